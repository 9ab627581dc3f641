// Spin-projected hopping terms shared by the site and line kernels.
//   D_mu psi(x) = P-^mu U_mu(x) psi(x+mu) + P+^mu U_mu(x-mu)^dag psi(x-mu)
// The time-boundary phase is folded into the stored U_t(Lt-1).
#pragma once
#include "tp_device.h"

// out += c * D_t psi at p3 site (t, s); psi and the links live on the same parity.
// In the Dirac-Pauli basis P- = lower spins, P+ = upper spins.
template <typename S, typename R, typename Lt>
TP_DEV void hop_time_p3(const SpinorF<S>& f, const LinkF<Lt>& ut, const Geom& g, int t, int s, R c,
                        cx<R>* out) {
  int tf = t + 1 == g.Lt ? 0 : t + 1;
  int tb = t == 0 ? g.Lt - 1 : t - 1;
  const uint32_t i = p3_idx32(g, t, s);
  const uint32_t jf = p3_idx32(g, tf, s), jb = p3_idx32(g, tb, s);
  cx<R> v[6], w[6];
  load_half<S, R>(f, 1, jf, v);
  su3<R> U = load_su3<R, Lt>(ut, i);
  mv(U, v, w);
  mv(U, v + 3, w + 3);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[6 + k] += c * w[k];
  load_half<S, R>(f, 0, jb, v);
  su3<R> V = load_su3<R, Lt>(ut, jb);
  mvd(V, v, w);
  mvd(V, v + 3, w + 3);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] += c * w[k];
}

// One spatial direction K of the projected hop; c already includes the 1/2 of P+-.
// ROWS: stored rows of the links (2 = SU(3), third row rebuilt).
template <int K, typename S, typename R, typename Lt, int ROWS = 3>
TP_DEV void hop_dir(const SpinorF<S>& nb, const LinkF<Lt>& u_fwd, uint32_t i_fwd_link,
                    uint32_t jf, const LinkF<Lt>& u_bwd, uint32_t jb, R c, cx<R>* out) {
  cx<R> psi[12], h[6], w[6];
  load_spinor<S, R>(nb, jf, psi);
  proj_minus<K, R>(psi, h);
  su3<R> U = load_su3<R, Lt, ROWS>(u_fwd, i_fwd_link);
  mv(U, h, w);
  mv(U, h + 3, w + 3);
  recon_minus<K, R>(out, w, c);
  load_spinor<S, R>(nb, jb, psi);
  proj_plus<K, R>(psi, h);
  su3<R> V = load_su3<R, Lt, ROWS>(u_bwd, jb);
  mvd(V, h, w);
  mvd(V, h + 3, w + 3);
  recon_plus<K, R>(out, w, c);
}

// out += c * D_s psi at p3 site (p, t, s): nb is the field on parity 1-p,
// u_here[k] the links on parity p, u_there[k] those on parity 1-p.
template <typename S, typename R, typename Lt, int ROWS = 3>
TP_DEV void hop_space_p3(const SpinorF<S>& nb, const LinkF<Lt>* u_here, const LinkF<Lt>* u_there,
                         const Geom& g, int p, int t, int s, R c, cx<R>* out) {
  C3 q = p3_coords(g, p, s);
  const uint32_t i = p3_idx32(g, t, s);
  int xp = q.x + 1 == g.Lx ? 0 : q.x + 1, xm = q.x == 0 ? g.Lx - 1 : q.x - 1;
  int yp = q.y + 1 == g.Ly ? 0 : q.y + 1, ym = q.y == 0 ? g.Ly - 1 : q.y - 1;
  int zp = q.z + 1 == g.Lz ? 0 : q.z + 1, zm = q.z == 0 ? g.Lz - 1 : q.z - 1;
  hop_dir<0, S, R, Lt, ROWS>(nb, u_here[0], i, p3_idx32(g, t, p3_index(g, xp, q.y, q.z)), u_there[0],
                       p3_idx32(g, t, p3_index(g, xm, q.y, q.z)), c, out);
  hop_dir<1, S, R, Lt, ROWS>(nb, u_here[1], i, p3_idx32(g, t, p3_index(g, q.x, yp, q.z)), u_there[1],
                       p3_idx32(g, t, p3_index(g, q.x, ym, q.z)), c, out);
  hop_dir<2, S, R, Lt, ROWS>(nb, u_here[2], i, p3_idx32(g, t, p3_index(g, q.x, q.y, zp)), u_there[2],
                       p3_idx32(g, t, p3_index(g, q.x, q.y, zm)), c, out);
}

// p4 layout: out += c_t * D_t psi + c_sp * D_s psi at site i of parity p;
// src on parity 1-p; c_sp excludes the 1/2 of the spatial projectors.
template <typename S, typename R, typename Lt>
TP_DEV void hop_4d_p4(const SpinorF<S>& src, const LinkF<Lt>* u_here, const LinkF<Lt>* u_there,
                      const Geom& g, int p, uint32_t i, R c_t, R c_sp, cx<R>* out) {
  int xh = int(i % uint32_t(g.Lxh));
  uint32_t r = i / uint32_t(g.Lxh);
  int y = int(r % uint32_t(g.Ly));
  r /= uint32_t(g.Ly);
  int z = int(r % uint32_t(g.Lz));
  int t = int(r / uint32_t(g.Lz));
  int x = 2 * xh + ((y + z + t + p) & 1);
  auto idx = [&](int X, int Y, int Z, int T) -> uint32_t {
    return (uint32_t(X) + uint32_t(g.Lx) * (uint32_t(Y) + uint32_t(g.Ly) * (uint32_t(Z) + uint32_t(g.Lz) * uint32_t(T)))) >> 1;
  };
  int xp = x + 1 == g.Lx ? 0 : x + 1, xm = x == 0 ? g.Lx - 1 : x - 1;
  int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
  int zp = z + 1 == g.Lz ? 0 : z + 1, zm = z == 0 ? g.Lz - 1 : z - 1;
  int tp = t + 1 == g.Lt ? 0 : t + 1, tm = t == 0 ? g.Lt - 1 : t - 1;
  R ch = R(0.5) * c_sp;
  hop_dir<0, S, R, Lt>(src, u_here[0], i, idx(xp, y, z, t), u_there[0], idx(xm, y, z, t), ch, out);
  hop_dir<1, S, R, Lt>(src, u_here[1], i, idx(x, yp, z, t), u_there[1], idx(x, ym, z, t), ch, out);
  hop_dir<2, S, R, Lt>(src, u_here[2], i, idx(x, y, zp, t), u_there[2], idx(x, y, zm, t), ch, out);
  // time: forward -> lower spins, backward -> upper spins
  cx<R> v[6], w[6];
  const uint32_t jf = idx(x, y, z, tp), jb = idx(x, y, z, tm);
  load_half<S, R>(src, 1, jf, v);
  su3<R> U = load_su3<R, Lt>(u_here[3], i);
  mv(U, v, w);
  mv(U, v + 3, w + 3);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[6 + k] += c_t * w[k];
  load_half<S, R>(src, 0, jb, v);
  su3<R> V = load_su3<R, Lt>(u_there[3], jb);
  mvd(V, v, w);
  mvd(V, v + 3, w + 3);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] += c_t * w[k];
}
