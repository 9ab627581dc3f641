// Spin-projected hopping terms shared by the site and line kernels.
//   D_mu psi(x) = P-^mu U_mu(x) psi(x+mu) + P+^mu U_mu(x-mu)^dag psi(x-mu)
// The time-boundary phase is folded into the stored U_t(Lt-1).
#pragma once
#include <type_traits>

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

// FP16 storage, two-row links: the operands of one projected hop in storage form, i.e. the
// neighbour's two half spinors (three 8-byte pairs of FP16 complex values each, and their FP32
// scales) and the first two rows of the link (three pairs).
struct HopRawH {
  Half2x2 sp[2][3];
  float sc[2];
  Half2x2 lk[3];
};

TP_DEV void hop_raw_load(HopRawH& r, const SpinorF<__half2>& nb, uint32_t j,
                         const LinkF<__half2>& u, uint32_t il) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      r.sp[h][q] = *reinterpret_cast<const Half2x2*>(at(nb.p[h] + (int64_t)(2 * q) * nb.stride, 2 * j));
    r.sc[h] = *at(nb.nrm[h], j);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q)
    r.lk[q] = *reinterpret_cast<const Half2x2*>(at(u.p + (int64_t)(2 * q) * u.stride, 2 * il));
}

// The same arithmetic as hop_dir's forward (FWD) or backward half, from operands in storage form.
template <int K, bool FWD>
TP_DEV void hop_raw_apply(const HopRawH& r, float c, cx<float>* out) {
  cx<float> psi[12], h[6], w[6];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float2 a = __half22float2(r.sp[hh][q].a), b = __half22float2(r.sp[hh][q].b);
      psi[6 * hh + 2 * q] = r.sc[hh] * cx<float>{a.x, a.y};
      psi[6 * hh + 2 * q + 1] = r.sc[hh] * cx<float>{b.x, b.y};
    }
  su3<float> U;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float2 a = __half22float2(r.lk[q].a), b = __half22float2(r.lk[q].b);
    U.e[2 * q] = {a.x, a.y};
    U.e[2 * q + 1] = {b.x, b.y};
  }
  su3_third_row(U);
  if constexpr (FWD) {
    proj_minus<K, float>(psi, h);
    mv(U, h, w);
    mv(U, h + 3, w + 3);
    recon_minus<K, float>(out, w, c);
  } else {
    proj_plus<K, float>(psi, h);
    mvd(U, h, w);
    mvd(U, h + 3, w + 3);
    recon_plus<K, float>(out, w, c);
  }
}

// Site index and the six neighbour indices of D_s at p3 site (p, t, s), in hop_dir's order
// (x forward, x backward, y forward, ...).
struct HopIdx {
  uint32_t i, j[6];
};
TP_DEV HopIdx hop_idx(const Geom& g, int p, int t, int s) {
  C3 q = p3_coords(g, p, s);
  int xp = q.x + 1 == g.Lx ? 0 : q.x + 1, xm = q.x == 0 ? g.Lx - 1 : q.x - 1;
  int yp = q.y + 1 == g.Ly ? 0 : q.y + 1, ym = q.y == 0 ? g.Ly - 1 : q.y - 1;
  int zp = q.z + 1 == g.Lz ? 0 : q.z + 1, zm = q.z == 0 ? g.Lz - 1 : q.z - 1;
  HopIdx r;
  r.i = p3_idx32(g, t, s);
  r.j[0] = p3_idx32(g, t, p3_index(g, xp, q.y, q.z));
  r.j[1] = p3_idx32(g, t, p3_index(g, xm, q.y, q.z));
  r.j[2] = p3_idx32(g, t, p3_index(g, q.x, yp, q.z));
  r.j[3] = p3_idx32(g, t, p3_index(g, q.x, ym, q.z));
  r.j[4] = p3_idx32(g, t, p3_index(g, q.x, q.y, zp));
  r.j[5] = p3_idx32(g, t, p3_index(g, q.x, q.y, zm));
  return r;
}

// D_s with FP16 storage and two-row links: each hop's loads are issued before the previous
// hop's arithmetic, so that every wavefront keeps two hops' loads in flight.  The operations and
// their order are hop_dir's (the compiler may still pair a few multiply-adds differently, which
// moves the FP16 result by at most its last bit).
TP_DEV void hop_space_raw(const HopIdx& x, const SpinorF<__half2>& nb, const LinkF<__half2>* u_here,
                          const LinkF<__half2>* u_there, float c, cx<float>* out) {
  HopRawH A, B;
  hop_raw_load(A, nb, x.j[0], u_here[0], x.i);
  hop_raw_load(B, nb, x.j[1], u_there[0], x.j[1]);
  hop_raw_apply<0, true>(A, c, out);
  hop_raw_load(A, nb, x.j[2], u_here[1], x.i);
  hop_raw_apply<0, false>(B, c, out);
  hop_raw_load(B, nb, x.j[3], u_there[1], x.j[3]);
  hop_raw_apply<1, true>(A, c, out);
  hop_raw_load(A, nb, x.j[4], u_here[2], x.i);
  hop_raw_apply<1, false>(B, c, out);
  hop_raw_load(B, nb, x.j[5], u_there[2], x.j[5]);
  hop_raw_apply<2, true>(A, c, out);
  hop_raw_apply<2, false>(B, c, out);
}

// Whether hop_space_p3 takes the FP16 pipeline above.
template <typename S, typename Lt, int ROWS>
constexpr bool hop_raw_path() {
  return std::is_same<S, __half2>::value && std::is_same<Lt, __half2>::value && ROWS == 2;
}

// out += c * D_s psi at p3 site (p, t, s): nb is the field on parity 1-p,
// u_here[k] the links on parity p, u_there[k] those on parity 1-p.
template <typename S, typename R, typename Lt, int ROWS = 3>
TP_DEV void hop_space_p3(const SpinorF<S>& nb, const LinkF<Lt>* u_here, const LinkF<Lt>* u_there,
                         const Geom& g, int p, int t, int s, R c, cx<R>* out) {
  const HopIdx x = hop_idx(g, p, t, s);
  if constexpr (hop_raw_path<S, Lt, ROWS>()) {
    hop_space_raw(x, nb, u_here, u_there, c, out);
  } else {
    hop_dir<0, S, R, Lt, ROWS>(nb, u_here[0], x.i, x.j[0], u_there[0], x.j[1], c, out);
    hop_dir<1, S, R, Lt, ROWS>(nb, u_here[1], x.i, x.j[2], u_there[1], x.j[3], c, out);
    hop_dir<2, S, R, Lt, ROWS>(nb, u_here[2], x.i, x.j[4], u_there[2], x.j[5], c, out);
  }
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
