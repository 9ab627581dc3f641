// One-off and layout kernels: canonical <-> internal spinor layouts, link
// packing, the per-time-line products W(t) and the FP64 closure of T^-1,
// the clover term in its chiral block form and (A + mu)^-1.
#include "tp_internal.h"

namespace {

constexpr int kBlock = 256;

TP_DEV void canon_coords(int64_t n, const Geom& g, int& x, int& y, int& z, int& t) {
  x = int(n % g.Lx);
  int64_t r = n / g.Lx;
  y = int(r % g.Ly);
  r /= g.Ly;
  z = int(r % g.Lz);
  t = int(r / g.Lz);
}

// internal (parity, index) of a site for the p3 or p4 layout
TP_DEV void site_pi(const Geom& g, bool l4, int x, int y, int z, int t, int& p, int64_t& i) {
  int64_t f3 = (int64_t)(x + g.Lx * (y + g.Ly * z));
  if (l4) {
    p = (x + y + z + t) & 1;
    i = (f3 + (int64_t)g.Lx * g.Ly * g.Lz * t) >> 1;
  } else {
    p = (x + y + z) & 1;
    i = p3_idx(g, t, int(f3 >> 1));
  }
}

// psi(colour) <- W^dag psi (to_axial) or W psi (from the axial frame), all four spins, FP64.
TP_DEV void rotate_spinor(const double2* __restrict__ w, int p, int64_t i, int64_t V2, bool dag,
                          cx<double>* v) {
  const double2* b = w + (int64_t)p * 9 * V2 + i;
  su3<double> W;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 e = b[(int64_t)k * V2];
    W.e[k] = cx<double>{e.x, e.y};
  }
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    cx<double> o[3];
    if (dag) mvd(W, v + 3 * sp, o);
    else mv(W, v + 3 * sp, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[3 * sp + c] = o[c];
  }
}

template <typename S>
__global__ void k_pack(const double2* __restrict__ canon, SpinorF<S> f0, SpinorF<S> f1, Geom g,
                       int64_t V, bool l4, bool g5, const double2* __restrict__ w) {
  using R = typename Prec<S>::R;
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  int x, y, z, t;
  canon_coords(n, g, x, y, z, t);
  int p;
  int64_t i;
  site_pi(g, l4, x, y, z, t, p, i);
  cx<double> d[12];
  const double2* src = canon + n * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) d[c] = cx<double>{src[c].x, src[c].y};
  if (w) rotate_spinor(w, p, i, g.V2, true, d);
  cx<R> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = cx<R>{R(d[c].re), R(d[c].im)};
  if (g5) {  // gamma5 = [[0,-1],[-1,0]] in the Dirac-Pauli basis
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      cx<R> a = v[c];
      v[c] = -v[6 + c];
      v[6 + c] = -a;
    }
  }
  store_spinor<S, R>(p ? f1 : f0, i, v);
}

template <typename S>
__global__ void k_unpack(double2* __restrict__ canon, SpinorF<S> f0, SpinorF<S> f1, Geom g,
                         int64_t V, bool l4, bool g5, const double2* __restrict__ w) {
  using R = typename Prec<S>::R;
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  int x, y, z, t;
  canon_coords(n, g, x, y, z, t);
  int p;
  int64_t i;
  site_pi(g, l4, x, y, z, t, p, i);
  cx<R> v[12];
  load_spinor<S, R>(p ? f1 : f0, i, v);
  if (g5) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      cx<R> a = v[c];
      v[c] = -v[6 + c];
      v[6 + c] = -a;
    }
  }
  cx<double> d[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) d[c] = cx<double>{double(v[c].re), double(v[c].im)};
  if (w) rotate_spinor(w, p, i, g.V2, false, d);
  double2* dst = canon + n * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) dst[c] = make_double2(d[c].re, d[c].im);
}

// links: canon [4][V][9] -> p4 FP64/FP32 (the 4D even-odd baseline), phase b folded
// into U_t(Lt-1)
__global__ void k_pack_links4(const double2* __restrict__ canon, double2* u4d, float2* u4f, Geom g,
                              int64_t V, double b) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mu = blockIdx.y;
  if (n >= V) return;
  int x, y, z, t;
  canon_coords(n, g, x, y, z, t);
  double ph = (mu == 3 && t == g.Lt - 1) ? b : 1.0;
  int p4;
  int64_t i4;
  site_pi(g, true, x, y, z, t, p4, i4);
  const double2* src = canon + ((int64_t)mu * V + n) * 9;
  int64_t V2 = V / 2;
  double2* d4 = u4d + ((int64_t)(mu * 2 + p4) * 9) * V2 + i4;
  float2* f4 = u4f + ((int64_t)(mu * 2 + p4) * 9) * V2;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 e = src[k];
    e.x *= ph;
    e.y *= ph;
    d4[(int64_t)k * V2] = e;
    f4[comp_off<float2>(k, 9, V2, i4)] = make_float2(float(e.x), float(e.y));
  }
}

TP_DEV void mm3(const cx<double>* a, const cx<double>* b, cx<double>* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = cmul(a[3 * i], b[j]);
      s += cmul(a[3 * i + 1], b[3 + j]);
      s += cmul(a[3 * i + 2], b[6 + j]);
      c[3 * i + j] = s;
    }
}

// W(t) = U'(t) U'(t+1) ... U'(Lt-1) per time line, U' the time links with the phase b
// folded into U'(Lt-1).  One thread per line: an Lt-step product, run once per gauge field.
__global__ void k_wline(const double2* __restrict__ canon, double2* wd, double2* poly, Geom g,
                        int64_t V, double b) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int p = blockIdx.y;
  if (s >= g.Vs2) return;
  int64_t V2 = g.V2;
  C3 q = p3_coords(g, p, s);
  int64_t f3 = (int64_t)q.x + (int64_t)g.Lx * (q.y + (int64_t)g.Ly * q.z);
  int64_t Vs = (int64_t)g.Lx * g.Ly * g.Lz;
  double2* w = wd + (int64_t)p * 9 * V2;
  cx<double> acc[9], u[9], nw[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = cx<double>{(k % 4 == 0) ? 1.0 : 0.0, 0.0};
  for (int t = g.Lt - 1; t >= 0; --t) {
    int64_t i = p3_idx(g, t, s);
    const double2* src = canon + ((int64_t)3 * V + f3 + Vs * t) * 9;
    double ph = t == g.Lt - 1 ? b : 1.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = cx<double>{ph * src[k].x, ph * src[k].y};
    mm3(u, acc, nw);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      acc[k] = nw[k];
      w[(int64_t)k * V2 + i] = make_double2(nw[k].re, nw[k].im);
    }
  }
  double2* pl = poly + (int64_t)p * 9 * g.Vs2;
#pragma unroll
  for (int k = 0; k < 9; ++k) pl[(int64_t)k * g.Vs2 + s] = make_double2(acc[k].re, acc[k].im);
}

// Axial-gauge links U^ax_mu(x) = W(x)^dag U'_mu(x) W(x+mu) with Omega = W^dag (Sec. II.C,
// App. C): every time link becomes the identity except U^ax_t(Lt-1) = W(0) = P.
// Writes the p3 layout (F64, F32) and a canonical copy for the clover build.
__global__ void k_axial_links(const double2* __restrict__ canon, const double2* __restrict__ wd,
                              double2* u3d, float2* u3f, double2* canon_ax, Geom g, int64_t V,
                              double b, int* flags) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mu = blockIdx.y;
  if (n >= V) return;
  int x, y, z, t;
  canon_coords(n, g, x, y, z, t);
  int xs[4] = {x, y, z, t};
  int ls[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
  xs[mu] = xs[mu] + 1 == ls[mu] ? 0 : xs[mu] + 1;
  int pa, pb;
  int64_t ia, ib;
  site_pi(g, false, x, y, z, t, pa, ia);
  site_pi(g, false, xs[0], xs[1], xs[2], xs[3], pb, ib);
  int64_t V2 = V / 2;
  cx<double> U[9], Wa[9], Wb[9], T1[9], T2[9];
  double ph = (mu == 3 && t == g.Lt - 1) ? b : 1.0;
  const double2* src = canon + ((int64_t)mu * V + n) * 9;
  bool finite = true;
  for (int k = 0; k < 9; ++k) {
    finite = finite && isfinite(src[k].x) && isfinite(src[k].y);
    U[k] = cx<double>{ph * src[k].x, ph * src[k].y};
    double2 ea = wd[((int64_t)pa * 9 + k) * V2 + ia];
    double2 eb = wd[((int64_t)pb * 9 + k) * V2 + ib];
    Wa[k] = cx<double>{ea.x, -ea.y};  // conj, transposed below
    Wb[k] = cx<double>{eb.x, eb.y};
  }
  cx<double> Wad[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Wad[3 * r + c] = Wa[3 * c + r];
  mm3(Wad, U, T1);
  mm3(T1, Wb, T2);
  {
    // spatial links: deviation of the axial-frame link from SU(3); time links: deviation of
    // the input link from unitarity (the axial frame is a gauge rotation only for unitary W)
    const cx<double>* m = mu < 3 ? T2 : U;
    double dev = 0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        cx<double> e = cx<double>{r == c ? -1.0 : 0.0, 0.0};
        for (int k = 0; k < 3; ++k) e += cmul(m[3 * r + k], conj(m[3 * c + k]));
        dev = fmax(dev, sqrt(norm2(e)));
      }
    if (mu < 3) {
      cx<double> c0 = cmul(m[4], m[8]) - cmul(m[5], m[7]);
      cx<double> c1 = cmul(m[5], m[6]) - cmul(m[3], m[8]);
      cx<double> c2 = cmul(m[3], m[7]) - cmul(m[4], m[6]);
      cx<double> det = cmul(m[0], c0) + cmul(m[1], c1) + cmul(m[2], c2);
      dev = fmax(dev, sqrt(norm2(det - cx<double>{1.0, 0.0})));
      if (!(dev <= 1e-9)) flags[0] = 1;
      if (!(dev <= 1e-13)) flags[3] = 1;
    } else if (!(dev <= 1e-10)) {
      flags[1] = 1;
    }
    if (!finite) flags[2] = 1;
  }
  double2* d3 = u3d + ((int64_t)(mu * 2 + pa) * 9) * V2 + ia;
  float2* f3 = u3f + ((int64_t)(mu * 2 + pa) * 9) * V2;
  double2* ca = canon_ax + ((int64_t)mu * V + n) * 9;
  for (int k = 0; k < 9; ++k) {
    d3[(int64_t)k * V2] = make_double2(T2[k].re, T2[k].im);
    f3[comp_off<float2>(k, 9, V2, ia)] = make_float2(float(T2[k].re), float(T2[k].im));
    ca[k] = make_double2(T2[k].re, T2[k].im);
  }
}

__global__ void k_to_half(const float2* __restrict__ src, __half2* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = __float22half2_rn(src[i]);
}

TP_DEV bool inv3(const cx<double>* m, cx<double>* r) {
  // adjugate / determinant
  cx<double> c00 = cmul(m[4], m[8]) - cmul(m[5], m[7]);
  cx<double> c01 = cmul(m[5], m[6]) - cmul(m[3], m[8]);
  cx<double> c02 = cmul(m[3], m[7]) - cmul(m[4], m[6]);
  cx<double> det = cmul(m[0], c00) + cmul(m[1], c01) + cmul(m[2], c02);
  double dn = norm2(det);
  if (!(dn > 0.0)) return false;
  cx<double> id = cx<double>{det.re / dn, -det.im / dn};
  r[0] = cmul(c00, id);
  r[3] = cmul(c01, id);
  r[6] = cmul(c02, id);
  r[1] = cmul(cmul(m[2], m[7]) - cmul(m[1], m[8]), id);
  r[4] = cmul(cmul(m[0], m[8]) - cmul(m[2], m[6]), id);
  r[7] = cmul(cmul(m[1], m[6]) - cmul(m[0], m[7]), id);
  r[2] = cmul(cmul(m[1], m[5]) - cmul(m[2], m[4]), id);
  r[5] = cmul(cmul(m[2], m[3]) - cmul(m[0], m[5]), id);
  r[8] = cmul(cmul(m[0], m[4]) - cmul(m[1], m[3]), id);
  return true;
}

TP_DEV double norm1(const cx<double>* m) {
  double best = 0;
  for (int j = 0; j < 3; ++j) {
    double s = 0;
    for (int i = 0; i < 3; ++i) s += sqrt(norm2(m[3 * i + j]));
    best = fmax(best, s);
  }
  return best;
}

// Closure of the temporal inverse per line: K = (I - mu^-Lt P)^-1 and G = K P / mu,
// so that delta = G sigma(0) for T^-1 and delta' = G^dagger rho(Lt-1) for T^dagger^-1.
__global__ void k_closure(const double2* __restrict__ poly, double2* gclos, float2* gclos_f,
                          double* cond, Geom g, double mu, double mu_mlt) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  int p = blockIdx.y;
  if (s >= g.Vs2) return;
  const double2* pl = poly + (int64_t)p * 9 * g.Vs2;
  cx<double> P[9], A[9], K[9], G[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 e = pl[(int64_t)k * g.Vs2 + s];
    P[k] = cx<double>{e.x, e.y};
    A[k] = cx<double>{(k % 4 == 0 ? 1.0 : 0.0) - mu_mlt * e.x, -mu_mlt * e.y};
  }
  double c;
  if (inv3(A, K)) {
    c = norm1(A) * norm1(K);
    mm3(K, P, G);
  } else {
    c = INFINITY;
    for (int k = 0; k < 9; ++k) G[k] = cx<double>{0, 0};
  }
  if (!isfinite(c)) c = INFINITY;
  cond[(int64_t)p * g.Vs2 + s] = c;
  double2* go = gclos + (int64_t)p * 9 * g.Vs2;
  float2* gf = gclos_f + (int64_t)p * 9 * g.Vs2;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    go[(int64_t)k * g.Vs2 + s] = make_double2(G[k].re / mu, G[k].im / mu);
    gf[(int64_t)k * g.Vs2 + s] = make_float2(float(G[k].re / mu), float(G[k].im / mu));
  }
}

// ---- clover ------------------------------------------------------------------------------
struct SigTab {
  double2 s[6][2][2][2];  // plane, chirality, row, col:  coef_p * V_chi^dag sigma_p V_chi / 2
};

TP_DEV void load_link(const double2* canon, const Geom& g, int64_t V, int mu, int x, int y, int z,
                      int t, cx<double>* u) {
  x = (x + g.Lx) % g.Lx;
  y = (y + g.Ly) % g.Ly;
  z = (z + g.Lz) % g.Lz;
  t = (t + g.Lt) % g.Lt;
  int64_t n = (int64_t)x + (int64_t)g.Lx * (y + (int64_t)g.Ly * (z + (int64_t)g.Lz * t));
  const double2* src = canon + ((int64_t)mu * V + n) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = cx<double>{src[k].x, src[k].y};
}
TP_DEV void dag3(const cx<double>* a, cx<double>* b) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) b[3 * i + j] = conj(a[3 * j + i]);
}
TP_DEV void chain4(const cx<double>* a, const cx<double>* b, const cx<double>* c,
                   const cx<double>* d, cx<double>* out) {
  cx<double> t1[9], t2[9];
  mm3(a, b, t1);
  mm3(t1, c, t2);
  mm3(t2, d, out);
}

// F_{mu nu}(x) = (Q - Q^dag)/8 - tr/3 with Q the four leaves, all oriented mu -> nu.
TP_DEV void field_strength(const double2* canon, const Geom& g, int64_t V, int mu, int nu, int x,
                           int y, int z, int t, cx<double>* F) {
  // U_d(x + am*mu + an*nu); the offsets are formed arithmetically (a direction table indexed
  // by mu and nu would live in scratch memory)
  auto L = [&](int d, int am, int an, cx<double>* u) {
    load_link(canon, g, V, d, x + am * (mu == 0) + an * (nu == 0), y + am * (mu == 1) + an * (nu == 1),
              z + am * (mu == 2) + an * (nu == 2), t + am * (mu == 3) + an * (nu == 3), u);
  };
  cx<double> a[9], b[9], c[9], d[9], cd[9], dd[9], leaf[9], Q[9];
  for (int k = 0; k < 9; ++k) Q[k] = cx<double>{0, 0};
  // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
  L(mu, 0, 0, a); L(nu, 1, 0, b); L(mu, 0, 1, c); L(nu, 0, 0, d);
  dag3(c, cd); dag3(d, dd); chain4(a, b, cd, dd, leaf);
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  // leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
  L(nu, 0, 0, a); L(mu, -1, 1, b); L(nu, -1, 0, c); L(mu, -1, 0, d);
  { cx<double> bd[9]; dag3(b, bd); dag3(c, cd); chain4(a, bd, cd, d, leaf); }
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  // leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
  L(mu, -1, 0, a); L(nu, -1, -1, b); L(mu, -1, -1, c); L(nu, 0, -1, d);
  { cx<double> ad[9], bd[9]; dag3(a, ad); dag3(b, bd); chain4(ad, bd, c, d, leaf); }
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  // leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
  L(nu, 0, -1, a); L(mu, 0, -1, b); L(nu, 1, -1, c); L(mu, 0, 0, d);
  { cx<double> ad[9]; dag3(a, ad); dag3(d, dd); chain4(ad, b, c, dd, leaf); }
  for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[3 * i + j] = 0.125 * (Q[3 * i + j] - conj(Q[3 * j + i]));
  cx<double> tr = (1.0 / 3.0) * (F[0] + F[4] + F[8]);
  F[0] -= tr; F[4] -= tr; F[8] -= tr;
}

// One chiral block C of the clover term at every site: the sum over the six planes of the
// sigma-table coefficients times F_{mu nu}, accumulated only into the stored entries of the
// hermitian 6x6 block (6 real diagonal, 15 complex below it), all at compile-time indices so
// that they stay in registers.
template <int C>
__global__ void __launch_bounds__(64) k_clover_build(const double2* __restrict__ canon, double2* a3d,
                                                     float2* a3f, double2* a4d, float2* a4f, Geom g,
                                                     int64_t V, SigTab sig) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  int x, y, z, t;
  canon_coords(n, g, x, y, z, t);
  double dg[6];
  cx<double> lo[15];
#pragma unroll
  for (int k = 0; k < 6; ++k) dg[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 15; ++k) lo[k] = cx<double>{0, 0};
#pragma unroll
  for (int pl = 0; pl < 6; ++pl) {
    // planes 03 13 23 01 02 12
    const int mu = pl < 3 ? pl : (pl == 5 ? 1 : 0);
    const int nu = pl < 3 ? 3 : (pl == 3 ? 1 : 2);
    const double2 w00 = sig.s[pl][C][0][0], w01 = sig.s[pl][C][0][1];
    const double2 w10 = sig.s[pl][C][1][0], w11 = sig.s[pl][C][1][1];
    if (fabs(w00.x) + fabs(w00.y) + fabs(w01.x) + fabs(w01.y) + fabs(w10.x) + fabs(w10.y) +
            fabs(w11.x) + fabs(w11.y) == 0.0)
      continue;  // coefficient zero
    cx<double> F[9];
    field_strength(canon, g, V, mu, nu, x, y, z, t, F);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q <= r; ++q) {
        const int sr = r / 3, a = r % 3, sq = q / 3, bb = q % 3;
        const double2 wv = sr == 0 ? (sq == 0 ? w00 : w01) : (sq == 0 ? w10 : w11);
        const cx<double> v = cmul(cx<double>{wv.x, wv.y}, F[3 * a + bb]);
        if (r == q) dg[r] += v.re;
        else lo[r * (r - 1) / 2 + q] += v;
      }
  }
  int p3, p4;
  int64_t i3, i4;
  site_pi(g, false, x, y, z, t, p3, i3);
  site_pi(g, true, x, y, z, t, p4, i4);
  const int64_t V2 = V / 2;
  double2* d3 = a3d ? a3d + ((int64_t)p3 * 36 + 18 * C) * V2 : nullptr;
  float2* f3 = a3f ? a3f + ((int64_t)p3 * 36 + 18 * C) * V2 : nullptr;
  double2* d4 = a4d ? a4d + ((int64_t)p4 * 36 + 18 * C) * V2 : nullptr;
  float2* f4 = a4f ? a4f + ((int64_t)p4 * 36 + 18 * C) * V2 : nullptr;
  // slots 0..2: diagonal pairs, 3..17: lower triangle row-major (the layout of store_herm6_parts)
#pragma unroll
  for (int slot = 0; slot < 18; ++slot) {
    const double2 v = slot < 3 ? make_double2(dg[2 * slot], dg[2 * slot + 1])
                               : make_double2(lo[slot - 3].re, lo[slot - 3].im);
    if (d3) d3[(int64_t)slot * V2 + i3] = v;
    if (f3) f3[comp_off<float2>(slot, 18, V2, i3)] = make_float2(float(v.x), float(v.y));
    if (d4) d4[(int64_t)slot * V2 + i4] = v;
    if (f4) f4[comp_off<float2>(slot, 18, V2, i4)] = make_float2(float(v.x), float(v.y));
  }
}

// Inverse of a hermitian 6x6 block from its stored form (real diagonal dg, lower triangle lo
// row-major), by H = L D L^dag with L unit lower triangular and D real: H^-1 = L^-dag D^-1 L^-1.
// Every loop has fixed bounds, so all entries stay in registers.  Returns false when a pivot
// falls below 1e-13 of the largest diagonal entry (the block is then reported singular).
TP_DEV bool inv_herm6(const double* dg, const cx<double>* lo, double* idg, cx<double>* ilo) {
  auto T = [](int r, int c) { return r * (r - 1) / 2 + c; };  // lower-triangle index, r > c
  double scale = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) scale = fmax(scale, fabs(dg[k]));
  double d[6];
  cx<double> L[15];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double dj = dg[j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= norm2(L[T(j, k)]) * d[k];
    d[j] = dj;
    if (!(fabs(dj) > 1e-13 * scale)) ok = false;
    const double id = 1.0 / dj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      cx<double> v = lo[T(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= d[k] * cmul(L[T(i, k)], conj(L[T(j, k)]));
      L[T(i, j)] = id * v;
    }
  }
  // M = L^-1 (unit lower triangular), by forward substitution
  cx<double> M[15];
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) {
      cx<double> v = -L[T(i, j)];
#pragma unroll
      for (int k = j + 1; k < i; ++k) v -= cmul(L[T(i, k)], M[T(k, j)]);
      M[T(i, j)] = v;
    }
  // H^-1[i][j] = sum_{k >= i} conj(M[k][i]) M[k][j] / d[k]  (i >= j; M[k][k] = 1)
  double id[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) id[k] = 1.0 / d[k];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double v = id[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) v += norm2(M[T(k, i)]) * id[k];
    idg[i] = v;
  }
#pragma unroll
  for (int i = 1; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) {
      cx<double> v = id[i] * M[T(i, j)];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) v += id[k] * cmul(conj(M[T(k, i)]), M[T(k, j)]);
      ilo[T(i, j)] = v;
    }
  return ok;
}

// Stored form of a hermitian block: slots 0..2 diagonal pairs, 3..17 the lower triangle
// row-major.  The clover kernels read this form (clover_apply, herm6_from_slots).
TP_DEV void load_herm6_parts(const double2* base, int64_t st, int64_t i, double* dg, cx<double>* lo) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double2 v = base[(int64_t)k * st + i];
    dg[2 * k] = v.x;
    dg[2 * k + 1] = v.y;
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    const double2 v = base[(int64_t)(3 + k) * st + i];
    lo[k] = cx<double>{v.x, v.y};
  }
}
TP_DEV void store_herm6_parts(const double* dg, const cx<double>* lo, double2* d, float2* f, int64_t st,
                              int64_t i) {
#pragma unroll
  for (int slot = 0; slot < 18; ++slot) {
    const double2 v = slot < 3 ? make_double2(dg[2 * slot], dg[2 * slot + 1])
                               : make_double2(lo[slot - 3].re, lo[slot - 3].im);
    d[(int64_t)slot * st + i] = v;
    if (f) f[comp_off<float2>(slot, 18, st, i)] = make_float2(float(v.x), float(v.y));
  }
}

// From the stored A/2 blocks (layout p3 or p4), write (A+mu)/2 and (A+mu)^-1/2 blocks.
__global__ void __launch_bounds__(64) k_clover_derived(const double2* __restrict__ a, double2* amu,
                                                       double2* ainv, float2* amu_f, float2* ainv_f,
                                                       int64_t V2, double mu, int* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int p = blockIdx.y;
  if (i >= V2) return;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t off = ((int64_t)p * 36 + 18 * c) * V2;
    double dg[6], idg[6];
    cx<double> lo[15], ilo[15];
    if (a) {
      load_herm6_parts(a + off, V2, i, dg, lo);
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) dg[k] = 0.0;
#pragma unroll
      for (int k = 0; k < 15; ++k) lo[k] = cx<double>{0, 0};
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) dg[k] += 0.5 * mu;  // (A + mu)/2
    store_herm6_parts(dg, lo, amu + off, amu_f ? amu_f + off : nullptr, V2, i);
    // (A+mu)^-1/2 = [(A+mu)/2]^-1 / 4
    if (!inv_herm6(dg, lo, idg, ilo)) {
      bad[0] = 1;
#pragma unroll
      for (int k = 0; k < 6; ++k) idg[k] = 0.0;
#pragma unroll
      for (int k = 0; k < 15; ++k) ilo[k] = cx<double>{0, 0};
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) idg[k] *= 0.25;
#pragma unroll
    for (int k = 0; k < 15; ++k) ilo[k] = 0.25 * ilo[k];
    store_herm6_parts(idg, ilo, ainv + off, ainv_f ? ainv_f + off : nullptr, V2, i);
  }
}

// Plaquette averages (1/3 Re tr) over spatial and temporal planes: per-block partials.
__global__ void k_plaquette(const double2* __restrict__ canon, Geom g, int64_t V, double* part) {
  __shared__ double sh[2][kBlock];
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ps = 0, pt = 0;
  if (n < V) {
    int x, y, z, t;
    canon_coords(n, g, x, y, z, t);
    // planes 01 02 12 03 13 23; offsets formed arithmetically, not from a table indexed by
    // the plane (which would live in scratch memory)
#pragma unroll 1
    for (int pl = 0; pl < 6; ++pl) {
      const int mu = pl == 2 || pl == 4 ? 1 : (pl == 5 ? 2 : 0);
      const int nu = pl < 3 ? (pl == 0 ? 1 : 2) : 3;
      cx<double> a[9], b[9], c[9], d[9], cd[9], dd[9], leaf[9];
      load_link(canon, g, V, mu, x, y, z, t, a);
      load_link(canon, g, V, nu, x + (mu == 0), y + (mu == 1), z + (mu == 2), t + (mu == 3), b);
      load_link(canon, g, V, mu, x + (nu == 0), y + (nu == 1), z + (nu == 2), t + (nu == 3), c);
      load_link(canon, g, V, nu, x, y, z, t, d);
      dag3(c, cd);
      dag3(d, dd);
      chain4(a, b, cd, dd, leaf);
      double re = (leaf[0].re + leaf[4].re + leaf[8].re) / 3.0;
      if (pl < 3) ps += re; else pt += re;
    }
  }
  sh[0][threadIdx.x] = ps;
  sh[1][threadIdx.x] = pt;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

inline unsigned nblk(int64_t n, int64_t b = kBlock) { return (unsigned)((n + b - 1) / b); }

template <typename S>
void pack_t(tp_ctx ctx, const double2* canon, Field& dst, bool l4, bool g5, const double2* w) {
  const Lattice& L = ctx->lat;
  hipLaunchKernelGGL(k_pack<S>, dim3(nblk(L.V)), dim3(kBlock), 0, ctx->stream, canon,
                     dst.template par<S>(0), dst.template par<S>(1), L.g, L.V, l4, g5, w);
  LAUNCH_CHECK();
}
template <typename S>
void unpack_t(tp_ctx ctx, const Field& src, double2* canon, bool l4, bool g5, const double2* w) {
  const Lattice& L = ctx->lat;
  hipLaunchKernelGGL(k_unpack<S>, dim3(nblk(L.V)), dim3(kBlock), 0, ctx->stream, canon,
                     src.template par<S>(0), src.template par<S>(1), L.g, L.V, l4, g5, w);
  LAUNCH_CHECK();
}


// ---- SW-term link force -----------------------------------------------------------------
// With x and lambda (dL = -Re <lambda, dM x>), the SW term contributes
//   s(U) = Re sum_x sum_p tr(Q_p(x) Yh_p(x)),  Yh_p = (c_p/2)(Z - Z^dag),
//   Z = W/8 - tr(W)/24,  W_p(x) = sum_{s s'} sigma_p[s][s'] x_s'(x) lambda_s(x)^dag,
// Q_p the four-leaf sum of plane p.  Each leaf is a plaquette read from one of its corners,
// so a link's derivative collects, from each plaquette that contains it, the product of the
// other three factors with Yh of every corner inserted at that corner.
struct SigmaTab {
  double2 s[6][4][4];  // sigma_{mu nu} = [gamma_mu, gamma_nu]/2, planes (03 13 23 01 02 12)
};

TP_DEV int plane_index(int a, int b) {  // a < b
  return b == 3 ? a : (a == 0 ? (b == 1 ? 3 : 4) : 5);
}

__global__ void __launch_bounds__(128) k_clover_Y(SpinorF<double2> x0, SpinorF<double2> x1,
                                                   SpinorF<double2> l0, SpinorF<double2> l1,
                                                   double2* Y, Geom g, int64_t V, SigmaTab sig,
                                                   double c_s, double c_t) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  int x, y, z, t;
  canon_coords(n, g, x, y, z, t);
  const int p = (x + y + z) & 1;
  const int64_t i = p3_idx(g, t, (x + g.Lx * (y + g.Ly * z)) >> 1);
  cx<double> xs[12], ls[12];
  load_spinor<double2, double>(p ? x1 : x0, i, xs);
  load_spinor<double2, double>(p ? l1 : l0, i, ls);
  // W_ba = sum_s v_sb conj(lambda_sa) with v_sb = sum_s' sigma_ss' x_s'b; every loop is
  // unrolled so that the spinor components and the table are read at constant indices (arrays
  // indexed by a loop variable would live in scratch memory)
#pragma unroll
  for (int pl = 0; pl < 6; ++pl) {
    cx<double> W[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = czero<double>();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cx<double> v[3] = {czero<double>(), czero<double>(), czero<double>()};
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const cx<double> sg = cx<double>{sig.s[pl][s][sp].x, sig.s[pl][s][sp].y};
#pragma unroll
        for (int b = 0; b < 3; ++b) v[b] += cmul(sg, xs[3 * sp + b]);
      }
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) W[3 * b + a] += cmul(v[b], conj(ls[3 * s + a]));
    }
    const cx<double> tr = W[0] + W[4] + W[8];
    const double c = 0.5 * (pl < 3 ? c_t : c_s);
    double2* out = Y + ((int64_t)pl * V + n) * 9;
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        cx<double> zrq = (1.0 / 8.0) * W[3 * r + q], zqr = (1.0 / 8.0) * W[3 * q + r];
        if (r == q) {
          zrq -= (1.0 / 24.0) * tr;
          zqr -= (1.0 / 24.0) * tr;
        }
        const cx<double> v = c * (zrq - conj(zqr));
        out[3 * r + q] = make_double2(v.re, v.im);
      }
  }
}

TP_DEV void load_y(const double2* Y, const Geom& g, int64_t V, int pl, int x, int y, int z, int t,
                   cx<double>* m) {
  x = (x + g.Lx) % g.Lx;
  y = (y + g.Ly) % g.Ly;
  z = (z + g.Lz) % g.Lz;
  t = (t + g.Lt) % g.Lt;
  const int64_t n = (int64_t)x + (int64_t)g.Lx * (y + (int64_t)g.Ly * (z + (int64_t)g.Lz * t));
  const double2* src = Y + ((int64_t)pl * V + n) * 9;
  for (int k = 0; k < 9; ++k) m[k] = cx<double>{src[k].x, src[k].y};
}

TP_DEV void madd3(const cx<double>* a, const cx<double>* b, cx<double>* acc) {
  cx<double> c[9];
  mm3(a, b, c);
  for (int k = 0; k < 9; ++k) acc[k] += c[k];
}

// R = Ya M1 M2 M3 + M1 Yb M2 M3 + M1 M2 Yc M3 + M1 M2 M3 Yd
TP_DEV void insert4(const cx<double>* M1, const cx<double>* M2, const cx<double>* M3, const cx<double>* Ya,
                    const cx<double>* Yb, const cx<double>* Yc, const cx<double>* Yd, cx<double>* R) {
  cx<double> P23[9], P123[9], T[9], P12[9];
  mm3(M2, M3, P23);
  mm3(M1, P23, P123);
  mm3(Ya, P123, R);
  mm3(Yb, P23, T);
  madd3(M1, T, R);
  mm3(M1, M2, P12);
  mm3(Yc, M3, T);
  madd3(P12, T, R);
  madd3(P123, Yd, R);
}

__global__ void __launch_bounds__(64) k_clover_force(const double2* __restrict__ canon,
                                                      const double2* __restrict__ Y, double2* grad,
                                                      Geom g, int64_t V, int projected) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  if (n >= V) return;
  int c[4];
  canon_coords(n, g, c[0], c[1], c[2], c[3]);
  auto at = [&](int d1, int s1, int d2, int s2, int& X, int& Yy, int& Z, int& T) {
    int q[4] = {c[0], c[1], c[2], c[3]};
    if (d1 >= 0) q[d1] += s1;
    if (d2 >= 0) q[d2] += s2;
    X = q[0]; Yy = q[1]; Z = q[2]; T = q[3];
  };
  cx<double> G[9];
  for (int k = 0; k < 9; ++k) G[k] = czero<double>();
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
    const int pl = plane_index(a, b);
    cx<double> L0[9], L1[9], L2[9], L3[9], T[9], Ya[9], Yb[9], Yc[9], Yd[9], R[9];
    int X, Yy, Z, Tt;
    // plaquette(base): L0 = U_a(base), L1 = U_b(base+a), L2 = U_a(base+b)^dag, L3 = U_b(base)^dag
    // corners c0 = base, c1 = base+a, c2 = base+a+b, c3 = base+b
    auto load_plaq = [&](int d, int sd) {  // base = x + sd * e_d (d < 0: base = x)
      at(d, sd, -1, 0, X, Yy, Z, Tt);
      const int bx = X, by = Yy, bz = Z, bt = Tt;
      int e[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
      load_link(canon, g, V, a, bx, by, bz, bt, L0);
      load_link(canon, g, V, b, bx + e[a][0], by + e[a][1], bz + e[a][2], bt + e[a][3], L1);
      load_link(canon, g, V, a, bx + e[b][0], by + e[b][1], bz + e[b][2], bt + e[b][3], T);
      dag3(T, L2);
      load_link(canon, g, V, b, bx, by, bz, bt, T);
      dag3(T, L3);
      load_y(Y, g, V, pl, bx, by, bz, bt, Ya);                                              // c0
      load_y(Y, g, V, pl, bx + e[a][0], by + e[a][1], bz + e[a][2], bt + e[a][3], Yb);      // c1
      load_y(Y, g, V, pl, bx + e[a][0] + e[b][0], by + e[a][1] + e[b][1], bz + e[a][2] + e[b][2],
             bt + e[a][3] + e[b][3], Yc);                                                   // c2
      load_y(Y, g, V, pl, bx + e[b][0], by + e[b][1], bz + e[b][2], bt + e[b][3], Yd);      // c3
    };
    if (mu == a) {
      // the link is L0 of the plaquette based at x, and L2 (daggered) of the one at x - b
      load_plaq(-1, 0);
      insert4(L1, L2, L3, Yb, Yc, Yd, Ya, R);  // R_0: corners c1 c2 c3 before L1 L2 L3, c0 last
      dag3(R, T);
      for (int k = 0; k < 9; ++k) G[k] += T[k];
      load_plaq(b, -1);
      insert4(L3, L0, L1, Yd, Ya, Yb, Yc, R);  // R_2
      for (int k = 0; k < 9; ++k) G[k] += R[k];
    } else {
      // the link is L1 of the plaquette based at x - a, and L3 (daggered) of the one at x
      load_plaq(a, -1);
      insert4(L2, L3, L0, Yc, Yd, Ya, Yb, R);  // R_1
      dag3(R, T);
      for (int k = 0; k < 9; ++k) G[k] += T[k];
      load_plaq(-1, 0);
      insert4(L0, L1, L2, Ya, Yb, Yc, Yd, R);  // R_3
      for (int k = 0; k < 9; ++k) G[k] += R[k];
    }
  }
  double2* out = grad + ((int64_t)mu * V + n) * 9;
  if (!projected) {
    for (int k = 0; k < 9; ++k) out[k] = make_double2(out[k].x + G[k].re, out[k].y + G[k].im);
    return;
  }
  // su(3) projection TH[i U G^dag]
  cx<double> U[9], Gd[9], M[9];
  load_link(canon, g, V, mu, c[0], c[1], c[2], c[3], U);
  dag3(G, Gd);
  mm3(U, Gd, M);
  for (int k = 0; k < 9; ++k) M[k] = cx<double>{-M[k].im, M[k].re};  // i U G^dag
  const double trh = (M[0].re + M[4].re + M[8].re) / 3.0;
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) {
      cx<double> h = 0.5 * (M[3 * r + q] + conj(M[3 * q + r]));
      if (r == q) h.re -= trh;
      out[3 * r + q] = make_double2(out[3 * r + q].x + h.re, out[3 * r + q].y + h.im);
    }
}

}  // namespace

void launch_pack(tp_ctx ctx, const double2* canon, Field& dst, bool l4, bool g5, const double2* w) {
  ProfScope ps(ctx, KID_PACK, double(ctx->lat.V) * (192 + 12 * dst.elem_bytes() + (w ? 144 : 0)));
  switch (dst.prec) {
    case TP_F64: pack_t<double2>(ctx, canon, dst, l4, g5, w); break;
    case TP_F32: pack_t<float2>(ctx, canon, dst, l4, g5, w); break;
    default: pack_t<__half2>(ctx, canon, dst, l4, g5, w); break;
  }
}

void launch_unpack(tp_ctx ctx, const Field& src, double2* canon, bool l4, bool g5, const double2* w) {
  ProfScope ps(ctx, KID_PACK, double(ctx->lat.V) * (192 + 12 * src.elem_bytes() + (w ? 144 : 0)));
  switch (src.prec) {
    case TP_F64: unpack_t<double2>(ctx, src, canon, l4, g5, w); break;
    case TP_F32: unpack_t<float2>(ctx, src, canon, l4, g5, w); break;
    default: unpack_t<__half2>(ctx, src, canon, l4, g5, w); break;
  }
}

void launch_pack_links(tp_ctx ctx, tp_gauge g) {
  const Lattice& L = ctx->lat;
  hipLaunchKernelGGL(k_pack_links4, dim3(nblk(L.V), 4), dim3(kBlock), 0, ctx->stream, g->canon,
                     g->u4_d, g->u4_f, L.g, L.V, double(ctx->bc));
  LAUNCH_CHECK();
}

void launch_wline(tp_ctx ctx, tp_gauge g) {
  const Lattice& L = ctx->lat;
  hipLaunchKernelGGL(k_wline, dim3((L.Vs2 + 63) / 64, 2), dim3(64), 0, ctx->stream, g->canon,
                     g->w_d, g->poly, L.g, L.V, double(ctx->bc));
  LAUNCH_CHECK();
}

void launch_to_half(tp_ctx ctx, const float2* src, __half2* dst, int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_to_half, dim3((unsigned)nb), dim3(256), 0, ctx->stream, src, dst, n);
  LAUNCH_CHECK();
}

void launch_axial_links(tp_ctx ctx, tp_gauge g, int* flags) {
  const Lattice& L = ctx->lat;
  hipLaunchKernelGGL(k_axial_links, dim3(nblk(L.V, 64), 4), dim3(64), 0, ctx->stream, g->canon,
                     g->w_d, g->u3_d, g->u3_f, g->canon_ax, L.g, L.V, double(ctx->bc), flags);
  LAUNCH_CHECK();
}

void launch_closure(tp_ctx ctx, tp_op op, double* cond) {
  const Lattice& L = ctx->lat;
  double mu_mlt = pow(op->mu, -double(L.L[3]));
  hipLaunchKernelGGL(k_closure, dim3((L.Vs2 + 63) / 64, 2), dim3(64), 0, ctx->stream,
                     op->g->poly, op->gclos, op->gclos_f, cond, L.g, op->mu, mu_mlt);
  LAUNCH_CHECK();
}

void launch_clover_build(tp_ctx ctx, tp_clover c, const double sig[6][2][2][2][2]) {
  // p3 blocks from the axial-gauge links (the frame of every p3 operator), p4 blocks
  // from the original links (the 4D even-odd baseline)
  const Lattice& L = ctx->lat;
  SigTab t;
  for (int p = 0; p < 6; ++p)
    for (int ch = 0; ch < 2; ++ch)
      for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) t.s[p][ch][r][q] = make_double2(sig[p][ch][r][q][0], sig[p][ch][r][q][1]);
  hipLaunchKernelGGL(k_clover_build<0>, dim3(nblk(L.V, 64)), dim3(64), 0, ctx->stream, c->g->canon_ax,
                     c->a3_d, c->a3_f, (double2*)nullptr, (float2*)nullptr, L.g, L.V, t);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_clover_build<1>, dim3(nblk(L.V, 64)), dim3(64), 0, ctx->stream, c->g->canon_ax,
                     c->a3_d, c->a3_f, (double2*)nullptr, (float2*)nullptr, L.g, L.V, t);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_clover_build<0>, dim3(nblk(L.V, 64)), dim3(64), 0, ctx->stream, c->g->canon,
                     (double2*)nullptr, (float2*)nullptr, c->a4_d, c->a4_f, L.g, L.V, t);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_clover_build<1>, dim3(nblk(L.V, 64)), dim3(64), 0, ctx->stream, c->g->canon,
                     (double2*)nullptr, (float2*)nullptr, c->a4_d, c->a4_f, L.g, L.V, t);
  LAUNCH_CHECK();
}

void launch_clover_derived(tp_ctx ctx, tp_op op, int* bad) {
  const Lattice& L = ctx->lat;
  const double2* a4 = op->c ? op->c->a4_d : nullptr;
  const double2* a3 = op->c ? op->c->a3_d : nullptr;
  hipLaunchKernelGGL(k_clover_derived, dim3(nblk(L.V2, 64), 2), dim3(64), 0, ctx->stream, a4,
                     op->a4_mu, op->a4_inv, op->a4_mu_f, op->a4_inv_f, L.V2, op->mu, bad);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_clover_derived, dim3(nblk(L.V2, 64), 2), dim3(64), 0, ctx->stream, a3,
                     op->a3_mu, op->a3_inv, op->a3_mu_f, op->a3_inv_f, L.V2, op->mu, bad);
  LAUNCH_CHECK();
}

void launch_plaquette(tp_ctx ctx, tp_gauge g, double* part) {
  const Lattice& L = ctx->lat;
  hipLaunchKernelGGL(k_plaquette, dim3(nblk(L.V)), dim3(kBlock), 0, ctx->stream, g->canon, L.g,
                     L.V, part);
  LAUNCH_CHECK();
}

void launch_clover_force(tp_op op, const Field& x, const Field& lam, double2* grad, bool projected,
                         const double sig[6][4][4][2]) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  SigmaTab t;
  for (int p = 0; p < 6; ++p)
    for (int r = 0; r < 4; ++r)
      for (int q = 0; q < 4; ++q) t.s[p][r][q] = make_double2(sig[p][r][q][0], sig[p][r][q][1]);
  double2* Y = static_cast<double2*>(dev_alloc(ctx, size_t(6) * L.V * 9 * sizeof(double2)));
  try {
    hipLaunchKernelGGL(k_clover_Y, dim3(nblk(L.V, 128)), dim3(128), 0, ctx->stream, x.par<double2>(0),
                       x.par<double2>(1), lam.par<double2>(0), lam.par<double2>(1), Y, L.g, L.V, t,
                       op->c->cs, op->c->ct);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_clover_force, dim3(nblk(L.V, 64), 4), dim3(64), 0, ctx->stream, op->g->canon, Y,
                       grad, L.g, L.V, projected ? 1 : 0);
    LAUNCH_CHECK();
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  } catch (...) {
    dev_free(ctx, Y);
    throw;
  }
  dev_free(ctx, Y);
}
