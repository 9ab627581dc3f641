// Time-line kernels: the exact inverse of the temporal matrix T (and T^dagger)
// inside C_L, C_R, fused with the spatial hop and the clover term.
//
// Sec. II.A inverts T = mu - U_t(t) delta_{t+1,t'} (with the boundary corner)
// per spatial site by Sherman-Morrison-Woodbury: an open back-substitution
// plus a rank-3 correction built from partial Polyakov loops X(t).  Here the
// same exact inverse is evaluated in the frame rotated by
// W(t) = U_t(t) U_t(t+1) ... U_t(Lt-1) (the product the closed form of X
// contains; W(0) = P, the Polyakov loop with the boundary phase):
//   psi(t) = W(t) r(t)  turns  T psi = eta  into
//   mu r(t) - r(t+1) = xi(t) := W(t)^dag eta(t)   (t < Lt-1),
//   mu r(Lt-1) - P r(0) = xi(Lt-1),
// whose solution is the scalar discounted suffix sum
//   sigma(t) = (xi(t) + sigma(t+1)) / mu,  sigma(Lt) = 0,
//   r(t) = sigma(t) + mu^-(Lt-1-t) delta,  delta = (I - mu^-Lt P)^-1 P sigma(0) / mu.
// T^dagger mirrors it with a prefix sum and delta' = G^dagger rho(Lt-1).
// This is the axial-gauge form of Sec. II.C applied on the fly.  Because the
// recurrence has a scalar coefficient, a line splits into chunks whose
// partial sums combine exactly through LDS (carry = mu^-k times the neighbour
// chunk's head), so every time slice of a line gets its own thread.  The
// closure G = (I - mu^-Lt P)^-1 P / mu is FP64 and applied in FP64.
//
// Workgroup = LPB consecutive lines x NCH chunks of CH consecutive time
// slices; lanes run over lines first, so a wavefront reads LPB consecutive
// sites per time slice.
#pragma once
#include "tp_internal.h"
#include "tp_hop.h"

namespace {

template <typename R>
struct ScanCtx {
  int l, j, LPB, NCH, t0, Lt;
  int s;
  bool active;
  R inv_mu, f;  // 1/mu and mu^-CH
  const R* mupow;  // mu^-k, k = 0..Lt
  const double2* G;  // closure planes [9][Vs2] of this parity
  int64_t gstride;
};

// v: per time slice of the chunk, NV complex values (NV/3 colour vectors) that are
// already rotated by W^dagger.  On return v holds r(t) (still in the rotated frame).
template <typename R, int CH, int NV, bool BWD>
TP_DEV void scan_core(cx<R> (&v)[CH][NV], cx<R>* lds, const ScanCtx<R>& sc) {
  cx<R> X[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    cx<R> acc = czero<R>();
    if constexpr (BWD) {
#pragma unroll
      for (int k = CH - 1; k >= 0; --k) {
        acc = sc.inv_mu * (v[k][c] + acc);
        v[k][c] = acc;
      }
    } else {
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        acc = sc.inv_mu * (v[k][c] + acc);
        v[k][c] = acc;
      }
    }
    X[c] = acc;
  }
  cx<R> C[NV], Z[NV];
  const int me = (sc.j * sc.LPB + sc.l) * 6;
#pragma unroll
  for (int g = 0; g < NV / 6; ++g) {
    R fd = sc.f;
    for (int d = 1; d < sc.NCH; d <<= 1) {
#pragma unroll
      for (int c = 0; c < 6; ++c) lds[me + c] = X[6 * g + c];
      __syncthreads();
      int jj = BWD ? sc.j + d : sc.j - d;
      if (jj >= 0 && jj < sc.NCH) {
        const int o = (jj * sc.LPB + sc.l) * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) X[6 * g + c] += fd * lds[o + c];
      }
      __syncthreads();
      fd = fd * fd;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) lds[me + c] = X[6 * g + c];
    __syncthreads();
    int jc = BWD ? sc.j + 1 : sc.j - 1;
    bool has = jc >= 0 && jc < sc.NCH;
    const int oc = (has ? jc : 0) * sc.LPB * 6 + sc.l * 6;
    const int oz = ((BWD ? 0 : sc.NCH - 1) * sc.LPB + sc.l) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      C[6 * g + c] = has ? lds[oc + c] : czero<R>();
      Z[6 * g + c] = lds[oz + c];
    }
    __syncthreads();
  }
  // closure in FP64: delta = G z (backward) or G^dagger z (forward), per colour vector
  cx<R> D[NV];
  if (sc.active) {
    cx<double> G[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 e = sc.G[(int64_t)k * sc.gstride + sc.s];
      G[k] = cx<double>{e.x, e.y};
    }
#pragma unroll
    for (int q = 0; q < NV / 3; ++q) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cx<double> acc = czero<double>();
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          cx<double> z = cx<double>{double(Z[3 * q + b].re), double(Z[3 * q + b].im)};
          if constexpr (BWD) acc += cmul(G[3 * a + b], z);
          else acc += cmulc(G[3 * b + a], z);
        }
        D[3 * q + a] = cx<R>{R(acc.re), R(acc.im)};
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < NV; ++c) D[c] = czero<R>();
  }
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    int t = sc.t0 + k;
    R ca = BWD ? sc.mupow[CH - k] : sc.mupow[k + 1];
    R cb = BWD ? sc.mupow[sc.Lt - 1 - t] : sc.mupow[t];
#pragma unroll
    for (int c = 0; c < NV; ++c) v[k][c] += ca * C[c] + cb * D[c];
  }
}

// v[3q..3q+2] <- W^dag v (dag = true) or W v, for NV/3 colour vectors.
template <typename R, int NV, bool DAG>
TP_DEV void rotate(const su3<R>& w, cx<R>* v) {
#pragma unroll
  for (int q = 0; q < NV / 3; ++q) {
    cx<R> o[3];
    if constexpr (DAG) mvd(w, v + 3 * q, o);
    else mv(w, v + 3 * q, o);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[3 * q + a] = o[a];
  }
}

template <int N> struct Arr { static constexpr int n = N > 0 ? N : 1; };

// Which halves each mode scans: backward (T^-1) and forward (T^dagger^-1).
//   CL: lower bwd.  CR: upper fwd.  CRCL: lower bwd + upper fwd.
//   TINV: both bwd.  TDINV: both fwd.
template <int MODE> struct ModeT;
template <> struct ModeT<LM_CL> { static constexpr int nb = 6, nf = 0; static constexpr bool up_b = false, lo_b = true, up_f = false, lo_f = false; };
template <> struct ModeT<LM_CR> { static constexpr int nb = 0, nf = 6; static constexpr bool up_b = false, lo_b = false, up_f = true, lo_f = false; };
template <> struct ModeT<LM_CRCL> { static constexpr int nb = 6, nf = 6; static constexpr bool up_b = false, lo_b = true, up_f = true, lo_f = false; };
template <> struct ModeT<LM_TINV> { static constexpr int nb = 12, nf = 0; static constexpr bool up_b = true, lo_b = true, up_f = false, lo_f = false; };
template <> struct ModeT<LM_TDINV> { static constexpr int nb = 0, nf = 12; static constexpr bool up_b = false, lo_b = false, up_f = true, lo_f = true; };

template <typename S>
struct LineArgs {
  SpinorF<S> in, out, nb, self, base;
  LinkF<typename Prec<S>::L> w;     // W(t) of this parity
  LinkF<typename Prec<S>::L> u[2][4];
  const typename Prec<S>::L* clov;  // A/2 blocks of this parity
  const double2* G;
  const typename Prec<S>::R* mupow;
  double inv_mu, f, c_s, c_A, c_self, c_out, c_base;
  Geom g;
  int par, LPB, NCH;
};

template <typename S>
TP_DEV ScanCtx<typename Prec<S>::R> make_ctx(const LineArgs<S>& a, int CH) {
  using R = typename Prec<S>::R;
  ScanCtx<R> sc;
  sc.l = threadIdx.x % a.LPB;
  sc.j = threadIdx.x / a.LPB;
  sc.LPB = a.LPB;
  sc.NCH = a.NCH;
  sc.t0 = sc.j * CH;
  sc.Lt = a.g.Lt;
  sc.s = blockIdx.x * a.LPB + sc.l;
  sc.active = sc.s < a.g.Vs2;
  sc.inv_mu = R(a.inv_mu);
  sc.f = R(a.f);
  sc.mupow = a.mupow;
  sc.G = a.G + (int64_t)a.par * 9 * a.g.Vs2;
  sc.gstride = a.g.Vs2;
  return sc;
}

// Split a full spinor value into the backward/forward scan inputs of MODE.
template <int MODE, typename R>
TP_DEV void split(const cx<R>* v, cx<R>* vb, cx<R>* vf) {
  using M = ModeT<MODE>;
  int ib = 0, jf = 0;
  if constexpr (M::up_b) { for (int c = 0; c < 6; ++c) vb[ib + c] = v[c]; ib += 6; }
  if constexpr (M::lo_b) { for (int c = 0; c < 6; ++c) vb[ib + c] = v[6 + c]; ib += 6; }
  if constexpr (M::up_f) { for (int c = 0; c < 6; ++c) vf[jf + c] = v[c]; jf += 6; }
  if constexpr (M::lo_f) { for (int c = 0; c < 6; ++c) vf[jf + c] = v[6 + c]; jf += 6; }
}
template <int MODE, typename R>
TP_DEV void merge(cx<R>* v, const cx<R>* vb, const cx<R>* vf) {
  using M = ModeT<MODE>;
  int ib = 0, jf = 0;
  if constexpr (M::up_b) { for (int c = 0; c < 6; ++c) v[c] = vb[ib + c]; ib += 6; }
  if constexpr (M::lo_b) { for (int c = 0; c < 6; ++c) v[6 + c] = vb[ib + c]; ib += 6; }
  if constexpr (M::up_f) { for (int c = 0; c < 6; ++c) v[c] = vf[jf + c]; jf += 6; }
  if constexpr (M::lo_f) { for (int c = 0; c < 6; ++c) v[6 + c] = vf[jf + c]; jf += 6; }
}
template <int MODE> TP_DEV constexpr bool passes(int h) {
  using M = ModeT<MODE>;
  return h == 0 ? !(M::up_b || M::up_f) : !(M::lo_b || M::lo_f);
}

// Generic line kernel.
//   STEN: v = c_s D_s(nb) [+ c_A A(self)] [+ c_self self]   else v = in
//   r = MODE(v) on the scanned halves, v on the pass-through halves
//   out = c_out r + c_base base (BASE) or r
//   PASS = false: pass-through halves are not written (in-place or half outputs).
template <typename S, int CH, int MODE, bool STEN, bool CLOV, bool SELF, bool BASE, bool PASS>
__global__ void __launch_bounds__(1024) k_line(LineArgs<S> a) {
  using R = typename Prec<S>::R;
  using Lt = typename Prec<S>::L;
  using M = ModeT<MODE>;
  extern __shared__ char smem_raw[];
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
  ScanCtx<R> sc = make_ctx<S>(a, CH);
  const int s = sc.active ? sc.s : 0;
  cx<R> vb[CH][Arr<M::nb>::n], vf[CH][Arr<M::nf>::n];
  const R cout = R(a.c_out), cbase = R(a.c_base);
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const int64_t i = (int64_t)t * a.g.Vs2 + s;
    cx<R> v[12];
    if (sc.active) {
      if constexpr (STEN) {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = czero<R>();
        hop_space_p3<S, R, Lt>(a.nb, a.u[a.par], a.u[1 - a.par], a.g, a.par, t, s, R(0.5 * a.c_s), v);
        if constexpr (CLOV || SELF) {
          cx<R> x[12];
          load_spinor<S, R>(a.self, i, x);
          if constexpr (CLOV) {
            cx<R> ax[12];
            clover_apply<R, Lt>(a.clov, a.g.V2, i, x, ax);
            R ca = R(a.c_A);
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] += ca * ax[c];
          }
          if constexpr (SELF) {
            R cs = R(a.c_self);
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] += cs * x[c];
          }
        }
      } else {
        if constexpr (M::up_b || M::up_f || (PASS && passes<MODE>(0))) load_half<S, R>(a.in, 0, i, v);
        if constexpr (M::lo_b || M::lo_f || (PASS && passes<MODE>(1))) load_half<S, R>(a.in, 1, i, v + 6);
      }
      // pass-through halves go straight to the output
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (PASS && passes<MODE>(h)) {
          cx<R> o[6];
          if constexpr (BASE) {
            cx<R> bb[6];
            load_half<S, R>(a.base, h, i, bb);
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = cout * v[6 * h + c] + cbase * bb[c];
          } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = cout * v[6 * h + c];
          }
          store_half<S, R>(a.out, h, i, o);
        }
      }
      su3<R> w = load_su3<R, Lt>(a.w, i);
      if constexpr (M::nb > 0) {
        split<MODE, R>(v, vb[k], vf[k]);
        rotate<R, M::nb, true>(w, vb[k]);
      }
      if constexpr (M::nf > 0) {
        if constexpr (M::nb == 0) split<MODE, R>(v, vb[k], vf[k]);
        rotate<R, M::nf, true>(w, vf[k]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < Arr<M::nb>::n; ++c) vb[k][c] = czero<R>();
#pragma unroll
      for (int c = 0; c < Arr<M::nf>::n; ++c) vf[k][c] = czero<R>();
    }
  }
  if constexpr (M::nb > 0) scan_core<R, CH, M::nb, true>(vb, lds, sc);
  if constexpr (M::nf > 0) scan_core<R, CH, M::nf, false>(vf, lds, sc);
  if (!sc.active) return;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const int64_t i = (int64_t)t * a.g.Vs2 + s;
    su3<R> w = load_su3<R, Lt>(a.w, i);
    if constexpr (M::nb > 0) rotate<R, M::nb, false>(w, vb[k]);
    if constexpr (M::nf > 0) rotate<R, M::nf, false>(w, vf[k]);
    cx<R> v[12];
    merge<MODE, R>(v, vb[k], vf[k]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (passes<MODE>(h)) continue;
      cx<R> o[6];
      if constexpr (BASE) {
        cx<R> bb[6];
        load_half<S, R>(a.base, h, i, bb);
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = cout * v[6 * h + c] + cbase * bb[c];
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = cout * v[6 * h + c];
      }
      store_half<S, R>(a.out, h, i, o);
    }
  }
}

// ILU step K2a (even parity): u = D_s^eo a_o / gamma_f (a_o = (aup, psi_o lower)),
//   w = C_R (C_L u + psi_e) = (T^dag^-1 (u_up + psi_up), T^-1 u_lo + psi_lo),
//   y = A w.   Writes y and u.
template <typename S, int CH>
__global__ void __launch_bounds__(1024) k_ilu_k2a(LineArgs<S> a) {
  using R = typename Prec<S>::R;
  using Lt = typename Prec<S>::L;
  extern __shared__ char smem_raw[];
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
  ScanCtx<R> sc = make_ctx<S>(a, CH);
  const int s = sc.active ? sc.s : 0;
  cx<R> vb[CH][6], vf[CH][6], pl[CH][6];
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const int64_t i = (int64_t)t * a.g.Vs2 + s;
    if (sc.active) {
      cx<R> u[12], ps[6];
#pragma unroll
      for (int c = 0; c < 12; ++c) u[c] = czero<R>();
      hop_space_p3<S, R, Lt>(a.nb, a.u[a.par], a.u[1 - a.par], a.g, a.par, t, s, R(0.5 * a.c_s), u);
      store_spinor<S, R>(a.base, i, u);  // u, consumed by K2b
      load_half<S, R>(a.in, 0, i, ps);
      load_half<S, R>(a.in, 1, i, pl[k]);
      su3<R> w = load_su3<R, Lt>(a.w, i);
#pragma unroll
      for (int c = 0; c < 6; ++c) { vf[k][c] = u[c] + ps[c]; vb[k][c] = u[6 + c]; }
      rotate<R, 6, true>(w, vb[k]);
      rotate<R, 6, true>(w, vf[k]);
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) { vb[k][c] = czero<R>(); vf[k][c] = czero<R>(); pl[k][c] = czero<R>(); }
    }
  }
  scan_core<R, CH, 6, true>(vb, lds, sc);
  scan_core<R, CH, 6, false>(vf, lds, sc);
  if (!sc.active) return;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const int64_t i = (int64_t)t * a.g.Vs2 + s;
    su3<R> w = load_su3<R, Lt>(a.w, i);
    rotate<R, 6, false>(w, vb[k]);
    rotate<R, 6, false>(w, vf[k]);
    cx<R> x[12], y[12];
#pragma unroll
    for (int c = 0; c < 6; ++c) { x[c] = vf[k][c]; x[6 + c] = vb[k][c] + pl[k][c]; }
    clover_apply<R, Lt>(a.clov, a.g.V2, i, x, y);
    store_spinor<S, R>(a.out, i, y);
  }
}

// ILU step K2b (even parity): chi_e = psi_e + C_L y = (psi_up + y_up, psi_lo + T^-1 y_lo),
//   n_e = C_R C_L (y - u) = (T^dag^-1 (y_up - u_up), T^-1 (y_lo - u_lo)).
// in = psi_e, self = y, nb = u (same parity), out = chi_e, base = n_e.
template <typename S, int CH>
__global__ void __launch_bounds__(1024) k_ilu_k2b(LineArgs<S> a) {
  using R = typename Prec<S>::R;
  using Lt = typename Prec<S>::L;
  extern __shared__ char smem_raw[];
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
  ScanCtx<R> sc = make_ctx<S>(a, CH);
  const int s = sc.active ? sc.s : 0;
  cx<R> vb[CH][12], vf[CH][6], pl[CH][6];
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const int64_t i = (int64_t)t * a.g.Vs2 + s;
    if (sc.active) {
      cx<R> y[12], u[12], ps[6], o[6];
      load_spinor<S, R>(a.self, i, y);
      load_spinor<S, R>(a.nb, i, u);
      load_half<S, R>(a.in, 0, i, ps);
      load_half<S, R>(a.in, 1, i, pl[k]);
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = ps[c] + y[c];
      store_half<S, R>(a.out, 0, i, o);
      su3<R> w = load_su3<R, Lt>(a.w, i);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        vb[k][c] = y[6 + c];
        vb[k][6 + c] = y[6 + c] - u[6 + c];
        vf[k][c] = y[c] - u[c];
      }
      rotate<R, 12, true>(w, vb[k]);
      rotate<R, 6, true>(w, vf[k]);
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        vb[k][c] = czero<R>(); vb[k][6 + c] = czero<R>(); vf[k][c] = czero<R>(); pl[k][c] = czero<R>();
      }
    }
  }
  scan_core<R, CH, 12, true>(vb, lds, sc);
  scan_core<R, CH, 6, false>(vf, lds, sc);
  if (!sc.active) return;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const int64_t i = (int64_t)t * a.g.Vs2 + s;
    su3<R> w = load_su3<R, Lt>(a.w, i);
    rotate<R, 12, false>(w, vb[k]);
    rotate<R, 6, false>(w, vf[k]);
    cx<R> o[6], n[12];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      o[c] = pl[k][c] + vb[k][c];
      n[c] = vf[k][c];
      n[6 + c] = vb[k][6 + c];
    }
    store_half<S, R>(a.out, 1, i, o);
    store_spinor<S, R>(a.base, i, n);
  }
}

// ---------------------------------------------------------------- launch plumbing
struct Shape {
  int CH, NCH, LPB;
};

// Pick CH (time slices per thread) from `allowed`, NCH = Lt/CH chunks, and LPB lines so
// that LPB * NCH <= max_threads with LPB as close to lpb_target as possible.
Shape pick_shape(int Lt, int lpb_target, int max_threads, std::initializer_list<int> allowed) {
  for (int ch : allowed) {
    if (Lt % ch) continue;
    int nch = Lt / ch;
    if (nch > max_threads) continue;
    int lpb = lpb_target;
    while (lpb > 1 && lpb * nch > max_threads) lpb >>= 1;
    return Shape{ch, nch, lpb};
  }
  TP_THROW(TP_EDIMS, "time extent not supported by the line kernels");
}

template <typename S>
LineArgs<S> base_args(tp_op op, int par) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  LineArgs<S> a{};
  using Lk = typename Prec<S>::L;
  const Lk* w;
  const Lk* u3;
  if constexpr (sizeof(Lk) == 16) { w = (const Lk*)op->g->w_d; u3 = (const Lk*)op->g->u3_d; }
  else { w = (const Lk*)op->g->w_f; u3 = (const Lk*)op->g->u3_f; }
  a.w.p = w + (int64_t)par * 9 * L.V2;
  a.w.stride = L.V2;
  for (int p = 0; p < 2; ++p)
    for (int d = 0; d < 4; ++d) {
      a.u[p][d].p = u3 + (int64_t)(d * 2 + p) * 9 * L.V2;
      a.u[p][d].stride = L.V2;
    }
  a.clov = nullptr;
  if (op->c) {
    if constexpr (sizeof(Lk) == 16) a.clov = (const Lk*)op->c->a3_d + (int64_t)par * 36 * L.V2;
    else a.clov = (const Lk*)op->c->a3_f + (int64_t)par * 36 * L.V2;
  }
  a.G = op->gclos;
  if constexpr (sizeof(Lk) == 16) a.mupow = (const typename Prec<S>::R*)op->mupow_d;
  else a.mupow = (const typename Prec<S>::R*)op->mupow_f;
  a.inv_mu = 1.0 / op->mu;
  a.g = L.g;
  a.par = par;
  return a;
}

template <typename S>
SpinorF<S> pv(const Field* f, int p) {
  if (!f) {
    SpinorF<S> z{};
    return z;
  }
  return f->template par<S>(p);
}

template <typename S>
constexpr int max_threads() { return sizeof(typename Prec<S>::R) == 8 ? 512 : 1024; }
template <typename S>
constexpr int lpb_target() { return sizeof(typename Prec<S>::R) == 8 ? 8 : 16; }

template <typename S, typename K>
void go(tp_op op, K kern, LineArgs<S>& a, Shape sh) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  a.LPB = sh.LPB;
  a.NCH = sh.NCH;
  a.f = pow(op->mu, -double(sh.CH));
  size_t lds = size_t(sh.LPB) * sh.NCH * 6 * sizeof(cx<typename Prec<S>::R>);
  dim3 grid((unsigned)((L.Vs2 + sh.LPB - 1) / sh.LPB));
  hipLaunchKernelGGL(kern, grid, dim3(sh.LPB * sh.NCH), lds, ctx->stream, a);
  LAUNCH_CHECK();
}

// dispatch CH at compile time
#define TP_CH_DISPATCH(CHV, ...)                                   \
  switch (CHV) {                                                   \
    case 1: { constexpr int CH = 1; __VA_ARGS__; break; }          \
    case 2: { constexpr int CH = 2; __VA_ARGS__; break; }          \
    case 4: { constexpr int CH = 4; __VA_ARGS__; break; }          \
    default: TP_THROW(TP_EDIMS, "unsupported chunk length");       \
  }

template <typename S, int MODE>
void line_plain_t(tp_op op, int par, const Field& src, Field& dst, bool pass) {
  LineArgs<S> a = base_args<S>(op, par);
  a.in = pv<S>(&src, par);
  a.out = pv<S>(&dst, par);
  a.c_out = 1.0;
  constexpr bool heavy = ModeT<MODE>::nb + ModeT<MODE>::nf > 6;
  Shape sh = heavy ? pick_shape(op->g->ctx->lat.L[3], lpb_target<S>(), max_threads<S>(), {2, 1, 4})
                   : pick_shape(op->g->ctx->lat.L[3], lpb_target<S>(), max_threads<S>(), {4, 2, 1});
  if (pass) {
    TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, false, false, false, false, true>, a, sh))
  } else {
    TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, false, false, false, false, false>, a, sh))
  }
}

template <typename S>
void line_plain_s(tp_op op, int mode, int par, const Field& src, Field& dst) {
  switch (mode) {
    case LM_CL: line_plain_t<S, LM_CL>(op, par, src, dst, src.data != dst.data); break;
    case LM_CR: line_plain_t<S, LM_CR>(op, par, src, dst, src.data != dst.data); break;
    case LM_CRCL: line_plain_t<S, LM_CRCL>(op, par, src, dst, src.data != dst.data); break;
    case LM_TINV: line_plain_t<S, LM_TINV>(op, par, src, dst, src.data != dst.data); break;
    default: line_plain_t<S, LM_TDINV>(op, par, src, dst, src.data != dst.data); break;
  }
}

template <typename S, int MODE, bool CLOV, bool SELF, bool BASE>
void line_sten_t4(tp_op op, LineArgs<S>& a, Shape sh) {
  TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, true, CLOV, SELF, BASE, true>, a, sh))
}

template <typename S, int MODE>
void line_sten_t(tp_op op, int par, const LineStencilArgs& s, Field& dst) {
  const Lattice& L = op->g->ctx->lat;
  LineArgs<S> a = base_args<S>(op, par);
  SpinorF<S> up = pv<S>(s.nb_up, 1 - par), lo = pv<S>(s.nb_lo, 1 - par);
  a.nb = up;
  a.nb.p[1] = lo.p[1];
  a.nb.nrm[1] = lo.nrm[1];
  a.self = pv<S>(s.self, par);
  a.base = pv<S>(s.base, par);
  a.out = pv<S>(&dst, par);
  a.c_s = s.c_s;
  a.c_A = s.c_A;
  a.c_self = s.c_self;
  a.c_out = s.c_out;
  a.c_base = s.c_base;
  bool clov = s.self && s.c_A != 0.0 && a.clov != nullptr;
  bool self = s.self && s.c_self != 0.0;
  bool base = s.base != nullptr;
  Shape sh = pick_shape(L.L[3], lpb_target<S>(), max_threads<S>(), {2, 1, 4});
  if (clov) {
    if (base) line_sten_t4<S, MODE, true, false, true>(op, a, sh);
    else line_sten_t4<S, MODE, true, false, false>(op, a, sh);
  } else if (self) {
    if (base) line_sten_t4<S, MODE, false, true, true>(op, a, sh);
    else line_sten_t4<S, MODE, false, true, false>(op, a, sh);
  } else {
    if (base) line_sten_t4<S, MODE, false, false, true>(op, a, sh);
    else line_sten_t4<S, MODE, false, false, false>(op, a, sh);
  }
}

template <typename S>
void line_sten_s(tp_op op, int mode, int par, const LineStencilArgs& s, Field& dst) {
  switch (mode) {
    case LM_CL: line_sten_t<S, LM_CL>(op, par, s, dst); break;
    case LM_CR: line_sten_t<S, LM_CR>(op, par, s, dst); break;
    case LM_CRCL: line_sten_t<S, LM_CRCL>(op, par, s, dst); break;
    default: TP_THROW(TP_EINVAL, "stencil line mode");
  }
}

template <typename S>
void k2a_t(tp_op op, const Field& psi, const Field& aup, Field& y, Field& u) {
  const Lattice& L = op->g->ctx->lat;
  LineArgs<S> a = base_args<S>(op, 0);
  SpinorF<S> up = pv<S>(&aup, 1), lo = pv<S>(&psi, 1);
  a.nb = up;
  a.nb.p[1] = lo.p[1];
  a.nb.nrm[1] = lo.nrm[1];
  a.in = pv<S>(&psi, 0);
  a.out = pv<S>(&y, 0);
  a.base = pv<S>(&u, 0);
  a.c_s = 1.0 / op->gf;
  Shape sh = pick_shape(L.L[3], lpb_target<S>(), max_threads<S>(), {2, 1, 4});
  TP_CH_DISPATCH(sh.CH, go<S>(op, k_ilu_k2a<S, CH>, a, sh))
}

template <typename S>
void k2b_t(tp_op op, const Field& psi, const Field& y, const Field& u, Field& chi, Field& n) {
  const Lattice& L = op->g->ctx->lat;
  LineArgs<S> a = base_args<S>(op, 0);
  a.in = pv<S>(&psi, 0);
  a.self = pv<S>(&y, 0);
  a.nb = pv<S>(&u, 0);
  a.out = pv<S>(&chi, 0);
  a.base = pv<S>(&n, 0);
  Shape sh = pick_shape(L.L[3], lpb_target<S>(), max_threads<S>(), {2, 1, 4});
  TP_CH_DISPATCH(sh.CH, go<S>(op, k_ilu_k2b<S, CH>, a, sh))
}


template <typename S>
void k3_t(tp_op op, const Field& psi, const Field& aup, const Field& n, Field& chi) {
  const Lattice& L = op->g->ctx->lat;
  LineArgs<S> a = base_args<S>(op, 1);
  a.nb = pv<S>(&n, 0);
  a.self = pv<S>(&psi, 1);
  SpinorF<S> au = pv<S>(&aup, 1);
  a.self.p[0] = au.p[0];
  a.self.nrm[0] = au.nrm[0];
  a.base = pv<S>(&psi, 1);
  a.out = pv<S>(&chi, 1);
  a.c_s = 1.0 / op->gf;
  a.c_A = 1;
  a.c_out = 1;
  a.c_base = 1;
  Shape sh = pick_shape(L.L[3], lpb_target<S>(), max_threads<S>(), {2, 1, 4});
  if (op->c) line_sten_t4<S, LM_CL, true, false, true>(op, a, sh);
  else line_sten_t4<S, LM_CL, false, false, true>(op, a, sh);
}

}  // namespace

#define TP_CAT2(a, b) a##b
#define TP_CAT(a, b) TP_CAT2(a, b)
void TP_CAT(line_plain_, TP_LINE_SUFFIX)(tp_op op, int mode, int par, const Field& src, Field& dst) {
  line_plain_s<TP_LINE_S>(op, mode, par, src, dst);
}
void TP_CAT(line_half_cr_, TP_LINE_SUFFIX)(tp_op op, const Field& src, Field& dst) {
  line_plain_t<TP_LINE_S, LM_CR>(op, 1, src, dst, false);
}
void TP_CAT(line_sten_, TP_LINE_SUFFIX)(tp_op op, int mode, int par, const LineStencilArgs& s, Field& dst) {
  line_sten_s<TP_LINE_S>(op, mode, par, s, dst);
}
void TP_CAT(ilu_k2a_, TP_LINE_SUFFIX)(tp_op op, const Field& psi, const Field& aup, Field& y, Field& u) {
  k2a_t<TP_LINE_S>(op, psi, aup, y, u);
}
void TP_CAT(ilu_k2b_, TP_LINE_SUFFIX)(tp_op op, const Field& psi, const Field& y, const Field& u, Field& chi, Field& n) {
  k2b_t<TP_LINE_S>(op, psi, y, u, chi, n);
}
void TP_CAT(ilu_k3_, TP_LINE_SUFFIX)(tp_op op, const Field& psi, const Field& aup, const Field& n, Field& chi) {
  k3_t<TP_LINE_S>(op, psi, aup, n, chi);
}
