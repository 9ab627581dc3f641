// Exact inverse of the even p3 block M^ee = A + mu - D_t: the even-site solve of temporal
// preconditioning combined with 3D-Schur (Sec. II.B; App. A writes the block as a
// tridiagonal matrix plus a corner term).  The factors are computed in FP64; the sweeps run
// in FP64, or in FP32 on a rounded copy of the factors for the FP32 operator.
//
// In the axial frame every interior time link is the identity, so on an even time line
//   (M^ee psi)(t) = B(t) psi(t) - P_- psi(t+1) - P_+ psi(t-1),   B(t) = A(t) + mu,
// with the wrapping hops -P_- P psi(0) in row Lt-1 and -P_+ P^dag psi(Lt-1) in row 0 (P is
// the axial link U_t(Lt-1): the Polyakov loop times the boundary phase).  In the Dirac-Pauli
// basis P_+ keeps spins 0-1 (rows 0-5, spin*3 + colour) and P_- spins 2-3 (rows 6-11).
//
// Split M^ee = T0 + V W^dag: T0 is the open block-tridiagonal part, and the corner term has
// rank 12 with W^dag psi = (rows 0-5 of psi(Lt-1), rows 6-11 of psi(0)).  By
// Sherman-Morrison-Woodbury, as the paper does for the temporal matrix (Sec. II.A),
//   x = T0^-1 (eta + c(beta)),   beta = K W^dag T0^-1 eta,   K = (1 + W^dag T0^-1 V)^-1,
// where c(beta) = -V beta adds P^dag beta_0..5 to rows 0-5 of slice 0 and P beta_6..11 to
// rows 6-11 of slice Lt-1.  T0 is factored once by block LU,
//   S(0) = B(0),   S(t) = B(t) - P_+ S(t-1)^-1 P_-,
// and a solve is a forward sweep w(t) = S(t)^-1 (eta(t) + P_+ w(t-1)) and a backward sweep
// x(t) = w(t) + S(t)^-1 P_- x(t+1).  An apply is two such solves: the first only yields
// W^dag T0^-1 eta.  K comes from twelve solves with the unit vectors as beta and eta = 0.
//
// Storage: S(t)^-1 for every even site as [tile][t][column][row][line of the tile], so the
// 48 lanes (row, line) of one wavefront that handle a tile read one column in a single
// contiguous load (768 bytes in FP64).  K is [line][row][column].
#include "tp_internal.h"

namespace {

constexpr int kFacThreads = 32;  // lines per workgroup of the factorisation kernels

// In-place Gauss-Jordan inverse with partial pivoting of the 12x12 matrix of thread th,
// stored in LDS as m[(row * 12 + col) * NT + th]; perm[k * NT + th] records the row swaps.
// Returns false when a pivot is zero or not finite.
template <int NT>
__device__ bool gj_invert(double2* m, int* perm, int th) {
  auto at = [&](int r, int c) -> double2& { return m[(r * 12 + c) * NT + th]; };
  bool ok = true;
#pragma unroll 1
  for (int k = 0; k < 12; ++k) {
    int p = k;
    double best = -1.0;
#pragma unroll 1
    for (int i = k; i < 12; ++i) {
      double2 v = at(i, k);
      double a = v.x * v.x + v.y * v.y;
      if (a > best) { best = a; p = i; }
    }
    if (!(best > 1e-300) || !isfinite(best)) { ok = false; best = 1.0; }
    perm[k * NT + th] = p;
    if (p != k) {
#pragma unroll 1
      for (int j = 0; j < 12; ++j) {
        double2 a = at(k, j);
        at(k, j) = at(p, j);
        at(p, j) = a;
      }
    }
    double2 pv = at(k, k);
    double den = pv.x * pv.x + pv.y * pv.y;
    if (!(den > 1e-300)) den = 1.0;
    cx<double> ip{pv.x / den, -pv.y / den};
    at(k, k) = make_double2(1.0, 0.0);
#pragma unroll 1
    for (int j = 0; j < 12; ++j) {
      double2 a = at(k, j);
      cx<double> r = cmul(cx<double>{a.x, a.y}, ip);
      at(k, j) = make_double2(r.re, r.im);
    }
#pragma unroll 1
    for (int i = 0; i < 12; ++i) {
      if (i == k) continue;
      double2 fv = at(i, k);
      cx<double> f{fv.x, fv.y};
      at(i, k) = make_double2(0.0, 0.0);
#pragma unroll 1
      for (int j = 0; j < 12; ++j) {
        double2 a = at(i, j);
        double2 b = at(k, j);
        cx<double> r = cx<double>{a.x, a.y} - cmul(f, cx<double>{b.x, b.y});
        at(i, j) = make_double2(r.re, r.im);
      }
    }
  }
  // undo the row swaps as column swaps, in reverse order
#pragma unroll 1
  for (int k = 11; k >= 0; --k) {
    int p = perm[k * NT + th];
    if (p == k) continue;
#pragma unroll 1
    for (int i = 0; i < 12; ++i) {
      double2 a = at(i, k);
      at(i, k) = at(i, p);
      at(i, p) = a;
    }
  }
  return ok;
}

// Block LU of T0 along each even line (one thread per line): S(t)^-1 for t = 0..Lt-1.
// cl: even-parity clover planes (A, chiral blocks) or null for Wilson fermions.
__global__ __launch_bounds__(kFacThreads) void k_s3_factor(const double2* __restrict__ cl,
                                                           int64_t V2, double mu, Geom g,
                                                           int nlines,
                                                           double2* __restrict__ sinv,
                                                           int* bad) {
  constexpr int NT = kFacThreads;
  extern __shared__ double2 lds[];
  double2* m = lds;                // [144][NT] S(t), inverted in place
  double2* pv = lds + 144 * NT;    // [36][NT]  rows 0-5, columns 6-11 of S(t-1)^-1
  int* perm = reinterpret_cast<int*>(lds + 180 * NT);  // [12][NT]
  const int th = threadIdx.x;
  const int s = blockIdx.x * NT + th;
  if (s >= nlines) return;  // no barriers below: every thread works on its own line
#pragma unroll 1
  for (int k = 0; k < 36; ++k) pv[k * NT + th] = make_double2(0.0, 0.0);
  bool ok = true;
#pragma unroll 1
  for (int t = 0; t < g.Lt; ++t) {
    const int64_t i = p3_idx(g, t, s);
    // B(t) = A(t) + mu, one column per unit vector
#pragma unroll 1
    for (int j = 0; j < 12; ++j) {
      cx<double> e[12], out[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        e[k] = cx<double>{k == j ? 1.0 : 0.0, 0.0};
        out[k] = czero<double>();
      }
      if (cl) clover_apply<double, double2, int64_t>(cl, V2, i, e, out);
#pragma unroll
      for (int r = 0; r < 12; ++r)
        m[(r * 12 + j) * NT + th] = make_double2(out[r].re + (r == j ? mu : 0.0), out[r].im);
    }
    // S(t) = B(t) - P_+ S(t-1)^-1 P_-
#pragma unroll 1
    for (int r = 0; r < 6; ++r)
#pragma unroll 1
      for (int c = 0; c < 6; ++c) {
        double2 a = m[(r * 12 + 6 + c) * NT + th];
        double2 b = pv[(r * 6 + c) * NT + th];
        m[(r * 12 + 6 + c) * NT + th] = make_double2(a.x - b.x, a.y - b.y);
      }
    ok = gj_invert<NT>(m, perm, th) && ok;
    double2* dst = sinv + ((int64_t)(s >> 2) * g.Lt + t) * 576 + (s & 3);
#pragma unroll 1
    for (int c = 0; c < 12; ++c)
#pragma unroll 1
      for (int r = 0; r < 12; ++r) dst[(c * 12 + r) * 4] = m[(r * 12 + c) * NT + th];
#pragma unroll 1
    for (int r = 0; r < 6; ++r)
#pragma unroll 1
      for (int c = 0; c < 6; ++c) pv[(r * 6 + c) * NT + th] = m[(r * 12 + 6 + c) * NT + th];
  }
  if (!ok) *bad = 1;
}

// K = (1 - Q)^-1 per line, Q[r][j] = qcols[(j * nlines + s) * 12 + r] = -(W^dag T0^-1 V)[r][j].
__global__ __launch_bounds__(kFacThreads) void k_s3_capacitance(const double2* __restrict__ qcols,
                                                                int nlines,
                                                                double2* __restrict__ kmat,
                                                                int* bad) {
  constexpr int NT = kFacThreads;
  extern __shared__ double2 lds[];
  double2* m = lds;
  int* perm = reinterpret_cast<int*>(lds + 144 * NT);
  const int th = threadIdx.x;
  const int s = blockIdx.x * NT + th;
  if (s >= nlines) return;
#pragma unroll 1
  for (int r = 0; r < 12; ++r)
#pragma unroll 1
    for (int j = 0; j < 12; ++j) {
      double2 q = qcols[((int64_t)j * nlines + s) * 12 + r];
      m[(r * 12 + j) * NT + th] = make_double2((r == j ? 1.0 : 0.0) - q.x, -q.y);
    }
  if (!gj_invert<NT>(m, perm, th)) *bad = 1;
#pragma unroll 1
  for (int k = 0; k < 144; ++k) kmat[(int64_t)s * 144 + k] = m[k * NT + th];
}

// One wavefront per tile of 4 even lines; lane = row * 4 + line for rows 0-11 (lanes 48-63
// only join the barriers).
struct SweepLane {
  int tile, lane, r, l, s;
  bool active;
};
__device__ SweepLane sweep_lane() {
  SweepLane q;
  q.tile = blockIdx.x;
  q.lane = threadIdx.x;
  q.r = q.lane >> 2;
  q.l = q.lane & 3;
  q.s = q.tile * 4 + q.l;
  q.active = q.lane < 48;
  return q;
}

// Element (row r, site i) of an even-parity spinor field of storage T: half r / 6,
// component r % 6 (FP32 planes are paired).
template <typename T>
__device__ int64_t row_off(int r, int64_t V2, int64_t i) {
  return comp_off<T>(r < 6 ? r : r - 6, 6, V2, i);
}

// Forward sweep: w(t) = S(t)^-1 (eta(t) + P_+ w(t-1) + c(beta)(t)), storage T (double2:
// FP64; float2: FP32 factors and spinors, FP32 arithmetic).
// eta: even-parity halves, or null for eta = 0.  beta per line: K q when kmat is given,
// the unit vector `unit` when unit >= 0, else no corner term.
// link_t: FP64 planes [9][V2] of the even-parity axial time links (P at t = Lt-1).
template <typename T>
__global__ __launch_bounds__(64) void k_s3_forward(const T* __restrict__ eta_up,
                                                   const T* __restrict__ eta_lo, int64_t V2,
                                                   Geom g, const T* __restrict__ sinv,
                                                   const double2* __restrict__ link_t,
                                                   const T* __restrict__ kmat,
                                                   const T* __restrict__ q, int unit,
                                                   T* __restrict__ w_up, T* __restrict__ w_lo) {
  using R = typename Prec<T>::R;
  __shared__ cx<R> zb[4][12];
  __shared__ cx<R> db[4][12];
  const SweepLane ln = sweep_lane();
  const bool corner = kmat != nullptr || unit >= 0;
  if (ln.active && corner) {
    cx<R> d = czero<R>();
    if (kmat) {
      const T* kr = kmat + (int64_t)ln.s * 144 + ln.r * 12;
      const T* qs = q + (int64_t)ln.s * 12;
#pragma unroll
      for (int c = 0; c < 12; ++c) d += cmul(ld<R, T>(kr + c), ld<R, T>(qs + c));
    } else if (ln.r == unit) {
      d = cx<R>{R(1), R(0)};
    }
    db[ln.l][ln.r] = d;
  }
  __syncthreads();
  // this lane's corner term: rows 0-5 at t = 0, rows 6-11 at t = Lt-1
  cx<R> corr = czero<R>();
  if (ln.active && corner) {
    const int64_t ib = p3_idx(g, g.Lt - 1, ln.s);
    const int rr = ln.r < 6 ? ln.r : ln.r - 6;
    const int sp = rr / 3, a = rr % 3;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (ln.r < 6) {
        double2 u = link_t[(int64_t)(b * 3 + a) * V2 + ib];  // (P^dag)_{ab} = conj(P_{ba})
        corr += cmulc(cx<R>{R(u.x), R(u.y)}, db[ln.l][sp * 3 + b]);
      } else {
        double2 u = link_t[(int64_t)(a * 3 + b) * V2 + ib];
        corr += cmul(cx<R>{R(u.x), R(u.y)}, db[ln.l][6 + sp * 3 + b]);
      }
    }
  }
  const T* ep = ln.active && eta_up ? (ln.r < 6 ? eta_up : eta_lo) : nullptr;
  T* wp = ln.active ? (ln.r < 6 ? w_up : w_lo) : nullptr;
  const T* sbase = sinv + (int64_t)ln.tile * g.Lt * 576 + ln.lane;
  cx<R> wprev = czero<R>();
#pragma unroll 1
  for (int t = 0; t < g.Lt; ++t) {
    const int64_t i = p3_idx(g, t, ln.s);
    if (ln.active) {
      cx<R> z = czero<R>();
      if (ep) z = ld<R, T>(ep + row_off<T>(ln.r, V2, i));
      if (ln.r < 6) {
        z += wprev;
        if (t == 0) z += corr;
      } else if (t == g.Lt - 1) {
        z += corr;
      }
      zb[ln.l][ln.r] = z;
    }
    __syncthreads();
    if (ln.active) {
      const T* sc = sbase + (int64_t)t * 576;
      cx<R> w = czero<R>();
#pragma unroll
      for (int c = 0; c < 12; ++c) w += cmul(ld<R, T>(sc + c * 48), zb[ln.l][c]);
      st(wp + row_off<T>(ln.r, V2, i), w);
      wprev = w;
    }
    __syncthreads();
  }
}

// Backward sweep: x(t) = w(t) + S(t)^-1 P_- x(t+1).  x (optional) receives the solution;
// qout (optional) receives W^dag x = (rows 0-5 of x(Lt-1), rows 6-11 of x(0)) per line.
template <typename T>
__global__ __launch_bounds__(64) void k_s3_backward(const T* __restrict__ w_up,
                                                    const T* __restrict__ w_lo, int64_t V2,
                                                    Geom g, const T* __restrict__ sinv,
                                                    T* __restrict__ x_up, T* __restrict__ x_lo,
                                                    T* __restrict__ qout) {
  using R = typename Prec<T>::R;
  __shared__ cx<R> xb[4][12];
  const SweepLane ln = sweep_lane();
  const T* wp = ln.active ? (ln.r < 6 ? w_up : w_lo) : nullptr;
  T* xp = ln.active && x_up ? (ln.r < 6 ? x_up : x_lo) : nullptr;
  const T* sbase = sinv + (int64_t)ln.tile * g.Lt * 576 + ln.lane;
#pragma unroll 1
  for (int t = g.Lt - 1; t >= 0; --t) {
    const int64_t i = p3_idx(g, t, ln.s);
    cx<R> x = czero<R>();
    if (ln.active) {
      x = ld<R, T>(wp + row_off<T>(ln.r, V2, i));
      if (t < g.Lt - 1) {
        const T* sc = sbase + (int64_t)t * 576;
#pragma unroll
        for (int c = 6; c < 12; ++c) x += cmul(ld<R, T>(sc + c * 48), xb[ln.l][c]);
      }
    }
    __syncthreads();  // every lane has read x(t+1)
    if (ln.active) {
      if (ln.r >= 6) xb[ln.l][ln.r] = x;
      if (xp) st(xp + row_off<T>(ln.r, V2, i), x);
      if (qout && ((t == g.Lt - 1 && ln.r < 6) || (t == 0 && ln.r >= 6)))
        st(qout + (int64_t)ln.s * 12 + ln.r, x);
    }
    __syncthreads();
  }
}

__global__ void k_s3_round(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = make_float2(float(src[k].x), float(src[k].y));
}

size_t factor_lds() { return size_t(kFacThreads) * (180 * sizeof(double2) + 12 * sizeof(int)); }

}  // namespace

// Factorisation and capacitance of M^ee for this operator (even parity), FP64.
void schur3d_setup(tp_op op) {
  if (op->s3_inv) return;
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  if (factor_lds() > ctx->lds_max) TP_THROW(TP_EDIMS, "device LDS too small for the M^ee factorisation");
  const int nlines = L.Vs2;
  const int nblk = (nlines + kFacThreads - 1) / kFacThreads;
  double2* sinv = static_cast<double2*>(dev_alloc(ctx, size_t(L.V2) * 144 * sizeof(double2)));
  double2* kmat = nullptr;
  double2* qbuf = nullptr;
  int* bad = nullptr;
  Field w;
  try {
    kmat = static_cast<double2*>(dev_alloc(ctx, size_t(nlines) * 144 * sizeof(double2)));
    qbuf = static_cast<double2*>(dev_alloc(ctx, size_t(nlines) * 144 * sizeof(double2)));
    bad = static_cast<int*>(dev_alloc(ctx, sizeof(int)));
    w = field_alloc(ctx, TP_F64);
    HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    const double2* cl = op->c ? op->c->a3_d : nullptr;  // even parity first
    hipLaunchKernelGGL(k_s3_factor, dim3(nblk), dim3(kFacThreads), factor_lds(), ctx->stream, cl,
                       L.V2, op->mu, L.g, nlines, sinv, bad);
    LAUNCH_CHECK();
    const double2* link_t = op->g->u3_d + (int64_t)(3 * 2 + 0) * 9 * L.V2;
    SpinorF<double2> wf = w.par<double2>(0);
    for (int j = 0; j < 12; ++j) {
      hipLaunchKernelGGL(k_s3_forward<double2>, dim3(nlines / 4), dim3(64), 0, ctx->stream,
                         (const double2*)nullptr, (const double2*)nullptr, L.V2, L.g,
                         (const double2*)sinv, link_t, (const double2*)nullptr,
                         (const double2*)nullptr, j, wf.p[0], wf.p[1]);
      LAUNCH_CHECK();
      hipLaunchKernelGGL(k_s3_backward<double2>, dim3(nlines / 4), dim3(64), 0, ctx->stream,
                         (const double2*)wf.p[0], (const double2*)wf.p[1], L.V2, L.g,
                         (const double2*)sinv, (double2*)nullptr, (double2*)nullptr,
                         qbuf + (int64_t)j * nlines * 12);
      LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_s3_capacitance, dim3(nblk), dim3(kFacThreads),
                       size_t(kFacThreads) * (144 * sizeof(double2) + 12 * sizeof(int)),
                       ctx->stream, qbuf, nlines, kmat, bad);
    LAUNCH_CHECK();
    int hb = 0;
    HIP_CHECK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (hb) TP_THROW(TP_ESINGULAR, "M^ee factorisation: zero pivot");
  } catch (...) {
    field_free(ctx, w);
    dev_free(ctx, bad);
    dev_free(ctx, qbuf);
    dev_free(ctx, kmat);
    dev_free(ctx, sinv);
    throw;
  }
  field_free(ctx, w);
  dev_free(ctx, bad);
  op->s3_inv = sinv;
  op->s3_k = kmat;
  op->s3_q = qbuf;  // the first 12 complex per line serve the applies
}

// FP32 copies of the factors for the FP32 operator (rounded from the FP64 factorisation).
void schur3d_setup_f32(tp_op op) {
  schur3d_setup(op);
  if (op->s3_inv_f) return;
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  const int64_t ni = L.V2 * 144, nk = int64_t(L.Vs2) * 144;
  float2* fi = static_cast<float2*>(dev_alloc(ctx, size_t(ni) * sizeof(float2)));
  float2* fk = nullptr;
  float2* fq = nullptr;
  try {
    fk = static_cast<float2*>(dev_alloc(ctx, size_t(nk) * sizeof(float2)));
    fq = static_cast<float2*>(dev_alloc(ctx, size_t(L.Vs2) * 12 * sizeof(float2)));
    hipLaunchKernelGGL(k_s3_round, dim3(unsigned((ni + 255) / 256)), dim3(256), 0, ctx->stream,
                       op->s3_inv, fi, ni);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_round, dim3(unsigned((nk + 255) / 256)), dim3(256), 0, ctx->stream,
                       op->s3_k, fk, nk);
    LAUNCH_CHECK();
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  } catch (...) {
    dev_free(ctx, fq);
    dev_free(ctx, fk);
    dev_free(ctx, fi);
    throw;
  }
  op->s3_inv_f = fi;
  op->s3_k_f = fk;
  op->s3_q_f = fq;
}

void schur3d_free(tp_op op) {
  tp_ctx ctx = op->g->ctx;
  dev_free(ctx, op->s3_inv);
  dev_free(ctx, op->s3_k);
  dev_free(ctx, op->s3_q);
  dev_free(ctx, op->s3_inv_f);
  dev_free(ctx, op->s3_k_f);
  dev_free(ctx, op->s3_q_f);
  op->s3_inv = op->s3_k = op->s3_q = nullptr;
  op->s3_inv_f = op->s3_k_f = op->s3_q_f = nullptr;
}

namespace {
template <typename T>
void mee_inv_impl(tp_op op, const Field& src, Field& dst, Field& w, const T* sinv, const T* kmat,
                  T* q) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  const int nlines = L.Vs2;
  const double2* link_t = op->g->u3_d + (int64_t)(3 * 2 + 0) * 9 * L.V2;
  for (int r = 0; r < src.nr; ++r) {
    SpinorF<T> sf = src.view(r).template par<T>(0);
    SpinorF<T> df = dst.view(r).template par<T>(0);
    SpinorF<T> wf = w.view(r).template par<T>(0);
    hipLaunchKernelGGL(k_s3_forward<T>, dim3(nlines / 4), dim3(64), 0, ctx->stream,
                       (const T*)sf.p[0], (const T*)sf.p[1], L.V2, L.g, sinv, link_t,
                       (const T*)nullptr, (const T*)nullptr, -1, wf.p[0], wf.p[1]);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_backward<T>, dim3(nlines / 4), dim3(64), 0, ctx->stream,
                       (const T*)wf.p[0], (const T*)wf.p[1], L.V2, L.g, sinv, (T*)nullptr,
                       (T*)nullptr, q);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_forward<T>, dim3(nlines / 4), dim3(64), 0, ctx->stream,
                       (const T*)sf.p[0], (const T*)sf.p[1], L.V2, L.g, sinv, link_t, kmat,
                       (const T*)q, -1, wf.p[0], wf.p[1]);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_backward<T>, dim3(nlines / 4), dim3(64), 0, ctx->stream,
                       (const T*)wf.p[0], (const T*)wf.p[1], L.V2, L.g, sinv, df.p[0], df.p[1],
                       (T*)nullptr);
    LAUNCH_CHECK();
  }
}
}  // namespace

// dst_e = (M^ee)^-1 src_e for each right-hand side of the batch, in the fields' precision
// (F64, or F32 with the rounded factors).  dst may alias src; w is a work field of the same
// precision and batch size.
void launch_mee_inv(tp_op op, const Field& src, Field& dst, Field& w) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  if (src.prec != dst.prec || src.prec != w.prec || src.prec == TP_F16N)
    TP_THROW(TP_EINVAL, "the exact M^ee inverse runs in F64 or F32");
  // the one-off factorisation stays outside the timed scope of the sweeps
  if (src.prec == TP_F64) schur3d_setup(op);
  else schur3d_setup_f32(op);
  const double fb = src.prec == TP_F64 ? 16.0 : 8.0;
  ProfScope ps(ctx, KID_SCHUR3D_MEE,
               double(L.V2) * (2 * (144 + 72) * fb + 7 * spinor_bytes(src.prec)) * src.nr);
  if (src.prec == TP_F64)
    mee_inv_impl<double2>(op, src, dst, w, op->s3_inv, op->s3_k, op->s3_q);
  else
    mee_inv_impl<float2>(op, src, dst, w, op->s3_inv_f, op->s3_k_f, op->s3_q_f);
}
