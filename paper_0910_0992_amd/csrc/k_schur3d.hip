// Exact inverse of T = A + mu - D_t on the sites of one p3 parity.  On the even sites this is
// the block M^ee, the even-site solve of temporal preconditioning combined with 3D-Schur
// (Sec. II.B); on both parities it is the left factor of full SW temporal preconditioning on
// the whole lattice (Sec. II.A, App. A, which writes the matrix as a tridiagonal part plus a
// corner term).  The factors are computed in FP64; the sweeps run in FP64, or in FP32 on a
// rounded copy of the factors for the FP32 operator.
//
// In the axial frame every interior time link is the identity, so on a time line
//   (T psi)(t) = B(t) psi(t) - P_- psi(t+1) - P_+ psi(t-1),   B(t) = A(t) + mu,
// with the wrapping hops -P_- P psi(0) in row Lt-1 and -P_+ P^dag psi(Lt-1) in row 0 (P is
// the axial link U_t(Lt-1): the Polyakov loop times the boundary phase).  In the Dirac-Pauli
// basis P_+ keeps spins 0-1 (rows 0-5, spin*3 + colour) and P_- spins 2-3 (rows 6-11).
//
// Split T = T0 + V W^dag: T0 is the open block-tridiagonal part, and the corner term has
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
// Storage per parity: S(t)^-1 for every site as [tile][t][column][row][line of the tile], so the
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

// Block LU of T0 along each line of one parity (one thread per line): S(t)^-1 for t = 0..Lt-1.
// cl: that parity's clover planes (A, chiral blocks) or null for Wilson fermions.
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

// One wavefront per tile of 4 lines of parity slot blockIdx.y; lane = row * 4 + line for
// rows 0-11 (lanes 48-63 only join the barriers).
struct SweepLane {
  int tile, lane, r, l, s, k;
  bool active;
};
__device__ SweepLane sweep_lane() {
  SweepLane q;
  q.tile = blockIdx.x;
  q.k = blockIdx.y;
  q.lane = threadIdx.x;
  q.r = q.lane >> 2;
  q.l = q.lane & 3;
  q.s = q.tile * 4 + q.l;
  q.active = q.lane < 48;
  return q;
}

// Element (row r, site i) of one parity of a spinor field of storage T: half r / 6,
// component r % 6 (FP32 planes are paired).
template <typename T>
__device__ int64_t row_off(int r, int64_t V2, int64_t i) {
  return comp_off<T>(r < 6 ? r : r - 6, 6, V2, i);
}

// Operands of one sweep launch, per parity slot k = blockIdx.y (one or two parities).
template <typename T>
struct Sweep {
  const T* in_up[2] = {};    // forward: eta (null: eta = 0); backward: w
  const T* in_lo[2] = {};
  T* out_up[2] = {};         // forward: w; backward: x (null: not stored)
  T* out_lo[2] = {};
  const T* base_up[2] = {};  // backward: x is stored as base - x when given
  const T* base_lo[2] = {};
  const T* sinv[2] = {};
  const T* kmat[2] = {};     // forward: beta = K q per line when given
  const T* q[2] = {};
  T* qout[2] = {};           // backward: W^dag x per line when given
  const double2* link_t[2] = {};  // FP64 planes [9][V2] of the parity's axial time links
  int unit = -1;             // forward: beta = unit vector `unit` when >= 0
};

// Forward sweep: w(t) = S(t)^-1 (eta(t) + P_+ w(t-1) + c(beta)(t)), storage T (double2:
// FP64; float2: FP32 factors and spinors, FP32 arithmetic).  The corner term is K q when
// kmat is given, the unit vector `unit` when unit >= 0, else absent.
template <typename T>
__global__ __launch_bounds__(64) void k_s3_forward(Sweep<T> a, int64_t V2, Geom g) {
  using R = typename Prec<T>::R;
  __shared__ cx<R> zb[4][12];
  __shared__ cx<R> db[4][12];
  const SweepLane ln = sweep_lane();
  const T* kmat = a.kmat[ln.k];
  const bool corner = kmat != nullptr || a.unit >= 0;
  if (ln.active && corner) {
    cx<R> d = czero<R>();
    if (kmat) {
      const T* kr = kmat + (int64_t)ln.s * 144 + ln.r * 12;
      const T* qs = a.q[ln.k] + (int64_t)ln.s * 12;
#pragma unroll
      for (int c = 0; c < 12; ++c) d += cmul(ld<R, T>(kr + c), ld<R, T>(qs + c));
    } else if (ln.r == a.unit) {
      d = cx<R>{R(1), R(0)};
    }
    db[ln.l][ln.r] = d;
  }
  __syncthreads();
  // this lane's corner term: rows 0-5 at t = 0, rows 6-11 at t = Lt-1
  cx<R> corr = czero<R>();
  if (ln.active && corner) {
    const double2* link_t = a.link_t[ln.k];
    const int64_t ib = p3_idx(g, g.Lt - 1, ln.s);
    const int rr = ln.r < 6 ? ln.r : ln.r - 6;
    const int sp = rr / 3, c3 = rr % 3;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (ln.r < 6) {
        double2 u = link_t[(int64_t)(b * 3 + c3) * V2 + ib];  // (P^dag)_{ab} = conj(P_{ba})
        corr += cmulc(cx<R>{R(u.x), R(u.y)}, db[ln.l][sp * 3 + b]);
      } else {
        double2 u = link_t[(int64_t)(c3 * 3 + b) * V2 + ib];
        corr += cmul(cx<R>{R(u.x), R(u.y)}, db[ln.l][6 + sp * 3 + b]);
      }
    }
  }
  const T* ep = ln.active && a.in_up[ln.k] ? (ln.r < 6 ? a.in_up[ln.k] : a.in_lo[ln.k]) : nullptr;
  T* wp = ln.active ? (ln.r < 6 ? a.out_up[ln.k] : a.out_lo[ln.k]) : nullptr;
  const T* sbase = a.sinv[ln.k] + (int64_t)ln.tile * g.Lt * 576 + ln.lane;
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

// Backward sweep: x(t) = w(t) + S(t)^-1 P_- x(t+1).  out (optional) receives x, or base - x
// when base is given; qout (optional) receives W^dag x = (rows 0-5 of x(Lt-1), rows 6-11
// of x(0)) per line.
template <typename T>
__global__ __launch_bounds__(64) void k_s3_backward(Sweep<T> a, int64_t V2, Geom g) {
  using R = typename Prec<T>::R;
  __shared__ cx<R> xb[4][12];
  const SweepLane ln = sweep_lane();
  const T* wp = ln.active ? (ln.r < 6 ? a.in_up[ln.k] : a.in_lo[ln.k]) : nullptr;
  T* xp = ln.active && a.out_up[ln.k] ? (ln.r < 6 ? a.out_up[ln.k] : a.out_lo[ln.k]) : nullptr;
  const T* bp =
      ln.active && a.base_up[ln.k] ? (ln.r < 6 ? a.base_up[ln.k] : a.base_lo[ln.k]) : nullptr;
  T* qout = a.qout[ln.k];
  const T* sbase = a.sinv[ln.k] + (int64_t)ln.tile * g.Lt * 576 + ln.lane;
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
      if (xp) {
        const int64_t o = row_off<T>(ln.r, V2, i);
        st(xp + o, bp ? ld<R, T>(bp + o) - x : x);
      }
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

// Factorisation and capacitance of T = A + mu - D_t on p3 parity par for this operator, FP64.
void schur3d_setup(tp_op op, int par) {
  if (op->s3_inv[par]) return;
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  if (factor_lds() > ctx->lds_max) TP_THROW(TP_EDIMS, "device LDS too small for the T factorisation");
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
    const double2* cl = op->c ? op->c->a3_d + (int64_t)par * 36 * L.V2 : nullptr;
    hipLaunchKernelGGL(k_s3_factor, dim3(nblk), dim3(kFacThreads), factor_lds(), ctx->stream, cl,
                       L.V2, op->mu, L.g, nlines, sinv, bad);
    LAUNCH_CHECK();
    SpinorF<double2> wf = w.par<double2>(par);
    for (int j = 0; j < 12; ++j) {
      Sweep<double2> f;
      f.out_up[0] = wf.p[0];
      f.out_lo[0] = wf.p[1];
      f.sinv[0] = sinv;
      f.link_t[0] = op->g->u3_d + (int64_t)(3 * 2 + par) * 9 * L.V2;
      f.unit = j;
      hipLaunchKernelGGL(k_s3_forward<double2>, dim3(nlines / 4, 1), dim3(64), 0, ctx->stream, f,
                         L.V2, L.g);
      LAUNCH_CHECK();
      Sweep<double2> b;
      b.in_up[0] = wf.p[0];
      b.in_lo[0] = wf.p[1];
      b.sinv[0] = sinv;
      b.qout[0] = qbuf + (int64_t)j * nlines * 12;
      hipLaunchKernelGGL(k_s3_backward<double2>, dim3(nlines / 4, 1), dim3(64), 0, ctx->stream, b,
                         L.V2, L.g);
      LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_s3_capacitance, dim3(nblk), dim3(kFacThreads),
                       size_t(kFacThreads) * (144 * sizeof(double2) + 12 * sizeof(int)),
                       ctx->stream, qbuf, nlines, kmat, bad);
    LAUNCH_CHECK();
    int hb = 0;
    HIP_CHECK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (hb) TP_THROW(TP_ESINGULAR, "A + mu - D_t factorisation: zero pivot");
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
  op->s3_inv[par] = sinv;
  op->s3_k[par] = kmat;
  op->s3_q[par] = qbuf;  // the first 12 complex per line serve the applies
}

namespace {
// FP32 copies of the factors of parity par for the FP32 operator (rounded from FP64).
void schur3d_setup_f32(tp_op op, int par) {
  schur3d_setup(op, par);
  if (op->s3_inv_f[par]) return;
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
                       op->s3_inv[par], fi, ni);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_round, dim3(unsigned((nk + 255) / 256)), dim3(256), 0, ctx->stream,
                       op->s3_k[par], fk, nk);
    LAUNCH_CHECK();
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  } catch (...) {
    dev_free(ctx, fq);
    dev_free(ctx, fk);
    dev_free(ctx, fi);
    throw;
  }
  op->s3_inv_f[par] = fi;
  op->s3_k_f[par] = fk;
  op->s3_q_f[par] = fq;
}
}  // namespace

bool schur3d_ready(tp_op op, int prec, int par) {
  return prec == TP_F64 ? op->s3_inv[par] != nullptr : op->s3_inv_f[par] != nullptr;
}

void schur3d_free(tp_op op) {
  tp_ctx ctx = op->g->ctx;
  for (int p = 0; p < 2; ++p) {
    dev_free(ctx, op->s3_inv[p]);
    dev_free(ctx, op->s3_k[p]);
    dev_free(ctx, op->s3_q[p]);
    dev_free(ctx, op->s3_inv_f[p]);
    dev_free(ctx, op->s3_k_f[p]);
    dev_free(ctx, op->s3_q_f[p]);
    op->s3_inv[p] = op->s3_k[p] = op->s3_q[p] = nullptr;
    op->s3_inv_f[p] = op->s3_k_f[p] = op->s3_q_f[p] = nullptr;
  }
}

namespace {
// Two solves of T0 per parity (Sherman-Morrison-Woodbury): the first only yields the
// boundary values q = W^dag T0^-1 src, the second adds the corner term K q.  Both parities
// of a call run in the same launches (blockIdx.y).
template <typename T>
void tinv_impl(tp_op op, int par0, int npar, const Field& src, Field& dst, Field& w,
               const Field* base, T* const* sinv, T* const* kmat, T* const* q) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  const dim3 grid(L.Vs2 / 4, npar);
  for (int r = 0; r < src.nr; ++r) {
    Sweep<T> f1, b1, f2, b2;
    for (int k = 0; k < npar; ++k) {
      const int p = par0 + k;
      SpinorF<T> sf = src.view(r).template par<T>(p);
      SpinorF<T> df = dst.view(r).template par<T>(p);
      SpinorF<T> wf = w.view(r).template par<T>(p);
      const double2* link_t = op->g->u3_d + (int64_t)(3 * 2 + p) * 9 * L.V2;
      f1.in_up[k] = f2.in_up[k] = sf.p[0];
      f1.in_lo[k] = f2.in_lo[k] = sf.p[1];
      f1.out_up[k] = f2.out_up[k] = wf.p[0];
      f1.out_lo[k] = f2.out_lo[k] = wf.p[1];
      f1.sinv[k] = f2.sinv[k] = b1.sinv[k] = b2.sinv[k] = sinv[p];
      f1.link_t[k] = f2.link_t[k] = link_t;
      f2.kmat[k] = kmat[p];
      f2.q[k] = q[p];
      b1.in_up[k] = b2.in_up[k] = wf.p[0];
      b1.in_lo[k] = b2.in_lo[k] = wf.p[1];
      b1.qout[k] = q[p];
      b2.out_up[k] = df.p[0];
      b2.out_lo[k] = df.p[1];
      if (base) {
        SpinorF<T> bf = base->view(r).template par<T>(p);
        b2.base_up[k] = bf.p[0];
        b2.base_lo[k] = bf.p[1];
      }
    }
    hipLaunchKernelGGL(k_s3_forward<T>, grid, dim3(64), 0, ctx->stream, f1, L.V2, L.g);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_backward<T>, grid, dim3(64), 0, ctx->stream, b1, L.V2, L.g);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_forward<T>, grid, dim3(64), 0, ctx->stream, f2, L.V2, L.g);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_s3_backward<T>, grid, dim3(64), 0, ctx->stream, b2, L.V2, L.g);
    LAUNCH_CHECK();
  }
}
}  // namespace

void launch_tinv(tp_op op, int par0, int npar, const Field& src, Field& dst, Field& w,
                 const Field* base) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  if (src.prec != dst.prec || src.prec != w.prec || src.prec == TP_F16N ||
      (base && base->prec != src.prec))
    TP_THROW(TP_EINVAL, "the exact T^-1 runs in F64 or F32");
  if (par0 < 0 || npar < 1 || par0 + npar > 2) TP_THROW(TP_EINVAL, "bad parity range");
  // the one-off factorisation stays outside the timed scope of the sweeps
  for (int p = par0; p < par0 + npar; ++p) {
    if (src.prec == TP_F64) schur3d_setup(op, p);
    else schur3d_setup_f32(op, p);
  }
  const double fb = src.prec == TP_F64 ? 16.0 : 8.0;
  const double spin = (7 + (base ? 1 : 0)) * spinor_bytes(src.prec);
  ProfScope ps(ctx, KID_SCHUR3D_MEE, double(L.V2) * (2 * (144 + 72) * fb + spin) * src.nr * npar);
  if (src.prec == TP_F64)
    tinv_impl<double2>(op, par0, npar, src, dst, w, base, op->s3_inv, op->s3_k, op->s3_q);
  else
    tinv_impl<float2>(op, par0, npar, src, dst, w, base, op->s3_inv_f, op->s3_k_f, op->s3_q_f);
}

// dst_e = (M^ee)^-1 src_e for each right-hand side of the batch, in the fields' precision
// (F64, or F32 with the rounded factors).  dst may alias src; w is a work field of the same
// precision and batch size.
void launch_mee_inv(tp_op op, const Field& src, Field& dst, Field& w) {
  launch_tinv(op, 0, 1, src, dst, w);
}
