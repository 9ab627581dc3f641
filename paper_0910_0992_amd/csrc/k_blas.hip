// Level-1 kernels for the Krylov solvers: fused updates with FP64 reductions.
// Work unit = one half spinor (6 complex) of one site, so FP16 fields with a
// scale per half spinor are updated consistently.  The parity and the half are loop
// indices uniform across the grid, so every plane address is a uniform base plus a
// 32-bit site offset.  Reductions are deterministic: a fixed grid writes per-block
// partials, one block sums them in a fixed order.
#include "tp_internal.h"

namespace {

constexpr int kBlock = 256;
// Grid of the level-1 kernels: 4 workgroups per CU; enough loads in flight to stream HBM
// and few partials to sum.
constexpr int kBlasBlocks = 1024;
static_assert(kBlasBlocks <= kRedBlocks, "partials buffer too small");

template <typename S>
struct BlasK {
  SpinorF<S> f[6][2];
  double a[2], b[2], c[2];
  int par0, npar;
  uint32_t V2;
  int nr;                      // right-hand sides: block b works on field b % nr of each batch
  double coef[kMaxRhs][8];     // nr > 1: per right-hand side a, b, c (complex) and a skip flag
  double* partial;             // [nr][blocks per right-hand side][8]
  const double* dcoef;         // single right-hand side: a, b, c read from device memory
};
static_assert(BS_COUNT <= 8 * kMaxRhs, "pinned staging buffer too small for the solver scalars");

TP_DEV void block_reduce(double (&acc)[8], int nred, double* partial, uint32_t blk) {
  __shared__ double sh[kBlock / 64][8];
  for (int k = 0; k < nred; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)nred) {
    double s = 0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
    partial[(int64_t)blk * 8 + threadIdx.x] = s;
  }
}

template <typename R> TP_DEV cx<R> cc(const double* z) { return cx<R>{R(z[0]), R(z[1])}; }

// Streaming access for the reductions that write no field (norms and inner products): each field
// is read once, in vectors larger than the caches, so the loads carry the non-temporal hint.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T> TP_DEV T nt_load(const T* p) {
  if constexpr (sizeof(T) == 16) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p)));
  } else if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p)));
  } else {
    static_assert(sizeof(T) == 4, "4, 8 or 16 bytes");
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p)));
  }
}
// load_half of tp_device.h with non-temporal accesses (same values).
template <typename S, typename R = typename Prec<S>::R>
TP_DEV void nt_load_half(const SpinorF<S>& f, int h, uint32_t i, cx<R>* v) {
  const S* b = f.p[h];
  if constexpr (Prec<S>::half) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const Half2x2 e = nt_load(reinterpret_cast<const Half2x2*>(at(b + (int64_t)(2 * q) * f.stride, 2 * i)));
      const float2 fa = __half22float2(e.a), fb = __half22float2(e.b);
      v[2 * q] = {fa.x, fa.y};
      v[2 * q + 1] = {fb.x, fb.y};
    }
    const R sc = nt_load(at(f.nrm[h], i));
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = sc * v[c];
  } else if constexpr (paired<S>()) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float4 e = nt_load(reinterpret_cast<const float4*>(at(b + (int64_t)(2 * q) * f.stride, 2 * i)));
      v[2 * q] = {e.x, e.y};
      v[2 * q + 1] = {e.z, e.w};
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const S e = nt_load(at(b + (int64_t)c * f.stride, i));
      v[c] = {R(e.x), R(e.y)};
    }
  }
}




// acc[0..1] += <x, y> = sum conj(x) y over one half spinor, in FP64.
template <typename R>
TP_DEV void dot_acc(const cx<R>* x, const cx<R>* y, double* acc) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    acc[0] += double(x[c].re) * double(y[c].re) + double(x[c].im) * double(y[c].im);
    acc[1] += double(x[c].re) * double(y[c].im) - double(x[c].im) * double(y[c].re);
  }
}

template <typename S, int OP>
__global__ void __launch_bounds__(kBlock) k_blas(BlasK<S> k) {
  using R = typename Prec<S>::R;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const uint32_t nr = uint32_t(k.nr), rhs = blockIdx.x % nr, blk = blockIdx.x / nr, nblk = gridDim.x / nr;
  // coefficients from the kernel arguments (one set, or one per right-hand side) or from
  // device memory; separate branches, so that no pointer mixes the two address spaces (a
  // pointer that may point into the by-value arguments makes the compiler copy them to
  // scratch in every thread)
  cx<R> A, B, C;
  if (k.dcoef) {
    A = cc<R>(k.dcoef);
    B = cc<R>(k.dcoef + 2);
    C = cc<R>(k.dcoef + 4);
  } else if (nr > 1) {
    A = cc<R>(k.coef[rhs]);
    B = cc<R>(k.coef[rhs] + 2);
    C = cc<R>(k.coef[rhs] + 4);
  } else {
    A = cc<R>(k.a);
    B = cc<R>(k.b);
    C = cc<R>(k.c);
  }
  // a skipped right-hand side is left untouched
  const int npar = (nr > 1 && k.coef[rhs][6] != 0.0) ? 0 : k.npar;
  for (int q = 0; q < npar; ++q)
#pragma unroll
  for (int h = 0; h < 2; ++h)
  for (uint32_t i = blk * blockDim.x + threadIdx.x; i < k.V2; i += nblk * blockDim.x) {
    const int p = k.par0 + q;
    const SpinorF<S> f0 = rhs_view(k.f[0][p], rhs), f1 = rhs_view(k.f[1][p], rhs), f2 = rhs_view(k.f[2][p], rhs);
    const SpinorF<S> f3 = rhs_view(k.f[3][p], rhs), f4 = rhs_view(k.f[4][p], rhs), f5 = rhs_view(k.f[5][p], rhs);
    cx<R> x[6], y[6], z[6], w[6], v[6];
    if constexpr (OP == B_ZERO) {
      for (int c = 0; c < 6; ++c) y[c] = czero<R>();
      store_half<S, R>(f1, h, i, y);
    } else if constexpr (OP == B_COPY) {
      load_half<S, R>(f0, h, i, x);
      store_half<S, R>(f1, h, i, x);
    } else if constexpr (OP == B_AXPY) {
      load_half<S, R>(f0, h, i, x);
      load_half<S, R>(f1, h, i, y);
      for (int c = 0; c < 6; ++c) y[c] += cmul(A, x[c]);
      store_half<S, R>(f1, h, i, y);
    } else if constexpr (OP == B_XPAY) {
      load_half<S, R>(f0, h, i, x);
      load_half<S, R>(f1, h, i, y);
      for (int c = 0; c < 6; ++c) y[c] = x[c] + cmul(A, y[c]);
      store_half<S, R>(f1, h, i, y);
    } else if constexpr (OP == B_NORM2) {
      nt_load_half<S, R>(f0, h, i, x);
      for (int c = 0; c < 6; ++c) acc[0] += double(norm2(x[c]));
    } else if constexpr (OP == B_DOT || OP == B_DOT_NORM) {
      nt_load_half<S, R>(f0, h, i, x);
      nt_load_half<S, R>(f1, h, i, y);
      for (int c = 0; c < 6; ++c) {
        acc[0] += double(x[c].re) * double(y[c].re) + double(x[c].im) * double(y[c].im);
        acc[1] += double(x[c].re) * double(y[c].im) - double(x[c].im) * double(y[c].re);
        if constexpr (OP == B_DOT_NORM) acc[2] += double(norm2(y[c]));
      }
    } else if constexpr (OP == B_CAXPY_NORM) {
      load_half<S, R>(f0, h, i, x);
      load_half<S, R>(f1, h, i, y);
      for (int c = 0; c < 6; ++c) {
        y[c] += cmul(A, x[c]);
        acc[0] += double(norm2(y[c]));
      }
      store_half<S, R>(f1, h, i, y);
    } else if constexpr (OP == B_AXPYZ_NORM) {
      load_half<S, R>(f0, h, i, x);
      load_half<S, R>(f1, h, i, y);
      for (int c = 0; c < 6; ++c) {
        y[c] += cmul(A, x[c]);
        acc[0] += double(norm2(y[c]));
      }
      store_half<S, R>(f2, h, i, y);
    } else if constexpr (OP == B_DOT4_TS) {
      nt_load_half<S, R>(f0, h, i, x);  // t
      nt_load_half<S, R>(f1, h, i, y);  // s
      nt_load_half<S, R>(f2, h, i, z);  // rhat
      dot_acc(x, y, acc);
      for (int c = 0; c < 6; ++c) acc[2] += double(norm2(x[c]));
      dot_acc(z, y, acc + 3);
      dot_acc(z, x, acc + 5);
    } else if constexpr (OP == B_BICG_FUSED) {
      // f0 = x, f1 = p, f2 = s, f3 = t, f4 = v, f5 = r (out); A = alpha, B = omega, C = beta
      load_half<S, R>(f0, h, i, x);
      load_half<S, R>(f1, h, i, y);
      load_half<S, R>(f2, h, i, z);
      load_half<S, R>(f3, h, i, w);
      load_half<S, R>(f4, h, i, v);
      const cx<R> BC = cmul(B, C);
      for (int c = 0; c < 6; ++c) {
        x[c] += cmul(A, y[c]) + cmul(B, z[c]);
        z[c] = z[c] - cmul(B, w[c]);                  // r = s - omega t
        y[c] = z[c] + cmul(C, y[c]) - cmul(BC, v[c]);  // p = r + beta (p - omega v)
        acc[0] += double(norm2(z[c]));
      }
      store_half<S, R>(f0, h, i, x);
      store_half<S, R>(f5, h, i, z);
      store_half<S, R>(f1, h, i, y);
    } else if constexpr (OP == B_G5) {
      load_half<S, R>(f0, h, i, x);
      for (int c = 0; c < 6; ++c) x[c] = -x[c];
      store_half<S, R>(f1, 1 - h, i, x);
    }
  }
  constexpr int nred =
      (OP == B_NORM2 || OP == B_CAXPY_NORM || OP == B_AXPYZ_NORM || OP == B_BICG_FUSED) ? 1
      : (OP == B_DOT) ? 2
      : (OP == B_DOT_NORM) ? 3
      : (OP == B_DOT4_TS) ? 7 : 0;
  if constexpr (nred > 0) block_reduce(acc, nred, k.partial + (int64_t)rhs * nblk * 8, blk);
}

// y (precision SY) = x (precision SX) when MODE = 0, y += x when MODE = 1, y = z + x (z in
// precision SY) when MODE = 2.
template <typename SX, typename SY, int MODE>
__global__ void __launch_bounds__(kBlock) k_convert(SpinorF<SX> x0, SpinorF<SX> x1, SpinorF<SY> y0,
                                                    SpinorF<SY> y1, SpinorF<SY> z0, SpinorF<SY> z1,
                                                    int par0, int npar, int64_t V2) {
  using RX = typename Prec<SX>::R;
  using RY = typename Prec<SY>::R;
  for (int q = 0; q < npar; ++q)
#pragma unroll
  for (int h = 0; h < 2; ++h)
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < uint32_t(V2); i += gridDim.x * blockDim.x) {
    const int p = par0 + q;
    cx<RX> a[6];
    load_half<SX, RX>(p ? x1 : x0, h, i, a);
    cx<RY> b[6];
    if constexpr (MODE == 1) load_half<SY, RY>(p ? y1 : y0, h, i, b);
    if constexpr (MODE == 2) load_half<SY, RY>(p ? z1 : z0, h, i, b);
    for (int c = 0; c < 6; ++c) {
      cx<RY> t = cx<RY>{RY(a[c].re), RY(a[c].im)};
      b[c] = MODE ? b[c] + t : t;
    }
    store_half<SY, RY>(p ? y1 : y0, h, i, b);
  }
}

// BiCGStab's scalar steps on the device (single right-hand side), from the reduced values v
// of the op just finished; the same formulas as the host-side solver.
TP_DEV void bicg_post(int post, const double* v, double* st) {
  if (post == BP_RHO) {
    st[BS_RHO] = v[0];
    st[BS_RHO + 1] = v[1];
  } else if (post == BP_ALPHA) {  // v = <rhat, v>
    const double den = v[0] * v[0] + v[1] * v[1];
    const double rr = st[BS_RHO], ri = st[BS_RHO + 1];
    const double ar = (rr * v[0] + ri * v[1]) / den, ai = (ri * v[0] - rr * v[1]) / den;
    st[BS_ALPHA] = ar;
    st[BS_ALPHA + 1] = ai;
    st[BS_AXPY] = -ar;
    st[BS_AXPY + 1] = -ai;
    for (int q = 2; q < 6; ++q) st[BS_AXPY + q] = 0.0;
  } else if (post == BP_S2) {
    st[BS_S2] = v[0];
  } else if (post == BP_OMEGA) {  // v = <t, s>, |t|^2, <rhat, s>, <rhat, t>
    const double om_r = v[0] / v[2], om_i = v[1] / v[2];
    const double rn_r = v[3] - (om_r * v[5] - om_i * v[6]);
    const double rn_i = v[4] - (om_r * v[6] + om_i * v[5]);
    const double rho_r = st[BS_RHO], rho_i = st[BS_RHO + 1];
    const double al_r = st[BS_ALPHA], al_i = st[BS_ALPHA + 1];
    const double rr = rho_r * rho_r + rho_i * rho_i, oo = om_r * om_r + om_i * om_i;
    const double q_r = (rn_r * rho_r + rn_i * rho_i) / rr, q_i = (rn_i * rho_r - rn_r * rho_i) / rr;
    const double w_r = (al_r * om_r + al_i * om_i) / oo, w_i = (al_i * om_r - al_r * om_i) / oo;
    const double be_r = q_r * w_r - q_i * w_i, be_i = q_r * w_i + q_i * w_r;
    st[BS_BREAK] = (v[2] == 0.0 || !isfinite(oo) || oo == 0.0 || rr == 0.0) ? 1.0 : 0.0;
    st[BS_OMEGA] = om_r;
    st[BS_OMEGA + 1] = om_i;
    st[BS_BETA] = be_r;
    st[BS_BETA + 1] = be_i;
    st[BS_FUSED] = al_r;
    st[BS_FUSED + 1] = al_i;
    st[BS_FUSED + 2] = om_r;
    st[BS_FUSED + 3] = om_i;
    st[BS_FUSED + 4] = be_r;
    st[BS_FUSED + 5] = be_i;
    st[BS_RHO] = rn_r;
    st[BS_RHO + 1] = rn_i;
  } else if (post == BP_R2) {
    st[BS_R2] = v[0];
  }
}

// Block r sums the `nblocks` partials of right-hand side r into result[r][0..nred); with
// `post`, block 0 then updates the solver scalars st.
__global__ void k_finish(const double* partial, int nblocks, int nred, double* result, int post,
                         double* st) {
  __shared__ double sh[kBlock];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  partial += (int64_t)blockIdx.x * nblocks * 8;
  result += (int64_t)blockIdx.x * 8;
  for (int k = 0; k < nred; ++k) {
    double s = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(int64_t)b * 8 + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) result[k] = v[k] = sh[0];
    __syncthreads();
  }
  if (post != BP_NONE && blockIdx.x == 0 && threadIdx.x == 0) bicg_post(post, v, st);
}

template <typename S>
SpinorF<S> fv(const Field* f, int p) {
  if (!f) {
    SpinorF<S> z{};
    return z;
  }
  return f->template par<S>(p);
}

// Coefficients of one call: the same for every right-hand side (per == null) or one set per
// right-hand side, with optional skip flags.
struct BlasCall {
  BlasArgs k;
  int nr;
  const BlasArgs* per;
  const bool* skip;
  const double* dcoef;
};

template <typename S, int OP>
int blas_go(tp_ctx ctx, int par0, int npar, const Field* const* fs, const BlasCall& c) {
  BlasK<S> a;
  for (int q = 0; q < 6; ++q)
    for (int p = 0; p < 2; ++p) a.f[q][p] = fv<S>(fs[q], p);
  for (int r = 0; r < 2; ++r) { a.a[r] = c.k.a[r]; a.b[r] = c.k.b[r]; a.c[r] = c.k.c[r]; }
  a.nr = c.nr;
  for (int q = 0; q < kMaxRhs; ++q)
    for (int r = 0; r < 8; ++r) a.coef[q][r] = 0.0;
  if (c.nr > 1) {
    for (int q = 0; q < c.nr; ++q) {
      const BlasArgs& k = c.per ? c.per[q] : c.k;
      a.coef[q][0] = k.a[0]; a.coef[q][1] = k.a[1];
      a.coef[q][2] = k.b[0]; a.coef[q][3] = k.b[1];
      a.coef[q][4] = k.c[0]; a.coef[q][5] = k.c[1];
      a.coef[q][6] = (c.skip && c.skip[q]) ? 1.0 : 0.0;
    }
  }
  a.par0 = par0;
  a.npar = npar;
  a.V2 = uint32_t(ctx->lat.V2);
  a.partial = ctx->red_partial;
  a.dcoef = c.dcoef;
  // blocks per right-hand side: the whole grid stays near kBlasBlocks
  int64_t nb = ((int64_t)npar * 2 * a.V2 + kBlock - 1) / kBlock;
  // measured at 32^3x256: FP32 fields stream fastest with 2 workgroups per CU (5.4 against
  // 5.0 TB/s at 4), FP16 ones with 4 (4.5 against 4.4 at 2 or 16)
  const int blocks = std::is_same<S, float2>::value ? kBlasBlocks / 2 : kBlasBlocks;
  nb = std::min<int64_t>(nb, std::max(1, blocks / c.nr));
  hipLaunchKernelGGL((k_blas<S, OP>), dim3((unsigned)(nb * c.nr)), dim3(kBlock), 0, ctx->stream, a);
  LAUNCH_CHECK();
  return int(nb);
}

template <int OP>
int blas_prec(tp_ctx ctx, int prec, int par0, int npar, const Field* const* fs, const BlasCall& c) {
  switch (prec) {
    case TP_F64: return blas_go<double2, OP>(ctx, par0, npar, fs, c);
    case TP_F32: return blas_go<float2, OP>(ctx, par0, npar, fs, c);
    default: return blas_go<__half2, OP>(ctx, par0, npar, fs, c);
  }
}

template <typename SX, typename SY, int MODE>
void conv_go(tp_ctx ctx, int par0, int npar, const Field& x, const Field& y, const Field* z) {
  int64_t V2 = ctx->lat.V2;
  int64_t nb = (V2 + kBlock - 1) / kBlock;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL((k_convert<SX, SY, MODE>), dim3((unsigned)nb), dim3(kBlock), 0, ctx->stream,
                     x.template par<SX>(0), x.template par<SX>(1), y.template par<SY>(0),
                     y.template par<SY>(1), fv<SY>(z, 0), fv<SY>(z, 1), par0, npar, V2);
  LAUNCH_CHECK();
}

template <typename SX, int MODE>
void conv_y(tp_ctx ctx, int par0, int npar, const Field& x, const Field& y, const Field* z) {
  switch (y.prec) {
    case TP_F64: conv_go<SX, double2, MODE>(ctx, par0, npar, x, y, z); break;
    case TP_F32: conv_go<SX, float2, MODE>(ctx, par0, npar, x, y, z); break;
    default: conv_go<SX, __half2, MODE>(ctx, par0, npar, x, y, z); break;
  }
}

template <int MODE>
void conv(tp_ctx ctx, int par0, int npar, const Field& x, const Field& y, const Field* z = nullptr) {
  switch (x.prec) {
    case TP_F64: conv_y<double2, MODE>(ctx, par0, npar, x, y, z); break;
    case TP_F32: conv_y<float2, MODE>(ctx, par0, npar, x, y, z); break;
    default: conv_y<__half2, MODE>(ctx, par0, npar, x, y, z); break;
  }
}

}  // namespace

void blas(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fl,
          BlasArgs k, double* red_out) {
  blas_multi(ctx, op, par0, npar, fl, nullptr, nullptr, red_out, k);
}

namespace {
void blas_impl(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fl,
               const BlasArgs* per, const bool* skip, double* red_out, BlasArgs k, const double* dcoef,
               int post, bool dev);
}  // namespace

void blas_multi(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fl,
                const BlasArgs* per, const bool* skip, double* red_out, BlasArgs k) {
  blas_impl(ctx, op, par0, npar, fl, per, skip, red_out, k, nullptr, BP_NONE, false);
}

void blas_dev(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fl,
              const double* dcoef, int post) {
  blas_impl(ctx, op, par0, npar, fl, nullptr, nullptr, nullptr, BlasArgs{}, dcoef, post, true);
}

void bicg_state(tp_ctx ctx, double* out) {
  HIP_CHECK(hipMemcpyAsync(ctx->red_host, ctx->bicg, sizeof(double) * BS_COUNT, hipMemcpyDeviceToHost,
                           ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  prof_flush(ctx);
  for (int q = 0; q < BS_COUNT; ++q) out[q] = ctx->red_host[q];
}

namespace {
void blas_impl(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fl,
               const BlasArgs* per, const bool* skip, double* red_out, BlasArgs k, const double* dcoef,
               int post, bool dev) {
  const Field* fs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int nr = 0;
  {
    int q = 0;
    for (const Field* f : fl) {
      fs[q++] = f;
      if (f) {
        if (nr && f->nr != nr) TP_THROW(TP_EINVAL, "blas: fields of different batch sizes");
        nr = f->nr;
      }
    }
  }
  if (nr < 1 || nr > kMaxRhs) TP_THROW(TP_EINVAL, "blas: batch size");
  if (dev && nr != 1) TP_THROW(TP_EINVAL, "blas: device-side coefficients take single fields");
  const BlasCall call{k, nr, per, skip, dcoef};
  const Field* x = fs[0];
  const Field* y = fs[1];
  int prec = x ? x->prec : y->prec;
  // bytes per site and field: 12 components, plus the two FP32 half-spinor scales of F16N
  double S = spinor_bytes(prec);
  double n = double(npar) * ctx->lat.V2 * nr;
  if (op == B_CONVERT || op == B_MIXED_ACC) {
    if (nr != 1) TP_THROW(TP_EINVAL, "blas: conversions take single fields");
    ProfScope ps(ctx, KID_BLAS_OTHER, n * (S + spinor_bytes(y->prec) * (op == B_MIXED_ACC ? 2 : 1)));
    if (op == B_CONVERT) conv<0>(ctx, par0, npar, *x, *y);
    else conv<1>(ctx, par0, npar, *x, *y);
    return;
  }
  if (op == B_MIXED_ADD) {
    // fields x (any precision), z and y (same precision): y = z + x
    const Field* z = fs[1];
    const Field* out = fs[2];
    if (nr != 1) TP_THROW(TP_EINVAL, "blas: conversions take single fields");
    if (!x || !z || !out || z->prec != out->prec) TP_THROW(TP_EINVAL, "blas: mixed add fields");
    ProfScope ps(ctx, KID_BLAS_OTHER, n * (S + spinor_bytes(out->prec) * 2));
    conv<2>(ctx, par0, npar, *x, *out, z);
    return;
  }
  int nb = 0, nred = 0;
  {
    double passes = 2;
    switch (op) {
      case B_AXPY: case B_XPAY: case B_DOT_NORM: case B_CAXPY_NORM: case B_AXPYZ_NORM: passes = 3; break;
      case B_DOT4_TS: passes = 3; break;
      case B_BICG_FUSED: passes = 8; break;
      case B_NORM2: passes = 1; break;
      case B_ZERO: passes = 1; break;
      default: break;
    }
    const int kid = op == B_DOT ? KID_BLAS_DOT
                    : op == B_AXPYZ_NORM ? KID_BLAS_AXPYZ
                    : op == B_DOT4_TS ? KID_BLAS_DOT4
                    : op == B_BICG_FUSED ? KID_BLAS_FUSED : KID_BLAS_OTHER;
    ProfScope ps(ctx, kid, n * S * passes);
    switch (op) {
      case B_ZERO: nb = blas_prec<B_ZERO>(ctx, prec, par0, npar, fs, call); break;
      case B_COPY: nb = blas_prec<B_COPY>(ctx, prec, par0, npar, fs, call); break;
      case B_AXPY: nb = blas_prec<B_AXPY>(ctx, prec, par0, npar, fs, call); break;
      case B_XPAY: nb = blas_prec<B_XPAY>(ctx, prec, par0, npar, fs, call); break;
      case B_NORM2: nb = blas_prec<B_NORM2>(ctx, prec, par0, npar, fs, call); nred = 1; break;
      case B_DOT: nb = blas_prec<B_DOT>(ctx, prec, par0, npar, fs, call); nred = 2; break;
      case B_DOT_NORM: nb = blas_prec<B_DOT_NORM>(ctx, prec, par0, npar, fs, call); nred = 3; break;
      case B_CAXPY_NORM: nb = blas_prec<B_CAXPY_NORM>(ctx, prec, par0, npar, fs, call); nred = 1; break;
      case B_AXPYZ_NORM: nb = blas_prec<B_AXPYZ_NORM>(ctx, prec, par0, npar, fs, call); nred = 1; break;
      case B_DOT4_TS: nb = blas_prec<B_DOT4_TS>(ctx, prec, par0, npar, fs, call); nred = 7; break;
      case B_BICG_FUSED: nb = blas_prec<B_BICG_FUSED>(ctx, prec, par0, npar, fs, call); nred = 1; break;
      case B_G5: nb = blas_prec<B_G5>(ctx, prec, par0, npar, fs, call); break;
      default: TP_THROW(TP_EINVAL, "blas op");
    }
  }
  if (nred > 0) {
    {
      ProfScope ps(ctx, KID_REDUCE, double(nb) * nr * 8 * 8);
      hipLaunchKernelGGL(k_finish, dim3(nr), dim3(kBlock), 0, ctx->stream, ctx->red_partial, nb, nred,
                         ctx->red_result, post, ctx->bicg);
      LAUNCH_CHECK();
    }
    if (dev) return;
    HIP_CHECK(hipMemcpyAsync(ctx->red_host, ctx->red_result, sizeof(double) * 8 * nr,
                             hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    prof_flush(ctx);
    for (int q = 0; q < 8 * (nr - 1) + nred; ++q) red_out[q] = ctx->red_host[q];
  }
}
}  // namespace

// Sum of the first `nblocks` partials written by a norm-producing site kernel.
double finish_norm(tp_ctx ctx, int nblocks) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, ctx->stream, ctx->red_partial, nblocks, 1,
                     ctx->red_result, int(BP_NONE), ctx->bicg);
  LAUNCH_CHECK();
  HIP_CHECK(hipMemcpyAsync(ctx->red_host, ctx->red_result, sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  prof_flush(ctx);
  return ctx->red_host[0];
}
