// Site-parallel stencil kernels: the fermion matrix and its pieces on the p3
// ("line") layout, the 4D even-odd Schur pieces on the p4 layout, and the
// link-gradient kernel.  One thread per output site; spin projection in the
// Dirac-Pauli basis (only two colour matvecs per hop direction).
#include <type_traits>

#include "tp_internal.h"
#include "tp_hop.h"

namespace {

constexpr int kBlock = 256;

// Order in which the blocks of a one-block-per-chunk launch visit the tiles.  Workgroups go to
// the 8 XCDs (each with its own L2) in turn, so block b runs on XCD b % 8.  A tile of 4 lines
// spans Q = Lt / 64 blocks; XCD x takes the time range x % Q of the tiles in part x / Q of a
// z-blocked tile sequence (x fastest, then z inside blocks of BZ planes, then y, then the z
// block), so that the tiles holding a site's x, y and z neighbours were visited by the same
// XCD 1, TX*BZ and TX blocks earlier.  off = identity.
struct TileOrder {
  uint32_t Q, TX, Ly, BZ, per_part;
  int on;
};

TP_DEV uint32_t ordered_block(const TileOrder& o, uint32_t b) {
  const uint32_t x = b & 7u, n = b >> 3;
  const uint32_t q = (x / o.Q) * o.per_part + n;
  const uint32_t tx = q % o.TX;
  uint32_t r = q / o.TX;
  const uint32_t zi = r % o.BZ;
  r /= o.BZ;
  const uint32_t y = r % o.Ly, zb = r / o.Ly;
  const uint32_t tile = tx + o.TX * (y + o.Ly * (zb * o.BZ + zi));
  return tile * o.Q + x % o.Q;
}

// The XCD-aware order where the launch shape allows it (one block per chunk of 256 sites,
// whole tiles per block group, tiles inside x rows), else off.
TileOrder tile_order(const Lattice& L, int64_t nblocks, int nr, bool half) {
  TileOrder o{1, 1, 1, 1, 0, 0};
  const Geom& g = L.g;
  if (nr != 1 || int64_t(nblocks) * kBlock != g.V2) return o;
  if (g.Lt % 64 || (8 % (g.Lt / 64)) || g.Lxh % kTile) return o;
  const uint32_t Q = uint32_t(g.Lt / 64), tiles = uint32_t(g.Vs2 / kTile);
  if ((uint64_t(tiles) * Q) % 8) return o;
  o.Q = Q;
  o.TX = uint32_t(g.Lxh / kTile);
  o.Ly = uint32_t(g.Ly);
  o.BZ = g.Lz % 8 == 0 ? 8u : g.Lz % 4 == 0 ? 4u : g.Lz % 2 == 0 ? 2u : 1u;
  o.per_part = tiles * Q / 8;
  o.on = 1;
  // measured: with FP16 storage and four blocks per tile (256-slice lines) the identity
  // order was 2.7% faster; everywhere else this order was 4-19% faster
  o.on = !(half && Q >= 4);
  return o;
}

template <typename S>
struct SiteArgsP3 {
  // for output parity p: self[p] (parity p operand of mu, A, D_t), nb[p] (parity 1-p
  // operand of D_s), in2[p]
  SpinorF<S> self[2], nb[2], dst[2], in2[2];
  LinkF<typename Prec<S>::L> u[2][4];  // [parity][direction]
  const typename Prec<S>::L* clov[2];
  double c_mu, c_A, c_t, c_s, c_in;
  Geom g;
  int par;  // output parity of this launch
  int nr;   // right-hand sides: block b works on field b % nr of each batch
  double* partial;
  TileOrder ord;
};

// DS: 0 = no spatial hop, 3 = spatial links read whole, 2 = read as two rows (SU(3))
template <typename S, bool DT, int DS, bool CLOV, bool IN2, bool NORM>
__global__ void __launch_bounds__(kBlock) k_site_p3(SiteArgsP3<S> a) {
  using R = typename Prec<S>::R;
  using Lt = typename Prec<S>::L;
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  const int p = a.par;  // one parity per launch: every field plane address is uniform
  const uint32_t nr = uint32_t(a.nr), rhs = blockIdx.x % nr, blk = blockIdx.x / nr, nblk = gridDim.x / nr;
  const SpinorF<S> self = rhs_view(a.self[p], rhs), nbf = rhs_view(a.nb[p], rhs);
  const SpinorF<S> in2 = rhs_view(a.in2[p], rhs), dst = rhs_view(a.dst[p], rhs);
  const uint32_t first = a.ord.on ? ordered_block(a.ord, blk) : blk;
  for (uint32_t i = first * blockDim.x + threadIdx.x; i < uint32_t(a.g.V2); i += nblk * blockDim.x) {
    int t, s;
    p3_ts32(a.g, i, t, s);
    cx<R> out[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = czero<R>();
    if (a.c_mu != 0.0 || CLOV) {
      cx<R> psi[12];
      load_spinor<S, R>(self, i, psi);
      R cm = R(a.c_mu);
#pragma unroll
      for (int c = 0; c < 12; ++c) out[c] = cm * psi[c];
      if constexpr (CLOV) {
        cx<R> ap[12];
        clover_apply<R, Lt>(a.clov[p], a.g.V2, i, psi, ap);
        R ca = R(a.c_A);
#pragma unroll
        for (int c = 0; c < 12; ++c) out[c] += ca * ap[c];
      }
    }
    if constexpr (DT) {
      hop_time_p3<S, R, Lt>(self, a.u[p][3], a.g, t, s, R(a.c_t), out);
    }
    if constexpr (DS != 0) {
      hop_space_p3<S, R, Lt, DS>(nbf, a.u[p], a.u[1 - p], a.g, p, t, s, R(0.5 * a.c_s), out);
    }
    if constexpr (IN2) {
      cx<R> e[12];
      load_spinor<S, R>(in2, i, e);
      R ci = R(a.c_in);
#pragma unroll
      for (int c = 0; c < 12; ++c) out[c] += ci * e[c];
    }
    if constexpr (NORM) {
#pragma unroll
      for (int c = 0; c < 12; ++c) acc += double(norm2(out[c]));
    }
    store_spinor<S, R>(dst, i, out);
  }
  if constexpr (NORM) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0;
      for (int w = 0; w < kBlock / 64; ++w) s += red[w];
      a.partial[(int64_t)blockIdx.x * 8] = s;
    }
  }
}

// ---- 4D even-odd Schur (p4 layout) ---------------------------------------------------------
template <typename S>
struct ArgsP4 {
  SpinorF<S> src, dst, in2;  // src on parity 1-p; dst and in2 on parity p
  LinkF<typename Prec<S>::L> u[2][4];
  const typename Prec<S>::L* clov;  // blocks on parity p
  double c_h, c_in, inv_gf;
  Geom g;
  int p;
};

// CL: 0 none; 1 clover applied to (c_in*in2 + c_h*D_w src); 2 clover applied to in2,
// then + c_h*D_w src.
template <typename S, bool HOP, bool IN2, int CL>
__global__ void __launch_bounds__(kBlock) k_schur4d(ArgsP4<S> a) {
  using R = typename Prec<S>::R;
  using Lt = typename Prec<S>::L;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.V2) return;
  cx<R> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = czero<R>();
  if constexpr (IN2) {
    cx<R> e[12];
    load_spinor<S, R>(a.in2, i, e);
    if constexpr (CL == 2) {
      clover_apply<R, Lt>(a.clov, a.g.V2, i, e, v);
    } else {
      R ci = R(a.c_in);
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = ci * e[c];
    }
  }
  if constexpr (HOP) {
    hop_4d_p4<S, R, Lt>(a.src, a.u[a.p], a.u[1 - a.p], a.g, a.p, i, R(a.c_h), R(a.c_h * a.inv_gf), v);
  }
  if constexpr (CL == 1) {
    cx<R> w[12];
    clover_apply<R, Lt>(a.clov, a.g.V2, i, v, w);
    store_spinor<S, R>(a.dst, i, w);
  } else {
    store_spinor<S, R>(a.dst, i, v);
  }
}

// ---- link gradient ----------------------------------------------------------------------------
// Per link U_mu(s):  K = Y + Z^dag with
//   Y_ca = sum_a [P-^mu x(s+mu)]_{a c} conj(lambda(s)_{a a'}),
//   Z_ca = sum_a [P+^mu x(s)]_{a c} conj(lambda(s+mu)_{a a'});
// raw gradient k b K^dag, projected k b TH(i U K).
TP_DEV void proj_full(int mu, bool minus, const cx<double>* x, cx<double>* out) {
  // out = (1 -+ gamma_mu)/2 x, as a full 4-spinor
  if (mu == 3) {
    for (int c = 0; c < 12; ++c) out[c] = czero<double>();
    int off = minus ? 6 : 0;
    for (int c = 0; c < 6; ++c) out[off + c] = x[off + c];
    return;
  }
  cx<double> h[6], a[3], b[3];
  double sg = minus ? 1.0 : -1.0;  // h = x_up + sg * i s_k x_lo
  if (mu == 0) is_k<0, double>(x + 6, x + 9, a, b);
  else if (mu == 1) is_k<1, double>(x + 6, x + 9, a, b);
  else is_k<2, double>(x + 6, x + 9, a, b);
  for (int c = 0; c < 3; ++c) { h[c] = x[c] + sg * a[c]; h[3 + c] = x[3 + c] + sg * b[c]; }
  if (mu == 0) is_k<0, double>(h, h + 3, a, b);
  else if (mu == 1) is_k<1, double>(h, h + 3, a, b);
  else is_k<2, double>(h, h + 3, a, b);
  // lower = -sg * i s_k h
  for (int c = 0; c < 3; ++c) {
    out[c] = 0.5 * h[c];
    out[3 + c] = 0.5 * h[3 + c];
    out[6 + c] = (-0.5 * sg) * a[c];
    out[9 + c] = (-0.5 * sg) * b[c];
  }
}

// One direction mu (a compile-time constant, so that no array is indexed by it: such arrays
// would live in scratch memory).
template <int mu>
TP_DEV void force_site(SpinorF<double2> x0, SpinorF<double2> x1, SpinorF<double2> l0,
                       SpinorF<double2> l1, const double2* __restrict__ canon, double2* grad,
                       const Geom& g, int64_t V, double inv_gf, double b, int projected, int64_t n) {
  int x = int(n % g.Lx);
  int64_t r = n / g.Lx;
  int y = int(r % g.Ly);
  r /= g.Ly;
  int z = int(r % g.Lz);
  int t = int(r / g.Lz);
  // s + mu
  const int xn = mu == 0 ? (x + 1 == g.Lx ? 0 : x + 1) : x;
  const int yn = mu == 1 ? (y + 1 == g.Ly ? 0 : y + 1) : y;
  const int zn = mu == 2 ? (z + 1 == g.Lz ? 0 : z + 1) : z;
  const int tn = mu == 3 ? (t + 1 == g.Lt ? 0 : t + 1) : t;
  auto p3 = [&](int X, int Y, int Z, int T, int& p, int64_t& i) {
    p = (X + Y + Z) & 1;
    i = p3_idx(g, T, (X + g.Lx * (Y + g.Ly * Z)) >> 1);
  };
  int pa, pb;
  int64_t ia, ib;
  p3(x, y, z, t, pa, ia);
  p3(xn, yn, zn, tn, pb, ib);
  cx<double> xa[12], xb[12], la[12], lb[12], px[12];
  load_spinor<double2, double>(pa ? x1 : x0, ia, xa);
  load_spinor<double2, double>(pb ? x1 : x0, ib, xb);
  load_spinor<double2, double>(pa ? l1 : l0, ia, la);
  load_spinor<double2, double>(pb ? l1 : l0, ib, lb);
  cx<double> K[9];
  for (int k = 0; k < 9; ++k) K[k] = czero<double>();
  proj_full(mu, true, xb, px);  // P- x(s+mu)
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a) {
      cx<double> s = czero<double>();
      for (int al = 0; al < 4; ++al) s += cmulc(la[3 * al + a], px[3 * al + c]);
      K[3 * c + a] += s;  // Y_ca
    }
  proj_full(mu, false, xa, px);  // P+ x(s)
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a) {
      cx<double> s = czero<double>();
      for (int al = 0; al < 4; ++al) s += cmulc(lb[3 * al + a], px[3 * al + c]);
      K[3 * a + c] += conj(s);  // (Z^dag)_ac = conj(Z_ca)
    }
  double fac = (mu == 3 ? 1.0 : inv_gf) * ((mu == 3 && t == g.Lt - 1) ? b : 1.0);
  double2* out = grad + ((int64_t)mu * V + n) * 9;
  if (!projected) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cx<double> v = fac * conj(K[3 * j + i]);
        out[3 * i + j] = make_double2(v.re, v.im);
      }
    return;
  }
  const double2* u = canon + ((int64_t)mu * V + n) * 9;
  cx<double> U[9], M[9];
  for (int k = 0; k < 9; ++k) U[k] = cx<double>{u[k].x, u[k].y};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cx<double> s = czero<double>();
      for (int k = 0; k < 3; ++k) s += cmul(U[3 * i + k], K[3 * k + j]);
      M[3 * i + j] = ti(s);  // i U K
    }
  double tr = (M[0].re + M[4].re + M[8].re) / 3.0;  // tr of (M + M^dag)/2 over 3
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cx<double> h = 0.5 * (M[3 * i + j] + conj(M[3 * j + i]));
      if (i == j) h.re -= tr;
      out[3 * i + j] = make_double2(fac * h.re, fac * h.im);
    }
}

__global__ void __launch_bounds__(128) k_force(SpinorF<double2> x0, SpinorF<double2> x1, SpinorF<double2> l0,
                        SpinorF<double2> l1, const double2* __restrict__ canon, double2* grad,
                        Geom g, int64_t V, double inv_gf, double b, int projected) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  switch (blockIdx.y) {
    case 0: force_site<0>(x0, x1, l0, l1, canon, grad, g, V, inv_gf, b, projected, n); break;
    case 1: force_site<1>(x0, x1, l0, l1, canon, grad, g, V, inv_gf, b, projected, n); break;
    case 2: force_site<2>(x0, x1, l0, l1, canon, grad, g, V, inv_gf, b, projected, n); break;
    default: force_site<3>(x0, x1, l0, l1, canon, grad, g, V, inv_gf, b, projected, n); break;
  }
}

template <typename S>
SpinorF<S> view(const Field* f, int p) {
  if (!f) {
    SpinorF<S> z;
    z.p[0] = z.p[1] = nullptr;
    z.nrm[0] = z.nrm[1] = nullptr;
    z.stride = 0;
    return z;
  }
  return f->template par<S>(p);
}

template <typename S>
struct LinkSrc;
template <> struct LinkSrc<double2> {
  static const double2* get(tp_gauge g, bool l4) { return l4 ? g->u4_d : g->u3_d; }
};
template <> struct LinkSrc<float2> {
  static const float2* get(tp_gauge g, bool l4) { return l4 ? g->u4_f : g->u3_f; }
};
template <> struct LinkSrc<__half2> {
  // F16N runs only in the p3 layout (the 4D scheme is F64/F32)
  static const __half2* get(tp_gauge g, bool l4) { return l4 ? nullptr : g->u3_h; }
};

template <typename S>
void fill_links(tp_gauge g, bool l4, LinkF<typename Prec<S>::L> (&u)[2][4], int64_t V2) {
  const typename Prec<S>::L* base = LinkSrc<S>::get(g, l4);
  for (int p = 0; p < 2; ++p)
    for (int d = 0; d < 4; ++d) {
      u[p][d].p = base + (int64_t)(d * 2 + p) * 9 * V2;
      u[p][d].stride = V2;
    }
}

template <typename S>
const typename Prec<S>::L* clover_base(tp_op op, int kind, bool l4);
template <> const double2* clover_base<double2>(tp_op op, int kind, bool l4) {
  if (kind == 1) return op->c ? (l4 ? op->c->a4_d : op->c->a3_d) : nullptr;
  if (kind == 2) return l4 ? op->a4_mu : op->a3_mu;
  if (kind == 3) return l4 ? op->a4_inv : op->a3_inv;
  return nullptr;
}
template <> const float2* clover_base<float2>(tp_op op, int kind, bool l4) {
  if (kind == 1) return op->c ? (l4 ? op->c->a4_f : op->c->a3_f) : nullptr;
  if (kind == 2) return l4 ? op->a4_mu_f : op->a3_mu_f;
  if (kind == 3) return l4 ? op->a4_inv_f : op->a3_inv_f;
  return nullptr;
}
template <> const __half2* clover_base<__half2>(tp_op op, int kind, bool l4) {
  if (l4) return nullptr;
  if (kind == 1) return op->c ? op->c->a3_h : nullptr;
  if (kind == 2) return op->a3_mu_h;
  if (kind == 3) return op->a3_inv_h;
  return nullptr;
}

template <typename S, bool DT, int DS, bool CLOV, bool IN2, bool NORM>
void site_go(tp_op op, SiteArgsP3<S> a, int64_t nblocks, int par0, int npar) {
  tp_ctx ctx = op->g->ctx;
  for (int q = 0; q < npar; ++q) {
    a.par = par0 + q;
    a.partial = ctx->red_partial + (int64_t)q * nblocks * 8;
    hipLaunchKernelGGL((k_site_p3<S, DT, DS, CLOV, IN2, NORM>), dim3((unsigned)(nblocks * a.nr)), dim3(kBlock),
                       0, ctx->stream, a);
    LAUNCH_CHECK();
  }
}

template <typename S, bool DT, int DS, bool CLOV>
void site_in2(tp_op op, SiteArgsP3<S>& a, int64_t nb, bool in2, bool norm, int par0, int npar) {
  if (in2) {
    if (norm) site_go<S, DT, DS, CLOV, true, true>(op, a, nb, par0, npar);
    else site_go<S, DT, DS, CLOV, true, false>(op, a, nb, par0, npar);
  } else {
    if (norm) site_go<S, DT, DS, CLOV, false, true>(op, a, nb, par0, npar);
    else site_go<S, DT, DS, CLOV, false, false>(op, a, nb, par0, npar);
  }
}

template <typename S>
SpinorF<S> halves(const Field* up, const Field* lo, int p) {
  SpinorF<S> a = view<S>(up, p), b = view<S>(lo, p);
  a.p[1] = b.p[1];
  a.nrm[1] = b.nrm[1];
  if (!up) a.stride = b.stride;
  return a;
}

template <typename S>
int site_t(tp_op op, const SiteIO& io, Field& dst, SiteCoef cf, int ck, int par0, int npar, bool norm) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  const Field* in2 = io.in2;
  SiteArgsP3<S> a;
  for (int p = 0; p < 2; ++p) {
    a.self[p] = halves<S>(io.self_up, io.self_lo, p);
    a.nb[p] = halves<S>(io.nb_up, io.nb_lo, 1 - p);
    a.dst[p] = view<S>(&dst, p);
    a.in2[p] = view<S>(in2, p);
  }
  fill_links<S>(op->g, false, a.u, L.V2);
  const typename Prec<S>::L* cb = clover_base<S>(op, ck, false);
  bool clov = cb != nullptr && cf.c_A != 0.0;
  for (int p = 0; p < 2; ++p) a.clov[p] = cb ? cb + (int64_t)p * 36 * L.V2 : nullptr;
  a.c_mu = cf.c_mu;
  a.c_A = cf.c_A;
  a.c_t = cf.c_t;
  a.c_s = cf.c_s;
  a.c_in = cf.c_in;
  a.g = L.g;
  // one launch per output parity; with a norm, each launch's partials follow the previous
  a.nr = dst.nr;
  if (norm && a.nr != 1) TP_THROW(TP_EINVAL, "a fused norm needs a single right-hand side");
  int64_t nb = (L.V2 + kBlock - 1) / kBlock;
  if (norm) nb = std::min<int64_t>(nb, kRedBlocks / 2);
  a.ord = tile_order(L, nb, a.nr, Prec<S>::half);
  bool dt = cf.c_t != 0.0, ds = cf.c_s != 0.0;
  bool i2 = in2 != nullptr;
  // spatial hops read SU(3) links as two rows (FP64: only links SU(3) to 1e-13)
  constexpr bool kReduced = !std::is_same<S, double2>::value;
  const bool two = kReduced ? op->g->su3_spatial : op->g->su3_spatial_f64;
  if (dt && ds) {
    if (two) {
      if (clov) site_in2<S, true, 2, true>(op, a, nb, i2, norm, par0, npar);
      else site_in2<S, true, 2, false>(op, a, nb, i2, norm, par0, npar);
    } else {
      if (clov) site_in2<S, true, 3, true>(op, a, nb, i2, norm, par0, npar);
      else site_in2<S, true, 3, false>(op, a, nb, i2, norm, par0, npar);
    }
  } else if (ds) {
    if (two) {
      if (clov) site_in2<S, false, 2, true>(op, a, nb, i2, norm, par0, npar);
      else site_in2<S, false, 2, false>(op, a, nb, i2, norm, par0, npar);
    } else {
      if (clov) site_in2<S, false, 3, true>(op, a, nb, i2, norm, par0, npar);
      else site_in2<S, false, 3, false>(op, a, nb, i2, norm, par0, npar);
    }
  } else if (dt) {
    if (clov) site_in2<S, true, 0, true>(op, a, nb, i2, norm, par0, npar);
    else site_in2<S, true, 0, false>(op, a, nb, i2, norm, par0, npar);
  } else {
    if (clov) site_in2<S, false, 0, true>(op, a, nb, i2, norm, par0, npar);
    else site_in2<S, false, 0, false>(op, a, nb, i2, norm, par0, npar);
  }
  return norm ? int(nb * npar) : 0;
}

template <typename S, bool HOP, bool IN2, int CL>
void s4_go(tp_ctx ctx, ArgsP4<S>& a) {
  unsigned nb = (unsigned)((a.g.V2 + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_schur4d<S, HOP, IN2, CL>), dim3(nb), dim3(kBlock), 0, ctx->stream, a);
  LAUNCH_CHECK();
}

template <typename S>
void schur4d_t(tp_op op, int mode, int p, const Field* src, Field& dst, const Field* in2, double c_h,
               double c_in, int ck) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  ArgsP4<S> a;
  a.src = view<S>(src, 1 - p);
  a.dst = view<S>(&dst, p);
  a.in2 = view<S>(in2, p);
  fill_links<S>(op->g, true, a.u, L.V2);
  const typename Prec<S>::L* cb = clover_base<S>(op, ck, true);
  a.clov = cb ? cb + (int64_t)p * 36 * L.V2 : nullptr;
  a.c_h = c_h;
  a.c_in = c_in;
  a.inv_gf = 1.0 / op->gf;
  a.g = L.g;
  a.p = p;
  switch (mode) {
    case 0: s4_go<S, true, false, 1>(ctx, a); break;
    case 1: s4_go<S, true, true, 2>(ctx, a); break;
    case 2: s4_go<S, true, true, 0>(ctx, a); break;
    case 3: s4_go<S, true, true, 1>(ctx, a); break;
    default: s4_go<S, false, true, 2>(ctx, a); break;
  }
}

}  // namespace

int launch_site(tp_op op, int prec, const SiteIO& io, Field& dst, SiteCoef cf, int ck, int par0,
                int npar, bool norm) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  double S = spinor_bytes(prec), Lb = link_bytes(prec), C = clov_bytes(prec);
  // spatial links read as two rows (12 reals) when they are SU(3) (to 1e-13 for FP64)
  double Ls = (prec != TP_F64 ? op->g->su3_spatial : op->g->su3_spatial_f64) ? Lb * 2 / 3 : Lb;
  bool self = cf.c_mu != 0 || (ck && cf.c_A != 0);
  // spinor bytes per right-hand side; links and clover once for a whole batch
  double sp = S + (self ? S : 0) + (cf.c_s != 0 ? S : 0) + (cf.c_t != 0 ? S : 0) + (io.in2 ? S : 0);
  double lk = (cf.c_s != 0 ? 6 * Ls : 0) + (cf.c_t != 0 ? 2 * Lb : 0) + (ck && cf.c_A != 0 ? C : 0);
  double bytes = double(npar) * L.V2 * (dst.nr * sp + lk);
  // the time-line pipeline's stencils are accounted separately from M / residual applies
  const int kid = cf.c_t != 0 || io.in2 ? KID_SITE_P3 : (ck && cf.c_A != 0 ? KID_HOP_CLOVER : KID_HOP_DS);
  ProfScope ps(ctx, kid, bytes);
  switch (prec) {
    case TP_F64: return site_t<double2>(op, io, dst, cf, ck, par0, npar, norm);
    case TP_F32: return site_t<float2>(op, io, dst, cf, ck, par0, npar, norm);
    default: return site_t<__half2>(op, io, dst, cf, ck, par0, npar, norm);
  }
}

int launch_site_p3(tp_op op, int prec, const Field& src, Field& dst, const Field* in2, SiteCoef cf,
                   int ck, int par0, int npar, bool norm) {
  SiteIO io;
  io.self_up = io.self_lo = io.nb_up = io.nb_lo = &src;
  io.in2 = in2;
  return launch_site(op, prec, io, dst, cf, ck, par0, npar, norm);
}

void launch_schur4d(tp_op op, int prec, int mode, int p, const Field* src, Field& dst, const Field* in2,
                    double c_h, double c_in, int ck) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  double S = double(dst.elem_bytes()) * 12;
  double Lb = prec == TP_F64 ? 144 : 72;
  double C = prec == TP_F64 ? 576 : 288;
  double bytes = double(L.V2) * (S + (mode != 4 ? S + 8 * Lb : 0) + (in2 ? S : 0) + (ck ? C : 0));
  ProfScope ps(ctx, mode == 0 ? KID_SCHUR4D_EO : KID_SCHUR4D_OE, bytes);
  switch (prec) {
    case TP_F64: schur4d_t<double2>(op, mode, p, src, dst, in2, c_h, c_in, ck); break;
    default: schur4d_t<float2>(op, mode, p, src, dst, in2, c_h, c_in, ck); break;
  }
}

void launch_force(tp_op op, const Field& x, const Field& lam, double2* grad, bool projected) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  ProfScope ps(ctx, KID_FORCE, double(L.V) * 4 * (4 * 192 + 144 + 144));
  hipLaunchKernelGGL(k_force, dim3((unsigned)((L.V + 127) / 128), 4), dim3(128), 0, ctx->stream,
                     x.par<double2>(0), x.par<double2>(1), lam.par<double2>(0), lam.par<double2>(1),
                     op->g->canon, grad, L.g, L.V, 1.0 / op->gf, double(ctx->bc), projected ? 1 : 0);
  LAUNCH_CHECK();
}
