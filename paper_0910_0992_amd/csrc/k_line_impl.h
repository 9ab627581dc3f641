// Time-line kernels: the exact inverse of the temporal matrix T (and T^dagger)
// inside C_L, C_R, and the fused middle step of the 3D ILU operator.
//
// Sec. II.A inverts T = mu - U_t(t) delta_{t+1,t'} (with the boundary corner)
// per spatial site by Sherman-Morrison-Woodbury: an open back-substitution
// plus a rank-3 correction built from partial Polyakov loops X(t).  The p3
// operators here live in the axial gauge of Sec. II.C / App. C, fixed once per
// gauge field with Omega(x) = W(x)^dag, W(t) = U_t(t) U_t(t+1) ... U_t(Lt-1):
// every interior time link is the identity and U_t(Lt-1) = P, the Polyakov
// loop with the boundary phase.  T psi = eta then reads
//   mu psi(t) - psi(t+1) = eta(t)   (t < Lt-1),   mu psi(Lt-1) - P psi(0) = eta(Lt-1),
// whose exact solution is the scalar discounted suffix sum
//   sigma(t) = (eta(t) + sigma(t+1)) / mu,  sigma(Lt) = 0,
//   psi(t) = sigma(t) + mu^-(Lt-1-t) delta,  delta = (I - mu^-Lt P)^-1 P sigma(0) / mu,
// i.e. the SMW back-substitution with X(t) = -b mu^-(Lt-t) P.  T^dagger mirrors
// it with a prefix sum and delta' = G^dagger rho(Lt-1).  No link is read by a
// scan.  Because the recurrence has a scalar coefficient, a line splits into
// chunks whose partial sums combine exactly (carry = mu^-k times the neighbour
// chunk's head), by DPP row operations within a wavefront and through LDS across
// wavefronts.  The closure G = (I - mu^-Lt P)^-1 P / mu is formed
// in FP64 at set-up (mu^-Lt is far below FP32 range on long lines) and applied in the
// kernel's arithmetic precision.  With the cutoff trick (Sec. II.A, eq:cutoff) the closure
// term is applied only on the slices whose Woodbury vector survives, t >= cut for T^-1 and
// t < Lt - cut for T^dagger^-1; threads whose slices all fall outside skip the closure.
//
// Workgroup = LPB lines (whole tiles of 4 lines) x NCH chunks of CH consecutive
// time slices.  A wavefront covers one contiguous run of the tiled p3 layout (16
// slices x 4 lines when NCH is a multiple of 16, with one line per 16-lane DPP row;
// otherwise threads in memory order), so loads and stores are contiguous across it.
#pragma once
#include "tp_internal.h"

namespace {

template <typename R> struct Cplx2;
template <> struct Cplx2<double> { using T = double2; };
template <> struct Cplx2<float> { using T = float2; };

template <typename R>
struct ScanCtx {
  int l, j, LPB, NCH, t0, Lt, CH;
  int cut;      // cutoff trick: time slices (from the open end) without the closure term
  int s;
  int tile;     // tile of 4 lines within the workgroup
  bool active;
  bool fast;    // NCH % 16 == 0: each wavefront holds 16 chunks of the 4 lines of one tile
  R inv_mu, f;  // 1/mu and mu^-CH
  const R* mupow;  // mu^-k, k = 0..Lt
  // fast combine (lane = line * 16 + chunk within the wavefront)
  int jw, lt, seg, nseg;  // chunk within the wavefront, line within the tile, segment, segments
  R F;                    // mu^-(16 CH): factor between neighbouring segments
  cx<R>* tabs;            // combine tables: [2 buffers][2 sets] x [tile][16 segments][4 lines][6]
  int slot;               // complex values per table
  int buf;                // table buffer of the next combine (alternates, so no trailing barrier)
  const cx<R>* gl;        // closure G of the workgroup's lines, staged in LDS: [line][9]
};

// DPP move inside rows of 16 lanes: with CTRL = 0x100 + d (row_shl) lane i receives lane i + d
// of its row, with 0x110 + d (row_shr) lane i - d; lanes whose source lies outside the row
// receive zero.
template <int CTRL> TP_DEV float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> TP_DEV double dpp_f(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xF, 0xF, false));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
// The value d chunks further along the scan direction (backward scans run from high to low t,
// so they take the value of chunk j + d; forward scans that of chunk j - d), zero past the row.
template <typename R, bool BWD, int D> TP_DEV cx<R> from_next(cx<R> v) {
  constexpr int ctrl = BWD ? 0x100 + D : 0x110 + D;
  return cx<R>{dpp_f<ctrl>(v.re), dpp_f<ctrl>(v.im)};
}
template <typename R, bool BWD, int D> TP_DEV void ks_step(cx<R> (&X)[6], R fd) {
#pragma unroll
  for (int c = 0; c < 6; ++c) X[c] += fd * from_next<R, BWD, D>(X[c]);
}

// Level 1 of the fast combine: inclusive suffix (BWD) / prefix (FWD) of the chunk heads X over
// the 16 chunks of each line held by the wavefront (one DPP row per line), factor f per chunk;
// Cin receives the exclusive value (the neighbour chunk's inclusive value).
template <typename R, bool BWD>
TP_DEV void lvl1(cx<R> (&X)[6], cx<R> (&Cin)[6], R f) {
  const R f2 = f * f, f4 = f2 * f2, f8 = f4 * f4;
  ks_step<R, BWD, 1>(X, f);
  ks_step<R, BWD, 2>(X, f2);
  ks_step<R, BWD, 4>(X, f4);
  ks_step<R, BWD, 8>(X, f8);
#pragma unroll
  for (int c = 0; c < 6; ++c) Cin[c] = from_next<R, BWD, 1>(X[c]);
}

template <typename R>
TP_DEV cx<R>* tab_of(const ScanCtx<R>& sc, int set) {
  return sc.tabs + (sc.buf * 2 + set) * sc.slot + sc.tile * 16 * 24 + sc.lt * 6;
}

// The segment total of each line and segment (the inclusive value at the segment's first chunk
// for BWD, its last for FWD) goes to the table.
template <typename R, bool BWD>
TP_DEV void lvl2_put(const cx<R> (&X)[6], const ScanCtx<R>& sc, int set) {
  if (sc.jw == (BWD ? 0 : 15)) {
    cx<R>* p = tab_of(sc, set) + sc.seg * 24;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = X[c];
  }
}

// Level 2, run by the tile's first wavefront (lane = line * 16 + segment): the segment totals of
// each line are scanned in place with factor F per segment.
template <typename R, bool BWD>
TP_DEV void lvl2_scan(const ScanCtx<R>& sc, int set) {
  cx<R>* p = tab_of(sc, set) + sc.jw * 24;
  const bool in = sc.jw < sc.nseg;
  cx<R> T[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) T[c] = in ? p[c] : czero<R>();
  const R F2 = sc.F * sc.F, F4 = F2 * F2, F8 = F4 * F4;
  ks_step<R, BWD, 1>(T, sc.F);
  ks_step<R, BWD, 2>(T, F2);
  ks_step<R, BWD, 4>(T, F4);
  ks_step<R, BWD, 8>(T, F8);
  if (in) {
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = T[c];
  }
}

// Carry from the other segments and the line total Z (at chunk 0 for BWD, at the last chunk for FWD).
template <typename R, bool BWD>
TP_DEV void lvl2_get(cx<R> (&C)[6], cx<R> (&Z)[6], R w, const ScanCtx<R>& sc, int set) {
  const cx<R>* p = tab_of(sc, set);
  const int nxt = BWD ? sc.seg + 1 : sc.seg - 1;
  const bool hasn = BWD ? (nxt < sc.nseg) : (nxt >= 0);
  const cx<R>* pn = p + (hasn ? nxt : 0) * 24;
  const cx<R>* pz = p + (BWD ? 0 : sc.nseg - 1) * 24;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    if (hasn) C[c] += w * pn[c];
    Z[c] = pz[c];
  }
}

// Weight of the carried-in segment total for this thread's chunk: f^(15-jw) (BWD), f^jw (FWD);
// every index is below 16 CH <= Lt on the fast path.
template <typename R, bool BWD> TP_DEV R seg_weight(const ScanCtx<R>& sc) {
  return sc.mupow[sc.CH * (BWD ? 15 - sc.jw : sc.jw)];
}
// Closure weights of this thread's slices: mu^-(Lt-1-t) (BWD), mu^-t (FWD), 0 where the cutoff
// drops the closure.
template <typename R, int CH, bool BWD> TP_DEV void closure_weights(R (&cb)[CH], const ScanCtx<R>& sc) {
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int t = sc.t0 + k;
    const bool keep = BWD ? (t >= sc.cut) : (t < sc.Lt - sc.cut);
    cb[k] = keep ? sc.mupow[BWD ? sc.Lt - 1 - t : t] : R(0);
  }
}

// Exclusive carries across the line in LDS (Hillis-Steele), for lines whose chunk count is not
// a multiple of 16.  Z = the line's total at chunk 0 (BWD) or at the last chunk (FWD).
template <typename R, bool BWD>
TP_DEV void combine_lds(cx<R> (&X)[6], cx<R> (&C)[6], cx<R> (&Z)[6], cx<R>* lds, const ScanCtx<R>& sc) {
  const int me = (sc.j * sc.LPB + sc.l) * 6;
  R fd = sc.f;
  for (int d = 1; d < sc.NCH; d <<= 1) {
#pragma unroll
    for (int c = 0; c < 6; ++c) lds[me + c] = X[c];
    __syncthreads();
    int jj = BWD ? sc.j + d : sc.j - d;
    if (jj >= 0 && jj < sc.NCH) {
      const int o = (jj * sc.LPB + sc.l) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) X[c] += fd * lds[o + c];
    }
    __syncthreads();
    fd = fd * fd;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) lds[me + c] = X[c];
  __syncthreads();
  int jc = BWD ? sc.j + 1 : sc.j - 1;
  bool has = jc >= 0 && jc < sc.NCH;
  const int oc = ((has ? jc : 0) * sc.LPB + sc.l) * 6;
  const int oz = ((BWD ? 0 : sc.NCH - 1) * sc.LPB + sc.l) * 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    C[c] = has ? lds[oc + c] : czero<R>();
    Z[c] = lds[oz + c];
  }
  __syncthreads();
}

// Chunk-local recurrence of one group of 6 values; returns the chunk head (BWD) / tail (FWD).
template <typename R, int CH, int NV, bool BWD>
TP_DEV void local_scan(cx<R> (&v)[CH][NV], int g, cx<R> (&X)[6], const ScanCtx<R>& sc) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    cx<R> acc = czero<R>();
    if constexpr (BWD) {
#pragma unroll
      for (int k = CH - 1; k >= 0; --k) {
        acc = sc.inv_mu * (v[k][6 * g + c] + acc);
        v[k][6 * g + c] = acc;
      }
    } else {
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        acc = sc.inv_mu * (v[k][6 * g + c] + acc);
        v[k][6 * g + c] = acc;
      }
    }
    X[c] = acc;
  }
}

// Closure delta = G z (backward) or G^dagger z (forward), per colour vector, on the slices the
// cutoff keeps (all of them when cut = 0), and the final values of the group:
// v(t) += mu^-(distance to the carried-in chunk) C + mu^-(distance to the line's end) delta.
template <typename R, int CH, int NV, bool BWD>
TP_DEV void finish(cx<R> (&v)[CH][NV], int g, const cx<R> (&C)[6], const cx<R> (&Z)[6],
                   const R (&cb)[CH], const ScanCtx<R>& sc) {
  cx<R> D[6];
  const bool band = BWD ? (sc.t0 + CH - 1 >= sc.cut) : (sc.t0 < sc.Lt - sc.cut);
  if (sc.active && band) {
    const cx<R>* G = sc.gl + sc.l * 9;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> acc0 = czero<R>(), acc1 = czero<R>();
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const cx<R> gk = G[BWD ? 3 * a + b : 3 * b + a];
        if constexpr (BWD) {
          acc0 += cmul(gk, Z[b]);
          acc1 += cmul(gk, Z[3 + b]);
        } else {
          acc0 += cmulc(gk, Z[b]);
          acc1 += cmulc(gk, Z[3 + b]);
        }
      }
      D[a] = acc0;
      D[3 + a] = acc1;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) D[c] = czero<R>();
  }
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const R ca = BWD ? sc.mupow[CH - k] : sc.mupow[k + 1];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[k][6 * g + c] += ca * C[c] + cb[k] * D[c];
  }
}

// Scans of one or two sets of values per time slice (v1: NV1 values scanned in direction B1,
// v2: NV2 values in direction B2; NV2 = 0 for one set): on return each holds the scan result
// (T^-1 for a backward scan, T^dagger^-1 for a forward one).  Groups of 6 values (two colour
// vectors) are finished one at a time; the two sets' groups share the combine's barriers.
template <typename R, int CH, int NV1, bool B1, int NV2, bool B2, int N1, int N2>
TP_DEV void scan_sets(cx<R> (&v1)[CH][N1], cx<R> (&v2)[CH][N2], cx<R>* lds, ScanCtx<R>& sc) {
  constexpr int G1 = NV1 / 6, G2 = NV2 / 6, G = G1 > G2 ? G1 : G2;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    cx<R> X1[6], X2[6], C1[6], C2[6], Z1[6], Z2[6];
    if (g < G1) local_scan<R, CH, N1, B1>(v1, g, X1, sc);
    if (g < G2) local_scan<R, CH, N2, B2>(v2, g, X2, sc);
    // weights, loaded ahead of the barriers that hide their latency
    R cb1[CH], cb2[CH], w1 = R(0), w2 = R(0);
    if (sc.fast) {
      if (g < G1) { lvl1<R, B1>(X1, C1, sc.f); lvl2_put<R, B1>(X1, sc, 0); w1 = seg_weight<R, B1>(sc); }
      if (g < G2) { lvl1<R, B2>(X2, C2, sc.f); lvl2_put<R, B2>(X2, sc, 1); w2 = seg_weight<R, B2>(sc); }
      if (g < G1) closure_weights<R, CH, B1>(cb1, sc);
      if (g < G2) closure_weights<R, CH, B2>(cb2, sc);
      __syncthreads();
      if (sc.seg == 0) {  // uniform per wavefront
        if (g < G1) lvl2_scan<R, B1>(sc, 0);
        if (g < G2) lvl2_scan<R, B2>(sc, 1);
      }
      __syncthreads();
      if (g < G1) lvl2_get<R, B1>(C1, Z1, w1, sc, 0);
      if (g < G2) lvl2_get<R, B2>(C2, Z2, w2, sc, 1);
      sc.buf ^= 1;
    } else {
      if (g < G1) { closure_weights<R, CH, B1>(cb1, sc); combine_lds<R, B1>(X1, C1, Z1, lds, sc); }
      if (g < G2) { closure_weights<R, CH, B2>(cb2, sc); combine_lds<R, B2>(X2, C2, Z2, lds, sc); }
    }
    if (g < G1) finish<R, CH, N1, B1>(v1, g, C1, Z1, cb1, sc);
    if (g < G2) finish<R, CH, N2, B2>(v2, g, C2, Z2, cb2, sc);
  }
}

// One set (NV values, direction BWD).
template <typename R, int CH, int NV, bool BWD>
TP_DEV void scan_core(cx<R> (&v)[CH][NV], cx<R>* lds, ScanCtx<R>& sc) {
  cx<R> dummy[CH][1];
  scan_sets<R, CH, NV, BWD, 0, BWD, NV, 1>(v, dummy, lds, sc);
}

// The line kernels read every input once per launch (the middle kernel parks what it needs
// twice in LDS), in fields larger than the caches: their loads carry the non-temporal hint.
typedef unsigned int lu32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int lu32x4 __attribute__((ext_vector_type(4)));
template <typename T> TP_DEV T nt_ld(const T* p) {
  if constexpr (sizeof(T) == 16) return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const lu32x4*>(p)));
  else if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const lu32x2*>(p)));
  else return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p)));
}
// load_half (64-bit index form) with non-temporal loads: the same values.
template <typename S, typename R = typename Prec<S>::R>
TP_DEV void nt_load_half(const SpinorF<S>& f, int h, int64_t i, cx<R>* v) {
  const S* b = f.p[h];
  if constexpr (Prec<S>::half) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const Half2x2 e = nt_ld(reinterpret_cast<const Half2x2*>(b + (int64_t)(2 * q) * f.stride + 2 * i));
      const float2 fa = __half22float2(e.a), fb = __half22float2(e.b);
      v[2 * q] = {fa.x, fa.y};
      v[2 * q + 1] = {fb.x, fb.y};
    }
    const R sc = nt_ld(f.nrm[h] + i);
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = sc * v[c];
  } else if constexpr (paired<S>()) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float4 e = nt_ld(reinterpret_cast<const float4*>(b + (int64_t)(2 * q) * f.stride + 2 * i));
      v[2 * q] = {e.x, e.y};
      v[2 * q + 1] = {e.z, e.w};
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const S e = nt_ld(b + (int64_t)c * f.stride + i);
      v[c] = {R(e.x), R(e.y)};
    }
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
  SpinorF<S> in, out, aux, self, base;
  const typename Prec<S>::L* clov;  // A/2 blocks of this parity
  const typename Cplx2<typename Prec<S>::R>::T* G;  // closure, FP64 or FP32
  const typename Prec<S>::R* mupow;
  double inv_mu, f, c_out, c_base;
  int cut;        // cutoff trick: slices without the closure term (0: exact inverse)
  Geom g;
  int par, LPB, NCH;
  int lds_table;  // complex elements of LDS used by the chunk combine (the rest follows it)
  int nr;         // right-hand sides: block b works on field b % nr of each batch
  int lds_extra;  // LDS bytes after the table and the parked complex values
};

// Selects this block's right-hand side in every spinor argument; returns the block index
// within that right-hand side.
template <typename S>
TP_DEV uint32_t batch_select(LineArgs<S>& a) {
  const uint32_t nr = uint32_t(a.nr), rhs = blockIdx.x % nr;
  a.in = rhs_view(a.in, rhs);
  a.out = rhs_view(a.out, rhs);
  a.aux = rhs_view(a.aux, rhs);
  a.self = rhs_view(a.self, rhs);
  a.base = rhs_view(a.base, rhs);
  return blockIdx.x / nr;
}

// Thread layout and scan constants; stages the closure G of the workgroup's lines in LDS
// (visible after the first barrier of the combine, which precedes every use).
// Lines whose chunk count is a multiple of 16: a wavefront holds 16 consecutive chunks of the 4
// lines of one tile, lane = line * 16 + chunk, so each line's chunks form one DPP row.  Its 64
// lanes still cover one contiguous run of 16 slices x 4 lines of the tiled layout.  Otherwise
// threads run in memory order (line in tile fastest, then chunk, then tile).
template <typename S>
TP_DEV ScanCtx<typename Prec<S>::R> make_ctx(const LineArgs<S>& a, int CH, uint32_t blk, cx<typename Prec<S>::R>* lds) {
  using R = typename Prec<S>::R;
  ScanCtx<R> sc;
  const int tid = threadIdx.x;
  sc.fast = (a.NCH % 16) == 0;
  if (sc.fast) {
    const int lane = tid & 63, wv = tid >> 6, wpt = a.NCH >> 4;
    sc.jw = lane & 15;
    sc.lt = lane >> 4;
    sc.seg = wv % wpt;
    sc.nseg = wpt;
    sc.tile = wv / wpt;
    sc.j = sc.seg * 16 + sc.jw;
    sc.l = sc.tile * kTile + sc.lt;
  } else {
    const int rest = tid / kTile;
    sc.j = rest % a.NCH;
    sc.tile = rest / a.NCH;
    sc.lt = tid % kTile;
    sc.l = sc.tile * kTile + sc.lt;
    sc.jw = sc.seg = 0;
    sc.nseg = 1;
  }
  sc.CH = CH;
  sc.LPB = a.LPB;
  sc.NCH = a.NCH;
  sc.t0 = sc.j * CH;
  sc.Lt = a.g.Lt;
  sc.s = int(blk) * a.LPB + sc.l;
  sc.active = sc.s < a.g.Vs2;
  sc.inv_mu = R(a.inv_mu);
  sc.cut = a.cut;
  sc.f = R(a.f);
  sc.mupow = a.mupow;
  sc.F = sc.fast ? a.mupow[16 * CH] : R(0);  // fast path: Lt = 16 CH nseg >= 16 CH
  sc.tabs = lds;
  sc.slot = a.LPB * 16 * 6;
  sc.buf = 0;
  cx<R>* gl = lds + (a.lds_table - a.LPB * 9);
  sc.gl = gl;
  // LPB * 9 entries; a workgroup can have fewer threads (short lines: LPB * NCH < LPB * 9)
  for (int q = tid; q < a.LPB * 9; q += int(blockDim.x)) {
    const int ln = q / 9, k = q % 9;
    const int sl = int(blk) * a.LPB + ln;
    if (sl < a.g.Vs2) {
      const auto e = a.G[((int64_t)a.par * 9 + k) * a.g.Vs2 + sl];
      gl[ln * 9 + k] = cx<R>{R(e.x), R(e.y)};
    }
  }
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

// out = c_out MODE(in) + c_base base  (BASE), else c_out MODE(in).
// Halves that MODE does not scan pass through (PASS), or are left untouched.
// Largest workgroup of the line kernels: FP64 lines take at most 512 threads, which also
// lets the compiler give each FP64 thread up to 256 VGPRs.
template <typename S>
constexpr int max_threads() { return sizeof(typename Prec<S>::R) == 8 ? 512 : 1024; }

// One-slice FP32-arithmetic scans of one half spinor fit in 64 VGPRs: two 1024-thread
// workgroups per CU, so one workgroup's loads overlap the other's barriers.
template <typename S, int CH, int MODE> constexpr int line_waves() {
  return (CH == 1 && sizeof(typename Prec<S>::R) == 4 && ModeT<MODE>::nb + ModeT<MODE>::nf == 6) ? 8 : 1;
}

template <typename S, int CH, int MODE, bool BASE, bool PASS>
__global__ void __launch_bounds__(max_threads<S>()) __attribute__((amdgpu_waves_per_eu(line_waves<S, CH, MODE>())))
k_line(LineArgs<S> a) {
  using R = typename Prec<S>::R;
  using M = ModeT<MODE>;
  extern __shared__ char smem_raw[];
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
  const uint32_t blk = batch_select(a);
  ScanCtx<R> sc = make_ctx<S>(a, CH, blk, lds);
  const int s = sc.active ? sc.s : 0;
  cx<R> vb[CH][Arr<M::nb>::n], vf[CH][Arr<M::nf>::n];
  const R cout = R(a.c_out), cbase = R(a.c_base);
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int64_t i = p3_idx(a.g, sc.t0 + k, s);
    cx<R> v[12];
    if (sc.active) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool scanned = !passes<MODE>(h);
        if (scanned || PASS) nt_load_half<S, R>(a.in, h, i, v + 6 * h);
        if (PASS && !scanned) {
          cx<R> o[6];
          if constexpr (BASE) {
            cx<R> bb[6];
            nt_load_half<S, R>(a.base, h, i, bb);
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = cout * v[6 * h + c] + cbase * bb[c];
          } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = cout * v[6 * h + c];
          }
          store_half<S, R>(a.out, h, i, o);
        }
      }
      split<MODE, R>(v, vb[k], vf[k]);
    } else {
#pragma unroll
      for (int c = 0; c < Arr<M::nb>::n; ++c) vb[k][c] = czero<R>();
#pragma unroll
      for (int c = 0; c < Arr<M::nf>::n; ++c) vf[k][c] = czero<R>();
    }
  }
  if constexpr (M::nb > 0 && M::nf > 0)
    scan_sets<R, CH, M::nb, true, M::nf, false, Arr<M::nb>::n, Arr<M::nf>::n>(vb, vf, lds, sc);
  else if constexpr (M::nb > 0)
    scan_core<R, CH, M::nb, true>(vb, lds, sc);
  else
    scan_core<R, CH, M::nf, false>(vf, lds, sc);
  if (!sc.active) return;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int64_t i = p3_idx(a.g, sc.t0 + k, s);
    cx<R> v[12];
    merge<MODE, R>(v, vb[k], vf[k]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (passes<MODE>(h)) continue;
      cx<R> o[6];
      if constexpr (BASE) {
        cx<R> bb[6];
        nt_load_half<S, R>(a.base, h, i, bb);
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

// Middle step of the 3D ILU operator on the even parity, all scans of one line in one
// workgroup.  in = psi_e, aux = u = D_s^eo a_o / gamma_f:
//   b   = T^-1 u_lo,  f = T^dag^-1 (u_up + psi_up)
//   y   = A w,  w = C_R (C_L u + psi_e) = (f, b + psi_lo)
//   chi_e = psi_e + C_L y = (psi_up + y_up, psi_lo + T^-1 y_lo)               -> out
//   n_e = C_R C_L (y - u) = (T^dag^-1 (y_up - u_up), T^-1 y_lo - b)          -> base
// Threads per workgroup of the middle kernel: one slice per thread needs 1024-thread groups on
// 256-slice lines; two or more slices per thread run in 512-thread groups with twice the
// registers per thread.
template <int CH> constexpr int mid_threads() { return CH == 1 ? 1024 : 512; }

// A half spinor in the storage form of its field (FP16 pairs and the FP32 scale for the FP16
// form, else six complex values of the arithmetic precision), as parked in LDS by the middle
// kernel: one per thread and time slice.
template <typename S>
struct RawHalf {
  using R = typename Prec<S>::R;
  static constexpr bool half = Prec<S>::half;
  static constexpr int bytes = half ? 6 * 4 + 4 : 6 * int(sizeof(cx<R>));  // LDS per thread and slice
  typename std::conditional<half, Half2x2, cx<R>>::type e[half ? 3 : 6];
  float s;

  TP_DEV void load(const SpinorF<S>& f, int h, int64_t i) {
    if constexpr (half) {
#pragma unroll
      for (int q = 0; q < 3; ++q) e[q] = nt_ld(reinterpret_cast<const Half2x2*>(f.p[h] + (int64_t)(2 * q) * f.stride + 2 * i));
      s = nt_ld(f.nrm[h] + i);
    } else {
      nt_load_half<S, R>(f, h, i, e);
    }
  }
  TP_DEV void zero() {
    if constexpr (half) {
#pragma unroll
      for (int q = 0; q < 3; ++q) e[q] = Half2x2{__half2{}, __half2{}};
      s = 0.f;
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = czero<R>();
    }
  }
  TP_DEV void unpack(cx<R>* v) const {
    if constexpr (half) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float2 fa = __half22float2(e[q].a), fb = __half22float2(e[q].b);
        v[2 * q] = {s * fa.x, s * fa.y};
        v[2 * q + 1] = {s * fb.x, s * fb.y};
      }
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = e[c];
    }
  }
  // LDS slot `k` of the region at `base` ([CH][3][n] pairs then [CH][n] scales for FP16,
  // [CH][6][n] complex values otherwise; n threads, consecutive threads adjacent)
  TP_DEV void put(char* base, int CH, int n, int k) const {
    if constexpr (half) {
      Half2x2* pr = reinterpret_cast<Half2x2*>(base);
#pragma unroll
      for (int q = 0; q < 3; ++q) pr[(k * 3 + q) * n + threadIdx.x] = e[q];
      reinterpret_cast<float*>(pr + 3 * CH * n)[k * n + threadIdx.x] = s;
    } else {
      cx<R>* pr = reinterpret_cast<cx<R>*>(base);
#pragma unroll
      for (int c = 0; c < 6; ++c) pr[(k * 6 + c) * n + threadIdx.x] = e[c];
    }
  }
  TP_DEV void get(const char* base, int CH, int n, int k) {
    if constexpr (half) {
      const Half2x2* pr = reinterpret_cast<const Half2x2*>(base);
#pragma unroll
      for (int q = 0; q < 3; ++q) e[q] = pr[(k * 3 + q) * n + threadIdx.x];
      s = reinterpret_cast<const float*>(pr + 3 * CH * n)[k * n + threadIdx.x];
    } else {
      const cx<R>* pr = reinterpret_cast<const cx<R>*>(base);
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = pr[(k * 6 + c) * n + threadIdx.x];
    }
  }
};

// The ILU middle step on the even sites of each tile (App. B sequence, steps 2-5):
//   b = T^-1 u_lo, f = T^dag^-1 (u_up + psi_up), y = A (f, b + psi_lo),
//   chi = (psi_up + y_up, psi_lo + T^-1 y_lo), n = (T^dag^-1 (y_up - u_up), T^-1 y_lo - b).
// b waits in LDS from the first scans to the end (in registers when PB is false).  NP inputs are parked in LDS in storage
// form instead of being held in registers or read twice from HBM: NP = 2 parks u_up and
// psi_up, psi_lo taking u_up's slot once the clover product has consumed it; NP = 3 gives
// psi_lo its own slot, parked before the product.  Each thread touches only its own slots,
// so no barrier guards them.
template <typename S, int CH, int NP, bool PB = true>
__global__ void __launch_bounds__(mid_threads<CH>() < max_threads<S>() ? mid_threads<CH>() : max_threads<S>())
k_ilu_mid(LineArgs<S> a) {
  using R = typename Prec<S>::R;
  using Lk = typename Prec<S>::L;
  using Raw = RawHalf<S>;
  extern __shared__ char smem_raw[];
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
  const int nthr = blockDim.x;
  cx<R>* park_b = lds + a.lds_table;  // [CH][6][threads]
  char* raw0 = reinterpret_cast<char*>(park_b + 6 * CH * nthr);
  char* park_u = raw0;                                           // u_up, then (NP = 2) psi_lo
  char* park_p = raw0 + size_t(Raw::bytes) * CH * nthr;          // psi_up
  char* park_l = raw0 + size_t(Raw::bytes) * CH * nthr * 2;      // psi_lo (NP = 3)
  // PB = false (FP64 on lines too long for its LDS): b stays in registers
  cx<R> bkeep[PB ? 1 : CH][6];
  auto bslot = [&](int k, int c) -> cx<R>& {
    if constexpr (PB) return park_b[(k * 6 + c) * nthr + threadIdx.x];
    else return bkeep[k][c];
  };
  const uint32_t blk = batch_select(a);
  ScanCtx<R> sc = make_ctx<S>(a, CH, blk, lds);
  const int s = sc.active ? sc.s : 0;
  cx<R> b[CH][6], f[CH][6], uup[NP ? 1 : CH][6];
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int64_t i = p3_idx(a.g, sc.t0 + k, s);
    cx<R> u[6], ps[6];
    if constexpr (NP > 0) {
      Raw ru, rp;
      if (sc.active) {
        ru.load(a.aux, 0, i);
        rp.load(a.in, 0, i);
        nt_load_half<S, R>(a.aux, 1, i, b[k]);
      } else {
        ru.zero();
        rp.zero();
#pragma unroll
        for (int c = 0; c < 6; ++c) b[k][c] = czero<R>();
      }
      ru.put(park_u, CH, nthr, k);
      rp.put(park_p, CH, nthr, k);
      ru.unpack(u);
      rp.unpack(ps);
    } else {
      if (sc.active) {
        nt_load_half<S, R>(a.aux, 0, i, u);
        nt_load_half<S, R>(a.aux, 1, i, b[k]);
        nt_load_half<S, R>(a.in, 0, i, ps);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) { u[c] = czero<R>(); b[k][c] = czero<R>(); ps[c] = czero<R>(); }
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) uup[k][c] = u[c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) f[k][c] = u[c] + ps[c];
  }
  scan_sets<R, CH, 6, true, 6, false, 6, 6>(b, f, lds, sc);
#pragma unroll
  for (int k = 0; k < CH; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) bslot(k, c) = b[k][c];
  // y = A w; write chi_up; second-phase inputs y_lo (backward, kept in b) and y_up - u_up
  // (forward, kept in f)
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int64_t i = p3_idx(a.g, sc.t0 + k, s);
    if (sc.active) {
      cx<R> w[12], y[12], pl[6], ps[6];
      Raw rl;
      if constexpr (NP > 0) {
        rl.load(a.in, 1, i);
        rl.unpack(pl);
        if constexpr (NP == 3) rl.put(park_l, CH, nthr, k);
      } else {
        nt_load_half<S, R>(a.in, 1, i, pl);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) { w[c] = f[k][c]; w[6 + c] = bslot(k, c) + pl[c]; }
      clover_apply<R, Lk>(a.clov, a.g.V2, i, w, y);
      cx<R> u[6];
      if constexpr (NP > 0) {
        Raw rp, ru;
        rp.get(park_p, CH, nthr, k);
        rp.unpack(ps);
        ru.get(park_u, CH, nthr, k);
        ru.unpack(u);
        if constexpr (NP == 2) rl.put(park_u, CH, nthr, k);
      } else {
        nt_load_half<S, R>(a.in, 0, i, ps);
#pragma unroll
        for (int c = 0; c < 6; ++c) u[c] = uup[k][c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) ps[c] += y[c];
      store_half<S, R>(a.out, 0, i, ps);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        f[k][c] = y[c] - u[c];
        b[k][c] = y[6 + c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) { f[k][c] = czero<R>(); b[k][c] = czero<R>(); }
    }
  }
  scan_sets<R, CH, 6, true, 6, false, 6, 6>(b, f, lds, sc);  // T^-1 y_lo, T^dag^-1 (y_up - u_up)
  if (!sc.active) return;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int64_t i = p3_idx(a.g, sc.t0 + k, s);
    cx<R> pl[6], n[6];
    if constexpr (NP > 0) {
      Raw rl;
      rl.get(NP == 3 ? park_l : park_u, CH, nthr, k);
      rl.unpack(pl);
    } else {
      nt_load_half<S, R>(a.in, 1, i, pl);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      pl[c] += b[k][c];
      n[c] = b[k][c] - bslot(k, c);
    }
    store_half<S, R>(a.out, 1, i, pl);
    store_half<S, R>(a.base, 0, i, f[k]);
    store_half<S, R>(a.base, 1, i, n);
  }
}

// ---------------------------------------------------------------- launch plumbing
struct Shape {
  int CH, NCH, LPB;
};

// Pick CH (time slices per thread) from `allowed`, NCH = Lt/CH chunks, and LPB lines
// (a multiple of the 4-line tile) so that LPB * NCH <= max_threads.
Shape pick_shape(int Lt, int lpb_target, int max_threads, std::initializer_list<int> allowed) {
  for (int ch : allowed) {
    if (Lt % ch) continue;
    int nch = Lt / ch;
    if (nch * kTile > max_threads) continue;
    int lpb = lpb_target;
    while (lpb > kTile && lpb * nch > max_threads) lpb >>= 1;
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
  a.clov = nullptr;
  if (op->c) {
    if constexpr (sizeof(Lk) == 16) a.clov = (const Lk*)op->c->a3_d + (int64_t)par * 36 * L.V2;
    else if constexpr (sizeof(Lk) == 8) a.clov = (const Lk*)op->c->a3_f + (int64_t)par * 36 * L.V2;
    else a.clov = (const Lk*)op->c->a3_h + (int64_t)par * 36 * L.V2;
  }
  if constexpr (sizeof(Lk) == 16) {
    a.G = op->gclos;
    a.mupow = (const typename Prec<S>::R*)op->mupow_d;
  } else {
    a.G = op->gclos_f;
    a.mupow = (const typename Prec<S>::R*)op->mupow_f;
  }
  a.inv_mu = 1.0 / op->mu;
  a.cut = op->cut;
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


// LDS of a line kernel: the chunk-combine tables (DPP path: [2 buffers][2 sets] x [tile][16
// segments][4 lines][6]; LDS path: [chunk][line][6]) and the staged closure G ([line][9]),
// followed by `park` complex values per thread.
int lds_table_of(Shape sh) {
  return (sh.NCH % 16 == 0 ? 4 * sh.LPB * 16 * 6 : sh.LPB * sh.NCH * 6) + sh.LPB * 9;
}

template <typename S>
size_t lds_bytes(Shape sh, int park) {
  return (size_t(lds_table_of(sh)) + size_t(park) * sh.LPB * sh.NCH) * sizeof(cx<typename Prec<S>::R>);
}

template <typename S, typename K>
void go(tp_op op, K kern, LineArgs<S>& a, Shape sh, int park = 0) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  a.LPB = sh.LPB;
  a.NCH = sh.NCH;
  a.f = pow(op->mu, -double(sh.CH));
  a.lds_table = lds_table_of(sh);
  const size_t lds = lds_bytes<S>(sh, park) + size_t(a.lds_extra);
  if (lds > ctx->lds_max) TP_THROW(TP_EDIMS, "time extent too long for the line kernels' LDS");
  dim3 grid((unsigned)((L.Vs2 + sh.LPB - 1) / sh.LPB * a.nr));
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
void line_t(tp_op op, int par, const LineIO& io, Field& dst) {
  LineArgs<S> a = base_args<S>(op, par);
  SpinorF<S> up = pv<S>(io.in_up, par), lo = pv<S>(io.in_lo, par);
  a.in = up;
  a.in.p[1] = lo.p[1];
  a.in.nrm[1] = lo.nrm[1];
  a.out = pv<S>(&dst, par);
  a.base = pv<S>(io.base, par);
  a.nr = dst.nr;
  a.c_out = io.c_out;
  a.c_base = io.c_base;
  Shape sh = pick_shape(op->g->ctx->lat.L[3], 16, max_threads<S>(), {1, 2, 4});
  if (io.base) {
    if (io.pass) { TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, true, true>, a, sh)) }
    else { TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, true, false>, a, sh)) }
  } else {
    if (io.pass) { TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, false, true>, a, sh)) }
    else { TP_CH_DISPATCH(sh.CH, go<S>(op, k_line<S, CH, MODE, false, false>, a, sh)) }
  }
}

template <typename S>
void line_s(tp_op op, int mode, int par, const LineIO& io, Field& dst) {
  switch (mode) {
    case LM_CL: line_t<S, LM_CL>(op, par, io, dst); break;
    case LM_CR: line_t<S, LM_CR>(op, par, io, dst); break;
    case LM_CRCL: line_t<S, LM_CRCL>(op, par, io, dst); break;
    case LM_TINV: line_t<S, LM_TINV>(op, par, io, dst); break;
    default: line_t<S, LM_TDINV>(op, par, io, dst); break;
  }
}

template <typename S>
void mid_t(tp_op op, const Field& psi, const Field& u, Field& chi, Field& n) {
  const Lattice& L = op->g->ctx->lat;
  LineArgs<S> a = base_args<S>(op, 0);
  a.in = pv<S>(&psi, 0);
  a.aux = pv<S>(&u, 0);
  a.out = pv<S>(&chi, 0);
  a.base = pv<S>(&n, 0);
  a.nr = chi.nr;
  const int Lt = L.L[3];
  // one slice per thread where the line fits a workgroup (measured fastest), else more
  Shape sh{0, 0, 0};
  for (int ch : {1, 2, 4}) {
    const int mt = std::min(max_threads<S>(), ch == 1 ? mid_threads<1>() : mid_threads<2>());
    if (Lt % ch || (Lt / ch) * kTile > mt) continue;
    sh = pick_shape(Lt, 16, mt, {ch});
    break;
  }
  if (sh.CH == 0) TP_THROW(TP_EDIMS, "time extent not supported by the line kernels");
  // park as many inputs in LDS as the workgroup's LDS allows (each costs RawHalf bytes)
  auto bytes = [&](int np) {
    return lds_bytes<S>(sh, 6 * sh.CH) + size_t(np) * RawHalf<S>::bytes * sh.CH * sh.LPB * sh.NCH;
  };
  const int park = 6 * sh.CH;
  // FP64 scans already fill the register file: they park only b
  if constexpr (sizeof(typename Prec<S>::R) == 4) {
    const size_t cap = op->g->ctx->lds_max;
    if (bytes(3) <= cap) {
      a.lds_extra = int(bytes(3) - lds_bytes<S>(sh, park));
      TP_CH_DISPATCH(sh.CH, go<S>(op, k_ilu_mid<S, CH, 3>, a, sh, park))
      return;
    }
    if (bytes(2) <= cap) {
      a.lds_extra = int(bytes(2) - lds_bytes<S>(sh, park));
      TP_CH_DISPATCH(sh.CH, go<S>(op, k_ilu_mid<S, CH, 2>, a, sh, park))
      return;
    }
  }
  if (lds_bytes<S>(sh, park) <= op->g->ctx->lds_max) {
    TP_CH_DISPATCH(sh.CH, go<S>(op, k_ilu_mid<S, CH, 0>, a, sh, park))
  } else {
    TP_CH_DISPATCH(sh.CH, go<S>(op, k_ilu_mid<S, CH, 0, false>, a, sh, 0))
  }
}

}  // namespace

#define TP_CAT2(a, b) a##b
#define TP_CAT(a, b) TP_CAT2(a, b)
void TP_CAT(line_, TP_LINE_SUFFIX)(tp_op op, int mode, int par, const LineIO& io, Field& dst) {
  line_s<TP_LINE_S>(op, mode, par, io, dst);
}
void TP_CAT(ilu_mid_, TP_LINE_SUFFIX)(tp_op op, const Field& psi, const Field& u, Field& chi, Field& n) {
  mid_t<TP_LINE_S>(op, psi, u, chi, n);
}
