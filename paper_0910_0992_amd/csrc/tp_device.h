// Device-side arithmetic and storage helpers for gfx950.
//
// Complex numbers, SU(3) matrix-vector products, Dirac-Pauli spin projection
// and the storage formats of spinors, links and clover blocks.  All fields are
// stored as structure-of-arrays "planes": plane c of a field holds component c
// of every site contiguously, so the 64 lanes of a wavefront that handle 64
// consecutive sites issue one fully coalesced load per component.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#define TP_DEV __device__ __forceinline__
#define TP_HD __host__ __device__ __forceinline__

template <typename R>
struct cx {
  R re, im;
};

template <typename R> TP_DEV cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> TP_DEV cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> TP_DEV cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> TP_DEV cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> TP_DEV cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> TP_DEV cx<R>& operator+=(cx<R>& a, cx<R> b) { a.re += b.re; a.im += b.im; return a; }
template <typename R> TP_DEV cx<R>& operator-=(cx<R>& a, cx<R> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename R> TP_DEV cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R> TP_DEV cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> TP_DEV cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R> TP_DEV cx<R> ti(cx<R> a) { return {-a.im, a.re}; }   // i a
template <typename R> TP_DEV cx<R> tmi(cx<R> a) { return {a.im, -a.re}; }  // -i a
template <typename R> TP_DEV R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }
template <typename R> TP_DEV cx<R> czero() { return {R(0), R(0)}; }

// ---- SU(3) -------------------------------------------------------------------------
template <typename R>
struct su3 {
  cx<R> e[9];  // row-major
};

// out = U v
template <typename R> TP_DEV void mv(const su3<R>& u, const cx<R>* v, cx<R>* out) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = cmul(u.e[3 * a], v[0]);
    s += cmul(u.e[3 * a + 1], v[1]);
    s += cmul(u.e[3 * a + 2], v[2]);
    out[a] = s;
  }
}
// out = U^dagger v
template <typename R> TP_DEV void mvd(const su3<R>& u, const cx<R>* v, cx<R>* out) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> s = cmulc(u.e[a], v[0]);
    s += cmulc(u.e[3 + a], v[1]);
    s += cmulc(u.e[6 + a], v[2]);
    out[a] = s;
  }
}

// ---- storage -----------------------------------------------------------------------
// Spinor storage element types: double2 (FP64), float2 (FP32), __half2 (FP16 with
// an FP32 scale per half-spinor and site).  Links and clover blocks use double2 or
// float2.
template <typename S> struct Prec;
template <> struct Prec<double2> { using R = double; using L = double2; static constexpr bool half = false; };
template <> struct Prec<float2> { using R = float; using L = float2; static constexpr bool half = false; };
// F16N: FP16 spinors with per-site scales; p3 links and clover stored in FP16 as well
template <> struct Prec<__half2> { using R = float; using L = __half2; static constexpr bool half = true; };

template <typename R, typename S> TP_DEV cx<R> ld(const S* p) {
  S v = *p;
  return {R(v.x), R(v.y)};
}
template <> TP_DEV cx<float> ld<float, __half2>(const __half2* p) {
  float2 f = __half22float2(*p);
  return {f.x, f.y};
}
template <typename R> TP_DEV void st(double2* p, cx<R> v) { *p = make_double2(double(v.re), double(v.im)); }
template <typename R> TP_DEV void st(float2* p, cx<R> v) { *p = make_float2(float(v.re), float(v.im)); }
template <typename R> TP_DEV void st(__half2* p, cx<R> v) { *p = __floats2half2_rn(float(v.re), float(v.im)); }

// ---- field storage --------------------------------------------------------------------------
// A field of n complex components per site is stored as planes of `stride` sites.  FP32 and
// FP16 fields pair the planes (2k, 2k+1): the two values of one site are adjacent, so a
// single 16-byte (FP32) or 8-byte (FP16) load fetches both, halving the load instructions of
// the bandwidth-bound kernels.  A last odd plane (links: 9 components) stays single.  FP64
// fields keep one plane per component (a pair would exceed one 16-byte load).
template <typename T> TP_HD constexpr bool paired() { return sizeof(T) <= 8; }
template <typename T> TP_HD int64_t comp_off(int c, int n, int64_t stride, int64_t i) {
  if (paired<T>() && c < (n & ~1)) return (int64_t)(c & ~1) * stride + 2 * i + (c & 1);
  return (int64_t)c * stride + i;
}
// Two adjacent components of a paired field: p points at the even one.
template <typename R, typename T> TP_DEV void ld2(const T* p, cx<R>& a, cx<R>& b);
template <> TP_DEV void ld2<float, float2>(const float2* p, cx<float>& a, cx<float>& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = {v.x, v.y};
  b = {v.z, v.w};
}
struct alignas(8) Half2x2 { __half2 a, b; };
template <> TP_DEV void ld2<float, __half2>(const __half2* p, cx<float>& a, cx<float>& b) {
  const Half2x2 v = *reinterpret_cast<const Half2x2*>(p);
  const float2 fa = __half22float2(v.a), fb = __half22float2(v.b);
  a = {fa.x, fa.y};
  b = {fb.x, fb.y};
}
template <typename R> TP_DEV void st2(float2* p, cx<R> a, cx<R> b) {
  *reinterpret_cast<float4*>(p) = make_float4(float(a.re), float(a.im), float(b.re), float(b.im));
}
template <typename R> TP_DEV void st2(__half2* p, cx<R> a, cx<R> b) {
  Half2x2 v;
  v.a = __floats2half2_rn(float(a.re), float(a.im));
  v.b = __floats2half2_rn(float(b.re), float(b.im));
  *reinterpret_cast<Half2x2*>(p) = v;
}

// A spinor field of one parity, seen as two half-spinor fields: h = 0 holds spins
// 0-1 (the P+ = (1+gamma_t)/2 subspace in the Dirac-Pauli basis), h = 1 spins 2-3.
// Each half is 6 components [6][stride] (component = spin_in_half*3 + colour, paired as
// above for FP32 / FP16); for FP16,
// nrm[h] holds one FP32 scale per site.  The two halves may live in different
// buffers, so a field can be assembled from the halves of two others.
template <typename S>
struct SpinorF {
  S* p[2];
  float* nrm[2];
  int64_t stride;
};
// Field r of a batch of fields allocated back to back (24 planes of `stride` sites and 4
// scale planes apart): the right-hand sides of a batched solve share one launch.
template <typename S> TP_DEV SpinorF<S> rhs_view(SpinorF<S> f, uint32_t r) {
  const int64_t e = (int64_t)r * 24 * f.stride, n = (int64_t)r * 4 * f.stride;
  if (f.p[0]) f.p[0] += e;
  if (f.p[1]) f.p[1] += e;
  if (f.nrm[0]) f.nrm[0] += n;
  if (f.nrm[1]) f.nrm[1] += n;
  return f;
}

// Element i of a plane, addressed as plane + a 32-bit byte offset: with the plane pointer
// uniform across the wavefront this is the scalar-base + vector-offset load form, with no
// per-load 64-bit address arithmetic.  Every field here is below 2^32 bytes per plane
// (the context limits the volume to 2^29 sites).
template <typename T> TP_DEV const T* at(const T* plane, uint32_t i) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + uint32_t(i * uint32_t(sizeof(T))));
}
template <typename T> TP_DEV T* at(T* plane, uint32_t i) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + uint32_t(i * uint32_t(sizeof(T))));
}

template <typename S, typename R = typename Prec<S>::R>
TP_DEV void load_half(const SpinorF<S>& f, int h, uint32_t i, cx<R>* v) {
  const S* b = f.p[h];
  if constexpr (paired<S>()) {
#pragma unroll
    for (int q = 0; q < 3; ++q) ld2<R, S>(at(b + (int64_t)(2 * q) * f.stride, 2 * i), v[2 * q], v[2 * q + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = ld<R, S>(at(b + (int64_t)c * f.stride, i));
  }
  if constexpr (Prec<S>::half) {
    R s = *at(f.nrm[h], i);
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = s * v[c];
  }
}

template <typename S, typename R = typename Prec<S>::R>
TP_DEV void store_half(const SpinorF<S>& f, int h, uint32_t i, const cx<R>* v) {
  S* b = f.p[h];
  if constexpr (Prec<S>::half) {
    R m = R(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    // below the smallest normal FP32 value 1/m would overflow (a point source decaying as
    // mu^-t along a long line gets there): such a half spinor is stored as zero.  A NaN
    // fails the comparison and propagates.
    if (m < R(1.17549435e-38f)) m = R(0);
    R inv = m > R(0) ? R(1) / m : R(0);
#pragma unroll
    for (int q = 0; q < 3; ++q) st2(at(b + (int64_t)(2 * q) * f.stride, 2 * i), inv * v[2 * q], inv * v[2 * q + 1]);
    *at(f.nrm[h], i) = m;
  } else if constexpr (paired<S>()) {
#pragma unroll
    for (int q = 0; q < 3; ++q) st2(at(b + (int64_t)(2 * q) * f.stride, 2 * i), v[2 * q], v[2 * q + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) st(at(b + (int64_t)c * f.stride, i), v[c]);
  }
}

// The same with a 64-bit site index and 64-bit addresses (the line kernels, whose
// register budget is better spent elsewhere than on uniform plane bases).
template <typename S, typename R = typename Prec<S>::R>
TP_DEV void load_half(const SpinorF<S>& f, int h, int64_t i, cx<R>* v) {
  const S* b = f.p[h];
  if constexpr (paired<S>()) {
#pragma unroll
    for (int q = 0; q < 3; ++q) ld2<R, S>(b + (int64_t)(2 * q) * f.stride + 2 * i, v[2 * q], v[2 * q + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = ld<R, S>(b + (int64_t)c * f.stride + i);
  }
  if constexpr (Prec<S>::half) {
    R s = f.nrm[h][i];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = s * v[c];
  }
}
template <typename S, typename R = typename Prec<S>::R>
TP_DEV void store_half(const SpinorF<S>& f, int h, int64_t i, const cx<R>* v) {
  S* b = f.p[h];
  if constexpr (Prec<S>::half) {
    R m = R(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    // below the smallest normal FP32 value 1/m would overflow (a point source decaying as
    // mu^-t along a long line gets there): such a half spinor is stored as zero.  A NaN
    // fails the comparison and propagates.
    if (m < R(1.17549435e-38f)) m = R(0);
    R inv = m > R(0) ? R(1) / m : R(0);
#pragma unroll
    for (int q = 0; q < 3; ++q) st2(b + (int64_t)(2 * q) * f.stride + 2 * i, inv * v[2 * q], inv * v[2 * q + 1]);
    f.nrm[h][i] = m;
  } else if constexpr (paired<S>()) {
#pragma unroll
    for (int q = 0; q < 3; ++q) st2(b + (int64_t)(2 * q) * f.stride + 2 * i, v[2 * q], v[2 * q + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) st(b + (int64_t)c * f.stride + i, v[c]);
  }
}

template <typename S, typename R = typename Prec<S>::R>
TP_DEV void load_spinor(const SpinorF<S>& f, uint32_t i, cx<R>* v) {
  load_half<S, R>(f, 0, i, v);
  load_half<S, R>(f, 1, i, v + 6);
}
template <typename S, typename R = typename Prec<S>::R>
TP_DEV void store_spinor(const SpinorF<S>& f, uint32_t i, const cx<R>* v) {
  store_half<S, R>(f, 0, i, v);
  store_half<S, R>(f, 1, i, v + 6);
}

// Gauge links of one parity and direction: planes [9][stride].
template <typename L>
struct LinkF {
  const L* p;
  int64_t stride;
};
// The third row of an SU(3) matrix from its first two: the rows are orthonormal with unit
// determinant, so the third row is the complex conjugate of the cross product of the first two.
template <typename R> TP_DEV void su3_third_row(su3<R>& u) {
  const cx<R>* a = u.e;
  const cx<R>* b = u.e + 3;
  u.e[6] = conj(cmul(a[1], b[2]) - cmul(a[2], b[1]));
  u.e[7] = conj(cmul(a[2], b[0]) - cmul(a[0], b[2]));
  u.e[8] = conj(cmul(a[0], b[1]) - cmul(a[1], b[0]));
}
// ROWS = 3 reads all nine entries; ROWS = 2 reads the first two rows of an SU(3) link and
// rebuilds the third.
template <typename R, typename L, int ROWS = 3>
TP_DEV su3<R> load_su3(const LinkF<L>& f, uint32_t i) {
  su3<R> u;
  if constexpr (paired<L>()) {
    constexpr int npair = ROWS == 2 ? 3 : 4;
#pragma unroll
    for (int q = 0; q < npair; ++q) ld2<R, L>(at(f.p + (int64_t)(2 * q) * f.stride, 2 * i), u.e[2 * q], u.e[2 * q + 1]);
    if constexpr (ROWS == 3) u.e[8] = ld<R, L>(at(f.p + (int64_t)8 * f.stride, i));
  } else {
#pragma unroll
    for (int k = 0; k < 3 * ROWS; ++k) u.e[k] = ld<R, L>(at(f.p + (int64_t)k * f.stride, i));
  }
  if constexpr (ROWS == 2) su3_third_row(u);
  return u;
}

// ---- Dirac-Pauli spin structure --------------------------------------------------------
// gamma_t = diag(1,1,-1,-1); gamma_k = [[0, -i s_k], [i s_k, 0]].
// (1 -+ gamma_k) psi = (h, -+ i s_k h) with h = psi_up +- i s_k psi_lo, so a
// projected hop needs two colour matvecs on h and a reconstruction.
// i s_x (a, b) = (i b, i a);  i s_y (a, b) = (b, -a);  i s_z (a, b) = (i a, -i b).
template <int K, typename R> TP_DEV void is_k(const cx<R>* a, const cx<R>* b, cx<R>* oa, cx<R>* ob) {
  // (oa, ob) = i sigma_K (a, b), each a colour vector (3 components)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (K == 0) { oa[c] = ti(b[c]); ob[c] = ti(a[c]); }
    else if constexpr (K == 1) { oa[c] = b[c]; ob[c] = -a[c]; }
    else { oa[c] = ti(a[c]); ob[c] = tmi(b[c]); }
  }
}

// Half spinor for the forward hop in spatial direction K: h = psi_up + i s_K psi_lo.
template <int K, typename R> TP_DEV void proj_minus(const cx<R>* psi, cx<R>* h) {
  cx<R> a[3], b[3];
  is_k<K, R>(psi + 6, psi + 9, a, b);
#pragma unroll
  for (int c = 0; c < 3; ++c) { h[c] = psi[c] + a[c]; h[3 + c] = psi[3 + c] + b[c]; }
}
// Backward hop: h = psi_up - i s_K psi_lo.
template <int K, typename R> TP_DEV void proj_plus(const cx<R>* psi, cx<R>* h) {
  cx<R> a[3], b[3];
  is_k<K, R>(psi + 6, psi + 9, a, b);
#pragma unroll
  for (int c = 0; c < 3; ++c) { h[c] = psi[c] - a[c]; h[3 + c] = psi[3 + c] - b[c]; }
}
// out += w * (1 - gamma_K)/2-reconstruction of the transported half spinor g:
// upper += g, lower += -i s_K g   (forward hop), times the overall factor w.
template <int K, typename R> TP_DEV void recon_minus(cx<R>* out, const cx<R>* g, R w) {
  cx<R> a[3], b[3];
  is_k<K, R>(g, g + 3, a, b);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[c] += w * g[c];
    out[3 + c] += w * g[3 + c];
    out[6 + c] -= w * a[c];
    out[9 + c] -= w * b[c];
  }
}
// Backward: upper += g, lower += +i s_K g.
template <int K, typename R> TP_DEV void recon_plus(cx<R>* out, const cx<R>* g, R w) {
  cx<R> a[3], b[3];
  is_k<K, R>(g, g + 3, a, b);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[c] += w * g[c];
    out[3 + c] += w * g[3 + c];
    out[6 + c] += w * a[c];
    out[9 + c] += w * b[c];
  }
}

// ---- clover blocks -------------------------------------------------------------------------
// A commutes with gamma5 = [[0,-1],[-1,0]] and is stored as two hermitian 6x6 blocks
// acting on u+ = psi_up - psi_lo and u- = psi_up + psi_lo (index spin_in_pair*3 + colour),
// pre-multiplied by 1/2 so that
//   (A psi)_up = B+ u+ + B- u-,   (A psi)_lo = B- u- - B+ u+.
// Per block: 18 complex slots (36 components per site, paired for FP32 / FP16).
// out = B v for one hermitian 6x6 block from its 18 slots: slots 0..2 hold the six real
// diagonal entries in pairs, slots 3..17 the strictly lower triangle in row-major order.
template <typename R>
TP_DEV void herm6_from_slots(const cx<R>* sl, const cx<R>* v, cx<R>* out) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out[2 * k] = sl[k].re * v[2 * k];
    out[2 * k + 1] = sl[k].im * v[2 * k + 1];
  }
  int slot = 3;
#pragma unroll
  for (int r = 1; r < 6; ++r) {
#pragma unroll
    for (int c = 0; c < r; ++c) {
      out[r] += cmul(sl[slot], v[c]);
      out[c] += cmulc(sl[slot], v[r]);
      ++slot;
    }
  }
}

// The 18 slots of the block whose planes start at `base` (an even component index).
template <typename R, typename L>
TP_DEV void herm6_slots(const L* base, int64_t stride, uint32_t i, cx<R>* sl) {
  if constexpr (paired<L>()) {
#pragma unroll
    for (int q = 0; q < 9; ++q) ld2<R, L>(at(base + (int64_t)(2 * q) * stride, 2 * i), sl[2 * q], sl[2 * q + 1]);
  } else {
#pragma unroll
    for (int k = 0; k < 18; ++k) sl[k] = ld<R, L>(at(base + (int64_t)k * stride, i));
  }
}
template <typename R, typename L>
TP_DEV void herm6_slots(const L* base, int64_t stride, int64_t i, cx<R>* sl) {
  if constexpr (paired<L>()) {
#pragma unroll
    for (int q = 0; q < 9; ++q) ld2<R, L>(base + (int64_t)(2 * q) * stride + 2 * i, sl[2 * q], sl[2 * q + 1]);
  } else {
#pragma unroll
    for (int k = 0; k < 18; ++k) sl[k] = ld<R, L>(base + (int64_t)k * stride + i);
  }
}

// A psi for the clover term stored as two chiral blocks acting on psi_up -+ psi_lo
// (planes [36][stride], block c at component 18c), with I = uint32_t (uniform plane
// addressing) or int64_t.
template <typename R, typename L, typename I>
TP_DEV void clover_apply(const L* cl, int64_t stride, I i, const cx<R>* psi, cx<R>* out) {
  cx<R> up[6], um[6], bp[6], bm[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) { up[c] = psi[c] - psi[6 + c]; um[c] = psi[c] + psi[6 + c]; }
  {
    cx<R> sl[18];
    herm6_slots<R, L>(cl, stride, i, sl);
    herm6_from_slots<R>(sl, up, bp);
  }
  {
    cx<R> sl[18];
    herm6_slots<R, L>(cl + 18 * stride, stride, i, sl);
    herm6_from_slots<R>(sl, um, bm);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) { out[c] = bp[c] + bm[c]; out[6 + c] = bm[c] - bp[c]; }
}

// ---- lattice geometry ----------------------------------------------------------------------
// p3 ("line") layout: parity p = (x+y+z)&1; spatial index s = (x + Lx*(y + Ly*z)) >> 1;
// a time line (fixed s) stays inside one parity.  Lines are grouped in tiles of 4 and
// a tile stores all its time slices contiguously:
//   index(t, s) = ((s / 4) * Lt + t) * 4 + s % 4,
// so a workgroup that owns whole lines reads and writes contiguous memory in thread
// order.  Vs/2 is always a multiple of 4 (every spatial extent is even).
// p4 layout: parity p = (x+y+z+t)&1; index = (x + Lx*(y + Ly*(z + Lz*t))) >> 1.
struct Geom {
  int Lx, Ly, Lz, Lt;
  int Lxh, Vs2;
  int64_t V2;
};

struct C3 { int x, y, z; };
TP_DEV C3 p3_coords(const Geom& g, int p, int s) {
  int xh = s % g.Lxh;
  int r = s / g.Lxh;
  int y = r % g.Ly;
  int z = r / g.Ly;
  int x = 2 * xh + ((y + z + p) & 1);
  return {x, y, z};
}
TP_DEV int p3_index(const Geom& g, int x, int y, int z) { return (x + g.Lx * (y + g.Ly * z)) >> 1; }
constexpr int kTile = 4;
TP_HD int64_t p3_idx(const Geom& g, int t, int s) {
  return ((int64_t)(s >> 2) * g.Lt + t) * kTile + (s & 3);
}
TP_DEV uint32_t p3_idx32(const Geom& g, int t, int s) {
  return (uint32_t(s >> 2) * uint32_t(g.Lt) + uint32_t(t)) * kTile + uint32_t(s & 3);
}
TP_DEV void p3_ts32(const Geom& g, uint32_t i, int& t, int& s) {
  const uint32_t per = uint32_t(kTile) * uint32_t(g.Lt);
  const uint32_t tile = i / per;
  const uint32_t r = i - tile * per;
  t = int(r >> 2);
  s = int(tile * kTile + (r & 3));
}
TP_HD void p3_ts(const Geom& g, int64_t i, int& t, int& s) {
  int64_t tile = i / ((int64_t)kTile * g.Lt);
  int r = int(i - tile * kTile * g.Lt);
  t = r >> 2;
  s = int(tile * kTile) + (r & 3);
}
