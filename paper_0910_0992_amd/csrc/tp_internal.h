// Host-side internals of the tprec library: handle structures, internal field
// descriptors, kernel launcher declarations and error plumbing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>
#include <string>
#include <unordered_map>
#include <vector>

#include "tp_device.h"
#include "../../include/tprec.h"

// ---------------------------------------------------------------- errors
void tp_set_error(const std::string& msg);
struct TpError {
  tp_status code;
  std::string msg;
};
#define TP_THROW(code, msg) throw TpError{code, msg}
#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw TpError{e_ == hipErrorOutOfMemory ? TP_ENOMEM : TP_EHIP,                      \
                    std::string(#expr) + ": " + hipGetErrorString(e_)};                   \
  } while (0)
#define LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// ---------------------------------------------------------------- profiling ids
// One slot per kernel (or per pair of sweep kernels for KID_SCHUR3D_MEE).
enum KernelId {
  KID_PACK = 0,
  KID_SITE_P3,      // M / D_s / clover / residual on the p3 layout
  KID_SCHUR4D_EO,   // (A+mu)^-1 D_w^eo
  KID_SCHUR4D_OE,   // (A+mu) psi_o - D_w^oe t_e (and the other p4 site kernels)
  KID_SCAN_CR,      // C_R scans
  KID_SCAN_CL,      // C_L scans
  KID_SCAN_OTHER,   // C_R C_L, T^-1 and T^dag^-1 scans
  KID_ILU_MID,      // fused scans + clover of the 3D ILU operator (even parity)
  KID_HOP_DS,       // D_s hop feeding the scans (no clover)
  KID_HOP_CLOVER,   // A self + D_s hop feeding the scans
  KID_BLAS_DOT,     // <x, y>
  KID_BLAS_AXPYZ,   // z = y + a x with |z|^2
  KID_BLAS_DOT4,    // <t,s>, |t|^2, <rhat,s>, <rhat,t>
  KID_BLAS_FUSED,   // BiCGStab x, r, p update with |r|^2
  KID_BLAS_OTHER,   // every other level-1 kernel
  KID_REDUCE,
  KID_FORCE,
  KID_SCHUR3D_MEE,  // exact (A + mu - D_t)^-1: forward and backward block-LU sweeps
  KID_COUNT
};
extern const char* const kKernelNames[KID_COUNT];

// ---------------------------------------------------------------- internal fields
// A spinor field in an internal layout (p3 or p4), both parities:
// data [2 parity][12 component][V2] of the storage type of `prec`,
// nrm [2 parity][2 half][V2] FP32 scales for TP_F16N (else null).
// A batch of nr such fields is one allocation of nr consecutive fields (kernels offset by
// the right-hand-side index, see rhs_view); view(r) is field r alone.
struct Field {
  int prec = TP_F64;
  void* data = nullptr;
  float* nrm = nullptr;
  int64_t V2 = 0;
  int nr = 1;
  bool owned = false;

  size_t elem_bytes() const { return prec == TP_F64 ? 16 : (prec == TP_F32 ? 8 : 4); }
  template <typename S>
  SpinorF<S> par(int p) const {
    S* b = static_cast<S*>(data) + (int64_t)p * 12 * V2;
    SpinorF<S> f;
    f.p[0] = b;
    f.p[1] = b + 6 * V2;
    f.nrm[0] = nrm ? nrm + (int64_t)(2 * p) * V2 : nullptr;
    f.nrm[1] = nrm ? nrm + (int64_t)(2 * p + 1) * V2 : nullptr;
    f.stride = V2;
    return f;
  }
  Field view(int r) const {
    Field f = *this;
    f.data = static_cast<char*>(data) + (size_t)r * 24 * V2 * elem_bytes();
    f.nrm = nrm ? nrm + (int64_t)r * 4 * V2 : nullptr;
    f.nr = 1;
    f.owned = false;
    return f;
  }
};

// Geometry helpers shared by host launchers.
struct Lattice {
  int L[4];        // Lx, Ly, Lz, Lt
  int64_t V, V2;   // volume, half volume
  int Vs, Vs2;     // spatial volume, half
  Geom g;
};

// ---------------------------------------------------------------- handles
struct ProfSlot {
  int64_t launches = 0;
  double ms = 0;
  double bytes = 0;
};

struct tp_ctx_s {
  Lattice lat;
  int bc = -1;
  int device = 0;
  size_t lds_max = 65536;  // LDS bytes a workgroup may allocate on this device
  hipStream_t stream = nullptr;
  bool prof = false;
  uint32_t prof_mask = 0xffffffffu;  // kernel groups that record events while prof is on
  ProfSlot prof_slots[KID_COUNT];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  struct EvRec { int kid; double bytes; bool done; };
  std::vector<EvRec> ev_pending;  // per used event pair
  size_t ev_used = 0;
  // reduction scratch
  double* red_partial = nullptr;  // [kRedBlocks][8]
  double* red_result = nullptr;   // [8]
  double* red_host = nullptr;     // pinned [8]
  // BiCGStab scalars kept on the device (inside red_result's allocation): see BicgSlot
  double* bicg = nullptr;
  // device memory: registered allocator (null: hipMalloc), live allocations and their sizes
  tp_alloc_fn alloc_fn = nullptr;
  tp_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  std::unordered_map<void*, size_t> live;
  size_t live_bytes = 0;
  int nchildren = 0;  // gauge fields created from this context and not yet destroyed
  // device address of the library's fixed scratch array on this context's device
  // (tp_apply_prec_noalloc)
  char* scratch = nullptr;
};

struct tp_gauge_s {
  tp_ctx ctx = nullptr;
  double2* canon = nullptr;  // device copy of the canonical links [4][V][9]
  // p3 layout [4 dir][2 par][9][V2] in the axial gauge W(x)^dag U(x) W(x+mu): interior
  // time links are the identity, U_t(Lt-1) = P (Polyakov loop with the phase b)
  double2* u3_d = nullptr;
  float2* u3_f = nullptr;
  __half2* u3_h = nullptr;   // FP16 copy of u3 for the F16N operators
  double2* u4_d = nullptr;   // p4 layout [4 dir][2 par][9][V2], time phase folded
  float2* u4_f = nullptr;
  double2* w_d = nullptr;    // p3 layout W(t) = U(t)...U(Lt-1) [2 par][9][V2], FP64
  double2* canon_ax = nullptr;  // axial-gauge links, canonical order (clover build)
  double2* poly = nullptr;   // W(0) per line [2 par][9][Vs2]
  // every axial-frame spatial link is SU(3) to 1e-9: FP32/FP16 kernels read two rows
  bool su3_spatial = false;
  // ... and to 1e-13: the FP64 site kernels read two rows as well (the rebuilt third row is
  // then exact to that level)
  bool su3_spatial_f64 = false;
};

struct tp_clover_s {
  tp_gauge g = nullptr;
  double cs = 0, ct = 0;
  double2* a3_d = nullptr;  // p3 layout chiral blocks of A/2 [2 par][36][V2]
  float2* a3_f = nullptr;
  __half2* a3_h = nullptr;  // FP16 copy for the F16N operators
  double2* a4_d = nullptr;  // p4 layout chiral blocks of A/2 [2 par][36][V2]
  float2* a4_f = nullptr;
};

struct Workspace;

struct tp_op_s {
  tp_gauge g = nullptr;
  tp_clover c = nullptr;
  double m0 = 0, gf = 1, mu = 1;
  // cutoff trick (tp_op_set_cutoff): time slices whose Woodbury correction the scans drop
  // (T^-1: t < cut; T^dagger^-1: t >= Lt - cut); 0 keeps the exact inverse
  int cut = 0;
  double2* gclos = nullptr;  // per line G = (I - mu^-Lt P)^-1 P / mu  [2 par][9][Vs2]
  float2* gclos_f = nullptr;  // the same, rounded to FP32 (for the FP32 and FP16 scans)
  double2* a4_mu = nullptr;     // p4 (A+mu)/2 chiral blocks [2][36][V2]
  double2* a4_inv = nullptr;    // p4 (A+mu)^-1 / 2 chiral blocks [2][36][V2]
  float2* a4_mu_f = nullptr;
  float2* a4_inv_f = nullptr;
  double2* a3_mu = nullptr;     // p3 (A+mu)/2 and (A+mu)^-1/2 for apply checks
  double2* a3_inv = nullptr;
  float2* a3_mu_f = nullptr;
  float2* a3_inv_f = nullptr;
  __half2* a3_mu_h = nullptr;
  __half2* a3_inv_h = nullptr;
  double* mupow_d = nullptr;    // mu^-k, k = 0..Lt
  float* mupow_f = nullptr;
  // exact inverse of A + mu - D_t per p3 parity (FP64, built on first use; the even parity
  // serves the 3D-Schur scheme, both the whole-lattice full-SW scheme):
  double2* s3_inv[2] = {};  // block-LU S(t)^-1 [tile][t][12 col][12 row][4 line]
  double2* s3_k[2] = {};    // Woodbury capacitance K per line [Vs2][12][12]
  double2* s3_q[2] = {};    // boundary values W^dag T0^-1 eta [Vs2][12] (set-up: [12][Vs2][12])
  float2* s3_inv_f[2] = {};  // the factors rounded to FP32 for the FP32 operator
  float2* s3_k_f[2] = {};
  float2* s3_q_f[2] = {};
  Workspace* ws = nullptr;
  int batch_nr = 1;  // right-hand sides of the batched apply in progress (workspace size)
  // No-allocation mode (tp_apply_prec_noalloc): while arena is set, workspace fields are
  // carved from that fixed device region for the duration of one call instead of being
  // allocated; at most kArenaSlots distinct fields.
  struct ArenaSlot {
    int prec, slot, nr;
    Field f;
  };
  static constexpr int kArenaSlots = 16;
  char* arena = nullptr;
  size_t arena_cap = 0, arena_top = 0;
  ArenaSlot arena_slots[kArenaSlots];
  int arena_n = 0;
};

// ---------------------------------------------------------------- memory helpers
// Device memory of a context and of the handles created from it: through the allocator
// registered with tp_ctx_set_allocator, else hipMalloc / hipFree.  Fields are zeroed on the
// context's stream.
void* dev_alloc(tp_ctx ctx, size_t bytes);
void dev_free(tp_ctx ctx, void* p);
Field field_alloc(tp_ctx ctx, int prec, int nr = 1);
void field_free(tp_ctx ctx, Field& f);
// Device bytes of one field of `prec` (data, and the FP32 scales of F16N), 256-byte aligned.
size_t field_bytes(const Lattice& lat, int prec, int nr = 1);

// ---------------------------------------------------------------- profiling helpers
struct ProfScope {
  tp_ctx ctx;
  int kid;
  double bytes;
  size_t slot;
  bool on;
  ProfScope(tp_ctx c, int k, double b);
  ~ProfScope();
};
void prof_flush(tp_ctx ctx);

// ---------------------------------------------------------------- launchers (layout / setup)
// pack canonical c128 spinor (device) into an internal field; layout4 selects p4; w (p3
// only) rotates into the axial frame, psi -> W^dag psi (unpack: psi -> W psi).
void launch_pack(tp_ctx ctx, const double2* canon, Field& dst, bool layout4, bool gamma5,
                 const double2* w);
void launch_unpack(tp_ctx ctx, const Field& src, double2* canon, bool layout4, bool gamma5,
                   const double2* w);
void launch_pack_links(tp_ctx ctx, tp_gauge g);   // p4 layout (original frame)
void launch_wline(tp_ctx ctx, tp_gauge g);        // W(t), P from the canonical links
// p3 layout, axial frame.  flags: three device ints zeroed by the caller; [0] is set when an
// axial-frame spatial link deviates from SU(3) by more than 1e-9, [1] when a time link
// deviates from unitarity by more than 1e-10, [2] when an input entry is NaN or Inf
void launch_axial_links(tp_ctx ctx, tp_gauge g, int* flags);
// dst = src rounded to FP16 (n complex values)
void launch_to_half(tp_ctx ctx, const float2* src, __half2* dst, int64_t n);
void launch_closure(tp_ctx ctx, tp_op op, double* cond_out /*device [2*Vs2]*/);
void launch_clover_build(tp_ctx ctx, tp_clover c, const double sig[6][2][2][2][2]);
void launch_clover_derived(tp_ctx ctx, tp_op op, int* bad /*device counter*/);
void launch_plaquette(tp_ctx ctx, tp_gauge g, double* out2 /*device partial sums*/);

// ---------------------------------------------------------------- launchers (operators)
// p3 site kernel: dst = c_mu*src + c_A*(A src) + c_t*(D_t src) + c_s*(D_s src) + c_in*in2,
// for parities [par0, par0+npar); optional |dst|^2 into the reduction scratch.
struct SiteCoef {
  double c_mu, c_A, c_t, c_s, c_in;
};
// Returns the number of reduction partials written (0 unless want_norm).
int launch_site_p3(tp_op op, int prec, const Field& src, Field& dst, const Field* in2,
                   SiteCoef cf, int clover_kind /*0 none,1 A,2 (A+mu),3 (A+mu)^-1*/,
                   int par0, int npar, bool want_norm);

// 4D Schur pieces on the p4 layout (FP64 and FP32 storage).
//   mode 0: dst_e = (A+mu)^-1 (c_h D_w^eo src_o)              [clover after hop]
//   mode 1: dst_o = (A+mu) src_o + c_h D_w^oe t_e             [clover on self]
//   mode 2: dst_p = c_in*in2_p + c_h D_w src_(1-p)            [plain hop + axpy]
//   mode 3: dst_p = (A+mu)^-1 (in2_p + c_h D_w src_(1-p))     [reconstruction]
//   mode 4: dst_p = clover(in2_p) with clover_kind             [site only]
void launch_schur4d(tp_op op, int prec, int mode, int out_par, const Field* src, Field& dst,
                    const Field* in2, double c_h, double c_in, int clover_kind);

// Line (time-line scan) kernels on the p3 layout.
enum LineMode { LM_CL = 0, LM_CR = 1, LM_CRCL = 2, LM_TINV = 3, LM_TDINV = 4 };
// dst = c_out MODE(in) + c_base base on parity par.  The input's halves may come from
// different fields; halves that MODE does not scan pass through when `pass`, else they
// are not written.
struct LineIO {
  const Field* in_up = nullptr;
  const Field* in_lo = nullptr;
  const Field* base = nullptr;
  double c_out = 1.0, c_base = 1.0;
  bool pass = true;
};
void launch_line(tp_op op, int prec, int mode, int par, const LineIO& io, Field& dst);
// Fused middle step of the 3D ILU operator (even parity): from psi_e and
// u = D_s^eo a_o / gamma_f, chi_e = psi_e + C_L y and n_e = C_R C_L (y - u) with
// y = A C_R (C_L u + psi_e).
void launch_ilu_mid(tp_op op, int prec, const Field& psi, const Field& u, Field& chi, Field& n);
// Exact T^-1, T = A + mu - D_t on the sites of one p3 parity (M^ee on the even sites): block
// LU of each time line plus a rank-12 Woodbury correction for the wrapping hops.
// schur3d_setup builds the FP64 factors of parity par once per operator (TP_ESINGULAR on a
// zero pivot); schur3d_ready tells whether those of precision prec exist.
// launch_tinv writes dst_p = T^-1 src_p on the parities par0 .. par0+npar-1 per right-hand
// side in F64, or in F32 with the factors rounded to FP32 on first use (w: work field of the
// same precision and batch size).  With base given it writes dst_p = base_p - T^-1 src_p.
// launch_mee_inv is the even-parity case.
void schur3d_setup(tp_op op, int par);
bool schur3d_ready(tp_op op, int prec, int par);
void schur3d_free(tp_op op);
void launch_tinv(tp_op op, int par0, int npar, const Field& src, Field& dst, Field& w,
                 const Field* base = nullptr);
void launch_mee_inv(tp_op op, const Field& src, Field& dst, Field& w);

// Site kernel with operands assembled from half fields: for output parity p,
//   dst = c_mu self + c_A A self + c_t D_t self + c_s D_s nb + c_in in2,
// self (and in2) read on parity p, nb on parity 1-p.
struct SiteIO {
  const Field* self_up = nullptr;
  const Field* self_lo = nullptr;
  const Field* nb_up = nullptr;
  const Field* nb_lo = nullptr;
  const Field* in2 = nullptr;
};
int launch_site(tp_op op, int prec, const SiteIO& io, Field& dst, SiteCoef cf, int clover_kind,
                int par0, int npar, bool want_norm);
double spinor_bytes(int prec);
double link_bytes(int prec);
double clov_bytes(int prec);

// ---------------------------------------------------------------- BLAS
constexpr int kRedBlocks = 32768;  // one block per 256 sites of a parity at 32^3x256 (fused norms)
constexpr int kMaxRhs = 16;  // right-hand sides of one batched solve
// Generic unit-wise BLAS on fields over parities [par0, par0+npar).
enum BlasOp {
  B_ZERO,         // y = 0
  B_COPY,         // y = x                          (same precision)
  B_CONVERT,      // y = x                          (any precisions)
  B_AXPY,         // y = y + a x                    (a complex)
  B_XPAY,         // y = x + a y
  B_NORM2,        // |x|^2
  B_DOT,          // <x, y>
  B_DOT_NORM,     // <x, y>, |y|^2
  B_CAXPY_NORM,   // y = y + a x ; |y|^2
  B_AXPYZ_NORM,   // z = y + a x ; |z|^2            (s = r - alpha v)
  B_DOT4_TS,      // <t, s>, |t|^2, <rhat, s>, <rhat, t>   (fields t, s, rhat)
  B_BICG_FUSED,   // x += a p + b s ; r = s - b t ; p = r + c (p - b v) ; |r|^2
                  //                                (fields x, p, s, t, v, r)
  B_G5,           // y = gamma5 x
  B_MIXED_ACC,    // y(F64) += x(any)
  B_MIXED_ADD     // y = z + x (fields x, z, y; z and y of one precision, x any)
};
// Device-resident BiCGStab scalars (doubles in tp_ctx_s::bicg): the reduction that ends a
// level-1 op can turn its results into the next op's coefficients without a host round trip.
enum BicgSlot {
  BS_RHO = 0,      // rho = <rhat, r> (complex)
  BS_ALPHA = 2,    // alpha = rho / <rhat, v>
  BS_OMEGA = 4,    // omega = <t, s> / |t|^2
  BS_BETA = 6,     // beta = (rho_new / rho) (alpha / omega)
  BS_S2 = 8,       // |s|^2
  BS_R2 = 9,       // |r|^2 after the fused update
  BS_BREAK = 10,   // nonzero: |t|^2, omega or rho vanished or is not finite
  BS_AXPY = 16,    // coefficients (a, b, c) of s = r - alpha v
  BS_FUSED = 24,   // coefficients (alpha, omega, beta) of the fused update
  BS_COUNT = 32
};
enum BicgPost { BP_NONE, BP_RHO, BP_ALPHA, BP_S2, BP_OMEGA, BP_R2 };

struct BlasArgs {
  double a[2], b[2], c[2];  // complex coefficients
};
// fs: up to six fields (see each op); returns reduction values (up to 8 doubles, so
// red_out must hold 8)
// synchronously in red_out when the op reduces.
void blas(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fs,
          BlasArgs k = BlasArgs{}, double* red_out = nullptr);
// The same on batches of nr fields: per[r] (or k for all when null) are the coefficients of
// right-hand side r, skip[r] leaves it untouched (and its reductions zero); red_out holds
// [nr][8] values.
void blas_multi(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fs,
                const BlasArgs* per, const bool* skip, double* red_out, BlasArgs k = BlasArgs{});
// The same op with its coefficients (a, b, c as six doubles) read from device memory when
// dcoef is not null, and its reductions post-processed on the device by `post` (BicgPost);
// nothing is copied to the host and the host does not wait.
void blas_dev(tp_ctx ctx, BlasOp op, int par0, int npar, std::initializer_list<const Field*> fs,
              const double* dcoef, int post);
// Copies the BS_COUNT device scalars to out and waits for the stream.
void bicg_state(tp_ctx ctx, double* out);
// Sum of the first nblocks per-block partials written by a site kernel with want_norm.
double finish_norm(tp_ctx ctx, int nblocks);

// ---------------------------------------------------------------- force
// SW-term part of the link gradient (added to grad), sig = sigma_{mu nu} of planes 03 13 23 01 02 12
void launch_clover_force(tp_op op, const Field& x, const Field& lam, double2* grad, bool projected,
                         const double sig[6][4][4][2]);
void launch_force(tp_op op, const Field& x, const Field& lam, double2* grad, bool projected);

// ---------------------------------------------------------------- composite operators (ops.cpp)
void op_apply_M(tp_op op, int prec, const Field& src, Field& dst, bool dagger);
void op_apply_prec(tp_op op, int scheme, int prec, const Field& src, Field& dst, bool dagger);
// The operator N with Mt^dagger = gamma5 N gamma5: Mt itself for the gamma5-hermitian
// schemes, 1 - D_s T^-1 / gamma_f for TEMPORAL_FULLSW.
void op_apply_prec_adj(tp_op op, int scheme, int prec, const Field& src, Field& dst);
void op_apply_odd(tp_op op, int scheme, int prec, const Field& src, Field& dst, bool dagger);
bool scheme_sub(tp_op op, int scheme);
void op_prepare(tp_op op, int scheme, int prec, const Field& eta, Field& et);
void op_reconstruct(tp_op op, int scheme, int prec, const Field& y, Field& x);
bool scheme_layout4(int scheme);
// Workspace vectors (allocated lazily, owned by the op).
// Workspace field `slot` in `prec`, a batch of op->batch_nr fields (1 outside batched
// operator applications).
Field& ws_get(tp_op op, int prec, int slot);
Field& ws_get_n(tp_op op, int prec, int slot, int nr);
void ws_free(tp_op op);
