// C ABI of the tprec library: handle life cycle, argument checks, canonical
// <-> internal conversions around every apply, and the solve / force entry
// points.  Every entry point catches TpError and returns its status.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <mutex>
#include <vector>

#include "tp_internal.h"

tp_status op_solve(tp_op op, const tp_solve_params& P, Field& x64, const Field& eta64,
                   tp_solve_info& info);
tp_status op_solve_multi(tp_op op, const tp_solve_params& P, int nr, Field& x64, const Field& eta64,
                         tp_solve_info* info);

const char* const kKernelNames[KID_COUNT] = {
    "pack_unpack", "site_p3",   "schur4d_eo_clover_inv", "schur4d_oe_clover", "scan_cr",
    "scan_cl",     "scan_other", "ilu_mid",              "hop_ds",            "hop_clover",
    "blas_dot",    "blas_axpyz_norm", "blas_dot4",       "blas_bicg_fused",   "blas_other",
    "reduce_finish", "force",   "schur3d_mee"};

namespace {
thread_local std::string g_last_error;

template <typename F>
tp_status guard(F&& f) {
  try {
    f();
    g_last_error.clear();
    return TP_OK;
  } catch (const TpError& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return TP_ENOMEM;
  }
}

void check_prec(int prec) {
  if (prec != TP_F64 && prec != TP_F32 && prec != TP_F16N) TP_THROW(TP_EINVAL, "bad precision");
}
void check_scheme(int s) {
  if (s < TP_UNPREC || s > TP_TEMPORAL_FULLSW) TP_THROW(TP_EINVAL, "bad scheme");
}
// Schemes with an exact block inverse (SCHUR4D's (A+mu)^-1, the block-LU T^-1) run in F64
// and F32 only.
void check_scheme_prec(int scheme, int prec) {
  if (scheme == TP_SCHUR4D && prec == TP_F16N) TP_THROW(TP_EINVAL, "SCHUR4D supports F64 and F32");
  if (scheme == TP_TEMPORAL_SCHUR3D && prec == TP_F16N)
    TP_THROW(TP_EINVAL, "TEMPORAL_SCHUR3D runs in F64 and F32");
  if (scheme == TP_TEMPORAL_FULLSW && prec == TP_F16N)
    TP_THROW(TP_EINVAL, "TEMPORAL_FULLSW runs in F64 and F32");
}
void need(const void* p, const char* what) {
  if (!p) TP_THROW(TP_EINVAL, std::string("null pointer: ") + what);
}
void set_device(tp_ctx ctx) { HIP_CHECK(hipSetDevice(ctx->device)); }

// The spin matrices of the Dirac-Pauli basis and the chiral projections of
// sigma_{mu nu} used to build the clover blocks on the device.
typedef std::complex<double> zc;
void gammas(zc g[4][4][4]) {
  const zc I(0, 1);
  zc s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  for (int m = 0; m < 4; ++m)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) g[m][a][b] = 0;
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g[k][a][2 + b] = -I * s[k][a][b];
        g[k][2 + a][b] = I * s[k][a][b];
      }
  g[3][0][0] = g[3][1][1] = 1;
  g[3][2][2] = g[3][3][3] = -1;
}

// sig[p][chi][r][c] = coef_p * (V_chi^dag sigma_p V_chi)[r][c] / 2 with
// V_+ = (1, -1)/sqrt2 and V_- = (1, 1)/sqrt2 on the (upper, lower) spin pairs.
void clover_sigma_table(double cs, double ct, double sig[6][2][2][2][2]) {
  zc g[4][4][4];
  gammas(g);
  const int planes[6][2] = {{0, 3}, {1, 3}, {2, 3}, {0, 1}, {0, 2}, {1, 2}};
  for (int p = 0; p < 6; ++p) {
    int mu = planes[p][0], nu = planes[p][1];
    double coef = p < 3 ? -0.5 * ct : -0.5 * cs;
    zc sg[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        zc v = 0;
        for (int c = 0; c < 4; ++c) v += g[mu][a][c] * g[nu][c][b] - g[nu][a][c] * g[mu][c][b];
        sg[a][b] = 0.5 * v;
      }
    for (int chi = 0; chi < 2; ++chi) {
      double sgn = chi == 0 ? -1.0 : 1.0;  // V_+ lower component -1, V_- +1
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
          // (V^dag S V)[r][c] = (S[r][c] + sgn S[r][2+c] + sgn S[2+r][c] + S[2+r][2+c]) / 2
          zc v = 0.5 * (sg[r][c] + sgn * sg[r][2 + c] + sgn * sg[2 + r][c] + sg[2 + r][2 + c]);
          v *= 0.5 * coef;
          sig[p][chi][r][c][0] = v.real();
          sig[p][chi][r][c][1] = v.imag();
        }
    }
  }
}

// sigma_{mu nu} = [gamma_mu, gamma_nu]/2 for the planes 03 13 23 01 02 12
void sigma_planes(double out[6][4][4][2]) {
  zc g[4][4][4];
  gammas(g);
  const int planes[6][2] = {{0, 3}, {1, 3}, {2, 3}, {0, 1}, {0, 2}, {1, 2}};
  for (int p = 0; p < 6; ++p)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        zc v = 0;
        for (int c = 0; c < 4; ++c)
          v += g[planes[p][0]][a][c] * g[planes[p][1]][c][b] - g[planes[p][1]][a][c] * g[planes[p][0]][c][b];
        v *= 0.5;
        out[p][a][b][0] = v.real();
        out[p][a][b][1] = v.imag();
      }
}

Lattice make_lattice(const int32_t d[4]) {
  Lattice L;
  for (int k = 0; k < 4; ++k) L.L[k] = d[k];
  L.Vs = d[0] * d[1] * d[2];
  L.Vs2 = L.Vs / 2;
  L.V = (int64_t)L.Vs * d[3];
  L.V2 = L.V / 2;
  L.g.Lx = d[0];
  L.g.Ly = d[1];
  L.g.Lz = d[2];
  L.g.Lt = d[3];
  L.g.Lxh = d[0] / 2;
  L.g.Vs2 = L.Vs2;
  L.g.V2 = L.V2;
  return L;
}

Field& tmp_field(tp_op op, int prec, int k) { return ws_get(op, prec, 100 + k); }

}  // namespace

// ---------------------------------------------------------------- memory / profiling helpers
void tp_set_error(const std::string& m) { g_last_error = m; }

void* dev_alloc(tp_ctx ctx, size_t bytes) {
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  if (ctx->alloc_fn) {
    p = ctx->alloc_fn(bytes, ctx->stream, ctx->alloc_user);
    if (!p) TP_THROW(TP_ENOMEM, "registered allocator returned no memory");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      TP_THROW(e == hipErrorOutOfMemory ? TP_ENOMEM : TP_EHIP,
               std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  ctx->live[p] = bytes;
  ctx->live_bytes += bytes;
  return p;
}
void dev_free(tp_ctx ctx, void* p) {
  if (!p) return;
  size_t n = 0;
  auto it = ctx->live.find(p);
  if (it != ctx->live.end()) {
    n = it->second;
    ctx->live.erase(it);
    ctx->live_bytes -= n;
  }
  if (ctx->free_fn) ctx->free_fn(p, n, ctx->stream, ctx->alloc_user);
  else (void)hipFree(p);
}

size_t field_bytes(const Lattice& lat, int prec, int nr) {
  const size_t eb = prec == TP_F64 ? 16 : (prec == TP_F32 ? 8 : 4);
  size_t db = (size_t(nr) * 2 * 12 * lat.V2 * eb + 255) & ~size_t(255);
  if (prec == TP_F16N) db += (size_t(nr) * 2 * 2 * lat.V2 * sizeof(float) + 255) & ~size_t(255);
  return db;
}

Field field_alloc(tp_ctx ctx, int prec, int nr) {
  const Lattice& lat = ctx->lat;
  Field f;
  f.prec = prec;
  f.V2 = lat.V2;
  f.nr = nr;
  const size_t db = size_t(nr) * 2 * 12 * lat.V2 * f.elem_bytes();
  f.data = dev_alloc(ctx, db);
  f.owned = true;
  HIP_CHECK(hipMemsetAsync(f.data, 0, db, ctx->stream));
  if (prec == TP_F16N) {
    const size_t nb = size_t(nr) * 2 * 2 * lat.V2 * sizeof(float);
    f.nrm = static_cast<float*>(dev_alloc(ctx, nb));
    HIP_CHECK(hipMemsetAsync(f.nrm, 0, nb, ctx->stream));
  }
  return f;
}
void field_free(tp_ctx ctx, Field& f) {
  if (f.owned) {
    dev_free(ctx, f.data);
    dev_free(ctx, f.nrm);
  }
  f.data = nullptr;
  f.nrm = nullptr;
}

ProfScope::ProfScope(tp_ctx c, int k, double b)
    : ctx(c), kid(k), bytes(b), slot(0), on(c && c->prof && ((c->prof_mask >> k) & 1u)) {
  if (!on) return;
  if (ctx->ev_used >= 4096) prof_flush(ctx);
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t a, e;
    HIP_CHECK(hipEventCreate(&a));
    HIP_CHECK(hipEventCreate(&e));
    ctx->ev_pool.push_back({a, e});
    ctx->ev_pending.push_back({0, 0.0, false});
  }
  slot = ctx->ev_used++;
  ctx->ev_pending[slot] = {kid, bytes, false};
  HIP_CHECK(hipEventRecord(ctx->ev_pool[slot].first, ctx->stream));
}
ProfScope::~ProfScope() {
  if (!on) return;
  (void)hipEventRecord(ctx->ev_pool[slot].second, ctx->stream);
  ctx->ev_pending[slot].done = true;
}

// Accumulates the recorded (start, stop) pairs.  While a profiled launch is still
// open (its stop event not yet recorded) nothing is flushed; a later call will.
void prof_flush(tp_ctx ctx) {
  if (!ctx || ctx->ev_used == 0) return;
  for (size_t k = 0; k < ctx->ev_used; ++k)
    if (!ctx->ev_pending[k].done) return;
  HIP_CHECK(hipEventSynchronize(ctx->ev_pool[ctx->ev_used - 1].second));
  for (size_t k = 0; k < ctx->ev_used; ++k) {
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev_pool[k].first, ctx->ev_pool[k].second));
    ProfSlot& s = ctx->prof_slots[ctx->ev_pending[k].kid];
    s.launches++;
    s.ms += ms;
    s.bytes += ctx->ev_pending[k].bytes;
  }
  ctx->ev_used = 0;
}

// ---------------------------------------------------------------- fixed scratch
// Device memory of tp_apply_prec_noalloc: a file-scope array that every device the library
// runs on holds from the library's first use on it until the process ends.  Host code
// never uses the array's name as an address: its device address is taken once per device
// with hipGetSymbolAddress (with that device current) at context creation, and kept.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
char* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device`, which must be the current device.
char* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) TP_THROW(TP_EINVAL, "device ordinal");
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) TP_THROW(TP_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[device] = static_cast<char*>(p);
  }
  return g_scratch_dev[device];
}

// Workspace fields an apply of `scheme` takes (the packed input and output, and the composite
// operator's temporaries), all of the apply's precision.
int noalloc_fields(int scheme) {
  switch (scheme) {
    case TP_UNPREC: return 2;
    case TP_SCHUR4D: return 3;
    case TP_TEMPORAL: return 4;
    case TP_TEMPORAL_SCHUR: return 6;
    case TP_TEMPORAL_FULLSW: return 4;
    default: return 7;  // TP_TEMPORAL_SCHUR3D
  }
}

// The context's own device buffers: reduction partials and results, and the solver's
// device-side scalars.
void ctx_buffers_alloc(tp_ctx c) {
  c->red_partial = static_cast<double*>(dev_alloc(c, sizeof(double) * 8 * kRedBlocks));
  c->red_result = static_cast<double*>(dev_alloc(c, sizeof(double) * (8 * kMaxRhs + BS_COUNT)));
  c->bicg = c->red_result + 8 * kMaxRhs;
  HIP_CHECK(hipMemsetAsync(c->bicg, 0, sizeof(double) * BS_COUNT, c->stream));
}
void ctx_buffers_free(tp_ctx c) {
  dev_free(c, c->red_partial);
  dev_free(c, c->red_result);
  c->red_partial = c->red_result = c->bicg = nullptr;
}

// Canonical-in / canonical-out wrapper for the internal applies.
template <typename F>
tp_status apply_wrap(tp_op op, int prec, void* dst, const void* src, bool l4, bool g5, F&& f) {
  return guard([&] {
    need(op, "op");
    need(dst, "dst");
    need(src, "src");
    check_prec(prec);
    if (dst == src) TP_THROW(TP_EINVAL, "dst and src must differ");
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    if (l4 && ctx->lat.L[3] % 2) TP_THROW(TP_EDIMS, "SCHUR4D needs an even time extent");
    Field& a = tmp_field(op, prec, 0);
    Field& b = tmp_field(op, prec, 1);
    const double2* w = l4 ? nullptr : op->g->w_d;  // p3 operators act in the axial frame
    launch_pack(ctx, static_cast<const double2*>(src), a, l4, g5, w);
    f(a, b);
    launch_unpack(ctx, b, static_cast<double2*>(dst), l4, g5, w);
  });
}


// ---------------------------------------------------------------- fields in the library's layouts
namespace {
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

void check_tpfield(tp_op op, const tp_field* f, const char* what) {
  need(f, what);
  need(f->data, what);
  if (f->nrhs < 1 || f->nrhs > kMaxRhs) TP_THROW(TP_EINVAL, std::string(what) + ": nrhs must be 1..16");
  if (f->layout < TP_LAYOUT_CANONICAL || f->layout > TP_LAYOUT_P4) TP_THROW(TP_EINVAL, std::string(what) + ": bad layout");
  if (f->subset < TP_SUBSET_FULL || f->subset > TP_SUBSET_ODD) TP_THROW(TP_EINVAL, std::string(what) + ": bad subset");
  if (f->layout == TP_LAYOUT_CANONICAL) {
    if (f->prec != TP_F64 || f->subset != TP_SUBSET_FULL)
      TP_THROW(TP_EINVAL, std::string(what) + ": canonical fields are F64 and FULL");
  } else {
    check_prec(f->prec);
  }
  if (f->layout == TP_LAYOUT_P4 && op->g->ctx->lat.L[3] % 2) TP_THROW(TP_EDIMS, "the P4 layout needs an even time extent");
}

size_t tpfield_bytes(const Lattice& L, int layout, int prec, int subset) {
  if (layout == TP_LAYOUT_CANONICAL) return size_t(L.V) * 12 * sizeof(double2);
  const size_t eb = prec == TP_F64 ? 16 : (prec == TP_F32 ? 8 : 4);
  const size_t npar = subset == TP_SUBSET_FULL ? 2 : 1;
  size_t b = al256(npar * 12 * L.V2 * eb);
  if (prec == TP_F16N) b += al256(npar * 2 * L.V2 * sizeof(float));
  return b;
}

// Right-hand side r of an internal field as a Field.  For a one-parity field, parity p of the
// view is the caller's buffer; the view is only used with kernels restricted to parity p
// (one-parity copies and conversions), so the other parity's addresses are never formed into
// accesses.
Field tpfield_view(const Lattice& L, const tp_field& f, int r) {
  Field v;
  v.prec = f.prec;
  v.V2 = L.V2;
  v.nr = 1;
  v.owned = false;
  const size_t per = tpfield_bytes(L, f.layout, f.prec, f.subset);
  const uintptr_t base = reinterpret_cast<uintptr_t>(f.data) + size_t(r) * per;
  const size_t npar = f.subset == TP_SUBSET_FULL ? 2 : 1;
  const size_t dbytes = al256(npar * 12 * L.V2 * v.elem_bytes());
  const int p = f.subset == TP_SUBSET_ODD ? 1 : 0;
  const uintptr_t back = f.subset == TP_SUBSET_FULL ? 0 : uintptr_t(p);
  v.data = reinterpret_cast<void*>(base - back * 12 * L.V2 * v.elem_bytes());
  v.nrm = f.prec == TP_F16N ? reinterpret_cast<float*>(base + dbytes - back * 2 * L.V2 * sizeof(float)) : nullptr;
  return v;
}

double2* tpfield_canon(const Lattice& L, const tp_field& f, int r) {
  return static_cast<double2*>(f.data) + size_t(r) * L.V * 12;
}

int subset_par(int subset) { return subset == TP_SUBSET_ODD ? 1 : 0; }
bool layout4_of(int layout) { return layout == TP_LAYOUT_P4; }
int scheme_layout(int scheme) { return scheme == TP_SCHUR4D ? TP_LAYOUT_P4 : TP_LAYOUT_P3; }

// One right-hand side: internal dst = internal src, same layout (precision and subset change).
void convert_internal(tp_ctx ctx, const tp_field& dst, const Field& dv, const tp_field& src, const Field& sv) {
  if (src.subset == TP_SUBSET_FULL) {
    if (dst.subset == TP_SUBSET_FULL) blas(ctx, B_CONVERT, 0, 2, {&sv, &dv});
    else blas(ctx, B_CONVERT, subset_par(dst.subset), 1, {&sv, &dv});
    return;
  }
  const int p = subset_par(src.subset);
  if (dst.subset != TP_SUBSET_FULL && subset_par(dst.subset) != p)
    TP_THROW(TP_EINVAL, "field convert: one-parity fields of different parities");
  blas(ctx, B_CONVERT, p, 1, {&sv, &dv});
  if (dst.subset == TP_SUBSET_FULL) blas(ctx, B_ZERO, 1 - p, 1, {nullptr, &dv});
}

// One right-hand side of a field as a FULL internal Field of (layout, prec): the field itself
// when it already is one, else a conversion into workspace slot `slot`.
Field full_internal(tp_op op, const tp_field& f, int r, int layout, int prec, int slot) {
  tp_ctx ctx = op->g->ctx;
  const Lattice& L = ctx->lat;
  if (f.layout == layout && f.prec == prec && f.subset == TP_SUBSET_FULL) return tpfield_view(L, f, r);
  Field& w = tmp_field(op, prec, slot);
  if (f.layout == TP_LAYOUT_CANONICAL) {
    const double2* wd = layout4_of(layout) ? nullptr : op->g->w_d;
    launch_pack(ctx, tpfield_canon(L, f, r), w, layout4_of(layout), false, wd);
  } else {
    if (f.layout != layout) TP_THROW(TP_EINVAL, "field in another internal layout");
    tp_field full{nullptr, layout, prec, TP_SUBSET_FULL, 1};
    convert_internal(ctx, full, w, f, tpfield_view(L, f, r));
  }
  return w;
}
}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

const char* tp_status_string(tp_status s) {
  switch (s) {
    case TP_OK: return "ok";
    case TP_EINVAL: return "invalid argument";
    case TP_EDIMS: return "unsupported lattice dimensions";
    case TP_ESINGULAR: return "numerically singular matrix";
    case TP_ENOCONV: return "solver did not converge";
    case TP_EBREAKDOWN: return "solver breakdown";
    case TP_ENOMEM: return "out of device memory";
    case TP_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* tp_last_error(void) { return g_last_error.c_str(); }

tp_status tp_ctx_create(const int32_t dims[4], int32_t bc_t, int32_t device, tp_ctx* out) {
  return guard([&] {
    need(dims, "dims");
    need(out, "out");
    *out = nullptr;
    for (int k = 0; k < 3; ++k)
      if (dims[k] < 2 || dims[k] % 2) TP_THROW(TP_EDIMS, "spatial extents must be even and >= 2");
    if (dims[3] < 2) TP_THROW(TP_EDIMS, "time extent must be >= 2");
    if (bc_t != 1 && bc_t != -1) TP_THROW(TP_EINVAL, "bc_t must be +1 or -1");
    // device code addresses a field plane with 32-bit byte offsets: V/2 * 16 B < 2^32
    if ((int64_t)dims[0] * dims[1] * dims[2] * (int64_t)dims[3] > (int64_t)1 << 29)
      TP_THROW(TP_EDIMS, "volume too large");
    int ndev = 0;
    HIP_CHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) TP_THROW(TP_EINVAL, "bad device ordinal");
    tp_ctx c = new tp_ctx_s();
    c->lat = make_lattice(dims);
    c->bc = bc_t;
    c->device = device;
    try {
      HIP_CHECK(hipSetDevice(device));
      int lds = 0;
      HIP_CHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
      c->lds_max = size_t(lds);
      c->scratch = scratch_address(device);
      ctx_buffers_alloc(c);
      HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&c->red_host), sizeof(double) * 8 * kMaxRhs,
                              hipHostMallocDefault));
    } catch (...) {
      ctx_buffers_free(c);
      delete c;
      throw;
    }
    *out = c;
  });
}

tp_status tp_ctx_destroy(tp_ctx ctx) {
  return guard([&] {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto& e : ctx->ev_pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    ctx_buffers_free(ctx);
    if (ctx->red_host) (void)hipHostFree(ctx->red_host);
    delete ctx;
  });
}

tp_status tp_ctx_set_allocator(tp_ctx ctx, tp_alloc_fn alloc_fn, tp_free_fn free_fn, void* user) {
  return guard([&] {
    need(ctx, "ctx");
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
      TP_THROW(TP_EINVAL, "alloc_fn and free_fn must both be set or both be null");
    if (ctx->nchildren) TP_THROW(TP_EINVAL, "set the allocator before the first tp_gauge_create");
    set_device(ctx);
    if (ctx->stream) HIP_CHECK(hipStreamSynchronize(ctx->stream));
    ctx_buffers_free(ctx);
    ctx->alloc_fn = alloc_fn;
    ctx->free_fn = free_fn;
    ctx->alloc_user = user;
    ctx_buffers_alloc(ctx);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  });
}

tp_status tp_ctx_device_bytes(tp_ctx ctx, size_t* bytes) {
  return guard([&] {
    need(ctx, "ctx");
    need(bytes, "bytes");
    *bytes = ctx->live_bytes;
  });
}

tp_status tp_ctx_set_stream(tp_ctx ctx, void* stream) {
  return guard([&] {
    need(ctx, "ctx");
    prof_flush(ctx);
    ctx->stream = static_cast<hipStream_t>(stream);
  });
}

tp_status tp_gauge_create(tp_ctx ctx, const void* links, int32_t where, tp_gauge* out) {
  return guard([&] {
    need(ctx, "ctx");
    need(links, "links");
    need(out, "out");
    if (where != TP_HOST && where != TP_DEVICE) TP_THROW(TP_EINVAL, "bad `where`");
    *out = nullptr;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    tp_gauge g = new tp_gauge_s();
    g->ctx = ctx;
    ctx->nchildren++;
    try {
      size_t lb = size_t(4) * L.V * 9 * sizeof(double2);
      g->canon = static_cast<double2*>(dev_alloc(ctx, lb));
      HIP_CHECK(hipMemcpyAsync(g->canon, links, lb,
                               where == TP_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                               ctx->stream));
      g->u3_d = static_cast<double2*>(dev_alloc(ctx, lb));
      g->u3_f = static_cast<float2*>(dev_alloc(ctx, lb / 2));
      g->u3_h = static_cast<__half2*>(dev_alloc(ctx, lb / 4));
      g->u4_d = static_cast<double2*>(dev_alloc(ctx, lb));
      g->u4_f = static_cast<float2*>(dev_alloc(ctx, lb / 2));
      g->w_d = static_cast<double2*>(dev_alloc(ctx, size_t(2) * 9 * L.V2 * sizeof(double2)));
      g->poly = static_cast<double2*>(dev_alloc(ctx, size_t(2) * 9 * L.Vs2 * sizeof(double2)));
      g->canon_ax = static_cast<double2*>(dev_alloc(ctx, lb));
      int* flags = static_cast<int*>(dev_alloc(ctx, 4 * sizeof(int)));
      int hf[4] = {1, 1, 1, 1};
      try {
        HIP_CHECK(hipMemsetAsync(flags, 0, 4 * sizeof(int), ctx->stream));
        launch_wline(ctx, g);
        launch_axial_links(ctx, g, flags);
        launch_to_half(ctx, g->u3_f, g->u3_h, int64_t(lb / sizeof(double2)));
        launch_pack_links(ctx, g);
        HIP_CHECK(hipMemcpyAsync(hf, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
      } catch (...) {
        dev_free(ctx, flags);
        throw;
      }
      dev_free(ctx, flags);
      if (hf[2]) TP_THROW(TP_EINVAL, "links contain NaN or Inf");
      if (hf[1]) TP_THROW(TP_EINVAL, "time links must be unitary (U U^dag = 1 to 1e-10)");
      g->su3_spatial = hf[0] == 0;
      g->su3_spatial_f64 = hf[3] == 0;
    } catch (...) {
      tp_gauge_destroy(g);
      throw;
    }
    *out = g;
  });
}

tp_status tp_gauge_destroy(tp_gauge g) {
  return guard([&] {
    if (!g) return;
    tp_ctx ctx = g->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    dev_free(ctx, g->canon);
    dev_free(ctx, g->u3_d);
    dev_free(ctx, g->u3_f);
    dev_free(ctx, g->u3_h);
    dev_free(ctx, g->u4_d);
    dev_free(ctx, g->u4_f);
    dev_free(ctx, g->w_d);
    dev_free(ctx, g->canon_ax);
    dev_free(ctx, g->poly);
    ctx->nchildren--;
    delete g;
  });
}

tp_status tp_gauge_plaquette(tp_gauge g, double* ps, double* pt) {
  return guard([&] {
    need(g, "gauge");
    need(ps, "plaq_s");
    need(pt, "plaq_t");
    tp_ctx ctx = g->ctx;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    int64_t nb = (L.V + 255) / 256;
    double* part = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * nb));
    std::vector<double> h(2 * nb);
    try {
      launch_plaquette(ctx, g, part);
      HIP_CHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost,
                               ctx->stream));
      HIP_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (...) {
      dev_free(ctx, part);
      throw;
    }
    dev_free(ctx, part);
    double s = 0, t = 0;
    for (int64_t b = 0; b < nb; ++b) {
      s += h[2 * b];
      t += h[2 * b + 1];
    }
    *ps = s / (3.0 * L.V);
    *pt = t / (3.0 * L.V);
  });
}

tp_status tp_clover_create(tp_gauge g, double c_s, double c_t, tp_clover* out) {
  return guard([&] {
    need(g, "gauge");
    need(out, "out");
    if (!isfinite(c_s) || !isfinite(c_t)) TP_THROW(TP_EINVAL, "clover coefficients");
    *out = nullptr;
    tp_ctx ctx = g->ctx;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    tp_clover c = new tp_clover_s();
    c->g = g;
    c->cs = c_s;
    c->ct = c_t;
    try {
      size_t cb = size_t(2) * 36 * L.V2;
      c->a3_d = static_cast<double2*>(dev_alloc(ctx, cb * sizeof(double2)));
      c->a3_f = static_cast<float2*>(dev_alloc(ctx, cb * sizeof(float2)));
      c->a3_h = static_cast<__half2*>(dev_alloc(ctx, cb * sizeof(__half2)));
      c->a4_d = static_cast<double2*>(dev_alloc(ctx, cb * sizeof(double2)));
      c->a4_f = static_cast<float2*>(dev_alloc(ctx, cb * sizeof(float2)));
      double sig[6][2][2][2][2];
      clover_sigma_table(c_s, c_t, sig);
      launch_clover_build(ctx, c, sig);
      launch_to_half(ctx, c->a3_f, c->a3_h, int64_t(cb));
      HIP_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (...) {
      tp_clover_destroy(c);
      throw;
    }
    *out = c;
  });
}

tp_status tp_clover_destroy(tp_clover c) {
  return guard([&] {
    if (!c) return;
    tp_ctx ctx = c->g->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(c->g->ctx->stream);
    dev_free(ctx, c->a3_d);
    dev_free(ctx, c->a3_f);
    dev_free(ctx, c->a3_h);
    dev_free(ctx, c->a4_d);
    dev_free(ctx, c->a4_f);
    delete c;
  });
}

tp_status tp_op_create(tp_gauge g, tp_clover c, double m0, double gamma_f, tp_op* out) {
  return guard([&] {
    need(g, "gauge");
    need(out, "out");
    if (!isfinite(m0) || !isfinite(gamma_f) || gamma_f <= 0) TP_THROW(TP_EINVAL, "m0 / gamma_f");
    if (c && c->g != g) TP_THROW(TP_EINVAL, "clover built from another gauge field");
    *out = nullptr;
    tp_ctx ctx = g->ctx;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    tp_op op = new tp_op_s();
    op->g = g;
    op->c = c;
    op->m0 = m0;
    op->gf = gamma_f;
    op->mu = m0 + 1.0 + 3.0 / gamma_f;
    double* cond = nullptr;
    int* bad = nullptr;
    try {
      if (!(op->mu > 0)) TP_THROW(TP_EINVAL, "mass term mu = m0 + 1 + 3/gamma_f must be positive");
      op->gclos = static_cast<double2*>(dev_alloc(ctx, size_t(2) * 9 * L.Vs2 * sizeof(double2)));
      op->gclos_f = static_cast<float2*>(dev_alloc(ctx, size_t(2) * 9 * L.Vs2 * sizeof(float2)));
      size_t cb = size_t(2) * 36 * L.V2;
      op->a4_mu = static_cast<double2*>(dev_alloc(ctx, cb * sizeof(double2)));
      op->a4_inv = static_cast<double2*>(dev_alloc(ctx, cb * sizeof(double2)));
      op->a4_mu_f = static_cast<float2*>(dev_alloc(ctx, cb * sizeof(float2)));
      op->a4_inv_f = static_cast<float2*>(dev_alloc(ctx, cb * sizeof(float2)));
      op->a3_mu = static_cast<double2*>(dev_alloc(ctx, cb * sizeof(double2)));
      op->a3_inv = static_cast<double2*>(dev_alloc(ctx, cb * sizeof(double2)));
      op->a3_mu_f = static_cast<float2*>(dev_alloc(ctx, cb * sizeof(float2)));
      op->a3_inv_f = static_cast<float2*>(dev_alloc(ctx, cb * sizeof(float2)));
      op->a3_mu_h = static_cast<__half2*>(dev_alloc(ctx, cb * sizeof(__half2)));
      op->a3_inv_h = static_cast<__half2*>(dev_alloc(ctx, cb * sizeof(__half2)));
      std::vector<double> pw(L.L[3] + 1);
      std::vector<float> pwf(L.L[3] + 1);
      for (int k = 0; k <= L.L[3]; ++k) {
        pw[k] = pow(op->mu, -double(k));
        pwf[k] = float(pw[k]);
      }
      op->mupow_d = static_cast<double*>(dev_alloc(ctx, sizeof(double) * pw.size()));
      op->mupow_f = static_cast<float*>(dev_alloc(ctx, sizeof(float) * pwf.size()));
      HIP_CHECK(hipMemcpy(op->mupow_d, pw.data(), sizeof(double) * pw.size(), hipMemcpyHostToDevice));
      HIP_CHECK(hipMemcpy(op->mupow_f, pwf.data(), sizeof(float) * pwf.size(), hipMemcpyHostToDevice));
      cond = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * L.Vs2));
      bad = static_cast<int*>(dev_alloc(ctx, sizeof(int)));
      HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
      launch_closure(ctx, op, cond);
      launch_clover_derived(ctx, op, bad);
      launch_to_half(ctx, op->a3_mu_f, op->a3_mu_h, int64_t(cb));
      launch_to_half(ctx, op->a3_inv_f, op->a3_inv_h, int64_t(cb));
      std::vector<double> hc(2 * L.Vs2);
      int hb = 0;
      HIP_CHECK(hipMemcpyAsync(hc.data(), cond, sizeof(double) * hc.size(), hipMemcpyDeviceToHost,
                               ctx->stream));
      HIP_CHECK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
      HIP_CHECK(hipStreamSynchronize(ctx->stream));
      double worst = 0;
      for (double v : hc) worst = std::max(worst, isfinite(v) ? v : INFINITY);
      if (!(worst <= 1e12))
        TP_THROW(TP_ESINGULAR, "closure (I - mu^-Lt P) is singular or ill-conditioned");
      if (hb) TP_THROW(TP_ESINGULAR, "(A + mu) has a numerically singular 6x6 block");
    } catch (...) {
      dev_free(ctx, cond);
      dev_free(ctx, bad);
      tp_op_destroy(op);
      throw;
    }
    dev_free(ctx, cond);
    dev_free(ctx, bad);
    *out = op;
  });
}

tp_status tp_op_destroy(tp_op op) {
  return guard([&] {
    if (!op) return;
    tp_ctx ctx = op->g->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(op->g->ctx->stream);
    ws_free(op);
    schur3d_free(op);
    dev_free(ctx, op->gclos);
    dev_free(ctx, op->gclos_f);
    dev_free(ctx, op->a4_mu);
    dev_free(ctx, op->a4_inv);
    dev_free(ctx, op->a4_mu_f);
    dev_free(ctx, op->a4_inv_f);
    dev_free(ctx, op->a3_mu);
    dev_free(ctx, op->a3_inv);
    dev_free(ctx, op->a3_mu_f);
    dev_free(ctx, op->a3_inv_f);
    dev_free(ctx, op->a3_mu_h);
    dev_free(ctx, op->a3_inv_h);
    dev_free(ctx, op->mupow_d);
    dev_free(ctx, op->mupow_f);
    delete op;
  });
}

tp_status tp_op_set_cutoff(tp_op op, double eps, int32_t* dropped) {
  return guard([&] {
    need(op, "op");
    if (!(eps >= 0) || !isfinite(eps)) TP_THROW(TP_EINVAL, "cutoff threshold must be finite and >= 0");
    const int lt = op->g->ctx->lat.L[3];
    // |X(t)|_F = sqrt(3) mu^-(Lt-t) (eq:cutoff) decreases towards t = 0: the dropped slices
    // are t = 0 .. cut-1, and by symmetry t = Lt-cut .. Lt-1 for T^dagger
    int cut = 0;
    for (int t = 0; t < lt; ++t)
      if (std::sqrt(3.0) * std::pow(op->mu, -double(lt - t)) < eps) cut = t + 1;
    op->cut = cut;
    if (dropped) *dropped = cut;
  });
}

tp_status tp_op_mass(tp_op op, double* mu) {
  return guard([&] {
    need(op, "op");
    need(mu, "mu");
    *mu = op->mu;
  });
}

tp_status tp_apply_M(tp_op op, int32_t prec, void* dst, const void* src, int32_t dagger) {
  return apply_wrap(op, prec, dst, src, false, dagger != 0,
                    [&](Field& a, Field& b) { op_apply_M(op, prec, a, b, false); });
}

tp_status tp_apply_Ds(tp_op op, int32_t prec, void* dst, const void* src) {
  return apply_wrap(op, prec, dst, src, false, false, [&](Field& a, Field& b) {
    SiteCoef cf{0.0, 0.0, 0.0, 1.0, 0.0};
    launch_site_p3(op, prec, a, b, nullptr, cf, 0, 0, 2, false);
  });
}

tp_status tp_apply_clover(tp_op op, int32_t prec, void* dst, const void* src, int32_t plus_mu) {
  return apply_wrap(op, prec, dst, src, false, false, [&](Field& a, Field& b) {
    int kind = plus_mu == 0 ? 1 : (plus_mu > 0 ? 2 : 3);
    if (kind == 1 && !op->c) {
      blas(op->g->ctx, B_ZERO, 0, 2, {nullptr, &b});
      return;
    }
    SiteCoef cf{0.0, 1.0, 0.0, 0.0, 0.0};
    launch_site_p3(op, prec, a, b, nullptr, cf, kind, 0, 2, false);
  });
}

static void line_both(tp_op op, int prec, int mode, Field& a, Field& b) {
  LineIO io;
  io.in_up = io.in_lo = &a;
  for (int p = 0; p < 2; ++p) launch_line(op, prec, mode, p, io, b);
}

tp_status tp_apply_Tinv(tp_op op, int32_t prec, void* dst, const void* src, int32_t dagger) {
  return apply_wrap(op, prec, dst, src, false, false,
                    [&](Field& a, Field& b) { line_both(op, prec, dagger ? LM_TDINV : LM_TINV, a, b); });
}

tp_status tp_apply_CL(tp_op op, int32_t prec, void* dst, const void* src) {
  return apply_wrap(op, prec, dst, src, false, false,
                    [&](Field& a, Field& b) { line_both(op, prec, LM_CL, a, b); });
}

tp_status tp_apply_CR(tp_op op, int32_t prec, void* dst, const void* src) {
  return apply_wrap(op, prec, dst, src, false, false,
                    [&](Field& a, Field& b) { line_both(op, prec, LM_CR, a, b); });
}

tp_status tp_apply_prec(tp_op op, int32_t scheme, int32_t prec, void* dst, const void* src,
                        int32_t dagger) {
  return guard([&] {
    check_scheme(scheme);
    check_scheme_prec(scheme, prec);
    // dagger: gamma5 on the way in and out around N (Mt^dagger = gamma5 N gamma5)
    tp_status s = apply_wrap(op, prec, dst, src, scheme_layout4(scheme), dagger != 0,
                             [&](Field& a, Field& b) {
                               if (dagger) op_apply_prec_adj(op, scheme, prec, a, b);
                               else op_apply_prec(op, scheme, prec, a, b, false);
                             });
    if (s != TP_OK) TP_THROW(s, g_last_error);
  });
}

tp_status tp_apply_prec_noalloc(tp_op op, int32_t scheme, int32_t prec, void* dst, const void* src,
                                int32_t dagger) {
  return guard([&] {
    need(op, "op");
    check_scheme(scheme);
    check_prec(prec);
    check_scheme_prec(scheme, prec);
    if ((scheme == TP_TEMPORAL_SCHUR3D && !schur3d_ready(op, prec, 0)) ||
        (scheme == TP_TEMPORAL_FULLSW && !(schur3d_ready(op, prec, 0) && schur3d_ready(op, prec, 1))))
      TP_THROW(TP_EINVAL, "TEMPORAL_SCHUR3D, TEMPORAL_FULLSW: their factors are built (and allocated) "
                          "by the first tp_apply_prec of the scheme in this precision");
    tp_ctx ctx = op->g->ctx;
    const size_t needb = size_t(noalloc_fields(scheme)) * field_bytes(ctx->lat, prec);
    if (needb > kScratchBytes)
      TP_THROW(TP_EINVAL, "lattice too large for the no-allocation scratch (" +
                              std::to_string(needb >> 20) + " MiB needed, " +
                              std::to_string(kScratchBytes >> 20) + " MiB available)");
    if (!ctx->scratch) TP_THROW(TP_EHIP, "no scratch address on this device");
    // workspace fields from the scratch array; no profiling events (they would be created)
    struct Scope {
      tp_op op;
      bool prof;
      Scope(tp_op o, char* base) : op(o), prof(o->g->ctx->prof) {
        op->arena = base;
        op->arena_cap = kScratchBytes;
        op->arena_top = 0;
        op->arena_n = 0;
        op->g->ctx->prof = false;
      }
      ~Scope() {
        op->arena = nullptr;
        op->arena_n = 0;
        op->g->ctx->prof = prof;
      }
    } scope(op, ctx->scratch);
    // dagger: gamma5 on the way in and out around N (Mt^dagger = gamma5 N gamma5)
    tp_status s = apply_wrap(op, prec, dst, src, scheme_layout4(scheme), dagger != 0,
                             [&](Field& a, Field& b) {
                               if (dagger) op_apply_prec_adj(op, scheme, prec, a, b);
                               else op_apply_prec(op, scheme, prec, a, b, false);
                             });
    if (s != TP_OK) TP_THROW(s, g_last_error);
  });
}

tp_status tp_prepare_source(tp_op op, int32_t scheme, int32_t prec, void* et, const void* eta) {
  return guard([&] {
    check_scheme(scheme);
    check_scheme_prec(scheme, prec);
    tp_status s = apply_wrap(op, prec, et, eta, scheme_layout4(scheme), false,
                             [&](Field& a, Field& b) { op_prepare(op, scheme, prec, a, b); });
    if (s != TP_OK) TP_THROW(s, g_last_error);
  });
}

tp_status tp_reconstruct(tp_op op, int32_t scheme, int32_t prec, void* x, const void* y) {
  return guard([&] {
    check_scheme(scheme);
    check_scheme_prec(scheme, prec);
    tp_status s = apply_wrap(op, prec, x, y, scheme_layout4(scheme), false,
                             [&](Field& a, Field& b) { op_reconstruct(op, scheme, prec, a, b); });
    if (s != TP_OK) TP_THROW(s, g_last_error);
  });
}

tp_status tp_field_bytes(tp_op op, int32_t layout, int32_t prec, int32_t subset, size_t* bytes) {
  return guard([&] {
    need(op, "op");
    need(bytes, "bytes");
    tp_field f{bytes, layout, prec, subset, 1};
    check_tpfield(op, &f, "field");
    *bytes = tpfield_bytes(op->g->ctx->lat, layout, prec, subset);
  });
}

tp_status tp_field_convert(tp_op op, const tp_field* dst, const tp_field* src) {
  return guard([&] {
    need(op, "op");
    check_tpfield(op, dst, "dst");
    check_tpfield(op, src, "src");
    if (dst->nrhs != src->nrhs) TP_THROW(TP_EINVAL, "field convert: different nrhs");
    if (dst->data == src->data) TP_THROW(TP_EINVAL, "field convert: dst and src must differ");
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    const bool dc = dst->layout == TP_LAYOUT_CANONICAL, sc = src->layout == TP_LAYOUT_CANONICAL;
    if (!dc && !sc && dst->layout != src->layout)
      TP_THROW(TP_EINVAL, "field convert: internal layouts differ (convert through the canonical layout)");
    for (int r = 0; r < src->nrhs; ++r) {
      if (dc && sc) {
        HIP_CHECK(hipMemcpyAsync(tpfield_canon(L, *dst, r), tpfield_canon(L, *src, r), size_t(L.V) * 12 * sizeof(double2),
                                 hipMemcpyDeviceToDevice, ctx->stream));
      } else if (sc) {  // canonical -> internal
        const double2* wd = layout4_of(dst->layout) ? nullptr : op->g->w_d;
        Field dv = tpfield_view(L, *dst, r);
        if (dst->subset == TP_SUBSET_FULL) {
          launch_pack(ctx, tpfield_canon(L, *src, r), dv, layout4_of(dst->layout), false, wd);
        } else {
          Field& w = tmp_field(op, dst->prec, 0);
          launch_pack(ctx, tpfield_canon(L, *src, r), w, layout4_of(dst->layout), false, wd);
          blas(ctx, B_COPY, subset_par(dst->subset), 1, {&w, &dv});
        }
      } else if (dc) {  // internal -> canonical
        const double2* wd = layout4_of(src->layout) ? nullptr : op->g->w_d;
        Field w = full_internal(op, *src, r, src->layout, src->prec, 0);
        launch_unpack(ctx, w, tpfield_canon(L, *dst, r), layout4_of(src->layout), false, wd);
      } else {
        Field dv = tpfield_view(L, *dst, r);
        convert_internal(ctx, *dst, dv, *src, tpfield_view(L, *src, r));
      }
    }
  });
}

tp_status tp_apply_prec_field(tp_op op, int32_t scheme, const tp_field* dst, const tp_field* src,
                              int32_t dagger) {
  return guard([&] {
    need(op, "op");
    check_scheme(scheme);
    check_tpfield(op, dst, "dst");
    check_tpfield(op, src, "src");
    const int lay = scheme_layout(scheme);
    if (dst->layout != lay || src->layout != lay)
      TP_THROW(TP_EINVAL, "apply_prec_field: fields must be in the scheme's internal layout");
    if (dst->prec != src->prec || dst->subset != src->subset || dst->nrhs != src->nrhs)
      TP_THROW(TP_EINVAL, "apply_prec_field: fields of different precision, subset or nrhs");
    const int prec = src->prec;
    check_scheme_prec(scheme, prec);
    if (src->subset == TP_SUBSET_EVEN) TP_THROW(TP_EINVAL, "apply_prec_field: FULL or ODD fields");
    if (src->subset == TP_SUBSET_ODD && !scheme_sub(op, scheme))
      TP_THROW(TP_EINVAL, "apply_prec_field: ODD fields only for schemes solved on the odd block");
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    const size_t per = tpfield_bytes(L, src->layout, prec, src->subset);
    const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst->data), s0 = reinterpret_cast<uintptr_t>(src->data);
    if (d0 < s0 + per * src->nrhs && s0 < d0 + per * dst->nrhs) TP_THROW(TP_EINVAL, "apply_prec_field: dst overlaps src");
    for (int r = 0; r < src->nrhs; ++r) {
      Field sv = tpfield_view(L, *src, r), dv = tpfield_view(L, *dst, r);
      if (src->subset == TP_SUBSET_FULL) {
        op_apply_prec(op, scheme, prec, sv, dv, dagger != 0);
      } else {
        // the odd block through full work fields: copy parity 1 in, apply, copy parity 1 out
        Field& a = tmp_field(op, prec, 0);
        Field& b = tmp_field(op, prec, 1);
        blas(ctx, B_COPY, 1, 1, {&sv, &a});
        op_apply_odd(op, scheme, prec, a, b, dagger != 0);
        blas(ctx, B_COPY, 1, 1, {&b, &dv});
      }
    }
  });
}

tp_status tp_prepare_source_field(tp_op op, int32_t scheme, const tp_field* et, const tp_field* eta) {
  return guard([&] {
    need(op, "op");
    check_scheme(scheme);
    check_tpfield(op, et, "eta_tilde");
    check_tpfield(op, eta, "eta");
    const int lay = scheme_layout(scheme);
    if (et->layout != lay || et->subset != TP_SUBSET_FULL)
      TP_THROW(TP_EINVAL, "prepare_source_field: eta_tilde must be a FULL field of the scheme's layout");
    if (eta->nrhs != et->nrhs) TP_THROW(TP_EINVAL, "prepare_source_field: different nrhs");
    if (eta->data == et->data) TP_THROW(TP_EINVAL, "prepare_source_field: eta_tilde and eta must differ");
    const int prec = et->prec;
    check_scheme_prec(scheme, prec);
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    for (int r = 0; r < et->nrhs; ++r) {
      Field in = full_internal(op, *eta, r, lay, prec, 0);
      Field ov = tpfield_view(ctx->lat, *et, r);
      op_prepare(op, scheme, prec, in, ov);
    }
  });
}

tp_status tp_reconstruct_field(tp_op op, int32_t scheme, const tp_field* x, const tp_field* y) {
  return guard([&] {
    need(op, "op");
    check_scheme(scheme);
    check_tpfield(op, x, "x");
    check_tpfield(op, y, "y");
    const int lay = scheme_layout(scheme);
    if (y->layout != lay || y->subset != TP_SUBSET_FULL)
      TP_THROW(TP_EINVAL, "reconstruct_field: y must be a FULL field of the scheme's layout");
    if (x->nrhs != y->nrhs) TP_THROW(TP_EINVAL, "reconstruct_field: different nrhs");
    if (x->data == y->data) TP_THROW(TP_EINVAL, "reconstruct_field: x and y must differ");
    const int prec = y->prec;
    if (x->layout != TP_LAYOUT_CANONICAL && (x->layout != lay || x->prec != prec || x->subset != TP_SUBSET_FULL))
      TP_THROW(TP_EINVAL, "reconstruct_field: x must be canonical or a FULL field like y");
    check_scheme_prec(scheme, prec);
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    const Lattice& L = ctx->lat;
    for (int r = 0; r < y->nrhs; ++r) {
      Field yv = tpfield_view(L, *y, r);
      if (x->layout == TP_LAYOUT_CANONICAL) {
        Field& w = tmp_field(op, prec, 1);
        op_reconstruct(op, scheme, prec, yv, w);
        launch_unpack(ctx, w, tpfield_canon(L, *x, r), layout4_of(lay), false,
                      layout4_of(lay) ? nullptr : op->g->w_d);
      } else {
        Field xv = tpfield_view(L, *x, r);
        op_reconstruct(op, scheme, prec, yv, xv);
      }
    }
  });
}

tp_status tp_solve(tp_op op, const tp_solve_params* params, void* x, const void* eta,
                   tp_solve_info* info) {
  tp_status st = TP_OK;
  tp_status g = guard([&] {
    need(op, "op");
    need(params, "params");
    need(x, "x");
    need(eta, "eta");
    need(info, "info");
    if (x == eta) TP_THROW(TP_EINVAL, "x and eta must differ");
    const tp_solve_params& P = *params;
    check_scheme(P.scheme);
    check_prec(P.prec);
    if (P.solver != TP_CGNR && P.solver != TP_BICGSTAB) TP_THROW(TP_EINVAL, "bad solver");
    if (P.dagger != 0 && P.dagger != 1) TP_THROW(TP_EINVAL, "dagger must be 0 or 1");
    check_scheme_prec(P.scheme, P.prec);
    if (!(P.tol >= 0) || !(P.inner_tol >= 0)) TP_THROW(TP_EINVAL, "tolerances");
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    bool l4 = scheme_layout4(P.scheme);
    if (l4 && ctx->lat.L[3] % 2) TP_THROW(TP_EDIMS, "SCHUR4D needs an even time extent");
    Field& eta64 = ws_get(op, TP_F64, 60);
    Field& x64 = ws_get(op, TP_F64, 61);
    const double2* w = l4 ? nullptr : op->g->w_d;  // p3 schemes solve in the axial frame
    // M^dagger x = eta  <=>  M (g5 x) = g5 eta: g5 on the way in and out
    const bool g5 = P.dagger != 0;
    launch_pack(ctx, static_cast<const double2*>(eta), eta64, l4, g5, w);
    if (P.use_x0) launch_pack(ctx, static_cast<const double2*>(x), x64, l4, g5, w);
    st = op_solve(op, P, x64, eta64, *info);
    launch_unpack(ctx, x64, static_cast<double2*>(x), l4, g5, w);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    prof_flush(ctx);
    if (st != TP_OK)
      g_last_error = st == TP_ENOCONV ? "iteration cap reached before the target residual"
                                      : "Krylov breakdown";
  });
  if (g != TP_OK) return g;
  return st;
}

tp_status tp_solve_multi(tp_op op, const tp_solve_params* params, int32_t nrhs, void* const* x,
                         const void* const* eta, tp_solve_info* info) {
  tp_status st = TP_OK;
  tp_status g = guard([&] {
    need(op, "op");
    need(params, "params");
    need(x, "x");
    need(eta, "eta");
    need(info, "info");
    if (nrhs < 1 || nrhs > kMaxRhs) TP_THROW(TP_EINVAL, "nrhs must be 1..16");
    for (int q = 0; q < nrhs; ++q) {
      need(x[q], "x[k]");
      need(eta[q], "eta[k]");
      for (int k = 0; k < nrhs; ++k)
        if (x[q] == eta[k] || (k != q && x[q] == x[k])) TP_THROW(TP_EINVAL, "x[k] must be distinct buffers");
    }
    const tp_solve_params& P = *params;
    check_scheme(P.scheme);
    check_prec(P.prec);
    if (P.solver != TP_CGNR && P.solver != TP_BICGSTAB) TP_THROW(TP_EINVAL, "bad solver");
    if (P.dagger != 0 && P.dagger != 1) TP_THROW(TP_EINVAL, "dagger must be 0 or 1");
    check_scheme_prec(P.scheme, P.prec);
    if (!(P.tol >= 0) || !(P.inner_tol >= 0)) TP_THROW(TP_EINVAL, "tolerances");
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    bool l4 = scheme_layout4(P.scheme);
    if (l4 && ctx->lat.L[3] % 2) TP_THROW(TP_EDIMS, "SCHUR4D needs an even time extent");
    Field& eta64 = ws_get_n(op, TP_F64, 62, nrhs);
    Field& x64 = ws_get_n(op, TP_F64, 63, nrhs);
    const double2* w = l4 ? nullptr : op->g->w_d;  // p3 schemes solve in the axial frame
    const bool g5 = P.dagger != 0;  // M^dagger x = eta  <=>  M (g5 x) = g5 eta
    for (int q = 0; q < nrhs; ++q) {
      Field e = eta64.view(q), xq = x64.view(q);
      launch_pack(ctx, static_cast<const double2*>(eta[q]), e, l4, g5, w);
      if (P.use_x0) launch_pack(ctx, static_cast<const double2*>(x[q]), xq, l4, g5, w);
    }
    st = op_solve_multi(op, P, nrhs, x64, eta64, info);
    for (int q = 0; q < nrhs; ++q) {
      Field xq = x64.view(q);
      launch_unpack(ctx, xq, static_cast<double2*>(x[q]), l4, g5, w);
    }
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    prof_flush(ctx);
    if (st != TP_OK)
      g_last_error = st == TP_ENOCONV ? "iteration cap reached before the target residual"
                                      : "Krylov breakdown";
  });
  if (g != TP_OK) return g;
  return st;
}

tp_status tp_force(tp_op op, const void* x, const void* lambda, void* grad, int32_t flags) {
  return guard([&] {
    need(op, "op");
    need(x, "x");
    need(lambda, "lambda");
    need(grad, "grad_links");
    tp_ctx ctx = op->g->ctx;
    set_device(ctx);
    Field& a = tmp_field(op, TP_F64, 0);
    Field& b = tmp_field(op, TP_F64, 1);
    launch_pack(ctx, static_cast<const double2*>(x), a, false, false, nullptr);
    launch_pack(ctx, static_cast<const double2*>(lambda), b, false, false, nullptr);
    if (flags & ~(TP_FORCE_PROJECTED | TP_FORCE_HOPPING_ONLY)) TP_THROW(TP_EINVAL, "bad force flags");
    const bool projected = (flags & TP_FORCE_PROJECTED) != 0;
    launch_force(op, a, b, static_cast<double2*>(grad), projected);
    if (op->c && !(flags & TP_FORCE_HOPPING_ONLY)) {
      double sig[6][4][4][2];
      sigma_planes(sig);
      launch_clover_force(op, a, b, static_cast<double2*>(grad), projected, sig);
    }
  });
}

tp_status tp_prof_enable(tp_ctx ctx, int32_t on) {
  return guard([&] {
    need(ctx, "ctx");
    prof_flush(ctx);
    ctx->prof = on != 0;
  });
}

tp_status tp_prof_select(tp_ctx ctx, uint32_t mask) {
  return guard([&] {
    need(ctx, "ctx");
    prof_flush(ctx);
    ctx->prof_mask = mask;
  });
}

tp_status tp_prof_reset(tp_ctx ctx) {
  return guard([&] {
    need(ctx, "ctx");
    prof_flush(ctx);
    for (auto& s : ctx->prof_slots) s = ProfSlot{};
  });
}

int32_t tp_prof_count(void) { return KID_COUNT; }
const char* tp_prof_name(int32_t id) { return (id >= 0 && id < KID_COUNT) ? kKernelNames[id] : ""; }

tp_status tp_prof_get(tp_ctx ctx, int32_t id, int64_t* launches, double* ms, double* bytes) {
  return guard([&] {
    need(ctx, "ctx");
    if (id < 0 || id >= KID_COUNT) TP_THROW(TP_EINVAL, "kernel id");
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    prof_flush(ctx);
    if (launches) *launches = ctx->prof_slots[id].launches;
    if (ms) *ms = ctx->prof_slots[id].ms;
    if (bytes) *bytes = ctx->prof_slots[id].bytes;
  });
}

}  // extern "C"
