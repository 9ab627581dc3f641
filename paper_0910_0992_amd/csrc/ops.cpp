// Composite operators and the Krylov solvers, on internal fields.
//
// Schemes (Sec. II.A-B):
//   UNPREC          M
//   SCHUR4D         p4 parity: Mt = diag(A+mu, S-hat), S-hat = (A+mu) - D_w^oe (A+mu)^-1 D_w^eo
//   TEMPORAL        Mt = C_L M C_R = 1 + C_L (A - D_s/gamma_f) C_R   (eq:ContaminatedUnprec)
//   TEMPORAL_SCHUR  p3 parity: Mt3 = S_L M S_R.  Wilson: diag(1, 1 - Dbar^oe Dbar^eo/gamma_f^2)
//                   (eq:TPrecFull); clover: eq:TPrecPartial (3D ILU), applied as
//                     a_o   = C_R^o psi_o                          (scan, upper half only)
//                     u     = D_s^eo a_o / gamma_f                 (site hop)
//                     y     = A^ee C_R^e (C_L^e u + psi_e)         \
//                     chi_e = psi_e + C_L^e y                      } (fused scans + clover)
//                     n_e   = C_R^e C_L^e (y - u)                  /
//                     v     = A^oo a_o + D_s^oe n_e / gamma_f      (site hop + clover)
//                     chi_o = psi_o + C_L^o v                      (scan)
//                   which is the appendix's ILU sequence with t1 = C_L u, t2 = C_L y,
//                   C_R(t2 - t1) = C_R C_L (y - u) and the Dbar/Abar products expanded.
//   TEMPORAL_SCHUR3D  p3 parity with the even block inverted exactly (temporal
//                   preconditioning combined with 3D-Schur):
//                     Mt = diag(1, C_L^o S_o C_R^o),  S_o = M^oo - M^oe (M^ee)^-1 M^eo,
//                   applied as a_o = C_R^o psi_o, u = D_s^eo a_o, f = (M^ee)^-1 u,
//                   v = A^oo a_o - D_s^oe f / gamma_f^2, chi_o = psi_o + C_L^o v
//                   (M^oo = C_L^-1 C_R^-1 + A^oo on odd sites); F64 or F32.
//   TEMPORAL_FULLSW full SW temporal preconditioning on the whole lattice: C_L = T^-1 with
//                   T = A + mu - D_t inverted exactly on both parities, C_R = 1:
//                     Mt = 1 - T^-1 D_s / gamma_f,  Mt^dagger = g5 (1 - D_s T^-1 / gamma_f) g5,
//                   applied as u = D_s psi / gamma_f (site hop), chi = psi - T^-1 u (block-LU
//                   sweeps, the subtraction fused into the last one); F64 or F32.
// All p3 operators act in the axial gauge (interior time links = 1), see k_line_impl.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "tp_internal.h"

struct Workspace {
  std::map<std::tuple<int, int, int>, Field> f;
};

// A workspace field carved from the no-allocation arena (one per (prec, slot, nr) and call),
// cleared by a fill kernel on first use.
Field& arena_get(tp_op op, int prec, int slot, int nr) {
  for (int k = 0; k < op->arena_n; ++k) {
    auto& a = op->arena_slots[k];
    if (a.prec == prec && a.slot == slot && a.nr == nr) return a.f;
  }
  const Lattice& lat = op->g->ctx->lat;
  const size_t need = field_bytes(lat, prec, nr);
  if (op->arena_n == tp_op_s::kArenaSlots || op->arena_top + need > op->arena_cap)
    TP_THROW(TP_EINVAL, "no-allocation scratch exhausted");
  Field f;
  f.prec = prec;
  f.V2 = lat.V2;
  f.nr = nr;
  f.data = op->arena + op->arena_top;
  if (prec == TP_F16N) {
    const size_t db = size_t(nr) * 2 * 12 * lat.V2 * f.elem_bytes();
    f.nrm = reinterpret_cast<float*>(op->arena + op->arena_top + ((db + 255) & ~size_t(255)));
  }
  f.owned = false;
  op->arena_top += need;
  auto& a = op->arena_slots[op->arena_n++];
  a.prec = prec;
  a.slot = slot;
  a.nr = nr;
  a.f = f;
  blas(op->g->ctx, B_ZERO, 0, 2, {nullptr, &a.f});
  return a.f;
}

Field& ws_get_n(tp_op op, int prec, int slot, int nr) {
  if (op->arena) return arena_get(op, prec, slot, nr);
  if (!op->ws) op->ws = new Workspace();
  auto key = std::make_tuple(prec, slot, nr);
  auto it = op->ws->f.find(key);
  if (it != op->ws->f.end()) return it->second;
  Field nf = field_alloc(op->g->ctx, prec, nr);
  return op->ws->f.emplace(key, nf).first->second;
}

Field& ws_get(tp_op op, int prec, int slot) { return ws_get_n(op, prec, slot, op->batch_nr); }

void ws_free(tp_op op) {
  if (!op->ws) return;
  for (auto& kv : op->ws->f) field_free(op->g->ctx, kv.second);
  delete op->ws;
  op->ws = nullptr;
}

bool scheme_layout4(int scheme) { return scheme == TP_SCHUR4D; }

// Schemes whose even block is solved directly, so the Krylov solver runs on the odd sites.
bool scheme_sub(tp_op op, int scheme) {
  return scheme == TP_SCHUR4D || (scheme == TP_TEMPORAL_SCHUR && !op->c) ||
         scheme == TP_TEMPORAL_SCHUR3D;
}

namespace {

// workspace slot numbers
enum {
  W_T1 = 0, W_T2, W_T3, W_T4, W_G5A, W_G5B, W_PREP, W_PREP2,
  // solver vectors
  W_R = 16, W_RHAT, W_P, W_V, W_S, W_T, W_X, W_B, W_Y, W_Z, W_D,
  W_X64 = 40, W_R64, W_ETA64, W_TMP64,
  W_S3W = 48, W_S3F
};

BlasArgs cplx(double ar, double ai, double br = 0, double bi = 0, double cr = 0, double ci = 0) {
  BlasArgs k;
  k.a[0] = ar; k.a[1] = ai; k.b[0] = br; k.b[1] = bi; k.c[0] = cr; k.c[1] = ci;
  return k;
}

// S-hat on the odd p4 parity: dst_o = (A+mu) src_o - D^oe (A+mu)^-1 D^eo src_o
void schur4d_odd(tp_op op, int prec, const Field& src, Field& dst) {
  Field& t = ws_get(op, prec, W_T1);
  launch_schur4d(op, prec, 0, 0, &src, t, nullptr, 1.0, 0.0, 3);
  launch_schur4d(op, prec, 1, 1, &t, dst, &src, -1.0, 0.0, 2);
}

LineIO lio(const Field* in, const Field* base = nullptr, bool pass = true) {
  LineIO io;
  io.in_up = io.in_lo = in;
  io.base = base;
  io.pass = pass;
  return io;
}
SiteIO sio_nb(const Field* nb_up, const Field* nb_lo) {
  SiteIO io;
  io.nb_up = nb_up;
  io.nb_lo = nb_lo;
  return io;
}

// Wilson S_o on the odd p3 parity: dst_o = src_o - C_L D_s (C_R C_L) D_s C_R src_o / gamma_f^2
void wilson_so_odd(tp_op op, int prec, const Field& src, Field& dst) {
  Field& aup = ws_get(op, prec, W_T1);
  Field& u = ws_get(op, prec, W_T2);
  Field& m = ws_get(op, prec, W_T3);
  Field& v = ws_get(op, prec, W_T4);
  launch_line(op, prec, LM_CR, 1, lio(&src, nullptr, false), aup);          // a_o upper
  launch_site(op, prec, sio_nb(&aup, &src), u, SiteCoef{0, 0, 0, 1.0, 0}, 0, 0, 1, false);
  launch_line(op, prec, LM_CRCL, 0, lio(&u), m);
  launch_site(op, prec, sio_nb(&m, &m), v,
              SiteCoef{0, 0, 0, -1.0 / (op->gf * op->gf), 0}, 0, 1, 1, false);
  launch_line(op, prec, LM_CL, 1, lio(&v, &src), dst);
}

void ilu_full(tp_op op, int prec, const Field& src, Field& dst) {
  Field& aup = ws_get(op, prec, W_T1);
  Field& u = ws_get(op, prec, W_T2);
  Field& n = ws_get(op, prec, W_T3);
  Field& v = ws_get(op, prec, W_T4);
  const double ig = 1.0 / op->gf;
  launch_line(op, prec, LM_CR, 1, lio(&src, nullptr, false), aup);          // a_o upper
  launch_site(op, prec, sio_nb(&aup, &src), u, SiteCoef{0, 0, 0, ig, 0}, 0, 0, 1, false);
  launch_ilu_mid(op, prec, src, u, dst, n);                                 // chi_e, n_e
  SiteIO io3;
  io3.self_up = &aup;
  io3.self_lo = &src;
  io3.nb_up = io3.nb_lo = &n;
  launch_site(op, prec, io3, v, SiteCoef{0, 1.0, 0, ig, 0}, 1, 1, 1, false);
  launch_line(op, prec, LM_CL, 1, lio(&v, &src), dst);                      // chi_o
}

// C_L^o S_o C_R^o on the odd p3 parity (F64 or F32):
//   dst_o = src_o + C_L^o [A^oo a_o - D_s^oe (M^ee)^-1 D_s^eo a_o / gamma_f^2],  a_o = C_R^o src_o
void schur3d_so_odd(tp_op op, int prec, const Field& src, Field& dst) {
  Field& aup = ws_get(op, prec, W_T1);
  Field& u = ws_get(op, prec, W_T2);
  Field& f = ws_get(op, prec, W_T3);
  Field& v = ws_get(op, prec, W_T4);
  launch_line(op, prec, LM_CR, 1, lio(&src, nullptr, false), aup);          // a_o upper
  launch_site(op, prec, sio_nb(&aup, &src), u, SiteCoef{0, 0, 0, 1.0, 0}, 0, 0, 1, false);
  launch_mee_inv(op, u, f, ws_get(op, prec, W_S3W));
  SiteIO io3;
  io3.self_up = &aup;
  io3.self_lo = &src;
  io3.nb_up = io3.nb_lo = &f;
  const double ig2 = 1.0 / (op->gf * op->gf);
  launch_site(op, prec, io3, v, SiteCoef{0, op->c ? 1.0 : 0.0, 0, -ig2, 0}, op->c ? 1 : 0, 1, 1,
              false);
  launch_line(op, prec, LM_CL, 1, lio(&v, &src), dst);                      // chi_o
}

// Full SW temporal preconditioning on the whole lattice, T = A + mu - D_t:
//   Mt dst = src - T^-1 D_s src / gamma_f, or with adj the operator N = 1 - D_s T^-1 / gamma_f
//   of Mt^dagger = gamma5 N gamma5 (Mt is not gamma5-hermitian).
void fullsw_full(tp_op op, int prec, const Field& src, Field& dst, bool adj) {
  Field& t = ws_get(op, prec, W_T1);
  Field& w = ws_get(op, prec, W_S3W);
  const double ig = 1.0 / op->gf;
  if (!adj) {
    launch_site(op, prec, sio_nb(&src, &src), t, SiteCoef{0, 0, 0, ig, 0}, 0, 0, 2, false);
    launch_tinv(op, 0, 2, t, dst, w, &src);
  } else {
    launch_tinv(op, 0, 2, src, t, w);
    SiteIO io = sio_nb(&t, &t);
    io.in2 = &src;
    launch_site(op, prec, io, dst, SiteCoef{0, 0, 0, -ig, 1.0}, 0, 0, 2, false);
  }
}

void temporal_full(tp_op op, int prec, const Field& src, Field& dst) {
  // C_L M C_R = 1 + C_L (A - D_s / gamma_f) C_R
  Field& a = ws_get(op, prec, W_T1);
  Field& v = ws_get(op, prec, W_T2);
  launch_line(op, prec, LM_CR, 0, lio(&src), a);
  launch_line(op, prec, LM_CR, 1, lio(&src), a);
  SiteIO io;
  io.self_up = io.self_lo = io.nb_up = io.nb_lo = &a;
  launch_site(op, prec, io, v, SiteCoef{0, 1.0, 0, -1.0 / op->gf, 0}, op->c ? 1 : 0, 0, 2, false);
  launch_line(op, prec, LM_CL, 0, lio(&v, &src), dst);
  launch_line(op, prec, LM_CL, 1, lio(&v, &src), dst);
}

void apply_M_noalias(tp_op op, int prec, const Field& src, Field& dst) {
  SiteCoef cf{op->mu, 1.0, -1.0, -1.0 / op->gf, 0.0};
  launch_site_p3(op, prec, src, dst, nullptr, cf, op->c ? 1 : 0, 0, 2, false);
}

void apply_M_p4(tp_op op, int prec, const Field& src, Field& dst) {
  // M psi on parity p = (A+mu) psi_p - D_w psi_(1-p)
  launch_schur4d(op, prec, 1, 0, &src, dst, &src, -1.0, 0.0, 2);
  launch_schur4d(op, prec, 1, 1, &src, dst, &src, -1.0, 0.0, 2);
}

// Mt of the scheme; with adj, the operator N with Mt^dagger = gamma5 N gamma5 (N = Mt for
// every scheme but TEMPORAL_FULLSW).
void prec_noalias(tp_op op, int scheme, int prec, const Field& src, Field& dst, bool adj = false) {
  switch (scheme) {
    case TP_UNPREC:
      apply_M_noalias(op, prec, src, dst);
      break;
    case TP_SCHUR4D:
      schur4d_odd(op, prec, src, dst);
      launch_schur4d(op, prec, 4, 0, nullptr, dst, &src, 0.0, 0.0, 2);  // (A+mu) psi_e
      break;
    case TP_TEMPORAL:
      temporal_full(op, prec, src, dst);
      break;
    case TP_TEMPORAL_SCHUR:
      if (op->c) {
        ilu_full(op, prec, src, dst);
      } else {
        wilson_so_odd(op, prec, src, dst);
        blas(op->g->ctx, B_COPY, 0, 1, {&src, &dst});
      }
      break;
    case TP_TEMPORAL_SCHUR3D:
      schur3d_so_odd(op, prec, src, dst);
      blas(op->g->ctx, B_COPY, 0, 1, {&src, &dst});
      break;
    case TP_TEMPORAL_FULLSW:
      fullsw_full(op, prec, src, dst, adj);
      break;
    default:
      TP_THROW(TP_EINVAL, "unknown scheme");
  }
}

// The operator the Krylov solver iterates on: the whole of Mt, or its odd block
// when the even block is trivial (SCHUR4D; Wilson TEMPORAL_SCHUR).
struct KrylovOp {
  tp_op op;
  int scheme, prec;
  int par0, npar;
  int nr = 1;  // right-hand sides per field (batched applies)
  void apply(const Field& src, Field& dst, bool dagger) const {
    tp_ctx ctx = op->g->ctx;
    // the composite operators' temporaries are batches of nr fields while this runs
    struct BatchScope {
      tp_op op;
      int saved;
      BatchScope(tp_op o, int n) : op(o), saved(o->batch_nr) { o->batch_nr = n; }
      ~BatchScope() { op->batch_nr = saved; }
    } scope(op, nr);
    const Field* in = &src;
    Field* out = &dst;
    Field* ga = nullptr;
    if (dagger) {
      ga = &ws_get(op, prec, W_G5A);
      blas(ctx, B_G5, par0, npar, {&src, ga});
      in = ga;
      out = &ws_get(op, prec, W_G5B);
    }
    if (npar == 1) {
      if (scheme == TP_SCHUR4D) schur4d_odd(op, prec, *in, *out);
      else if (scheme == TP_TEMPORAL_SCHUR3D) schur3d_so_odd(op, prec, *in, *out);
      else wilson_so_odd(op, prec, *in, *out);
    } else {
      prec_noalias(op, scheme, prec, *in, *out, dagger);
    }
    if (dagger) blas(ctx, B_G5, par0, npar, {out, &dst});
  }
};

}  // namespace

// The odd block of a scheme whose even block is solved directly (scheme_sub): the operator
// the Krylov solver iterates on, reading and writing parity 1 of src and dst only.
void op_apply_odd(tp_op op, int scheme, int prec, const Field& src, Field& dst, bool dagger) {
  KrylovOp A{op, scheme, prec, 1, 1};
  A.apply(src, dst, dagger);
}

void op_apply_M(tp_op op, int prec, const Field& src, Field& dst, bool dagger) {
  tp_ctx ctx = op->g->ctx;
  if (!dagger) {
    apply_M_noalias(op, prec, src, dst);
    return;
  }
  Field& a = ws_get(op, prec, W_G5A);
  Field& b = ws_get(op, prec, W_G5B);
  blas(ctx, B_G5, 0, 2, {&src, &a});
  apply_M_noalias(op, prec, a, b);
  blas(ctx, B_G5, 0, 2, {&b, &dst});
}

void op_apply_prec(tp_op op, int scheme, int prec, const Field& src, Field& dst, bool dagger) {
  tp_ctx ctx = op->g->ctx;
  if (!dagger) {
    prec_noalias(op, scheme, prec, src, dst);
    return;
  }
  Field& a = ws_get(op, prec, W_G5A);
  Field& b = ws_get(op, prec, W_G5B);
  blas(ctx, B_G5, 0, 2, {&src, &a});
  prec_noalias(op, scheme, prec, a, b, true);
  blas(ctx, B_G5, 0, 2, {&b, &dst});
}

void op_apply_prec_adj(tp_op op, int scheme, int prec, const Field& src, Field& dst) {
  prec_noalias(op, scheme, prec, src, dst, true);
}

void op_prepare(tp_op op, int scheme, int prec, const Field& eta, Field& et) {
  tp_ctx ctx = op->g->ctx;
  switch (scheme) {
    case TP_UNPREC:
      blas(ctx, B_COPY, 0, 2, {&eta, &et});
      break;
    case TP_SCHUR4D: {
      // eta~_o = eta_o + D_w^oe (A+mu)^-1 eta_e ;  eta~_e = eta_e
      Field& t = ws_get(op, prec, W_PREP);
      launch_schur4d(op, prec, 4, 0, nullptr, t, &eta, 0.0, 0.0, 3);
      launch_schur4d(op, prec, 2, 1, &t, et, &eta, 1.0, 1.0, 0);
      blas(ctx, B_COPY, 0, 1, {&eta, &et});
      break;
    }
    case TP_TEMPORAL:
      launch_line(op, prec, LM_CL, 0, lio(&eta), et);
      launch_line(op, prec, LM_CL, 1, lio(&eta), et);
      break;
    case TP_TEMPORAL_SCHUR: {
      // eta~_e = C_L^e eta_e ; eta~_o = C_L^o [eta_o + D_s^oe C_R^e C_L^e eta_e / gamma_f]
      Field& t = ws_get(op, prec, W_PREP);
      Field& v = ws_get(op, prec, W_PREP2);
      launch_line(op, prec, LM_CL, 0, lio(&eta), et);
      launch_line(op, prec, LM_CRCL, 0, lio(&eta), t);
      SiteIO io = sio_nb(&t, &t);
      io.in2 = &eta;
      launch_site(op, prec, io, v, SiteCoef{0, 0, 0, 1.0 / op->gf, 1.0}, 0, 1, 1, false);
      launch_line(op, prec, LM_CL, 1, lio(&v), et);
      break;
    }
    case TP_TEMPORAL_SCHUR3D: {
      // eta~_e = (M^ee)^-1 eta_e ; eta~_o = C_L^o [eta_o + D_s^oe eta~_e / gamma_f]
      Field& v = ws_get(op, prec, W_PREP);
      launch_mee_inv(op, eta, et, ws_get(op, prec, W_S3W));
      SiteIO io = sio_nb(&et, &et);
      io.in2 = &eta;
      launch_site(op, prec, io, v, SiteCoef{0, 0, 0, 1.0 / op->gf, 1.0}, 0, 1, 1, false);
      launch_line(op, prec, LM_CL, 1, lio(&v), et);
      break;
    }
    case TP_TEMPORAL_FULLSW:
      // eta~ = T^-1 eta on both parities
      launch_tinv(op, 0, 2, eta, et, ws_get(op, prec, W_S3W));
      break;
    default:
      TP_THROW(TP_EINVAL, "unknown scheme");
  }
}

void op_reconstruct(tp_op op, int scheme, int prec, const Field& y, Field& x) {
  tp_ctx ctx = op->g->ctx;
  switch (scheme) {
    case TP_UNPREC:
      blas(ctx, B_COPY, 0, 2, {&y, &x});
      break;
    case TP_SCHUR4D: {
      // x_o = y_o ; x_e = y_e + (A+mu)^-1 D_w^eo y_o
      Field& t = ws_get(op, prec, W_PREP);
      launch_schur4d(op, prec, 0, 0, &y, t, nullptr, 1.0, 0.0, 3);
      blas(ctx, B_COPY, 0, 2, {&y, &x});
      blas(ctx, B_AXPY, 0, 1, {&t, &x}, cplx(1, 0));
      break;
    }
    case TP_TEMPORAL:
      launch_line(op, prec, LM_CR, 0, lio(&y), x);
      launch_line(op, prec, LM_CR, 1, lio(&y), x);
      break;
    case TP_TEMPORAL_SCHUR: {
      // x_o = C_R^o y_o ; x_e = C_R^e [y_e + C_L^e D_s^eo x_o / gamma_f]
      Field& v = ws_get(op, prec, W_PREP);
      Field& t = ws_get(op, prec, W_PREP2);
      launch_line(op, prec, LM_CR, 1, lio(&y), x);
      launch_site(op, prec, sio_nb(&x, &x), v, SiteCoef{0, 0, 0, 1.0 / op->gf, 0}, 0, 0, 1, false);
      launch_line(op, prec, LM_CL, 0, lio(&v, &y), t);
      launch_line(op, prec, LM_CR, 0, lio(&t), x);
      break;
    }
    case TP_TEMPORAL_SCHUR3D: {
      // x_o = C_R^o y_o ; x_e = y_e + (M^ee)^-1 D_s^eo x_o / gamma_f
      Field& t = ws_get(op, prec, W_PREP);
      Field& f = ws_get(op, prec, W_S3F);
      launch_line(op, prec, LM_CR, 1, lio(&y), x);
      launch_site(op, prec, sio_nb(&x, &x), t, SiteCoef{0, 0, 0, 1.0 / op->gf, 0}, 0, 0, 1, false);
      launch_mee_inv(op, t, f, ws_get(op, prec, W_S3W));
      blas(ctx, B_COPY, 0, 1, {&y, &x});
      blas(ctx, B_AXPY, 0, 1, {&f, &x}, cplx(1, 0));
      break;
    }
    case TP_TEMPORAL_FULLSW:  // S_R = 1
      blas(ctx, B_COPY, 0, 2, {&y, &x});
      break;
    default:
      TP_THROW(TP_EINVAL, "unknown scheme");
  }
}

// ---------------------------------------------------------------- Krylov solvers
namespace {

struct KrylovResult {
  int iters = 0, applies = 0, restarts = 0;
  double rel = 0;
  bool converged = false, breakdown = false, stalled = false;
  std::vector<double> alphas, betas;
};

double nrm2(tp_ctx ctx, const KrylovOp& A, const Field& x) {
  double r[4];
  blas(ctx, B_NORM2, A.par0, A.npar, {&x}, BlasArgs{}, r);
  return r[0];
}

// van der Vorst's BiCGStab on A y = b from y = 0; stops on |r| <= eps |b| (recursive).
KrylovResult bicgstab(const KrylovOp& A, const Field& b, Field& y, double eps, int maxit) {
  tp_ctx ctx = A.op->g->ctx;
  int pr = A.prec, p0 = A.par0, np = A.npar;
  Field& r = ws_get(A.op, pr, W_R);
  Field& rh = ws_get(A.op, pr, W_RHAT);
  Field& p = ws_get(A.op, pr, W_P);
  Field& v = ws_get(A.op, pr, W_V);
  Field& s = ws_get(A.op, pr, W_S);
  Field& t = ws_get(A.op, pr, W_T);
  KrylovResult res;
  double red[8];
  blas(ctx, B_ZERO, p0, np, {nullptr, &y});
  blas(ctx, B_COPY, p0, np, {&b, &r});
  blas(ctx, B_COPY, p0, np, {&b, &rh});
  blas(ctx, B_COPY, p0, np, {&b, &p});
  blas(ctx, B_DOT_NORM, p0, np, {&rh, &r}, BlasArgs{}, red);
  double bn2 = red[2];
  if (bn2 == 0.0) {
    res.converged = true;
    return res;
  }
  double rho_r = red[0], rho_i = red[1];
  double r2 = bn2;
  const double tgt2 = eps * eps * bn2;
  double best2 = bn2;
  int best_it = 0;
  while (res.iters < maxit) {
    // guard: stop on divergence, or when no new minimum appeared for a long stretch
    if (r2 > 1e8 * best2 || res.iters - best_it > std::max(500, 2 * best_it)) {
      res.stalled = true;
      break;
    }
    A.apply(p, v, false);
    res.applies++;
    blas(ctx, B_DOT, p0, np, {&rh, &v}, BlasArgs{}, red);
    double den = red[0] * red[0] + red[1] * red[1];
    if (den == 0.0 || !isfinite(den)) { res.breakdown = true; break; }
    // alpha = rho / <rhat, v>
    double al_r = (rho_r * red[0] + rho_i * red[1]) / den;
    double al_i = (rho_i * red[0] - rho_r * red[1]) / den;
    blas(ctx, B_AXPYZ_NORM, p0, np, {&v, &r, &s}, cplx(-al_r, -al_i), red);
    double s2 = red[0];
    res.iters++;
    if (s2 <= tgt2) {
      blas(ctx, B_AXPY, p0, np, {&p, &y}, cplx(al_r, al_i));
      r2 = s2;
      res.converged = true;
      break;
    }
    A.apply(s, t, false);
    res.applies++;
    // <t,s>, |t|^2, <rhat,s>, <rhat,t>: omega, and rho_new = <rhat, s - omega t> before r exists,
    // so the x, r and p updates share one pass over the fields
    blas(ctx, B_DOT4_TS, p0, np, {&t, &s, &rh}, BlasArgs{}, red);
    double om_r = red[0] / red[2], om_i = red[1] / red[2];
    double rn_r = red[3] - (om_r * red[5] - om_i * red[6]);
    double rn_i = red[4] - (om_r * red[6] + om_i * red[5]);
    // beta = (rho_new / rho) (alpha / omega)
    double rr = rho_r * rho_r + rho_i * rho_i;
    double oo = om_r * om_r + om_i * om_i;
    if (red[2] == 0.0 || !isfinite(oo) || oo == 0.0 || rr == 0.0) {
      // keep the half step: y + alpha p has residual s
      blas(ctx, B_AXPY, p0, np, {&p, &y}, cplx(al_r, al_i));
      r2 = s2;
      res.breakdown = true;
      break;
    }
    double q_r = (rn_r * rho_r + rn_i * rho_i) / rr, q_i = (rn_i * rho_r - rn_r * rho_i) / rr;
    double w_r = (al_r * om_r + al_i * om_i) / oo, w_i = (al_i * om_r - al_r * om_i) / oo;
    double be_r = q_r * w_r - q_i * w_i, be_i = q_r * w_i + q_i * w_r;
    blas(ctx, B_BICG_FUSED, p0, np, {&y, &p, &s, &t, &v, &r}, cplx(al_r, al_i, om_r, om_i, be_r, be_i),
         red);
    r2 = red[0];
    if (!isfinite(r2)) { res.breakdown = true; break; }
    if (r2 < best2) { best2 = r2; best_it = res.iters; }
    if (r2 <= tgt2) { res.converged = true; break; }
    rho_r = rn_r;
    rho_i = rn_i;
    if (rho_r * rho_r + rho_i * rho_i < 1e-60 * bn2 * bn2) {
      // rho breakdown: restart the shadow residual
      blas(ctx, B_COPY, p0, np, {&r, &rh});
      blas(ctx, B_COPY, p0, np, {&r, &p});
      rho_r = r2;
      rho_i = 0;
      res.restarts++;
    }
  }
  res.rel = sqrt(r2 / bn2);
  return res;
}

// CG on A^dag A y = A^dag b from y = 0; stops on |b - A y| <= eps |b|.
KrylovResult cgnr(const KrylovOp& A, const Field& b, Field& y, double eps, int maxit) {
  tp_ctx ctx = A.op->g->ctx;
  int pr = A.prec, p0 = A.par0, np = A.npar;
  Field& r = ws_get(A.op, pr, W_R);
  Field& z = ws_get(A.op, pr, W_Z);
  Field& p = ws_get(A.op, pr, W_P);
  Field& w = ws_get(A.op, pr, W_V);
  KrylovResult res;
  double red[8];
  blas(ctx, B_ZERO, p0, np, {nullptr, &y});
  blas(ctx, B_COPY, p0, np, {&b, &r});
  double bn2 = nrm2(ctx, A, b);
  if (bn2 == 0.0) {
    res.converged = true;
    return res;
  }
  A.apply(r, z, true);
  res.applies++;
  blas(ctx, B_COPY, p0, np, {&z, &p});
  double zz = nrm2(ctx, A, z);
  double r2 = bn2;
  const double tgt2 = eps * eps * bn2;
  while (res.iters < maxit) {
    A.apply(p, w, false);
    double ww = nrm2(ctx, A, w);
    if (ww == 0.0 || !isfinite(ww)) { res.breakdown = true; break; }
    double alpha = zz / ww;
    blas(ctx, B_AXPY, p0, np, {&p, &y}, cplx(alpha, 0));
    blas(ctx, B_CAXPY_NORM, p0, np, {&w, &r}, cplx(-alpha, 0), red);
    r2 = red[0];
    A.apply(r, z, true);
    res.applies += 2;
    double zz_new = nrm2(ctx, A, z);
    double beta = zz_new / zz;
    res.alphas.push_back(alpha);
    res.betas.push_back(beta);
    res.iters++;
    if (r2 <= tgt2) { res.converged = true; break; }
    blas(ctx, B_XPAY, p0, np, {&z, &p}, cplx(beta, 0));
    zz = zz_new;
  }
  res.rel = sqrt(r2 / bn2);
  return res;
}

// Extreme eigenvalues of the symmetric tridiagonal matrix (d, e) by Sturm bisection.
double sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t k = 0; k < d.size(); ++k) {
    double off = k ? e[k - 1] * e[k - 1] : 0.0;
    q = d[k] - x - (k ? off / (q == 0.0 ? 1e-300 : q) : 0.0);
    if (q < 0) ++cnt;
  }
  return cnt;
}
double tri_eig(const std::vector<double>& d, const std::vector<double>& e, int which) {
  double lo = 1e300, hi = -1e300;
  for (size_t k = 0; k < d.size(); ++k) {
    double rad = (k ? fabs(e[k - 1]) : 0) + (k + 1 < d.size() ? fabs(e[k]) : 0);
    lo = std::min(lo, d[k] - rad);
    hi = std::max(hi, d[k] + rad);
  }
  // which = 0: smallest (count >= 1), 1: largest (count >= n)
  double target = which == 0 ? 1 : double(d.size());
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, mid) >= target) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

void lanczos_kappa(const KrylovResult& kr, double& lmin, double& lmax) {
  size_t n = kr.alphas.size();
  lmin = lmax = 0;
  if (n == 0) return;
  std::vector<double> d(n), e(n > 1 ? n - 1 : 0);
  for (size_t k = 0; k < n; ++k) {
    d[k] = 1.0 / kr.alphas[k] + (k ? kr.betas[k - 1] / kr.alphas[k - 1] : 0.0);
    if (k + 1 < n) e[k] = sqrt(kr.betas[k]) / kr.alphas[k];
  }
  lmin = tri_eig(d, e, 0);
  lmax = tri_eig(d, e, 1);
}

// r = eta - M x in FP64, returns |r|^2
double true_residual(tp_op op, bool l4, const Field& x, const Field& eta, Field& r) {
  tp_ctx ctx = op->g->ctx;
  if (!l4) {
    SiteCoef cf{-op->mu, -1.0, 1.0, 1.0 / op->gf, 1.0};
    int nb = launch_site_p3(op, TP_F64, x, r, &eta, cf, op->c ? 1 : 0, 0, 2, true);
    return finish_norm(ctx, nb);
  }
  apply_M_p4(op, TP_F64, x, r);
  blas(ctx, B_XPAY, 0, 2, {&eta, &r}, cplx(-1, 0));
  double red[8];
  blas(ctx, B_NORM2, 0, 2, {&r}, BlasArgs{}, red);
  return red[0];
}

// Mixed-precision BiCGStab with reliable updates (Sleijpen and van der Vorst 1996): the
// inner recurrences run in the low precision on the preconditioned operator, and whenever
// the recursive residual has dropped by `delta` below its largest value since the last
// update (or reached the target), the accumulated correction is folded into the FP64
// solution and the recursive residual is replaced by the preconditioned FP64 true residual.
// The search direction and the shadow residual carry on, so the Krylov space is kept
// across updates.  Returns false (x64 holds the best iterate, r64 its residual) when the
// recurrence stalls or diverges, for the caller's fallback.
bool bicgstab_reliable(tp_op op, const tp_solve_params& P, const KrylovOp& A, bool l4, bool sub,
                       double delta, Field& x64, const Field& eta64, Field& r64, double eta2, double& r2,
                       double tol, int max_iter, tp_solve_info& info) {
  tp_ctx ctx = op->g->ctx;
  // The FP64 iterate lives in x64 or in a spare field: xc is the current one, xb the best seen.
  // A fold writes the new iterate next to the best one instead of over it, so keeping the best
  // costs no copy; x64 receives the result once, at the end.
  Field& spare = ws_get(op, TP_F64, W_TMP64);
  Field* xc = &x64;
  Field* xb = &x64;
  auto finish = [&](bool ok) {
    if (xc != &x64) blas(ctx, B_COPY, 0, 2, {xc, &x64});
    return ok;
  };
  const int pr = A.prec, p0 = A.par0, np = A.npar;
  Field& r = ws_get(op, pr, W_R);
  Field& rh = ws_get(op, pr, W_RHAT);
  Field& p = ws_get(op, pr, W_P);
  Field& v = ws_get(op, pr, W_V);
  Field& s = ws_get(op, pr, W_S);
  Field& t = ws_get(op, pr, W_T);
  Field& y = ws_get(op, pr, W_Y);
  Field& rin = ws_get(op, pr, W_B);
  Field& et = ws_get(op, pr, W_D);
  Field& d = ws_get(op, pr, W_X);
  double red[8];
  // preconditioned residual of the current iterate (r64) into `et` (and r), y = 0; returns |r|^2
  auto restart_residual = [&]() {
    blas(ctx, B_CONVERT, 0, 2, {&r64, &rin});
    op_prepare(op, P.scheme, pr, rin, et);
    blas(ctx, B_COPY, p0, np, {&et, &r});
    blas(ctx, B_ZERO, p0, np, {nullptr, &y});
    blas(ctx, B_NORM2, p0, np, {&r}, BlasArgs{}, red);
    return red[0];
  };
  // x += S_R y (with the even block of a subset scheme from the segment's source)
  auto fold = [&]() {
    if (sub) {
      if (P.scheme == TP_SCHUR4D) launch_schur4d(op, pr, 4, 0, nullptr, y, &et, 0.0, 0.0, 3);
      else blas(ctx, B_COPY, 0, 1, {&et, &y});
    }
    op_reconstruct(op, P.scheme, pr, y, d);
    if (xc == xb) {
      Field* next = xb == &x64 ? &spare : &x64;
      blas(ctx, B_MIXED_ADD, 0, 2, {&d, xc, next});
      xc = next;
    } else {
      blas(ctx, B_MIXED_ACC, 0, 2, {&d, xc});
    }
    r2 = true_residual(op, l4, *xc, eta64, r64);
    info.outer_iters++;
  };
  // on failure: back to the best FP64 iterate seen
  auto give_up = [&]() {
    if (xc != xb) {
      xc = xb;
      r2 = true_residual(op, l4, *xc, eta64, r64);
    }
    return finish(false);
  };
  double rr2 = restart_residual();
  // the preconditioned residual that corresponds to the true target, scaled per segment
  double seg_r2 = r2, seg_rr2 = rr2;
  blas(ctx, B_COPY, p0, np, {&r, &rh});
  blas(ctx, B_COPY, p0, np, {&r, &p});
  double rho_r = 0, rho_i = 0;
  double rmax2 = rr2;
  double best2 = r2;
  int since_best = 0;
  // stall / divergence guard on the recursive residual within a segment
  double seg_best = rr2;
  int seg_start = info.iters, seg_best_it = info.iters;
  // one iteration runs without host round trips: the reductions turn into the next op's
  // coefficients on the device (BicgPost), and the host reads the scalars once at its end
  double* st = ctx->bicg;
  double S[BS_COUNT];
  auto set_rho = [&]() {
    blas_dev(ctx, B_DOT, p0, np, {&rh, &r}, nullptr, BP_RHO);
    bicg_state(ctx, S);
    rho_r = S[BS_RHO];
    rho_i = S[BS_RHO + 1];
  };
  set_rho();
  while (true) {
    const double tgt2 = 0.25 * tol * tol * eta2 / seg_r2 * seg_rr2;
    if (info.iters >= max_iter) return give_up();
    A.apply(p, v, false);
    blas_dev(ctx, B_DOT, p0, np, {&rh, &v}, nullptr, BP_ALPHA);              // alpha
    blas_dev(ctx, B_AXPYZ_NORM, p0, np, {&v, &r, &s}, st + BS_AXPY, BP_S2);  // s = r - alpha v
    A.apply(s, t, false);
    // <t,s>, |t|^2, <rhat,s>, <rhat,t>: omega, rho_new = <rhat, s - omega t> and beta before r
    // exists, so the x, r and p updates share one pass over the fields
    blas_dev(ctx, B_DOT4_TS, p0, np, {&t, &s, &rh}, nullptr, BP_OMEGA);
    blas_dev(ctx, B_BICG_FUSED, p0, np, {&y, &p, &s, &t, &v, &r}, st + BS_FUSED, BP_R2);
    info.applies += 2;
    info.iters++;
    bicg_state(ctx, S);
    // a vanishing <rhat, v> makes alpha and everything after it non-finite
    rr2 = S[BS_R2];
    if (S[BS_BREAK] != 0.0 || !isfinite(rr2)) return give_up();
    if (rr2 < seg_best) {
      seg_best = rr2;
      seg_best_it = info.iters;
    }
    if (rr2 > 1e8 * seg_best || info.iters - seg_best_it > std::max(500, 2 * (seg_best_it - seg_start)))
      return give_up();
    rho_r = S[BS_RHO];
    rho_i = S[BS_RHO + 1];
    rmax2 = std::max(rmax2, rr2);
    const bool upd = rr2 <= tgt2 || rr2 <= delta * delta * rmax2;
    if (!upd) continue;
    fold();
    if (getenv("TPREC_VERBOSE"))
      fprintf(stderr, "[tprec] reliable update %d at iteration %d: true %.3e\n", info.outer_iters,
              info.iters, sqrt(r2 / eta2));
    if (sqrt(r2 / eta2) <= tol) return finish(true);
    if (r2 < best2) {
      best2 = r2;
      since_best = 0;
      xb = xc;
    } else if (++since_best >= 3 || r2 > 1e4 * best2) {
      return give_up();  // the low-precision recurrence no longer reduces the true residual
    }
    if (info.outer_iters >= (P.max_restarts > 0 ? P.max_restarts : 200)) return give_up();
    rr2 = restart_residual();
    seg_r2 = r2;
    seg_rr2 = rr2;
    rmax2 = rr2;
    seg_best = rr2;
    seg_start = seg_best_it = info.iters;
    set_rho();
    if (rho_r * rho_r + rho_i * rho_i < 1e-24 * rr2 * rr2) {
      // the shadow residual has become orthogonal to the new residual: restart it
      blas(ctx, B_COPY, p0, np, {&r, &rh});
      blas(ctx, B_COPY, p0, np, {&r, &p});
      set_rho();
      info.restarts++;
    }
  }
}

}  // namespace

tp_status op_solve(tp_op op, const tp_solve_params& P, Field& x64, const Field& eta64,
                   tp_solve_info& info) {
  tp_ctx ctx = op->g->ctx;
  auto t0 = std::chrono::steady_clock::now();
  bool l4 = scheme_layout4(P.scheme);
  int pr = P.prec;
  Field& r64 = ws_get(op, TP_F64, W_R64);
  double red[8];
  blas(ctx, B_NORM2, 0, 2, {&eta64}, BlasArgs{}, red);
  double eta2 = red[0];
  if (!isfinite(eta2)) TP_THROW(TP_EINVAL, "source contains NaN or Inf");
  if (!P.use_x0) blas(ctx, B_ZERO, 0, 2, {nullptr, &x64});
  info = tp_solve_info{};
  if (eta2 == 0.0) {
    blas(ctx, B_ZERO, 0, 2, {nullptr, &x64});
    info.true_rel_resid = 0;
    return TP_OK;
  }
  double r2 = true_residual(op, l4, x64, eta64, r64);
  double tol = P.tol > 0 ? P.tol : 1e-10;
  double inner_default = pr == TP_F64 ? 0.0 : (pr == TP_F32 ? 1e-6 : 2e-3);
  double inner = P.inner_tol > 0 ? P.inner_tol : inner_default;
  int max_iter = P.max_iter > 0 ? P.max_iter : 100000;
  int max_restarts = P.max_restarts > 0 ? P.max_restarts : 50;
  KrylovOp A{op, P.scheme, pr, 0, 2};
  bool sub = scheme_sub(op, P.scheme);
  if (sub) {
    A.par0 = 1;
    A.npar = 1;
  }
  Field& rin = ws_get(op, pr, W_B);
  Field& et = ws_get(op, pr, W_D);
  Field& y = ws_get(op, pr, W_Y);
  Field& d = ws_get(op, pr, W_X);
  Field& xsave = ws_get(op, TP_F64, W_TMP64);
  tp_status st = TP_OK;
  int solver = P.solver;
  int failures = 0;  // cycles rolled back
  if (pr != TP_F64 && solver == TP_BICGSTAB && sqrt(r2 / eta2) > tol) {
    // reliable updates; on a stall the defect-correction loop below continues with CGNR
    double delta = P.inner_tol > 0 ? P.inner_tol : (pr == TP_F32 ? 1e-3 : 0.01);
    if (!bicgstab_reliable(op, P, A, l4, sub, delta, x64, eta64, r64, eta2, r2, tol, max_iter, info))
      solver = TP_CGNR;
  }
  int cycles = 0;
  while (sqrt(r2 / eta2) > tol) {
    if (cycles++ >= max_restarts || info.iters >= max_iter) { st = TP_ENOCONV; break; }
    // inner source in the inner precision
    const Field* rsrc = &r64;
    if (pr != TP_F64) {
      blas(ctx, B_CONVERT, 0, 2, {&r64, &rin});
      rsrc = &rin;
    }
    op_prepare(op, P.scheme, pr, *rsrc, et);
    // relative target for this cycle
    double need = 0.5 * tol * sqrt(eta2 / r2);
    double eps = std::max(inner, need);
    if (pr == TP_F64) eps = need;
    eps = std::min(eps, 0.5);
    KrylovResult kr = solver == TP_CGNR ? cgnr(A, et, y, eps, max_iter - info.iters)
                                        : bicgstab(A, et, y, eps, max_iter - info.iters);
    info.iters += kr.iters;
    info.applies += kr.applies;
    info.restarts += kr.restarts;
    info.prec_rel_resid = kr.rel;
    if (P.estimate_kappa && P.solver == TP_CGNR && info.outer_iters == 0) {
      lanczos_kappa(kr, info.lambda_min, info.lambda_max);
      info.kappa_est = info.lambda_min > 0 ? info.lambda_max / info.lambda_min : 0;
    }
    // fill the trivially solved even block
    if (sub) {
      if (P.scheme == TP_SCHUR4D) launch_schur4d(op, pr, 4, 0, nullptr, y, &et, 0.0, 0.0, 3);
      else blas(ctx, B_COPY, 0, 1, {&et, &y});
    }
    op_reconstruct(op, P.scheme, pr, y, d);
    blas(ctx, B_COPY, 0, 2, {&x64, &xsave});
    blas(ctx, B_MIXED_ACC, 0, 2, {&d, &x64});
    double r2_prev = r2;
    r2 = true_residual(op, l4, x64, eta64, r64);
    info.outer_iters++;
    if (getenv("TPREC_VERBOSE"))
      fprintf(stderr, "[tprec] cycle %d: inner %d iters rel %.3e (eps %.1e)%s%s, true %.3e\n",
              info.outer_iters, kr.iters, kr.rel, eps, kr.converged ? "" : " not-converged",
              kr.breakdown ? " breakdown" : "", sqrt(r2 / eta2));
    if (!(r2 < r2_prev)) {
      // the cycle did not help (inner divergence or breakdown in the low precision):
      // undo it and continue with CGNR, whose residual cannot grow
      blas(ctx, B_COPY, 0, 2, {&xsave, &x64});
      r2 = true_residual(op, l4, x64, eta64, r64);
      ++failures;
      if (solver == TP_CGNR) {
        st = kr.breakdown || kr.stalled ? TP_EBREAKDOWN : TP_ENOCONV;
        break;
      }
      solver = TP_CGNR;
    }
  }
  info.true_rel_resid = sqrt(r2 / eta2);
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  prof_flush(ctx);
  info.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

// ---------------------------------------------------------------- batched right-hand sides
// nr right-hand sides solved together: the Krylov recurrences of every right-hand side run in
// lockstep, so each operator application is one batched launch per kernel (links and clover
// read once per site for all of them) and each reduction one synchronisation.  Scalars,
// reliable updates and stopping are per right-hand side; a right-hand side that has
// converged (or stalled) is skipped by the vector updates.  Mixed-precision BiCGStab on the
// full-lattice schemes only; everything else runs the right-hand sides one after another.
tp_status op_solve_multi(tp_op op, const tp_solve_params& P, int nr, Field& x64, const Field& eta64,
                         tp_solve_info* info) {
  tp_ctx ctx = op->g->ctx;
  auto t0 = std::chrono::steady_clock::now();
  const bool l4 = scheme_layout4(P.scheme);
  const bool sub = scheme_sub(op, P.scheme);
  const int pr = P.prec;
  tp_status worst = TP_OK;
  auto merge = [&](tp_status st) {
    if (st != TP_OK && (worst == TP_OK || st == TP_EBREAKDOWN)) worst = st;
  };
  if (nr == 1 || pr == TP_F64 || P.solver != TP_BICGSTAB || sub) {
    for (int q = 0; q < nr; ++q) {
      Field xq = x64.view(q);
      merge(op_solve(op, P, xq, eta64.view(q), info[q]));
    }
    return worst;
  }
  const double tol = P.tol > 0 ? P.tol : 1e-10;
  const double delta = P.inner_tol > 0 ? P.inner_tol : (pr == TP_F32 ? 1e-3 : 0.01);
  const int max_iter = P.max_iter > 0 ? P.max_iter : 100000;
  const int max_upd = P.max_restarts > 0 ? P.max_restarts : 200;
  KrylovOp A{op, P.scheme, pr, 0, 2, nr};
  Field& r = ws_get_n(op, pr, W_R, nr);
  Field& rh = ws_get_n(op, pr, W_RHAT, nr);
  Field& p = ws_get_n(op, pr, W_P, nr);
  Field& v = ws_get_n(op, pr, W_V, nr);
  Field& s = ws_get_n(op, pr, W_S, nr);
  Field& t = ws_get_n(op, pr, W_T, nr);
  Field& y = ws_get_n(op, pr, W_Y, nr);
  // FP64 iterates of right-hand side q live in x64.view(q) or spare.view(q) (as in the single
  // solver: a fold writes the new iterate beside the best one, so the best needs no copy)
  Field& spare = ws_get_n(op, TP_F64, W_TMP64, nr);
  Field& r64 = ws_get_n(op, TP_F64, W_R64, 1);
  Field& rin = ws_get_n(op, pr, W_B, 1);
  Field& et = ws_get_n(op, pr, W_D, 1);
  Field& d = ws_get_n(op, pr, W_X, 1);
  struct St {
    double eta2 = 0, r2 = 0, rr2 = 0, rho_r = 0, rho_i = 0, rmax2 = 0, seg_r2 = 0, seg_rr2 = 0;
    double best2 = 0, seg_best = 0, al_r = 0, al_i = 0;
    int since_best = 0, seg_start = 0, seg_best_it = 0;
    bool done = false, failed = false, upd = false;
    bool cur_spare = false, best_spare = false;  // where the current and the best iterate live
  };
  std::vector<St> S(nr);
  std::vector<double> red(8 * nr);
  std::vector<BlasArgs> args(nr);
  std::unique_ptr<bool[]> skip(new bool[nr]);
  for (int q = 0; q < nr; ++q) info[q] = tp_solve_info{};
  blas_multi(ctx, B_NORM2, 0, 2, {&eta64}, nullptr, nullptr, red.data());
  for (int q = 0; q < nr; ++q) {
    S[q].eta2 = red[8 * q];
    if (!isfinite(S[q].eta2)) TP_THROW(TP_EINVAL, "source contains NaN or Inf");
  }
  if (!P.use_x0) blas(ctx, B_ZERO, 0, 2, {nullptr, &x64});
  auto xview = [&](int q, bool in_spare) { return in_spare ? spare.view(q) : x64.view(q); };
  // preconditioned FP64 residual of right-hand side q into r[q]; y[q] = 0
  auto restart_residual = [&](int q) {
    Field rq = r.view(q), yq = y.view(q);
    double rr[8];
    blas(ctx, B_CONVERT, 0, 2, {&r64, &rin});
    op_prepare(op, P.scheme, pr, rin, et);
    blas(ctx, B_COPY, 0, 2, {&et, &rq});
    blas(ctx, B_ZERO, 0, 2, {nullptr, &yq});
    blas(ctx, B_NORM2, 0, 2, {&rq}, BlasArgs{}, rr);
    St& z = S[q];
    z.rr2 = z.seg_rr2 = z.rmax2 = z.seg_best = rr[0];
    z.seg_r2 = z.r2;
    z.seg_start = z.seg_best_it = info[q].iters;
  };
  auto give_up = [&](int q) {
    S[q].cur_spare = S[q].best_spare;
    S[q].failed = true;
  };
  for (int q = 0; q < nr; ++q) {
    St& z = S[q];
    if (z.eta2 == 0.0) {
      Field xq = x64.view(q);
      blas(ctx, B_ZERO, 0, 2, {nullptr, &xq});
      z.done = true;
      continue;
    }
    Field xq = x64.view(q);
    z.r2 = z.best2 = true_residual(op, l4, xq, eta64.view(q), r64);
    if (sqrt(z.r2 / z.eta2) <= tol) {
      z.done = true;
      continue;
    }
    restart_residual(q);
  }
  blas(ctx, B_COPY, 0, 2, {&r, &rh});
  blas(ctx, B_COPY, 0, 2, {&r, &p});
  blas_multi(ctx, B_DOT, 0, 2, {&rh, &r}, nullptr, nullptr, red.data());
  for (int q = 0; q < nr; ++q) {
    S[q].rho_r = red[8 * q];
    S[q].rho_i = red[8 * q + 1];
  }
  int iter = 0;
  while (true) {
    bool any = false;
    for (int q = 0; q < nr; ++q) {
      skip[q] = S[q].done || S[q].failed;
      any = any || !skip[q];
    }
    if (!any || iter >= max_iter) break;
    ++iter;
    A.apply(p, v, false);
    blas_multi(ctx, B_DOT, 0, 2, {&rh, &v}, nullptr, skip.get(), red.data());
    for (int q = 0; q < nr; ++q) {
      St& z = S[q];
      if (skip[q]) continue;
      const double dr = red[8 * q], di = red[8 * q + 1];
      const double den = dr * dr + di * di;
      if (den == 0.0 || !isfinite(den)) {
        give_up(q);
        skip[q] = true;
        continue;
      }
      z.al_r = (z.rho_r * dr + z.rho_i * di) / den;
      z.al_i = (z.rho_i * dr - z.rho_r * di) / den;
      args[q] = cplx(-z.al_r, -z.al_i);
    }
    blas_multi(ctx, B_AXPYZ_NORM, 0, 2, {&v, &r, &s}, args.data(), skip.get(), red.data());
    for (int q = 0; q < nr; ++q) {
      St& z = S[q];
      z.upd = false;
      if (skip[q]) continue;
      info[q].iters++;
      info[q].applies += 2;
      const double tgt2 = 0.25 * tol * tol * z.eta2 / z.seg_r2 * z.seg_rr2;
      if (red[8 * q] <= tgt2) {
        // converged at the half step: y += alpha p, r = s, and no second half
        Field yq = y.view(q), pq = p.view(q), sq = s.view(q), rq = r.view(q);
        blas(ctx, B_AXPY, 0, 2, {&pq, &yq}, cplx(z.al_r, z.al_i));
        blas(ctx, B_COPY, 0, 2, {&sq, &rq});
        z.rr2 = red[8 * q];
        z.upd = true;
        skip[q] = true;
      }
    }
    bool second = false;
    for (int q = 0; q < nr; ++q) second = second || !skip[q];
    if (second) {
      A.apply(s, t, false);
      blas_multi(ctx, B_DOT4_TS, 0, 2, {&t, &s, &rh}, nullptr, skip.get(), red.data());
      for (int q = 0; q < nr; ++q) {
        St& z = S[q];
        if (skip[q]) continue;
        const double* w = &red[8 * q];
        const double om_r = w[0] / w[2], om_i = w[1] / w[2];
        const double rn_r = w[3] - (om_r * w[5] - om_i * w[6]);
        const double rn_i = w[4] - (om_r * w[6] + om_i * w[5]);
        const double rr = z.rho_r * z.rho_r + z.rho_i * z.rho_i;
        const double oo = om_r * om_r + om_i * om_i;
        if (w[2] == 0.0 || !isfinite(oo) || oo == 0.0 || rr == 0.0) {
          give_up(q);
          skip[q] = true;
          continue;
        }
        const double q_r = (rn_r * z.rho_r + rn_i * z.rho_i) / rr, q_i = (rn_i * z.rho_r - rn_r * z.rho_i) / rr;
        const double w_r = (z.al_r * om_r + z.al_i * om_i) / oo, w_i = (z.al_i * om_r - z.al_r * om_i) / oo;
        args[q] = cplx(z.al_r, z.al_i, om_r, om_i, q_r * w_r - q_i * w_i, q_r * w_i + q_i * w_r);
        z.rho_r = rn_r;
        z.rho_i = rn_i;
      }
      blas_multi(ctx, B_BICG_FUSED, 0, 2, {&y, &p, &s, &t, &v, &r}, args.data(), skip.get(), red.data());
      for (int q = 0; q < nr; ++q) {
        St& z = S[q];
        if (skip[q]) continue;
        z.rr2 = red[8 * q];
        if (!isfinite(z.rr2)) {
          give_up(q);
          continue;
        }
        if (z.rr2 < z.seg_best) {
          z.seg_best = z.rr2;
          z.seg_best_it = info[q].iters;
        }
        if (z.rr2 > 1e8 * z.seg_best ||
            info[q].iters - z.seg_best_it > std::max(500, 2 * (z.seg_best_it - z.seg_start))) {
          give_up(q);
          continue;
        }
        z.rmax2 = std::max(z.rmax2, z.rr2);
        const double tgt2 = 0.25 * tol * tol * z.eta2 / z.seg_r2 * z.seg_rr2;
        z.upd = z.rr2 <= tgt2 || z.rr2 <= delta * delta * z.rmax2;
      }
    }
    // reliable updates, one right-hand side at a time
    for (int q = 0; q < nr; ++q) {
      St& z = S[q];
      if (!z.upd || z.failed) continue;
      Field yq = y.view(q), rq = r.view(q), rhq = rh.view(q), pq = p.view(q);
      op_reconstruct(op, P.scheme, pr, yq, d);
      Field xq = xview(q, z.cur_spare);
      if (z.cur_spare == z.best_spare) {
        Field nq = xview(q, !z.cur_spare);
        blas(ctx, B_MIXED_ADD, 0, 2, {&d, &xq, &nq});
        z.cur_spare = !z.cur_spare;
        xq = nq;
      } else {
        blas(ctx, B_MIXED_ACC, 0, 2, {&d, &xq});
      }
      z.r2 = true_residual(op, l4, xq, eta64.view(q), r64);
      info[q].outer_iters++;
      if (sqrt(z.r2 / z.eta2) <= tol) {
        z.done = true;
        continue;
      }
      if (z.r2 < z.best2) {
        z.best2 = z.r2;
        z.since_best = 0;
        z.best_spare = z.cur_spare;
      } else if (++z.since_best >= 3 || z.r2 > 1e4 * z.best2 || info[q].outer_iters >= max_upd) {
        give_up(q);
        continue;
      }
      restart_residual(q);
      double rr[8];
      blas(ctx, B_DOT, 0, 2, {&rhq, &rq}, BlasArgs{}, rr);
      z.rho_r = rr[0];
      z.rho_i = rr[1];
      if (z.rho_r * z.rho_r + z.rho_i * z.rho_i < 1e-24 * z.rr2 * z.rr2) {
        blas(ctx, B_COPY, 0, 2, {&rq, &rhq});
        blas(ctx, B_COPY, 0, 2, {&rq, &pq});
        z.rho_r = z.rr2;
        z.rho_i = 0;
        info[q].restarts++;
      }
    }
  }
  // every result (the converged iterate, or the best one of a stalled right-hand side) into x64
  for (int q = 0; q < nr; ++q) {
    if (!S[q].cur_spare) continue;
    Field from = spare.view(q), to = x64.view(q);
    blas(ctx, B_COPY, 0, 2, {&from, &to});
  }
  // right-hand sides that stalled continue alone from their best iterate
  for (int q = 0; q < nr; ++q) {
    St& z = S[q];
    Field xq = x64.view(q);
    if (z.done) {
      info[q].true_rel_resid = z.eta2 > 0 ? sqrt(z.r2 / z.eta2) : 0.0;
      continue;
    }
    tp_solve_params P2 = P;
    P2.use_x0 = 1;
    tp_solve_info extra{};
    merge(op_solve(op, P2, xq, eta64.view(q), extra));
    info[q].iters += extra.iters;
    info[q].applies += extra.applies;
    info[q].outer_iters += extra.outer_iters;
    info[q].restarts += extra.restarts;
    info[q].true_rel_resid = extra.true_rel_resid;
  }
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  prof_flush(ctx);
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int q = 0; q < nr; ++q) info[q].ms = ms;
  return worst;
}
