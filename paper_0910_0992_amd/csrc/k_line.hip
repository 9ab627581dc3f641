// Dispatch of the time-line kernels to their per-precision instantiations
// (k_line_f64.hip, k_line_f32.hip, k_line_f16.hip) and their byte accounting.
#include "tp_internal.h"

#define TP_DECL(sfx)                                                                             \
  void line_plain_##sfx(tp_op, int, int, const Field&, Field&);                                   \
  void line_half_cr_##sfx(tp_op, const Field&, Field&);                                           \
  void line_sten_##sfx(tp_op, int, int, const LineStencilArgs&, Field&);                          \
  void ilu_k2a_##sfx(tp_op, const Field&, const Field&, Field&, Field&);                          \
  void ilu_k2b_##sfx(tp_op, const Field&, const Field&, const Field&, Field&, Field&);            \
  void ilu_k3_##sfx(tp_op, const Field&, const Field&, const Field&, Field&);
TP_DECL(f64)
TP_DECL(f32)
TP_DECL(f16)

#define TP_DISPATCH(prec, fn, ...)          \
  switch (prec) {                           \
    case TP_F64: fn##f64(__VA_ARGS__); break; \
    case TP_F32: fn##f32(__VA_ARGS__); break; \
    default: fn##f16(__VA_ARGS__); break;     \
  }

namespace {
double spinor_bytes(int prec) { return prec == TP_F64 ? 192 : (prec == TP_F32 ? 96 : 56); }
double link_bytes(int prec) { return prec == TP_F64 ? 144 : 72; }
double clov_bytes(int prec) { return prec == TP_F64 ? 576 : 288; }
}  // namespace

void launch_line_plain(tp_op op, int prec, int mode, int par, const Field& src, Field& dst) {
  const Lattice& L = op->g->ctx->lat;
  double S = spinor_bytes(prec), Lb = link_bytes(prec);
  double nhalf = (mode == LM_CRCL || mode == LM_TINV || mode == LM_TDINV) ? 2 : 1;
  bool pass = src.data != dst.data;
  double per = nhalf * S + Lb + (pass ? (2 - nhalf) * S : 0);
  ProfScope ps(op->g->ctx, KID_LINE_CR, double(L.V2) * per);
  TP_DISPATCH(prec, line_plain_, op, mode, par, src, dst)
}

void launch_line_stencil(tp_op op, int prec, int mode, int par, const LineStencilArgs& s, Field& dst) {
  const Lattice& L = op->g->ctx->lat;
  double S = spinor_bytes(prec), Lb = link_bytes(prec), C = clov_bytes(prec);
  double per = S + 6 * Lb + Lb + S + (s.self ? S : 0) + (s.self && s.c_A != 0 && op->c ? C : 0) +
               (s.base ? S : 0);
  ProfScope ps(op->g->ctx, KID_LINE_STENCIL, double(L.V2) * per);
  TP_DISPATCH(prec, line_sten_, op, mode, par, s, dst)
}

void launch_ilu_k1(tp_op op, int prec, const Field& psi, Field& aup) {
  // a_o = C_R psi_o: only the scanned upper half is written (the lower half is psi_o's)
  const Lattice& L = op->g->ctx->lat;
  ProfScope ps(op->g->ctx, KID_LINE_CR, double(L.V2) * (spinor_bytes(prec) + link_bytes(prec)));
  TP_DISPATCH(prec, line_half_cr_, op, psi, aup)
}

void launch_ilu_k2a(tp_op op, int prec, const Field& psi, const Field& aup, Field& y, Field& u) {
  const Lattice& L = op->g->ctx->lat;
  double S = spinor_bytes(prec), Lb = link_bytes(prec), C = clov_bytes(prec);
  ProfScope ps(op->g->ctx, KID_ILU_K2A, double(L.V2) * (S + 6 * Lb + S + Lb + C + 2 * S));
  TP_DISPATCH(prec, ilu_k2a_, op, psi, aup, y, u)
}

void launch_ilu_k2b(tp_op op, int prec, const Field& psi, const Field& y, const Field& u, Field& chi,
                    Field& n) {
  const Lattice& L = op->g->ctx->lat;
  double S = spinor_bytes(prec), Lb = link_bytes(prec);
  ProfScope ps(op->g->ctx, KID_ILU_K2B, double(L.V2) * (5 * S + Lb));
  TP_DISPATCH(prec, ilu_k2b_, op, psi, y, u, chi, n)
}

void launch_ilu_k3(tp_op op, int prec, const Field& psi, const Field& aup, const Field& n, Field& chi) {
  // chi_o = psi_o + C_L [A a_o + D_s^oe n_e / gamma_f],  a_o = (aup upper, psi_o lower)
  const Lattice& L = op->g->ctx->lat;
  double S = spinor_bytes(prec), Lb = link_bytes(prec), C = clov_bytes(prec);
  ProfScope ps(op->g->ctx, KID_ILU_K3, double(L.V2) * (S + 6 * Lb + 1.5 * S + (op->c ? C : 0) + Lb + S));
  TP_DISPATCH(prec, ilu_k3_, op, psi, aup, n, chi)
}
