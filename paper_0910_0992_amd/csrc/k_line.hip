// Dispatch of the time-line kernels to their per-precision instantiations
// (k_line_f64.hip, k_line_f32.hip, k_line_f16.hip) and their byte accounting.
#include "tp_internal.h"

#define TP_DECL(sfx)                                                                    \
  void line_##sfx(tp_op, int, int, const LineIO&, Field&);                               \
  void ilu_mid_##sfx(tp_op, const Field&, const Field&, Field&, Field&);
TP_DECL(f64)
TP_DECL(f32)
TP_DECL(f16)

#define TP_DISPATCH(prec, fn, ...)            \
  switch (prec) {                             \
    case TP_F64: fn##f64(__VA_ARGS__); break; \
    case TP_F32: fn##f32(__VA_ARGS__); break; \
    default: fn##f16(__VA_ARGS__); break;     \
  }

double spinor_bytes(int prec) { return prec == TP_F64 ? 192 : (prec == TP_F32 ? 96 : 56); }
double link_bytes(int prec) { return prec == TP_F64 ? 144 : (prec == TP_F32 ? 72 : 36); }
double clov_bytes(int prec) { return prec == TP_F64 ? 576 : (prec == TP_F32 ? 288 : 144); }

void launch_line(tp_op op, int prec, int mode, int par, const LineIO& io, Field& dst) {
  const Lattice& L = op->g->ctx->lat;
  double hs = spinor_bytes(prec) / 2;
  int nscan = (mode == LM_CRCL || mode == LM_TINV || mode == LM_TDINV) ? 2 : 1;
  int nio = io.pass ? 2 : nscan;  // halves read and written
  double per = nio * 2 * hs + (io.base ? nio * hs : 0);
  const int kid = mode == LM_CR ? KID_SCAN_CR : (mode == LM_CL ? KID_SCAN_CL : KID_SCAN_OTHER);
  ProfScope ps(op->g->ctx, kid, double(L.V2) * per * dst.nr);
  TP_DISPATCH(prec, line_, op, mode, par, io, dst)
}

void launch_ilu_mid(tp_op op, int prec, const Field& psi, const Field& u, Field& chi, Field& n) {
  // reads psi_e, u, A_e; writes chi_e, n_e
  const Lattice& L = op->g->ctx->lat;
  double S = spinor_bytes(prec), C = clov_bytes(prec);
  ProfScope ps(op->g->ctx, KID_ILU_MID, double(L.V2) * (4 * S * chi.nr + C));
  TP_DISPATCH(prec, ilu_mid_, op, psi, u, chi, n)
}
