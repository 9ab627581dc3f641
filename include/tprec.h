/*
 * tprec.h - C ABI of the temporally preconditioned anisotropic Wilson / SW
 * fermion solver for AMD Instinct MI355X (gfx950).
 *
 * Method: B. Joo, R. G. Edwards, M. J. Peardon, "An anisotropic preconditioning
 * for the Wilson fermion matrix on the lattice" (arXiv:0910.0992).  Section
 * references below are to that paper.
 *
 * The library solves (Sec. I)  M x = eta  with (Sec. II)
 *     M = A + mu - D_t - D_s / gamma_f,   mu = m0 + 1 + 3 / gamma_f,
 * on an Lx x Ly x Lz x Lt lattice, periodic in space, with time boundary
 * phase b = +1 (periodic) or -1 (antiperiodic).  A is the SW clover term
 * (zero for Wilson fermions).  The temporal matrix T (Sec. II.A) is inverted
 * exactly per time line, and combined with 3D even-odd ("temporal + Schur")
 * preconditioning (Sec. II.B).
 *
 * Conventions
 *   Canonical spinor: complex128, C order [Lt][Lz][Ly][Lx][4 spin][3 colour],
 *     spin in the Dirac-Pauli basis (gamma_t = diag(1,1,-1,-1)),
 *     gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_5 = g_x g_y g_z g_t.
 *   Canonical links: complex128 [4 dir][Lt][Lz][Ly][Lx][3][3], dir 0=x 1=y 2=z 3=t;
 *     U_mu(x) multiplies psi(x + mu) in the forward hop.
 *   Every spinor pointer passed to an apply/solve entry point is a DEVICE
 *   pointer to a canonical spinor, owned by the caller.  The library never
 *   frees caller memory and keeps no caller pointer after a call returns.
 *   Requirements: Lx, Ly, Lz even and >= 2, Lt >= 2; SCHUR4D needs Lt even.
 *
 * Streams and synchronisation
 *   All GPU work is enqueued on the stream set with tp_ctx_set_stream (default:
 *   the null stream).  Apply entry points do not synchronise.  tp_solve and
 *   the create functions synchronise the stream (they need scalars on the host).
 *   A context, together with the gauge, clover and operator handles created from
 *   it, may be used by one host thread at a time: they share the context's
 *   reduction buffers and the solver's device-side scalars.
 *
 * Errors
 *   Every entry point returns a tp_status.  On failure a message is available
 *   from tp_last_error() (thread-local, valid until the next call on the thread).
 */
#ifndef TPREC_H
#define TPREC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tp_status;
enum {
  TP_OK = 0,
  TP_EINVAL = -1,      /* null pointer, bad enum value, NaN/Inf in an input     */
  TP_EDIMS = -2,       /* odd spatial extent, Lt < 2, odd Lt for SCHUR4D        */
  TP_ESINGULAR = -3,   /* closure matrix or clover block numerically singular  */
  TP_ENOCONV = -4,     /* solver hit its iteration cap; x holds the best iterate */
  TP_EBREAKDOWN = -5,  /* BiCGStab breakdown that restarts could not cure      */
  TP_ENOMEM = -6,      /* device allocation failed                             */
  TP_EHIP = -7         /* other HIP runtime error                              */
};

enum { TP_HOST = 0, TP_DEVICE = 1 };

/* Preconditioning schemes (Sec. II.A-B). */
enum {
  TP_UNPREC = 0,          /* M itself                                              */
  TP_SCHUR4D = 1,         /* 4D even-odd Schur: diag(A+mu, S-hat) with p4 parity  */
  TP_TEMPORAL = 2,        /* C_L M C_R  (eq:ContaminatedUnprec for clover)        */
  TP_TEMPORAL_SCHUR = 3,  /* S_L M S_R with p3 parity: eq:TPrecFull (Wilson),
                             eq:TPrecPartial = 3D ILU (clover)                    */
  TP_TEMPORAL_SCHUR3D = 4 /* temporal preconditioning combined with 3D-Schur
                             (Sec. II.B, App. A): the even block M^ee = A + mu - D_t
                             is inverted exactly, Mt = diag(1, C_L^o S_o C_R^o) with
                             S_o = M^oo - M^oe (M^ee)^-1 M^eo.  F64 and F32 (not
                             F16N); the first use on an operator factors M^ee (FP64,
                             2304 bytes per even site, plus an FP32 copy of 1152 bytes
                             on the first F32 use, kept until tp_op_destroy)       */,
  TP_TEMPORAL_FULLSW = 5  /* full SW temporal preconditioning on the whole lattice
                             (Sec. II.A, App. A): T = A + mu - D_t inverted exactly,
                             C_L = T^-1, C_R = 1, so Mt = 1 - T^-1 D_s / gamma_f,
                             S_L = T^-1, S_R = 1.  Mt is not gamma5-hermitian
                             (Mt^dagger = gamma5 (1 - D_s T^-1 / gamma_f) gamma5).
                             F64 and F32 (not F16N); the first use factors T on
                             both parities (2304 bytes per site, plus 1152 per site
                             for FP32, kept until tp_op_destroy)                   */
};

enum { TP_CGNR = 0, TP_BICGSTAB = 1 };

/* Arithmetic/storage precision of the operator applies. */
enum {
  TP_F64 = 0,    /* FP64 storage and arithmetic                                  */
  TP_F32 = 1,    /* FP32 storage and arithmetic                                  */
  TP_F16N = 2    /* FP16 spinors with one FP32 scale per half-spinor and site,
                    FP16 links and clover, FP32 arithmetic (3D-parity schemes;
                    SCHUR4D takes F64 and F32)                                    */
};

typedef struct tp_ctx_s* tp_ctx;
typedef struct tp_gauge_s* tp_gauge;
typedef struct tp_clover_s* tp_clover;
typedef struct tp_op_s* tp_op;

/* Device allocator hooks (tp_ctx_set_allocator).  alloc returns `bytes` bytes of device
 * memory of the context's device, aligned to at least 256 bytes and usable on `stream`, or
 * NULL if it cannot; free releases a pointer that alloc returned, given the size asked for
 * and the stream bound to the context at the time of the free.  `user` is passed through. */
typedef void* (*tp_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*tp_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

/* ---- context ------------------------------------------------------------- */

/* Lattice geometry (dims = {Lx, Ly, Lz, Lt}), fermion time boundary phase
 * bc_t = +1 or -1 (Sec. II.A, the corner of T), and HIP device ordinal.
 * Returns TP_EDIMS for odd spatial extents or Lt < 2. */
tp_status tp_ctx_create(const int32_t dims[4], int32_t bc_t, int32_t device, tp_ctx* out);
tp_status tp_ctx_destroy(tp_ctx ctx);
/* hip_stream is a hipStream_t (NULL = default stream). */
tp_status tp_ctx_set_stream(tp_ctx ctx, void* hip_stream);
/* Routes every device allocation of the context and of the gauge, clover and operator
 * handles created from it (fields, workspaces, set-up temporaries) through alloc_fn and
 * free_fn, e.g. a framework's caching allocator, so that the caller owns all device memory.
 * Both NULL: back to hipMalloc / hipFree.  Must be called before the first tp_gauge_create
 * on the context (else TP_EINVAL); the context's own buffers move to the new allocator.
 * Every allocation made through the hooks is freed through them by the destroy calls.
 * Pinned host memory for reduction read-back is not device memory and stays hipHostMalloc. */
tp_status tp_ctx_set_allocator(tp_ctx ctx, tp_alloc_fn alloc_fn, tp_free_fn free_fn, void* user);
/* Device bytes currently held by the context and its handles. */
tp_status tp_ctx_device_bytes(tp_ctx ctx, size_t* bytes);

/* ---- gauge field ------------------------------------------------------------
 * Copies the canonical links (host or device pointer, per `where`) into the
 * library's layouts and prepares the per-time-line products used by T^-1:
 * W(t) = U_t(t) U_t(t+1) ... U_t(Lt-1) with the boundary phase folded into the
 * last link; W(0) is the Polyakov loop (Sec. II.A, the closed form of X).
 * Time links must be unitary (checked to 1e-10, else TP_EINVAL): the p3 operators
 * work in the axial frame rotated by W^dag (Sec. II.C), a gauge rotation only for
 * unitary W.  Spatial links may be any complex 3x3 matrices; when all of them are
 * SU(3) to 1e-9, the FP32 and FP16 kernels read their first two rows and rebuild
 * the third (FP64 kernels always read all nine entries).  Links containing NaN or
 * Inf are refused with TP_EINVAL. */
tp_status tp_gauge_create(tp_ctx ctx, const void* links, int32_t where, tp_gauge* out);
tp_status tp_gauge_destroy(tp_gauge g);
/* Mean plaquette diagnostics: spatial and temporal (1/3 Re tr) averages. */
tp_status tp_gauge_plaquette(tp_gauge g, double* plaq_s, double* plaq_t);

/* ---- clover term --------------------------------------------------------------
 * A = -(c_t/2) sum_i sigma_{it} F_{it} - (c_s/2) sum_{i<j} sigma_{ij} F_{ij}
 * (Sec. II, SW term) from four-leaf clover F_{mu nu}.  c_s, c_t are the
 * literal coefficients of that formula. */
tp_status tp_clover_create(tp_gauge g, double c_s, double c_t, tp_clover* out);
tp_status tp_clover_destroy(tp_clover c);

/* ---- operator -------------------------------------------------------------------
 * Binds M to (links, clover or NULL for Wilson, m0, gamma_f).  Computes the
 * closure of the temporal inverse per line, K = (I - mu^-Lt P)^-1 with P the
 * Polyakov loop including the phase (the Woodbury matrix Lambda of Sec. II.A),
 * in FP64; returns TP_ESINGULAR if its condition number exceeds 1e12.  Also
 * factorises (A + mu) per site for SCHUR4D (TP_ESINGULAR on a zero pivot). */
tp_status tp_op_create(tp_gauge g, tp_clover c, double m0, double gamma_f, tp_op* out);
tp_status tp_op_destroy(tp_op op);
/* The cutoff trick (Sec. II.A, eq:cutoff): every T^-1 and T^dagger^-1 of the operator's
 * applies, in every precision, drops the Woodbury correction X(t) Lambda chi(0) on the time
 * slices where its norm bound sqrt(3) mu^-(Lt-t) (T^-1) or sqrt(3) mu^-(t+1) (T^dagger^-1) is
 * below eps, and skips computing it there.  C_L and C_R, and the preconditioned operators
 * built from them, then differ from the exact ones by terms bounded that way; solves still
 * reach their FP64 true-residual target, whose residual uses M itself.  eps = 0 (the default)
 * restores the exact inverse.  dropped (may be NULL) receives the number of slices dropped
 * at each line's suppressed end.  TP_EINVAL for a negative or non-finite eps. */
tp_status tp_op_set_cutoff(tp_op op, double eps, int32_t* dropped);
/* The diagonal mass term mu = m0 + 1 + 3/gamma_f of M (Sec. II, a_t = 1). */
tp_status tp_op_mass(tp_op op, double* mu);

/* ---- applies (canonical device spinors in and out, dst != src) -----------------
 * `prec` selects the precision of the internal apply (TP_F64/F32/F16N); input
 * and output stay complex128.  `dagger` = 1 applies the adjoint. */

/* M psi (Sec. II). */
tp_status tp_apply_M(tp_op op, int32_t prec, void* dst, const void* src, int32_t dagger);
/* D_s psi = sum_i [P-^i U_i(x) psi(x+i) + P+^i U_i(x-i)^dag psi(x-i)] (Sec. II). */
tp_status tp_apply_Ds(tp_op op, int32_t prec, void* dst, const void* src);
/* A psi, or (A+mu) psi when plus_mu = 1, or (A+mu)^-1 psi when plus_mu = -1. */
tp_status tp_apply_clover(tp_op op, int32_t prec, void* dst, const void* src, int32_t plus_mu);
/* T^-1 (dagger=0) or (T^dagger)^-1 (dagger=1) on all four spins, each spatial
 * site independently (Sec. II.A, SMW algorithm). */
tp_status tp_apply_Tinv(tp_op op, int32_t prec, void* dst, const void* src, int32_t dagger);
/* C_L = P+ + P- T^-1 and C_R = P- + P+ (T^dagger)^-1 (Sec. II.A). */
tp_status tp_apply_CL(tp_op op, int32_t prec, void* dst, const void* src);
tp_status tp_apply_CR(tp_op op, int32_t prec, void* dst, const void* src);
/* The preconditioned operator Mt of `scheme` on the full lattice:
 *   UNPREC M; SCHUR4D diag(A+mu, (A+mu) - D_w^oe (A+mu)^-1 D_w^eo) in p4 parity;
 *   TEMPORAL C_L M C_R; TEMPORAL_SCHUR S_L M S_R in p3 parity; TEMPORAL_SCHUR3D
 *   diag(1, C_L^o S_o C_R^o) in p3 parity; TEMPORAL_FULLSW 1 - T^-1 D_s / gamma_f with
 *   T = A + mu - D_t, in p3 parity.  dagger = 1 applies Mt^dagger: gamma5 Mt gamma5 for all
 *   but TEMPORAL_FULLSW, whose adjoint is gamma5 (1 - D_s T^-1 / gamma_f) gamma5. */
tp_status tp_apply_prec(tp_op op, int32_t scheme, int32_t prec, void* dst, const void* src,
                        int32_t dagger);
/* tp_apply_prec for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same arguments, same
 * result; its work fields come from a fixed 64 MiB device array of the library (held by
 * every device the library runs on until the process ends) instead of the allocator, and it
 * calls no allocation routine.  Takes (fields of the apply's precision) x V x field bytes:
 * 2 (UNPREC), 3 (SCHUR4D), 4 (TEMPORAL), 6 (TEMPORAL_SCHUR), 7 (TEMPORAL_SCHUR3D),
 * 4 (TEMPORAL_FULLSW), with V x 192 bytes per F64 field, V x 96 per F32 and V x 56 per F16N;
 * a lattice that needs more than 64 MiB is refused with TP_EINVAL, as are TEMPORAL_SCHUR3D
 * and TEMPORAL_FULLSW before a tp_apply_prec of that scheme and precision has built their
 * factors.  All calls on one device share the
 * array: calls that overlap on one device (other streams, threads or contexts) race, and
 * the caller serialises them.  No per-kernel timing events are recorded. */
tp_status tp_apply_prec_noalloc(tp_op op, int32_t scheme, int32_t prec, void* dst, const void* src,
                                int32_t dagger);
/* eta~ = S_L eta and x = S_R y, with M = S_L^-1 Mt S_R^-1 for `scheme`
 * (SCHUR4D: S_L = L^-1, S_R = U^-1 of the LDU factorisation, Sec. II.B;
 * TEMPORAL_SCHUR3D: S_L = diag((M^ee)^-1, C_L^o) L^-1, S_R = U^-1 diag(1, C_R^o) with the
 * p3 LDU factorisation; TEMPORAL_FULLSW: S_L = (A + mu - D_t)^-1, S_R = 1). */
tp_status tp_prepare_source(tp_op op, int32_t scheme, int32_t prec, void* eta_tilde,
                            const void* eta);
tp_status tp_reconstruct(tp_op op, int32_t scheme, int32_t prec, void* x, const void* y);

/* ---- fields in the library's layouts -----------------------------------------------
 * The paper's flow is a one-off set-up, then per right-hand side a source preparation,
 * applies of the preconditioned operator and a reconstruction (Sec. II.A-B).  A tp_field lets
 * a caller (for example its own Krylov solver) keep fields in the library's internal layout
 * and precision between calls instead of converting from and to canonical complex128 in every
 * call.  Internal buffers are opaque device memory of tp_field_bytes() bytes per right-hand
 * side, owned by the caller; the right-hand sides of a batch lie back to back.
 *   TP_LAYOUT_CANONICAL  complex128 [Lt][Lz][Ly][Lx][4][3] (prec TP_F64, subset FULL only)
 *   TP_LAYOUT_P3         3D-parity (x+y+z) layout in the axial frame of the gauge field: the
 *                        layout of UNPREC, TEMPORAL, TEMPORAL_SCHUR, TEMPORAL_SCHUR3D and
 *                        TEMPORAL_FULLSW
 *   TP_LAYOUT_P4         4D-parity (x+y+z+t) layout: the layout of SCHUR4D
 * Both internal layouts are unitary images of the canonical field (a permutation of sites
 * and components, and for P3 a colour rotation per site), so inner products and norms of F64
 * internal fields, read as complex128 vectors, equal those of the canonical fields.
 * subset: TP_SUBSET_FULL, or one parity of the layout (TP_SUBSET_EVEN / TP_SUBSET_ODD),
 * stored alone in half the memory. */
enum { TP_LAYOUT_CANONICAL = 0, TP_LAYOUT_P3 = 1, TP_LAYOUT_P4 = 2 };
enum { TP_SUBSET_FULL = 0, TP_SUBSET_EVEN = 1, TP_SUBSET_ODD = 2 };
typedef struct {
  void* data;      /* device pointer                                                   */
  int32_t layout;  /* TP_LAYOUT_*                                                      */
  int32_t prec;    /* TP_F64, TP_F32, TP_F16N (internal layouts); TP_F64 for canonical  */
  int32_t subset;  /* TP_SUBSET_*                                                      */
  int32_t nrhs;    /* right-hand sides stored back to back (1..16)                      */
} tp_field;

/* Bytes of one right-hand side of a field with this layout, precision and subset. */
tp_status tp_field_bytes(tp_op op, int32_t layout, int32_t prec, int32_t subset, size_t* bytes);
/* dst = src between layouts, precisions and subsets (same nrhs).  Canonical <-> internal
 * converts (with the axial-frame rotation for P3); internal -> internal needs one layout and
 * changes precision (FP16 storage rounds, with a scale per half spinor) and subset: a FULL
 * source gives the chosen parity, a one-parity source fills the same parity, and the other
 * parity of a FULL destination is set to zero. */
tp_status tp_field_convert(tp_op op, const tp_field* dst, const tp_field* src);
/* dst = Mt src (Mt^dagger with dagger = 1) on internal fields of `scheme`'s layout, one
 * precision: FULL fields, or TP_SUBSET_ODD fields for the schemes whose even block is solved
 * directly (SCHUR4D, TEMPORAL_SCHUR3D, TEMPORAL_SCHUR without clover), where the odd block is
 * the operator a Krylov solver iterates on.  dst and src must not overlap. */
tp_status tp_apply_prec_field(tp_op op, int32_t scheme, const tp_field* dst, const tp_field* src,
                              int32_t dagger);
/* eta_tilde = S_L eta and x = S_R y with fields: eta_tilde and y are FULL internal fields of
 * the scheme's layout (their precision is the precision of the maps); eta and x may be
 * canonical or FULL internal fields of that layout and precision.  For the schemes solved on
 * the odd block the even part of y is eta_tilde's (TEMPORAL_SCHUR without clover,
 * TEMPORAL_SCHUR3D) or (A + mu)^-1 eta_tilde_e (SCHUR4D). */
tp_status tp_prepare_source_field(tp_op op, int32_t scheme, const tp_field* eta_tilde,
                                  const tp_field* eta);
tp_status tp_reconstruct_field(tp_op op, int32_t scheme, const tp_field* x, const tp_field* y);

/* ---- solve ------------------------------------------------------------------------ */
typedef struct {
  int32_t scheme;          /* TP_UNPREC ... TP_TEMPORAL_FULLSW                      */
  int32_t solver;          /* TP_CGNR or TP_BICGSTAB                                */
  int32_t prec;            /* inner precision: TP_F64, TP_F32, TP_F16N              */
  int32_t max_iter;        /* cap on inner Krylov iterations summed over restarts  */
  int32_t max_restarts;    /* cap on FP64 corrections (updates or cycles)           */
  int32_t use_x0;          /* 1: x holds the initial guess on entry                 */
  int32_t estimate_kappa;  /* 1 (CGNR only): Lanczos estimate of kappa(Mt^dag Mt)  */
  int32_t dagger;          /* 1: solve M^dagger x = eta instead (as M (g5 x) = g5 eta,
                              M^dagger = g5 M g5, with the same preconditioned solver) */
  double tol;              /* target true relative residual |eta - M x| / |eta|     */
  double inner_tol;        /* BiCGStab in F32/F16N: reliable-update threshold delta
                              (0 = default 1e-3 F32, 0.01 F16N); CGNR: relative
                              reduction per inner solve (0 = 1e-6 F32, 2e-3 F16N)   */
} tp_solve_params;

typedef struct {
  int32_t iters;           /* inner Krylov iterations, all cycles                   */
  int32_t outer_iters;     /* FP64 corrections: reliable updates or cycles          */
  int32_t applies;         /* preconditioned-operator applies                       */
  int32_t restarts;        /* BiCGStab breakdown restarts                           */
  double true_rel_resid;   /* FP64 |eta - M x| / |eta| at exit                      */
  double prec_rel_resid;   /* last inner relative residual                          */
  double kappa_est;        /* Lanczos kappa of Mt^dag Mt (CGNR), else 0             */
  double lambda_min, lambda_max;
  double ms;               /* wall time of the solve                                */
} tp_solve_info;

/* Solves M x = eta (or M^dagger x = eta with params->dagger; canonical device
 * spinors) to the FP64 true relative
 * residual `tol` with the preconditioned operator Mt = S_L M S_R of `scheme`
 * (eta~ = S_L r, Krylov on Mt y = eta~ in `prec`, x += S_R y, r = eta - M x in
 * FP64).  F64: one Krylov solve.  F32/F16N BiCGStab: reliable updates (Sleijpen
 * and van der Vorst 1996): when the recursive residual has dropped by delta below
 * its maximum since the last update, y is folded into x in FP64 and the recursion
 * continues from the preconditioned FP64 true residual, keeping its search
 * direction.  CGNR, and BiCGStab after a stall, use defect correction: each cycle
 * restarts the Krylov solve on the new residual.  Returns TP_ENOCONV with x = best
 * iterate if the caps are reached. */
tp_status tp_solve(tp_op op, const tp_solve_params* params, void* x, const void* eta,
                   tp_solve_info* info);

/* Solves M x[k] = eta[k] (M^dagger with params->dagger) for k < nrhs (1..16) with the
 * same parameters.  For
 * mixed-precision BiCGStab on the full-lattice schemes (UNPREC, TEMPORAL, and
 * TEMPORAL_SCHUR with clover) the right-hand sides iterate in lockstep: every
 * operator application is one launch per kernel for all of them, so links and
 * clover are read once per site for the batch, and each inner product is one
 * synchronisation; scalars, reliable updates and stopping are per right-hand
 * side.  Other settings solve the right-hand sides one after another.  x[k],
 * eta[k]: canonical device spinors (x[k] distinct, none equal to any eta);
 * info: array of nrhs.  Returns the worst status over the right-hand sides. */
tp_status tp_solve_multi(tp_op op, const tp_solve_params* params, int32_t nrhs, void* const* x,
                         const void* const* eta, tp_solve_info* info);

/* ---- gradient ----------------------------------------------------------------------
 * Link gradient of a real L(x) with x = M^-1 eta and lambda = M^-dagger dL/dx* (for
 * L = |x|^2: M^dagger lambda = 2x), dL = -Re <lambda, dM x>.  The hopping terms give, per
 * link U_mu(s),
 *   Y = sum_a [P-^mu x(s+mu)]_a lambda(s)_a^dag,  Z = sum_a [P+^mu x(s)]_a lambda(s+mu)_a^dag,
 *   grad_U = k_mu b_mu(s) (Y + Z^dag)^dag,
 * with k_t = 1, k_i = 1/gamma_f, b_mu(s) = bc_t on time links of the last slice.  With a
 * clover term the SW part is added (unless TP_FORCE_HOPPING_ONLY): A depends on the links
 * through the four-leaf field strength (Sec. II), and each plaquette containing the link
 * contributes the product of its other three links with, at every corner x,
 * (c/2)(Zc - Zc^dag), Zc = W/8 - tr(W)/24, W = sum sigma_{mu nu}[s][s'] x_s'(x) lambda_s(x)^dag.
 * Raw form: d L = Re <grad_U, dU>.  TP_FORCE_PROJECTED: G = TH[i U grad_U^dag] with
 * dL/dh = tr(omega G) for U -> exp(i h omega) U, TH = traceless hermitian part.
 * x, lambda: canonical device spinors; grad_links: device complex128
 * [4][Lt][Lz][Ly][Lx][3][3], overwritten. */
enum { TP_FORCE_PROJECTED = 1, TP_FORCE_HOPPING_ONLY = 2 };
tp_status tp_force(tp_op op, const void* x, const void* lambda, void* grad_links, int32_t flags);

/* ---- diagnostics -------------------------------------------------------------------- */
const char* tp_status_string(tp_status s);
const char* tp_last_error(void);
/* Per-kernel timing with HIP events on the bound stream. */
tp_status tp_prof_enable(tp_ctx ctx, int32_t on);
/* Time only the kernel groups whose bit (1 << id) is set in mask (all groups until this is
 * called); launches of the other groups record no events, so timing one group costs the
 * others nothing.  EINVAL for a null context. */
tp_status tp_prof_select(tp_ctx ctx, uint32_t mask);
tp_status tp_prof_reset(tp_ctx ctx);
/* id in [0, tp_prof_count()): launches, summed milliseconds, algorithmic bytes. */
int32_t tp_prof_count(void);
const char* tp_prof_name(int32_t id);
tp_status tp_prof_get(tp_ctx ctx, int32_t id, int64_t* launches, double* total_ms,
                      double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* TPREC_H */
