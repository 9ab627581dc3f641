/* A C client of the tprec library: everything through include/tprec.h and the HIP runtime,
 * no Python.  Built and run by tests/test_c_client.py.
 *
 *   c_client --host-checks   argument checks that need no GPU
 *   c_client                 a temporally preconditioned clover solve on a free-field
 *                            lattice, FP16 and FP32 inner precision, whose FP64 residual is
 *                            recomputed here from tp_apply_M; a dagger solve checked the same
 *                            way; links with a NaN refused
 *   c_client --allocator     every device allocation of the library goes through a counting
 *                            allocator registered with tp_ctx_set_allocator (a bump allocator
 *                            over an arena of the client's): the device's free memory outside
 *                            the arena does not move, and the destroy calls free all of it
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tprec.h"

#define CHECK(call)                                                                       \
  do {                                                                                    \
    tp_status s_ = (call);                                                                \
    if (s_ != TP_OK) {                                                                    \
      fprintf(stderr, "FAIL %s -> %d (%s)\n", #call, (int)s_, tp_last_error());          \
      return 1;                                                                           \
    }                                                                                     \
  } while (0)

/* Counting allocator: a bump allocator over one arena the client allocates up front, so that
 * after the arena exists any device allocation that bypassed the hooks would lower the
 * device's free memory. */
typedef struct {
  char* arena;
  size_t cap, top;
  long n_alloc, n_free;
  size_t live;
} counter_t;

static void* count_alloc(size_t bytes, void* stream, void* user) {
  counter_t* c = (counter_t*)user;
  (void)stream;
  size_t need = (bytes + 255) & ~(size_t)255;
  if (c->top + need > c->cap) return NULL;
  void* p = c->arena + c->top;
  c->top += need;
  c->n_alloc++;
  c->live += bytes;
  return p;
}

static void count_free(void* p, size_t bytes, void* stream, void* user) {
  counter_t* c = (counter_t*)user;
  (void)stream;
  (void)p;
  c->n_free++;
  c->live -= bytes;
}

/* One clover solve on a 16^3x8 free field with the counting allocator; with `measure`, the
 * device's free memory after the arena exists is compared before and after the set-up and
 * the solves. */
static int allocator_pass(int measure) {
  const int32_t dims[4] = {16, 16, 16, 8};
  const size_t V = 16 * 16 * 16 * 8;
  const size_t nsp = V * 12, nlk = 4 * V * 9;
  double* links = (double*)calloc(2 * nlk, sizeof(double));
  double* eta = (double*)calloc(2 * nsp, sizeof(double));
  for (size_t l = 0; l < 4 * V; ++l)
    for (int a = 0; a < 3; ++a) links[2 * (l * 9 + 4 * a)] = 1.0;
  eta[2 * 7] = 1.0;
  void *d_eta, *d_x;
  counter_t cnt = {NULL, (size_t)1 << 30, 0, 0, 0, 0};
  if (hipMalloc((void**)&cnt.arena, cnt.cap) != hipSuccess) return 1;
  if (hipMalloc(&d_eta, 2 * nsp * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&d_x, 2 * nsp * sizeof(double)) != hipSuccess) return 1;
  if (hipMemcpy(d_eta, eta, 2 * nsp * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 1;
  if (hipDeviceSynchronize() != hipSuccess) return 1;
  size_t free0 = 0, free1 = 0, total = 0;
  if (hipMemGetInfo(&free0, &total) != hipSuccess) return 1;
  tp_ctx ctx;
  tp_gauge g;
  tp_clover c;
  tp_op op;
  CHECK(tp_ctx_create(dims, -1, 0, &ctx));
  CHECK(tp_ctx_set_allocator(ctx, count_alloc, count_free, &cnt));
  CHECK(tp_gauge_create(ctx, links, TP_HOST, &g));
  if (tp_ctx_set_allocator(ctx, NULL, NULL, NULL) != TP_EINVAL) return 1; /* too late */
  CHECK(tp_clover_create(g, 0.5, 1.0, &c));
  CHECK(tp_op_create(g, c, -0.05, 2.0, &op));
  tp_solve_params P;
  memset(&P, 0, sizeof P);
  P.scheme = TP_TEMPORAL_SCHUR;
  P.solver = TP_BICGSTAB;
  P.prec = TP_F16N;
  P.tol = 1e-10;
  tp_solve_info info;
  CHECK(tp_solve(op, &P, d_x, d_eta, &info));
  P.scheme = TP_SCHUR4D;
  P.prec = TP_F64;
  CHECK(tp_solve(op, &P, d_x, d_eta, &info));
  P.scheme = TP_TEMPORAL_SCHUR3D;
  CHECK(tp_solve(op, &P, d_x, d_eta, &info));
  if (hipDeviceSynchronize() != hipSuccess) return 1;
  if (hipMemGetInfo(&free1, &total) != hipSuccess) return 1;
  size_t lib_bytes = 0;
  CHECK(tp_ctx_device_bytes(ctx, &lib_bytes));
  const double drop = (double)free0 - (double)free1;
  if (measure)
    printf("allocator: %ld allocations, %.1f MB live (library reports %.1f MB); device free memory "
           "outside the arena changed by %.2f MB\n", cnt.n_alloc, cnt.live / 1e6, lib_bytes / 1e6,
           drop / 1e6);
  if (lib_bytes != cnt.live || cnt.n_alloc == 0) return 1;
  /* nothing but the runtime's own bookkeeping (far below one field of 9.4 MB) left the pool */
  if (measure && drop > 2.0 * (1 << 20)) {
    printf("device memory allocated outside the registered allocator\n");
    return 1;
  }
  CHECK(tp_op_destroy(op));
  CHECK(tp_clover_destroy(c));
  CHECK(tp_gauge_destroy(g));
  CHECK(tp_ctx_destroy(ctx));
  if (cnt.live != 0 || cnt.n_free != cnt.n_alloc) {
    printf("allocator: %ld allocations, %ld frees, %zu bytes left\n", cnt.n_alloc, cnt.n_free, cnt.live);
    return 1;
  }
  hipFree(d_eta);
  hipFree(d_x);
  hipFree(cnt.arena);
  free(links);
  free(eta);
  return 0;
}

static int host_checks(void) {
  tp_ctx ctx = NULL;
  const int32_t odd[4] = {3, 4, 4, 8};
  if (tp_ctx_create(odd, -1, 0, &ctx) != TP_EDIMS || ctx) return 1;
  const int32_t ok[4] = {4, 4, 4, 8};
  if (tp_ctx_create(ok, 0, 0, &ctx) != TP_EINVAL) return 1;
  if (tp_solve(NULL, NULL, NULL, NULL, NULL) != TP_EINVAL) return 1;
  if (tp_force(NULL, NULL, NULL, NULL, 0) != TP_EINVAL) return 1;
  if (tp_ctx_set_allocator(NULL, count_alloc, count_free, NULL) != TP_EINVAL) return 1;
  if (tp_op_mass(NULL, NULL) != TP_EINVAL) return 1;
  if (strcmp(tp_status_string(TP_ENOCONV), "solver did not converge") != 0) return 1;
  printf("host checks ok\n");
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && strcmp(argv[1], "--host-checks") == 0) return host_checks();
  if (argc > 1 && strcmp(argv[1], "--allocator") == 0) {
    /* the first pass loads the code objects; the second is measured */
    if (allocator_pass(0) || allocator_pass(1)) return 1;
    printf("allocator ok\n");
    return 0;
  }
  const int32_t dims[4] = {4, 4, 4, 8};
  const size_t V = 4 * 4 * 4 * 8;
  const size_t nsp = V * 12, nlk = 4 * V * 9;
  double* links = (double*)calloc(2 * nlk, sizeof(double));
  double* eta = (double*)calloc(2 * nsp, sizeof(double));
  double* out = (double*)calloc(2 * nsp, sizeof(double));
  for (size_t l = 0; l < 4 * V; ++l)
    for (int a = 0; a < 3; ++a) links[2 * (l * 9 + 4 * a)] = 1.0; /* unit links */
  eta[2 * (12 * 5 + 3 * 1 + 2)] = 1.0;                          /* spin 1, colour 2, site 5 */

  tp_ctx ctx;
  tp_gauge g;
  tp_clover c;
  tp_op op;
  CHECK(tp_ctx_create(dims, -1, 0, &ctx));
  CHECK(tp_gauge_create(ctx, links, TP_HOST, &g));
  CHECK(tp_clover_create(g, 0.5, 1.0, &c));
  CHECK(tp_op_create(g, c, -0.05, 2.0, &op));
  double mu = 0;
  CHECK(tp_op_mass(op, &mu));
  if (fabs(mu - (-0.05 + 1.0 + 3.0 / 2.0)) > 1e-15) return 1;
  void *d_eta, *d_x, *d_mx;
  if (hipMalloc(&d_eta, 2 * nsp * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&d_x, 2 * nsp * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&d_mx, 2 * nsp * sizeof(double)) != hipSuccess) return 1;
  if (hipMemcpy(d_eta, eta, 2 * nsp * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 1;
  const int32_t precs[2] = {TP_F16N, TP_F32};
  for (int k = 0; k < 2; ++k) {
    tp_solve_params P;
    memset(&P, 0, sizeof P);
    P.scheme = TP_TEMPORAL_SCHUR;
    P.solver = TP_BICGSTAB;
    P.prec = precs[k];
    P.tol = 1e-10;
    tp_solve_info info;
    CHECK(tp_solve(op, &P, d_x, d_eta, &info));
    CHECK(tp_apply_M(op, TP_F64, d_mx, d_x, 0));
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    if (hipMemcpy(out, d_mx, 2 * nsp * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;
    double r2 = 0, e2 = 0;
    for (size_t q = 0; q < 2 * nsp; ++q) {
      r2 += (eta[q] - out[q]) * (eta[q] - out[q]);
      e2 += eta[q] * eta[q];
    }
    const double rel = sqrt(r2 / e2);
    printf("prec %d: %d iterations, reported %.3e, recomputed %.3e\n", (int)precs[k], (int)info.iters,
           info.true_rel_resid, rel);
    if (!(info.true_rel_resid <= 1e-10) || !(rel <= 1.05e-10)) return 1;
    /* M^dagger x = eta, checked with tp_apply_M(dagger = 1) */
    P.dagger = 1;
    CHECK(tp_solve(op, &P, d_x, d_eta, &info));
    CHECK(tp_apply_M(op, TP_F64, d_mx, d_x, 1));
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    if (hipMemcpy(out, d_mx, 2 * nsp * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;
    r2 = 0;
    for (size_t q = 0; q < 2 * nsp; ++q) r2 += (eta[q] - out[q]) * (eta[q] - out[q]);
    printf("prec %d dagger: %d iterations, recomputed %.3e\n", (int)precs[k], (int)info.iters,
           sqrt(r2 / e2));
    if (!(sqrt(r2 / e2) <= 1.05e-10)) return 1;
  }
  {
    /* links with a NaN are refused */
    tp_gauge gbad = NULL;
    links[2 * (9 * 17 + 4) + 1] = NAN;
    if (tp_gauge_create(ctx, links, TP_HOST, &gbad) != TP_EINVAL || gbad) return 1;
    links[2 * (9 * 17 + 4) + 1] = 0.0;
  }
  hipFree(d_eta);
  hipFree(d_x);
  hipFree(d_mx);
  CHECK(tp_op_destroy(op));
  CHECK(tp_clover_destroy(c));
  CHECK(tp_gauge_destroy(g));
  CHECK(tp_ctx_destroy(ctx));
  free(links);
  free(eta);
  free(out);
  printf("solve ok\n");
  return 0;
}
