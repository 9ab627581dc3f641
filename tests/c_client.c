/* A C client of the tprec library: everything through include/tprec.h and the HIP runtime,
 * no Python.  Built and run by tests/test_c_client.py.
 *
 *   c_client --host-checks   argument checks that need no GPU
 *   c_client                 a temporally preconditioned clover solve on a free-field
 *                            lattice, FP16 and FP32 inner precision, whose FP64 residual is
 *                            recomputed here from tp_apply_M
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

static int host_checks(void) {
  tp_ctx ctx = NULL;
  const int32_t odd[4] = {3, 4, 4, 8};
  if (tp_ctx_create(odd, -1, 0, &ctx) != TP_EDIMS || ctx) return 1;
  const int32_t ok[4] = {4, 4, 4, 8};
  if (tp_ctx_create(ok, 0, 0, &ctx) != TP_EINVAL) return 1;
  if (tp_solve(NULL, NULL, NULL, NULL, NULL) != TP_EINVAL) return 1;
  if (tp_force(NULL, NULL, NULL, NULL, 0) != TP_EINVAL) return 1;
  if (strcmp(tp_status_string(TP_ENOCONV), "solver did not converge") != 0) return 1;
  printf("host checks ok\n");
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && strcmp(argv[1], "--host-checks") == 0) return host_checks();
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
