/* Host-side checks of the C ABI's argument validation, built against a library whose
 * host code carries AddressSanitizer and UndefinedBehaviorSanitizer (device code is
 * not compiled in): every call here must be rejected (or be a no-op) on the host
 * before any GPU work, so it runs without a GPU.  Pointers are fake and never
 * dereferenced.  Exit status 0 when every status matches. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mlpcp.h"

static int failures = 0;

#define EXPECT(call, want)                                                              \
  do {                                                                                  \
    const int got_ = (int)(call);                                                       \
    if (got_ != (want)) {                                                               \
      fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, got_, \
              (int)(want));                                                             \
      ++failures;                                                                       \
    }                                                                                   \
  } while (0)

static int coarse_ref(int n, int levels) {
  if (levels < 0 || n < 1) return MLPCP_E_LEVELS;
  for (int l = 0; l < levels; ++l) {
    if (n < 2) return MLPCP_E_LEVELS;
    n = (n % 2 == 0) ? n / 2 : (n + 1) / 2;
  }
  return n;
}

int main(void) {
  const float* D = (const float*)4096;
  float* L = (float*)8192;
  float* S = (float*)12288;
  float* Y = (float*)16384;
  const uint8_t* Q = (const uint8_t*)20480;
  void* ws = (void*)24576;
  mlpcp_opts o;
  mlpcp_default_opts(NULL);
  mlpcp_default_opts(&o);
  if (o.levels != 0 || o.tol != 1e-6 || o.max_iter != 500 || o.rho != 1.5 || o.prec != MLPCP_FP32) ++failures;

  for (int n = 0; n < 300; ++n)
    for (int l = -1; l < 10; ++l) EXPECT(mlpcp_coarse_dim(n, l), coarse_ref(n, l));

  EXPECT(mlpcp_workspace_bytes(10, 20, &o), 0);
  if (mlpcp_workspace_bytes(2000, 2000, NULL) == 0) ++failures;
  for (int s = -9; s <= 2; ++s)
    if (mlpcp_status_string(s) == NULL || strlen(mlpcp_status_string(s)) == 0) ++failures;

  /* pcp / cpcp solve */
  EXPECT(mlpcp_pcp_solve(10, 20, D, 20, 0.1f, 1.0, NULL, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_SHAPE);
  EXPECT(mlpcp_pcp_solve(20, 10, D, 5, 0.1f, 1.0, NULL, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.0f, 1.0, NULL, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, NAN, NULL, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_pcp_solve(20, 10, NULL, 10, 0.1f, 1.0, NULL, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 1.0, NULL, NULL, NULL, L, L, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 0.0, NULL, L, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  mlpcp_opts bad = o;
  bad.levels = 9;
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 1.0, &bad, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_LEVELS);
  bad = o;
  bad.tol = -1.0;
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 1.0, &bad, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  bad = o;
  bad.check_every = 2;
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 1.0, &bad, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_UNSUPPORTED);
  bad = o;
  bad.svt_method = 5;
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 1.0, &bad, NULL, NULL, L, S, NULL, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_pcp_solve(20, 10, D, 10, 0.1f, 1.0, NULL, NULL, NULL, L, S, NULL, ws, 16, NULL, NULL),
         MLPCP_E_WORKSPACE);
  EXPECT(mlpcp_cpcp_solve(20, 10, D, 10, NULL, 0.1f, 1.0, NULL, NULL, NULL, L, S, Y, NULL, 0, NULL, NULL),
         MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_cpcp_solve(5, 10, D, 10, Q, 0.1f, 1.0, NULL, NULL, NULL, L, S, Y, NULL, 0, NULL, NULL), MLPCP_E_SHAPE);

  /* svt_prox and its allocation-free variant */
  EXPECT(mlpcp_svt_prox(20, 10, D, 10, 1, 0.0f, L, NULL, NULL, 0, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_svt_prox(20, 10, D, 10, 7, 1.0f, L, NULL, NULL, 0, NULL), MLPCP_E_LEVELS);
  EXPECT(mlpcp_svt_prox(20, 10, D, 10, 1, 1.0f, L, NULL, ws, 8, NULL), MLPCP_E_WORKSPACE);
  EXPECT(mlpcp_svt_prox_static(10, 20, D, 20, 1, 1.0f, L, NULL, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_svt_prox_static(20, 10, NULL, 10, 1, 1.0f, L, NULL, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_svt_prox_static(40000, 1000, D, 1000, 0, 1.0f, L, NULL, NULL), MLPCP_E_WORKSPACE);

  /* streaming operators */
  EXPECT(mlpcp_shrink(0, NULL, 0.5f, NULL, NULL), MLPCP_OK);
  EXPECT(mlpcp_shrink(16, NULL, 0.5f, L, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_shrink(16, D, -1.0f, L, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_shrink(16, D, INFINITY, L, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_restrict(0, 10, D, 10, 1, L, 5, NULL), MLPCP_OK);
  EXPECT(mlpcp_restrict(4, 10, D, 9, 1, L, 5, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_restrict(4, 10, D, 10, 1, L, 4, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_restrict(4, 10, D, 10, 9, L, 5, NULL), MLPCP_E_LEVELS);
  EXPECT(mlpcp_restrict(4, 10, NULL, 10, 1, L, 5, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_prolong(0, 10, D, 5, 1, L, 10, NULL), MLPCP_OK);
  EXPECT(mlpcp_prolong(4, 10, D, 4, 1, L, 10, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_prolong(4, 10, D, 5, -1, L, 10, NULL), MLPCP_E_LEVELS);

  /* differentiation form */
  EXPECT(mlpcp_ialm_step(10, 20, 0, D, 20, NULL, NULL, 0.1f, 1.0, L, S, Y, NULL, NULL, 0, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_ialm_step(20, 10, 0, D, 10, NULL, NULL, 0.0f, 1.0, L, S, Y, NULL, NULL, 0, NULL), MLPCP_E_INVALID_ARG);
  EXPECT(mlpcp_ialm_step_vjp(20, 10, 0, D, 10, NULL, NULL, 0.1f, -1.0, NULL, NULL, NULL, L, S, Y, NULL, NULL, 0,
                             NULL),
         MLPCP_E_INVALID_ARG);
  if (mlpcp_step_workspace_bytes(10, 20, 0) != 0) ++failures;

  /* Frank-Wolfe thresholding */
  EXPECT(mlpcp_cpcp_fwt(10, 20, D, 20, NULL, 0.1f, 0.1f, 0, 1e-3, 10, L, S, NULL, 0, NULL, NULL), MLPCP_E_SHAPE);
  EXPECT(mlpcp_cpcp_fwt(20, 10, D, 10, NULL, 0.0f, 0.1f, 0, 1e-3, 10, L, S, NULL, 0, NULL, NULL), MLPCP_E_INVALID_ARG);
  if (mlpcp_fwt_workspace_bytes(10, 20, 0, 0) != 0) ++failures;

  /* kernel timing: off, nothing recorded */
  mlpcp_kernel_time kt[32];
  EXPECT(mlpcp_profile_enable(0), MLPCP_OK);
  if (mlpcp_profile_read(kt, 32) <= 0) ++failures;

  if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
  else printf("abi host checks passed\n");
  return failures ? 1 : 0;
}
