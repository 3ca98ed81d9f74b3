/* Host-side exercise of the C ABI for the sanitizer test: every call here
 * runs host code only (argument validation, workspace layouts, status
 * strings, the no-device path), so the program runs without a GPU.  Exit
 * status 0 when every call returned what the header promises. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fastcpd.h"

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

static cpd_params params(int M, int N, int method, int precision, int eig_mode, int K) {
  cpd_params p;
  memset(&p, 0, sizeof p);
  p.abi_version = CPD_ABI_VERSION;
  p.M = M;
  p.N = N;
  p.D = 3;
  p.beta = 2.0;
  p.lambda = 3.0;
  p.w = 0.1;
  p.method = method;
  p.precision = precision;
  p.eig_mode = eig_mode;
  p.K = K;
  p.oversample = 20;
  p.power_iters = 2;
  p.tol = 1e-8;
  p.max_iter = 100;
  return p;
}

int main(void) {
  EXPECT(cpd_abi_version() == CPD_ABI_VERSION);
  EXPECT(cpd_build_info() != NULL && strlen(cpd_build_info()) > 0);
  for (int s = -6; s <= 1; ++s) EXPECT(cpd_status_str((cpd_status)s) != NULL);
  EXPECT(cpd_status_str((cpd_status)99) != NULL);

  /* workspace sizes over methods, precisions, modes and sizes */
  const int sizes[][2] = {{1, 1}, {2, 3}, {500, 500}, {1023, 1025}, {4000, 3000}, {50000, 50000}};
  for (size_t i = 0; i < sizeof sizes / sizeof sizes[0]; ++i)
    for (int method = 0; method <= 2; ++method)
      for (int prec = 0; prec <= 2; ++prec)
        for (int mode = 0; mode <= 2; ++mode) {
          const int M = sizes[i][0], N = sizes[i][1];
          const int K = M < 300 ? M : 300;
          cpd_params p = params(M, N, method, prec, mode, K);
          size_t b = 0;
          const cpd_status s = cpd_workspace_size(&p, &b);
          EXPECT(s == CPD_OK || s == CPD_E_ARG || s == CPD_E_UNSUPPORTED);
          if (s == CPD_OK) EXPECT(b > 0);
        }

  /* invalid parameters are rejected before any device work */
  {
    cpd_params p = params(100, 100, CPD_METHOD_FAST, CPD_PREC_FP32, CPD_EIG_FULL, 0);
    size_t b = 0;
    cpd_params q = p;
    q.w = 1.0;
    EXPECT(cpd_workspace_size(&q, &b) == CPD_E_ARG);
    q = p;
    q.beta = 0.0;
    EXPECT(cpd_workspace_size(&q, &b) == CPD_E_ARG);
    q = p;
    q.D = 4;
    EXPECT(cpd_workspace_size(&q, &b) == CPD_E_ARG);
    q = p;
    q.M = 0;
    EXPECT(cpd_workspace_size(&q, &b) == CPD_E_ARG);
    q = p;
    q.abi_version = 0;
    EXPECT(cpd_workspace_size(&q, &b) == CPD_E_ARG);
    EXPECT(cpd_workspace_size(NULL, &b) == CPD_E_ARG);
    EXPECT(cpd_workspace_size(&p, NULL) == CPD_E_ARG);
  }

  /* batches of uneven sizes: header and per-instance layouts */
  {
    const int B = 300;
    cpd_params* ps = (cpd_params*)calloc(B, sizeof(cpd_params));
    unsigned r = 12345u;
    for (int i = 0; i < B; ++i) {
      r = r * 1103515245u + 12345u;
      const int M = 500 + (int)((r >> 8) % 7501);
      r = r * 1103515245u + 12345u;
      const int N = 500 + (int)((r >> 8) % 7501);
      ps[i] = params(M, N, CPD_METHOD_FAST, CPD_PREC_FP32, CPD_EIG_FULL, 0);
    }
    size_t b = 0;
    EXPECT(cpd_batch_workspace_size(B, ps, &b) == CPD_OK && b > 0);
    EXPECT(cpd_batch_workspace_size(0, ps, &b) == CPD_E_ARG);
    ps[7].precision = CPD_PREC_BF16X;
    EXPECT(cpd_batch_workspace_size(B, ps, &b) != CPD_OK);
    free(ps);
  }

  /* network sizes */
  {
    size_t n = 0, b = 0;
    EXPECT(cpdnet_param_count(&n) == CPD_OK && n > 0);
    EXPECT(cpdnet_workspace_size(32, 2000, 2000, CPDNET_BF16, &b) == CPD_OK && b > 0);
    EXPECT(cpdnet_workspace_size(2, 1, 1, CPDNET_FP32, &b) == CPD_OK && b > 0);
    EXPECT(cpdnet_workspace_size(1, 100, 100, 7, &b) == CPD_E_ARG);
    EXPECT(cpdnet_workspace_size(0, 100, 100, CPDNET_BF16, &b) == CPD_E_ARG);
  }

  /* NULL handles and arguments */
  {
    cpd_handle h = NULL;
    cpd_params p = params(100, 120, CPD_METHOD_FAST, CPD_PREC_FP32, CPD_EIG_FULL, 0);
    EXPECT(cpd_init(&h, &p, NULL, NULL, NULL, 0, NULL) == CPD_E_ARG && h == NULL);
    EXPECT(cpd_init(NULL, &p, NULL, NULL, NULL, 0, NULL) == CPD_E_ARG);
    EXPECT(cpd_step(NULL, NULL) == CPD_E_ARG);
    EXPECT(cpd_eig_prepare(NULL, NULL, NULL, NULL) == CPD_E_ARG);
    EXPECT(cpd_register(NULL, NULL, NULL, NULL, NULL) == CPD_E_ARG);
    EXPECT(cpd_destroy(NULL) == CPD_OK);
    EXPECT(cpd_batch_prepare(NULL, 1) == CPD_E_ARG);
    EXPECT(cpd_batch_destroy(NULL) == CPD_OK);
    EXPECT(cpd_last_error(NULL) != NULL);
  }

  /* a valid call without a device (host memory stands in for the arrays,
   * which the library must not touch before checking for a device) */
  {
    cpd_params p = params(64, 64, CPD_METHOD_FAST, CPD_PREC_FP32, CPD_EIG_FULL, 0);
    size_t b = 0;
    EXPECT(cpd_workspace_size(&p, &b) == CPD_OK);
    void* ws = aligned_alloc(256, (b + 255) / 256 * 256);
    float* X = (float*)calloc(64 * 3, sizeof(float));
    cpd_handle h = NULL;
    const cpd_status s = cpd_init(&h, &p, X, X, ws, b, NULL);
    EXPECT(s == CPD_E_DEVICE && h == NULL);
    free(X);
    free(ws);
  }

  if (fails) fprintf(stderr, "%d checks failed\n", fails);
  else printf("host ABI check: all checks passed\n");
  return fails ? 1 : 0;
}
