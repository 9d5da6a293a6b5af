/*
 * Host-side checks of the C ABI under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_abi_sanitizers.py builds libkqr with both on its host
 * code and this driver with both, then runs it).  Every call here is one the
 * library answers on the host: argument validation, option defaults, status
 * strings, the tuning-file reader and writer, the test hook, and -- only when
 * no GPU is present -- the no-device status of an otherwise valid call.  No
 * call hands a device pointer to a kernel.
 *
 * Exit status 0 when every status is the expected one; the sanitizers abort
 * with their own report on a memory or UB error.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "kqr.h"

static int failures = 0;

#define EXPECT(call, want)                                                                 \
  do {                                                                                     \
    int got_ = (call);                                                                     \
    if (got_ != (want)) {                                                                  \
      fprintf(stderr, "%s:%d %s -> %d, expected %d (%s)\n", __FILE__, __LINE__, #call, got_, \
              (want), kqr_last_error());                                                   \
      ++failures;                                                                          \
    }                                                                                      \
  } while (0)

int main(int argc, char** argv) {
  const char* tmpdir = argc > 1 ? argv[1] : "/tmp";
  void* P = (void*)(uintptr_t)4096; /* never dereferenced: every call below is rejected first */
  double beta = 0.0;
  kqr_options o;
  EXPECT(kqr_default_options(&o), KQR_OK);
  EXPECT(kqr_default_options(NULL), KQR_EINVAL);
  for (int s = -6; s <= 2; ++s)
    if (strlen(kqr_status_string(s)) == 0) ++failures;

  /* kqr_fit: argument and option validation */
  EXPECT(kqr_fit(P, P, 1, 3, 0.5, 1.0, KQR_RBF, 1.0, NULL, P, &beta, NULL, NULL), KQR_EINVAL);
  EXPECT(kqr_fit(P, P, 10, 3, 1.5, 1.0, KQR_RBF, 1.0, NULL, P, &beta, NULL, NULL), KQR_EINVAL);
  EXPECT(kqr_fit(P, P, 10, 3, 0.5, -1.0, KQR_RBF, 1.0, NULL, P, &beta, NULL, NULL), KQR_EINVAL);
  EXPECT(kqr_fit(P, P, 10, 65, 0.5, 1.0, KQR_RBF, 1.0, NULL, P, &beta, NULL, NULL), KQR_EINVAL);
  EXPECT(kqr_fit(NULL, P, 10, 3, 0.5, 1.0, KQR_RBF, 1.0, NULL, P, &beta, NULL, NULL), KQR_EINVAL);
  o.admm_step = 2.0;
  EXPECT(kqr_fit(P, P, 10, 3, 0.5, 1.0, KQR_RBF, 1.0, &o, P, &beta, NULL, NULL), KQR_EINVAL);
  if (strstr(kqr_last_error(), "admm_step") == NULL) ++failures;
  kqr_default_options(&o);
  o.warm_alpha = (const double*)P;
  EXPECT(kqr_fit(P, P, 10, 3, 0.5, 1.0, KQR_RBF, 1.0, &o, P, &beta, NULL, NULL), KQR_EINVAL);
  kqr_default_options(&o);
  o.trace_cap = 5; /* without a trace buffer */
  EXPECT(kqr_fit(P, P, 10, 3, 0.5, 1.0, KQR_RBF, 1.0, &o, P, &beta, NULL, NULL), KQR_EINVAL);

  /* kernel operators */
  EXPECT(kqr_kernel_build(P, 10, 3, 9, 1.0, KQR_FP32, P, 16, NULL), KQR_EINVAL);
  EXPECT(kqr_kernel_build(P, 10, 3, KQR_RBF, 1.0, KQR_FP32, P, 12, NULL), KQR_EINVAL);
  EXPECT(kqr_kernel_apply(P, 10, 3, KQR_RBF, 1.0, NULL, 0, 0, P, 17, 17, P, 17, 0, NULL), KQR_EINVAL);
  EXPECT(kqr_predict(P, 10, 3, P, 0.0, 0.0, KQR_RBF, 1.0, P, 5, P, NULL), KQR_EINVAL);
  EXPECT(kqr_woodbury_apply(P, 10, 2000, 4, 1.0, P, P, P, NULL), KQR_EINVAL);
  if (kqr_packed_bytes(-1, KQR_FP32) >= 0) ++failures;

  /* batched entry points */
  const float* Xs[2] = {(const float*)P, (const float*)P};
  const double* ys[2] = {(const double*)P, (const double*)P};
  double* as[2] = {(double*)P, (double*)P};
  int64_t ns[2] = {10, 1};
  double taus[2] = {0.5, 0.5}, lams[2] = {1.0, 1.0}, gams[2] = {1.0, 1.0}, betas[2];
  int st[2];
  EXPECT(kqr_fit_batch(2, Xs, ys, ns, 3, taus, lams, KQR_RBF, gams, NULL, as, betas, NULL, st, NULL), KQR_EINVAL);
  EXPECT(kqr_fit_multi_tau(P, P, 10, 3, taus, 0, 1.0, KQR_RBF, 1.0, NULL, P, betas, NULL, st, NULL), KQR_EINVAL);
  EXPECT(kqr_fit_path(P, P, 10, 3, 0.5, lams, 0, KQR_RBF, 1.0, NULL, P, betas, NULL, st, NULL), KQR_EINVAL);

  /* tuning file: null path, missing file, a malformed file */
  int cnt = -1;
  EXPECT(kqr_tune_save(NULL, &cnt), KQR_EINVAL);
  EXPECT(kqr_tune_load("/nonexistent/kqr_tune.json", &cnt), KQR_EINVAL);
  char path[512];
  snprintf(path, sizeof(path), "%s/kqr_tune_bad.json", tmpdir);
  FILE* f = fopen(path, "w");
  if (f) {
    fputs("{\"entries\": [\n{\"kind\": \"apply\"}\n]}\n", f); /* no "arch" */
    fclose(f);
    EXPECT(kqr_tune_load(path, &cnt), KQR_EINVAL);
  }

  /* test hook */
  EXPECT(kqr_test_core_breakdowns(-1, 1), KQR_EINVAL);
  EXPECT(kqr_test_core_breakdowns(0, 0), KQR_OK);
  EXPECT(kqr_test_batch_steps(-1), KQR_EINVAL);
  EXPECT(kqr_test_batch_steps(1), KQR_OK);

  /* a valid call without a GPU */
  if (kqr_device_count() == 0) {
    EXPECT(kqr_fit(P, P, 10, 3, 0.5, 1.0, KQR_RBF, 1.0, NULL, P, &beta, NULL, NULL), KQR_ENODEVICE);
  }
  if (failures) fprintf(stderr, "%d unexpected statuses\n", failures);
  else printf("abi_sanitize: all statuses as expected\n");
  return failures ? 1 : 0;
}
