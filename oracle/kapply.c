/*
 * FP64 kernel products for the full-size certificates of the oracle.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
 * and the benchmark's CPU-baseline and certificate legs load this library.
 *
 * U = K(Xr, X) V with the kernels of Section 1,
 *     RBF        k(x, x') = exp(-gamma sum_k (x_k - x'_k)^2)
 *     Laplacian  k(x, x') = exp(-gamma sum_k |x_k - x'_k|),
 * every entry formed from direct coordinate differences in FP64 (never the
 * norm expansion), exponentials from the C library, and each output a plain
 * left-to-right FP64 sum over the columns.  Rows are shared out over OpenMP
 * threads; nothing else is reordered.
 *
 *  X   n x p row-major (FP64), Xr m x p row-major, V n x nv row-major,
 *  U   m x nv row-major (written).  kind 0 = RBF, 1 = Laplacian; nv <= 16.
 *  Returns 0, or -1 for invalid arguments.
 */
#include <math.h>
#include <stdint.h>

int kqr_oracle_kernel_apply(const double* X, int64_t n, int64_t p, const double* Xr, int64_t m, int kind,
                            double gamma, const double* V, int64_t nv, double* U) {
  if (n < 0 || m < 0 || p < 1 || nv < 1 || nv > 16 || (kind != 0 && kind != 1)) return -1;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < m; ++i) {
    double acc[16];
    for (int64_t c = 0; c < nv; ++c) acc[c] = 0.0;
    const double* xi = Xr + i * p;
    for (int64_t j = 0; j < n; ++j) {
      const double* xj = X + j * p;
      double d = 0.0;
      for (int64_t k = 0; k < p; ++k) {
        const double t = xi[k] - xj[k];
        d += kind == 0 ? t * t : fabs(t);
      }
      const double e = exp(-gamma * d);
      for (int64_t c = 0; c < nv; ++c) acc[c] += e * V[j * nv + c];
    }
    for (int64_t c = 0; c < nv; ++c) U[i * nv + c] = acc[c];
  }
  return 0;
}
