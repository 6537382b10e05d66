/*
 * Oracle (test infrastructure only): the adjoint of eq. (1) written as plain
 * float64 loops in C, for checking the GPU gradients element by element at
 * full problem sizes, where the numpy definition in adjoint.py is too slow.
 *
 * eq. (1) with zero history, y_r[n] = sum_{k<M} h_r[k] s[n-k] (s[m<0] = 0),
 * is linear in s and in h_r.  For a real loss with upstream gradient g_r[n]
 * (complex convention dL/d(conj z)) the gradients are the adjoint maps:
 *
 *   ds[m]   = sum_r sum_{k<M, m+k<N_s} conj(h_r[k]) g_r[m+k]
 *   dh_r[k] = sum_{n=k}^{N_s-1} conj(s[n-k]) g_r[n]
 *
 * Both are computed here by those sums and nothing else: no transform, no
 * blocking of the arithmetic.  The loops are ordered so that every output is
 * accumulated by one thread in a fixed order (r, then k, for ds; n for dh), so
 * the result does not depend on the thread count.
 *
 * Data: complex values as interleaved {double re, double im}; g is [K][N_s],
 * h and dh are [K][M], s and ds are [N_s].  Nothing here is shared with the
 * GPU library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ds[m] for m in [0, N_s).  Outputs are split into blocks of consecutive m;
 * each block is owned by one thread, which adds the terms in (r, k) order. */
void oracle_grad_signal(const double* g, int64_t K, int64_t Ns, const double* h, int64_t M, double* ds) {
  const int64_t B = 4096;
  const int64_t nblk = (Ns + B - 1) / B;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t m0 = b * B;
    const int64_t m1 = m0 + B < Ns ? m0 + B : Ns;
    double* acc = ds + 2 * m0;
    memset(acc, 0, (size_t)(m1 - m0) * 2 * sizeof(double));
    for (int64_t r = 0; r < K; ++r) {
      const double* gr = g + 2 * r * Ns;
      for (int64_t k = 0; k < M; ++k) {
        const double hr = h[2 * (r * M + k)], hi = -h[2 * (r * M + k) + 1]; /* conj(h_r[k]) */
        /* m + k < N_s */
        const int64_t mend = (Ns - k) < m1 ? (Ns - k) : m1;
        for (int64_t m = m0; m < mend; ++m) {
          const double gre = gr[2 * (m + k)], gim = gr[2 * (m + k) + 1];
          acc[2 * (m - m0)] += hr * gre - hi * gim;
          acc[2 * (m - m0) + 1] += hr * gim + hi * gre;
        }
      }
    }
  }
}

/* dh_r[k] for r in [0, K), k in [0, M).  The sum over n runs in blocks of
 * consecutive n, one block after the other; inside a block every (r, k) is
 * owned by one thread, which adds its terms in n order. */
void oracle_grad_filters(const double* g, int64_t K, int64_t Ns, const double* s, int64_t M, double* dh) {
  memset(dh, 0, (size_t)(K * M) * 2 * sizeof(double));
  const int64_t B = 16384;
  for (int64_t n0 = 0; n0 < Ns; n0 += B) {
    const int64_t n1 = n0 + B < Ns ? n0 + B : Ns;
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t r = 0; r < K; ++r) {
      for (int64_t k = 0; k < M; ++k) {
        const double* gr = g + 2 * r * Ns;
        double are = dh[2 * (r * M + k)], aim = dh[2 * (r * M + k) + 1];
        const int64_t nb = n0 > k ? n0 : k; /* n - k >= 0 */
        for (int64_t n = nb; n < n1; ++n) {
          const double sre = s[2 * (n - k)], sim = -s[2 * (n - k) + 1]; /* conj(s[n-k]) */
          const double gre = gr[2 * n], gim = gr[2 * n + 1];
          are += sre * gre - sim * gim;
          aim += sre * gim + sim * gre;
        }
        dh[2 * (r * M + k)] = are;
        dh[2 * (r * M + k) + 1] = aim;
      }
    }
  }
}

/* eq. (1) itself, y_r[n] = sum_{k<M, k<=n} h_r[k] s[n-k], for n in [0, N_s):
 * the forward map these two are the adjoints of (used by the tests that pin
 * them through <A s, g> = <s, A^H g>). */
void oracle_direct_conv(const double* s, int64_t Ns, const double* h, int64_t K, int64_t M, double* y) {
  const int64_t B = 4096;
  const int64_t nblk = (Ns + B - 1) / B;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
  for (int64_t r = 0; r < K; ++r) {
    for (int64_t b = 0; b < nblk; ++b) {
      const int64_t n0 = b * B;
      const int64_t n1 = n0 + B < Ns ? n0 + B : Ns;
      double* acc = y + 2 * (r * Ns + n0);
      memset(acc, 0, (size_t)(n1 - n0) * 2 * sizeof(double));
      for (int64_t k = 0; k < M; ++k) {
        const double hre = h[2 * (r * M + k)], him = h[2 * (r * M + k) + 1];
        const int64_t nb = n0 > k ? n0 : k; /* n - k >= 0 */
        for (int64_t n = nb; n < n1; ++n) {
          const double sre = s[2 * (n - k)], sim = s[2 * (n - k) + 1];
          acc[2 * (n - n0)] += hre * sre - him * sim;
          acc[2 * (n - n0) + 1] += hre * sim + him * sre;
        }
      }
    }
  }
}
