/*
 * CPU oracle: the plain modular matrix product.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  It shares no code with the GPU library.
 *
 * Definition (Dumas, Fousse, Salvy, "Compressed Modular Matrix Multiplication",
 * section 2, the dot product whose value the compressed product recovers):
 *     C[i][j] = ( sum_{l<k} A[i][l] * B[l][j] ) mod p
 * computed with 64-bit unsigned accumulators and ONE reduction per entry.
 * Entries are bytes (0..255), so k*255*255 < 2^64 for every k < 2^47: the
 * accumulation never overflows for any size this oracle can be asked about.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Full product, i-l-j loop order, rows split over OpenMP threads. */
int qmm_oracle_modmul(int64_t m, int64_t n, int64_t k, uint32_t p,
                      const uint8_t *A, int64_t lda,
                      const uint8_t *B, int64_t ldb,
                      uint8_t *C, int64_t ldc)
{
    if (p < 2 || m < 0 || n < 0 || k < 0) return 1;
    int err = 0;
#pragma omp parallel
    {
        uint64_t *acc = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
        if (!acc) {
#pragma omp atomic write
            err = 2;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            if (!acc) continue;
            memset(acc, 0, (size_t)n * sizeof(uint64_t));
            for (int64_t l = 0; l < k; ++l) {
                const uint64_t a = A[i * lda + l];
                const uint8_t *brow = B + l * ldb;
                for (int64_t j = 0; j < n; ++j) acc[j] += a * (uint64_t)brow[j];
            }
            for (int64_t j = 0; j < n; ++j) C[i * ldc + j] = (uint8_t)(acc[j] % p);
        }
        free(acc);
    }
    return err;
}

/* Selected entries only: out[e] = C[rows[e]][cols[e]], each one a plain dot product. */
int qmm_oracle_modmul_entries(int64_t count, const int64_t *rows, const int64_t *cols,
                              int64_t k, uint32_t p,
                              const uint8_t *A, int64_t lda,
                              const uint8_t *B, int64_t ldb,
                              uint8_t *out)
{
    if (p < 2 || k < 0 || count < 0) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) {
        uint64_t acc = 0;
        for (int64_t l = 0; l < k; ++l)
            acc += (uint64_t)A[rows[e] * lda + l] * (uint64_t)B[l * ldb + cols[e]];
        out[e] = (uint8_t)(acc % p);
    }
    return 0;
}

/* Threads the OpenMP runtime will use for the full product. */
int qmm_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following products (n >= 1; the benchmark times the oracle on all
 * host cores and on one). */
void qmm_oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
