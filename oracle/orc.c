/*
 * Oracle inner loops -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU loops used by the Python oracle in
 * oracle/core.py.  Nothing in the product library links or calls this file;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Built with gcc -O2 -fopenmp -ffp-contract=off (no reassociation, no FMA
 * contraction): every sum below is accumulated in the order written.
 */
#include <stdint.h>

/* Linear convolution, eq. (1) of Section II:
 *   r[m] = sum_{n=0}^{N-1} s[m-n] * k[n],   0 <= m < L+N-1,
 * with s[i] = 0 outside [0, L).  FP64, each output summed sequentially over n. */
void orc_conv_f64(const double* s, int64_t L, const double* k, int64_t N, double* r)
{
    int64_t M = L + N - 1;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        double acc = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            int64_t i = m - n;
            if (i < 0 || i >= L) continue;
            acc += s[i] * k[n];
        }
        r[m] = acc;
    }
}

/* The same definition in exact 64-bit integer arithmetic, evaluated only for
 * outputs m in [m0, m1); r has m1-m0 entries.  Used for the integer fields
 * r~ = s~ * k~ of Section III.B. */
void orc_conv_i64_range(const int64_t* s, int64_t L, const int64_t* k, int64_t N,
                        int64_t m0, int64_t m1, int64_t* r)
{
#pragma omp parallel for schedule(static)
    for (int64_t m = m0; m < m1; ++m) {
        int64_t acc = 0;
        for (int64_t n = 0; n < N; ++n) {
            int64_t i = m - n;
            if (i < 0 || i >= L) continue;
            acc += s[i] * k[n];
        }
        r[m - m0] = acc;
    }
}

/* Many independent integer convolutions at once (one per overlap-save block):
 * block b has window s + b*Wb (Wb samples), kept outputs [m0[b], m1[b]) written
 * contiguously to r + off[b].  Same arithmetic as orc_conv_i64_range. */
void orc_conv_i64_blocks(const int64_t* s, int64_t nblocks, int64_t Wb,
                         const int64_t* k, int64_t N,
                         const int64_t* m0, const int64_t* m1, const int64_t* off,
                         int64_t* r)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblocks; ++b) {
        const int64_t* sb = s + b * Wb;
        for (int64_t m = m0[b]; m < m1[b]; ++m) {
            int64_t acc = 0;
            for (int64_t n = 0; n < N; ++n) {
                int64_t i = m - n;
                if (i < 0 || i >= Wb) continue;
                acc += sb[i] * k[n];
            }
            r[off[b] + (m - m0[b])] = acc;
        }
    }
}

int orc_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
