/*
 * Per-output-bin sums for checking sampled outputs of large transforms.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle).  Shares no code, table or
 * constant with the GPU library.
 *
 * oracle_dft_bins:  y_k = sum_j x_j w_N^{(j k) mod N},  w_N = exp(-2 pi i / N)
 *                   (the DFT definition of Sec. 2), no normalisation.
 * oracle_aqft_bins: y = sum_x x_j exp(-2 pi i P(j, y) / N) with
 *                   P(j, y) = sum_a j_a C_a(y) mod N and
 *                   C_a(y) = sum_{b : n-1-k <= a+b <= n-1} y_b 2^{a+b},
 *                   the closed form of the range-k AQFT (natural output
 *                   order) that follows from the circuit of Fig. 1.
 *
 * The phase index is exact integer arithmetic modulo N.  w_N^m is a two-level
 * product of long-double cos/sin values rounded to double; the sums are
 * accumulated in long double.  One OpenMP thread per bin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { double re, im; } cplx;

static void omega_tables(int n, int h, cplx **lo, cplx **hi)
{
    /* lo[m] = w_N^m for m < 2^h, hi[m] = w_N^{m 2^h} for m < 2^{n-h} */
    const long double twopi = 6.283185307179586476925286766559L;
    const long double N = ldexpl(1.0L, n);
    long nlo = 1L << h, nhi = 1L << (n - h);
    *lo = (cplx *)malloc(sizeof(cplx) * (size_t)nlo);
    *hi = (cplx *)malloc(sizeof(cplx) * (size_t)nhi);
    for (long m = 0; m < nlo; ++m) {
        long double a = twopi * (long double)m / N;
        (*lo)[m].re = (double)cosl(a);
        (*lo)[m].im = (double)-sinl(a);
    }
    for (long m = 0; m < nhi; ++m) {
        long double a = twopi * (long double)(m << h) / N;
        (*hi)[m].re = (double)cosl(a);
        (*hi)[m].im = (double)-sinl(a);
    }
}

static void sum_with_phase(const cplx *x, long N, int h, const cplx *lo,
                           const cplx *hi, const uint64_t *plo,
                           const uint64_t *phi, cplx *out)
{
    /* phase(j) = plo[j mod 2^h] + phi[j >> h]  (mod N): P is linear in the
       bits of j, so the low and high halves of j contribute independently */
    const uint64_t mask = (uint64_t)N - 1;
    const uint64_t hmask = (1ULL << h) - 1;
    long double sr = 0.0L, si = 0.0L;
    for (long j = 0; j < N; ++j) {
        uint64_t m = (plo[(uint64_t)j & hmask] + phi[(uint64_t)j >> h]) & mask;
        const cplx a = lo[m & hmask];
        const cplx b = hi[m >> h];
        long double wr = (long double)a.re * b.re - (long double)a.im * b.im;
        long double wi = (long double)a.re * b.im + (long double)a.im * b.re;
        sr += (long double)x[j].re * wr - (long double)x[j].im * wi;
        si += (long double)x[j].re * wi + (long double)x[j].im * wr;
    }
    out->re = (double)sr;
    out->im = (double)si;
}

static void bin_sums(const cplx *x, int n, int k, const int64_t *bins,
                     long nbins, cplx *out, int exact)
{
    const long N = 1L << n;
    const int h = (n + 1) / 2;
    cplx *lo, *hi;
    omega_tables(n, h, &lo, &hi);
#pragma omp parallel for schedule(dynamic, 1)
    for (long q = 0; q < nbins; ++q) {
        const uint64_t y = (uint64_t)bins[q];
        const uint64_t mask = (uint64_t)N - 1;
        uint64_t C[64];
        for (int a = 0; a < n; ++a) {
            uint64_t c = 0;
            if (exact) {
                c = (y << a) & mask; /* j*y = sum_a j_a 2^a y */
            } else {
                for (int b = 0; b < n; ++b)
                    if (a + b >= n - 1 - k && a + b <= n - 1 && ((y >> b) & 1))
                        c += 1ULL << (a + b);
                c &= mask;
            }
            C[a] = c;
        }
        long nlo = 1L << h, nhi = 1L << (n - h);
        uint64_t *plo = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nlo);
        uint64_t *phi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nhi);
        for (long j = 0; j < nlo; ++j) {
            uint64_t p = 0;
            for (int a = 0; a < h; ++a)
                if ((j >> a) & 1) p += C[a];
            plo[j] = p & mask;
        }
        for (long j = 0; j < nhi; ++j) {
            uint64_t p = 0;
            for (int a = 0; a < n - h; ++a)
                if ((j >> a) & 1) p += C[h + a];
            phi[j] = p & mask;
        }
        sum_with_phase(x, N, h, lo, hi, plo, phi, &out[q]);
        free(plo);
        free(phi);
    }
    free(lo);
    free(hi);
}

void oracle_dft_bins(const cplx *x, int n, const int64_t *bins, long nbins, cplx *out)
{
    bin_sums(x, n, n - 1, bins, nbins, out, 1);
}

void oracle_aqft_bins(const cplx *x, int n, int k, const int64_t *bins, long nbins,
                      cplx *out)
{
    bin_sums(x, n, k, bins, nbins, out, 0);
}
