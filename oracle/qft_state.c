/*
 * Whole-vector FP64 reference of the (approximate) QFT for large n.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle).  Shares no code, table or
 * constant with the GPU library.
 *
 * It is the circuit of Fig. 1 with the controlled phases of each target
 * collapsed into one diagonal (Sec. 2, gate fusion: commuting diagonal gates
 * multiply into one diagonal), the same per-target form as
 * qft_fused_targets in qft_oracle.py, written in plain C so that the whole
 * output of a 2^28- or 2^30-element transform can be computed in seconds:
 *
 *   for t = n-1 down to 0:
 *     for every index i with bit t clear (partner j = i + 2^t):
 *       (a, b) = (psi[i], psi[j])
 *       psi[i] = (a + b) / sqrt(2)                       H on qubit t
 *       psi[j] = (a - b) / sqrt(2) * exp(-/+ 2 pi i u / 2^{t+1})
 *   where u is (i mod 2^t) with its bits below t - k cleared: the controlled
 *   R_{d+1} with control c = t - d and d <= k multiplies amplitudes whose
 *   bits c and t are set by exp(-2 pi i 2^c / 2^{t+1}), and these factors
 *   multiply to the one above (Sec. 2 "Approximate QFT" keeps d <= k).
 *   The sign is + for the inverse (conjugate-phase) circuit.
 *
 * Then the output scale (Sec. 3 step 4) and, for the natural order, the final
 * swaps as the index permutation out[m] = psi[rev_n(m)] (Sec. 3 step 2).
 *
 * Every angle is 2 pi u / 2^{t+1} with u an exact integer; cos and sin are
 * the C library's double routines.  The loops over pairs are independent, so
 * they are split over OpenMP threads; the arithmetic of each element is the
 * same whatever the thread count.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static uint64_t reverse_bits(uint64_t x, int n)
{
    uint64_t r = 0;
    for (int b = 0; b < n; ++b) r |= ((x >> b) & 1ULL) << (n - 1 - b);
    return r;
}

/* psi: 2^n elements, transformed in place into the bit-reversed order
 * (psi[rev_n(m)] = bin m).  out: NULL, or 2^n elements that receive the
 * natural order (out[m] = bin m).  k: largest control-target distance kept
 * (k >= n-1 is the exact transform).  scale: the output norm factor. */
void oracle_qft_state(cplx *psi, cplx *out, int n, int k, int inverse, double scale)
{
    const int64_t half_n = (int64_t)1 << (n > 0 ? n - 1 : 0);
    const double s = 1.0 / sqrt(2.0);
    const double twopi = 6.283185307179586476925286766559;
    const double sign = inverse ? 1.0 : -1.0;
    for (int t = n - 1; t >= 0; --t) {
        const int64_t span = (int64_t)1 << t;
        const int low = t - k > 0 ? t - k : 0;
        const double denom = ldexp(1.0, t + 1);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < half_n; ++p) {
            const int64_t blk = p >> t;
            const int64_t u = p & (span - 1);
            const int64_t i = (blk << (t + 1)) | u;
            const int64_t j = i + span;
            const cplx a = psi[i], b = psi[j];
            psi[i].re = (a.re + b.re) * s;
            psi[i].im = (a.im + b.im) * s;
            const double dr = (a.re - b.re) * s, di = (a.im - b.im) * s;
            const int64_t uu = (u >> low) << low;
            const double ang = sign * twopi * (double)uu / denom;
            const double c = cos(ang), sn = sin(ang);
            psi[j].re = dr * c - di * sn;
            psi[j].im = dr * sn + di * c;
        }
    }
    const int64_t N = (int64_t)1 << n;
    if (scale != 1.0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            psi[i].re *= scale;
            psi[i].im *= scale;
        }
    }
    if (out) {
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < N; ++m) out[m] = psi[reverse_bits((uint64_t)m, n)];
    }
}

/* Threads the loops above run on (OpenMP's current maximum), for reporting. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
