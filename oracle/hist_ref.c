/*
 * Plain C version of the exact int64 spectral histogram (test infrastructure
 * only; see gw_oracle.histogram for the definition it follows).
 *
 * Spectral function of the free response, Section 5.A eq. chi_by_spectra,
 * with the pair weights of the closed form in Section 7.A and the factor 2 of
 * the spin sum (Section 2, eq. more_screening).  Each pole is split linearly
 * between bins m_p and m_p + 1 in fixed point with 2^-s resolution:
 *     t    = nearbyint(ldexp(P[mu,p] * P[nu,p], s))
 *     t_hi = nearbyint((P[mu,p] * ldexp(frac_p, s)) * P[nu,p])
 *     H[m_p]   += 2 (t - t_hi),  H[m_p + 1] += 2 t_hi.
 * Compiled with -ffp-contract=off so every product is rounded on its own.
 * ldexp(x, s) is written as x times the exact power 2^s (the same correctly
 * rounded value), and nearbyint as llrint (both round to nearest, ties to
 * even, in the default rounding mode; every value here is below 2^62).
 * One entry (mu, nu) per loop iteration, pairs in ascending order; the sums
 * are exact integers, so the order does not matter anyway.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

int hist_ref_entries(const double *P, int64_t n_prod, int64_t n_pairs,
                     const int64_t *m, const double *frac, int s,
                     const int64_t *mu, const int64_t *nu, int64_t n_entries,
                     int64_t nhb, int64_t *H, int64_t *n_dropped)
{
    int64_t dropped = 0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(n_pairs > 0 ? n_pairs : 1));
    if (!w) return -1;
    /* 2^s is exact, and multiplying by it rounds exactly as ldexp does */
    const double two_s = ldexp(1.0, s);
    for (int64_t p = 0; p < n_pairs; ++p) {
        w[p] = ldexp(frac[p], s);
        if (m[p] + 1 >= nhb) dropped++;
    }
    for (int64_t e = 0; e < n_entries; ++e) {
        if (mu[e] < 0 || nu[e] >= n_prod || mu[e] > nu[e]) { free(w); return -2; }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < n_entries; ++e) {
        const double *pm = P + mu[e] * n_pairs;
        const double *pn = P + nu[e] * n_pairs;
        for (int64_t p = 0; p < n_pairs; ++p) {
            int64_t mp = m[p];
            if (mp + 1 >= nhb) continue;
            double prod = pm[p] * pn[p];
            int64_t t = llrint(prod * two_s);      /* RNE(2^s * fl(P_mu P_nu)) */
            double y = pm[p] * w[p];
            double yy = y * pn[p];
            int64_t th = llrint(yy);               /* RNE(fl(fl(P_mu 2^s frac) P_nu)) */
            H[mp * n_entries + e] += 2 * (t - th);
            H[(mp + 1) * n_entries + e] += 2 * th;
        }
    }
    *n_dropped = dropped;
    free(w);
    return 0;
}
