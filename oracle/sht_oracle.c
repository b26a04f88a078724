/*
 * sht_oracle.c -- plain, slow, FP64 CPU oracle for the Legendre stage of the
 * inverse spherical harmonic transform (alm2map) and of its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the HIP path.
 *
 * What it computes (Hupca, Falcou, Grigori, Stompor, "Spherical harmonic
 * transform with GPUs", INRIA RR-7409):
 *
 *   Delta_m(theta) = sum_{l=m}^{lmax} a_lm P_lm(cos theta)       Eq. (DeltaDef), Sec. 2.1
 *
 * with P_lm the orthonormalised associated Legendre functions built by the
 * two-point recurrence in l (Eq. assLegRec), seeded by Eq. (pmm) and
 * Eq. (pm1m), coefficients beta_lm of Eq. (betaDef), and guarded against
 * under/overflow by real-time rescaling (Sec. 2.2.2, Algorithm 2).
 *
 * Readings of the printed equations (each pinned by a CPU test):
 *  - Eq. (assLegRec) is printed with "+"; the recurrence that yields the
 *    orthonormal functions has "-":
 *       P_{l,m} = beta_{l,m} * ( x P_{l-1,m} - P_{l-2,m} / beta_{l-1,m} ).
 *  - Eq. (pmm) is printed with (1-x^2)^m; the orthonormal seed is
 *       P_mm = mu_m (1-x^2)^{m/2} = mu_m sin^m(theta).
 *  - Eq. (pm1m) is printed with beta_{l+1,m}; the coefficient is
 *       beta_{m+1,m} = sqrt(2m+3).
 *  - No Condon-Shortley phase: mu_m > 0 as printed in Eq. (pmm).
 *  - For m = 0 only the real part of a_l0 enters (the map is real, Sec. 2.1).
 *
 * Rescaling (Algorithm 2): every freshly computed value is compared with a
 * threshold 2^S; when it exceeds it, it and its predecessor are multiplied by
 * 2^-S and an integer exponent k is incremented.  The value is scaled back
 * by 2^(S k) before it is used.  The rescale "table" of the paper is here
 * the set of powers 2^(S k).
 *
 * Structure: plm_column evaluates the column P_lm(x), l = m..lmax, of one
 * m at one colatitude from the seed and the recurrence; Delta_m is then the
 * dot product of that column with the a_lm of the m (Eq. DeltaDef), and the
 * adjoint adds the column times a ring's Delta~_m into the coefficients.
 * Rings (forward) or m (adjoint) are independent and are spread over OpenMP
 * threads, which changes no arithmetic.  Build with -ffp-contract=off so that
 * every expression is evaluated as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_S 256 /* power-of-two rescale step */

/* mu_m of Eq. (pmm): mu_m = sqrt((2m+1)!/(4 pi)) / (2^m m!).
 * Evaluated as the running product mu_0 = 1/sqrt(4 pi),
 * mu_m = mu_{m-1} * sqrt((2m+1)/(2m)), which is the same quantity
 * (the ratio of consecutive terms of the printed formula). */
void oracle_mu(int mmax, double *mu)
{
    mu[0] = 1.0 / sqrt(4.0 * M_PI);
    for (int m = 1; m <= mmax; ++m)
        mu[m] = mu[m - 1] * sqrt((2.0 * m + 1.0) / (2.0 * m));
}

/* beta_lm of Eq. (betaDef). */
static double beta(int l, int m)
{
    double L = (double)l, M = (double)m;
    return sqrt((4.0 * L * L - 1.0) / (L * L - M * M));
}

/* sin^m(theta) * mu as a scaled pair (v, k): value = v * 2^(S k), k <= 0.
 * The power is taken by repeated squaring, renormalising the mantissa with
 * frexp after every product so that nothing underflows. */
static void seed_mm(double mu, double s, int m, double *v, int *k)
{
    if (m == 0) { *v = mu; *k = 0; return; }
    if (s == 0.0) { *v = 0.0; *k = 0; return; }
    double rm = 1.0, base; /* result mantissa */
    long re = 0, be;       /* result / base exponents */
    int e;
    base = frexp(s, &e); be = e;
    int p = m;
    while (p) {
        if (p & 1) {
            rm = rm * base; re += be;
            rm = frexp(rm, &e); re += e;
        }
        p >>= 1;
        if (p) {
            base = base * base; be = 2 * be;
            base = frexp(base, &e); be += e;
        }
    }
    /* value = mu * rm * 2^re;  choose k <= 0 with re - S k in (-S, 0]. */
    long kk = 0;
    if (re < 0) kk = -((-re) / ORACLE_S);
    *v = ldexp(mu * rm, (int)(re - (long)ORACLE_S * kk));
    *k = (int)kk;
}

/* The column P_lm(x), l = m..lmax, of one m at one point (x = cos theta,
 * s = sin theta): P[l - m] for l = m..lmax.  mu_m is the seed constant of
 * Eq. (pmm); b[l - m] = beta_{l,m} of Eq. (betaDef) for l = m+1..lmax.  The
 * values are carried as v 2^(S k) (seed_mm) through the recurrence of
 * Eq. (assLegRec) and the start of Eq. (pm1m); whenever |v_l| passes 2^S the
 * last two values are scaled by 2^-S and k grows by one (Sec. 2.2.2).  Each
 * P_lm is returned as v 2^(S k), which is 0 for values below about 2^-1074. */
static void plm_column(int lmax, int m, double x, double s, double mu_m, const double *b,
                       double *P)
{
    double v0, v1;
    int k;
    seed_mm(mu_m, s, m, &v0, &k);
    double scale = ldexp(1.0, ORACLE_S * k);
    P[0] = v0 * scale;
    if (m + 1 > lmax) return;
    v1 = b[1] * x * v0;
    P[1] = v1 * scale;
    for (int l = m + 2; l <= lmax; ++l) {
        const int j = l - m;
        double v2 = b[j] * (x * v1 - v0 / b[j - 1]);
        if (fabs(v2) > 0x1p256) {
            v2 = ldexp(v2, -ORACLE_S);
            v1 = ldexp(v1, -ORACLE_S);
            k += 1;
            scale = ldexp(1.0, ORACLE_S * k);
        }
        P[j] = v2 * scale;
        v0 = v1;
        v1 = v2;
    }
}

/* P_lm(x) for l = 0..lmax at one point (x = cos theta, s = sin theta);
 * entries with l < m are set to 0.  Returns 0 on success. */
int oracle_lambda(int lmax, int m, double x, double s, double *out)
{
    if (lmax < 0 || m < 0 || m > lmax) return -1;
    double *mu = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *b = (double *)malloc(sizeof(double) * (size_t)(lmax - m + 1));
    if (!mu || !b) { free(mu); free(b); return -2; }
    oracle_mu(m, mu);
    b[0] = 0.0;
    for (int l = m + 1; l <= lmax; ++l) b[l - m] = beta(l, m);
    for (int l = 0; l < m; ++l) out[l] = 0.0;
    plm_column(lmax, m, x, s, mu[m], b, out + m);
    free(mu);
    free(b);
    return 0;
}

/* Offsets of the m-major packed coefficient array: for the i-th m of the
 * set, l = m..lmax are stored contiguously from off[i]. */
static int64_t *alm_offsets(int lmax, int nm, const int32_t *mval)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nm + 1));
    if (!off) return NULL;
    off[0] = 0;
    for (int i = 0; i < nm; ++i) off[i + 1] = off[i] + (lmax - mval[i] + 1);
    return off;
}

/* beta_{l,m} of every m of the set, computed once (the same numbers serve
 * every ring), in the packed m-major layout of the coefficients. */
static double *beta_tables(int lmax, int nm, const int32_t *mval, const int64_t *off)
{
    double *b = (double *)malloc(sizeof(double) * (size_t)off[nm]);
    if (!b) return NULL;
    for (int i = 0; i < nm; ++i) {
        int m = mval[i];
        b[off[i]] = 0.0; /* beta_{m,m} is never used (0/0) */
        for (int l = m + 1; l <= lmax; ++l) b[off[i] + (l - m)] = beta(l, m);
    }
    return b;
}

static int check_mset(int lmax, int nm, const int32_t *mval)
{
    if (lmax < 0 || nm < 1 || nm > lmax + 1) return -1;
    for (int i = 0; i < nm; ++i) {
        if (mval[i] < 0 || mval[i] > lmax) return -1;
        if (i && mval[i] <= mval[i - 1]) return -1;
    }
    return 0;
}

/* Delta_m(r) for every ring r and every m of the set (Eq. DeltaDef): the
 * dot product of the column P_lm(cos theta_r), l = m..lmax, with the a_lm
 * of the m (only the real part of a_l0 enters).
 *   alm   : complex [nalm] interleaved (re, im), m-major packed
 *   delta : complex [nrings][nm] interleaved, written
 * nthreads <= 0 uses the OpenMP default. */
int oracle_delta(int lmax, int nm, const int32_t *mval, int nrings,
                 const double *cth, const double *sth, const double *alm,
                 double *delta, int nthreads)
{
    if (check_mset(lmax, nm, mval) || nrings < 1) return -1;
    int64_t *off = alm_offsets(lmax, nm, mval);
    double *mu = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    double *bt = off ? beta_tables(lmax, nm, mval, off) : NULL;
    if (!off || !mu || !bt) { free(off); free(mu); free(bt); return -2; }
    oracle_mu(lmax, mu);
    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int r = 0; r < nrings; ++r) {
        double *P = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        if (!P) { fail = 1; continue; }
        for (int i = 0; i < nm; ++i) {
            const int m = mval[i];
            const int len = lmax - m + 1;
            const double *a = alm + 2 * off[i];
            plm_column(lmax, m, cth[r], sth[r], mu[m], bt + off[i], P);
            double dre = 0.0, dim = 0.0;
            for (int j = 0; j < len; ++j) {
                dre += a[2 * j] * P[j];
                if (m > 0) dim += a[2 * j + 1] * P[j];
            }
            delta[2 * ((int64_t)r * nm + i)] = dre;
            delta[2 * ((int64_t)r * nm + i) + 1] = dim;
        }
        free(P);
    }
    free(off); free(mu); free(bt);
    return fail ? -2 : 0;
}

/* Transposed Legendre stage of the adjoint transform:
 *   out_lm = sum_r P_lm(cos theta_r) * dt_m(r)
 * dt    : complex [nrings][nm] interleaved
 * out   : complex [nalm] interleaved, written; imaginary part of m = 0
 *         entries is set to 0 (those coefficients are real).
 * Parallel over m (each thread owns whole m rows, so no two threads write
 * the same output). */
int oracle_delta_adjoint(int lmax, int nm, const int32_t *mval, int nrings,
                         const double *cth, const double *sth, const double *dt,
                         double *out, int nthreads)
{
    if (check_mset(lmax, nm, mval) || nrings < 1) return -1;
    int64_t *off = alm_offsets(lmax, nm, mval);
    double *mu = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    double *bt = off ? beta_tables(lmax, nm, mval, off) : NULL;
    if (!off || !mu || !bt) { free(off); free(mu); free(bt); return -2; }
    oracle_mu(lmax, mu);
    memset(out, 0, sizeof(double) * 2 * (size_t)off[nm]);
    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int i = 0; i < nm; ++i) {
        const int m = mval[i];
        const int len = lmax - m + 1;
        double *o = out + 2 * off[i];
        double *P = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        if (!P) { fail = 1; continue; }
        for (int r = 0; r < nrings; ++r) {
            const double gre = dt[2 * ((int64_t)r * nm + i)];
            const double gim = dt[2 * ((int64_t)r * nm + i) + 1];
            plm_column(lmax, m, cth[r], sth[r], mu[m], bt + off[i], P);
            for (int j = 0; j < len; ++j) {
                o[2 * j] += P[j] * gre;
                o[2 * j + 1] += P[j] * gim;
            }
        }
        if (m == 0)
            for (int l = 0; l <= lmax; ++l) o[2 * l + 1] = 0.0;
        free(P);
    }
    free(off); free(mu); free(bt);
    return fail ? -2 : 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
