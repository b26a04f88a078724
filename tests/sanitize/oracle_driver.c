/* Exercises the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_host_sanitizers.py): mu_m, single P_lm columns,
 * Delta and its transpose on small grids, with the edge cases the oracle
 * handles (l_max 0, m = l_max, the pole rings with sin theta = 0, partial
 * m-sets, one ring), and its argument checks.  Exit status 0 means every call
 * returned as expected; the sanitizers abort on any finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_mu(int mmax, double *mu);
int oracle_lambda(int lmax, int m, double x, double s, double *out);
int oracle_delta(int lmax, int nm, const int32_t *mval, int nrings, const double *cth,
                 const double *sth, const double *alm, double *delta, int nthreads);
int oracle_delta_adjoint(int lmax, int nm, const int32_t *mval, int nrings, const double *cth,
                         const double *sth, const double *dt, double *out, int nthreads);

static int run(int lmax, int nm, const int32_t *mval, int nrings)
{
    int64_t nalm = 0;
    for (int i = 0; i < nm; ++i) nalm += lmax - mval[i] + 1;
    double *cth = malloc(sizeof(double) * nrings), *sth = malloc(sizeof(double) * nrings);
    double *alm = malloc(sizeof(double) * 2 * nalm), *out = malloc(sizeof(double) * 2 * nalm);
    double *delta = malloc(sizeof(double) * 2 * (size_t)nrings * nm);
    if (!cth || !sth || !alm || !out || !delta) return 1;
    for (int r = 0; r < nrings; ++r) {
        /* both poles, the equator and points between */
        const double th = (nrings == 1) ? 0.0 : M_PI * r / (nrings - 1);
        cth[r] = (r == 0) ? 1.0 : (r == nrings - 1 ? -1.0 : cos(th));
        sth[r] = (r == 0 || r == nrings - 1) ? 0.0 : sin(th);
    }
    for (int64_t i = 0; i < 2 * nalm; ++i) alm[i] = 1.0 / (1.0 + (double)(i % 97));
    int rc = oracle_delta(lmax, nm, mval, nrings, cth, sth, alm, delta, 2);
    rc |= oracle_delta_adjoint(lmax, nm, mval, nrings, cth, sth, delta, out, 2);
    for (int64_t i = 0; i < 2 * (int64_t)nrings * nm; ++i)
        if (!isfinite(delta[i])) rc |= 2;
    for (int64_t i = 0; i < 2 * nalm; ++i)
        if (!isfinite(out[i])) rc |= 4;
    free(cth); free(sth); free(alm); free(out); free(delta);
    return rc;
}

int main(void)
{
    int fail = 0;
    double mu[65];
    oracle_mu(64, mu);
    double col[301];
    for (int m = 0; m <= 300; m += 50) {
        fail |= oracle_lambda(300, m, 0.3, sqrt(1.0 - 0.09), col) != 0;
        fail |= oracle_lambda(300, m, 1.0, 0.0, col) != 0;   /* pole */
    }
    fail |= oracle_lambda(0, 0, 0.5, sqrt(0.75), col) != 0;
    fail |= oracle_lambda(5, 6, 0.5, sqrt(0.75), col) != -1;  /* m > l_max refused */
    int32_t all[65], part[3] = {0, 7, 64}, top[1] = {64}, zero[1] = {0};
    for (int i = 0; i <= 64; ++i) all[i] = i;
    fail |= run(64, 65, all, 9) != 0;
    fail |= run(64, 3, part, 5) != 0;
    fail |= run(64, 1, top, 4) != 0;
    fail |= run(0, 1, zero, 1) != 0;
    fail |= run(300, 65, all, 3) != 0;
    /* argument checks: unsorted and out-of-range m-sets are refused */
    int32_t bad[2] = {5, 3};
    double c = 0.0, s = 1.0, a[32] = {0}, d[4] = {0};
    fail |= oracle_delta(8, 2, bad, 1, &c, &s, a, d, 1) != -1;
    fail |= oracle_delta(4, 1, top, 1, &c, &s, a, d, 1) != -1;
    if (fail) fprintf(stderr, "oracle driver: unexpected return code\n");
    else printf("oracle driver ok\n");
    return fail ? 1 : 0;
}
