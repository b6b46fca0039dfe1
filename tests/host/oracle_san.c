/* Host driver for the oracle under AddressSanitizer / UndefinedBehaviorSanitizer
 * (test infrastructure, built by tests/test_host_sanitizers.py): every transform of
 * every sampling at small sizes, with the exact round trips of the sampling
 * theorems as a functional check.  Prints "OK" and exits 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_num_rings(int L, int sampling, int nside);
void or_s2_inverse(int L, int s, int sampling, int nside, const double *flm, double *f, int nsel, const int *rings);
void or_s2_forward(int L, int s, int sampling, int nside, const double *f, double *flm, int nsel, const int *msel);
void or_s2_inverse_adjoint(int L, int s, int sampling, int nside, const double *g, double *gflm, int nsel,
                           const int *msel);
void or_so3_inverse(int L, int N, const double *flmn, double *f);
void or_so3_forward(int L, int N, const double *f, double *flmn);
void or_wigner_d_ell(int L, int m, int n, double beta, double *out);

static unsigned long long rng = 88172645463325252ULL;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0 - 0.5;
}

static long long map_size(int L, int sampling, int nside)
{
    switch (sampling) {
    case 0: return (long long)L * (2 * L - 1);            /* MW */
    case 1: return 12LL * nside * nside;                   /* HEALPix */
    case 2: return 2LL * L * (2 * L - 1);                  /* DH */
    case 3: return (long long)L * (2 * L - 1);            /* GL */
    default: return (long long)(L + 1) * 2 * L;           /* MWSS */
    }
}

/* band-limited coefficients: zero below max(|m|, |s|) */
static void draw(int L, int s, double *flm)
{
    const int M = 2 * L - 1;
    memset(flm, 0, sizeof(double) * 2 * (size_t)L * M);
    for (int l = 0; l < L; ++l)
        for (int m = -l; m <= l; ++m)
            if (l >= abs(s)) {
                flm[2 * ((size_t)l * M + m + L - 1)] = urand();
                flm[2 * ((size_t)l * M + m + L - 1) + 1] = urand();
            }
}

static double rel_err(const double *a, const double *b, size_t n)
{
    double num = 0.0, den = 0.0;
    for (size_t i = 0; i < n; ++i) {
        num += (a[i] - b[i]) * (a[i] - b[i]);
        den += b[i] * b[i];
    }
    return sqrt(num / den);
}

int main(void)
{
    int fails = 0;
    const int samplings[5] = {0, 1, 2, 3, 4};
    for (int k = 0; k < 5; ++k) {
        const int sampling = samplings[k];
        for (int s = -2; s <= 2; s += 2) {
            const int L = 8, nside = 4, M = 2 * L - 1;
            const size_t nc = 2 * (size_t)L * M;
            const long long np = map_size(L, sampling, nside);
            double *flm = malloc(sizeof(double) * nc), *back = malloc(sizeof(double) * nc);
            double *g = malloc(sizeof(double) * nc);
            double *f = malloc(sizeof(double) * 2 * (size_t)np);
            draw(L, s, flm);
            or_s2_inverse(L, s, sampling, nside, flm, f, -1, NULL);
            or_s2_forward(L, s, sampling, nside, f, back, -1, NULL);
            or_s2_inverse_adjoint(L, s, sampling, nside, f, g, -1, NULL);
            const int ring[2] = {0, or_num_rings(L, sampling, nside) - 1};
            const int ms[3] = {0, 3, -5};
            or_s2_inverse(L, s, sampling, nside, flm, f, 2, ring);
            or_s2_forward(L, s, sampling, nside, f, g, 3, ms);
            if (sampling != 1) {                                  /* sampling theorems: exact */
                or_s2_inverse(L, s, sampling, nside, flm, f, -1, NULL);
                or_s2_forward(L, s, sampling, nside, f, back, -1, NULL);
                const double e = rel_err(back, flm, nc);
                if (!(e < 1e-11)) { printf("round trip sampling %d spin %d: %.3e\n", sampling, s, e); ++fails; }
            }
            free(flm); free(back); free(g); free(f);
        }
    }
    {
        const int L = 6, N = 3, M = 2 * L - 1, G = 2 * N - 1;
        const size_t nc = 2 * (size_t)G * L * M;
        double *x = malloc(sizeof(double) * nc), *y = malloc(sizeof(double) * nc);
        double *f = malloc(sizeof(double) * 2 * (size_t)G * L * M);
        memset(x, 0, sizeof(double) * nc);
        for (int n = -(N - 1); n <= N - 1; ++n)
            for (int l = 0; l < L; ++l)
                for (int m = -l; m <= l; ++m)
                    if (l >= abs(n)) {
                        const size_t i = ((size_t)(n + N - 1) * L + l) * M + m + L - 1;
                        x[2 * i] = urand();
                        x[2 * i + 1] = urand();
                    }
        or_so3_inverse(L, N, x, f);
        or_so3_forward(L, N, f, y);
        const double e = rel_err(y, x, nc);
        if (!(e < 1e-11)) { printf("SO(3) round trip: %.3e\n", e); ++fails; }
        free(x); free(y); free(f);
    }
    {
        double d[16];
        or_wigner_d_ell(16, 3, -2, 0.7, d);
        double s2 = 0.0;                                          /* |d^l_{m,n}| <= 1 */
        for (int l = 3; l < 16; ++l) s2 = fmax(s2, fabs(d[l]));
        if (!(s2 <= 1.0 + 1e-12)) { printf("|d| > 1\n"); ++fails; }
    }
    if (fails) return 1;
    printf("OK\n");
    return 0;
}
