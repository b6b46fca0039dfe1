/*
 * s2oracle.c -- plain, slow, direct-summation CPU oracle for the spin
 * spherical-harmonic and Wigner transforms of Price & McEwen,
 * "Differentiable and accelerated spherical harmonic and Wigner transforms"
 * (arXiv 2311.14670).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls this code;
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, table or constant generator with the
 * GPU library: its own sampling geometry, its own Wigner-d (a recursion in
 * degree ell, not the paper's recursion in order m), its own DFTs (direct
 * sums with exact integer phase indices, never an FFT).
 *
 * Conventions (paper Sec. 2):
 *   sY_lm(theta,phi) = (-1)^s sqrt((2l+1)/4pi) e^{i m phi} d^l_{m,-s}(theta)
 *       -- the D <-> spin-harmonic relation (Eq. 9) with the D = e d e
 *          decomposition (Eq. 10); spin 0 reduces to Eq. 1 with the
 *          Condon-Shortley phase.
 *   Coefficient layout: flm[l][m + L - 1], complex interleaved (re, im).
 *   Entries with l < max(|m|, |s|) are ignored on input, zero on output.
 *
 * Samplings (paper Sec. 4.2), codes 0..3:
 *   0 MW:      theta_t = (2t+1) pi / (2L-1), t < L;  phi_p = 2 pi p / (2L-1).
 *   1 HEALPix: RING-ordered pixels, geometry of Gorski et al. (2005).
 *   2 DH:      theta_t = (2t+1) pi / (4L), t < 2L;   phi_p = 2 pi p / (2L-1);
 *              forward by the explicit DH quadrature weights.
 *   3 GL:      cos(theta_t) = roots of P_L (theta ascending), t < L;
 *              phi_p = 2 pi p / (2L-1); forward by Gauss-Legendre weights.
 *   4 MWSS:    theta_t = pi t / L, t = 0..L (both poles); phi_p = 2 pi p / (2L);
 *              forward exact like MW, on the 2L-point theta-torus.
 *   SO(3):   MW in (beta, alpha), gamma_k = 2 pi k / (2N-1) (Sec. 4.5).
 *
 * Every complex exponential whose phase is a rational multiple of pi is
 * evaluated from an integer phase index (k mod period) into a table of
 * roots of unity, so no large floating-point angle is ever formed.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define OR_PI_L 3.141592653589793238462643383279502884L

/* ------------------------------------------------------------------------ */
/* Sampling geometry                                                         */
/* ------------------------------------------------------------------------ */

/* MW colatitudes (Sec. 4.2, MW sampling theorem). */
void or_mw_thetas(int L, double *theta)
{
    for (int t = 0; t < L; ++t)
        theta[t] = (double)((2.0L * t + 1.0L) * OR_PI_L / (2.0L * L - 1.0L));
    theta[L - 1] = M_PI;                       /* t = L-1 is the south pole */
}

/* HEALPix RING geometry (Gorski et al. 2005; referenced in Sec. 4.2).
 * Ring r = 0 .. 4 nside - 2 (ring index i = r + 1).
 *   north cap  i <  nside : z = 1 - i^2/(3 nside^2), 4i pixels,
 *                           phi_j = pi/(2i) (j + 1/2)
 *   belt  nside <= i <= 3 nside : z = 4/3 - 2i/(3 nside), 4 nside pixels,
 *                           phi_j = pi/(2 nside) (j + shift/2),
 *                           shift = 1 if (i - nside) even else 0
 *   south cap i > 3 nside : mirror of ring 4 nside - i.
 * Outputs per ring: theta, number of pixels, first pixel index, and the
 * half-pixel shift flag s_r so that phi_j = (pi / nphi) (2 j + s_r).      */
void or_healpix_rings(int nside, double *theta, int *nphi, long long *start,
                      int *shift)
{
    const int nring = 4 * nside - 1;
    const long double ns = nside;
    long long pix = 0;
    for (int r = 0; r < nring; ++r) {
        const int i = r + 1;
        long double th;
        int np, sh;
        if (i < nside) {                        /* north cap */
            th = 2.0L * asinl((long double)i / (sqrtl(6.0L) * ns));
            np = 4 * i; sh = 1;
        } else if (i <= 3 * nside) {            /* belt */
            long double z = 4.0L / 3.0L - 2.0L * (long double)i / (3.0L * ns);
            th = acosl(z);
            np = 4 * nside; sh = ((i - nside) % 2 == 0) ? 1 : 0;
        } else {                                /* south cap */
            const int ii = 4 * nside - i;
            th = OR_PI_L - 2.0L * asinl((long double)ii / (sqrtl(6.0L) * ns));
            np = 4 * ii; sh = 1;
        }
        theta[r] = (double)th; nphi[r] = np; start[r] = pix; shift[r] = sh;
        pix += np;
    }
}

/* The same ring colatitudes kept in long double. */
static void hp_thetas_ld(int nside, long double *theta)
{
    const long double ns = nside;
    for (int r = 0; r < 4 * nside - 1; ++r) {
        const int i = r + 1;
        if (i < nside) theta[r] = 2.0L * asinl((long double)i / (sqrtl(6.0L) * ns));
        else if (i <= 3 * nside) theta[r] = acosl(4.0L / 3.0L - 2.0L * (long double)i / (3.0L * ns));
        else theta[r] = OR_PI_L - 2.0L * asinl((long double)(4 * nside - i) / (sqrtl(6.0L) * ns));
    }
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n, long double). */
/* ------------------------------------------------------------------------ */
void or_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        /* Tricomi-style initial guess, node i in decreasing order of x. */
        long double z = cosl(OR_PI_L * (i + 0.75L) / (n + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0L; }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L * (1.0L + fabsl(z))) {
                /* one more derivative evaluation at the converged node */
                p0 = 1.0L; p1 = z;
                for (int k = 2; k <= n; ++k) {
                    long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                    p0 = p1; p1 = p2;
                }
                if (n == 1) { p1 = z; p0 = 1.0L; }
                dp = n * (z * p1 - p0) / (z * z - 1.0L);
                break;
            }
        }
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

/* GL nodes as colatitudes, kept in long double (no rounding to double). */
static void gl_nodes_ld(int n, long double *theta, double *w)
{
    for (int i = 0; i < n; ++i) {
        long double z = cosl(OR_PI_L * (i + 0.75L) / (n + 0.5L)), dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0L; }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L * (1.0L + fabsl(z))) break;
        }
        long double p0 = 1.0L, p1 = z;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
            p0 = p1; p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0L; }
        dp = n * (z * p1 - p0) / (z * z - 1.0L);
        theta[i] = acosl(z);
        w[i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

/* DH colatitudes and theta weights (Sec. 4.2, DH sampling theorem):
 *   theta_t = (2t+1) pi / (4L),  t < 2L,
 *   w_t = (2/L) sin(theta_t) sum_{k<L} sin((2k+1) theta_t) / (2k+1),
 * so that sum_t w_t g(theta_t) = int_0^pi g sin(theta) dtheta for g of degree
 * < 2L in cos(theta); the paper's weight is (2 pi/(2L-1)) w_t.             */
static void dh_nodes_ld(int L, long double *theta, double *w)
{
    for (int t = 0; t < 2 * L; ++t) {
        const long double th = (2.0L * t + 1.0L) * OR_PI_L / (4.0L * L);
        long double acc = 0.0L;
        for (int k = 0; k < L; ++k) acc += sinl((2.0L * k + 1.0L) * th) / (2.0L * k + 1.0L);
        theta[t] = th;
        w[t] = (double)(2.0L / L * sinl(th) * acc);
    }
}

void or_dh_nodes(int L, double *theta, double *w)
{
    long double *th = (long double *)malloc(sizeof(long double) * 2 * L);
    dh_nodes_ld(L, th, w);
    for (int t = 0; t < 2 * L; ++t) theta[t] = (double)th[t];
    free(th);
}

void or_gl_nodes(int L, double *theta, double *w)
{
    long double *th = (long double *)malloc(sizeof(long double) * L);
    gl_nodes_ld(L, th, w);
    for (int t = 0; t < L; ++t) theta[t] = (double)th[t];
    free(th);
}

/* ------------------------------------------------------------------------ */
/* Wigner d by the three-term recursion in degree ell at fixed (m, n, beta). */
/* ------------------------------------------------------------------------ */
/*
 * d^l_{ln}(beta) (Eq. 27) as sign * 2^{log2mag}.  lg2 of the factorial
 * ratio is formed in long double from lgammal.  Requires 0 < beta < pi.
 */
static void d_top(int l, int n, long double beta, int *sign, long double *log2mag)
{
    const long double lf = lgammal(2.0L * l + 1.0L) - lgammal((long double)(l + n) + 1.0L)
                         - lgammal((long double)(l - n) + 1.0L);
    const long double sh = sinl(0.5L * beta), ch = cosl(0.5L * beta);
    *log2mag = (0.5L * lf + (l - n) * logl(sh) + (l + n) * logl(ch)) / logl(2.0L);
    *sign = ((l - n) % 2 == 0) ? 1 : -1;          /* (-sin(beta/2))^{l-n} */
}

/*
 * Starting value at l0 = max(|m|, |n|) from Eq. 27 and the symmetries
 * d^l_{mn} = (-1)^{m-n} d^l_{nm} = d^l_{-n,-m} (stated with Eq. 27).
 */
static void d_start(int m, int n, long double beta, int *sign, long double *log2mag)
{
    const int am = abs(m), an = abs(n);
    int sg; long double lm;
    if (am >= an) {
        const int l = am;
        if (m >= 0) { d_top(l, n, beta, &sg, &lm); }
        else {        /* d^l_{-l,n} = (-1)^{l+n} d^l_{l,-n} */
            d_top(l, -n, beta, &sg, &lm);
            if (((l + n) % 2 + 2) % 2) sg = -sg;
        }
    } else {
        const int l = an;
        if (n > 0) {  /* d^l_{m,l} = (-1)^{m-l} d^l_{l,m} */
            d_top(l, m, beta, &sg, &lm);
            if (((m - l) % 2 + 2) % 2) sg = -sg;
        } else {      /* d^l_{m,-l} = d^l_{l,-m} */
            d_top(l, -m, beta, &sg, &lm);
        }
    }
    *sign = sg; *log2mag = lm;
}

/*
 * out[l] = d^l_{mn}(beta) for l = 0 .. L-1 (zero for l < max(|m|,|n|)).
 * Poles use the closed forms of Eqs. 28-29.  Elsewhere: start value at l0,
 * then the standard upward three-term recursion in l,
 *   d^{l+1} = A_l (cos b - m n / (l (l+1))) d^l - B_l d^{l-1},
 *   A_l = (l+1)(2l+1) / sqrt(((l+1)^2 - m^2)((l+1)^2 - n^2)),
 *   B_l = (l+1) sqrt((l^2 - m^2)(l^2 - n^2)) / (l sqrt(((l+1)^2 - m^2)((l+1)^2 - n^2))),
 * carried as a mantissa pair with a common binary exponent so that values far
 * below the double range are followed exactly until they become representable.
 */
static void wigner_d_ld(int L, int m, int n, long double beta, double *out)
{
    for (int l = 0; l < L; ++l) out[l] = 0.0;
    const int l0 = abs(m) > abs(n) ? abs(m) : abs(n);
    if (l0 >= L) return;
    if (beta == 0.0L) {                      /* Eq. 28: d(0) = delta_mn */
        if (m == n) for (int l = l0; l < L; ++l) out[l] = 1.0;
        return;
    }
    if (beta == OR_PI_L || beta == (long double)M_PI) {   /* Eq. 29: (-1)^{l+m} delta_{m,-n} */
        if (m == -n)
            for (int l = l0; l < L; ++l) out[l] = (((l + m) % 2 + 2) % 2) ? -1.0 : 1.0;
        return;
    }
    int sg; long double lg2;
    d_start(m, n, beta, &sg, &lg2);
    long double fl = floorl(lg2);
    int e = (int)fl;
    /* the recursion is carried in long double: near the poles it depends on
       1 - cos(beta), which a double cos(beta) would only hold to eps/(1-cos) */
    long double a = sg * exp2l(lg2 - fl);    /* d^{l0} = a * 2^e */
    long double b = 0.0L;                     /* d^{l0-1} = 0     */
    const long double cb = cosl(beta);
    const long double mm = (long double)m * m, nn = (long double)n * n, mn = (long double)m * n;
    out[l0] = (double)ldexpl(a, e);
    for (int l = l0; l < L - 1; ++l) {
        const long double lp1 = l + 1.0L;
        const long double den = sqrtl((lp1 * lp1 - mm) * (lp1 * lp1 - nn));
        const long double A = lp1 * (2.0L * l + 1.0L) / den;
        long double c;
        if (l == 0) c = A * cb * a;
        else {
            const long double B = lp1 * sqrtl(((long double)l * l - mm) * ((long double)l * l - nn)) / (l * den);
            c = A * (cb - mn / ((long double)l * lp1)) * a - B * b;
        }
        b = a; a = c;
        /* keep the mantissa pair in a comfortable range */
        const long double mx = fmaxl(fabsl(a), fabsl(b));
        if (mx > 0x1p+300L || (mx < 0x1p-300L && mx > 0.0L)) {
            int k; frexpl(mx, &k);
            a = ldexpl(a, -k); b = ldexpl(b, -k); e += k;
        }
        out[l + 1] = (double)ldexpl(a, e);
    }
}

void or_wigner_d_ell(int L, int m, int n, double beta, double *out)
{
    wigner_d_ld(L, m, n, (long double)beta, out);
}

/* ------------------------------------------------------------------------ */
/* Helpers                                                                   */
/* ------------------------------------------------------------------------ */

/* roots[k] = e^{sgn * i * 2 pi k / P}, k < P (long double evaluation). */
static double *root_table(int P, int sgn)
{
    double *r = (double *)malloc(sizeof(double) * 2 * (size_t)P);
    for (int k = 0; k < P; ++k) {
        long double a = 2.0L * OR_PI_L * (long double)k / (long double)P;
        r[2 * k] = (double)cosl(a);
        r[2 * k + 1] = sgn * (double)sinl(a);
    }
    return r;
}

static inline long long pmod(long long a, long long p) { long long r = a % p; return r < 0 ? r + p : r; }

static inline int iabs_(int a) { return a < 0 ? -a : a; }

/* w_l = (-1)^s sqrt((2l+1)/(4 pi))  (Eqs. 30 and 33) */
static double w_sht(int l, int s)
{
    double v = (double)sqrtl((2.0L * l + 1.0L) / (4.0L * OR_PI_L));
    return (iabs_(s) % 2) ? -v : v;
}

/* ------------------------------------------------------------------------ */
/* Inverse spin SHT (Eq. 4 with the spin harmonics of Eq. 9), direct sum.    */
/* ------------------------------------------------------------------------ */
/*
 * sampling 0 = MW, 1 = HEALPix (nside).  f receives the map for the selected
 * rings (rings == NULL: all rings), each ring's samples packed one after the
 * other in selection order.  For a single ring theta:
 *   f(theta, phi_p) = sum_m e^{i m phi_p} sum_l w_l flm[l][m] d^l_{m,-s}(theta)
 * which is Eq. 4 with the sum over m taken outermost, as the paper writes it
 * in Eqs. 32-33.
 */
static void ring_inverse(int L, int s, long double theta, int nphi, int shift, int mwphi,
                         const double *flm, double *fr, double *dbuf, double *ft)
{
    const int M = 2 * L - 1;
    for (int m = -(L - 1); m <= L - 1; ++m) {
        wigner_d_ld(L, m, -s, theta, dbuf);
        long double re = 0.0L, im = 0.0L;
        const int l0 = iabs_(m) > iabs_(s) ? iabs_(m) : iabs_(s);
        for (int l = l0; l < L; ++l) {
            const long double c = (long double)w_sht(l, s) * dbuf[l];
            re += c * flm[2 * ((size_t)l * M + m + L - 1)];
            im += c * flm[2 * ((size_t)l * M + m + L - 1) + 1];
        }
        ft[2 * (m + L - 1)] = (double)re; ft[2 * (m + L - 1) + 1] = (double)im;
    }
    /* phase of sample p: MW    phi_p = 2 pi p / (2L-1)        -> index m p mod (2L-1)
     *                    HEALPix phi_p = pi (2p + shift) / nphi -> index m (2p+shift) mod 2 nphi */
    const int P = mwphi ? M : 2 * nphi;
    double *rt = root_table(P, +1);
    for (int p = 0; p < nphi; ++p) {
        long double re = 0.0L, im = 0.0L;
        const long long q = mwphi ? p : (2LL * p + shift);
        for (int m = -(L - 1); m <= L - 1; ++m) {
            const long long k = pmod((long long)m * q, P);
            const long double cr = rt[2 * k], ci = rt[2 * k + 1];
            const long double ar = ft[2 * (m + L - 1)], ai = ft[2 * (m + L - 1) + 1];
            re += ar * cr - ai * ci;
            im += ar * ci + ai * cr;
        }
        fr[2 * p] = (double)re; fr[2 * p + 1] = (double)im;
    }
    free(rt);
}

/* Ring list helper: number of rings, theta, nphi, shift, offset in the map;
 * for DH and GL also the theta weights of the forward quadrature.          */
typedef struct { int nring; double *theta; long double *thl; int *nphi; int *shift; long long *start; double *wq; } rings_t;

static rings_t make_rings(int L, int sampling, int nside)
{
    rings_t R;
    R.wq = NULL;
    if (sampling == 4) {
        R.nring = L + 1;
        R.theta = (double *)malloc(sizeof(double) * R.nring);
        R.nphi = (int *)malloc(sizeof(int) * R.nring);
        R.shift = (int *)malloc(sizeof(int) * R.nring);
        R.start = (long long *)malloc(sizeof(long long) * R.nring);
        R.thl = (long double *)malloc(sizeof(long double) * R.nring);
        for (int t = 0; t <= L; ++t) {
            R.thl[t] = (t == L) ? OR_PI_L : OR_PI_L * t / L;
            R.theta[t] = (double)R.thl[t];
            R.nphi[t] = 2 * L; R.shift[t] = 0; R.start[t] = (long long)t * 2 * L;
        }
    } else if (sampling == 2 || sampling == 3) {
        R.nring = sampling == 2 ? 2 * L : L;
        R.theta = (double *)malloc(sizeof(double) * R.nring);
        R.nphi = (int *)malloc(sizeof(int) * R.nring);
        R.shift = (int *)malloc(sizeof(int) * R.nring);
        R.start = (long long *)malloc(sizeof(long long) * R.nring);
        R.thl = (long double *)malloc(sizeof(long double) * R.nring);
        R.wq = (double *)malloc(sizeof(double) * R.nring);
        if (sampling == 2) dh_nodes_ld(L, R.thl, R.wq);
        else gl_nodes_ld(L, R.thl, R.wq);
        for (int t = 0; t < R.nring; ++t) {
            R.theta[t] = (double)R.thl[t];
            R.nphi[t] = 2 * L - 1; R.shift[t] = 0; R.start[t] = (long long)t * (2 * L - 1);
        }
    } else if (sampling == 0) {
        R.nring = L;
        R.theta = (double *)malloc(sizeof(double) * L);
        R.nphi = (int *)malloc(sizeof(int) * L);
        R.shift = (int *)malloc(sizeof(int) * L);
        R.start = (long long *)malloc(sizeof(long long) * L);
        or_mw_thetas(L, R.theta);
        R.thl = (long double *)malloc(sizeof(long double) * L);
        for (int t = 0; t < L; ++t) {
            R.nphi[t] = 2 * L - 1; R.shift[t] = 0; R.start[t] = (long long)t * (2 * L - 1);
            R.thl[t] = (t == L - 1) ? OR_PI_L : (2.0L * t + 1.0L) * OR_PI_L / (2.0L * L - 1.0L);
        }
    } else {
        R.nring = 4 * nside - 1;
        R.theta = (double *)malloc(sizeof(double) * R.nring);
        R.nphi = (int *)malloc(sizeof(int) * R.nring);
        R.shift = (int *)malloc(sizeof(int) * R.nring);
        R.start = (long long *)malloc(sizeof(long long) * R.nring);
        or_healpix_rings(nside, R.theta, R.nphi, R.start, R.shift);
        R.thl = (long double *)malloc(sizeof(long double) * R.nring);
        hp_thetas_ld(nside, R.thl);
    }
    return R;
}

static void free_rings(rings_t *R)
{
    free(R->theta); free(R->thl); free(R->nphi); free(R->shift); free(R->start); free(R->wq);
}


/* e^{-i pi k / nphi} tables for every distinct HEALPix ring length (index nphi/4). */
static double **hp_root_tables(const rings_t *R)
{
    int maxq = 0;
    for (int r = 0; r < R->nring; ++r) if (R->nphi[r] / 4 > maxq) maxq = R->nphi[r] / 4;
    double **tab = (double **)calloc((size_t)maxq + 1, sizeof(double *));
    for (int r = 0; r < R->nring; ++r) {
        const int q = R->nphi[r] / 4;
        if (!tab[q]) tab[q] = root_table(2 * R->nphi[r], -1);
    }
    return tab;
}

static void free_hp_root_tables(const rings_t *R, double **tab)
{
    int maxq = 0;
    for (int r = 0; r < R->nring; ++r) if (R->nphi[r] / 4 > maxq) maxq = R->nphi[r] / 4;
    for (int q = 0; q <= maxq; ++q) free(tab[q]);
    free(tab);
}

int or_num_rings(int L, int sampling, int nside)
{
    return sampling == 0 || sampling == 3 ? L : sampling == 2 ? 2 * L : sampling == 4 ? L + 1 : 4 * nside - 1;
}

/* phi_p = 2 pi p / (2L-1) (MW, DH, GL) */
static int phi_2l1(int sampling) { return sampling == 0 || sampling == 2 || sampling == 3; }

void or_s2_inverse(int L, int s, int sampling, int nside, const double *flm, double *f,
                   int nsel, const int *rings)
{
    rings_t R = make_rings(L, sampling, nside);
    const int nr = (nsel < 0) ? R.nring : nsel;
    long long *off = (long long *)malloc(sizeof(long long) * (nr + 1));
    off[0] = 0;
    for (int i = 0; i < nr; ++i) {
        const int r = (nsel < 0) ? i : rings[i];
        off[i + 1] = off[i] + R.nphi[r];
    }
    #pragma omp parallel
    {
        double *dbuf = (double *)malloc(sizeof(double) * L);
        double *ft = (double *)malloc(sizeof(double) * 2 * (2 * L - 1));
        #pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nr; ++i) {
            const int r = (nsel < 0) ? i : rings[i];
            /* MWSS (phi_p = pi p / L) goes through the HEALPix-style phase index 2p / (2 nphi) */
            ring_inverse(L, s, R.thl[r], R.nphi[r], R.shift[r], phi_2l1(sampling),
                         flm, f + 2 * off[i], dbuf, ft);
        }
        free(dbuf); free(ft);
    }
    free(off);
    free_rings(&R);
}

/* ------------------------------------------------------------------------ */
/* Direct forward phi-DFT of one ring at order m (Eq. 31 without weight).    */
/* ------------------------------------------------------------------------ */
static void ring_dft(const double *fr, int nphi, int shift, int mwphi, int m, int L,
                     const double *rt, int P, double *out)
{
    long double re = 0.0L, im = 0.0L;
    for (int p = 0; p < nphi; ++p) {
        const long long q = mwphi ? p : (2LL * p + shift);
        const long long k = pmod((long long)m * q, P);     /* rt holds e^{-i 2 pi k / P} */
        const long double cr = rt[2 * k], ci = rt[2 * k + 1];
        const long double ar = fr[2 * p], ai = fr[2 * p + 1];
        re += ar * cr - ai * ci;
        im += ar * ci + ai * cr;
    }
    (void)L;
    out[0] = (double)re; out[1] = (double)im;
}

/* ------------------------------------------------------------------------ */
/* MW forward: <I(f), sY_lm> = w_l int_0^pi g_m(theta) d(theta) sin(theta).  */
/* ------------------------------------------------------------------------ */
/* g(theta) = sum_k ghat_k e^{ik theta} at one colatitude (long double rotation). */
static void eval_interp(int L, const double *gh, long double th, double *out)
{
    const long double c1 = cosl(th), s1 = sinl(th);
    long double cr = cosl((long double)(L - 1) * th), ci = -sinl((long double)(L - 1) * th);
    long double re = 0.0L, im = 0.0L;
    for (int k = -(L - 1); k <= L - 1; ++k) {
        const long double ar = gh[2 * (k + L - 1)], ai = gh[2 * (k + L - 1) + 1];
        re += ar * cr - ai * ci;
        im += ar * ci + ai * cr;
        const long double nr = cr * c1 - ci * s1, ni = cr * s1 + ci * c1;
        cr = nr; ci = ni;
    }
    out[0] = (double)re; out[1] = (double)im;
}

/*
 * For one order m and the L-ring MW samples gt[t] = ftilde_m(theta_t):
 *  (1) extend to the 2L-1 torus samples with g(2pi - theta) = parity * g(theta),
 *      parity = (-1)^{m+s} (reflection with the pi phi-shift and the (-1)^s
 *      sign, Sec. 4.2 MW); the pole sample t = L-1 is its own mirror and is
 *      used as given.  MWSS (ss = 1): the L+1 samples t = 0..L (theta_t = pi t/L)
 *      extend to the 2L torus samples, mirror of t being 2L - t (both poles are
 *      their own mirrors);
 *  (2) the torus interpolant of degree L-1, g(theta) = sum_k ghat_k e^{ik theta},
 *      ghat_k = (1/N) sum_t g_t e^{-ik theta_t}, N = 2L-1 (MW) or 2L (MWSS; the
 *      Nyquist frequency L is left out, it vanishes for band-limited samples);
 *  (3) out_l = wl[l] * int_0^pi g(theta) d^l_{mn}(theta) sin(theta) dtheta,
 *      evaluated exactly: with d(-theta) = parity d(theta), the integrand splits
 *      into G+ = d (g(th) + parity g(-th))/2, a polynomial of degree <= 2L-2 in
 *      cos(theta) (L-node Gauss-Legendre is exact), and
 *      G- = d (g(th) - parity g(-th))/2 = sin(theta) Q(cos theta), deg Q <= 2L-3,
 *      whose integral int sqrt(1-x^2) Q(x) dx is exact with L-node Gauss-Chebyshev
 *      of the second kind.  G- vanishes for samples of a band-limited signal.
 */
static void mw_theta_forward(int L, int m, int n, int parity, const double *gt,
                             const double *wl, const long double *thgl, const double *wgl,
                             const double *rt2N, double *out, double *dbuf, int ss)
{
    const int N = ss ? 2 * L : 2 * L - 1;
    const int ngiven = ss ? L + 1 : L;
    double *g = (double *)malloc(sizeof(double) * 2 * N);
    for (int t = 0; t < N; ++t) {
        if (t < ngiven) { g[2 * t] = gt[2 * t]; g[2 * t + 1] = gt[2 * t + 1]; }
        else {
            const int tr = ss ? N - t : N - 1 - t;
            g[2 * t] = parity * gt[2 * tr]; g[2 * t + 1] = parity * gt[2 * tr + 1];
        }
    }
    /* ghat_k, k = -(L-1)..L-1; e^{-ik theta_t} = e^{-i pi idx / N} with idx = k(2t+1) (MW)
     * or 2kt (MWSS), mod 2N, from rt2N */
    double *gh = (double *)malloc(sizeof(double) * 2 * N);
    for (int k = -(L - 1); k <= L - 1; ++k) {
        long double re = 0.0L, im = 0.0L;
        for (int t = 0; t < N; ++t) {
            const long long idx = pmod((long long)k * (ss ? 2 * t : 2 * t + 1), 2LL * N);
            const long double cr = rt2N[2 * idx], ci = rt2N[2 * idx + 1];  /* e^{-i pi idx / N} */
            re += g[2 * t] * cr - g[2 * t + 1] * ci;
            im += g[2 * t] * ci + g[2 * t + 1] * cr;
        }
        gh[2 * (k + L - 1)] = (double)(re / N); gh[2 * (k + L - 1) + 1] = (double)(im / N);
    }
    long double *acc = (long double *)calloc(2 * (size_t)L, sizeof(long double));
    double gp[2], gm[2];
    /* even part: Gauss-Legendre */
    for (int j = 0; j < L; ++j) {
        eval_interp(L, gh, thgl[j], gp);
        eval_interp(L, gh, -thgl[j], gm);
        const long double ar = 0.5L * wgl[j] * ((long double)gp[0] + parity * (long double)gm[0]);
        const long double ai = 0.5L * wgl[j] * ((long double)gp[1] + parity * (long double)gm[1]);
        wigner_d_ld(L, m, n, thgl[j], dbuf);
        for (int l = 0; l < L; ++l) { acc[2 * l] += ar * dbuf[l]; acc[2 * l + 1] += ai * dbuf[l]; }
    }
    /* odd part: Gauss-Chebyshev (second kind), nodes j pi/(L+1), weights pi/(L+1) sin^2 */
    for (int j = 1; j <= L; ++j) {
        const long double th = OR_PI_L * j / (L + 1.0L);
        eval_interp(L, gh, th, gp);
        eval_interp(L, gh, -th, gm);
        const long double dr = (long double)gp[0] - parity * (long double)gm[0];
        const long double di = (long double)gp[1] - parity * (long double)gm[1];
        if (dr == 0.0L && di == 0.0L) continue;
        const long double wq = 0.5L * OR_PI_L / (L + 1.0L) * sinl(th);
        wigner_d_ld(L, m, n, th, dbuf);
        for (int l = 0; l < L; ++l) { acc[2 * l] += wq * dr * dbuf[l]; acc[2 * l + 1] += wq * di * dbuf[l]; }
    }
    const int l0 = iabs_(m) > iabs_(n) ? iabs_(m) : iabs_(n);
    for (int l = 0; l < L; ++l) {
        const long double c = (l < l0) ? 0.0L : (long double)wl[l];
        out[2 * l] = (double)(acc[2 * l] * c); out[2 * l + 1] = (double)(acc[2 * l + 1] * c);
    }
    free(acc); free(g); free(gh);
}

/*
 * Forward spin SHT.  MW: the exact transform of Sec. 4.2 (torus extension of
 * the ring DFTs, computed here by GL quadrature of the interpolant).
 * HEALPix: the plain quadrature of Eq. 19 with q = 4 pi / Npix.
 * DH, GL: the quadrature of Eq. 19 with the sampling theorem's weights
 * q_t = (2 pi / (2L-1)) w_t (exact for band-limited maps).
 * Only the orders in msel (nsel >= 0) are computed; other columns are zero.
 */
void or_s2_forward(int L, int s, int sampling, int nside, const double *f, double *flm,
                   int nsel, const int *msel)
{
    const int M = 2 * L - 1;
    memset(flm, 0, sizeof(double) * 2 * (size_t)L * M);
    rings_t R = make_rings(L, sampling, nside);
    const int nm = (nsel < 0) ? M : nsel;
    double *wl = (double *)malloc(sizeof(double) * L);
    for (int l = 0; l < L; ++l) wl[l] = w_sht(l, s);
    long double *thgl = (long double *)malloc(sizeof(long double) * L);
    double *wgl = (double *)malloc(sizeof(double) * L);
    if (sampling == 0 || sampling == 4) gl_nodes_ld(L, thgl, wgl);
    double *rt2N = root_table(2 * M, -1);          /* e^{-i pi k / M} */
    double *rt4L = root_table(4 * L, -1);          /* e^{-i pi k / (2L)}: MWSS torus */
    double *rt2L = root_table(2 * L, -1);          /* e^{-2 pi i k / (2L)}: MWSS rings */
    double *rtM = root_table(M, -1);
    double **hpt = (sampling == 1) ? hp_root_tables(&R) : NULL;
    const long long npix = 12LL * nside * nside;
    #pragma omp parallel
    {
        double *dbuf = (double *)malloc(sizeof(double) * L);
        double *gt = (double *)malloc(sizeof(double) * 2 * R.nring);
        double *col = (double *)malloc(sizeof(double) * 2 * L);
        #pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nm; ++i) {
            const int m = (nsel < 0) ? i - (L - 1) : msel[i];
            if (sampling == 0) {
                const double q = (double)(2.0L * OR_PI_L / M);       /* Eq. 31 weight */
                for (int t = 0; t < L; ++t) {
                    ring_dft(f + 2 * R.start[t], M, 0, 1, m, L, rtM, M, gt + 2 * t);
                    gt[2 * t] *= q; gt[2 * t + 1] *= q;
                }
                const int parity = (iabs_(m + s) % 2) ? -1 : 1;
                mw_theta_forward(L, m, -s, parity, gt, wl, thgl, wgl, rt2N, col, dbuf, 0);
            } else if (sampling == 4) {
                const double q = (double)(2.0L * OR_PI_L / (2 * L));   /* phi rule of 2L samples */
                for (int t = 0; t <= L; ++t) {
                    ring_dft(f + 2 * R.start[t], 2 * L, 0, 1, m, L, rt2L, 2 * L, gt + 2 * t);
                    gt[2 * t] *= q; gt[2 * t + 1] *= q;
                }
                const int parity = (iabs_(m + s) % 2) ? -1 : 1;
                mw_theta_forward(L, m, -s, parity, gt, wl, thgl, wgl, rt4L, col, dbuf, 1);
            } else {
                for (int l = 0; l < L; ++l) { col[2 * l] = 0.0; col[2 * l + 1] = 0.0; }
                for (int r = 0; r < R.nring; ++r) {
                    double fm[2];
                    double q;
                    if (sampling == 1) {
                        q = (double)(4.0L * OR_PI_L / (long double)npix);
                        ring_dft(f + 2 * R.start[r], R.nphi[r], R.shift[r], 0, m, L, hpt[R.nphi[r] / 4],
                                 2 * R.nphi[r], fm);
                    } else {
                        q = (double)(2.0L * OR_PI_L / M) * R.wq[r];
                        ring_dft(f + 2 * R.start[r], M, 0, 1, m, L, rtM, M, fm);
                    }
                    wigner_d_ld(L, m, -s, R.thl[r], dbuf);
                    for (int l = 0; l < L; ++l) {
                        const double c = q * wl[l] * dbuf[l];
                        col[2 * l] += c * fm[0]; col[2 * l + 1] += c * fm[1];
                    }
                }
                const int l0 = iabs_(m) > iabs_(s) ? iabs_(m) : iabs_(s);
                for (int l = 0; l < l0; ++l) { col[2 * l] = 0.0; col[2 * l + 1] = 0.0; }
            }
            for (int l = 0; l < L; ++l) {
                flm[2 * ((size_t)l * M + m + L - 1)] = col[2 * l];
                flm[2 * ((size_t)l * M + m + L - 1) + 1] = col[2 * l + 1];
            }
        }
        free(dbuf); free(gt); free(col);
    }
    free(wl); free(thgl); free(wgl); free(rt2N); free(rtM); free(rt4L); free(rt2L);
    if (hpt) free_hp_root_tables(&R, hpt);
    free_rings(&R);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the inverse SHT: gflm_lm = sum_{t,p} g(t,p) conj(sY_lm(t,p)).  */
/* The Hermitian adjoint in the sense used for complex gradients (Eq. 58).   */
/* ------------------------------------------------------------------------ */
void or_s2_inverse_adjoint(int L, int s, int sampling, int nside, const double *g, double *gflm,
                           int nsel, const int *msel)
{
    const int M = 2 * L - 1;
    memset(gflm, 0, sizeof(double) * 2 * (size_t)L * M);
    rings_t R = make_rings(L, sampling, nside);
    const int nm = (nsel < 0) ? M : nsel;
    double *rtM = root_table(M, -1);
    double *rt2L = root_table(2 * L, -1);
    double **hpt = (sampling == 1) ? hp_root_tables(&R) : NULL;
    #pragma omp parallel
    {
        double *dbuf = (double *)malloc(sizeof(double) * L);
        double *col = (double *)malloc(sizeof(double) * 2 * L);
        #pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nm; ++i) {
            const int m = (nsel < 0) ? i - (L - 1) : msel[i];
            for (int l = 0; l < L; ++l) { col[2 * l] = 0.0; col[2 * l + 1] = 0.0; }
            for (int r = 0; r < R.nring; ++r) {
                double fm[2];
                if (sampling == 4) ring_dft(g + 2 * R.start[r], 2 * L, 0, 1, m, L, rt2L, 2 * L, fm);
                else if (sampling != 1) ring_dft(g + 2 * R.start[r], M, 0, 1, m, L, rtM, M, fm);
                else ring_dft(g + 2 * R.start[r], R.nphi[r], R.shift[r], 0, m, L,
                              hpt[R.nphi[r] / 4], 2 * R.nphi[r], fm);
                wigner_d_ld(L, m, -s, R.thl[r], dbuf);
                for (int l = 0; l < L; ++l) {
                    const double c = w_sht(l, s) * dbuf[l];
                    col[2 * l] += c * fm[0]; col[2 * l + 1] += c * fm[1];
                }
            }
            const int l0 = iabs_(m) > iabs_(s) ? iabs_(m) : iabs_(s);
            for (int l = l0; l < L; ++l) {
                gflm[2 * ((size_t)l * M + m + L - 1)] = col[2 * l];
                gflm[2 * ((size_t)l * M + m + L - 1) + 1] = col[2 * l + 1];
            }
        }
        free(dbuf); free(col);
    }
    free(rtM); free(rt2L);
    if (hpt) free_hp_root_tables(&R, hpt);
    free_rings(&R);
}

/* ------------------------------------------------------------------------ */
/* Wigner (SO(3)) transforms, MW in (beta, alpha), gamma_k = 2 pi k/(2N-1).  */
/* Layouts: flmn[n + N-1][l][m + L-1], f[k][t][p].                           */
/* ------------------------------------------------------------------------ */
/*
 * Inverse (Eq. 13 with D of Eq. 10):
 *   f(alpha_p, beta_t, gamma_k) = sum_n e^{i n gamma_k} sum_m e^{i m alpha_p}
 *                                 sum_l (2l+1)/(8 pi^2) flmn d^l_{mn}(beta_t)
 */
void or_so3_inverse(int L, int N, const double *flmn, double *f)
{
    const int M = 2 * L - 1, G = 2 * N - 1;
    long double *th = (long double *)malloc(sizeof(long double) * L);
    for (int t = 0; t < L; ++t) th[t] = (t == L - 1) ? OR_PI_L : (2.0L * t + 1.0L) * OR_PI_L / (2.0L * L - 1.0L);
    double *rtM = root_table(M, +1), *rtG = root_table(G, +1);
    const size_t slab = (size_t)L * M;
    #pragma omp parallel
    {
        double *dbuf = (double *)malloc(sizeof(double) * L);
        double *fn = (double *)malloc(sizeof(double) * 2 * (size_t)G * M);  /* [n][m] at this beta */
        double *fa = (double *)malloc(sizeof(double) * 2 * (size_t)G * M);  /* [n][p] */
        #pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < L; ++t) {
            for (int n = -(N - 1); n <= N - 1; ++n) {
                const double *fl = flmn + 2 * (size_t)(n + N - 1) * slab;
                for (int m = -(L - 1); m <= L - 1; ++m) {
                    wigner_d_ld(L, m, n, th[t], dbuf);
                    double re = 0.0, im = 0.0;
                    for (int l = 0; l < L; ++l) {
                        const double c = (double)((2.0L * l + 1.0L) / (8.0L * OR_PI_L * OR_PI_L)) * dbuf[l];
                        re += c * fl[2 * ((size_t)l * M + m + L - 1)];
                        im += c * fl[2 * ((size_t)l * M + m + L - 1) + 1];
                    }
                    fn[2 * ((size_t)(n + N - 1) * M + m + L - 1)] = re;
                    fn[2 * ((size_t)(n + N - 1) * M + m + L - 1) + 1] = im;
                }
                for (int p = 0; p < M; ++p) {
                    double re = 0.0, im = 0.0;
                    for (int m = -(L - 1); m <= L - 1; ++m) {
                        const long long k = pmod((long long)m * p, M);
                        const double ar = fn[2 * ((size_t)(n + N - 1) * M + m + L - 1)];
                        const double ai = fn[2 * ((size_t)(n + N - 1) * M + m + L - 1) + 1];
                        re += ar * rtM[2 * k] - ai * rtM[2 * k + 1];
                        im += ar * rtM[2 * k + 1] + ai * rtM[2 * k];
                    }
                    fa[2 * ((size_t)(n + N - 1) * M + p)] = re;
                    fa[2 * ((size_t)(n + N - 1) * M + p) + 1] = im;
                }
            }
            for (int k = 0; k < G; ++k)
                for (int p = 0; p < M; ++p) {
                    double re = 0.0, im = 0.0;
                    for (int n = -(N - 1); n <= N - 1; ++n) {
                        const long long q = pmod((long long)n * k, G);
                        const double ar = fa[2 * ((size_t)(n + N - 1) * M + p)];
                        const double ai = fa[2 * ((size_t)(n + N - 1) * M + p) + 1];
                        re += ar * rtG[2 * q] - ai * rtG[2 * q + 1];
                        im += ar * rtG[2 * q + 1] + ai * rtG[2 * q];
                    }
                    f[2 * (((size_t)k * L + t) * M + p)] = re;
                    f[2 * (((size_t)k * L + t) * M + p) + 1] = im;
                }
        }
        free(dbuf); free(fn); free(fa);
    }
    free(th); free(rtM); free(rtG);
}

/*
 * Forward (Eq. 14): gamma and alpha integrals by their exact equispaced
 * rules (weights 2pi/(2N-1), 2pi/(2L-1)), beta integral exactly through the
 * torus extension with parity (-1)^{m-n} (spin -n, Eq. 15) and GL quadrature
 * of the interpolant; per-l weight 1.
 */
void or_so3_forward(int L, int N, const double *f, double *flmn)
{
    const int M = 2 * L - 1, G = 2 * N - 1;
    const size_t slab = (size_t)L * M;
    memset(flmn, 0, sizeof(double) * 2 * (size_t)G * slab);
    double *rtM = root_table(M, -1), *rtG = root_table(G, -1), *rt2N = root_table(2 * M, -1);
    long double *thgl = (long double *)malloc(sizeof(long double) * L);
    double *wgl = (double *)malloc(sizeof(double) * L);
    gl_nodes_ld(L, thgl, wgl);
    double *wl = (double *)malloc(sizeof(double) * L);
    for (int l = 0; l < L; ++l) wl[l] = 1.0;
    const double qa = (double)(2.0L * OR_PI_L / M), qg = (double)(2.0L * OR_PI_L / G);
    #pragma omp parallel
    {
        double *dbuf = (double *)malloc(sizeof(double) * L);
        double *gt = (double *)malloc(sizeof(double) * 2 * L);
        double *col = (double *)malloc(sizeof(double) * 2 * L);
        #pragma omp for schedule(dynamic, 1) collapse(2)
        for (int n = -(N - 1); n <= N - 1; ++n)
            for (int m = -(L - 1); m <= L - 1; ++m) {
                for (int t = 0; t < L; ++t) {
                    double re = 0.0, im = 0.0;
                    for (int k = 0; k < G; ++k)
                        for (int p = 0; p < M; ++p) {
                            /* rtM, rtG hold e^{-i 2 pi k / P} */
                            const long long ia = pmod((long long)m * p, M);
                            const long long ig = pmod((long long)n * k, G);
                            const double cr = rtM[2 * ia] * rtG[2 * ig] - rtM[2 * ia + 1] * rtG[2 * ig + 1];
                            const double ci = rtM[2 * ia] * rtG[2 * ig + 1] + rtM[2 * ia + 1] * rtG[2 * ig];
                            const double ar = f[2 * (((size_t)k * L + t) * M + p)];
                            const double ai = f[2 * (((size_t)k * L + t) * M + p) + 1];
                            re += ar * cr - ai * ci;
                            im += ar * ci + ai * cr;
                        }
                    gt[2 * t] = re * qa * qg; gt[2 * t + 1] = im * qa * qg;
                }
                const int parity = (iabs_(m - n) % 2) ? -1 : 1;
                mw_theta_forward(L, m, n, parity, gt, wl, thgl, wgl, rt2N, col, dbuf, 0);
                double *fl = flmn + 2 * (size_t)(n + N - 1) * slab;
                for (int l = 0; l < L; ++l) {
                    fl[2 * ((size_t)l * M + m + L - 1)] = col[2 * l];
                    fl[2 * ((size_t)l * M + m + L - 1) + 1] = col[2 * l + 1];
                }
            }
        free(dbuf); free(gt); free(col);
    }
    free(rtM); free(rtG); free(rt2N); free(thgl); free(wgl); free(wl);
}
