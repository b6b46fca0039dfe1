// s2mi_consts.cpp -- host-side generation of the plan constants in quad
// precision (libquadmath), rounded once to double or split into double-double.
//
// Nothing here touches the GPU; s2mi_capi.hip uploads the arrays.
//
// Paper references (Price & McEwen, arXiv 2311.14670):
//   ring geometry      Sec. 4.2 (MW: theta_t = (2t+1) pi/(2L-1); HEALPix RING
//                      geometry of Gorski et al. 2005)
//   recursion          Sec. 3.3, Eqs. 25-26 (descending-m three-term recursion)
//   initial values     Eq. 27, computed in log space (Sec. 3.3)
//   MW theta weights   Sec. 4.2, Eqs. 41-42 (band-limited sin(theta) 1_[0,pi])
#include <algorithm>
#include <quadmath.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "s2mi_internal.h"

namespace s2mi {

namespace {
using q = __float128;
const q QPI = M_PIq;

inline void split_dd(q v, double *hi, double *lo)
{
    const double h = (double)v;
    *hi = h;
    *lo = (double)(v - (q)h);
}
}  // namespace

// Regular (non-polar) MW colatitudes t = 0 .. L-2.
void host_mw_rings(int L, RingConsts *rc)
{
    const int nreg = L - 1;
    rc->theta.resize(nreg);
    rc->cot.resize(nreg);
    rc->csc.resize(nreg);
    rc->lsin.resize(2 * nreg);
    rc->lcos.resize(2 * nreg);
    for (int t = 0; t < nreg; ++t) {
        const q th = (2 * (q)t + 1) * QPI / (2 * (q)L - 1);
        fill_ring(rc, t, th);
    }
}

void fill_ring(RingConsts *rc, int r, __float128 th)
{
    const q s = sinq(th), c = cosq(th);
    rc->theta[r] = (double)th;
    rc->cot[r] = (double)(c / s);
    rc->csc[r] = (double)(1 / s);
    split_dd(log2q(sinq(th / 2)), &rc->lsin[2 * r], &rc->lsin[2 * r + 1]);
    split_dd(log2q(cosq(th / 2)), &rc->lcos[2 * r], &rc->lcos[2 * r + 1]);
}

// MWSS (Sec. 4.2): the swept rings theta = pi t / L, t = 1 .. L-1 (ring r = t - 1);
// the poles t = 0 and t = L are handled in closed form.
void host_mwss_rings(int L, RingConsts *rc)
{
    const int nreg = L - 1;
    rc->theta.resize(nreg);
    rc->cot.resize(nreg);
    rc->csc.resize(nreg);
    rc->lsin.resize(2 * nreg);
    rc->lcos.resize(2 * nreg);
    for (int r = 0; r < nreg; ++r) fill_ring(rc, r, QPI * (q)(r + 1) / (q)L);
}

// DH sampling theorem (Sec. 4.2): 2L rings theta_t = (2t+1) pi / (4L); the forward
// weight of ring t (the phi rule 2 pi / (2L-1) included) is
//   (4 pi / (L (2L-1))) sin(theta_t) sum_{k<L} sin((2k+1) theta_t) / (2k+1),
// the sines by the recurrence s_{k+1} = 2 cos(2 theta) s_k - s_{k-1} in quad precision.
void host_dh_rings(int L, RingConsts *rc, std::vector<double> *wq)
{
    const int nring = 2 * L;
    rc->theta.resize(nring);
    rc->cot.resize(nring);
    rc->csc.resize(nring);
    rc->lsin.resize(2 * nring);
    rc->lcos.resize(2 * nring);
    wq->resize(nring);
    for (int t = 0; t < nring; ++t) {
        const q th = (2 * (q)t + 1) * QPI / (4 * (q)L);
        fill_ring(rc, t, th);
        const q c2 = 2 * cosq(2 * th);
        q sm = -sinq(th), sk = sinq(th), acc = 0;            // sin(-theta), sin(theta)
        for (int k = 0; k < L; ++k) {
            acc += sk / (2 * (q)k + 1);
            const q sn = c2 * sk - sm;
            sm = sk;
            sk = sn;
        }
        (*wq)[t] = (double)(4 * QPI / ((q)L * (2 * (q)L - 1)) * sinq(th) * acc);
    }
}

// GL sampling theorem (Sec. 4.2): L rings with cos(theta_t) the roots of P_L (theta
// ascending), by Newton's method on the three-term Legendre recurrence in quad
// precision; forward weight (phi rule included) (2 pi / (2L-1)) 2 / ((1 - x^2) P_L'(x)^2).
void host_gl_rings(int L, RingConsts *rc, std::vector<double> *wq)
{
    rc->theta.resize(L);
    rc->cot.resize(L);
    rc->csc.resize(L);
    rc->lsin.resize(2 * L);
    rc->lcos.resize(2 * L);
    wq->resize(L);
    auto legendre = [L](q x, q *p, q *dp) {              // P_L(x) and P_L'(x)
        q p0 = 1, p1 = x;
        for (int k = 2; k <= L; ++k) {
            const q p2 = ((2 * (q)k - 1) * x * p1 - ((q)k - 1) * p0) / (q)k;
            p0 = p1;
            p1 = p2;
        }
        if (L == 1) { p1 = x; p0 = 1; }
        *p = p1;
        *dp = (q)L * (x * p1 - p0) / (x * x - 1);
    };
    for (int t = 0; t < L; ++t) {
        long double xl = cosl(3.14159265358979323846264338327950288L * (t + 0.75L) / (L + 0.5L));
        for (int it = 0; it < 60; ++it) {                  // long double Newton from the classical guess
            long double p0 = 1, p1 = xl;
            for (int k = 2; k <= L; ++k) {
                const long double p2 = ((2.0L * k - 1) * xl * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (L == 1) { p1 = xl; p0 = 1; }
            const long double dpl = L * (xl * p1 - p0) / (xl * xl - 1);
            const long double dx = p1 / dpl;
            xl -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        q x = xl, p, dp;
        for (int it = 0; it < 2; ++it) {                   // polish in quad precision
            legendre(x, &p, &dp);
            x -= p / dp;
        }
        legendre(x, &p, &dp);
        fill_ring(rc, t, acosq(x));
        (*wq)[t] = (double)(2 * QPI / (2 * (q)L - 1) * 2 / ((1 - x * x) * dp * dp));
    }
}

// HEALPix RING geometry (Gorski et al. 2005), ring r = 0 .. 4 nside - 2, i = r + 1:
//   i <  nside:          cos(theta) = 1 - i^2/(3 nside^2), 4i pixels, half-pixel shift
//   nside <= i <= 3nside: cos(theta) = 4/3 - 2i/(3 nside), 4 nside pixels,
//                         shift when (i - nside) is even
//   i > 3 nside:          mirror of ring 4 nside - i.
// Pixel j of ring r sits at phi = pi (2j + shift_r) / nphi_r.
void host_healpix_rings(int nside, RingConsts *rc, std::vector<int> *nphi,
                        std::vector<long long> *start, std::vector<int> *shift)
{
    const int nring = 4 * nside - 1;
    rc->theta.resize(nring);
    rc->cot.resize(nring);
    rc->csc.resize(nring);
    rc->lsin.resize(2 * nring);
    rc->lcos.resize(2 * nring);
    nphi->resize(nring);
    start->resize(nring);
    shift->resize(nring);
    long long pix = 0;
    const q ns = nside;
    for (int r = 0; r < nring; ++r) {
        const int i = r + 1;
        q th;
        int np, sh;
        if (i < nside) {
            th = 2 * asinq((q)i / (sqrtq((q)6) * ns));
            np = 4 * i;
            sh = 1;
        } else if (i <= 3 * nside) {
            th = acosq((q)4 / 3 - 2 * (q)i / (3 * ns));
            np = 4 * nside;
            sh = ((i - nside) % 2 == 0) ? 1 : 0;
        } else {
            const int ii = 4 * nside - i;
            th = QPI - 2 * asinq((q)ii / (sqrtq((q)6) * ns));
            np = 4 * ii;
            sh = 1;
        }
        fill_ring(rc, r, th);
        (*nphi)[r] = np;
        (*start)[r] = pix;
        (*shift)[r] = sh;
        pix += np;
    }
}

// 0.5 * log2 binom(2l, l - n) for l = |n| .. L-1 as double-double (zero below |n|).
void host_log2_binom(int L, int n, std::vector<double> *out)
{
    out->assign(2 * (size_t)L, 0.0);
    const int an = n < 0 ? -n : n;
    for (int l = an; l < L; ++l) {
        const q v = 0.5q * (lgammaq(2 * (q)l + 1) - lgammaq((q)(l - n) + 1) - lgammaq((q)(l + n) + 1)) / logq((q)2);
        split_dd(v, &(*out)[2 * l], &(*out)[2 * l + 1]);
    }
}

// Rescaled recursion.  With alpha_k = sqrt((l+k)(l-k+1)), Eq. 25 reads
//   alpha_m d_{m-1} = 2 lambda_m d_m - alpha_{m+1} d_{m+1}.
// Writing d_m = e_m g_m with g_l = g_{l-1} = 1, g_{m-1} = g_{m+1} alpha_{m+1}/alpha_m
// turns it into  e_{m-1} = kappa_m lambda_m e_m - e_{m+1},
//   kappa_m = 2 g_m / (alpha_m g_{m-1}).
// Tables are indexed by the order being produced: kap[m][l] = kappa_{m+1} (m < l),
// gtab[m][l] = g_m (m <= l).  Both [L][L], l fastest.  Long double: the even
// and odd g-chains accumulate ~1e-19 per step, and every product of consecutive
// kappas telescopes to exact alpha ratios, so no error drifts through the sweep.
// kappa / g tables of the rescaled recursion for orders m in [-nx, L): row (m + nx).
// The negative rows serve the continuation of a run past m = 0 (stable-direction
// remedy near the poles); entries outside the recursion's range are zero.
void host_recursion_tables(int L, int nx, std::vector<double> *kap, std::vector<double> *gtab)
{
    const size_t rows = (size_t)L + nx;
    kap->assign(rows * L, 0.0);
    gtab->assign(rows * L, 0.0);
    std::vector<long double> g(L + 2 + 2 * (size_t)nx);   // g[m + nx + 1], m in [-nx-1, l+1)
    for (int l = 0; l < L; ++l) {
        auto al = [l](int k) { return sqrtl((long double)(l + k) * (long double)(l - k + 1)); };
        auto G = [&](int m) -> long double & { return g[(size_t)(m + nx + 1)]; };
        G(l) = 1.0L;
        if (l >= 1) G(l - 1) = 1.0L;
        const int mlow = std::max(-nx, -l + 1);             // alpha_m > 0 for m > -l
        for (int m = l - 1; m >= mlow; --m) G(m - 1) = G(m + 1) * al(m + 1) / al(m);
        for (int m = std::max(-nx, -l); m <= l; ++m) (*gtab)[(size_t)(m + nx) * L + l] = (double)G(m);
        for (int m = std::max(-nx, -l); m < l; ++m) {
            const int mp = m + 1;   // kappa_{m+1} produces order m
            (*kap)[(size_t)(m + nx) * L + l] = (double)(2.0L * G(mp) / (al(mp) * G(mp - 1)));
        }
    }
}

// e^{-2 pi i k / n}, k < n, interleaved (long double evaluation of the reduced angle).
void host_roots(int n, std::vector<double> *out)
{
    out->resize(2 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < n; ++k) {
        const long double a = 2.0L * pi * (long double)k / (long double)n;
        (*out)[2 * k] = (double)cosl(a);
        (*out)[2 * k + 1] = -(double)sinl(a);
    }
}

// Bluestein chirp c_k = e^{i pi (k^2 mod 2n) / n}, k < n.
void host_chirp(int n, std::vector<double> *out)
{
    out->resize(2 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (long long k = 0; k < n; ++k) {
        const long long r = (k * k) % (2LL * n);
        const long double a = pi * (long double)r / (long double)n;
        (*out)[2 * k] = (double)cosl(a);
        (*out)[2 * k + 1] = (double)sinl(a);
    }
}

// MW theta filter constants for N = 2L-1 torus points theta_t = (2t+1) pi/N and
// midpoints mu_t = theta_t + pi/N:
//   wq[t], wq[N + t]  = P_{2L-2}[sin(theta) 1_[0,pi]] at theta_t and mu_t.  The
//       Fourier coefficients c_d = (1/2pi) int_0^pi sin(th) e^{-i d th} are
//       c_{+-1} = -+ i/4, c_d = 1/(pi (1 - d^2)) for even d, 0 for other odd d
//       (Eq. 42 up to the 2pi normalisation and the sign of d), so
//       P[...](th) = sin(th)/2 + c_0 + 2 sum_{even d >= 2} c_d cos(d th);
//   ph[k] = e^{i k' pi / N} / N for DFT bin k with signed frequency
//       k' = k (k <= L-1) or k - N (k >= L): the half-sample shift.
void host_mw_filter(int L, bool ss, std::vector<double> *wq, std::vector<double> *ph)
{
    const int N = ss ? 2 * L : 2 * L - 1;
    const long double pi = 3.141592653589793238462643383279502884L;
    wq->assign(2 * (size_t)N, 0.0);
    for (int which = 0; which < 2; ++which) {
        for (int t = 0; t < N; ++t) {
            // MW theta_t = (2t+1) pi/N, MWSS theta_t = 2t pi/N; midpoints one half-step on
            const long double th = (2.0L * t + (ss ? 0.0L : 1.0L) + which) * pi / (long double)N;
            long double acc = 1.0L / pi + 0.5L * sinl(th);
            const long double c2 = cosl(2.0L * th);
            long double cprev = 1.0L, ccur = c2;   // cos(0 th), cos(2 th)
            for (int d = 2; d <= 2 * L - 2; d += 2) {
                if ((d & 127) == 0) {                                   // re-anchor the recurrence
                    ccur = cosl((long double)d * th);
                    cprev = cosl((long double)(d - 2) * th);
                }
                acc += 2.0L / (pi * (1.0L - (long double)d * d)) * ccur;
                const long double cnext = 2.0L * c2 * ccur - cprev;
                cprev = ccur; ccur = cnext;
            }
            (*wq)[(size_t)which * N + t] = (double)acc;
        }
    }
    ph->resize(2 * (size_t)N);
    for (int k = 0; k < N; ++k) {
        const int ks = (k <= L - 1) ? k : k - N;
        const long double a = (long double)ks * pi / (long double)N;
        const bool nyquist = ss && k == L;                  // MWSS: the Nyquist frequency is left out
        (*ph)[2 * k] = nyquist ? 0.0 : (double)(cosl(a) / (long double)N);
        (*ph)[2 * k + 1] = nyquist ? 0.0 : (double)(sinl(a) / (long double)N);
    }
}

// Half-step shifts of the MW theta filter as convolutions.  The filter moves the
// torus samples g (length N = 2L - 1, band |k| < L) onto the midpoints and back:
// (S g)_t = sum_j c_{t-j} g_j with c_s = (1/N) sum_{|k|<L} e^{i pi k (2s+1)/N}, a
// Dirichlet sum equal to (-1)^s / (N sin(pi (2s+1) / (2N))), and the way back with
// c'_s = (1/N) sum_{|k|<L} e^{i pi k (2s-1)/N} = -(-1)^s / (N sin(pi (2s-1) / (2N)))
// (indices mod N).  Placed cyclically in M >= 2N - 1 points (e_{s mod M} = c_{s mod N}
// for |s| < N, zero elsewhere), an M-point cyclic convolution of g (zero past N) with e
// equals the circular one of length N at t < N, with no wrap-around.  out = the M-point
// spectra E_k = (1/M) sum_j e_j e^{-2 pi i j k / M} of the two kernels (S, then the way
// back), interleaved complex, each M entries; M a power of two.
static void fft_ld(std::vector<long double> &re, std::vector<long double> &im, int M)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 1, j = 0; i < M; ++i) {                   // bit reversal
        int bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j |= bit;
        if (i < j) { std::swap(re[i], re[j]); std::swap(im[i], im[j]); }
    }
    for (int len = 2; len <= M; len <<= 1) {
        const int h = len / 2;
        for (int k = 0; k < h; ++k) {
            const long double a = -2.0L * pi * (long double)k / (long double)len;
            const long double wr = cosl(a), wi = sinl(a);
            for (int b = 0; b < M; b += len) {
                const int u = b + k, v = u + h;
                const long double xr = re[v] * wr - im[v] * wi, xi = re[v] * wi + im[v] * wr;
                re[v] = re[u] - xr; im[v] = im[u] - xi;
                re[u] += xr; im[u] += xi;
            }
        }
    }
}

void host_shift_spectra(int L, int M, std::vector<double> *out)
{
    const int N = 2 * L - 1;
    const long double pi = 3.141592653589793238462643383279502884L;
    out->assign(4 * (size_t)M, 0.0);
    for (int which = 0; which < 2; ++which) {
        std::vector<long double> re(M, 0.0L), im(M, 0.0L);
        for (int d = -(N - 1); d <= N - 1; ++d) {
            const int s = (d % N + N) % N;                  // kernel index mod N
            const long double sg = (s & 1) ? -1.0L : 1.0L;
            re[(d % M + M) % M] = which == 0 ? sg / ((long double)N * sinl(pi * (2.0L * s + 1.0L) / (2.0L * N)))
                                             : -sg / ((long double)N * sinl(pi * (2.0L * s - 1.0L) / (2.0L * N)));
        }
        fft_ld(re, im, M);
        for (int k = 0; k < M; ++k) {
            (*out)[2 * ((size_t)which * M + k)] = (double)(re[k] / M);
            (*out)[2 * ((size_t)which * M + k) + 1] = (double)(im[k] / M);
        }
    }
}

// Per-l weights: SHT (-1)^s sqrt((2l+1)/4pi) (Eqs. 30, 33); SO(3) inverse
// (2l+1)/(8 pi^2) (Eq. 13); SO(3) forward 1 (Eq. 14).
void host_weights(int L, int kind, int spin, std::vector<double> *w)
{
    w->resize(L);
    for (int l = 0; l < L; ++l) {
        q v;
        if (kind == 0) {
            v = sqrtq((2 * (q)l + 1) / (4 * QPI));
            if ((spin < 0 ? -spin : spin) % 2) v = -v;
        } else if (kind == 1) {
            v = (2 * (q)l + 1) / (8 * QPI * QPI);
        } else {
            v = 1;
        }
        (*w)[l] = (double)v;
    }
}

}  // namespace s2mi
