// Host driver for the plan builder's constant tables under AddressSanitizer /
// UndefinedBehaviorSanitizer (test infrastructure, built by
// tests/test_host_sanitizers.py).  Besides running every table generator at small
// sizes it checks properties fixed by the mathematics:
//  - cot^2 + 1 = csc^2 on every ring of every sampling;
//  - the GL nodes integrate every Legendre polynomial of degree < 2L exactly
//    (sum of weights 2 over cos theta, after removing the phi rule 2 pi / (2L-1));
//  - the half-step shift spectra move each band-limited exponential e^{i k theta}
//    (|k| < L) on the MW theta-torus by exactly half a step, pi / (2L-1), when
//    applied as the M-point cyclic convolution the theta filter runs (result at
//    t < N).
// Prints "OK" and exits 0 on success.
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "s2mi_internal.h"

using namespace s2mi;
using cd = std::complex<double>;

static int fails = 0;
static void check(bool ok, const char *what)
{
    if (!ok) { std::printf("failed: %s\n", what); ++fails; }
}

static void check_rings(const RingConsts &rc, const char *what)
{
    for (size_t r = 0; r < rc.cot.size(); ++r) {
        const double c = rc.cot[r], s = rc.csc[r];
        check(std::fabs(c * c + 1.0 - s * s) <= 1e-12 * s * s, what);
    }
}

// naive DFT of length M, sign -1 forward / +1 inverse (unnormalised)
static std::vector<cd> dft(const std::vector<cd> &x, int sign)
{
    const int M = (int)x.size();
    std::vector<cd> y(M);
    for (int k = 0; k < M; ++k) {
        cd acc = 0.0;
        for (int j = 0; j < M; ++j) acc += x[j] * std::polar(1.0, sign * 2.0 * M_PI * ((long long)j * k % M) / M);
        y[k] = acc;
    }
    return y;
}

int main()
{
    {
        RingConsts rc;
        host_mw_rings(16, &rc);
        check_rings(rc, "MW rings");
        RingConsts rs;
        host_mwss_rings(16, &rs);
        check_rings(rs, "MWSS rings");
        RingConsts rd;
        std::vector<double> wd;
        host_dh_rings(16, &rd, &wd);
        check_rings(rd, "DH rings");
        check(wd.size() == 32, "DH weights size");
    }
    {
        const int L = 12;
        RingConsts rc;
        std::vector<double> wq;
        host_gl_rings(L, &rc, &wq);
        check_rings(rc, "GL rings");
        double sum = 0.0;
        for (double w : wq) sum += w / (2.0 * M_PI / (2 * L - 1));
        check(std::fabs(sum - 2.0) < 1e-13, "GL weights integrate 1 over cos theta");
    }
    {
        RingConsts rc;
        std::vector<int> nphi;
        std::vector<long long> start;
        std::vector<int> shift;
        host_healpix_rings(8, &rc, &nphi, &start, &shift);
        check_rings(rc, "HEALPix rings");
        long long tot = 0;
        for (int n : nphi) tot += n;
        check(tot == 12LL * 8 * 8, "HEALPix pixel count");
    }
    {
        std::vector<double> a, b, kap, g;
        host_log2_binom(16, 2, &a);
        host_log2_binom(16, -3, &b);
        host_recursion_tables(16, 3, &kap, &g);
        check(kap.size() == (size_t)(16 + 3) * 16 && g.size() == kap.size(), "recursion table sizes");
        std::vector<double> r, c, w;
        host_roots(12, &r);
        host_chirp(13, &c);
        for (int kind = 0; kind < 3; ++kind) host_weights(16, kind, -1, &w);
        std::vector<double> wq, ph;
        host_mw_filter(16, false, &wq, &ph);
        host_mw_filter(16, true, &wq, &ph);
    }
    {
        // half-step shifts as cyclic convolutions: L = 7, N = 13, M = 32 >= 2N - 1
        const int L = 7, N = 2 * L - 1, M = 32;
        std::vector<double> spec;
        host_shift_spectra(L, M, &spec);
        check(spec.size() == 4 * (size_t)M, "shift spectra size");
        for (int which = 0; which < 2; ++which) {
            std::vector<cd> E(M);
            for (int k = 0; k < M; ++k) E[k] = cd(spec[2 * ((size_t)which * M + k)], spec[2 * ((size_t)which * M + k) + 1]);
            double worst = 0.0;
            for (int kk = -(L - 1); kk <= L - 1; ++kk) {
                std::vector<cd> x(M, 0.0);
                for (int t = 0; t < N; ++t) x[t] = std::polar(1.0, 2.0 * M_PI * kk * t / N);
                std::vector<cd> X = dft(x, -1);
                for (int k = 0; k < M; ++k) X[k] *= E[k];
                std::vector<cd> y = dft(X, +1);
                const double step = which == 0 ? M_PI / N : -M_PI / N;   // S, then the way back
                for (int t = 0; t < N; ++t) {
                    const cd want = std::polar(1.0, 2.0 * M_PI * kk * t / N + kk * step);
                    worst = std::fmax(worst, std::abs(y[t] - want));
                }
            }
            check(worst < 1e-12, which == 0 ? "half-step shift" : "half-step shift back");
        }
    }
    if (fails) return 1;
    std::printf("OK\n");
    return 0;
}
