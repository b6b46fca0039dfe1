// s2mi_capi.hip -- the C ABI of include/s2mi.h: plan construction, argument
// validation and the launch sequence of each transform.
//
// Paper: Price & McEwen, arXiv 2311.14670.  Spin SHT = phi-DFT (Eqs. 31-32) +
// Wigner d-stage (Eqs. 30, 33) on an isolatitude sampling (Sec. 4.1-4.2);
// Wigner transform = gamma-DFT + one spin SHT per n (Sec. 4.5, Eqs. 15-18).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/s2mi.h"
#include "s2mi_internal.h"
#include "s2mi_kernels.h"
#include "s2mi_mfma.h"

using namespace s2mi;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hipfail(hipError_t e, const char *what)
{
    return fail(S2_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr, what)                      \
    do {                                        \
        hipError_t _e = (expr);                 \
        if (_e != hipSuccess) return hipfail(_e, what); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------------ plan
struct s2_plan_s {
    int L = 0, spin = 0, N = 1, sampling = 0, nside = 0, max_batch = 1, prec = 0;
    int nslice = 1;                       // 1 for S2, 2N-1 for SO(3)
    std::vector<int> slice_spin;          // spin of each slice (SO(3) slice k: n = k-(N-1), spin -n)
    int nring = 0, nreg = 0;              // rings of the sampling; rings the d-stage sweeps
    int nsw = 0;                          // rings the inverse sweep's lanes run (nreg, or the northern
                                          // half when mirror rings come from the symmetry)
    long long nsamp = 0;                  // samples per slice map
    std::vector<Run> runs;

    // device memory owned by the plan
    std::vector<void *> allocs;
    size_t plan_bytes = 0;

    // geometry (regular rings first; MW adds the south pole as ring nreg)
    double *cot = nullptr, *csc = nullptr, *lsin = nullptr, *lcos = nullptr;
    int *ring_nphi = nullptr, *ring_shift = nullptr, *ring_fft = nullptr;
    int *ring_pairs = nullptr;             // real signals: [npair][2] rings sharing one complex DFT (-1: none)
    int npair = 0;
    long long *ring_start = nullptr;
    // recursion tables
    double *kap = nullptr, *gtab = nullptr;
    std::vector<double *> lbin;   // per run
    std::vector<double *> lam;    // per run [L][hstride]
    std::vector<double2 *> init;  // per run [nreg][L]: start values of Eq. 27
    // per-slice weights: SHT (Eqs. 30, 33), SO(3) inverse (Eq. 13), SO(3) forward (Eq. 14)
    std::vector<double *> w_sht, w_so3i, w_so3f;
    double *w_so3f_n1 = nullptr;          // one-slice Wigner forward on the matrix cores: w_so3f times the gamma rule 2 pi
    std::vector<double *> w_fadj;         // HEALPix: (4 pi / Npix) w_l, the adjoint of the forward quadrature
    // FFT
    std::vector<FftArgs> ffts_h;
    FftArgs *ffts = nullptr;
    int fft_threads = 64;
    size_t fft_lds = 0;
    FftArgs fN{};                          // MW ring / theta-torus length 2L-1
    double *wq = nullptr, *ph = nullptr;   // MW theta filter
    int conv_idx = -1;                     // MW, 2L - 1 not 13-smooth: the filter's two shifts as cyclic
                                           // convolutions (FftArgs conv_idx and conv_idx + 1)
    double *ringq = nullptr;               // DH / GL: forward quadrature weight of each ring (phi rule included)
    double *groots = nullptr;              // e^{-2 pi i k/(2N-1)}
    // d-stage work assignment
    // stable-direction remedy: a run with n cos(theta) < 0 at a ring continues to
    // orders -(|n|-1) and supplies the other run's orders |m| < |n| there
    int nxp = 0;                           // max |n| over the runs (orders below it are remedied)
    int nx = 0;                            // negative orders held in the tables: max(0, nxp - 1)
    int inv_nblk = 1, inv_waves = 4;
    int *lslot = nullptr, *lchunk = nullptr, *mtop = nullptr;
    int fwd_nblk = 1, fwd_waves = 4, G = 1;
    // forward sweep over the northern rings (spin 0, symmetric samplings: nsw < nreg)
    bool fwd_pair = false;
    int fwdp_nblk = 1, fwdp_waves = 4, Gp = 1, pstride = 0;
    size_t off_Fp = 0;                    // workspace: sums and differences of mirror-ring spectra
    int hstride = 0;                       // ring stride of the forward spectra (padded to the sweep's slots)
    // order tiles of the FP64 sweeps and, per run, the recursion state at their cuts
    OrderTiles tiles{};
    std::vector<double *> ck;
    // workspace layout (bytes)
    size_t off_C = 0, off_P = 0, off_maps = 0, off_F = 0, off_Q = 0, off_hpole = 0, ws_bytes = 0;
    size_t off_fscr = 0, sz_fscr = 0;      // split-Bluestein scratch: FFT_SCRATCH complex per FFT workgroup
    size_t off_hsym = 0;                   // spin-0 S2 plans: Hermitian part of a coefficient cotangent
    size_t szC = 0, szP = 0, szF = 0, szQ = 0;
    size_t off_Hx = 0, off_Qx = 0, szHx = 0, szQx = 0;

    // matrix-core contraction path (precision FP32 / split BF16): batched over maps
    bool mfma = false;
    MfmaGeom mg{};
    int mch = 1;                           // orders per generated d chunk
    int gen_nblk = 1, gen_waves = 1;
    int *gen_lchunk = nullptr, *gen_mtop = nullptr, *mtop1 = nullptr;
    double2 *kg = nullptr;                 // [m][lrow] {kappa, g}
    size_t nslots = 0;                     // recursion state slots (l) of the generator
    size_t off_D = 0, off_S = 0, off_AH = 0, off_mP = 0, off_mF = 0, off_mQ = 0, off_mhp = 0, off_mmaps = 0;
    size_t off_mQx = 0;
    size_t state_bytes = 0;

    // stage timing
    bool timing = false;
    struct TimedLaunch { int stage; hipEvent_t a, b; };
    std::vector<TimedLaunch> tl;

    template <typename T>
    int dalloc(T **p, size_t count, const char *what)
    {
        void *q = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return fail(S2_ERR_OOM, "hipMalloc(%zu) for %s: %s", bytes, what, hipGetErrorString(e));
        allocs.push_back(q);
        plan_bytes += bytes;
        *p = static_cast<T *>(q);
        return S2_OK;
    }
    ~s2_plan_s()
    {
        for (auto &t : tl) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
        for (void *q : allocs) (void)hipFree(q);
    }
};

namespace {

// factor n over the engine radices; returns remainder (1 if fully factored)
int factor_radices(int n, std::vector<int> &rad)
{
    rad.clear();
    while (n % 8 == 0) { rad.push_back(8); n /= 8; }
    while (n % 4 == 0) { rad.push_back(4); n /= 4; }
    while (n % 2 == 0) { rad.push_back(2); n /= 2; }
    while (n % 9 == 0) { rad.push_back(9); n /= 9; }       // one stage instead of two radix-3 ones
    for (int p : {13, 11, 7, 5, 3})
        while (n % p == 0) { rad.push_back(p); n /= p; }
    return n;
}

// host staging kept alive until the plan's upload has completed (deque: references
// to earlier entries stay valid while later ones are added)
struct Staging {
    std::deque<std::vector<double>> d;
    std::deque<std::vector<int>> i;
    std::deque<std::vector<long long>> ll;
};

template <typename T>
int upload(s2_plan_s *P, T **dst, const std::vector<T> &src, hipStream_t st, const char *what)
{
    int rc = P->dalloc(dst, src.size(), what);
    if (rc) return rc;
    if (!src.empty()) HIPCHK(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st), what);
    return S2_OK;
}

int build_fft(s2_plan_s *P, int n, Staging &stg, hipStream_t st, FftArgs *out)
{
    FftArgs f{};
    std::vector<int> rad;
    const int rem = factor_radices(n, rad);
    f.n = n;
    if (rem == 1) {
        f.blue = 0;
        f.len = n;
    } else {
        f.blue = 1;
        int M = 1;
        while (M < 2 * n - 1) M *= 2;
        f.len = M;
        if (M > FFT_MAX_LEN && M / 2 <= FFT_MAX_LEN && n < M / 2) {
            f.split = 1;                                   // two LDS-resident halves of length M/2
            f.len = M / 2;
        }
        factor_radices(f.len, rad);
    }
    if (f.len > FFT_MAX_LEN)
        return fail(S2_ERR_UNSUPPORTED, "DFT length %d needs an engine of %d points (> %d)", n, f.len, FFT_MAX_LEN);
    if ((int)rad.size() > FFT_MAX_STAGES) return fail(S2_ERR_UNSUPPORTED, "too many FFT stages for %d", n);
    f.nst = (int)rad.size();
    for (int s = 0; s < f.nst; ++s) f.rad[s] = rad[s];
    stg.d.emplace_back();
    host_roots(f.len, &stg.d.back());
    double *tw;
    int rc = upload(P, &tw, stg.d.back(), st, "fft twiddles");
    if (rc) return rc;
    f.tw = tw;
    if (f.blue) {
        stg.d.emplace_back();
        host_chirp(n, &stg.d.back());
        double *ch, *bf;
        if ((rc = upload(P, &ch, stg.d.back(), st, "bluestein chirp"))) return rc;
        const int conv = f.split ? 2 * f.len : f.len;    // convolution length
        if ((rc = P->dalloc(&bf, 2 * (size_t)conv, "bluestein filter"))) return rc;
        f.chirp = ch;
        f.bflt = bf;
        if (f.split) {
            stg.d.emplace_back();
            host_roots(conv, &stg.d.back());
            stg.d.back().resize(2 * (size_t)f.len);       // e^{-2 pi i k/conv}, k < len
            double *wm;
            if ((rc = upload(P, &wm, stg.d.back(), st, "bluestein split roots"))) return rc;
            f.twm = wm;
        }
    }
    *out = f;
    return S2_OK;
}

int fft_threads_for(int len) { return std::min(1024, std::max(64, ((len / 8 + 63) / 64) * 64)); }

// Inverse d-stage: l is cut into chunks of 8 consecutive degrees; chunks are
// dealt in decreasing order of work (work of chunk c ~ c) over the (block,
// wave) bins in snake order, two per wave, so every wave's sum_l (l + 1) is
// balanced.  lchunk[bin] = {base of chunk A, base of chunk B} (or -1);
// lslot[bin][16] = the degree of each slot (slot j of a chunk: base + 7 - j),
// -1 where the chunk runs past L-1.
void assign_inverse(int L, int nblk, int W, int nchw, std::vector<int> &lchunk, std::vector<int> &lslot,
                    std::vector<int> &mtop)
{
    const int nbin = nblk * W;
    const int jw = 8 * nchw;
    const int nch = (L + 7) / 8;
    lchunk.assign((size_t)nbin * nchw, -1);
    lslot.assign((size_t)nbin * jw, -1);
    std::vector<int> fill(nbin, 0);
    for (int idx = 0, c = nch - 1; c >= 0; --c, ++idx) {
        const int round = idx / nbin, pos = idx % nbin;
        const int bin = (round % 2 == 0) ? pos : nbin - 1 - pos;
        const int g = fill[bin]++;
        lchunk[(size_t)bin * nchw + g] = 8 * c;
        for (int j = 0; j < 8; ++j) {
            const int l = 8 * c + 7 - j;
            lslot[(size_t)bin * jw + g * 8 + j] = l < L ? l : -1;
        }
    }
    mtop.assign(nblk, 0);
    for (int b = 0; b < nblk; ++b)
        for (int k = 0; k < W * jw; ++k) mtop[b] = std::max(mtop[b], lslot[(size_t)b * W * jw + k]);
}

}  // namespace

extern "C" {

const char *s2_error_string(int code)
{
    switch (code) {
    case S2_OK: return "ok";
    case S2_ERR_INVALID_ARG: return "invalid argument";
    case S2_ERR_UNSUPPORTED: return "unsupported";
    case S2_ERR_OOM: return "out of memory";
    case S2_ERR_HIP: return "HIP runtime error";
    case S2_ERR_CHECK: return "debug check failed";
    default: return "unknown error";
    }
}

const char *s2_last_error_message(void) { return g_last_error.c_str(); }

int s2_plan_info(s2_plan_t P, s2_plan_info_t *info)
{
    if (!P || !info) return fail(S2_ERR_INVALID_ARG, "s2_plan_info: null argument");
    info->L = P->L;
    info->spin = P->spin;
    info->N = P->N;
    info->nside = P->nside;
    info->sampling = P->sampling;
    info->precision = P->prec;
    info->max_batch = P->max_batch;
    info->nrings = P->nring;
    info->nsamples = P->nsamp;
    info->ncoeffs = (long long)P->L * (2 * P->L - 1);
    info->workspace_bytes = P->ws_bytes;
    info->plan_device_bytes = P->plan_bytes;
    info->swept_rings = P->nsw;
    info->order_tiles = P->ck.empty() ? 1 : P->tiles.nt;
    return S2_OK;
}

int s2_plan_destroy(s2_plan_t P)
{
    if (!P) return S2_OK;
    (void)hipDeviceSynchronize();
    delete P;
    return S2_OK;
}

static int plan_create_impl(s2_plan_t *out, int L, int spin, int N, s2_sampling_t sampling, int nside, int max_batch,
                            s2_precision_t prec, void *hip_stream)
{
    if (!out) return fail(S2_ERR_INVALID_ARG, "s2_plan_create: out is NULL");
    *out = nullptr;
    if (L < 2 || L > 4096) return fail(S2_ERR_INVALID_ARG, "L=%d outside [2, 4096]", L);
    if (N < 1 || N > L) return fail(S2_ERR_INVALID_ARG, "N=%d outside [1, L]", N);
    if (N > 8) return fail(S2_ERR_UNSUPPORTED, "N=%d: SO(3) plans support N <= 8", N);
    if (N > 1 && spin != 0) return fail(S2_ERR_INVALID_ARG, "SO(3) plans (N > 1) take spin 0");
    if (spin <= -L || spin >= L) return fail(S2_ERR_INVALID_ARG, "|spin|=%d must be < L=%d", spin, L);
    if (sampling != S2_MW && sampling != S2_HEALPIX && sampling != S2_DH && sampling != S2_GL && sampling != S2_MWSS)
        return fail(S2_ERR_INVALID_ARG, "unknown sampling %d", (int)sampling);
    if (sampling == S2_HEALPIX && (nside < 1 || nside > 2048)) return fail(S2_ERR_INVALID_ARG, "nside=%d outside [1, 2048]", nside);
    if (sampling != S2_MW && N > 1) return fail(S2_ERR_UNSUPPORTED, "SO(3) plans need MW sampling");
    if (sampling != S2_HEALPIX) nside = 0;
    if (max_batch < 1) return fail(S2_ERR_INVALID_ARG, "max_batch=%d < 1", max_batch);
    if (prec != S2_FP64 && prec != S2_CONTRACT_FP32 && prec != S2_CONTRACT_SPLIT_BF16)
        return fail(S2_ERR_INVALID_ARG, "unknown precision mode %d", (int)prec);
    hipStream_t st = (hipStream_t)hip_stream;

    s2_plan_s *P = new (std::nothrow) s2_plan_s();
    if (!P) return fail(S2_ERR_OOM, "host allocation of the plan failed");
    P->L = L; P->spin = spin; P->N = N; P->sampling = sampling; P->nside = nside; P->max_batch = max_batch; P->prec = prec;
    P->nslice = 2 * N - 1;
    const bool so3 = N > 1;
    Staging stg;
    int rc;
    auto bail = [&](int code) { delete P; return code; };
    // a HIP failure while the plan is built releases everything it holds
#define PLANCHK(expr, what)                                  \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return bail(hipfail(_e, what)); \
    } while (0)

    // slices and runs
    P->slice_spin.resize(P->nslice);
    if (!so3) P->slice_spin[0] = spin;
    else for (int k = 0; k < P->nslice; ++k) P->slice_spin[k] = -(k - (N - 1));
    auto slice_of_spin = [&](int s) {
        for (int k = 0; k < P->nslice; ++k) if (P->slice_spin[k] == s) return k;
        return -1;
    };
    {
        std::vector<int> ns;
        for (int k = 0; k < P->nslice; ++k) {
            const int s = P->slice_spin[k];
            for (int n : {-s, s}) if (std::find(ns.begin(), ns.end(), n) == ns.end()) ns.push_back(n);
        }
        for (int n : ns) P->runs.push_back(Run{n, slice_of_spin(-n), slice_of_spin(n)});
    }

    // geometry
    RingConsts rc_h;
    std::vector<int> nphi, shift;
    std::vector<long long> start;
    if (sampling == S2_MW) {
        host_mw_rings(L, &rc_h);
        P->nreg = L - 1;
        P->nring = L;
        nphi.assign(L, 2 * L - 1);
        shift.assign(L, 0);
        start.resize(L);
        for (int t = 0; t < L; ++t) start[t] = (long long)t * (2 * L - 1);
        P->nsamp = (long long)L * (2 * L - 1);
    } else if (sampling == S2_MWSS) {
        // rings 0 .. L-2: theta = pi (r+1)/L; ring L-1: south pole; ring L: north pole
        host_mwss_rings(L, &rc_h);
        P->nreg = L - 1;
        P->nring = L + 1;
        nphi.assign(L + 1, 2 * L);
        shift.assign(L + 1, 0);
        start.resize(L + 1);
        for (int r = 0; r < L - 1; ++r) start[r] = (long long)(r + 1) * 2 * L;
        start[L - 1] = (long long)L * 2 * L;
        start[L] = 0;
        P->nsamp = (long long)(L + 1) * 2 * L;
    } else if (sampling == S2_DH || sampling == S2_GL) {
        // equiangular-phi rings without poles, each ring swept; forward by quadrature
        stg.d.emplace_back(); std::vector<double> &rq = stg.d.back();
        if (sampling == S2_DH) host_dh_rings(L, &rc_h, &rq);
        else host_gl_rings(L, &rc_h, &rq);
        P->nring = (int)rq.size();
        P->nreg = P->nring;
        nphi.assign(P->nring, 2 * L - 1);
        shift.assign(P->nring, 0);
        start.resize(P->nring);
        for (int t = 0; t < P->nring; ++t) start[t] = (long long)t * (2 * L - 1);
        P->nsamp = (long long)P->nring * (2 * L - 1);
        if ((rc = upload(P, &P->ringq, rq, st, "ring weights"))) return bail(rc);
    } else {
        host_healpix_rings(nside, &rc_h, &nphi, &start, &shift);
        P->nring = 4 * nside - 1;
        P->nreg = P->nring;
        P->nsamp = 12LL * nside * nside;
    }
    if ((rc = upload(P, &P->cot, rc_h.cot, st, "cot"))) return bail(rc);
    if ((rc = upload(P, &P->csc, rc_h.csc, st, "csc"))) return bail(rc);
    if ((rc = upload(P, &P->lsin, rc_h.lsin, st, "lsin"))) return bail(rc);
    if ((rc = upload(P, &P->lcos, rc_h.lcos, st, "lcos"))) return bail(rc);
    if ((rc = upload(P, &P->ring_nphi, nphi, st, "ring_nphi"))) return bail(rc);
    if ((rc = upload(P, &P->ring_shift, shift, st, "ring_shift"))) return bail(rc);
    if ((rc = upload(P, &P->ring_start, start, st, "ring_start"))) return bail(rc);
    {
        // real signals: rings of equal length and phase offset pair up in ring order
        // (MW-type grids: (0,1), (2,3), ...; HEALPix: a cap ring with its mirror ring)
        stg.i.emplace_back();
        std::vector<int> &pr = stg.i.back();
        std::map<std::pair<int, int>, int> open_ring;
        for (int r = 0; r < P->nring; ++r) {
            const auto key = std::make_pair(nphi[r], shift[r]);
            auto it = open_ring.find(key);
            if (it == open_ring.end()) { open_ring[key] = r; continue; }
            pr.push_back(it->second);
            pr.push_back(r);
            open_ring.erase(it);
        }
        for (const auto &kv : open_ring) { pr.push_back(kv.second); pr.push_back(-1); }
        P->npair = (int)pr.size() / 2;
        if ((rc = upload(P, &P->ring_pairs, pr, st, "ring pairs"))) return bail(rc);
    }

    // FFTs: one per distinct ring length
    {
        std::vector<int> lens, rf(P->nring);
        for (int r = 0; r < P->nring; ++r) {
            auto it = std::find(lens.begin(), lens.end(), nphi[r]);
            if (it == lens.end()) { lens.push_back(nphi[r]); rf[r] = (int)lens.size() - 1; }
            else rf[r] = (int)(it - lens.begin());
        }
        int maxlen = 0;
        for (int n : lens) {
            FftArgs f;
            if ((rc = build_fft(P, n, stg, st, &f))) return bail(rc);
            P->ffts_h.push_back(f);
            maxlen = std::max(maxlen, f.len);
        }
        if (sampling == S2_MW || sampling == S2_MWSS) P->fN = P->ffts_h[0];
        // MW with a ring length N = 2L - 1 that needs Bluestein's identity: the theta
        // filter's two half-step shifts are circular convolutions of length N, each run
        // by the Bluestein driver as one cyclic convolution of the same length M (unit
        // chirp, the shift kernel's spectrum as the filter; two FFTs of M points, or four
        // of M/2 where the driver splits it) instead of two Bluestein DFTs
        if (sampling == S2_MW && P->fN.blue) {
            const int M = P->fN.split ? 2 * P->fN.len : P->fN.len;
            stg.d.emplace_back();
            host_shift_spectra(L, M, &stg.d.back());
            double *cs;
            if ((rc = upload(P, &cs, stg.d.back(), st, "theta filter shift spectra"))) return bail(rc);
            FftArgs f = P->fN;                             // same engine; its chirp is never applied
            f.conv = 1;
            P->conv_idx = (int)P->ffts_h.size();
            f.bflt = cs;
            P->ffts_h.push_back(f);
            f.bflt = cs + 2 * (size_t)M;
            P->ffts_h.push_back(f);
        }
        P->fft_threads = fft_threads_for(maxlen);
        P->fft_lds = (size_t)maxlen * sizeof(double2);
        if ((rc = upload(P, &P->ring_fft, rf, st, "ring_fft"))) return bail(rc);
        if ((rc = upload(P, &P->ffts, P->ffts_h, st, "fft table"))) return bail(rc);
        PLANCHK(set_kernel_lds_limits(P->fft_lds), "LDS limits");
        int nblue = 0;
        for (auto &f : P->ffts_h) nblue += f.blue;
        if (nblue) PLANCHK(launch_bluestein_filter(st, (int)P->ffts_h.size(), P->ffts, P->fft_threads, P->fft_lds), "bluestein filters");
    }
    if (sampling == S2_MW || sampling == S2_MWSS) {
        stg.d.emplace_back(); std::vector<double> &wq = stg.d.back();
        stg.d.emplace_back(); std::vector<double> &ph = stg.d.back();
        host_mw_filter(L, sampling == S2_MWSS, &wq, &ph);
        if ((rc = upload(P, &P->wq, wq, st, "mw filter weights"))) return bail(rc);
        if ((rc = upload(P, &P->ph, ph, st, "mw half-shift phases"))) return bail(rc);
    }
    if (sampling == S2_MW && spin == 0) {
        stg.d.emplace_back();
        host_roots(2 * N - 1, &stg.d.back());
        if ((rc = upload(P, &P->groots, stg.d.back(), st, "gamma roots"))) return bail(rc);
    }

    // recursion tables, rows m in [-nx, L) (device pointers at row m = 0)
    {
        for (const Run &r : P->runs) P->nxp = std::max(P->nxp, r.n < 0 ? -r.n : r.n);
        P->nx = std::max(0, P->nxp - 1);
        stg.d.emplace_back(); std::vector<double> &kap = stg.d.back();
        stg.d.emplace_back(); std::vector<double> &g = stg.d.back();
        host_recursion_tables(L, P->nx, &kap, &g);
        if ((rc = upload(P, &P->kap, kap, st, "kappa table"))) return bail(rc);
        if ((rc = upload(P, &P->gtab, g, st, "g table"))) return bail(rc);
        P->kap += (size_t)P->nx * L;
        P->gtab += (size_t)P->nx * L;
    }
    for (const Run &r : P->runs) {
        stg.d.emplace_back();
        host_log2_binom(L, r.n, &stg.d.back());
        double *lb;
        if ((rc = upload(P, &lb, stg.d.back(), st, "log2 binomials"))) return bail(rc);
        P->lbin.push_back(lb);
    }
    for (int k = 0; k < P->nslice; ++k) {
        for (int kind = 0; kind < 3; ++kind) {
            stg.d.emplace_back();
            host_weights(L, kind, P->slice_spin[k], &stg.d.back());
            double *a;
            if ((rc = upload(P, &a, stg.d.back(), st, "weights"))) return bail(rc);
            (kind == 0 ? P->w_sht : kind == 1 ? P->w_so3i : P->w_so3f).push_back(a);
        }
    }
    if (!so3 && sampling == S2_MW && spin == 0 && prec != S2_FP64) {
        // so3_forward with N = 1 on the matrix-core path folds the gamma rule 2 pi/(2N-1) = 2 pi
        // (Eq. 16) into the finish's weights instead of scaling a copy of the samples
        stg.d.emplace_back();
        host_weights(L, 2, 0, &stg.d.back());
        for (double &v : stg.d.back()) v *= 2.0 * M_PI;
        if ((rc = upload(P, &P->w_so3f_n1, stg.d.back(), st, "one-slice Wigner forward weights"))) return bail(rc);
    }

    // inverse d-stage assignment: waves of INV_NCH 8-degree chunks, W a multiple of 4.
    // Spin-0 plans of the N/S-symmetric samplings sweep only the northern rings and
    // produce each mirror ring from d^l_{m,0}(pi - theta) = (-1)^{l+m} d^l_{m,0}(theta),
    // when the halved grid still has a workgroup for every compute unit (splitting the
    // l-range over more blocks instead does not pay: the per-order reduction dominates
    // sparsely filled waves).
    {
        const int nch = (L + 7) / 8;
        const int per_blk = DSTAGE_MAX_WAVES * INV_NCH;
        P->inv_nblk = (nch + per_blk - 1) / per_blk;
        const int wneed = (nch + INV_NCH * P->inv_nblk - 1) / (INV_NCH * P->inv_nblk);
        P->inv_waves = std::min(DSTAGE_MAX_WAVES, std::max(4, (wneed + 3) / 4 * 4));
        // S2MI_RING_PAIRING=0 / 1 turns the mirror-ring sweep off / on wherever it applies
        // (tests, tuning); unset, the plan decides from the grid size.
        P->nsw = P->nreg;
        int dev = 0, ncu = 0;
        PLANCHK(hipGetDevice(&dev), "hipGetDevice");
        PLANCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
        const bool sym = sampling == S2_DH || sampling == S2_GL || sampling == S2_MWSS || sampling == S2_HEALPIX;
        const char *pm = std::getenv("S2MI_RING_PAIRING");
        const int mode = pm && pm[0] == '0' ? 0 : pm && pm[0] == '1' ? 1 : -1;
        if (sym && spin == 0 && !so3 && prec == S2_FP64 && mode != 0) {
            const int half_rings = (P->nreg + 1) / 2;
            if (mode == 1 || (half_rings + 63) / 64 * P->inv_nblk >= ncu) P->nsw = half_rings;
        }
        // Order tiles (FP64 sweeps; see OrderTiles): a grid of fewer than two waves per
        // SIMD is run as nt tiles aiming at four (more, shorter workgroups also even out
        // the tail), at most one per 64 orders (128 for the mirror-ring sweeps, whose
        // forward degree groups span 128).  Measured, MW L = 1024 spin 0: sweeps 0.90 +
        // 1.00 ms untiled, 0.46 + 0.58 ms in 8 tiles; at L = 2048, where the grid already
        // holds two waves per SIMD, 2 tiles made the forward sweep slower (3.05 -> 3.5 ms).
        // If the tiled grid still holds fewer than two waves per SIMD, four-wave
        // workgroups over twice the l-blocks (MW L = 512: inverse 0.206 -> 0.193 ms; at
        // L = 1024 in 8 tiles the eight-wave form is faster, 0.72 -> 0.46 ms, its l-blocks
        // writing half the partial sums).  S2MI_ORDER_TILES=k forces k tiles (1: none),
        // S2MI_INV_WAVES=4 / 8 the inverse workgroup size (tests, tuning).
        {
            const long long base = (long long)((P->nsw + 63) / 64) * P->inv_nblk * P->inv_waves;
            const long long two = 8LL * ncu, four = 16LL * ncu;
            const int q = P->nsw < P->nreg ? 128 : 64;
            int nt = base >= two ? 1 : (int)std::min<long long>(MAX_ORDER_TILES, (four + base - 1) / base);
            if (const char *ev = std::getenv("S2MI_ORDER_TILES"))
                nt = std::max(1, std::min(MAX_ORDER_TILES, std::atoi(ev)));
            if (prec != S2_FP64) nt = 1;                     // the matrix-core path has no FP64 sweeps
            nt = std::min(nt, std::max(1, L / q));
            P->tiles.nt = nt;
            const char *iw = std::getenv("S2MI_INV_WAVES");
            if (P->inv_waves == DSTAGE_MAX_WAVES && (iw ? iw[0] == '4' : base * nt < two)) {
                P->inv_waves = 4;
                P->inv_nblk *= 2;
            }
        }
        stg.i.emplace_back(); std::vector<int> &lch = stg.i.back();
        stg.i.emplace_back(); std::vector<int> &ls = stg.i.back();
        stg.i.emplace_back(); std::vector<int> &mt = stg.i.back();
        assign_inverse(L, P->inv_nblk, P->inv_waves, INV_NCH, lch, ls, mt);
        if ((rc = upload(P, &P->lchunk, lch, st, "inverse chunks"))) return bail(rc);
        if ((rc = upload(P, &P->lslot, ls, st, "inverse slots"))) return bail(rc);
        if ((rc = upload(P, &P->mtop, mt, st, "inverse mtop"))) return bail(rc);
    }
    // forward d-stage assignment: wave w of block b sweeps rings (b W + w) FWD_R ..
    // + FWD_R - 1; rings past the last regular ring are inert padding.  W is 4, 8
    // or 16 (rotating groups of four reducer waves); larger workgroups mean fewer
    // ring blocks and so fewer partial sums to write and add up in the finish.  At
    // most 16 ring blocks where the waves allow (MW L = 1024 in 8 order tiles: 32
    // blocks of 4 waves 0.62 ms, 16 blocks of 8 waves 0.58 ms, finish 0.15 -> 0.07 ms).
    {
        P->G = (L + 63) / 64;
        const int pairs = (P->G + 1) / 2;
        int nb = std::max(1, std::min({16, 256 / pairs, (P->nreg + 4 * FWD_R - 1) / (4 * FWD_R)}));
        int W = (P->nreg + nb * FWD_R - 1) / (nb * FWD_R);
        while (W > FWD_MAX_WAVES) { ++nb; W = (P->nreg + nb * FWD_R - 1) / (nb * FWD_R); }
        W = W <= 4 ? 4 : W <= 8 ? 8 : 16;                    // 1, 2 or 4 groups of four waves
        if (W > FWD_MAX_WAVES) W = FWD_MAX_WAVES;
        if (const char *fw = std::getenv("S2MI_FWD_WAVES")) {   // 4, 8 or 16 forced (tuning)
            const int Wf = std::atoi(fw);
            if (Wf == 4 || Wf == 8 || Wf == 16) {
                W = Wf;
                nb = (P->nreg + W * FWD_R - 1) / (W * FWD_R);
            }
        }
        P->fwd_nblk = nb;
        P->fwd_waves = W;
        P->hstride = std::max(nb * W * FWD_R, P->nring);
        // the mirror-ring form sweeps nsw rings with groups of 64 degrees of one parity
        // (Gp groups), on the same rule
        if (P->nsw < P->nreg) {
            P->fwd_pair = true;
            P->Gp = 2 * ((L + 127) / 128);
            const int pp = (P->Gp + 1) / 2;
            int nbp = std::max(1, std::min({16, 256 / pp, (P->nsw + 4 * FWD_R - 1) / (4 * FWD_R)}));
            int Wp = (P->nsw + nbp * FWD_R - 1) / (nbp * FWD_R);
            while (Wp > FWD_MAX_WAVES) { ++nbp; Wp = (P->nsw + nbp * FWD_R - 1) / (nbp * FWD_R); }
            Wp = Wp <= 4 ? 4 : Wp <= 8 ? 8 : 16;
            if (Wp > FWD_MAX_WAVES) Wp = FWD_MAX_WAVES;
            P->fwdp_nblk = nbp;
            P->fwdp_waves = Wp;
            P->pstride = nbp * Wp * FWD_R;
            P->hstride = std::max(P->hstride, P->pstride);  // the lambda table's columns cover every slot
        }
    }

    for (size_t ri = 0; ri < P->runs.size(); ++ri) {
        const Run &r = P->runs[ri];
        double *lam;
        double2 *ini;
        if ((rc = P->dalloc(&lam, (size_t)(L + P->nx) * P->hstride, "lambda table"))) return bail(rc);
        lam += (size_t)P->nx * P->hstride;                 // rows m in [-nx, L)
        PLANCHK(launch_lambda_table(st, L, P->nx, P->nreg, P->hstride, r.n, P->cot, P->csc, lam), "lambda table");
        if ((rc = P->dalloc(&ini, (size_t)L * P->nreg, "start values"))) return bail(rc);
        PLANCHK(launch_init_table(st, L, P->nreg, r.n, P->lsin, P->lcos, P->lbin[ri], ini), "start values");
        P->lam.push_back(lam);
        P->init.push_back(ini);
    }

    // order-tile cuts (tile count chosen with the inverse geometry above): tiles of about
    // equal work (the work above order m grows like (L - m)^2), cut at whole forward
    // degree groups, and per run the recursion state at each cut
    if (P->tiles.nt > 1) {
        const int q = P->fwd_pair ? 128 : 64;
        const int nt = P->tiles.nt;
        OrderTiles &ot = P->tiles;
        ot.c[0] = L;
        int k = 1;
        for (int j = 1; j < nt; ++j) {
            const double c = (double)L * (1.0 - std::sqrt((double)j / nt));
            int cq = (int)std::lround(c / q) * q;
            cq = std::max(q, std::min(cq, (L - 1) / q * q));
            if (cq < ot.c[k - 1]) ot.c[k++] = cq;
        }
        ot.nt = k;
        ot.rp = (P->nreg + 63) / 64 * 64;
        size_t tot = 0;
        for (int j = 1; j < ot.nt; ++j) {
            ot.off[j] = (long long)tot;
            tot += (size_t)(L - ot.c[j]) * 3 * ot.rp;
        }
        for (size_t ri = 0; ri < P->runs.size() && ot.nt > 1; ++ri) {
            double *ck;
            if ((rc = P->dalloc(&ck, tot, "order-tile states"))) return bail(rc);
            PLANCHK(launch_order_ckpt(st, L, P->nreg, P->runs[ri].n, P->cot, P->csc, P->init[ri], P->kap, ot, ck),
                    "order-tile states");
            P->ck.push_back(ck);
        }
    }

    // S2MI_DEBUG_CHECKS=1: check sum_{|m| <= l} (d^l_{m,n})^2 = 1 (d^l is orthogonal) on
    // sampled rings, for every degree and every run whose partner -n is in the plan,
    // with the same start values, tables and stable-direction continuation as the
    // sweeps; a violation fails the plan (S2_ERR_CHECK).  S2MI_DEBUG_CHECKS_TOL sets
    // the tolerance on |sum - 1| (default 1e-10).
    if (const char *dc = std::getenv("S2MI_DEBUG_CHECKS"); dc && dc[0] == '1' && P->nreg > 0) {
        const int nreg = P->nreg;
        std::vector<int> rs = {0, 1, nreg / 8, nreg / 4, nreg / 2, (3 * nreg) / 4, nreg - 2, nreg - 1};
        std::sort(rs.begin(), rs.end());
        rs.erase(std::unique(rs.begin(), rs.end()), rs.end());
        rs.erase(std::remove_if(rs.begin(), rs.end(), [&](int r) { return r < 0 || r >= nreg; }), rs.end());
        const int nsel = (int)rs.size();
        double tol = 1e-10;
        if (const char *tv = std::getenv("S2MI_DEBUG_CHECKS_TOL")) tol = std::atof(tv);
        int *rsel = nullptr;
        double *sums = nullptr;
        if ((rc = upload(P, &rsel, rs, st, "check rings"))) return bail(rc);
        const size_t per_run = (size_t)nsel * L * 2;
        if ((rc = P->dalloc(&sums, per_run * P->runs.size(), "check sums"))) return bail(rc);
        for (size_t ri = 0; ri < P->runs.size(); ++ri)
            PLANCHK(launch_unitarity(st, L, P->runs[ri].n, nsel, rsel, P->cot, P->csc, P->lsin, P->lcos, P->lbin[ri],
                                     P->kap, P->gtab, sums + ri * per_run),
                    "unitarity check");
        std::vector<double> h(per_run * P->runs.size());
        PLANCHK(hipMemcpyAsync(h.data(), sums, h.size() * sizeof(double), hipMemcpyDeviceToHost, st), "check copy");
        PLANCHK(hipStreamSynchronize(st), "check sync");
        for (size_t ri = 0; ri < P->runs.size(); ++ri) {
            const int n = P->runs[ri].n, an = n < 0 ? -n : n;
            int rj = -1;
            for (size_t k = 0; k < P->runs.size(); ++k)
                if (P->runs[k].n == -n) rj = (int)k;
            if (rj < 0) continue;
            const double *a = h.data() + ri * per_run, *b = h.data() + rj * per_run;
            for (int i = 0; i < nsel; ++i)
                for (int l = an; l < L; ++l) {
                    const size_t o = ((size_t)i * L + l) * 2;
                    // m >= 0 from run n, m < 0 from run -n at -m > 0
                    const double sum = a[o] + b[o] - b[o + 1] * b[o + 1];
                    if (!(std::fabs(sum - 1.0) <= tol))
                        return bail(fail(S2_ERR_CHECK,
                                         "debug check: sum over |m| <= l of d^l_{m,n}(theta)^2 = %.17g at l = %d, "
                                         "n = %d, ring %d (tolerance %g)", sum, l, n, rs[i], tol));
                }
        }
    }

    // workspace layout
    {
        const size_t S = P->nslice;
        P->szC = (size_t)P->inv_nblk * P->inv_waves * INV_J * (L + P->nx) * 5 * sizeof(double);
        P->szP = (size_t)P->inv_nblk * P->nreg * L * 4 * sizeof(double);
        P->szF = (size_t)L * P->hstride * 4 * sizeof(double);
        // forward partials [blk][l][m][4]; the adjoint of the MW / MWSS forward reuses the
        // buffer for ring partials [nring][m][4] (nring = L + 1 for MWSS)
        const int adj_rows = (sampling == S2_MW || sampling == S2_MWSS) ? P->nring : 0;
        P->szQ = (size_t)std::max({P->fwd_nblk * L, P->fwdp_nblk * L, adj_rows}) * L * 4 * sizeof(double);
        size_t o = 0;
        P->off_C = o; o += align256(P->szC * P->runs.size());
        P->off_P = o; o += align256(P->szP * S);
        P->off_maps = o; o += (sampling == S2_MW && spin == 0) ? align256((size_t)P->nsamp * S * sizeof(double2)) : 0;
        P->off_F = o; o += align256(P->szF * S);
        P->off_Q = o; o += align256(P->szQ * S);
        P->off_hpole = o; o += align256((size_t)(2 * L - 1) * S * 2 * sizeof(double2));   // south, north
        // low-order machinery of runs with n != 0: masked spectra copies per run, continuation sums per slice
        P->szHx = (size_t)std::max(P->nxp, 1) * P->hstride * 4 * sizeof(double);
        P->szQx = (size_t)P->fwd_nblk * L * std::max(P->nxp, 1) * 4 * sizeof(double);
        P->off_Hx = o; o += P->nxp > 0 ? align256(2 * P->szHx * P->runs.size()) : 0;
        P->off_Qx = o; o += P->nxp > 0 ? align256(P->szQx * S) : 0;
        bool split = false;
        for (const FftArgs &f : P->ffts_h) split = split || (f.blue && f.split);
        // one FFT_SCRATCH slice per workgroup of the phi-DFT (hstride), inverse phi-DFT
        // (nring) and MW filter (L) launches
        P->sz_fscr = split ? (size_t)std::max({P->hstride, P->nring, L}) * FFT_SCRATCH * sizeof(double2) : 0;
        P->off_fscr = o; o += align256(P->sz_fscr);
        P->off_hsym = o; o += (spin == 0 && !so3) ? align256((size_t)L * (2 * L - 1) * sizeof(double2)) : 0;
        P->off_Fp = o; o += P->fwd_pair ? align256(2 * (size_t)L * P->pstride * 4 * sizeof(double)) : 0;
        P->ws_bytes = o;
    }

    {
        stg.i.emplace_back(1, L - 1);
        if ((rc = upload(P, &P->mtop1, stg.i.back(), st, "single-block mtop"))) return bail(rc);
    }
    // HEALPix forward = q x adjoint of the inverse, so its adjoint is the inverse with weights q w_l;
    // DH / GL: the inverse with weights w_l, then each ring scaled by its quadrature weight
    if (sampling != S2_MW && sampling != S2_MWSS && !so3) {
        stg.d.emplace_back();
        host_weights(L, 0, spin, &stg.d.back());
        if (sampling == S2_HEALPIX)
            for (double &v : stg.d.back()) v *= 4.0 * M_PI / (double)P->nsamp;
        double *a;
        if ((rc = upload(P, &a, stg.d.back(), st, "forward-adjoint weights"))) return bail(rc);
        P->w_fadj.push_back(a);
    }

    // matrix-core path: generator assignment, {kappa, g} table, batched workspace
    if (prec != S2_FP64) {
        P->mfma = true;
        MfmaGeom &g = P->mg;
        g.L = L;
        g.nreg = P->nreg;
        g.rpad = (P->nreg + 63) / 64 * 64;
        g.lp = (L + 63) / 64 * 64;
        g.kc = (L + 7) / 8;
        g.lrow = 8 * g.kc;
        g.rows = (4 * max_batch + 31) / 32 * 32;
        {
            const int nch = g.kc;
            const int per_blk = DSTAGE_MAX_WAVES * GEN_NCH;
            P->gen_nblk = (nch + per_blk - 1) / per_blk;
            P->gen_waves = std::max(1, (nch + GEN_NCH * P->gen_nblk - 1) / (GEN_NCH * P->gen_nblk));
            stg.i.emplace_back(); std::vector<int> &lch = stg.i.back();
            stg.i.emplace_back(); std::vector<int> &ls = stg.i.back();
            stg.i.emplace_back(); std::vector<int> &mt = stg.i.back();
            assign_inverse(L, P->gen_nblk, P->gen_waves, GEN_NCH, lch, ls, mt);
            if ((rc = upload(P, &P->gen_lchunk, lch, st, "generator chunks"))) return bail(rc);
            if ((rc = upload(P, &P->gen_mtop, mt, st, "generator mtop"))) return bail(rc);
            P->nslots = (size_t)P->gen_nblk * P->gen_waves * GEN_NCH * 8;
        }
        if ((rc = P->dalloc(&P->kg, (size_t)(L + P->nx) * g.lrow, "kappa/g table"))) return bail(rc);
        P->kg += (size_t)P->nx * g.lrow;                     // rows m in [-nx, L)
        PLANCHK(launch_kg_table(st, L, P->nx, g.lrow, P->kap, P->gtab, P->kg), "kappa/g table");
        const size_t per_m_d = std::max((size_t)g.kc * g.rpad, (size_t)(g.rpad / 8) * g.lp) * 32;
        // up to 4 GiB of staged D (256 orders at L = 2048): larger chunks mean fewer, larger
        // generator and product launches (64 maps at L = 2048, FP32 pair: 32 orders per
        // chunk 145 ms, 64: 130 ms, 128: 123 ms, 256: 119 ms; split BF16 115 -> 101 ms)
        P->mch = (int)std::max<size_t>(4, std::min<size_t>((size_t)L, ((size_t)4 << 30) / per_m_d));
        // S2MI_MFMA_ORDER_CHUNK=k stages k orders of D per generator launch instead (tests: the
        // recursion state carried across order chunks at small L; results do not depend on it)
        if (const char *mc = std::getenv("S2MI_MFMA_ORDER_CHUNK")) {
            const int k = std::atoi(mc);
            if (k > 0) P->mch = std::min(L, k);
        }
        const size_t per_m_ah = (size_t)std::max(g.kc, g.rpad / 8) * g.rows * 32;
        const size_t S = P->nslice, B = max_batch;
        const size_t nP1 = (size_t)P->nreg * L * 4, nQ1 = (size_t)L * L * 4;
        P->state_bytes = P->nslots * g.rpad * (2 * sizeof(double) + sizeof(int));
        size_t o = P->ws_bytes;
        P->off_D = o; o += align256(per_m_d * P->mch);
        P->off_S = o; o += align256(P->state_bytes);
        P->off_AH = o; o += align256(per_m_ah * P->mch);
        P->off_mP = o; o += align256(B * S * nP1 * sizeof(double));
        P->off_mF = o; o += align256(B * S * P->szF);
        P->off_mQ = o; o += align256(B * S * nQ1 * sizeof(double));
        P->off_mhp = o; o += align256(B * S * (2 * L - 1) * 2 * sizeof(double2));        // south, north
        P->off_mmaps = o; o += (S > 1) ? align256(B * S * (size_t)P->nsamp * sizeof(double2)) : 0;
        P->off_mQx = o; o += P->nxp > 0 ? align256(B * S * (size_t)L * P->nxp * 4 * sizeof(double)) : 0;
        P->ws_bytes = o;
    }
    PLANCHK(hipStreamSynchronize(st), "plan upload");
    PLANCHK(hipGetLastError(), "plan kernels");
    *out = P;
    return S2_OK;
}
#undef PLANCHK

int s2_plan_create(s2_plan_t *out, int L, int spin, int N, s2_sampling_t sampling, int nside, int max_batch,
                   s2_precision_t prec, void *hip_stream)
{
    try {
        return plan_create_impl(out, L, spin, N, sampling, nside, max_batch, prec, hip_stream);
    } catch (const std::bad_alloc &) {
        return fail(S2_ERR_OOM, "host allocation failed during plan creation");
    } catch (...) {
        return fail(S2_ERR_HIP, "unexpected exception during plan creation");
    }
}

}  // extern "C"

// ------------------------------------------------------------------ transforms
namespace {

// Bracket one launch with events when the plan records stage timing.
// Set for the duration of a call that must not allocate (s2_inverse_noalloc):
// event creation and the timing record are skipped.
thread_local bool g_no_timing = false;

struct StageTimer {
    s2_plan_t P;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(s2_plan_t P_, int stage_, hipStream_t st_) : P(P_), stage(stage_), st(st_)
    {
        if (P->timing && !g_no_timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, st);
    }
    ~StageTimer()
    {
        if (a && b) {
            (void)hipEventRecord(b, st);
            P->tl.push_back({stage, a, b});
        }
    }
};
#define S2_CAT2(a, b) a##b
#define S2_CAT(a, b) S2_CAT2(a, b)
#define TIMED(stage) StageTimer S2_CAT(_timer_, __LINE__)(P, stage, st)

int check_call(const char *fn, s2_plan_t P, const void *in, const void *out, int batch, void *ws)
{
    if (!P) return fail(S2_ERR_INVALID_ARG, "%s: plan is NULL", fn);
    if (batch == 0) return S2_OK;                 // an empty batch: nothing is read or written
    if (!in || !out) return fail(S2_ERR_INVALID_ARG, "%s: NULL data pointer", fn);
    if (!ws) return fail(S2_ERR_INVALID_ARG, "%s: NULL workspace", fn);
    if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(S2_ERR_INVALID_ARG, "%s: data pointers must be 16-byte aligned", fn);
    if ((uintptr_t)ws & 255) return fail(S2_ERR_INVALID_ARG, "%s: workspace must be 256-byte aligned", fn);
    if (batch < 0 || batch > P->max_batch)
        return fail(S2_ERR_INVALID_ARG, "%s: batch=%d outside [0, max_batch=%d]", fn, batch, P->max_batch);
    return S2_OK;
}

// the order tiles of run ri (one tile where the plan has no state tables)
OrderTiles run_tiles(const s2_plan_s *P, size_t ri)
{
    OrderTiles ot = P->tiles;
    if (ri < P->ck.size()) ot.ck = P->ck[ri];
    else ot.nt = 1;
    return ot;
}

// the theta filter's convolution form: its FFT, kernel spectra and length (none: nullptr)
#define CONV_ARGS(P) ((P)->conv_idx >= 0 ? (P)->ffts + (P)->conv_idx : nullptr)

// the workspace's split-Bluestein scratch (nullptr when no DFT of the plan needs it)
double2 *fft_scratch(const s2_plan_s *P, char *ws)
{
    return P->sz_fscr ? reinterpret_cast<double2 *>(ws + P->off_fscr) : nullptr;
}

// inverse d-stage of one (map, all slices): flm slices [S][L][2L-1] -> partials P[slice][blk][ring][m][4]
// (half: real signal of a spin-0 plan, orders m >= 0 and components 0,1 only)
int run_inverse_dstage(s2_plan_t P, const double2 *flm, const std::vector<double *> &wl, char *ws, hipStream_t st,
                       int half = 0)
{
    const int L = P->L;
    const size_t slab = (size_t)L * (2 * L - 1);
    double *C0 = (double *)(ws + P->off_C);
    double *P0 = (double *)(ws + P->off_P);
    const size_t nP = P->szP / sizeof(double), nC = P->szC / sizeof(double);
    for (size_t ri = 0; ri < P->runs.size(); ++ri) {
        const Run &r = P->runs[ri];
        const double2 *fa = r.sliceA >= 0 ? flm + r.sliceA * slab : nullptr;
        const double2 *fb = r.sliceB >= 0 ? flm + r.sliceB * slab : nullptr;
        // a run that feeds one side only (spin-s sphere plans) sweeps that side alone
        const int side = half ? 1 : (fa && fb) ? 0 : (fa ? 1 : 2);
        double *C = C0 + ri * nC;
        {
        TIMED(S2_STAGE_PACK);
        HIPCHK(launch_pack_inv(st, L, P->nx, r.n, P->inv_nblk, P->inv_waves * INV_J, P->lslot, fa, fb,
                               r.sliceA >= 0 ? wl[r.sliceA] : nullptr, r.sliceB >= 0 ? wl[r.sliceB] : nullptr, P->kap,
                               P->gtab, C, side), "pack");
        }
        TIMED(S2_STAGE_DSTAGE_INV);
        HIPCHK(launch_dstage_inv(st, P->inv_waves, P->inv_nblk, L, P->nx, P->nreg, r.n, P->cot, P->csc, P->init[ri], C,
                                 P->lchunk, P->mtop,
                                 r.sliceA >= 0 ? P0 + r.sliceA * nP : nullptr,
                                 r.sliceB >= 0 ? P0 + r.sliceB * nP : nullptr, side, P->nsw, run_tiles(P, ri)),
               "inverse d-stage");
    }
    return S2_OK;
}

// inverse of one (map, all slices): flm slices [S][L][2L-1] -> slice maps
int run_inverse(s2_plan_t P, const double2 *flm, double2 *const *slice_maps, const std::vector<double *> &wl,
                char *ws, hipStream_t st)
{
    const int L = P->L;
    const size_t slab = (size_t)L * (2 * L - 1);
    double *P0 = (double *)(ws + P->off_P);
    const size_t nP = P->szP / sizeof(double);
    int rc = run_inverse_dstage(P, flm, wl, ws, st);
    if (rc) return rc;
    for (int k = 0; k < P->nslice; ++k) {
        TIMED(S2_STAGE_PHI_INV);
        HIPCHK(launch_phi_inv(st, P->fft_threads, P->fft_lds, P->nring, L, P->nreg, P->inv_nblk, P->slice_spin[k],
                              P0 + k * nP, P->mtop, flm + k * slab, wl[k], P->ring_nphi, P->ring_start,
                              P->ring_shift, P->ring_fft, P->ffts, slice_maps[k], fft_scratch(P, ws)), "inverse phi-DFT");
    }
    return S2_OK;
}

// adjoint of the MW / MWSS forward of one map, all slices (finish weights wl[k],
// spin slice_spin[k]): coefficient cotangent slices -> slice maps.  The slices
// share one gather / filter / scatter buffer in turn.  MWSS adds the north-pole
// row and runs the adjoint form of its theta filter.
int run_forward_adjoint_mw(s2_plan_t P, const double2 *G, double2 *const *slice_maps,
                           const std::vector<double *> &wl, char *ws, hipStream_t st)
{
    const int L = P->L;
    const int ss = P->sampling == S2_MWSS;
    const size_t slab = (size_t)L * (2 * L - 1);
    int rc = run_inverse_dstage(P, G, wl, ws, st);
    if (rc) return rc;
    double *P0 = (double *)(ws + P->off_P);
    const size_t nP = P->szP / sizeof(double);
    double *F0 = (double *)(ws + P->off_F);
    double2 *hp0 = (double2 *)(ws + P->off_hpole);
    double2 *hpN0 = ss ? hp0 + (size_t)P->nslice * (2 * L - 1) : nullptr;
    double *Q0 = (double *)(ws + P->off_Q);
    const double q = 2.0 * M_PI / (double)(ss ? 2 * L : 2 * L - 1);
    for (int k = 0; k < P->nslice; ++k) {
        const int s = P->slice_spin[k];
        const double2 *Gk = G + k * slab;
        {
        TIMED(S2_STAGE_MW_THETA);
        HIPCHK(launch_fadj_gather(st, L, ss, P->inv_nblk, s, P0 + k * nP, P->mtop, Gk, wl[k], P->hstride, F0),
               "adjoint gather");
        HIPCHK(launch_mw_filter(st, P->fft_threads, P->fft_lds, L, ss, P->hstride, s, P->ffts, P->wq, P->ph, F0, hp0,
                                hpN0, fft_scratch(P, ws), 0, 1, CONV_ARGS(P)), "adjoint theta filter");
        HIPCHK(launch_fadj_scatter(st, L, ss, P->hstride, q, F0, hp0, hpN0, Q0), "adjoint scatter");
        }
        TIMED(S2_STAGE_PHI_INV);
        HIPCHK(launch_phi_inv(st, P->fft_threads, P->fft_lds, P->nring, L, P->nring, 1, s, Q0, P->mtop1, Gk, wl[k],
                              P->ring_nphi, P->ring_start, P->ring_shift, P->ring_fft, P->ffts, slice_maps[k],
                              fft_scratch(P, ws)), "adjoint phi-DFT");
    }
    return S2_OK;
}

// forward d-stage of one map from the filtered ring spectra H (slices) -> flm slices
int run_forward_dstage(s2_plan_t P, double *H0, const double2 *hpole0, const double2 *hpoleN0, double2 *flm,
                       const std::vector<double *> &wl,
                       char *ws, hipStream_t st, int half = 0)
{
    const int L = P->L;
    const size_t slab = (size_t)L * (2 * L - 1);
    const size_t nF = P->szF / sizeof(double), nQ = P->szQ / sizeof(double);
    const size_t nHx = P->szHx / sizeof(double), nQx = P->szQx / sizeof(double);
    double *Q0 = (double *)(ws + P->off_Q);
    double *Hx0 = P->nxp > 0 ? (double *)(ws + P->off_Hx) : nullptr;
    double *Qx0 = P->nxp > 0 ? (double *)(ws + P->off_Qx) : nullptr;
    if (Qx0) HIPCHK(launch_zero(st, Qx0, P->szQx * P->nslice), "continuation sums clear");
    if (P->fwd_pair) {
        // spin-0 S2 plan (one slice, run n = 0): sweep the northern rings on the sums and
        // differences of each ring's and its mirror's spectra
        double *S = (double *)(ws + P->off_Fp);
        double *D = S + (size_t)L * P->pstride * 4;
        TIMED(S2_STAGE_DSTAGE_FWD);
        HIPCHK(launch_pair_spectra(st, L, P->nreg, P->nsw, P->hstride, P->pstride, H0, S, D), "mirror spectra");
        HIPCHK(launch_dstage_fwd(st, P->fwdp_waves, P->fwdp_nblk, P->Gp, L, 1, P->nsw, P->pstride, P->hstride, 0,
                                 P->lam[0], P->init[0], P->kap, P->gtab, S, D, nullptr, nullptr, Q0, Q0, nullptr,
                                 nullptr, half, 1, run_tiles(P, 0)), "forward d-stage");
    }
    for (size_t ri = 0; ri < P->runs.size() && !P->fwd_pair; ++ri) {
        const Run &r = P->runs[ri];
        const int an = r.n < 0 ? -r.n : r.n;
        const double *HA = r.sliceA >= 0 ? H0 + r.sliceA * nF : H0 + r.sliceB * nF;
        const double *HB = r.sliceB >= 0 ? H0 + r.sliceB * nF : HA;
        double *HxA = an > 0 ? Hx0 + 2 * ri * nHx : nullptr;
        double *HxB = an > 0 ? HxA + nHx : nullptr;
        const int side = half ? 1 : (r.sliceA >= 0 && r.sliceB >= 0) ? 0 : (r.sliceA >= 0 ? 1 : 2);
        TIMED(S2_STAGE_DSTAGE_FWD);
        if (an > 0)
            HIPCHK(launch_mask_low(st, an, r.n, P->nreg, P->hstride, P->cot, P->csc, HA, HB, HxA, HxB),
                   "low-order spectra");
        HIPCHK(launch_dstage_fwd(st, P->fwd_waves, P->fwd_nblk, P->G, L, std::max(P->nxp, 1), P->nreg, P->hstride,
                                 P->hstride, r.n, P->lam[ri], P->init[ri], P->kap, P->gtab, HA, HB, HxA, HxB,
                                 r.sliceA >= 0 ? Q0 + r.sliceA * nQ : nullptr,
                                 r.sliceB >= 0 ? Q0 + r.sliceB * nQ : nullptr,
                                 (an > 0 && r.sliceA >= 0) ? Qx0 + r.sliceA * nQx : nullptr,
                                 (an > 0 && r.sliceB >= 0) ? Qx0 + r.sliceB * nQx : nullptr, side, 0,
                                 run_tiles(P, ri)), "forward d-stage");
    }
    for (int k = 0; k < P->nslice; ++k) {
        const int s = P->slice_spin[k];
        TIMED(S2_STAGE_FINISH);
        HIPCHK(launch_finish_fwd(st, L, P->fwd_pair ? P->fwdp_nblk : P->fwd_nblk, s, s, Q0 + k * nQ,
                                 Qx0 ? Qx0 + k * nQx : nullptr,
                                 std::max(P->nxp, 1), wl[k], hpole0 ? hpole0 + k * (2 * L - 1) : nullptr,
                                 hpoleN0 ? hpoleN0 + k * (2 * L - 1) : nullptr, flm + k * slab, half),
               "forward finish");
    }
    return S2_OK;
}

// forward of one map: slice maps -> flm slices.  adjoint: unit phi weight, no theta filter.
int run_forward(s2_plan_t P, const double2 *const *slice_maps, double2 *flm, const std::vector<double *> &wl,
                char *ws, hipStream_t st, bool adjoint)
{
    const int L = P->L;
    const size_t nF = P->szF / sizeof(double);
    double *F0 = (double *)(ws + P->off_F);
    double2 *hp0 = (double2 *)(ws + P->off_hpole);
    const bool mw = P->sampling == S2_MW || P->sampling == S2_MWSS;   // theta-torus samplings
    const int ss = P->sampling == S2_MWSS;
    double2 *hpN0 = ss ? hp0 + (size_t)P->nslice * (2 * L - 1) : nullptr;
    double q;
    if (adjoint) q = 1.0;
    else if (mw) q = 2.0 * M_PI / (double)(ss ? 2 * L : 2 * L - 1);
    else q = 4.0 * M_PI / (double)P->nsamp;
    for (int k = 0; k < P->nslice; ++k) {
        double *F = F0 + k * nF;
        {
        TIMED(S2_STAGE_PHI_FWD);
        HIPCHK(launch_phi_fwd(st, P->fft_threads, P->fft_lds, P->nring, P->hstride, L, q, slice_maps[k], P->ring_nphi,
                              P->ring_start, P->ring_shift, P->ring_fft, P->ffts, adjoint ? nullptr : P->ringq, F,
                              fft_scratch(P, ws)),
                   "forward phi-DFT");
        }
        TIMED(S2_STAGE_MW_THETA);
        if (mw && !adjoint)
            HIPCHK(launch_mw_filter(st, P->fft_threads, P->fft_lds, L, ss, P->hstride, P->slice_spin[k], P->ffts, P->wq,
                                    P->ph, F, hp0 + k * (2 * L - 1), ss ? hpN0 + k * (2 * L - 1) : nullptr,
                                    fft_scratch(P, ws), 0, 0, CONV_ARGS(P)), "MW theta filter");
        else if (mw) {
            HIPCHK(launch_pole_from_F(st, L, P->hstride, L - 1, F, hp0 + k * (2 * L - 1)), "pole line");
            if (ss) HIPCHK(launch_pole_from_F(st, L, P->hstride, L, F, hpN0 + k * (2 * L - 1)), "north pole line");
        }
    }
    return run_forward_dstage(P, F0, mw ? hp0 : nullptr, hpN0, flm, wl, ws, st);
}

// Real signals (spin-0 S2 plan, Hermitian symmetry of the coefficients): the
// sweeps carry the orders m >= 0 only and pairs of rings share a phi-DFT.
int run_inverse_real(s2_plan_t P, const double2 *flm, double *map, char *ws, hipStream_t st)
{
    int rc = run_inverse_dstage(P, flm, P->w_sht, ws, st, 1);
    if (rc) return rc;
    TIMED(S2_STAGE_PHI_INV);
    HIPCHK(launch_phi_inv_real(st, P->fft_threads, P->fft_lds, P->npair, P->L, P->nreg, P->inv_nblk, P->ring_pairs,
                               (const double *)(ws + P->off_P), P->mtop, flm, P->w_sht[0], P->ring_nphi,
                               P->ring_start, P->ring_shift, P->ring_fft, P->ffts, map, fft_scratch(P, ws)),
           "real inverse phi-DFT");
    return S2_OK;
}

// vjp: the gradient of run_inverse_real with respect to its complex input for a
// real map cotangent: 2 A^H g at m > 0 and Re (A^H g) at m = 0 (A the complex
// inverse), i.e. the unnormalised phi-DFT, no theta filter, the forward-type
// sweep with the SHT weights, and the finish in its gradient mode.
int run_forward_real(s2_plan_t P, const double *map, double2 *flm, char *ws, hipStream_t st, bool vjp = false)
{
    const int L = P->L;
    const bool mw = P->sampling == S2_MW || P->sampling == S2_MWSS;   // theta-torus samplings
    const int ss = P->sampling == S2_MWSS;
    double *F0 = (double *)(ws + P->off_F);
    double2 *hp0 = (double2 *)(ws + P->off_hpole);
    double2 *hpN0 = ss ? hp0 + (size_t)P->nslice * (2 * L - 1) : nullptr;
    double q;
    if (vjp) q = 1.0;
    else if (mw) q = 2.0 * M_PI / (double)(ss ? 2 * L : 2 * L - 1);
    else q = 4.0 * M_PI / (double)P->nsamp;               // HEALPix (DH / GL: per-ring weights)
    {
    TIMED(S2_STAGE_PHI_FWD);
    HIPCHK(launch_phi_fwd_real(st, P->fft_threads, P->fft_lds, P->nring, P->hstride, P->npair, L, q, P->ring_pairs,
                               map, P->ring_nphi, P->ring_start, P->ring_shift, P->ring_fft, P->ffts,
                               vjp ? nullptr : P->ringq, F0, fft_scratch(P, ws)), "real forward phi-DFT");
    }
    if (mw) {
        TIMED(S2_STAGE_MW_THETA);
        if (!vjp) {
            HIPCHK(launch_mw_filter(st, P->fft_threads, P->fft_lds, L, ss, P->hstride, 0, P->ffts, P->wq, P->ph, F0,
                                    hp0, hpN0, fft_scratch(P, ws), 1, 0, CONV_ARGS(P)), "MW theta filter");
        } else {
            HIPCHK(launch_pole_from_F(st, L, P->hstride, L - 1, F0, hp0), "pole line");
            if (ss) HIPCHK(launch_pole_from_F(st, L, P->hstride, L, F0, hpN0), "north pole line");
        }
    }
    return run_forward_dstage(P, F0, mw ? hp0 : nullptr, hpN0, flm, P->w_sht, ws, st, vjp ? 2 : 1);
}

// The adjoint of the forward transform restricted to real maps: Re(F^H G) =
// F^H h with h the Hermitian part of G, so the real-signal machinery applies:
// MW / MWSS as the complex adjoint (gather, adjoint theta filter on one side,
// scatter) ending in the paired real phi-DFT; DH / GL / HEALPix the real
// inverse with the forward-adjoint weights, then the ring weights (DH / GL).
int run_forward_real_adjoint(s2_plan_t P, const double2 *G, double *map, char *ws, hipStream_t st)
{
    const int L = P->L;
    const int ss = P->sampling == S2_MWSS;
    double2 *H = (double2 *)(ws + P->off_hsym);
    HIPCHK(launch_hermitian_part(st, L, G, H), "Hermitian part");
    if (P->sampling != S2_MW && P->sampling != S2_MWSS) {
        int rc = run_inverse_dstage(P, H, P->w_fadj, ws, st, 1);
        if (rc) return rc;
        {
        TIMED(S2_STAGE_PHI_INV);
        HIPCHK(launch_phi_inv_real(st, P->fft_threads, P->fft_lds, P->npair, L, P->nreg, P->inv_nblk, P->ring_pairs,
                                   (const double *)(ws + P->off_P), P->mtop, H, P->w_fadj[0], P->ring_nphi,
                                   P->ring_start, P->ring_shift, P->ring_fft, P->ffts, map, fft_scratch(P, ws)),
               "real inverse phi-DFT");
        }
        if (P->ringq)
            HIPCHK(launch_ring_scale_real(st, P->nring, P->ring_start, P->ring_nphi, P->ringq, map), "ring weights");
        return S2_OK;
    }
    int rc = run_inverse_dstage(P, H, P->w_sht, ws, st, 1);
    if (rc) return rc;
    double *P0 = (double *)(ws + P->off_P);
    double *F0 = (double *)(ws + P->off_F);
    double2 *hp0 = (double2 *)(ws + P->off_hpole);
    double2 *hpN0 = ss ? hp0 + (size_t)P->nslice * (2 * L - 1) : nullptr;
    double *Q0 = (double *)(ws + P->off_Q);
    const double q = 2.0 * M_PI / (double)(ss ? 2 * L : 2 * L - 1);
    {
    TIMED(S2_STAGE_MW_THETA);
    // side B of the gathered rows is not produced by the half sweep and is never read
    HIPCHK(launch_fadj_gather(st, L, ss, P->inv_nblk, 0, P0, P->mtop, H, P->w_sht[0], P->hstride, F0),
           "adjoint gather");
    HIPCHK(launch_mw_filter(st, P->fft_threads, P->fft_lds, L, ss, P->hstride, 0, P->ffts, P->wq, P->ph, F0, hp0,
                            hpN0, fft_scratch(P, ws), 1, 1, CONV_ARGS(P)), "adjoint theta filter");
    HIPCHK(launch_fadj_scatter(st, L, ss, P->hstride, q, F0, hp0, hpN0, Q0), "adjoint scatter");
    }
    TIMED(S2_STAGE_PHI_INV);
    HIPCHK(launch_phi_inv_real(st, P->fft_threads, P->fft_lds, P->npair, L, P->nring, 1, P->ring_pairs, Q0, P->mtop1,
                               H, P->w_sht[0], P->ring_nphi, P->ring_start, P->ring_shift, P->ring_fft, P->ffts, map,
                               fft_scratch(P, ws)), "real adjoint phi-DFT");
    return S2_OK;
}

// ---------------------------------------------------------------- matrix-core path
// Batched inverse: flm [B][S][L][2L-1] -> slice maps [B][S][nsamp].
int run_inverse_mfma(s2_plan_t P, const double2 *flm, int B, double2 *maps, const std::vector<double *> &wl, char *ws,
                     hipStream_t st)
{
    const int L = P->L, S = P->nslice, fmt = P->prec;
    const MfmaGeom &g = P->mg;
    const size_t slab = (size_t)L * (2 * L - 1);
    const size_t nP1 = (size_t)P->nreg * L * 4;
    uint4 *D = (uint4 *)(ws + P->off_D);
    uint4 *A = (uint4 *)(ws + P->off_AH);
    double *SX = (double *)(ws + P->off_S);
    double *SY = SX + P->nslots * g.rpad;
    int *SE = (int *)(SY + P->nslots * g.rpad);
    double *Pm = (double *)(ws + P->off_mP);
    for (size_t ri = 0; ri < P->runs.size(); ++ri) {
        const Run &r = P->runs[ri];
        const double2 *fa = r.sliceA >= 0 ? flm + r.sliceA * slab : nullptr;
        const double2 *fb = r.sliceB >= 0 ? flm + r.sliceB * slab : nullptr;
        double *PA = r.sliceA >= 0 ? Pm + r.sliceA * nP1 : nullptr;
        double *PB = r.sliceB >= 0 ? Pm + r.sliceB * nP1 : nullptr;
        const int an = r.n < 0 ? -r.n : r.n;
        const int mend = an > 1 ? -(an - 1) : 0;          // continuation below m = 0
        HIPCHK(launch_zero(st, SX, P->state_bytes), "recursion state clear");
        for (int mhi = L - 1; mhi >= mend; mhi -= P->mch) {
            const int mlo = std::max(mend, mhi - P->mch + 1), mcn = mhi - mlo + 1;
            {
            TIMED(S2_STAGE_DGEN);
            HIPCHK(launch_dgen(st, 0, fmt, P->gen_waves, P->gen_nblk, g, r.n, mhi, mlo, P->cot, P->csc, P->init[ri],
                               P->kg, P->gen_lchunk, P->gen_mtop, SX, SY, SE, D), "d-tile generator");
            }
            {
            TIMED(S2_STAGE_PACK);
            HIPCHK(launch_pack_a(st, fmt, g, r.n, mlo, mcn, B, (long long)(S * slab), fa, fb,
                                 r.sliceA >= 0 ? wl[r.sliceA] : nullptr, r.sliceB >= 0 ? wl[r.sliceB] : nullptr, A),
                   "coefficient pack");
            }
            TIMED(S2_STAGE_MFMA);
            HIPCHK(launch_mfma_inv(st, fmt, g, r.n, P->cot, P->csc, mlo, mcn, B, A, D, PA, PB, (long long)(S * nP1)),
                   "inverse contraction");
        }
    }
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < S; ++k) {
            TIMED(S2_STAGE_PHI_INV);
            HIPCHK(launch_phi_inv(st, P->fft_threads, P->fft_lds, P->nring, L, P->nreg, 1, P->slice_spin[k],
                                  Pm + ((size_t)b * S + k) * nP1, P->mtop1, flm + ((size_t)b * S + k) * slab, wl[k],
                                  P->ring_nphi, P->ring_start, P->ring_shift, P->ring_fft, P->ffts,
                                  maps + ((size_t)b * S + k) * P->nsamp, fft_scratch(P, ws)), "inverse phi-DFT");
        }
    return S2_OK;
}

// Batched forward (adjoint: unit phi weight, no theta filter): slice maps [B][S][nsamp] -> flm [B][S][L][2L-1].
int run_forward_mfma(s2_plan_t P, const double2 *maps, int B, double2 *flm, const std::vector<double *> &wl, char *ws,
                     hipStream_t st, bool adjoint)
{
    const int L = P->L, S = P->nslice, fmt = P->prec;
    const MfmaGeom &g = P->mg;
    const size_t slab = (size_t)L * (2 * L - 1);
    const size_t nF = P->szF / sizeof(double), nQ1 = (size_t)L * L * 4;
    const bool mw = P->sampling == S2_MW || P->sampling == S2_MWSS;   // theta-torus samplings
    const int ss = P->sampling == S2_MWSS;
    uint4 *D = (uint4 *)(ws + P->off_D);
    uint4 *H = (uint4 *)(ws + P->off_AH);
    double *SX = (double *)(ws + P->off_S);
    double *SY = SX + P->nslots * g.rpad;
    int *SE = (int *)(SY + P->nslots * g.rpad);
    double *Fm = (double *)(ws + P->off_mF);
    double *Qm = (double *)(ws + P->off_mQ);
    double2 *hp = (double2 *)(ws + P->off_mhp);
    double2 *hpN = ss ? hp + (size_t)B * S * (2 * L - 1) : nullptr;
    const int nxp1 = std::max(P->nxp, 1);
    const size_t nQx1 = (size_t)L * nxp1 * 4;
    double *Qxm = P->nxp > 0 ? (double *)(ws + P->off_mQx) : nullptr;
    if (Qxm) HIPCHK(launch_zero(st, Qxm, (size_t)B * S * nQx1 * sizeof(double)), "continuation sums clear");
    double q;
    if (adjoint) q = 1.0;
    else if (mw) q = 2.0 * M_PI / (double)(ss ? 2 * L : 2 * L - 1);
    else q = 4.0 * M_PI / (double)P->nsamp;
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < S; ++k) {
            const size_t bk = (size_t)b * S + k;
            double *F = Fm + bk * nF;
            {
            TIMED(S2_STAGE_PHI_FWD);
            HIPCHK(launch_phi_fwd(st, P->fft_threads, P->fft_lds, P->nring, P->hstride, L, q, maps + bk * P->nsamp,
                                  P->ring_nphi, P->ring_start, P->ring_shift, P->ring_fft, P->ffts,
                                  adjoint ? nullptr : P->ringq, F,
                                  fft_scratch(P, ws)),
                   "forward phi-DFT");
            }
            TIMED(S2_STAGE_MW_THETA);
            if (mw && !adjoint)
                HIPCHK(launch_mw_filter(st, P->fft_threads, P->fft_lds, L, ss, P->hstride, P->slice_spin[k], P->ffts,
                                        P->wq, P->ph, F, hp + bk * (2 * L - 1), ss ? hpN + bk * (2 * L - 1) : nullptr,
                                        fft_scratch(P, ws), 0, 0, CONV_ARGS(P)),
                   "MW theta filter");
            else if (mw) {
                HIPCHK(launch_pole_from_F(st, L, P->hstride, L - 1, F, hp + bk * (2 * L - 1)), "pole line");
                if (ss) HIPCHK(launch_pole_from_F(st, L, P->hstride, L, F, hpN + bk * (2 * L - 1)), "north pole line");
            }
        }
    for (size_t ri = 0; ri < P->runs.size(); ++ri) {
        const Run &r = P->runs[ri];
        const double *FA = r.sliceA >= 0 ? Fm + r.sliceA * nF : Fm + r.sliceB * nF;
        const double *FB = r.sliceB >= 0 ? Fm + r.sliceB * nF : FA;
        double *QA = r.sliceA >= 0 ? Qm + r.sliceA * nQ1 : nullptr;
        double *QB = r.sliceB >= 0 ? Qm + r.sliceB * nQ1 : nullptr;
        const int an = r.n < 0 ? -r.n : r.n;
        const int mend = an > 1 ? -(an - 1) : 0;          // continuation below m = 0
        double *QxA = (an > 0 && r.sliceA >= 0) ? Qxm + r.sliceA * nQx1 : nullptr;
        double *QxB = (an > 0 && r.sliceB >= 0) ? Qxm + r.sliceB * nQx1 : nullptr;
        HIPCHK(launch_zero(st, SX, P->state_bytes), "recursion state clear");
        for (int mhi = L - 1; mhi >= mend; mhi -= P->mch) {
            const int mlo = std::max(mend, mhi - P->mch + 1), mcn = mhi - mlo + 1;
            {
            TIMED(S2_STAGE_DGEN);
            HIPCHK(launch_dgen(st, 1, fmt, P->gen_waves, P->gen_nblk, g, r.n, mhi, mlo, P->cot, P->csc, P->init[ri],
                               P->kg, P->gen_lchunk, P->gen_mtop, SX, SY, SE, D), "d-tile generator");
            }
            {
            TIMED(S2_STAGE_PACK);
            HIPCHK(launch_pack_h(st, fmt, g, P->hstride, r.n, P->cot, P->csc, mlo, mcn, B, (long long)(S * nF), FA, FB, H),
                   "spectra pack");
            }
            TIMED(S2_STAGE_MFMA);
            HIPCHK(launch_mfma_fwd(st, fmt, g, r.n, nxp1, mlo, mcn, B, H, D, QA, QB, (long long)(S * nQ1), QxA, QxB,
                                   (long long)(S * nQx1)), "forward contraction");
        }
    }
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < S; ++k) {
            const size_t bk = (size_t)b * S + k;
            const int s = P->slice_spin[k];
            TIMED(S2_STAGE_FINISH);
            HIPCHK(launch_finish_fwd(st, L, 1, s, s, Qm + bk * nQ1, Qxm ? Qxm + bk * nQx1 : nullptr, nxp1, wl[k],
                                     mw ? hp + bk * (2 * L - 1) : nullptr, ss ? hpN + bk * (2 * L - 1) : nullptr,
                                     flm + bk * slab), "forward finish");
        }
    return S2_OK;
}

}  // namespace

extern "C" {

int s2_inverse(s2_plan_t P, const void *flm, void *f, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_inverse", P, flm, f, batch, workspace);
    if (rc) return rc;
    if (P->N != 1) return fail(S2_ERR_INVALID_ARG, "s2_inverse: plan was created for SO(3) (N=%d)", P->N);
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    if (P->mfma) return run_inverse_mfma(P, (const double2 *)flm, batch, (double2 *)f, P->w_sht, (char *)workspace, st);
    for (int b = 0; b < batch; ++b) {
        double2 *out = (double2 *)f + (size_t)b * P->nsamp;
        if ((rc = run_inverse(P, (const double2 *)flm + b * slab, &out, P->w_sht, (char *)workspace, st))) return rc;
    }
    return S2_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation inverse
// The workspace of s2_inverse_noalloc: a fixed device array, one copy per GPU the
// library runs on, held until the process ends.  Host code never uses the name
// `scratch` as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[S2_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};   // per device index; nullptr until looked up

// device address of `scratch` on the current device (looked up on the first call there)
int scratch_on_current_device(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(S2_ERR_UNSUPPORTED, "s2_inverse_noalloc: device index %d beyond %d", dev, SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return S2_OK;
}

// bytes of the workspace the FP64 inverse touches (records, partials, and the
// split-Bluestein scratch when a ring DFT needs it)
size_t inverse_extent(const s2_plan_s *P)
{
    if (P->sz_fscr) return P->off_fscr + P->sz_fscr;
    return P->off_P + P->szP * P->nslice;
}

}  // namespace

extern "C" {

int s2_inverse_noalloc(s2_plan_t P, const void *flm, void *f, int batch, void *hip_stream)
{
    if (!P) return fail(S2_ERR_INVALID_ARG, "s2_inverse_noalloc: plan is NULL");
    if (P->N != 1) return fail(S2_ERR_INVALID_ARG, "s2_inverse_noalloc: plan was created for SO(3) (N=%d)", P->N);
    if (P->mfma) return fail(S2_ERR_UNSUPPORTED, "s2_inverse_noalloc: available for FP64 plans");
    const size_t need = inverse_extent(P);
    if (need > (size_t)S2_NOALLOC_SCRATCH_BYTES)
        return fail(S2_ERR_INVALID_ARG,
                    "s2_inverse_noalloc: this plan's inverse needs %zu bytes of scratch, more than the fixed %zu "
                    "(use s2_inverse with a workspace)", need, (size_t)S2_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    int rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    if ((rc = check_call("s2_inverse_noalloc", P, flm, f, batch, ws))) return rc;
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    g_no_timing = true;
    for (int b = 0; b < batch && rc == S2_OK; ++b) {
        double2 *out = (double2 *)f + (size_t)b * P->nsamp;
        rc = run_inverse(P, (const double2 *)flm + b * slab, &out, P->w_sht, (char *)ws, st);
    }
    g_no_timing = false;
    return rc;
}

int s2_forward(s2_plan_t P, const void *f, void *flm, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_forward", P, f, flm, batch, workspace);
    if (rc) return rc;
    if (P->N != 1) return fail(S2_ERR_INVALID_ARG, "s2_forward: plan was created for SO(3) (N=%d)", P->N);
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    if (P->mfma)
        return run_forward_mfma(P, (const double2 *)f, batch, (double2 *)flm, P->w_sht, (char *)workspace, st, false);
    for (int b = 0; b < batch; ++b) {
        const double2 *in = (const double2 *)f + (size_t)b * P->nsamp;
        if ((rc = run_forward(P, &in, (double2 *)flm + b * slab, P->w_sht, (char *)workspace, st, false))) return rc;
    }
    return S2_OK;
}

int s2_inverse_adjoint(s2_plan_t P, const void *g, void *g_flm, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_inverse_adjoint", P, g, g_flm, batch, workspace);
    if (rc) return rc;
    if (P->N != 1) return fail(S2_ERR_INVALID_ARG, "s2_inverse_adjoint: plan was created for SO(3) (N=%d)", P->N);
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    if (P->mfma)
        return run_forward_mfma(P, (const double2 *)g, batch, (double2 *)g_flm, P->w_sht, (char *)workspace, st, true);
    for (int b = 0; b < batch; ++b) {
        const double2 *in = (const double2 *)g + (size_t)b * P->nsamp;
        if ((rc = run_forward(P, &in, (double2 *)g_flm + b * slab, P->w_sht, (char *)workspace, st, true))) return rc;
    }
    return S2_OK;
}

int s2_forward_adjoint(s2_plan_t P, const void *g_flm, void *g, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_forward_adjoint", P, g_flm, g, batch, workspace);
    if (rc) return rc;
    if (P->N != 1) return fail(S2_ERR_INVALID_ARG, "s2_forward_adjoint: plan was created for SO(3) (N=%d)", P->N);
    if (P->mfma) return fail(S2_ERR_UNSUPPORTED, "s2_forward_adjoint: available for FP64 plans");
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    for (int b = 0; b < batch; ++b) {
        const double2 *G = (const double2 *)g_flm + b * slab;
        double2 *out = (double2 *)g + (size_t)b * P->nsamp;
        if (P->sampling == S2_MW || P->sampling == S2_MWSS)
            rc = run_forward_adjoint_mw(P, G, &out, P->w_sht, (char *)workspace, st);
        else rc = run_inverse(P, G, &out, P->w_fadj, (char *)workspace, st);
        if (rc) return rc;
        if (P->ringq)
            HIPCHK(launch_ring_scale(st, P->nring, 2 * P->L - 1, P->ringq, out), "quadrature weights");
    }
    return S2_OK;
}

int so3_inverse(s2_plan_t P, const void *flmn, void *f, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("so3_inverse", P, flmn, f, batch, workspace);
    if (rc) return rc;
    if (P->sampling != S2_MW || P->spin != 0) return fail(S2_ERR_INVALID_ARG, "so3_inverse: needs an MW spin-0 plan");
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const int S = P->nslice;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    if (P->mfma) {
        double2 *tmp = (S > 1) ? (double2 *)((char *)workspace + P->off_mmaps) : (double2 *)f;
        if ((rc = run_inverse_mfma(P, (const double2 *)flmn, batch, tmp, P->w_so3i, (char *)workspace, st))) return rc;
        if (S > 1)
            for (int b = 0; b < batch; ++b) {
                TIMED(S2_STAGE_GAMMA);
                HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, +1, 1.0, P->groots, tmp + (size_t)b * S * P->nsamp,
                                        (double2 *)f + (size_t)b * S * P->nsamp), "gamma DFT");
            }
        return S2_OK;
    }
    for (int b = 0; b < batch; ++b) {
        double2 *out = (double2 *)f + (size_t)b * S * P->nsamp;
        std::vector<double2 *> maps(S);
        double2 *tmp = (S > 1) ? (double2 *)((char *)workspace + P->off_maps) : out;
        for (int k = 0; k < S; ++k) maps[k] = tmp + (size_t)k * P->nsamp;
        if ((rc = run_inverse(P, (const double2 *)flmn + (size_t)b * S * slab, maps.data(), P->w_so3i,
                              (char *)workspace, st))) return rc;
        if (S > 1) {
            TIMED(S2_STAGE_GAMMA);
            HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, +1, 1.0, P->groots, tmp, out), "gamma DFT");
        }
    }
    return S2_OK;
}

int so3_forward(s2_plan_t P, const void *f, void *flmn, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("so3_forward", P, f, flmn, batch, workspace);
    if (rc) return rc;
    if (P->sampling != S2_MW || P->spin != 0) return fail(S2_ERR_INVALID_ARG, "so3_forward: needs an MW spin-0 plan");
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const int S = P->nslice;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    if (P->mfma) {
        const double2 *src = (const double2 *)f;
        if (S > 1) {
            double2 *tmp = (double2 *)((char *)workspace + P->off_mmaps);
            for (int b = 0; b < batch; ++b) {
                TIMED(S2_STAGE_GAMMA);
                HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, -1, 2.0 * M_PI / (double)S, P->groots,
                                        (const double2 *)f + (size_t)b * S * P->nsamp, tmp + (size_t)b * S * P->nsamp),
                       "gamma DFT");
            }
            src = tmp;
        }
        // one slice (N = 1): the gamma rule is the weight 2 pi alone, folded into the finish
        const std::vector<double *> w1 = {P->w_so3f_n1};
        return run_forward_mfma(P, src, batch, (double2 *)flmn, S > 1 ? P->w_so3f : w1, (char *)workspace, st, false);
    }
    for (int b = 0; b < batch; ++b) {
        const double2 *in = (const double2 *)f + (size_t)b * S * P->nsamp;
        std::vector<const double2 *> maps(S);
        double2 *tmp = (double2 *)((char *)workspace + P->off_maps);
        // f_n = 2pi/(2N-1) sum_k f(gamma_k) e^{-i n gamma_k}  (Eq. 16, exact equispaced rule)
        {
        TIMED(S2_STAGE_GAMMA);
        HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, -1, 2.0 * M_PI / (double)S, P->groots, in, tmp), "gamma DFT");
        }
        for (int k = 0; k < S; ++k) maps[k] = tmp + (size_t)k * P->nsamp;
        if ((rc = run_forward(P, maps.data(), (double2 *)flmn + (size_t)b * S * slab, P->w_so3f, (char *)workspace,
                              st, false))) return rc;
    }
    return S2_OK;
}

static int check_real(const char *fn, s2_plan_t P)
{
    if (P->N != 1) return fail(S2_ERR_INVALID_ARG, "%s: plan was created for SO(3) (N=%d)", fn, P->N);
    if (P->spin != 0) return fail(S2_ERR_UNSUPPORTED, "%s: real signals need a spin-0 plan", fn);
    if (P->mfma) return fail(S2_ERR_UNSUPPORTED, "%s: available for FP64 plans", fn);
    return S2_OK;
}

int s2_inverse_real(s2_plan_t P, const void *flm, void *f, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_inverse_real", P, flm, f, batch, workspace);
    if (rc || (rc = check_real("s2_inverse_real", P))) return rc;
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    for (int b = 0; b < batch; ++b)
        if ((rc = run_inverse_real(P, (const double2 *)flm + b * slab, (double *)f + (size_t)b * P->nsamp,
                                   (char *)workspace, st))) return rc;
    return S2_OK;
}

int s2_forward_real(s2_plan_t P, const void *f, void *flm, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_forward_real", P, f, flm, batch, workspace);
    if (rc || (rc = check_real("s2_forward_real", P))) return rc;
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    for (int b = 0; b < batch; ++b)
        if ((rc = run_forward_real(P, (const double *)f + (size_t)b * P->nsamp, (double2 *)flm + b * slab,
                                   (char *)workspace, st))) return rc;
    return S2_OK;
}

int s2_inverse_real_adjoint(s2_plan_t P, const void *g, void *g_flm, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_inverse_real_adjoint", P, g, g_flm, batch, workspace);
    if (rc || (rc = check_real("s2_inverse_real_adjoint", P))) return rc;
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    for (int b = 0; b < batch; ++b)
        if ((rc = run_forward_real(P, (const double *)g + (size_t)b * P->nsamp, (double2 *)g_flm + b * slab,
                                   (char *)workspace, st, true))) return rc;
    return S2_OK;
}

int s2_forward_real_adjoint(s2_plan_t P, const void *g_flm, void *g, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("s2_forward_real_adjoint", P, g_flm, g, batch, workspace);
    if (rc || (rc = check_real("s2_forward_real_adjoint", P))) return rc;
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    for (int b = 0; b < batch; ++b)
        if ((rc = run_forward_real_adjoint(P, (const double2 *)g_flm + b * slab, (double *)g + (size_t)b * P->nsamp,
                                           (char *)workspace, st))) return rc;
    return S2_OK;
}

int so3_inverse_adjoint(s2_plan_t P, const void *g, void *g_flmn, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("so3_inverse_adjoint", P, g, g_flmn, batch, workspace);
    if (rc) return rc;
    if (P->sampling != S2_MW || P->spin != 0)
        return fail(S2_ERR_INVALID_ARG, "so3_inverse_adjoint: needs an MW spin-0 plan");
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const int S = P->nslice;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    // so3_inverse = (gamma synthesis, sign +1) after the per-n inverses, so its adjoint is the
    // gamma analysis with unit weight (sign -1) followed by the per-n inverse adjoints.
    if (P->mfma) {
        const double2 *src = (const double2 *)g;
        if (S > 1) {
            double2 *tmp = (double2 *)((char *)workspace + P->off_mmaps);
            for (int b = 0; b < batch; ++b) {
                TIMED(S2_STAGE_GAMMA);
                HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, -1, 1.0, P->groots,
                                        (const double2 *)g + (size_t)b * S * P->nsamp, tmp + (size_t)b * S * P->nsamp),
                       "gamma DFT");
            }
            src = tmp;
        }
        return run_forward_mfma(P, src, batch, (double2 *)g_flmn, P->w_so3i, (char *)workspace, st, true);
    }
    for (int b = 0; b < batch; ++b) {
        const double2 *in = (const double2 *)g + (size_t)b * S * P->nsamp;
        const double2 *src = in;
        if (S > 1) {
            double2 *tmp = (double2 *)((char *)workspace + P->off_maps);
            TIMED(S2_STAGE_GAMMA);
            HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, -1, 1.0, P->groots, in, tmp), "gamma DFT");
            src = tmp;
        }
        std::vector<const double2 *> maps(S);
        for (int k = 0; k < S; ++k) maps[k] = src + (size_t)k * P->nsamp;
        if ((rc = run_forward(P, maps.data(), (double2 *)g_flmn + (size_t)b * S * slab, P->w_so3i, (char *)workspace,
                              st, true))) return rc;
    }
    return S2_OK;
}

int so3_forward_adjoint(s2_plan_t P, const void *g_flmn, void *g, int batch, void *workspace, void *hip_stream)
{
    int rc = check_call("so3_forward_adjoint", P, g_flmn, g, batch, workspace);
    if (rc) return rc;
    if (P->sampling != S2_MW || P->spin != 0)
        return fail(S2_ERR_INVALID_ARG, "so3_forward_adjoint: needs an MW spin-0 plan");
    if (P->mfma) return fail(S2_ERR_UNSUPPORTED, "so3_forward_adjoint: available for FP64 plans");
    if (batch == 0) return S2_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const int S = P->nslice;
    const size_t slab = (size_t)P->L * (2 * P->L - 1);
    // so3_forward = per-n MW forwards after the gamma analysis (sign -1, weight 2pi/(2N-1)), so
    // its adjoint is the per-n forward adjoints followed by the gamma synthesis with that weight.
    double2 *tmp = (double2 *)((char *)workspace + P->off_maps);
    std::vector<double2 *> maps(S);
    for (int k = 0; k < S; ++k) maps[k] = tmp + (size_t)k * P->nsamp;
    for (int b = 0; b < batch; ++b) {
        if ((rc = run_forward_adjoint_mw(P, (const double2 *)g_flmn + (size_t)b * S * slab, maps.data(), P->w_so3f,
                                         (char *)workspace, st))) return rc;
        TIMED(S2_STAGE_GAMMA);
        HIPCHK(launch_gamma_dft(st, P->N, P->nsamp, +1, 2.0 * M_PI / (double)S, P->groots, tmp,
                                (double2 *)g + (size_t)b * S * P->nsamp), "gamma DFT");
    }
    return S2_OK;
}

int s2_plan_set_timing(s2_plan_t P, int enable)
{
    if (!P) return fail(S2_ERR_INVALID_ARG, "s2_plan_set_timing: plan is NULL");
    P->timing = enable != 0;
    return S2_OK;
}

int s2_plan_read_timing(s2_plan_t P, s2_timing_t *out)
{
    if (!P || !out) return fail(S2_ERR_INVALID_ARG, "s2_plan_read_timing: null argument");
    for (int s = 0; s < S2_NSTAGES; ++s) { out->ms[s] = 0.0; out->launches[s] = 0; }
    int rc = S2_OK;
    for (auto &t : P->tl) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess && rc == S2_OK) rc = hipfail(e, "stage timing");
        if (t.stage >= 0 && t.stage < S2_NSTAGES) { out->ms[t.stage] += ms; out->launches[t.stage] += 1; }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    P->tl.clear();
    return rc;
}

int s2_debug_wigner_d(s2_plan_t P, int n, void *out, void *hip_stream)
{
    if (!P || !out) return fail(S2_ERR_INVALID_ARG, "s2_debug_wigner_d: null argument");
    int ri = -1;
    for (size_t i = 0; i < P->runs.size(); ++i) if (P->runs[i].n == n) ri = (int)i;
    if (ri < 0) return fail(S2_ERR_INVALID_ARG, "s2_debug_wigner_d: n=%d is not a run of this plan", n);
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(hipMemsetAsync(out, 0, (size_t)P->nreg * P->L * P->L * sizeof(double), st), "memset");
    HIPCHK(launch_debug_d(st, P->L, P->nreg, n, P->cot, P->csc, P->lsin, P->lcos, P->lbin[ri], P->kap, P->gtab,
                          (double *)out), "debug d");
    return S2_OK;
}

}  // extern "C"
