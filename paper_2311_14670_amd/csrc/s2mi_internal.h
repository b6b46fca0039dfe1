// s2mi_internal.h -- library-internal declarations shared by the host constant
// generator (g++), the kernels and the C-ABI layer (hipcc).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace s2mi {

// ----------------------------------------------------------------- host constants
struct RingConsts {
    std::vector<double> theta, cot, csc;   // per ring
    std::vector<double> lsin, lcos;        // per ring, double-double (hi, lo): log2 sin(th/2), log2 cos(th/2)
};

#ifdef __SIZEOF_FLOAT128__
#if !defined(__HIP_DEVICE_COMPILE__) && !defined(__HIPCC__)
void fill_ring(RingConsts *rc, int r, __float128 th);
#endif
#endif
void host_mw_rings(int L, RingConsts *rc);
void host_mwss_rings(int L, RingConsts *rc);
void host_dh_rings(int L, RingConsts *rc, std::vector<double> *wq);
void host_gl_rings(int L, RingConsts *rc, std::vector<double> *wq);
void host_healpix_rings(int nside, RingConsts *rc, std::vector<int> *nphi,
                        std::vector<long long> *start, std::vector<int> *shift);
void host_log2_binom(int L, int n, std::vector<double> *out);
void host_recursion_tables(int L, int nx, std::vector<double> *kap, std::vector<double> *gtab);
void host_roots(int n, std::vector<double> *out);
void host_chirp(int n, std::vector<double> *out);
void host_mw_filter(int L, bool ss, std::vector<double> *wq, std::vector<double> *ph);
void host_shift_spectra(int L, int M, std::vector<double> *out);
void host_weights(int L, int kind, int spin, std::vector<double> *w);

// ----------------------------------------------------------------- FFT
constexpr int FFT_MAX_STAGES = 16;
constexpr int FFT_MAX_LEN = 8192;        // LDS-resident engine length (complex doubles)
constexpr int FFT_THREADS = 1024;
constexpr size_t FFT_SCRATCH = 2 * (size_t)FFT_MAX_LEN;   // split Bluestein: complex scratch entries per workgroup

// Everything a kernel needs to run one DFT of length n in LDS (passed by value).
struct FftArgs {
    int n;            // logical DFT length
    int len;          // engine length: n (mixed radix) or a power of two >= 2n-1 (Bluestein);
                      // split Bluestein: half the convolution length M = 2 len
    int blue;         // 1: Bluestein
    int split;        // 1: Bluestein convolution of length 2 len done as two LDS-resident halves
    int nst;          // engine stages
    int rad[FFT_MAX_STAGES];
    const double *tw;     // e^{-2 pi i k/len}, k < len (interleaved)
    const double *chirp;  // Bluestein: e^{+i pi k^2/n}, k < n
    const double *bflt;   // Bluestein: FFT of the chirp filter over the convolution length, divided by it
    const double *twm;    // split: e^{-2 pi i k/(2 len)}, k < len
    int conv;             // 1: a cyclic convolution, not a DFT: the chirp is 1 and bflt is
                          // the spectrum of a kernel the plan supplies (the Bluestein
                          // machinery then returns the convolution at t < n)
};

// ----------------------------------------------------------------- d-stage geometry
constexpr int INV_NCH = 4;              // 8-degree chunks per wave, inverse d-stage
constexpr int INV_J = 8 * INV_NCH;      // l-slots per wave
constexpr int FWD_NCH = 1;              // 8-ring chunks per wave, forward d-stage
constexpr int FWD_R = 8 * FWD_NCH;      // ring-slots per wave
constexpr int GEN_NCH = 2;              // 8-degree chunks per wave, d-tile generator (matrix-core path)
constexpr int DSTAGE_MAX_WAVES = 8;     // inverse sweep / d-tile generator workgroups: at most 512 threads
constexpr int FWD_MAX_WAVES = 16;       // forward sweep workgroups: at most 1024 threads (4, 8 or 16 waves)

// Order tiles of the sweeps.  Tile k runs the orders c[k] - 1 down to c[k+1]
// (c[0] = L; the last tile runs down to the run's lowest order), so that more
// workgroups share one run without adding partial sums (each order stays in one
// tile).  A tile k > 0 starts from the recursion state after order c[k], held per
// run in ck at offset off[k] as rows (l - c[k]), l >= c[k], of 3 x rp doubles:
// {e_{c[k]}[ring], e_{c[k]+1}[ring], E[ring]} (a recursion slot state; see renorm).
constexpr int MAX_ORDER_TILES = 8;
struct OrderTiles {
    int nt = 1;                             // tiles (1: the whole order range)
    int rp = 0;                             // ring stride of a state row
    int c[MAX_ORDER_TILES + 1] = {};
    long long off[MAX_ORDER_TILES] = {};
    const double *ck = nullptr;             // the run's state table (nt > 1)
};

// One recursion run: fixed second index n of d^l_{m,n}; its A side feeds the
// slice of spin -n at orders +m, its B side the slice of spin +n at orders -m.
struct Run {
    int n;
    int sliceA;   // slice index or -1
    int sliceB;   // slice index or -1
};

}  // namespace s2mi
