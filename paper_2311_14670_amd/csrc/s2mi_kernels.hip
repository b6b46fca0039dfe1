// s2mi_kernels.hip -- gfx950 kernels of the spin SHT / Wigner transforms.
//
// Paper: Price & McEwen, arXiv 2311.14670.
//   d-stage   Wigner d^l_{m,n}(theta) by the descending-m recursion (Sec. 3.3,
//             Eqs. 25-26) started from Eq. 27 in log space, renormalised as it
//             runs (Sec. 3.4), fused with the l-contraction of Eq. 33 (inverse)
//             or the theta-contraction of Eq. 30 (forward) -- Sec. 4.4.
//   phi-DFT   Eqs. 31-32 per isolatitude ring; HEALPix rings repeat / fold the
//             Fourier line (Sec. 4.2, HEALPix).
//   MW theta  the exact MW theta integral (Sec. 4.2, MW): torus extension,
//             band-limited sin(theta) weight, evaluated on the L rings.
//
// Recursion in rescaled form.  With alpha_k = sqrt((l+k)(l-k+1)) and
// d_m = e_m g_m (g from the plan tables), Eq. 25 becomes
//     e_{m-1} = kappa_m lambda_m e_m - e_{m+1},  lambda_m = (n - m cos th)/sin th,
// two FP64 operations per step.  Each (ring, l) carries (e_m, e_{m+1}, E) with
// d = e g 2^E.  While the value is below 2^-600 (E < 0) the pair is held scaled near
// 2^-600 and renormalised by an exact power of two every RN orders; the contraction
// uses e as it stands, so such a slot adds a negligible amount (below 2^-279 of its
// record) with no per-step scaling.  Once the value is within 2^-600 of unit scale
// it is realised (E = 0, d = e g): |d| <= 1 and the recursion runs downhill in m, so
// it can no longer overflow or meaningfully underflow.  A chunk whose lanes are all
// realised skips the renormalisation.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "s2mi_fft.h"
#include "s2mi_internal.h"
#include "s2mi_kernels.h"
#include "s2mi_recur.h"

namespace s2mi {

// ------------------------------------------------------------------ helpers
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_from(const double *p) { return DD{p[0], p[1]}; }

__device__ __forceinline__ DD two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return DD{s, e};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    DD s = two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return two_sum(s.hi, s.lo);
}

__device__ __forceinline__ DD dd_mul_d(DD a, double k)   // k an exact small integer
{
    const double p = a.hi * k;
    const double e = fma(a.hi, k, -p);
    return two_sum(p, e + a.lo * k);
}

// d^l_{l,n}(theta) of Eq. 27 as a recursion slot state (e, E): log2|d| =
// lbin + (l-n) log2 sin(th/2) + (l+n) log2 cos(th/2) in double-double, sign (-1)^{l-n}.
// Realised (E = 0) directly when the value is not tiny; otherwise e = v 2^-RT with
// v in [1, 2) and the value is e 2^E, E < 0 (see renorm).
__device__ __forceinline__ void d_init(int l, int n, DD lbin, DD ls, DD lc, double &e, int &E)
{
    DD x = dd_add(lbin, dd_add(dd_mul_d(ls, (double)(l - n)), dd_mul_d(lc, (double)(l + n))));
    double fl = floor(x.hi);
    double f = (x.hi - fl) + x.lo;
    if (f < 0.0) { f += 1.0; fl -= 1.0; }
    if (f >= 1.0) { f -= 1.0; fl += 1.0; }
    double v = exp2(f);
    if ((l - n) & 1) v = -v;
    int ex = (int)fl;
    if (ex >= -RT) { v = ldexp(v, ex); ex = 0; }
    else { v = ldexp(v, -RT); ex += RT; }
    e = v;
    E = ex;
}

// ------------------------------------------------------------------ start values
// init[r][l] = {mantissa, exponent} of d^l_{l,n}(theta_r) (Eq. 27) for every
// swept ring and l >= |n| (zeros below): computed once per plan so the sweeps
// only load them when a degree starts.
__global__ void k_init_table(int L, int nreg, int n, const double *__restrict__ lsin, const double *__restrict__ lcos,
                             const double *__restrict__ lbin, double2 *__restrict__ init)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nreg * L) return;
    const int r = (int)(i / L), l = (int)(i % L);
    const int an = n < 0 ? -n : n;
    double e = 0.0;
    int E = 0;
    if (l >= an) d_init(l, n, dd_from(lbin + 2 * l), dd_from(lsin + 2 * r), dd_from(lcos + 2 * r), e, E);
    init[i] = make_double2(e, (double)E);
}

// ------------------------------------------------------------------ inverse pack
// Records in the inverse sweep's slot order, C[blk][m + nx][wave][slot] = 5 doubles
//   {kappa_{m+1}^l, wA_l g_m^l flmA[l][m], wB_l g_m^l (-1)^{m-n} flmB[l][-m]}
// for l = lslot[blk][wave][slot] and orders m in [-nx, L); zeros where the run
// does not reach (l < max(m, |n|), empty slot) or the side is absent.  The
// B record is used at m > 0 and, for n != 0, at m <= 0 by the continuation of
// the run below m = 0 (orders m <= 0 then feed the B slice at -m >= 0 and the
// A slice at m < 0).  A wave reads the records of one order at fixed offsets
// from a single base address.  One side (rs = 3): the records hold kappa and the
// A side (real signals: the B side is its conjugate) or, with flmA absent, the
// B side (a spin-s sphere run that feeds only the orders -m of its slice).
__global__ void k_pack_inv(int L, int nx, int n, int nslot, int S, int rs, const int *__restrict__ lslot,
                           const double2 *__restrict__ flmA, const double2 *__restrict__ flmB,
                           const double *__restrict__ wA, const double *__restrict__ wB,
                           const double *__restrict__ kap, const double *__restrict__ gtab, double *__restrict__ C)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // i = (blk, slot-in-block)
    const int m = (int)blockIdx.y - nx;
    if (i >= (size_t)nslot) return;
    const int M = 2 * L - 1;
    const int an = n < 0 ? -n : n;
    const int l = lslot[i];
    double rec[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (l >= 0 && l >= m && l >= an) {
        const double g = gtab[(ptrdiff_t)m * L + l];
        if (l > m) rec[0] = kap[(ptrdiff_t)m * L + l];
        if (flmA) {
            const double2 a = flmA[(size_t)l * M + (L - 1) + m];
            const double sa = wA[l] * g;
            rec[1] = sa * a.x;
            rec[2] = sa * a.y;
        }
        if (flmB && (m > 0 || an > 0)) {
            const double2 b = flmB[(size_t)l * M + (L - 1) - m];
            double sb = wB[l] * g;
            if ((m - n) & 1) sb = -sb;
            rec[3] = sb * b.x;
            rec[4] = sb * b.y;
        }
    }
    // slot index i = blk * S + s (S slots per block); record at ((blk * (L + nx) + m + nx) * S + s)
    const int blk = (int)(i / S), s = (int)(i % S);
    double *o = C + (((size_t)blk * (L + nx) + (m + nx)) * S + s) * rs;
    if (rs == 3) {
        o[0] = rec[0];
        o[1] = flmA ? rec[1] : rec[3];
        o[2] = flmA ? rec[2] : rec[4];
    } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) o[q] = rec[q];
    }
}

// ------------------------------------------------------------------ inverse d-stage
// Lanes = 64 rings.  Each wave owns two chunks of SG = 8 consecutive l (a high
// and a low chunk, for balance; slot j of a chunk holds l = base + SG-1-j),
// waves of a workgroup share the rings and split the l-range.  A slot whose l
// has not started (l < m) has zero state and zero records, so chunks need no
// per-slot activity test: a chunk is skipped until its top l is reached, its
// SG starts happen in SG consecutive "ramp" orders, and afterwards it runs the
// branch-free step
//   e_{m-1} = (kappa lambda) e_m - e_{m+1};  acc += e * C[m][slot].{A,B}.
// The two state registers of a slot alternate roles between consecutive
// orders (PAR), so the recursion needs no register moves.  Per order, each
// wave's partial sums are reduced over the waves in LDS by a rotating group of
// four waves and written to partA/partB[blk][ring][m].
// Renormalisation pass over chunks that are not yet realised, every RN orders (see
// s2mi_recur.h); a chunk whose lanes all reached E = 0 stays realised while no degree
// starts in it.  (Passes every 8 orders: MW L = 2048 inverse 2.70 ms, forward 2.78 ms;
// every 16: 2.62 and 2.71-2.76 ms.)
// Orders of record / spectra prefetch ahead of use (both sweeps, every run).  Measured
// at MW L = 2048 spin 0 with the unscaled contraction and passes every 16 orders:
// inverse 2.61 / 2.60 / 2.62 ms and forward 2.72 / 2.68 / 2.74 ms at 3 / 2 / 4 orders
// ahead.
constexpr int PFD = 2;

// ------------------------------------------------------------------ order-tile states
// State of the descending recursion (Eq. 25 in the rescaled form of the sweeps)
// after order c of every order-tile cut c = ot.c[k], k >= 1, for ring r and degree
// l >= c: thread (r, l) starts at order l from d^l_{l,n} (Eq. 27) and steps down
// with the sweeps' operations (kappa lambda, then one fma), renormalising every RN
// orders by exact powers of two at the same orders as the sweeps, so a tile that
// starts from this state holds exactly the state of the uninterrupted sweep.  Rings past nreg and degrees below |n| (never started)
// hold zeros.
__global__ void k_order_ckpt(int L, int nreg, int n, const double *__restrict__ cot, const double *__restrict__ csc,
                             const double2 *__restrict__ init, const double *__restrict__ kap, OrderTiles ot,
                             double *__restrict__ ck)
{
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int l = (int)blockIdx.y;
    if (r >= ot.rp) return;
    const int an = n < 0 ? -n : n;
    const bool live = r < nreg && l >= an;
    double cur = 0.0, prev = 0.0;                        // e_m, e_{m+1}
    int E = 0;
    double ct = 0.0, ncs = 0.0;
    if (live) {
        const double2 v = init[(size_t)r * L + l];
        cur = v.x;
        E = (int)v.y;
        ct = cot[r];
        ncs = (double)n * csc[r];
    }
    int m = l;
    for (int k = 1; k < ot.nt; ++k) {
        const int c = ot.c[k];
        if (c > l) continue;
        if (live) {
            for (int mm = m - 1; mm >= c; --mm) {
                const double lam = fma(-(double)(mm + 1), ct, ncs);
                const double p = kap[(ptrdiff_t)mm * L + l] * lam;
                const double nw = fma(p, cur, -prev);
                prev = cur;
                cur = nw;
                if ((mm & (RN - 1)) == 0) renorm(cur, prev, E);
            }
            m = c;
        }
        double *q = ck + ot.off[k] + (size_t)(l - c) * 3 * ot.rp + r;
        q[0] = cur;
        q[ot.rp] = prev;
        q[2 * ot.rp] = (double)E;
    }
}

// Workgroups of the sweeps hold W = 4, 8 or 16 waves; the 4 x 64 outputs of an
// order are reduced by one group of four waves, rotating with the order.
__device__ __forceinline__ int reducer_group(int m, int W)
{
    return m & ((W >> 2) - 1);                            // positive residue, also for m < 0
}

// Sum over the W waves of one output's partials in LDS (NC components of 64 per
// wave).  The reads of all MAXW slots are issued together; slots of absent waves
// are read (inside the buffer) but selected away, so stale contents never enter
// the sum.  The sum is a pairwise tree (depth log2 MAXW instead of a chain of MAXW
// dependent adds).
template <int MAXW, int NC = 4>
__device__ __forceinline__ double wave_sum(const double *rb, int comp, int i, int W)
{
    double v[MAXW];
#pragma unroll
    for (int ww = 0; ww < MAXW; ++ww) v[ww] = ww < W ? rb[(ww * NC + comp) * 64 + i] : 0.0;
#pragma unroll
    for (int h = MAXW / 2; h >= 1; h /= 2)
#pragma unroll
        for (int ww = 0; ww < h; ++ww) v[ww] += v[ww + h];
    return v[0];
}

template <int NCH>
__device__ __forceinline__ void renorm_chunks(double (&X)[NCH][SG], double (&Y)[NCH][SG], int (&E)[NCH][SG], int p,
                                              uint32_t &real)
{
#pragma unroll
    for (int g = 0; g < NCH; ++g) {
        if (g >= p || ((real >> g) & 1u)) continue;
        bool z = true;
#pragma unroll
        for (int j = 0; j < SG; ++j) {
            renorm(X[g][j], Y[g][j], E[g][j]);
            z = z && (E[g][j] == 0);
        }
        if (__all(z)) real |= (1u << g);
    }
}

// One order of one chunk: e_{m-1} = (kappa lambda) e_m - e_{m+1}, plus the
// contribution e times the records (unscaled: a slot not yet realised holds e near
// 2^-RT, so its contribution is negligible; see renorm).
// SIDE 1 / 2 (one side present: real signals, or a spin-s sphere run, which
// feeds only the orders +m or only -m of its slice): records of RS = 3 doubles,
// {kappa, that side's coefficient}.  ac[0..3] are the sums {Re A, Im A, Re B,
// Im B}; PAIR: ac[0..3] over the even and ac[4..7] over the odd degrees (slot j
// of a chunk holds l = base + SG-1-j, base a multiple of SG, so l is odd
// exactly when j is even).
template <int PAR, int SIDE = 0, bool PAIR = false>
__device__ __forceinline__ void inv_chunk(double (&X)[SG], double (&Y)[SG], const double *__restrict__ rec, double lam,
                                          double (&ac)[PAIR ? 8 : 4])
{
    constexpr int RS = SIDE ? 3 : 5;
    // GROUPED: all kappa-lambda products, then all recurrence updates, then the
    // contractions, so that dependent FP64 operations issue several apart (the
    // operations and the summation order are those of one slot after another).
    // Measured at L = 2048, this pays only for the two-sided unpaired sweep (MW
    // inverse 3.62 -> 3.36 ms); the one-sided and the paired sweeps keep the
    // slot-by-slot order, which is faster for them (the paired form spills when
    // grouped).
    constexpr bool GROUPED = SIDE == 0 && !PAIR;
    double tt[SG];
    if constexpr (GROUPED) {
        double p[SG];
#pragma unroll
        for (int j = 0; j < SG; ++j) p[j] = rec[j * RS] * lam;
#pragma unroll
        for (int j = 0; j < SG; ++j) {
            double &nw = PAR == 0 ? Y[j] : X[j];          // receives order m
            double &od = PAR == 0 ? X[j] : Y[j];          // holds order m+1
            nw = fma(p[j], od, -nw);
            tt[j] = nw;
        }
    }
#pragma unroll
    for (int j = 0; j < SG; ++j) {
        const int o = (PAIR && (j & 1) == 0) ? 4 : 0;
        const double *c = rec + j * RS;
        double t = tt[j];
        if constexpr (!GROUPED) {
            double &nw = PAR == 0 ? Y[j] : X[j];
            double &od = PAR == 0 ? X[j] : Y[j];
            nw = fma(c[0] * lam, od, -nw);
            t = nw;
        }
        if constexpr (SIDE == 2) {
            ac[o + 2] = fma(t, c[1], ac[o + 2]);
            ac[o + 3] = fma(t, c[2], ac[o + 3]);
        } else {
            ac[o + 0] = fma(t, c[1], ac[o + 0]);
            ac[o + 1] = fma(t, c[2], ac[o + 1]);
            if constexpr (SIDE == 0) {
                ac[o + 2] = fma(t, c[3], ac[o + 2]);
                ac[o + 3] = fma(t, c[4], ac[o + 3]);
            }
        }
    }
}

// A degree l starts at order m = l from its start value (e0, E0) (Eq. 27) with
// e_{l+1} = 0.  Its slot holds zero state until then and its record at l == m
// has kappa = 0, so writing -e0 into the register that receives order m lets the
// ordinary step produce e_m = fma(0, 0, e0) = e0: every chunk runs one step form.
// jin is wave-uniform.
template <int PAR>
__device__ __forceinline__ void inv_preset(double (&X)[SG], double (&Y)[SG], int (&E)[SG], int jin, double e0, int E0)
{
#pragma unroll
    for (int j = 0; j < SG; ++j)
        if (j == jin) {
            (PAR == 0 ? Y[j] : X[j]) = -e0;
            E[j] = E0;
        }
}

// PAIR (spin 0, N/S-symmetric sampling): the lanes sweep the northern rings
// (nsw of nreg) and also produce the mirror ring nreg-1-r, using
// d^l_{m,0}(pi - theta) = (-1)^{l+m} d^l_{m,0}(theta): with E and O the sums
// over the even and odd degrees, ring r gets E + O and its mirror (-1)^m (E - O).
template <int SIDE, bool PAIR>
__device__ __forceinline__ void inv_reduce(int m, int L, int W, bool good, int ms, int ring0, int nreg, int nsw,
                                           const double *rb, int blk, double *__restrict__ partA,
                                           double *__restrict__ partB);

// One order of the inverse sweep: its partial sums go to LDS buffer m mod 8 (paired:
// m mod 4) and the caller reduces four orders (paired: two) after one barrier.
template <int NCH, int PAR, int SIDE = 0, bool PAIR = false>
__device__ __forceinline__ void inv_step(int m, int L, int nx, int n, int an, bool good, int ms, int ring0, int nreg,
                                         int nsw, int lane,
                                         int w, int W,
                                         const int (&lb)[NCH], double (&X)[NCH][SG], double (&Y)[NCH][SG],
                                         int (&E)[NCH][SG], uint32_t &fast, double ct, double ncs,
                                         const double2 *__restrict__ initr, const double *__restrict__ C, double *red,
                                         int blk, double *__restrict__ partA, double *__restrict__ partB)
{
    constexpr int RS = SIDE ? 3 : 5;
    constexpr int NA = PAIR ? 8 : 4;                     // sums per lane
    const double lam = fma(-(double)(m + 1), ct, ncs);   // lambda_{m+1}: produces order m
    double ac[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) ac[c] = 0.0;
    const double *Cw = C + (((size_t)blk * (L + nx) + (m + nx)) * W + w) * (NCH * SG) * RS;   // records at order m

#pragma unroll
    for (int g = 0; g < NCH; ++g) {
        const int base = lb[g];
        if (base < 0 || m > base + SG - 1) continue;     // chunk not started
        const double *rec = Cw + g * SG * RS;
        if (m >= base) {                                  // ramp: slot base + SG-1 - m starts at this order
            if (m >= an) {
                const double2 iv = initr[m];             // d^m_{m,n}(theta_ring) as (mantissa, exponent)
                inv_preset<PAR>(X[g], Y[g], E[g], base + SG - 1 - m, iv.x, (int)iv.y);
            }
            fast &= ~(1u << g);
        }
        inv_chunk<PAR, SIDE, PAIR>(X[g], Y[g], rec, lam, ac);
    }
    // renormalisation pass every RN orders over the started chunks not yet realised
    if ((m & (RN - 1)) == 0) {
#pragma unroll
        for (int g = 0; g < NCH; ++g) {
            const int base = lb[g];
            if (base < 0 || m > base + SG - 1 || ((fast >> g) & 1u)) continue;
            bool z = true;
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                renorm(X[g][j], Y[g][j], E[g][j]);
                z = z && (E[g][j] == 0);
            }
            if (__all(z)) fast |= (1u << g);
        }
    }
    constexpr int NBUF = PAIR ? 4 : 8;
    double *rb = red + (size_t)(m & (NBUF - 1)) * DSTAGE_MAX_WAVES * NA * 64;
#pragma unroll
    for (int c = 0; c < NA; ++c)
        if (SIDE == 0 || (SIDE == 1) == ((c & 3) < 2)) rb[(w * NA + c) * 64 + lane] = ac[c];
}

// Sum of one order's partials over the waves (LDS buffer rb) and its store.
template <int SIDE, bool PAIR>
__device__ __forceinline__ void inv_reduce(int m, int L, int W, bool good, int ms, int ring0, int nreg, int nsw,
                                           const double *rb, int blk, double *__restrict__ partA,
                                           double *__restrict__ partB)
{
    constexpr int NA = PAIR ? 8 : 4;
    // four waves, rotating with the order, reduce the 4 x 64 outputs over the waves
    // (only the present side's 2 x 64 for SIDE 1 / 2)
    const int tr = (int)threadIdx.x - 256 * reducer_group(m, W);
    if (tr >= 0 && tr < 256 && (SIDE == 0 || (SIDE == 1) == (tr < 128))) {
        const int rl = tr & 63, comp = tr >> 6;         // rl == lane: this thread's ring
        double s = 0.0, s2 = 0.0;                       // a plain loop: fewer scalar registers than wave_sum
        if (PAIR) {
            double se = 0.0, so = 0.0;
            for (int ww = 0; ww < W; ++ww) {
                se += rb[(ww * NA + comp) * 64 + rl];
                so += rb[(ww * NA + 4 + comp) * 64 + rl];
            }
            s = se + so;                                // ring ring0 + rl
            s2 = (m & 1) ? so - se : se - so;           // its mirror
        } else {
            for (int ww = 0; ww < W; ++ww) s += rb[(ww * NA + comp) * 64 + rl];
        }
        // Orders below the ring's switch order ms come from the run that is stable
        // there (n cos(theta) < 0): it writes its own sides at m >= 0 and, from its
        // continuation to m > -ms, the A slice at order m < 0 (components 2,3 at |m|)
        // and the B slice at order -m >= 0 (components 0,1 at |m|).  The other run
        // writes nothing below ms.
        double *dst = nullptr;
        int mo = m, co = comp;
        const bool ext_ok = good && m <= 0 && -m < ms;   // continuation output of the stable run
        if (comp < 2) {
            if (m >= 0 && (good || m >= ms)) dst = partA;                      // A slice at order m
            else if (m < 0 && ext_ok) { dst = partA; mo = -m; co = comp + 2; }  // A slice at order m < 0
        } else {
            if (m > 0 && (good || m >= ms)) dst = partB;                       // B slice at order -m
            else if (ext_ok) { dst = partB; mo = -m; co = comp - 2; }          // B slice at order -m >= 0
        }
        const int rr = ring0 + rl;
        if (dst && rr < nsw) {
            dst[(((size_t)blk * nreg + rr) * L + mo) * 4 + co] = s;
            if (PAIR && nreg - 1 - rr != rr) dst[(((size_t)blk * nreg + (nreg - 1 - rr)) * L + mo) * 4 + co] = s2;
        }
    }
}

template <int NCH, int WT, int SIDE = 0, bool PAIR = false>
__global__ __launch_bounds__(64 * WT) void k_dstage_inv(
    int L, int nx, int nreg, int nsw, int n, const double *__restrict__ cot, const double *__restrict__ csc,
    const double2 *__restrict__ init, const double *__restrict__ C, const int *__restrict__ lchunk,
    const int *__restrict__ mtop, double *__restrict__ partA, double *__restrict__ partB, OrderTiles ot)
{
    // unpaired sweeps reduce four orders per barrier (eight 16 KB buffers); the paired
    // sweep, with twice the sums, two orders per barrier (four 32 KB buffers)
    constexpr int DORD = PAIR ? 2 : 4;                   // orders per barrier
    __shared__ double red[2 * DORD * DSTAGE_MAX_WAVES * (PAIR ? 8 : 4) * 64];
    const int an = n < 0 ? -n : n;
    const int lane = threadIdx.x & 63;
    const int w = ufl(threadIdx.x >> 6);
    constexpr int W = WT;                                // waves per workgroup (== blockDim.x / 64)
    const int blk = blockIdx.y;
    const int ring0 = blockIdx.x * 64;
    const int ring = min(ring0 + lane, nsw - 1);        // swept rings 0 .. nsw-1 (nsw == nreg unless PAIR)
    const double ct = cot[ring], cs = csc[ring];
    const double ncs = (double)n * cs;
    const bool good = ring_good(n, ct);                 // this run is the stable one at this ring
    const int ms = switch_order(n, ct, cs);
    const int mend = an > 1 ? -(an - 1) : 0;            // continuation below m = 0
    const double2 *initr = init + (size_t)ring * L;

    int lb[NCH];
#pragma unroll
    for (int g = 0; g < NCH; ++g) lb[g] = ufl(lchunk[((size_t)blk * W + w) * NCH + g]);
    double X[NCH][SG], Y[NCH][SG];
    int E[NCH][SG];
#pragma unroll
    for (int g = 0; g < NCH; ++g)
#pragma unroll
        for (int j = 0; j < SG; ++j) { X[g][j] = 0.0; Y[g][j] = 0.0; E[g][j] = 0; }
    uint32_t fast = 0;

    // order tile blockIdx.z: orders ctop - 1 .. bot; the slots whose degree started
    // above the tile (l >= ctop) resume from the stored state after order ctop
    const int tile = blockIdx.z;
    const int ctop = tile == 0 ? L : ot.c[tile];
    const int bot = tile + 1 < ot.nt ? ot.c[tile + 1] : mend;
    const int mt = min(ufl(mtop[blk]), ctop - 1);
    if (mt < bot) return;                               // no degree of this block reaches the tile
    if (tile > 0) {
        const double *ck = ot.ck + ot.off[tile] + ring;
#pragma unroll
        for (int g = 0; g < NCH; ++g)
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                const int l = lb[g] + SG - 1 - j;
                if (lb[g] >= 0 && l >= ctop && l < L) {   // PAR 0 at order ctop - 1: X holds e_{ctop}
                    const double *q = ck + (size_t)(l - ctop) * 3 * ot.rp;
                    X[g][j] = q[0];
                    Y[g][j] = q[ot.rp];
                    E[g][j] = (int)q[2 * ot.rp];
                }
            }
    }
    int pf = 0;
    constexpr int RS = SIDE ? 3 : 5;                     // doubles per record
    constexpr int ROWB = NCH * SG * RS * 8;              // bytes of one wave's records per order
    static_assert(ROWB % 128 == 0, "a wave's record row spans whole cache lines");
    // Pull the records of orders mm - PFD and mm - PFD - 1 toward the caches (one
    // dword per 128-byte line); the result is consumed only at the next pair of
    // orders, so the load latency overlaps this pair's work.
    auto prefetch = [&](int mm) {
        asm volatile("" ::"v"(pf));
        if (mm - PFD - 1 >= -nx && lane < 2 * ROWB / 128) {
            const int row = mm - PFD - (lane >= ROWB / 128 ? 1 : 0);
            const int *Cp = reinterpret_cast<const int *>(C + (((size_t)blk * (L + nx) + (row + nx)) * W + w) *
                                                                  (NCH * SG) * RS);
            pf = Cp[(lane % (ROWB / 128)) * 32];
        }
    };
    // DORD orders per barrier, their sums in LDS buffers m mod 2 DORD; with 8 waves
    // the two reducer groups take DORD / 2 orders each.  An order's buffer is next
    // written two iterations on, after the next barrier, which every reducer
    // reaches only once done here.
    constexpr int NBUF = 2 * DORD;
    constexpr size_t SL = (size_t)DSTAGE_MAX_WAVES * (PAIR ? 8 : 4) * 64;
    for (int m = mt; m >= bot; m -= DORD) {
        prefetch(m);
        inv_step<NCH, 0, SIDE, PAIR>(m, L, nx, n, an, good, ms, ring0, nreg, nsw, lane, w, W, lb, X, Y, E, fast, ct,
                                     ncs, initr, C, red, blk, partA, partB);
        if (m - 1 >= bot)
            inv_step<NCH, 1, SIDE, PAIR>(m - 1, L, nx, n, an, good, ms, ring0, nreg, nsw, lane, w, W, lb, X, Y, E, fast,
                                         ct, ncs, initr, C, red, blk, partA, partB);
        if (DORD == 4 && m - 2 >= bot) {
            prefetch(m - 2);
            inv_step<NCH, 0, SIDE, PAIR>(m - 2, L, nx, n, an, good, ms, ring0, nreg, nsw, lane, w, W, lb, X, Y, E, fast,
                                         ct, ncs, initr, C, red, blk, partA, partB);
            if (m - 3 >= bot)
                inv_step<NCH, 1, SIDE, PAIR>(m - 3, L, nx, n, an, good, ms, ring0, nreg, nsw, lane, w, W, lb, X, Y, E,
                                             fast, ct, ncs, initr, C, red, blk, partA, partB);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DORD; ++q)
            if (m - q >= bot)
                inv_reduce<SIDE, PAIR>(m - q, L, W, good, ms, ring0, nreg, nsw,
                                       red + (size_t)((m - q) & (NBUF - 1)) * SL, blk, partA, partB);
    }
    asm volatile("" ::"v"(pf));
}

// ------------------------------------------------------------------ forward d-stage
// Lanes = 64 consecutive l (group g); each wave owns 2 x SG contiguous ring
// slots (ring rbase + k; rings past the last regular ring are inert: zero
// lambda, zero H, never initialised); waves of a workgroup share the l-group
// and split the rings.  A workgroup runs group p then group G-1-p so all
// workgroups carry equal work.  At order m:
//   acc(l) = g_m^l sum_{slots} e * H[m][ring]   (e unscaled; see renorm),
// reduced over the waves in LDS (rotating reducers) and written to
// QA/QB[blk][l][m].  kappa and g of the next order are loaded one step ahead.

// LDS reduction buffers of the forward sweep.  A two-sided run keeps the four
// components of an order (A re, A im, B re, B im; W x 4 x 64 sums) in buffer m mod 4;
// a one-sided run (SIDE 1 / 2) keeps its two (re, im) in buffer m mod 8 of half the
// size, so the same LDS holds eight orders and its main loop reduces four orders per
// barrier.  A buffer is rewritten only after a barrier that follows its reduction:
// two consecutive barrier intervals never span more orders than there are buffers.
// fwd_boff1: offset of a one-sided run's buffer for order m.
__device__ __forceinline__ size_t fwd_boff1(int m, int W)
{
    return (size_t)(m & 7) * W * 2 * 64;
}

// A one-sided run's sums of this order to its LDS buffer (wave w, lane).
template <int SIDE>
__device__ __forceinline__ void fwd_put1(double *red, int m, int w, int W, int lane, double g, double aAr, double aAi,
                                         double aBr, double aBi)
{
    double *rb = red + fwd_boff1(m, W);
    rb[(w * 2 + 0) * 64 + lane] = (SIDE == 1 ? aAr : aBr) * g;
    rb[(w * 2 + 1) * 64 + lane] = (SIDE == 1 ? aAi : aBi) * g;
}

__device__ __forceinline__ const double2 *init_tab_ptr(const double2 *init, int r0, int m, int L)
{
    return init + (size_t)r0 * L + m;
}

template <int PAR, bool HEAD, bool REAL = false, int SIDE = 0>
__device__ __forceinline__ void fwd_chunk(double (&X)[SG], double (&Y)[SG], int (&E)[SG], const double *__restrict__ Lm,
                                          const double *__restrict__ HA, const double *__restrict__ HB, double kk,
                                          bool init, int nval, const double2 *__restrict__ iv, int istride, double &aAr,
                                          double &aAi, double &aBr, double &aBi)
{
#pragma unroll
    for (int k = 0; k < SG; ++k) {
        double &nw = PAR == 0 ? Y[k] : X[k];
        double &od = PAR == 0 ? X[k] : Y[k];
        nw = fma(kk * Lm[k], od, -nw);
        if constexpr (HEAD) {
            if (init && k < nval) {                      // l == m starts at slot k's ring (a swept ring)
                const double2 v = iv[(size_t)k * istride];
                nw = v.x;
                E[k] = (int)v.y;
                od = 0.0;
            }
        }
        const double t = nw;                             // unscaled (see renorm)
        const double *ha = HA + k * 4;                   // components chosen by the caller's offsets
        const double *hb = HB + k * 4;
        if constexpr (SIDE != 2) {
            aAr = fma(t, ha[0], aAr);
            aAi = fma(t, ha[1], aAi);
        }
        if constexpr (SIDE != 1) {
            aBr = fma(t, hb[0], aBr);
            aBi = fma(t, hb[1], aBi);
        }
    }
}

// HEAD: degrees of the group start in this pair of orders.  MAIN: m >= |n|
// (no low-order copies, no continuation outputs).  SAME (with MAIN, m > 0): both
// sides read one spectra array (run n = 0), so a ring's four components form one
// contiguous record and the wave's row is fetched with wide scalar loads.
// REAL (with MAIN): every chunk is realised (all E == 0), which stays so in the
// main loop since no degree starts there: no scaling and no renormalisation.
// SIDE 1 / 2: only the A side (order +m) or only the B side (order -m) is
// accumulated (a real signal's run n = 0, whose order -m is the conjugate; a
// spin-s sphere run, which feeds one side of its slice).
// PAIRF (run n = 0, N/S-symmetric sampling): the slots are the northern rings,
// the lanes of group g hold degrees of one parity (l = 128 (g/2) + 2 lane + g%2),
// and by d^l_{m,0}(pi - theta) = (-1)^{l+m} d^l_{m,0}(theta) a slot contributes
// d (H(ring) + (-1)^{l+m} H(mirror)): HA holds the sums and HB the differences of
// the two rings' spectra, and l + m has one parity across the wave at each order.
template <int NCH, int PAR, bool HEAD, bool MAIN = false, bool SAME = false, bool REAL = false, int SIDE = 0,
          bool PAIRF = false>
__device__ __forceinline__ void fwd_step(int m, int mend, int g, int l, int L, int nxp, int n, int an, int lane, int w,
                                         int W, int hstride, int lstride, int nreg, int rbase, double (&X)[NCH][SG],
                                         double (&Y)[NCH][SG], int (&E)[NCH][SG], uint32_t &real, double &kk, double &gm,
                                         const double *__restrict__ lam, const double2 *__restrict__ init,
                                         const double *__restrict__ kap, const double *__restrict__ gtab,
                                         const double *__restrict__ HA, const double *__restrict__ HB,
                                         const double *__restrict__ HxA, const double *__restrict__ HxB, double *red,
                                         int blk, double *__restrict__ QA, double *__restrict__ QB,
                                         double *__restrict__ QxA, double *__restrict__ QxB)
{
    // kappa / g of this order were loaded one step ahead; fetch the next order's now
    const double kcur = kk, gcur = gm;
    if (m - 1 >= mend) {
        const int mn = m - 1;
        const int lc = min(l, L - 1);
        kk = (l > mn && l < L) ? kap[(ptrdiff_t)mn * L + lc] : 0.0;
        gm = (l >= mn && l < L) ? gtab[(ptrdiff_t)mn * L + lc] : 0.0;
    }
    const bool starts = HEAD && (l == m) && (l >= an);
    // start values of slot k: init[rbase + k][m] (rings past nreg stay zero)
    double aAr = 0.0, aAi = 0.0, aBr = 0.0, aBi = 0.0;
    const double *Lm = lam + (ptrdiff_t)m * lstride + rbase;
    // Ring spectra of the two sides.  Orders below |n| read copies in which the
    // rings where this run is unstable are zero (the other run covers them); the
    // continuation (m <= 0) reads the A slice at order m < 0 (components 2,3) and
    // the B slice at order -m >= 0 (components 0,1).
    const int am = MAIN ? m : (m < 0 ? -m : m);
    const bool low = !MAIN && m < an;
    const double *HAm, *HBm;
    if constexpr (PAIRF) {
        HAm = (((m + g) & 1) ? HB : HA) + ((size_t)am * hstride + rbase) * 4;
        HBm = HAm + 2;
    } else {
        HAm = (low ? HxA : HA) + ((size_t)am * hstride + rbase) * 4 + (!MAIN && m < 0 ? 2 : 0);
        HBm = SAME ? HAm + 2 : (low ? HxB : HB) + ((size_t)am * hstride + rbase) * 4 + (m > 0 ? 2 : 0);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const double *Lc = Lm + c * SG;
        const double *Ac = HAm + c * SG * 4;
        const double *Bc = HBm + c * SG * 4;
        if (HEAD) {
            const int r0 = min(rbase + c * SG, nreg - 1);
            // slots at or past the last swept ring (MW south pole, padding) are never
            // started: they stay zero, and their start values lie outside the table
            const int nval = nreg - (rbase + c * SG);
            const bool ok = starts && nval > 0;
            fwd_chunk<PAR, true, false, SIDE>(X[c], Y[c], E[c], Lc, Ac, Bc, kcur, ok, nval,
                                              init_tab_ptr(init, r0, m < 0 ? 0 : m, L), L, aAr, aAi, aBr, aBi);
        } else {
            fwd_chunk<PAR, false, REAL, SIDE>(X[c], Y[c], E[c], Lc, Ac, Bc, kcur, false, 0, nullptr, 0, aAr, aAi, aBr,
                                              aBi);
        }
    }
    if (HEAD) real = 0u;                                  // degrees start in this group: not realised
    if (!REAL && (m & (RN - 1)) == 0) renorm_chunks<NCH>(X, Y, E, NCH, real);
    // this order's sums go to its LDS buffer; the caller reduces two orders after
    // one barrier (fwd_reduce2)
    if constexpr (SIDE == 0) {
        double *rb = red + (size_t)(m & 3) * W * 4 * 64;
        rb[(w * 4 + 0) * 64 + lane] = aAr * gcur;
        rb[(w * 4 + 1) * 64 + lane] = aAi * gcur;
        rb[(w * 4 + 2) * 64 + lane] = aBr * gcur;
        rb[(w * 4 + 3) * 64 + lane] = aBi * gcur;
    } else {
        fwd_put1<SIDE>(red, m, w, W, lane, gcur, aAr, aAi, aBr, aBi);
    }
}

// The main-loop order of a run whose two sides read one spectra array (SAME: run
// n = 0, m > 0; a paired sweep reads the sums or the differences by the order's
// parity, and the caller passes the row of the array that this order reads): the
// wave's lambda and spectra rows and the lane's kappa and g are reached through
// pointers that step back (hstep: the spectra row's step per call), so an order
// carries no index arithmetic, and kappa and g of the next order are plain loads (in
// the main loop every lane's degree has started, l > m; lanes past L read row
// entries of L - 1 and are never stored).
template <int NCH, int PAR, bool REAL, int SIDE>
__device__ __forceinline__ void fwd_step_same(int m, int lane, int w, int W, int L, double (&X)[NCH][SG],
                                              double (&Y)[NCH][SG], int (&E)[NCH][SG], uint32_t &real, double &kk,
                                              double &gm, const double *__restrict__ &Lp,
                                              const double *__restrict__ &Hp, const double *__restrict__ &kp,
                                              const double *__restrict__ &gp, int lstride, int hstep, double *red)
{
    const double kcur = kk, gcur = gm;
    kp -= L;
    gp -= L;
    kk = *kp;                                            // order m - 1
    gm = *gp;
    double aAr = 0.0, aAi = 0.0, aBr = 0.0, aBi = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        fwd_chunk<PAR, false, REAL, SIDE>(X[c], Y[c], E[c], Lp + c * SG, Hp + c * SG * 4, Hp + c * SG * 4 + 2, kcur,
                                          false, 0, nullptr, 0, aAr, aAi, aBr, aBi);
    Lp -= lstride;
    Hp -= hstep;
    if (!REAL && (m & (RN - 1)) == 0) renorm_chunks<NCH>(X, Y, E, NCH, real);
    if constexpr (SIDE == 0) {
        double *rb = red + (size_t)(m & 3) * W * 4 * 64;
        rb[(w * 4 + 0) * 64 + lane] = aAr * gcur;
        rb[(w * 4 + 1) * 64 + lane] = aAi * gcur;
        rb[(w * 4 + 2) * 64 + lane] = aBr * gcur;
        rb[(w * 4 + 3) * 64 + lane] = aBi * gcur;
    } else {
        fwd_put1<SIDE>(red, m, w, W, lane, gcur, aAr, aAi, aBr, aBi);
    }
}

// Sum of order m's partials over the WT waves (its LDS buffer) and its store to
// QA/QB[blk][l][m] (continuation orders m < 0: QxA/QxB).
template <int WT, bool MAIN, int SIDE, bool PAIRF>
__device__ __forceinline__ void fwd_reduce(int m, int g, int L, int nxp, int n, int an, const double *red, int blk,
                                           double *__restrict__ QA, double *__restrict__ QB, double *__restrict__ QxA,
                                           double *__restrict__ QxB)
{
    const double *rb = SIDE == 0 ? red + (size_t)(m & 3) * WT * 4 * 64 : red + fwd_boff1(m, WT);
    const int am = MAIN ? m : (m < 0 ? -m : m);
    const int tr = (int)threadIdx.x - 256 * reducer_group(m, WT);
    if (tr >= 0 && tr < 256 && (SIDE == 0 || (SIDE == 1) == (tr < 128))) {
        const int ll = tr & 63, comp = tr >> 6;
        const int lo = PAIRF ? 128 * (g >> 1) + 2 * ll + (g & 1) : 64 * g + ll;
        double s;
        if constexpr (SIDE == 0) s = wave_sum<WT>(rb, comp, ll, WT);
        else s = wave_sum<WT, 2>(rb, comp & 1, ll, WT);
        if (MAIN) {
            if (lo < L && lo >= m && (m > 0 || comp < 2)) {
                double *dst = comp < 2 ? QA : QB;
                if (dst) dst[(((size_t)blk * L + lo) * L + m) * 4 + comp] = s;
            }
        } else if (lo < L && lo >= m) {
            if (m > 0 || comp < 2) {
                if (m >= 0) {
                    double *dst = comp < 2 ? QA : QB;
                    if (dst) dst[(((size_t)blk * L + lo) * L + m) * 4 + comp] = s;
                } else if (QxA) {
                    // A slice at order m < 0; the sign cancels the one the finish applies to m < 0
                    const double sg = ((am + n) & 1) ? -s : s;
                    QxA[(((size_t)blk * L + lo) * nxp + am) * 4 + comp + 2] = sg;
                }
            } else if (an > 0 && QxB) {
                // B slice at order -m >= 0: d^l_{-m,-n} = (-1)^{m-n} d^l_{m,n}
                const double sg = ((am + n) & 1) ? -s : s;
                QxB[(((size_t)blk * L + lo) * nxp + am) * 4 + comp - 2] = sg;
            }
        }
    }
}

// One barrier, then the reductions of orders m and (two) m - 1, whose buffers are
// next written two iterations on or later, after the next barrier, which every
// reducer reaches only once done here.  With 8 or 16 waves the two orders go to
// different reducer groups.
template <int WT, bool MAIN, int SIDE, bool PAIRF>
__device__ __forceinline__ void fwd_reduce2(int m, bool two, int g, int L, int nxp, int n, int an, const double *red,
                                            int blk, double *__restrict__ QA, double *__restrict__ QB,
                                            double *__restrict__ QxA, double *__restrict__ QxB)
{
    __syncthreads();
    fwd_reduce<WT, MAIN, SIDE, PAIRF>(m, g, L, nxp, n, an, red, blk, QA, QB, QxA, QxB);
    if (two) fwd_reduce<WT, MAIN, SIDE, PAIRF>(m - 1, g, L, nxp, n, an, red, blk, QA, QB, QxA, QxB);
}

template <int NCH, bool SAME, int WT, int SIDE = 0, bool PAIRF = false>
__global__ __launch_bounds__(64 * WT) void k_dstage_fwd(
    int gx, int gy, int gz, bool xcd, int L, int nxp, int nreg, int hstride, int lstride, int n, int G,
    const double *__restrict__ lam, const double2 *__restrict__ init, const double *__restrict__ kap,
    const double *__restrict__ gtab, const double *__restrict__ HA, const double *__restrict__ HB,
    const double *__restrict__ HxA, const double *__restrict__ HxB, double *__restrict__ QA, double *__restrict__ QB,
    double *__restrict__ QxA, double *__restrict__ QxB, OrderTiles ot)
{
    __shared__ double red[4 * WT * 4 * 64];         // four order buffers of WT x 4 x 64 sums
    const int an = n < 0 ? -n : n;
    const int mend = an > 1 ? -(an - 1) : 0;            // continuation below m = 0
    const int lane = threadIdx.x & 63;
    const int w = ufl(threadIdx.x >> 6);
    constexpr int W = WT;                                // waves per workgroup (== blockDim.x / 64)
    // l-group pair p, ring block blk, order tile bz (xcd: each XCD takes contiguous
    // pairs, so the workgroups of one ring block read its spectra rows through one L2)
    int p, blk, bz;
    if (!xcd_tile(gx, gy, gz, p, blk, bz, xcd)) return;
    // this wave's rings: rbase .. rbase + NCH SG - 1 (contiguous; >= nreg inert)
    const int rbase = (blk * W + w) * NCH * SG;
    // order tile bz: orders ctop - 1 .. lo
    const int tile = bz;
    const int ctop = tile == 0 ? L : ot.c[tile];
    const int lo = tile + 1 < ot.nt ? ot.c[tile + 1] : mend;

    for (int pass = 0; pass < 2; ++pass) {
        const int g = pass == 0 ? p : G - 1 - p;
        if (pass == 1 && g == p) break;
        const int lmin = PAIRF ? 128 * (g >> 1) + (g & 1) : 64 * g;     // lowest degree of the group
        const int l = PAIRF ? lmin + 2 * lane : lmin + lane;
        double X[NCH][SG], Y[NCH][SG];
        int E[NCH][SG];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int k = 0; k < SG; ++k) { X[c][k] = 0.0; Y[c][k] = 0.0; E[c][k] = 0; }
        uint32_t real = 0u;
        const int mstart = min(PAIRF ? lmin + 126 : lmin + 63, L - 1);
        // head: the orders at which lanes of this group start (an even number of
        // steps so the register roles line up with the main loop)
        const int hend = ((mstart - lmin + 1) % 2 == 0) ? lmin : lmin - 1;
        int m = min(mstart, ctop - 1);
        if (m < lo) continue;                            // the group's degrees lie below the tile
        if (tile > 0 && l >= ctop && l < L) {
            // lanes whose degree started above the tile resume from the stored state
            // (PAR 0 at order ctop - 1: X holds e_{ctop}); slots past the swept rings stay zero
            const double *q = ot.ck + ot.off[tile] + (size_t)(l - ctop) * 3 * ot.rp + rbase;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int k = 0; k < SG; ++k)
                    if (rbase + c * SG + k < nreg) {
                        X[c][k] = q[c * SG + k];
                        Y[c][k] = q[ot.rp + c * SG + k];
                        E[c][k] = (int)q[2 * ot.rp + c * SG + k];
                    }
        }
        const int lc = min(l, L - 1);
        double kk = (l > m && l < L) ? kap[(ptrdiff_t)m * L + lc] : 0.0;
        double gm = (l >= m && l < L) ? gtab[(ptrdiff_t)m * L + lc] : 0.0;
        // Pull the wave's lambda and spectra rows of orders m - PFF, m - PFF - 1 toward
        // the caches (one dword per 128-byte line, PQ lanes per order); the result is
        // consumed only at the next pair of orders, so the latency overlaps their work.
        constexpr int HL = NCH * SG * 4 * 8 / 128;           // 128-byte lines of one side's spectra row
        constexpr int PQ = 1 + 2 * HL;
        constexpr int PFF = PFD;
        int pf = 0;
        auto prefetch = [&](int mm) {
            asm volatile("" ::"v"(pf));
            const int mp = mm - PFF - (lane >= PQ ? 1 : 0);
            const int q = lane % PQ;
            if (lane < 2 * PQ && mp >= an) {
                // q = 0: the wave's lambdas; q = 1..HL / HL+1..2HL: the spectra rows of the two sides
                const int *a;
                if (q == 0) a = reinterpret_cast<const int *>(lam + (ptrdiff_t)mp * lstride + rbase);
                else if (q <= HL) a = reinterpret_cast<const int *>(HA + ((size_t)mp * hstride + rbase) * 4) + (q - 1) * 32;
                else a = reinterpret_cast<const int *>(HB + ((size_t)mp * hstride + rbase) * 4) + (q - 1 - HL) * 32;
                pf = *a;
            }
        };
        for (; m >= hend && m >= lo; m -= 2) {
            prefetch(m);
            fwd_step<NCH, 0, true, false, false, false, SIDE, PAIRF>(m, mend, g, l, L, nxp, n, an, lane, w, W, hstride,
                                                              lstride, nreg, rbase, X, Y, E, real, kk, gm, lam, init,
                                                              kap, gtab, HA, HB, HxA, HxB, red, blk, QA, QB, QxA, QxB);
            if (m - 1 >= lo)
                fwd_step<NCH, 1, true, false, false, false, SIDE, PAIRF>(m - 1, mend, g, l, L, nxp, n, an, lane, w, W,
                                                                  hstride, lstride, nreg, rbase, X, Y, E, real, kk, gm,
                                                                  lam, init, kap, gtab, HA, HB, HxA, HxB, red, blk, QA,
                                                                  QB, QxA, QxB);
            fwd_reduce2<WT, false, SIDE, PAIRF>(m, m - 1 >= lo, g, L, nxp, n, an, red, blk, QA, QB, QxA, QxB);
        }
        // both orders of the pair >= |n| (and > 0 when the sides share one array) and
        // in the tile
        constexpr uint32_t ALL = (1u << NCH) - 1u;
        const int mlo = max(SAME ? max(an, 1) : an, lo);
        if constexpr (SAME) {
            // Main loop with every per-order address stepped, not recomputed: the wave's
            // lambda and spectra rows, the lane's kappa / g, the prefetch lanes' lines and
            // each reducer thread's output column move back one order per step.
            // PAIRF: order m reads the sums (HA) or the differences (HB) by the parity of
            // m + g; the loop takes two orders per iteration, so each of its two steps
            // keeps one array and steps its row back two orders at a time.
            const bool hodd = PAIRF && ((m + g) & 1);
            const double *Lp = lam + (ptrdiff_t)m * lstride + rbase;
            const double *Hp = (hodd ? HB : HA) + ((size_t)m * hstride + rbase) * 4;
            const double *Hq = PAIRF ? (hodd ? HA : HB) + ((ptrdiff_t)(m - 1) * hstride + rbase) * 4 : nullptr;
            const double *kp = kap + (ptrdiff_t)m * L + lc;      // kk, gm hold order m already
            const double *gp = gtab + (ptrdiff_t)m * L + lc;
            const int hstep = hstride * 4;
            // prefetch: lanes [0, PS) pull the rows of order m - PFF, lanes [PS, 2 PS) those
            // of order m - PFF - 1 (lane q of a row: the lambdas for q = 0, else one
            // 128-byte line of the spectra row); both sides share the spectra
            constexpr int PS = 1 + HL;
            const int q = lane % PS;
            int pm = m - PFF - (lane >= PS ? 1 : 0);
            const double *HP = (PAIRF && ((pm + g) & 1)) ? HB : HA;    // a lane's rows keep their parity
            const char *pa = q == 0 ? reinterpret_cast<const char *>(lam + (ptrdiff_t)pm * lstride + rbase)
                                    : reinterpret_cast<const char *>(HP + ((ptrdiff_t)pm * hstride + rbase) * 4) +
                                          (q - 1) * 128;
            const ptrdiff_t pstep = q == 0 ? 2 * (ptrdiff_t)lstride * 8 : 2 * (ptrdiff_t)hstride * 32;
            const bool plane = lane < 2 * PS;
            // reducer thread (group threadIdx / 256, component, lane): its output column
            // at order m is dcol[m * 4] (every order of the main loop is > 0 and < l)
            const int rgrp = (int)threadIdx.x >> 8;
            const int rcomp = ((int)threadIdx.x >> 6) & 3;
            const int lo = PAIRF ? 128 * (g >> 1) + 2 * lane + (g & 1) : 64 * g + lane;
            double *dbase = rcomp < 2 ? QA : QB;
            const bool rok = lo < L && dbase != nullptr && (SIDE == 0 || (SIDE == 1) == (rcomp < 2));
            double *dcol = rok ? dbase + (((size_t)blk * L + lo) * L) * 4 + rcomp : nullptr;
            auto reduce_pair = [&](int mm) {
                __syncthreads();
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const int mo = mm - o;
                    if (rok && rgrp == reducer_group(mo, WT)) {
                        if constexpr (SIDE == 0) {
                            const double *rb = red + (size_t)(mo & 3) * WT * 4 * 64;
                            dcol[(size_t)mo * 4] = wave_sum<WT>(rb, rcomp, lane, WT);
                        } else {
                            dcol[(size_t)mo * 4] = wave_sum<WT, 2>(red + fwd_boff1(mo, WT), rcomp & 1, lane, WT);
                        }
                    }
                }
            };
            // one-sided runs: one barrier, then the reductions of four orders (a rolled
            // loop, so that the loads of one order's sum are live at a time)
            auto reduce_quad = [&](int mm) {
                __syncthreads();
#pragma unroll 1
                for (int o = 0; o < 4; ++o) {
                    const int mo = mm - o;
                    if (rok && rgrp == reducer_group(mo, WT)) {
                        dcol[(size_t)mo * 4] = wave_sum<WT, 2>(red + fwd_boff1(mo, WT), rcomp & 1, lane, WT);
                    }
                }
            };
            auto pull = [&]() {
                asm volatile("" ::"v"(pf));
                if (plane && pm >= an) pf = *reinterpret_cast<const int *>(pa);
                pa -= pstep;
                pm -= 2;
            };
            // one order's step; PAIRF: the second order of each pair reads Hq
            constexpr int HST = PAIRF ? 2 : 1;
            // two orders per iteration; a one-sided run reduces after every second
            // iteration (four orders per barrier), the last pair pending at most (not
            // the paired one-sided run: there the deferral costs registers and spills)
            bool pend = false;
            for (; m - 1 >= mlo && real != ALL; m -= 2) {
                pull();
                fwd_step_same<NCH, 0, false, SIDE>(m, lane, w, W, L, X, Y, E, real, kk, gm, Lp, Hp, kp, gp, lstride,
                                                   HST * hstep, red);
                fwd_step_same<NCH, 1, false, SIDE>(m - 1, lane, w, W, L, X, Y, E, real, kk, gm, Lp, PAIRF ? Hq : Hp,
                                                   kp, gp, lstride, HST * hstep, red);
                if constexpr (SIDE == 0 || PAIRF) {
                    reduce_pair(m);
                } else {
                    if (pend) reduce_quad(m + 2);
                    pend = !pend;
                }
            }
            for (; m - 1 >= mlo; m -= 2) {               // realised: plain contributions
                pull();
                fwd_step_same<NCH, 0, true, SIDE>(m, lane, w, W, L, X, Y, E, real, kk, gm, Lp, Hp, kp, gp, lstride,
                                                  HST * hstep, red);
                fwd_step_same<NCH, 1, true, SIDE>(m - 1, lane, w, W, L, X, Y, E, real, kk, gm, Lp, PAIRF ? Hq : Hp,
                                                  kp, gp, lstride, HST * hstep, red);
                if constexpr (SIDE == 0 || PAIRF) {
                    reduce_pair(m);
                } else {
                    if (pend) reduce_quad(m + 2);
                    pend = !pend;
                }
            }
            if constexpr (SIDE != 0 && !PAIRF)
                if (pend) reduce_pair(m + 2);            // the last pair's orders m + 2, m + 1
        }
        for (; m - 1 >= mlo && real != ALL; m -= 2) {
            prefetch(m);
            fwd_step<NCH, 0, false, true, SAME, false, SIDE, PAIRF>(m, mend, g, l, L, nxp, n, an, lane, w, W, hstride,
                                                             lstride, nreg, rbase, X, Y, E, real, kk, gm, lam, init,
                                                             kap, gtab, HA, HB, HxA, HxB, red, blk, QA, QB, QxA, QxB);
            fwd_step<NCH, 1, false, true, SAME, false, SIDE, PAIRF>(m - 1, mend, g, l, L, nxp, n, an, lane, w, W, hstride,
                                                             lstride, nreg, rbase, X, Y, E, real, kk, gm, lam, init,
                                                             kap, gtab, HA, HB, HxA, HxB, red, blk, QA, QB, QxA, QxB);
            fwd_reduce2<WT, true, SIDE, PAIRF>(m, true, g, L, nxp, n, an, red, blk, QA, QB, QxA, QxB);
        }
        for (; m - 1 >= mlo; m -= 2) {                   // realised: plain contributions
            prefetch(m);
            fwd_step<NCH, 0, false, true, SAME, true, SIDE, PAIRF>(m, mend, g, l, L, nxp, n, an, lane, w, W, hstride,
                                                            lstride, nreg, rbase, X, Y, E, real, kk, gm, lam, init,
                                                            kap, gtab, HA, HB, HxA, HxB, red, blk, QA, QB, QxA, QxB);
            fwd_step<NCH, 1, false, true, SAME, true, SIDE, PAIRF>(m - 1, mend, g, l, L, nxp, n, an, lane, w, W, hstride,
                                                            lstride, nreg, rbase, X, Y, E, real, kk, gm, lam, init,
                                                            kap, gtab, HA, HB, HxA, HxB, red, blk, QA, QB, QxA, QxB);
            fwd_reduce2<WT, true, SIDE, PAIRF>(m, true, g, L, nxp, n, an, red, blk, QA, QB, QxA, QxB);
        }
        for (; m >= lo; m -= 2) {
            prefetch(m);
            fwd_step<NCH, 0, false, false, false, false, SIDE, PAIRF>(m, mend, g, l, L, nxp, n, an, lane, w, W, hstride,
                                                               lstride, nreg, rbase, X, Y, E, real, kk, gm, lam, init,
                                                               kap, gtab, HA, HB, HxA, HxB, red, blk, QA, QB, QxA, QxB);
            if (m - 1 >= lo)
                fwd_step<NCH, 1, false, false, false, false, SIDE, PAIRF>(m - 1, mend, g, l, L, nxp, n, an, lane, w, W,
                                                                   hstride, lstride, nreg, rbase, X, Y, E, real, kk,
                                                                   gm, lam, init, kap, gtab, HA, HB, HxA, HxB, red,
                                                                   blk, QA, QB, QxA, QxB);
            fwd_reduce2<WT, false, SIDE, PAIRF>(m, m - 1 >= lo, g, L, nxp, n, an, red, blk, QA, QB, QxA, QxB);
        }
        asm volatile("" ::"v"(pf));
        __syncthreads();   // the LDS buffers are reused by the next pass
    }
}

// Sums and differences of the spectra of a ring and its mirror for the paired
// forward sweep: S[m][i] = H[m][i] + H[m][nreg-1-i], D[m][i] = H[m][i] -
// H[m][nreg-1-i] over whole 32-byte records (both sides); a ring that is its own
// mirror (the equator) enters once: S = D = H.  Pairs past nsw are zero padding.
__global__ void k_pair_spectra(int L, int nreg, int nsw, int hstride, int pstride, const double *__restrict__ H,
                               double *__restrict__ S, double *__restrict__ D)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)L * pstride) return;
    const int m = (int)(i / pstride), r = (int)(i % pstride);
    double4 a = make_double4(0.0, 0.0, 0.0, 0.0), b = a;
    if (r < nsw) {
        a = *reinterpret_cast<const double4 *>(H + ((size_t)m * hstride + r) * 4);
        const int rm = nreg - 1 - r;
        if (rm != r) {
            const double4 c = *reinterpret_cast<const double4 *>(H + ((size_t)m * hstride + rm) * 4);
            b = make_double4(a.x - c.x, a.y - c.y, a.z - c.z, a.w - c.w);
            a = make_double4(a.x + c.x, a.y + c.y, a.z + c.z, a.w + c.w);
        } else {
            b = a;
        }
    }
    *reinterpret_cast<double4 *>(S + ((size_t)m * pstride + r) * 4) = a;
    *reinterpret_cast<double4 *>(D + ((size_t)m * pstride + r) * 4) = b;
}

// Copies of the two sides' ring spectra at orders mu < |n| for the forward sweep
// of run n, restricted to the rings whose values this run supplies (switch
// order ms of the ring): the own orders (A components 0,1 at mu >= 0, B
// components 2,3 at mu > 0) where the run is stable or mu >= ms, and the
// continuation orders (A components 2,3 = A slice at -mu, B components 0,1 = B
// slice at +mu) where the run is the stable one and mu < ms.  Other entries 0.
__global__ void k_mask_low(int an_run, int n, int nreg, int hstride, const double *__restrict__ cot,
                           const double *__restrict__ csc, const double *__restrict__ FA,
                           const double *__restrict__ FB, double *__restrict__ HxA, double *__restrict__ HxB)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)an_run * hstride) return;
    const int r = (int)(i % hstride), mu = (int)(i / hstride);
    bool own = false, ext = false;
    if (r < nreg) {
        const double ct = cot[r];
        const bool good = ring_good(n, ct);
        const int ms = switch_order(n, ct, csc[r]);
        own = good || mu >= ms;
        ext = good && mu < ms;
    }
    HxA[i * 4 + 0] = own ? FA[i * 4 + 0] : 0.0;
    HxA[i * 4 + 1] = own ? FA[i * 4 + 1] : 0.0;
    HxA[i * 4 + 2] = ext ? FA[i * 4 + 2] : 0.0;
    HxA[i * 4 + 3] = ext ? FA[i * 4 + 3] : 0.0;
    HxB[i * 4 + 0] = ext ? FB[i * 4 + 0] : 0.0;
    HxB[i * 4 + 1] = ext ? FB[i * 4 + 1] : 0.0;
    HxB[i * 4 + 2] = own ? FB[i * 4 + 2] : 0.0;
    HxB[i * 4 + 3] = own ? FB[i * 4 + 3] : 0.0;
}

// 2 lambda table for the forward sweep: lam[m][r] = n csc_r - (m+1) cot_r
// (the same FMA the inverse sweep evaluates inline).
// Rows are padded to lstride rings; padding rings get lambda = 0 (inert).
__global__ void k_lambda_table(int L, int nx, int nreg, int lstride, int n, const double *__restrict__ cot,
                               const double *__restrict__ csc, double *__restrict__ lam)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // rows m in [-nx, L), lam at row 0
    if (i >= (size_t)(L + nx) * lstride) return;
    const int m = (int)(i / lstride) - nx, r = (int)(i % lstride);
    lam[(ptrdiff_t)m * lstride + r] = r < nreg ? fma(-(double)(m + 1), cot[r], (double)n * csc[r]) : 0.0;
}

// ------------------------------------------------------------------ phi-DFT: inverse
// One workgroup per (map, ring).  X_k = ftilde at orders m == k mod nphi
// (summed over the d-stage blocks), times the ring's half-pixel phase, then an
// inverse DFT of length nphi.  MW rings: nphi = 2L-1 and the order line maps
// one-to-one onto the bins.  The MW south pole (ring == nreg) has the closed
// form d^l_{m,-s}(pi) = (-1)^{l+m} delta_{m,s} (Eq. 29).
__global__ __launch_bounds__(1024) void k_phi_inv(
    int L, int nreg, int nblk, int spin, const double *__restrict__ part, const int *__restrict__ mtop,
    const double2 *__restrict__ flm,
    const double *__restrict__ wl, const int *__restrict__ ring_nphi, const long long *__restrict__ ring_start,
    const int *__restrict__ ring_shift, const int *__restrict__ ring_fft, const FftArgs *__restrict__ ffts,
    double2 *__restrict__ map, double2 *__restrict__ fscr)
{
    extern __shared__ double2 buf[];
    __shared__ double2 red[1024];
    const int r = blockIdx.x;
    const int T = blockDim.x, tid = threadIdx.x;
    const int nphi = ring_nphi[r];
    const FftArgs *f = ffts + ring_fft[r];
    const int shift = ring_shift[r];
    const int M = 2 * L - 1;
    if (r < nreg && nphi >= M) {
        // at most one order per bin (MW, and rings of nphi >= 2L - 1 samples: HEALPix
        // belt, DH, MWSS): a thread per |m| reads whole 32-byte records (order +|m| in
        // components 0,1, order -|m| in 2,3) and fills bins |m| and nphi - |m|; the bins
        // L .. nphi - L that no order reaches are zero
        for (int k = L + tid; k <= nphi - L; k += T) buf[k] = make_double2(0.0, 0.0);
        const double *pr = part + (size_t)r * L * 4;
        const size_t bstride = (size_t)nreg * L * 4;
        for (int am = tid; am < L; am += T) {
            double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
            for (int b = 0; b < nblk; ++b) {
                if (am > mtop[b]) continue;                  // that block's sweep never reached order am
                const double2 *pp = reinterpret_cast<const double2 *>(pr + b * bstride + am * 4);
                va = cadd(va, pp[0]);
                vb = cadd(vb, pp[1]);
            }
            if (shift) {
                double s, c;   // e^{+- i pi am / nphi}
                sincospi((double)(am % (2 * nphi)) / (double)nphi, &s, &c);
                va = cmul(va, make_double2(c, s));
                vb = cmul(vb, make_double2(c, -s));
            }
            buf[am] = va;
            if (am > 0) buf[nphi - am] = vb;
        }
    } else if (r < nreg) {
        // Bin k sums the orders m = k + q nphi within [-(L-1), L-1].  A short ring (nphi
        // below the thread count, HEALPix caps) spreads each bin's orders over `per`
        // threads, j-th taking every per-th order, and adds their sums in a fixed order.
        const double *pr = part + (size_t)r * L * 4;
        const size_t bstride = (size_t)nreg * L * 4;
        const int per = nphi >= T ? 1 : T / nphi;
        auto bin_sum = [&](int k, int j) {
            double2 acc = make_double2(0.0, 0.0);
            for (int m = k - ((k + L - 1) / nphi) * nphi + j * nphi; m <= L - 1; m += per * nphi) {
                const int am = m < 0 ? -m : m;
                const int off = am * 4 + (m < 0 ? 2 : 0);
                double2 v = make_double2(0.0, 0.0);
                for (int b = 0; b < nblk; ++b) {
                    if (am > mtop[b]) continue;              // that block's sweep never reached order m
                    const double *pp = pr + b * bstride + off;
                    v.x += pp[0];
                    v.y += pp[1];
                }
                if (shift) {
                    double s, c;   // e^{i pi m / nphi}
                    sincospi((double)(((long long)m % (2 * nphi) + 2 * nphi) % (2 * nphi)) / (double)nphi, &s, &c);
                    v = cmul(v, make_double2(c, s));
                }
                acc = cadd(acc, v);
            }
            return acc;
        };
        if (per == 1) {
            for (int k = tid; k < nphi; k += T) buf[k] = bin_sum(k, 0);
        } else {                                               // uniform over the workgroup
            if (tid < per * nphi) red[tid] = bin_sum(tid % nphi, tid / nphi);
            __syncthreads();
            for (int k = tid; k < nphi; k += T) {
                double2 acc = red[k];
                for (int j = 1; j < per; ++j) acc = cadd(acc, red[k + j * nphi]);
                buf[k] = acc;
            }
        }
    } else {
        // south pole (ring nreg): only m = s contributes, value sum_l (-1)^{l+s} w_l flm[l][s];
        // north pole (ring nreg + 1, MWSS): only m = -s, value sum_l w_l flm[l][-s]  (Eq. 29)
        const bool north = r > nreg;
        const int mp = north ? -spin : spin;
        double2 acc = make_double2(0.0, 0.0);
        const int as = spin < 0 ? -spin : spin;
        for (int l = as + tid; l < L; l += T) {
            double2 v = flm[(size_t)l * M + (L - 1) + mp];
            const double c = (!north && ((l + spin) & 1)) ? -wl[l] : wl[l];
            acc.x += c * v.x;
            acc.y += c * v.y;
        }
        red[tid] = acc;
        __syncthreads();
        int p2 = 1;
        while (p2 < T) p2 <<= 1;
        for (int s = p2 / 2; s > 0; s >>= 1) {   // T need not be a power of two
            if (tid < s && tid + s < T) red[tid] = cadd(red[tid], red[tid + s]);
            __syncthreads();
        }
        for (int k = tid; k < nphi; k += T) buf[k] = make_double2(0.0, 0.0);
        __syncthreads();
        if (tid == 0) buf[((mp % nphi) + nphi) % nphi] = red[0];
    }
    __syncthreads();
    dft_lds(buf, f, +1, fscr ? fscr + (size_t)blockIdx.x * FFT_SCRATCH : nullptr);
    double2 *out = map + ring_start[r];
    for (int k = tid; k < nphi; k += T) out[k] = buf[k];
}

// ------------------------------------------------------------------ phi-DFT: forward
// One workgroup per (map, ring): X = DFT_nphi(ring); ftilde_m = q e^{-i pi m s_r/nphi} X[m mod nphi]
// for |m| < L (the periodic repeat of Sec. 4.2 for short HEALPix rings), written
// to F[m][ring] = {ftilde_m, ftilde_-m}.
__global__ __launch_bounds__(1024) void k_phi_fwd(
    int L, int nring, int hstride, double q, const double2 *__restrict__ map, const int *__restrict__ ring_nphi,
    const long long *__restrict__ ring_start, const int *__restrict__ ring_shift,
    const int *__restrict__ ring_fft, const FftArgs *__restrict__ ffts, const double *__restrict__ ringq,
    double *__restrict__ F, double2 *__restrict__ fscr)
{
    extern __shared__ double2 buf[];
    const int r = blockIdx.x;
    const int T = blockDim.x, tid = threadIdx.x;
    if (r >= nring) {                       // padding rings of the forward sweep: zeros
        for (int m = tid; m < L; m += T) {
            double *o = F + ((size_t)m * hstride + r) * 4;
            *reinterpret_cast<double2 *>(o) = make_double2(0.0, 0.0);
            *reinterpret_cast<double2 *>(o + 2) = make_double2(0.0, 0.0);
        }
        return;
    }
    const int nphi = ring_nphi[r];
    const FftArgs *f = ffts + ring_fft[r];
    const int shift = ring_shift[r];
    if (ringq) q = ringq[r];                     // per-ring quadrature weight (DH, GL)
    const double2 *in = map + ring_start[r];
    for (int k = tid; k < nphi; k += T) buf[k] = in[k];
    __syncthreads();
    dft_lds(buf, f, -1, fscr ? fscr + (size_t)blockIdx.x * FFT_SCRATCH : nullptr);
    for (int m = tid; m < L; m += T) {
        double2 a = buf[m % nphi];
        double2 b = buf[(nphi - (m % nphi)) % nphi];
        if (shift) {
            double s, c;   // e^{-i pi m / nphi}
            sincospi((double)(m % (2 * nphi)) / (double)nphi, &s, &c);
            a = cmul(a, make_double2(c, -s));
            b = cmul(b, make_double2(c, s));
        }
        double *o = F + ((size_t)m * hstride + r) * 4;
        *reinterpret_cast<double2 *>(o) = make_double2(q * a.x, q * a.y);
        *reinterpret_cast<double2 *>(o + 2) = make_double2(q * b.x, q * b.y);
    }
}

// ------------------------------------------------------------------ phi-DFTs of real signals
// Spin 0.  The spectrum of a real ring is Hermitian (X[-k] = conj X[k], X[0]
// real), so two rings of equal length and phase offset share one complex DFT:
// ring r1 in the real and ring r2 in the imaginary part of z = x1 + i x2, with
// Z = X1 + i X2.  One workgroup per pair (r2 < 0: r1 alone); the pairs are
// built on the host.
//
// Inverse: the order-m spectrum of a swept ring is the sweep's side A (summed
// over its blocks) for m >= 0 and its conjugate for m < 0; the poles (MW south
// ring nreg, MWSS north ring nreg + 1) hold only order 0, sum_l (+-1)^l w_l
// Re flm[l][0] (Eq. 29).  Order 0 enters with its real part: the result is the
// real part of the complex transform of the Hermitian completion of the orders
// m >= 0.  Rings of 2L-1 samples without offset map orders one-to-one onto
// bins; other rings sum the orders of each bin (HEALPix repeat) with the
// half-pixel phase.
__global__ __launch_bounds__(1024) void k_phi_inv_real(
    int L, int nreg, int nblk, const int *__restrict__ pairs, const double *__restrict__ part,
    const int *__restrict__ mtop, const double2 *__restrict__ flm, const double *__restrict__ wl,
    const int *__restrict__ ring_nphi, const long long *__restrict__ ring_start, const int *__restrict__ ring_shift,
    const int *__restrict__ ring_fft, const FftArgs *__restrict__ ffts, double *__restrict__ map,
    double2 *__restrict__ fscr)
{
    extern __shared__ double2 buf[];
    __shared__ double2 red[1024];
    const int r1 = pairs[2 * blockIdx.x], r2 = pairs[2 * blockIdx.x + 1];
    const int T = blockDim.x, tid = threadIdx.x;
    const int M = 2 * L - 1;
    const int nphi = ring_nphi[r1];
    const FftArgs *f = ffts + ring_fft[r1];
    const int shift = ring_shift[r1];
    double2 pole = make_double2(0.0, 0.0);                 // (south, north) order-0 values
    if (r1 >= nreg || r2 >= nreg) {                        // uniform over the workgroup
        double2 acc = make_double2(0.0, 0.0);
        for (int l = tid; l < L; l += T) {
            const double v = wl[l] * flm[(size_t)l * M + (L - 1)].x;
            acc.x += (l & 1) ? -v : v;
            acc.y += v;
        }
        red[tid] = acc;
        __syncthreads();
        int p2 = 1;
        while (p2 < T) p2 <<= 1;
        for (int h = p2 / 2; h > 0; h >>= 1) {           // T need not be a power of two
            if (tid < h && tid + h < T) red[tid] = cadd(red[tid], red[tid + h]);
            __syncthreads();
        }
        pole = red[0];
    }
    const size_t bstride = (size_t)nreg * L * 4;
    auto spec = [&](int r, int am) {                       // order +am of ring r (real part only at am = 0)
        double2 v = make_double2(0.0, 0.0);
        if (r < 0) return v;
        if (r < nreg) {
            const double *pr = part + ((size_t)r * L + am) * 4;
            for (int b = 0; b < nblk; ++b) {
                if (am > mtop[b]) continue;                  // that block's sweep never reached order am
                v = cadd(v, *reinterpret_cast<const double2 *>(pr + b * bstride));
            }
        } else if (am == 0) {
            v.x = r == nreg ? pole.x : pole.y;
        }
        if (am == 0) v.y = 0.0;
        return v;
    };
    if (nphi == M && !shift) {
        for (int am = tid; am < L; am += T) {
            const double2 x1 = spec(r1, am), x2 = spec(r2, am);
            buf[am] = make_double2(x1.x - x2.y, x1.y + x2.x);                      // X1 + i X2
            if (am > 0) buf[M - am] = make_double2(x1.x + x2.y, x2.x - x1.y);     // conj X1 + i conj X2
        }
    } else {
        // bins sum the orders = k mod nphi; short rings spread a bin over `per` threads
        // (fixed-order combination, as in the complex inverse)
        const int per = nphi >= T ? 1 : T / nphi;
        auto bin_sum = [&](int k, int j) {
            double2 z = make_double2(0.0, 0.0);
            for (int m = k - ((k + L - 1) / nphi) * nphi + j * nphi; m <= L - 1; m += per * nphi) {
                const int am = m < 0 ? -m : m;
                double2 x1 = spec(r1, am), x2 = spec(r2, am);
                if (m < 0) { x1 = cconj(x1); x2 = cconj(x2); }
                if (shift) {
                    double sn, cs;   // e^{i pi m / nphi}
                    sincospi((double)(((long long)m % (2 * nphi) + 2 * nphi) % (2 * nphi)) / (double)nphi, &sn, &cs);
                    x1 = cmul(x1, make_double2(cs, sn));
                    x2 = cmul(x2, make_double2(cs, sn));
                }
                z.x += x1.x - x2.y;
                z.y += x1.y + x2.x;
            }
            return z;
        };
        if (per == 1) {
            for (int k = tid; k < nphi; k += T) buf[k] = bin_sum(k, 0);
        } else {
            __syncthreads();                                   // red may still hold the pole sums
            if (tid < per * nphi) red[tid] = bin_sum(tid % nphi, tid / nphi);
            __syncthreads();
            for (int k = tid; k < nphi; k += T) {
                double2 z = red[k];
                for (int j = 1; j < per; ++j) z = cadd(z, red[k + j * nphi]);
                buf[k] = z;
            }
        }
    }
    __syncthreads();
    dft_lds(buf, f, +1, fscr ? fscr + (size_t)blockIdx.x * FFT_SCRATCH : nullptr);
    double *o1 = map + ring_start[r1];
    double *o2 = r2 >= 0 ? map + ring_start[r2] : nullptr;
    for (int k = tid; k < nphi; k += T) {
        o1[k] = buf[k].x;
        if (o2) o2[k] = buf[k].y;
    }
}

// Forward: Z = DFT(x1 + i x2), X1[k] = (Z[k] + conj Z[-k]) / 2, X2[k] = (Z[k] -
// conj Z[-k]) / 2i; order m >= 0 of a ring is q e^{-i pi m s/nphi} X[m mod nphi]
// (q per ring for DH / GL), written as F[m][ring] = {X_m, conj X_m} (the layout
// of the complex phi-DFT).  Workgroups past the pairs zero the sweep's padding
// rings nring .. hstride-1, two per workgroup.
__global__ __launch_bounds__(1024) void k_phi_fwd_real(
    int L, int nring, int hstride, int npair, double q, const int *__restrict__ pairs, const double *__restrict__ map,
    const int *__restrict__ ring_nphi, const long long *__restrict__ ring_start, const int *__restrict__ ring_shift,
    const int *__restrict__ ring_fft, const FftArgs *__restrict__ ffts, const double *__restrict__ ringq,
    double *__restrict__ F, double2 *__restrict__ fscr)
{
    extern __shared__ double2 buf[];
    const int T = blockDim.x, tid = threadIdx.x;
    if ((int)blockIdx.x >= npair) {
        const int r0 = nring + 2 * ((int)blockIdx.x - npair);
        for (int m = tid; m < L; m += T)
            for (int r = r0; r < r0 + 2 && r < hstride; ++r) {
                double2 *o = reinterpret_cast<double2 *>(F + ((size_t)m * hstride + r) * 4);
                o[0] = make_double2(0.0, 0.0);
                o[1] = make_double2(0.0, 0.0);
            }
        return;
    }
    const int r1 = pairs[2 * blockIdx.x], r2 = pairs[2 * blockIdx.x + 1];
    const int nphi = ring_nphi[r1];
    const FftArgs *f = ffts + ring_fft[r1];
    const int shift = ring_shift[r1];
    const double q1 = 0.5 * (ringq ? ringq[r1] : q);
    const double q2 = 0.5 * (ringq && r2 >= 0 ? ringq[r2] : q);
    const double *x1 = map + ring_start[r1];
    const double *x2 = r2 >= 0 ? map + ring_start[r2] : nullptr;
    for (int k = tid; k < nphi; k += T) buf[k] = make_double2(x1[k], x2 ? x2[k] : 0.0);
    __syncthreads();
    dft_lds(buf, f, -1, fscr ? fscr + (size_t)blockIdx.x * FFT_SCRATCH : nullptr);
    for (int m = tid; m < L; m += T) {
        const int b = m % nphi;
        const double2 z = buf[b];
        const double2 zc = cconj(buf[b == 0 ? 0 : nphi - b]);
        double2 a = make_double2(q1 * (z.x + zc.x), q1 * (z.y + zc.y));     // q X1[m]
        double2 c = make_double2(q2 * (z.y - zc.y), -q2 * (z.x - zc.x));    // q X2[m]
        if (shift) {
            double sn, cs;   // e^{-i pi m / nphi}
            sincospi((double)(m % (2 * nphi)) / (double)nphi, &sn, &cs);
            a = cmul(a, make_double2(cs, -sn));
            c = cmul(c, make_double2(cs, -sn));
        }
        double2 *o1 = reinterpret_cast<double2 *>(F + ((size_t)m * hstride + r1) * 4);
        o1[0] = a;
        o1[1] = cconj(a);
        if (r2 >= 0) {
            double2 *o2 = reinterpret_cast<double2 *>(F + ((size_t)m * hstride + r2) * 4);
            o2[0] = c;
            o2[1] = cconj(c);
        }
    }
}

// ------------------------------------------------------------------ MW / MWSS theta filter
// One workgroup per order m >= 0, both signs.  For g = the torus extension of
// ftilde_{+-m} (g(2pi - th) = (-1)^{m+s} g(th)), on the N torus points
// (MW: N = 2L-1, theta_t = (2t+1) pi/N; MWSS: N = 2L, theta_t = 2 pi t/N)
//   h = P_{L-1}[g w'],   w' = P_{2L-2}[sin(theta) 1_[0,pi]],
// folded onto the rings: h~(theta_t) = (2pi/N) [h(theta_t) + (-1)^{m+s} h(mirror t)]
// (MW mirror N-1-t, MWSS N-t), unfolded at the poles, so that
// sum_t h~(theta_t) d(theta_t) = int_0^pi g d sin(theta) exactly.  On the doubled
// grid {theta_t} u {mu_t = theta_t + pi/N}:
//   h = (g w'_theta + S-[w'_mu S+ g]) / 2,
// S+-: band-limited half-sample shifts (DFT, phase e^{+-i k pi/N}/N, inverse DFT).
// MWSS: g is the torus interpolant without the Nyquist frequency L (it vanishes
// for band-limited samples); its value at theta_t is g_t - ghat_L (-1)^t.
// Torus point t <-> ring: MW t < L: ring t (t = L-1: south pole), MWSS t = 0:
// north pole (ring L), 0 < t < L: ring t-1, t = L: south pole (ring L-1).  In
// place: F[m][ring] -> H[m][ring] for the swept rings; the pole values go to
// hpole[(L-1) +- m] (south) and hpoleN (north, MWSS).  half (real signals):
// only the side of order +m is filtered, the filter being real and the side
// of order -m the conjugate.
// adj (MWSS): the Hermitian adjoint of the filter.  With the Nyquist projector
// P (real, symmetric) and (S+)^H = S-, the filter is sc E^T [(W P + S- W' S+) / 2] E,
// whose adjoint differs only in the first term: P W instead of W P, i.e. the
// Nyquist component is removed from g w'_theta rather than from g.  (MW has no
// Nyquist bin: its filter is Hermitian and adj changes nothing.)
__device__ __forceinline__ int torus_ring(int t, int L, int N, int ss, bool *mirrored)
{
    *mirrored = ss ? t > L : t >= L;
    const int u = *mirrored ? (ss ? N - t : N - 1 - t) : t;     // sample on [0, pi]
    if (!ss) return u;
    return u == 0 ? L : u - 1;
}

__global__ __launch_bounds__(1024) void k_mw_filter(int L, int ss, int hstride, int spin, const FftArgs *__restrict__ fN,
                                                    const double *__restrict__ wq, const double *__restrict__ ph,
                                                    double *__restrict__ F, double2 *__restrict__ hpole,
                                                    double2 *__restrict__ hpoleN, double2 *__restrict__ fscr,
                                                    int half, int adj, const FftArgs *__restrict__ fconv)
{
    extern __shared__ double2 buf[];
    __shared__ double2 nyq;
    __shared__ double2 wpart[16];                          // per-wave partial sums (<= 1024 threads)
    const int m = blockIdx.x;
    const int N = ss ? 2 * L : 2 * L - 1;
    const int T = blockDim.x, tid = threadIdx.x;
    const double par = ((m + spin) & 1) ? -1.0 : 1.0;
    const double2 *phc = reinterpret_cast<const double2 *>(ph);
    double2 *scr = fscr ? fscr + (size_t)blockIdx.x * FFT_SCRATCH : nullptr;
    for (int side = 0; side < 2; ++side) {
        if (side == 1 && (m == 0 || half)) break;
        // torus samples
        double2 acc = make_double2(0.0, 0.0);                // adj: sum_t (-1)^t w'_theta g
        for (int t = tid; t < N; t += T) {
            bool mir;
            const int r = torus_ring(t, L, N, ss, &mir);
            const double *src = F + ((size_t)m * hstride + r) * 4 + 2 * side;
            double2 g = make_double2(src[0], src[1]);
            if (mir) { g.x *= par; g.y *= par; }
            buf[t] = g;
            if (ss && adj) {
                const double sw = (t & 1) ? -wq[t] : wq[t];
                acc.x = fma(sw, g.x, acc.x);
                acc.y = fma(sw, g.y, acc.y);
            }
        }
        if (ss && adj) {                                    // uniform over the workgroup
            for (int o = 32; o > 0; o >>= 1) {
                acc.x += __shfl_xor(acc.x, o, 64);
                acc.y += __shfl_xor(acc.y, o, 64);
            }
            if ((tid & 63) == 0) wpart[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double2 tot = make_double2(0.0, 0.0);
                for (int w = 0; w < (T + 63) / 64; ++w) tot = cadd(tot, wpart[w]);
                nyq = make_double2(tot.x / N, tot.y / N);   // Nyquist component of g w'_theta
            }
        }
        // the midpoint samples S g times the weights w'', moved back: S^{-1} (w'' S g).
        // DFT form: four engine passes (forward, shift, inverse: midpoints; weights;
        // forward, shift back, inverse).  Convolution form (MW, N not 13-smooth, fconv:
        // the two shifts' FftArgs): each shift is a circular convolution of length N
        // with a fixed kernel, run by the Bluestein driver with a unit chirp and the
        // kernel's spectrum as its filter (one cyclic convolution, two FFTs or four
        // half-length ones where the engine splits it, instead of two Bluestein DFTs);
        // its result is at t < N.  One call site, so the engine is inlined once.
        const bool conv = fconv != nullptr;
        __syncthreads();                             // the torus samples are in LDS
#pragma nounroll
        for (int pass = 0; pass < 4; ++pass) {
            if (!conv || !(pass & 1))
                dft_lds(buf, conv ? fconv + (pass >> 1) : fN, conv ? -1 : ((pass & 1) ? +1 : -1), scr);
            if (pass == 0 && !conv) {
                for (int k = tid; k < N; k += T) {                                 // shift +pi/N
                    if (ss && !adj && k == L) nyq = make_double2(buf[k].x / N, buf[k].y / N);   // ghat_L (MWSS), read first
                    buf[k] = cmul(buf[k], phc[k]);
                }
            } else if (pass == 1) {
                for (int t = tid; t < N; t += T) {
                    const double wv = wq[N + t];
                    buf[t].x *= wv;
                    buf[t].y *= wv;
                }
            } else if (pass == 2 && !conv) {
                for (int k = tid; k < N; k += T) buf[k] = cmulc(buf[k], phc[k]);   // shift -pi/N
            }
            __syncthreads();
        }
        for (int t = tid; t < N; t += T) {          // + g w'_theta (g re-read: F is rewritten only below)
            bool mir;
            const int r = torus_ring(t, L, N, ss, &mir);
            const double *src = F + ((size_t)m * hstride + r) * 4 + 2 * side;
            double2 g = make_double2(src[0], src[1]);
            if (mir) { g.x *= par; g.y *= par; }
            const double wv = wq[t];
            const double sg = (t & 1) ? -1.0 : 1.0;
            if (ss && !adj) {                                // P g, then times w'
                g.x -= sg * nyq.x;
                g.y -= sg * nyq.y;
            }
            double2 gw = make_double2(g.x * wv, g.y * wv);
            if (ss && adj) {                                 // P (g w')
                gw.x -= sg * nyq.x;
                gw.y -= sg * nyq.y;
            }
            buf[t] = make_double2(0.5 * (gw.x + buf[t].x), 0.5 * (gw.y + buf[t].y));
        }
        __syncthreads();
        const double sc = 2.0 * M_PI / (double)N;
        const int hidx = side == 0 ? (L - 1) + m : (L - 1) - m;
        for (int t = tid; t < (ss ? L + 1 : L); t += T) {
            double2 h = buf[t];
            const bool pole = ss ? (t == 0 || t == L) : (t == L - 1);
            if (!pole) {
                const double2 hr = buf[ss ? N - t : N - 1 - t];
                h.x += par * hr.x;
                h.y += par * hr.y;
            }
            h.x *= sc;
            h.y *= sc;
            if (!pole) {
                double *dst = F + ((size_t)m * hstride + (ss ? t - 1 : t)) * 4 + 2 * side;
                dst[0] = h.x;
                dst[1] = h.y;
            } else if (ss && t == 0) {
                hpoleN[hidx] = h;
            } else {
                hpole[hidx] = h;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ adjoint of the forward (MW)
// The MW forward is F = Finish Dfwd Theta PhiFwd with the theta filter Theta =
// sc E^H A E (torus extension E, Hermitian A, fold sc E^H): Theta is
// Hermitian, so F^H = PhiFwd^H Theta Dfwd^H Finish^H, where Dfwd^H Finish^H
// is the inverse sweep with the SHT weights on the regular rings plus the
// closed-form south pole (Eq. 29).  gather: sum the sweep's blocks (and the
// pole) into the filter's [m][ring] layout; scatter: filtered rings and pole
// -> [ring][m] partials of a single block, scaled by the phi weight q.
// MWSS (ss): the rows are the L-1 regular rings, the south pole (row L-1) and the
// north pole (row L, the forward's w_l h~_{-s}(0) at order -s), and the adjoint
// filter runs in between.
__global__ void k_fadj_gather(int L, int ss, int nblk, int spin, const double *__restrict__ part,
                              const int *__restrict__ mtop, const double2 *__restrict__ flm,
                              const double *__restrict__ wl, int hstride, double *__restrict__ F)
{
    const int nrow = L + ss;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)L * nrow) return;
    const int m = (int)(i / nrow), t = (int)(i % nrow);
    const int nreg = L - 1, M = 2 * L - 1;
    const size_t bstride = (size_t)nreg * L * 4;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (t < nreg) {
        for (int b = 0; b < nblk; ++b) {
            if (m > mtop[b]) continue;                  // that block's sweep never reached order m
            const double *pp = part + b * bstride + ((size_t)t * L + m) * 4;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += pp[c];
        }
    } else {
        // south pole (t == nreg): only the signed order s is nonzero, sum_l (-1)^{l+s} w_l G[l][s];
        // north pole (t == nreg + 1): only the order -s, sum_l w_l G[l][-s]
        const bool north = t > nreg;
        const int mp = north ? -spin : spin;
        const int as = spin < 0 ? -spin : spin;
        if (m == as) {
            double2 acc = make_double2(0.0, 0.0);
            for (int l = as; l < L; ++l) {
                const double2 g = flm[(size_t)l * M + (L - 1) + mp];
                const double c = (!north && ((l + spin) & 1)) ? -wl[l] : wl[l];
                acc.x += c * g.x;
                acc.y += c * g.y;
            }
            const int off = (mp < 0) ? 2 : 0;
            v[off] = acc.x;
            v[off + 1] = acc.y;
        }
    }
    if (m == 0) { v[2] = 0.0; v[3] = 0.0; }
    double *dst = F + ((size_t)m * hstride + t) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[c] = v[c];
}

__global__ void k_fadj_scatter(int L, int ss, int hstride, double q, const double *__restrict__ F,
                               const double2 *__restrict__ hpole, const double2 *__restrict__ hpoleN,
                               double *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)(L + ss) * L) return;
    const int t = (int)(i / L), m = (int)(i % L);
    double v[4];
    if (t < L - 1) {
        const double *src = F + ((size_t)m * hstride + t) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = src[c];
    } else {
        const double2 *hp = t == L - 1 ? hpole : hpoleN;   // south pole; north pole (MWSS)
        const double2 a = hp[(L - 1) + m], b = hp[(L - 1) - m];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    if (m == 0) { v[2] = 0.0; v[3] = 0.0; }
    double *dst = out + ((size_t)t * L + m) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[c] = q * v[c];
}

// ------------------------------------------------------------------ forward finish
// flm[l][m] = w_l * (sum_b Q[b][l][|m|].side + Qx[b][l][|m|].side) * ((-1)^{|m|-nB} for m < 0)
//           + south pole: w_l (-1)^{l+s} h~_s(pi) at m = s  (Eq. 29)
//           + north pole (MWSS): w_l h~_{-s}(0) at m = -s.
// Zero where l < max(|m|, |spin|).  One thread per (l, |m|) reads whole 32-byte
// records (side A = order +|m| in components 0,1, side B = order -|m| in 2,3) and
// writes both orders.  half (real signals, spin 0): only side A is read, and
// half = 1: flm[l][-m] = (-1)^m conj(flm[l][m]) (Hermitian symmetry);
// half = 2 (gradient of the real-signal inverse with respect to its complex
// input, whose orders m > 0 enter twice and order 0 through its real part):
// 2 x side A at m > 0, its real part at m = 0, zero at m < 0.
__global__ void k_finish_fwd(int L, int nblk, int spin, int nB, const double *__restrict__ Q,
                             const double *__restrict__ Qx, int nxp, const double *__restrict__ wl,
                             const double2 *__restrict__ hpole, const double2 *__restrict__ hpoleN,
                             double2 *__restrict__ flm, int half)
{
    const int M = 2 * L - 1;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)L * L) return;
    const int l = (int)(i / L), am = (int)(i % L);
    const int as = spin < 0 ? -spin : spin;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (l >= am && l >= as) {
        for (int bb = 0; bb < nblk; ++bb) {
            const double2 *q = reinterpret_cast<const double2 *>(Q + (((size_t)bb * L + l) * L + am) * 4);
            a = cadd(a, q[0]);
            if (!half) b = cadd(b, q[1]);
            if (Qx && am < nxp) {                      // orders below |n| from the other run's continuation
                const double2 *qx = reinterpret_cast<const double2 *>(Qx + (((size_t)bb * L + l) * nxp + am) * 4);
                a = cadd(a, qx[0]);
                b = cadd(b, qx[1]);
            }
        }
        const double w = wl[l];
        const double wb = ((am - nB) & 1) ? -w : w;
        a = make_double2(a.x * w, a.y * w);
        b = make_double2(b.x * wb, b.y * wb);
        if (hpole) {
            const double c = ((l + spin) & 1) ? -w : w;
            if (am == spin) {
                const double2 hp = hpole[(L - 1) + am];
                a = make_double2(fma(c, hp.x, a.x), fma(c, hp.y, a.y));
            }
            if (am > 0 && -am == spin) {
                const double2 hp = hpole[(L - 1) - am];
                b = make_double2(fma(c, hp.x, b.x), fma(c, hp.y, b.y));
            }
        }
        if (hpoleN) {                                  // MWSS north pole: w_l h~_{-s}(0) at m = -s
            if (am == -spin) {
                const double2 hp = hpoleN[(L - 1) + am];
                a = make_double2(fma(w, hp.x, a.x), fma(w, hp.y, a.y));
            }
            if (am > 0 && -am == -spin) {
                const double2 hp = hpoleN[(L - 1) - am];
                b = make_double2(fma(w, hp.x, b.x), fma(w, hp.y, b.y));
            }
        }
    }
    if (half == 1) {
        b = (am & 1) ? make_double2(-a.x, a.y) : make_double2(a.x, -a.y);
    } else if (half == 2) {
        a = am == 0 ? make_double2(a.x, 0.0) : make_double2(2.0 * a.x, 2.0 * a.y);
        b = make_double2(0.0, 0.0);
    }
    double2 *row = flm + (size_t)l * M + (L - 1);
    row[am] = a;
    if (am > 0) row[-am] = b;
}

// ------------------------------------------------------------------ ring scaling
// map[t][p] *= w[t] for rings of nphi samples each (adjoint of a ring-weighted quadrature)
__global__ void k_ring_scale(int nring, int nphi, const double *__restrict__ w, double2 *__restrict__ map)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nring * nphi) return;
    const double s = w[i / nphi];
    map[i] = make_double2(map[i].x * s, map[i].y * s);
}

// real maps: map[t][p] *= w[t] over rings given by their start and length
__global__ void k_ring_scale_real(int nring, const long long *__restrict__ ring_start,
                                  const int *__restrict__ ring_nphi, const double *__restrict__ w,
                                  double *__restrict__ map)
{
    const int r = blockIdx.x;
    if (r >= nring) return;
    double *row = map + ring_start[r];
    const double s = w[r];
    for (int k = threadIdx.x; k < ring_nphi[r]; k += blockDim.x) row[k] *= s;
}

// Hermitian part of a coefficient cotangent: out[l][+-m] from
// h_m = (G[l][m] + (-1)^m conj G[l][-m]) / 2 (m > 0), h_0 = Re G[l][0], with
// out[l][-m] = (-1)^m conj h_m.  For a real map x and the forward transform F,
// Re <G, F x> = <h, F x>: the real-signal adjoint of the forward sees only h.
__global__ void k_hermitian_part(int L, const double2 *__restrict__ G, double2 *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)L * L) return;
    const int l = (int)(i / L), am = (int)(i % L);
    const int M = 2 * L - 1;
    const double2 *row = G + (size_t)l * M + (L - 1);
    double2 *orow = out + (size_t)l * M + (L - 1);
    const double2 a = row[am];
    if (am == 0) {
        orow[0] = make_double2(a.x, 0.0);
        return;
    }
    const double2 b = row[-am];
    const double sg = (am & 1) ? -1.0 : 1.0;
    const double2 h = make_double2(0.5 * (a.x + sg * b.x), 0.5 * (a.y - sg * b.y));
    orow[am] = h;
    orow[-am] = make_double2(sg * h.x, -sg * h.y);
}

// ------------------------------------------------------------------ SO(3) gamma DFT
// inverse: out[k][i] = sum_n e^{i n gamma_k} in[n][i];  forward: out[n][i] = q sum_k e^{-i n gamma_k} in[k][i]
__global__ void k_gamma_dft(int N, long long nper, int sign, double q, const double *__restrict__ roots,
                            const double2 *__restrict__ in, double2 *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nper) return;
    const int G = 2 * N - 1;
    double2 v[15];
    for (int a = 0; a < G; ++a) v[a] = in[(size_t)a * nper + i];
    for (int b = 0; b < G; ++b) {
        double2 acc = make_double2(0.0, 0.0);
        for (int a = 0; a < G; ++a) {
            // sign = +1 (inverse): a = n index (n = a-(N-1)), b = k;  sign = -1: a = k, b = n index
            const int nn = (sign > 0 ? a : b) - (N - 1);
            const int kk = sign > 0 ? b : a;
            const int idx = (int)((((long long)nn * kk) % G + G) % G);
            const double2 rt = ldroot(roots, idx, sign);
            acc = cadd(acc, cmul(v[a], rt));
        }
        out[(size_t)b * nper + i] = make_double2(q * acc.x, q * acc.y);
    }
}

// ------------------------------------------------------------------ debug export of d
// d^l_{m,n}(theta_r) for one (ring, l) from the same init / step / renormalisation
// as the sweeps, handed to put(m, d, cont) for m = l down to 0; where this run is the
// unstable one below the switch order ms, the run -n is then continued to order
// -(ms-1) and put(m, d^l_{m,n}, true) gives the orders m < ms again from
// d^l_{m,n} = (-1)^{m-n} d^l_{-m,-n} (those replace the first values).
template <typename Put>
__device__ __forceinline__ void d_walk(int L, int n, int r, int l, const double *__restrict__ cot,
                                       const double *__restrict__ csc, const double *__restrict__ lsin,
                                       const double *__restrict__ lcos, const double *__restrict__ lbin,
                                       const double *__restrict__ kap, const double *__restrict__ gtab, Put put)
{
    const int an = n < 0 ? -n : n;
    if (l < an) return;
    double e, ep = 0.0;
    int E;
    d_init(l, n, dd_from(lbin + 2 * l), dd_from(lsin + 2 * r), dd_from(lcos + 2 * r), e, E);
    put(l, ldexp(e * gtab[(size_t)l * L + l], E), false);
    for (int m = l - 1; m >= 0; --m) {
        const double lam = fma(-(double)(m + 1), cot[r], (double)n * csc[r]);
        const double en = fma(kap[(size_t)m * L + l] * lam, e, -ep);
        ep = e;
        e = en;
        if (E != 0) renorm(e, ep, E);
        put(m, ldexp(e * gtab[(size_t)m * L + l], E), false);
    }
    const double ct = cot[r];
    const int ms = switch_order(n, ct, csc[r]);
    if (an > 0 && !ring_good(n, ct) && ms > 0) {
        E = 0;
        ep = 0.0;
        d_init(l, -n, dd_from(lbin + 2 * l), dd_from(lsin + 2 * r), dd_from(lcos + 2 * r), e, E);
        for (int m = l - 1; m >= -(ms - 1); --m) {
            const double lam = fma(-(double)(m + 1), ct, -(double)n * csc[r]);
            const double en = fma(kap[(ptrdiff_t)m * L + l] * lam, e, -ep);
            ep = e;
            e = en;
            if (E != 0) renorm(e, ep, E);
            const int mm = -m;
            if (mm >= 0 && mm < ms) {
                const double v = ldexp(e * gtab[(ptrdiff_t)m * L + l], E);
                put(mm, ((mm - n) & 1) ? -v : v, true);
            }
        }
    }
}

// out[r][m][l] = d^l_{m,n}(theta_r), one thread per (ring, l).
__global__ void k_debug_d(int L, int nreg, int n, const double *__restrict__ cot, const double *__restrict__ csc,
                          const double *__restrict__ lsin, const double *__restrict__ lcos,
                          const double *__restrict__ lbin, const double *__restrict__ kap,
                          const double *__restrict__ gtab, double *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (r >= nreg) return;
    double *o = out + (size_t)r * L * L;
    for (int m = 0; m <= l; ++m) o[(size_t)m * L + l] = 0.0;
    d_walk(L, n, r, l, cot, csc, lsin, lcos, lbin, kap, gtab,
           [&](int m, double v, bool) { o[(size_t)m * L + l] = v; });
}

// Unitarity check (debug): for ring rsel[i] and degree l, out[i][l] = {sum over
// m >= 0 of (d^l_{m,n})^2, d^l_{0,n}} with the values the sweeps use.  d^l(theta) is
// the matrix of a rotation in the (2l+1)-dimensional representation, real and
// orthogonal, so with d^l_{-m,n} = (-1)^{m-n} d^l_{m,-n} the runs n and -n give
// sum_{|m| <= l} (d^l_{m,n})^2 = 1.
__global__ void k_unitarity(int L, int n, int nsel, const int *__restrict__ rsel, const double *__restrict__ cot,
                            const double *__restrict__ csc, const double *__restrict__ lsin,
                            const double *__restrict__ lcos, const double *__restrict__ lbin,
                            const double *__restrict__ kap, const double *__restrict__ gtab,
                            double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= nsel) return;
    const int r = rsel[i];
    const int an = n < 0 ? -n : n;
    const double ct = cot[r];
    const int ms = switch_order(n, ct, csc[r]);
    const int ovr = (an > 0 && !ring_good(n, ct) && ms > 0) ? ms : 0;   // orders the continuation replaces
    double sum = 0.0, d0 = 0.0;
    d_walk(L, n, r, l, cot, csc, lsin, lcos, lbin, kap, gtab, [&](int m, double v, bool cont) {
        if (!cont && m < ovr) return;
        sum = fma(v, v, sum);
        if (m == 0) d0 = v;
    });
    out[((size_t)i * L + l) * 2] = sum;
    out[((size_t)i * L + l) * 2 + 1] = d0;
}

// ------------------------------------------------------------------ Bluestein filters
// For every Bluestein transform: bflt = DFT_len(b) / len with b_j = c_j (j < n),
// b_{len-j} = c_j (0 < j < n), 0 elsewhere -- the circular form of the chirp.
// Split form (convolution length M = 2H, H = f.len): by decimation in
// frequency the even samples are DFT_H(b_j + b_{j+H}) and the odd ones
// DFT_H((b_j - b_{j+H}) w^j), w = e^{-2 pi i/M}; with n < H, b_j = c_j for
// j < n and b_{j+H} = c_{H-j} for j > H - n.
__global__ __launch_bounds__(1024) void k_bluestein_prep(const FftArgs *__restrict__ ffts)
{
    extern __shared__ double2 buf[];
    const FftArgs *f = ffts + blockIdx.x;
    if (!f->blue || f->conv) return;                    // convolutions carry their own filter
    const int n = f->n, len = f->len;
    const double2 *ch = reinterpret_cast<const double2 *>(f->chirp);
    if (f->split) {
        const double2 *wm = reinterpret_cast<const double2 *>(f->twm);
        double2 *out = reinterpret_cast<double2 *>(const_cast<double *>(f->bflt));
        const double inv = 1.0 / (2.0 * (double)len);
        for (int half = 0; half < 2; ++half) {
            for (int j = threadIdx.x; j < len; j += blockDim.x) {
                const double2 lo = j < n ? ch[j] : make_double2(0.0, 0.0);
                const double2 hi = (j > len - n) ? ch[len - j] : make_double2(0.0, 0.0);
                buf[j] = half == 0 ? cadd(lo, hi) : cmul(csub(lo, hi), wm[j]);
            }
            __syncthreads();
            fft_engine(buf, f, -1);
            for (int k = threadIdx.x; k < len; k += blockDim.x)
                out[2 * k + half] = make_double2(buf[k].x * inv, buf[k].y * inv);
            __syncthreads();
        }
        return;
    }
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (i < n) v = ch[i];
        else if (i > len - n) v = ch[len - i];
        buf[i] = v;
    }
    __syncthreads();
    fft_engine(buf, f, -1);
    double2 *out = reinterpret_cast<double2 *>(const_cast<double *>(f->bflt));
    const double inv = 1.0 / (double)len;
    for (int i = threadIdx.x; i < len; i += blockDim.x) out[i] = make_double2(buf[i].x * inv, buf[i].y * inv);
}

// pole[(L-1) + m] = F[|m|][ring].side(m): the MW south-pole ring's Fourier line
__global__ void k_pole_from_F(int L, int hstride, int ring, const double *__restrict__ F, double2 *__restrict__ pole)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * L - 1) return;
    const int m = i - (L - 1), am = m < 0 ? -m : m;
    const double *src = F + ((size_t)am * hstride + ring) * 4 + (m < 0 ? 2 : 0);
    pole[i] = make_double2(src[0], src[1]);
}

// ------------------------------------------------------------------ launchers
#define S2_LAUNCH_CHECK() do { hipError_t _e = hipGetLastError(); if (_e != hipSuccess) return _e; } while (0)

hipError_t launch_pack_inv(hipStream_t st, int L, int nx, int n, int nblk, int slots_per_blk, const int *lslot,
                           const double2 *flmA, const double2 *flmB, const double *wA, const double *wB,
                           const double *kap, const double *gtab, double *C, int half)
{   // half: 0 both sides, 1 the A side only, 2 the B side only
    const int nslot = nblk * slots_per_blk;
    dim3 grid((nslot + 255) / 256, L + nx);
    // side 1: A only (flmB not read), side 2: B only (flmA absent)
    if ((half == 1 && !flmA) || (half == 2 && (flmA || !flmB))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_inv, grid, dim3(256), 0, st, L, nx, n, nslot, slots_per_blk, half ? 3 : 5, lslot, flmA,
                       half == 1 ? nullptr : flmB, wA, wB, kap, gtab, C);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_dstage_inv(hipStream_t st, int nwaves, int nblk, int L, int nx, int nreg, int n, const double *cot,
                             const double *csc, const double2 *init, const double *C, const int *lchunk,
                             const int *mtop, double *partA, double *partB, int side, int nsw,
                             const OrderTiles &ot)
{
    if (ot.nt < 1 || ot.nt > MAX_ORDER_TILES || (ot.nt > 1 && !ot.ck)) return hipErrorInvalidValue;
    if (nwaves != 4 && nwaves != 8) return hipErrorInvalidValue;   // reducer rotation: one or two groups of 4
    if (side < 0 || side > 2 || (side == 1 && !partA) || (side == 2 && !partB) || (side == 0 && (!partA || !partB)))
        return hipErrorInvalidValue;                                // the side(s) swept must have outputs
    if (nsw <= 0) nsw = nreg;
    const bool pair = nsw < nreg;                                   // mirror rings from the northern sweep
    if (nsw > nreg || (pair && (n != 0 || side == 2 || 2 * nsw < nreg))) return hipErrorInvalidValue;
    dim3 grid((nsw + 63) / 64, nblk, ot.nt);
    // wave count, the real-signal half and the ring pairing as template arguments
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(64 * nwaves), 0, st, L, nx, nreg, nsw, n, cot, csc, init, C, lchunk, mtop,
                           partA, partB, ot);
    };
    if (nwaves == 8) {
        if (pair) side ? go(k_dstage_inv<INV_NCH, 8, 1, true>) : go(k_dstage_inv<INV_NCH, 8, 0, true>);
        else if (side == 1) go(k_dstage_inv<INV_NCH, 8, 1>);
        else if (side == 2) go(k_dstage_inv<INV_NCH, 8, 2>);
        else go(k_dstage_inv<INV_NCH, 8, 0>);
    } else {
        if (pair) side ? go(k_dstage_inv<INV_NCH, 4, 1, true>) : go(k_dstage_inv<INV_NCH, 4, 0, true>);
        else if (side == 1) go(k_dstage_inv<INV_NCH, 4, 1>);
        else if (side == 2) go(k_dstage_inv<INV_NCH, 4, 2>);
        else go(k_dstage_inv<INV_NCH, 4, 0>);
    }
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_dstage_fwd(hipStream_t st, int nwaves, int nblk, int G, int L, int nxp, int nreg, int hstride,
                             int lstride, int n, const double *lam, const double2 *init, const double *kap,
                             const double *gtab, const double *HA, const double *HB, const double *HxA,
                             const double *HxB, double *QA, double *QB, double *QxA, double *QxB, int side, int pair,
                             const OrderTiles &ot)
{
    if (ot.nt < 1 || ot.nt > MAX_ORDER_TILES || (ot.nt > 1 && !ot.ck)) return hipErrorInvalidValue;
    if ((nwaves != 4 && nwaves != 8 && nwaves != 16) || nwaves > FWD_MAX_WAVES)
        return hipErrorInvalidValue;                                // reducer rotation: 1, 2 or 4 groups of 4
    if (pair && (n != 0 || HA == HB || HxA || HxB || side == 2)) return hipErrorInvalidValue;   // mirror rings: n = 0
    // one side: both sides read one spectra array (the run's slice), and that side has outputs
    if (side && !pair && (HA != HB || (side == 1 && !QA) || (side == 2 && !QB))) return hipErrorInvalidValue;
    // XCD-aware tile order when the untiled grid is resident in one round (every
    // workgroup of a ring block then runs beside the others that read its spectra rows,
    // in step through one L2).  Measured (one map): MW L = 2048 forward 2.94 -> 2.82 ms
    // (spin 2: 5.43 -> 5.05 ms), HEALPix nside 1024 3.95 -> 3.80 ms, spectra read from
    // HBM 3.04 -> 1.58 GB; grids of several rounds were slower in that order (L = 3072
    // 10.7 -> 12.4 ms, L = 4096 19.5 -> 28.1 ms, L = 1024 in 8 order tiles 0.59 -> 0.75
    // ms) and keep the plain one.  The inverse sweep was slower in XCD order at every size
    // tried (L = 1024: 0.47 -> 0.79 ms; L = 2048 spin 2: 4.5 -> 5.1 ms).
    const int gx = (G + 1) / 2, gy = nblk, gz = ot.nt, T = gx * gy * gz;
    // (a failed query only selects the plain order; its error is cleared, not reported)
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
        hipSuccess) {
        ncu = 0;
        (void)hipGetLastError();
    }
    // the wave count is a template argument: the reducer rotation and the wave sum
    // then compile to fixed code; HA == HB (run n = 0) selects the one-array path
    auto go = [&](auto kern) {
        int per_cu = 0;
        if (ncu && hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * nwaves, 0) != hipSuccess) {
            per_cu = 0;
            (void)hipGetLastError();
        }
        const bool xcd = ot.nt == 1 && T <= per_cu * ncu;
        const dim3 grid((unsigned)(xcd ? (T + NXCD - 1) / NXCD * NXCD : T));
        hipLaunchKernelGGL(kern, grid, dim3(64 * nwaves), 0, st, gx, gy, gz, xcd, L, nxp, nreg, hstride, lstride, n,
                           G, lam, init, kap, gtab, HA, HB, HxA, HxB, QA, QB, QxA, QxB, ot);
    };
    const bool same = HA == HB;
    if (pair) {
        if (nwaves == 16) side ? go(k_dstage_fwd<FWD_NCH, true, 16, 1, true>) : go(k_dstage_fwd<FWD_NCH, true, 16, 0, true>);
        else if (nwaves == 8) side ? go(k_dstage_fwd<FWD_NCH, true, 8, 1, true>) : go(k_dstage_fwd<FWD_NCH, true, 8, 0, true>);
        else side ? go(k_dstage_fwd<FWD_NCH, true, 4, 1, true>) : go(k_dstage_fwd<FWD_NCH, true, 4, 0, true>);
    } else if (side == 1) {
        if (nwaves == 16) go(k_dstage_fwd<FWD_NCH, true, 16, 1>);
        else if (nwaves == 8) go(k_dstage_fwd<FWD_NCH, true, 8, 1>);
        else go(k_dstage_fwd<FWD_NCH, true, 4, 1>);
    } else if (side == 2) {
        if (nwaves == 16) go(k_dstage_fwd<FWD_NCH, true, 16, 2>);
        else if (nwaves == 8) go(k_dstage_fwd<FWD_NCH, true, 8, 2>);
        else go(k_dstage_fwd<FWD_NCH, true, 4, 2>);
    } else if (nwaves == 16) same ? go(k_dstage_fwd<FWD_NCH, true, 16>) : go(k_dstage_fwd<FWD_NCH, false, 16>);
    else if (nwaves == 8) same ? go(k_dstage_fwd<FWD_NCH, true, 8>) : go(k_dstage_fwd<FWD_NCH, false, 8>);
    else same ? go(k_dstage_fwd<FWD_NCH, true, 4>) : go(k_dstage_fwd<FWD_NCH, false, 4>);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_order_ckpt(hipStream_t st, int L, int nreg, int n, const double *cot, const double *csc,
                             const double2 *init, const double *kap, const OrderTiles &ot, double *ck)
{
    if (ot.nt < 2) return hipSuccess;
    if (ot.nt > MAX_ORDER_TILES || !ck || ot.rp < nreg) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_order_ckpt, dim3((ot.rp + 63) / 64, L), dim3(64), 0, st, L, nreg, n, cot, csc, init, kap, ot,
                       ck);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pair_spectra(hipStream_t st, int L, int nreg, int nsw, int hstride, int pstride, const double *H,
                               double *S, double *D)
{
    if (nsw > pstride || 2 * nsw < nreg || nreg > hstride) return hipErrorInvalidValue;
    const size_t tot = (size_t)L * pstride;
    hipLaunchKernelGGL(k_pair_spectra, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, nreg, nsw, hstride,
                       pstride, H, S, D);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_init_table(hipStream_t st, int L, int nreg, int n, const double *lsin, const double *lcos,
                             const double *lbin, double2 *init)
{
    const size_t tot = (size_t)L * nreg;
    hipLaunchKernelGGL(k_init_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, nreg, n, lsin, lcos,
                       lbin, init);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_lambda_table(hipStream_t st, int L, int nx, int nreg, int lstride, int n, const double *cot,
                               const double *csc, double *lam)
{
    const size_t tot = (size_t)(L + nx) * lstride;
    hipLaunchKernelGGL(k_lambda_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, nx, nreg, lstride, n,
                       cot, csc, lam);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_phi_inv(hipStream_t st, int nthreads, size_t lds, int nring, int L, int nreg, int nblk, int spin,
                          const double *part, const int *mtop, const double2 *flm, const double *wl,
                          const int *ring_nphi, const long long *ring_start, const int *ring_shift,
                          const int *ring_fft, const FftArgs *ffts, double2 *map, double2 *fscr)
{
    hipLaunchKernelGGL(k_phi_inv, dim3(nring), dim3(nthreads), lds, st, L, nreg, nblk, spin, part, mtop, flm, wl,
                       ring_nphi, ring_start, ring_shift, ring_fft, ffts, map, fscr);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_phi_fwd(hipStream_t st, int nthreads, size_t lds, int nring, int hstride, int L, double q,
                          const double2 *map, const int *ring_nphi, const long long *ring_start, const int *ring_shift,
                          const int *ring_fft, const FftArgs *ffts, const double *ringq, double *F,
                          double2 *fscr)
{
    hipLaunchKernelGGL(k_phi_fwd, dim3(hstride), dim3(nthreads), lds, st, L, nring, hstride, q, map, ring_nphi,
                       ring_start, ring_shift, ring_fft, ffts, ringq, F, fscr);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_phi_inv_real(hipStream_t st, int nthreads, size_t lds, int npair, int L, int nreg, int nblk,
                               const int *pairs, const double *part, const int *mtop, const double2 *flm,
                               const double *wl, const int *ring_nphi, const long long *ring_start,
                               const int *ring_shift, const int *ring_fft, const FftArgs *ffts, double *map,
                               double2 *fscr)
{
    if (nthreads > 1024 || npair < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_phi_inv_real, dim3(npair), dim3(nthreads), lds, st, L, nreg, nblk, pairs, part, mtop, flm, wl,
                       ring_nphi, ring_start, ring_shift, ring_fft, ffts, map, fscr);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_phi_fwd_real(hipStream_t st, int nthreads, size_t lds, int nring, int hstride, int npair, int L,
                               double q, const int *pairs, const double *map, const int *ring_nphi,
                               const long long *ring_start, const int *ring_shift, const int *ring_fft,
                               const FftArgs *ffts, const double *ringq, double *F, double2 *fscr)
{
    if (nthreads > 1024 || hstride < nring || npair < 1) return hipErrorInvalidValue;
    const int nblocks = npair + (hstride - nring + 1) / 2;
    hipLaunchKernelGGL(k_phi_fwd_real, dim3(nblocks), dim3(nthreads), lds, st, L, nring, hstride, npair, q, pairs, map,
                       ring_nphi, ring_start, ring_shift, ring_fft, ffts, ringq, F, fscr);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_mw_filter(hipStream_t st, int nthreads, size_t lds, int L, int ss, int hstride, int spin,
                            const FftArgs *fN, const double *wq, const double *ph, double *F, double2 *hpole,
                            double2 *hpoleN, double2 *fscr, int half, int adj, const FftArgs *fconv)
{
    if ((ss && !hpoleN) || nthreads > 1024) return hipErrorInvalidValue;
    if (fconv && ss) return hipErrorInvalidValue;               // the convolution form is MW's
    hipLaunchKernelGGL(k_mw_filter, dim3(L), dim3(nthreads), lds, st, L, ss, hstride, spin, fN, wq, ph, F, hpole,
                       hpoleN, fscr, half, adj, fconv);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_ring_scale_real(hipStream_t st, int nring, const long long *ring_start, const int *ring_nphi,
                                  const double *w, double *map)
{
    if (nring < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ring_scale_real, dim3(nring), dim3(256), 0, st, nring, ring_start, ring_nphi, w, map);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_hermitian_part(hipStream_t st, int L, const double2 *G, double2 *out)
{
    const size_t tot = (size_t)L * L;
    hipLaunchKernelGGL(k_hermitian_part, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, G, out);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_ring_scale(hipStream_t st, int nring, int nphi, const double *w, double2 *map)
{
    const size_t tot = (size_t)nring * nphi;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ring_scale, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nring, nphi, w, map);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_finish_fwd(hipStream_t st, int L, int nblk, int spin, int nB, const double *Q, const double *Qx,
                             int nxp, const double *wl, const double2 *hpole, const double2 *hpoleN, double2 *flm,
                             int half)
{
    if (half && (spin != 0 || Qx)) return hipErrorInvalidValue;   // real signals: spin 0
    const size_t tot = (size_t)L * L;
    hipLaunchKernelGGL(k_finish_fwd, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, nblk, spin, nB, Q, Qx,
                       nxp, wl, hpole, hpoleN, flm, half);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_gamma_dft(hipStream_t st, int N, long long nper, int sign, double q, const double *roots,
                            const double2 *in, double2 *out)
{
    hipLaunchKernelGGL(k_gamma_dft, dim3((unsigned)((nper + 255) / 256)), dim3(256), 0, st, N, nper, sign, q, roots,
                       in, out);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_unitarity(hipStream_t st, int L, int n, int nsel, const int *rsel, const double *cot,
                           const double *csc, const double *lsin, const double *lcos, const double *lbin,
                           const double *kap, const double *gtab, double *out)
{
    if (nsel < 1) return hipSuccess;
    dim3 grid((nsel + 63) / 64, L);
    hipLaunchKernelGGL(k_unitarity, grid, dim3(64), 0, st, L, n, nsel, rsel, cot, csc, lsin, lcos, lbin, kap, gtab,
                       out);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_debug_d(hipStream_t st, int L, int nreg, int n, const double *cot, const double *csc,
                          const double *lsin, const double *lcos, const double *lbin, const double *kap,
                          const double *gtab, double *out)
{
    dim3 grid((nreg + 63) / 64, L);
    hipLaunchKernelGGL(k_debug_d, grid, dim3(64), 0, st, L, nreg, n, cot, csc, lsin, lcos, lbin, kap, gtab, out);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_bluestein_filter(hipStream_t st, int nfft, const FftArgs *ffts, int nthreads, size_t lds)
{
    hipLaunchKernelGGL(k_bluestein_prep, dim3(nfft), dim3(nthreads), lds, st, ffts);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fadj_gather(hipStream_t st, int L, int ss, int nblk, int spin, const double *part, const int *mtop,
                              const double2 *flm, const double *wl, int hstride, double *F)
{
    if (hstride < L + ss) return hipErrorInvalidValue;
    const size_t tot = (size_t)L * (L + ss);
    hipLaunchKernelGGL(k_fadj_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, ss, nblk, spin, part,
                       mtop, flm, wl, hstride, F);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fadj_scatter(hipStream_t st, int L, int ss, int hstride, double q, const double *F,
                               const double2 *hpole, const double2 *hpoleN, double *out)
{
    if (ss && !hpoleN) return hipErrorInvalidValue;
    const size_t tot = (size_t)(L + ss) * L;
    hipLaunchKernelGGL(k_fadj_scatter, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, ss, hstride, q, F,
                       hpole, hpoleN, out);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_mask_low(hipStream_t st, int an, int n, int nreg, int hstride, const double *cot, const double *csc,
                           const double *FA, const double *FB, double *HxA, double *HxB)
{
    const size_t tot = (size_t)an * hstride;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mask_low, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, an, n, nreg, hstride, cot, csc,
                       FA, FB, HxA, HxB);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pole_from_F(hipStream_t st, int L, int hstride, int ring, const double *F, double2 *pole)
{
    hipLaunchKernelGGL(k_pole_from_F, dim3((2 * L - 1 + 255) / 256), dim3(256), 0, st, L, hstride, ring, F, pole);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

// Kernels with large dynamic LDS need the per-kernel limit raised.
hipError_t set_kernel_lds_limits(size_t max_dyn)
{
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_phi_inv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_phi_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_mw_filter, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_bluestein_prep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_phi_inv_real, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void *)k_phi_fwd_real, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace s2mi
