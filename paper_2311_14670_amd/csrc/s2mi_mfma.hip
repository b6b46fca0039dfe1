// s2mi_mfma.hip -- batched l- and theta-contractions on the matrix cores.
//
// For a batch of B maps, at each order m the l-contraction of Eq. 33 (inverse)
// and the theta-contraction of Eq. 30 (forward) are products of a (4B x K)
// matrix -- coefficients or ring spectra, one row per (map, component) -- with
// the Wigner-d matrix D_m[l][ring] of the run's second index n.  D_m comes
// from the same FP64 descending-m recursion as the fused FP64 sweeps
// (Eqs. 25-27, running renormalisation of Sec. 3.4), generated for a chunk of
// consecutive orders at a time, realised (d = e g; a value not yet realised is
// below 2^-279 and rounds to zero) and rounded to the
// contraction format:
//   FP32        fp32 operands, one MFMA pass, fp32 accumulation;
//   split BF16  x = hi + lo, hi = bf16(x), lo = bf16(x - hi); three MFMA passes
//               hi*hi + hi*lo + lo*hi with fp32 accumulation.
// The recursion state of every (l, ring) is carried across order chunks in the
// workspace, so only one chunk of D is ever staged.
//
// Product rows: 4b + {Re A, Im A, Re B, Im B}; side A is the slice fed at +m,
// side B the slice fed at -m (sign (-1)^{m-n}), exactly as in the FP64 sweeps.
//
// Staging element: 32 bytes holding 8 consecutive K values for one row or
// column (fp32: 8 floats; split BF16: 8 hi then 8 lo).  Lane l of a 32x32
// MFMA tile supplies K values from chunk (k0 + l/32) for row / column l%32, so
// each operand is one 32-byte load.  The pairing of K values between the two
// operands is the same on both sides, which is all the contraction needs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "s2mi_internal.h"
#include "s2mi_mfma.h"
#include "s2mi_recur.h"

namespace s2mi {

typedef __bf16 bf16x8_t __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x16_t __attribute__((__vector_size__(16 * sizeof(float))));
typedef unsigned v4u __attribute__((ext_vector_type(4)));     // 16 staging bytes as a native vector

// ------------------------------------------------------------------ formats
__device__ __forceinline__ unsigned bf16_bits(float f)   // round to nearest even
{
    const unsigned u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(unsigned h) { return __uint_as_float(h << 16); }

// 8 values -> one 32-byte staging element
template <int FMT>
__device__ __forceinline__ void store_elem(uint4 *dst, const float (&v)[SG])
{
    if constexpr (FMT == S2_CONTRACT_FP32) {
        dst[0] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3]));
        dst[1] = make_uint4(__float_as_uint(v[4]), __float_as_uint(v[5]), __float_as_uint(v[6]), __float_as_uint(v[7]));
    } else {
        unsigned h[SG], l[SG];
#pragma unroll
        for (int k = 0; k < SG; ++k) {
            h[k] = bf16_bits(v[k]);
            l[k] = bf16_bits(v[k] - bf16_value(h[k]));
        }
        dst[0] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
        dst[1] = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
    }
}

__device__ __forceinline__ bf16x8_t as_bf16x8(v4u u) { return __builtin_bit_cast(bf16x8_t, u); }

__device__ __forceinline__ float elem_f32(v4u a, v4u b, int s)   // s compile-time after unrolling
{
    return __uint_as_float(s < 4 ? a[s] : b[s - 4]);
}

// acc[i][t] += A(tile i) * B(tile t) over one K step (16 values; one 32-byte element
// per lane and operand) for all of a wave's tiles, interleaved so that consecutive
// matrix instructions accumulate into different tiles (each tile's products depend
// on its previous one).  FP32: eight 32x32x2 products per tile; split BF16: three
// 32x32x16 products per tile, hi*hi, hi*lo, lo*hi.
template <int FMT, int MTW>
__device__ __forceinline__ void mfma_tiles(f32x16_t (&acc)[MTW][2], const bool (&mv)[MTW], const v4u (&ah)[MTW],
                                           const v4u (&al)[MTW], const v4u (&bh)[2], const v4u (&bl)[2])
{
    if constexpr (FMT == S2_CONTRACT_FP32) {
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < MTW; ++i) {
                if (!mv[i]) continue;
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(elem_f32(ah[i], al[i], s), elem_f32(bh[t], bl[t], s),
                                                                     acc[i][t], 0, 0, 0);
            }
    } else {
#pragma unroll
        for (int pass = 0; pass < 3; ++pass)
#pragma unroll
            for (int i = 0; i < MTW; ++i) {
                if (!mv[i]) continue;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const v4u a = pass == 2 ? al[i] : ah[i];
                    const v4u b = pass == 1 ? bl[t] : bh[t];
                    acc[i][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a), as_bf16x8(b), acc[i][t], 0, 0, 0);
                }
            }
    }
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ fill
__global__ void k_zero_words(unsigned *__restrict__ p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------ recursion tables
// kg[m][l] = {kappa_{m+1}^l, g_m^l} for m in [-nx, L) with l padded to lrow (zeros
// past L and where the plan tables hold zeros), so a chunk of 8 degrees is one load.
__global__ void k_kg_table(int L, int nx, int lrow, const double *__restrict__ kap, const double *__restrict__ gtab,
                           double2 *__restrict__ kg)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // rows m in [-nx, L); pointers at row 0
    if (i >= (size_t)(L + nx) * lrow) return;
    const int m = (int)(i / lrow) - nx, l = (int)(i % lrow);
    kg[(ptrdiff_t)m * lrow + l] = l < L ? make_double2(kap[(ptrdiff_t)m * L + l], gtab[(ptrdiff_t)m * L + l])
                                        : make_double2(0.0, 0.0);
}

// ------------------------------------------------------------------ d-tile generator
// Same sweep geometry as the fused inverse sweep: lanes = 64 rings, each wave
// owns NCH chunks of 8 consecutive degrees (slot e holds l = base + e).  Runs
// the orders m_hi .. m_lo (register roles fixed by the parity of m so a chunk
// boundary needs no fix-up; m_lo < 0 continues the run below m = 0), writing
// realised d values (zero at orders below |n| on rings where the run is the
// unstable one):
//   LAY 0 (K = l):    D[m - m_lo][l/8][ring][8 degrees]
//   LAY 1 (K = ring): D[m - m_lo][ring/8][l][8 rings]   (8x8 transposes through LDS)
template <int PAR, bool SLOW>
__device__ __forceinline__ void gen_chunk(double (&X)[SG], double (&Y)[SG], int (&E)[SG], const double2 *__restrict__ rec,
                                          double lam, int ein, double e0, int E0, float (&dv)[SG])
{
#pragma unroll
    for (int e = 0; e < SG; ++e) {
        double &nw = PAR == 0 ? Y[e] : X[e];              // receives order m
        double &od = PAR == 0 ? X[e] : Y[e];              // holds order m+1
        const double2 kgv = rec[e];
        nw = fma(kgv.x * lam, od, -nw);
        double t = nw;
        if constexpr (SLOW) {
            if (e == ein) {                               // l == m starts here
                nw = e0;
                od = 0.0;
                E[e] = E0;
            }
            renorm(nw, od, E[e]);
            t = nw;                                       // not yet realised: below 2^-279, 0 as a float
        }
        dv[e] = (float)(t * kgv.y);
    }
}

template <int NCH, int LAY, int FMT, int PAR>
__device__ __forceinline__ void gen_step(int m, int m_lo, int an, bool good, int ms, int kc_tot, int rpad, int lp,
                                         int ring0, int lane, int w, const int (&lb)[NCH], double (&X)[NCH][SG], double (&Y)[NCH][SG],
                                         int (&E)[NCH][SG], uint32_t &fast, double ct, double ncs,
                                         const double2 *__restrict__ initr, const double2 *__restrict__ kgm,
                                         float *tr, uint4 *__restrict__ D)
{
    const double lam = fma(-(double)(m + 1), ct, ncs);   // lambda_{m+1}: produces order m
    const size_t mc = (size_t)(m - m_lo);
#pragma unroll
    for (int g = 0; g < NCH; ++g) {
        const int base = lb[g];
        if (base < 0 || m > base + SG - 1) continue;     // chunk not started
        const double2 *rec = kgm + base;
        float dv[SG];
        if (m >= base) {                                  // ramp: slot m - base starts at this order
            const double2 iv = initr[m];                 // d^m_{m,n}(theta_ring), zero if m < |n|
            gen_chunk<PAR, true>(X[g], Y[g], E[g], rec, lam, m >= an ? m - base : -1, iv.x, (int)iv.y, dv);
            bool z = true;
#pragma unroll
            for (int e = 0; e < SG; ++e) z = z && (E[g][e] == 0);
            fast = __all(z) ? (fast | (1u << g)) : (fast & ~(1u << g));
        } else if (((fast >> g) & 1u) || (m & (RN - 1)) != 0) {
            // realised, or not a renormalisation order (a value not yet realised
            // stays below 2^-279 between passes and rounds to a zero float)
            gen_chunk<PAR, false>(X[g], Y[g], E[g], rec, lam, -1, 0.0, 0, dv);
        } else {
            gen_chunk<PAR, true>(X[g], Y[g], E[g], rec, lam, -1, 0.0, 0, dv);
            bool z = true;
#pragma unroll
            for (int e = 0; e < SG; ++e) z = z && (E[g][e] == 0);
            if (__all(z)) fast |= (1u << g);
        }
        if (good ? (m < 0 && -m >= ms) : (m < ms)) {      // values this run does not supply at this ring
#pragma unroll                                            // (the other run covers them): emitted as 0
            for (int e = 0; e < SG; ++e) dv[e] = 0.0f;
        }
        if constexpr (LAY == 0) {
            store_elem<FMT>(D + ((mc * kc_tot + base / SG) * rpad + ring0 + lane) * 2, dv);
        } else {
#pragma unroll
            for (int e = 0; e < SG; ++e) tr[e * 64 + lane] = dv[e];
            wave_lds_sync();
            const int e2 = lane >> 3, rg = lane & 7;
            float v[SG];
#pragma unroll
            for (int k = 0; k < SG; ++k) v[k] = tr[e2 * 64 + rg * SG + k];
            wave_lds_sync();
            store_elem<FMT>(D + ((mc * (rpad / SG) + ring0 / SG + rg) * lp + base + e2) * 2, v);
        }
    }
}

template <int NCH, int LAY, int FMT>
__global__ __launch_bounds__(512) void k_dgen(
    int L, int nreg, int rpad, int lp, int kc_tot, int lrow, int n, int m_hi, int m_lo,
    const double *__restrict__ cot, const double *__restrict__ csc, const double2 *__restrict__ init,
    const double2 *__restrict__ kg, const int *__restrict__ lchunk, const int *__restrict__ mtop,
    double *__restrict__ SX, double *__restrict__ SY, int *__restrict__ SE, uint4 *__restrict__ D)
{
    __shared__ float trbuf[LAY == 1 ? DSTAGE_MAX_WAVES * SG * 64 : 1];
    const int an = n < 0 ? -n : n;
    const int lane = threadIdx.x & 63;
    const int w = ufl(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int blk = blockIdx.y;
    const int ring0 = blockIdx.x * 64;
    const int ring = min(ring0 + lane, nreg - 1);        // lanes past the last ring duplicate it
    const double ct = cot[ring], cs = csc[ring];
    const double ncs = (double)n * cs;
    const double2 *initr = init + (size_t)ring * L;
    float *tr = trbuf + (LAY == 1 ? w * SG * 64 : 0);
    const bool good = ring_good(n, ct);                 // this run is the stable one at this ring
    const int ms = switch_order(n, ct, cs);

    int lb[NCH];
#pragma unroll
    for (int g = 0; g < NCH; ++g) lb[g] = ufl(lchunk[((size_t)blk * W + w) * NCH + g]);
    double X[NCH][SG], Y[NCH][SG];
    int E[NCH][SG];
    // state of slot (g, e) at SXw[(g SG + e) rpad + lane] (zeroed before a run's first chunk)
    const size_t sbase = ((((size_t)blk * W + w) * NCH) * SG) * rpad + ring0;
    double *SXw = SX + sbase, *SYw = SY + sbase;
    int *SEw = SE + sbase;
#pragma unroll
    for (int g = 0; g < NCH; ++g)
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int so = (g * SG + e) * rpad + lane;
            X[g][e] = SXw[so];
            Y[g][e] = SYw[so];
            E[g][e] = SEw[so];
        }
    uint32_t fast = 0;

    const int mt = ufl(mtop[blk]);
    int m = min(m_hi, mt);
    if (m >= m_lo && (m & 1)) {
        gen_step<NCH, LAY, FMT, 1>(m, m_lo, an, good, ms, kc_tot, rpad, lp, ring0, lane, w, lb, X, Y, E, fast, ct, ncs,
                                   initr, kg + (ptrdiff_t)m * lrow, tr, D);
        --m;
    }
    for (; m >= m_lo; m -= 2) {
        gen_step<NCH, LAY, FMT, 0>(m, m_lo, an, good, ms, kc_tot, rpad, lp, ring0, lane, w, lb, X, Y, E, fast, ct, ncs,
                                   initr, kg + (ptrdiff_t)m * lrow, tr, D);
        if (m - 1 >= m_lo)
            gen_step<NCH, LAY, FMT, 1>(m - 1, m_lo, an, good, ms, kc_tot, rpad, lp, ring0, lane, w, lb, X, Y, E, fast, ct,
                                       ncs, initr, kg + (ptrdiff_t)(m - 1) * lrow, tr, D);
    }
#pragma unroll
    for (int g = 0; g < NCH; ++g)
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int so = (g * SG + e) * rpad + lane;
            SXw[so] = X[g][e];
            SYw[so] = Y[g][e];
            SEw[so] = E[g][e];
        }
}

// ------------------------------------------------------------------ operand packs
// Inverse: A[m - m_lo][l/8][row][8 degrees], row = 4b + comp,
//   comp 0,1: wA_l flmA[b][l][m]   comp 2,3: (-1)^{m-n} wB_l flmB[b][l][-m]
//   (the B rows at m > 0, and at m <= 0 for n != 0: the run's continuation)
// zero for l < max(m, |n|), l >= L, b >= B.
// A workgroup packs the tile (32 orders) x (one degree chunk kc) x (8 maps): the
// coefficients are read with lanes along the orders (contiguous in flm), staged in
// LDS as floats, and written with lanes along the tile's 32 rows (contiguous in A).
constexpr int PK_M = 32, PK_B = 8;                       // orders and maps per pack tile
template <int FMT>
__global__ __launch_bounds__(256) void k_pack_a(int L, int n, int m_lo, int mcn, int kc_tot, int rpad_rows, int B,
                                                long long mstride, const double2 *__restrict__ flmA,
                                                const double2 *__restrict__ flmB, const double *__restrict__ wA,
                                                const double *__restrict__ wB, uint4 *__restrict__ A)
{
    constexpr int RS = PK_M * (SG + 1) + 1;              // LDS row stride (floats): conflict-free both ways
    __shared__ float sh[4 * PK_B * RS];                  // [row = 4 b + comp][order][degree]
    const int kc = blockIdx.x, tb = blockIdx.y, m0 = blockIdx.z * PK_M;
    const int t = threadIdx.x;
    const int an = n < 0 ? -n : n;
    const int M = 2 * L - 1;
    {
        const int mi = t & (PK_M - 1), e = t >> 5;       // lanes along the orders; e: degree in the chunk
        const int m = m_lo + m0 + mi;
        const int l = kc * SG + e;
        const int lmin = m > an ? m : an;
        const bool ok = m0 + mi < mcn && l < L && l >= lmin;
        const bool sideB = flmB && (m > 0 || an > 0);
        const double sgB = ((m - n) & 1) ? -1.0 : 1.0;
        // a side that is absent (one-sided runs) has neither coefficients nor weights
        const double wa = ok && flmA ? wA[l] : 0.0, wb = ok && sideB ? sgB * wB[l] : 0.0;
#pragma unroll 2
        for (int bi = 0; bi < PK_B; ++bi) {
            const int b = PK_B * tb + bi;
            double2 xa = make_double2(0.0, 0.0), xb = make_double2(0.0, 0.0);
            if (ok && b < B) {
                if (flmA) {
                    const double2 v = flmA[(size_t)b * mstride + (size_t)l * M + (L - 1) + m];
                    xa = make_double2(wa * v.x, wa * v.y);
                }
                if (sideB) {
                    const double2 v = flmB[(size_t)b * mstride + (size_t)l * M + (L - 1) - m];
                    xb = make_double2(wb * v.x, wb * v.y);
                }
            }
            float *r = sh + (4 * bi) * RS + mi * (SG + 1) + e;
            r[0] = (float)xa.x;
            r[RS] = (float)xa.y;
            r[2 * RS] = (float)xb.x;
            r[3 * RS] = (float)xb.y;
        }
    }
    __syncthreads();
    const int row = t & 31;                              // lanes along the rows 4 b + comp of the tile
#pragma unroll
    for (int q = 0; q < PK_M / 8; ++q) {
        const int mi = (t >> 5) + 8 * q;
        if (m0 + mi >= mcn) break;
        float v[SG];
#pragma unroll
        for (int e = 0; e < SG; ++e) v[e] = sh[row * RS + mi * (SG + 1) + e];
        store_elem<FMT>(A + (((size_t)(m0 + mi) * kc_tot + kc) * rpad_rows + 4 * PK_B * tb + row) * 2, v);
    }
}

// Forward: H[m - m_lo][ring/8][row][8 rings] from the ring spectra F[b][|m|][ring][4]:
//   comp 0,1: FA components 0,1 (m >= 0) or 2,3 (m < 0: the A slice at order m);
//   comp 2,3: FB components 2,3 (m > 0) or 0,1 (m <= 0: the B slice at order -m);
// zero past the swept rings, for b >= B, and at orders below |n| where the ring's
// values come from the other run (see the switch order in s2mi_recur.h).
// A workgroup packs the tile (one order m) x (64 rings) x (8 maps): the ring records
// are read with lanes along the rings (contiguous in F), staged in LDS as floats, and
// written with lanes along the tile's 32 rows.
template <int FMT>
__global__ __launch_bounds__(256) void k_pack_h(int m_lo, int mcn, int rpad, int nreg, int hstride, int rpad_rows, int B,
                                                long long fstride, int n, const double *__restrict__ cot,
                                                const double *__restrict__ csc, const double *__restrict__ FA,
                                                const double *__restrict__ FB, uint4 *__restrict__ H)
{
    constexpr int RS = 64 + 1;                           // LDS row stride (floats)
    __shared__ float sh[4 * PK_B * RS];                  // [row = 4 b + comp][ring in the tile]
    const int kr0 = blockIdx.x * (64 / SG), tb = blockIdx.y, mc = blockIdx.z;
    const int t = threadIdx.x;
    const int m = m_lo + mc;
    const int am = m < 0 ? -m : m, an = n < 0 ? -n : n;
    const int cA = m < 0 ? 2 : 0;                        // A side: components 0,1 (m >= 0) or 2,3 (m < 0)
    const int cB = m > 0 ? 2 : 0;                        // B side: components 2,3 (m > 0) or 0,1 (m <= 0)
    {
        const int ri = t & 63;                           // lanes along the rings
        const int ring = kr0 * SG + ri;
        bool useA = ring < nreg, useB = ring < nreg;
        if (ring < nreg && m < an) {                     // low orders: own values or continuation
            const double ct = cot[ring];
            const bool good = ring_good(n, ct);
            const int ms = switch_order(n, ct, csc[ring]);
            useA = m < 0 ? (good && am < ms) : (good || m >= ms);
            useB = m <= 0 ? (good && am < ms) : (good || m >= ms);
        }
#pragma unroll
        for (int q = 0; q < PK_B / 4; ++q) {
            const int bi = (t >> 6) + 4 * q;
            const int b = PK_B * tb + bi;
            double2 xa = make_double2(0.0, 0.0), xb = make_double2(0.0, 0.0);
            if (b < B) {
                const size_t rec = (size_t)b * fstride + ((size_t)am * hstride + ring) * 4;
                if (FA && useA) xa = *reinterpret_cast<const double2 *>(FA + rec + cA);
                if (FB && useB) xb = *reinterpret_cast<const double2 *>(FB + rec + cB);
            }
            float *r = sh + (4 * bi) * RS + ri;
            r[0] = (float)xa.x;
            r[RS] = (float)xa.y;
            r[2 * RS] = (float)xb.x;
            r[3 * RS] = (float)xb.y;
        }
    }
    __syncthreads();
    const int row = t & 31, k8 = t >> 5;                 // lanes along the rows; k8: ring chunk of the tile
    float v[SG];
#pragma unroll
    for (int k = 0; k < SG; ++k) v[k] = sh[row * RS + k8 * SG + k];
    const int kr_tot = rpad / SG;
    store_elem<FMT>(H + (((size_t)mc * kr_tot + kr0 + k8) * rpad_rows + 4 * PK_B * tb + row) * 2, v);
}

// ------------------------------------------------------------------ contractions
// Contraction tiles are dispatched XCD-aware (xcd_tile): the tiles of one order share
// that order's coefficient or spectra operand (A_m / H_m, 2 MB at L = 2048, B = 64).

// 256 threads = 4 waves; each wave owns MTW 32-row tiles (rows of maps) and two
// 32-column tiles.  Inverse: columns = 64 rings, K = degrees l >= max(m, |n|).
// Output of map b, ring r, order m: partA[b][r][m][0,1], partB[b][r][m][2,3].
template <int FMT, int MTW>
__global__ __launch_bounds__(256) void k_mfma_inv(int gx, int gy, int gz, bool xcd, int L, int nreg, int rpad, int kc_tot, int n,
                                                  int m_lo, int B,
                                                  int rpad_rows, const double *__restrict__ cot,
                                                  const double *__restrict__ csc, const uint4 *__restrict__ A,
                                                  const uint4 *__restrict__ D,
                                                  double *__restrict__ PA, double *__restrict__ PB, long long pstride)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int half = lane >> 5, li = lane & 31;
    int bx, by, bz;
    if (!xcd_tile(gx, gy, gz, bx, by, bz, xcd)) return;
    const int ring0 = bx * 64;
    const int mc = by, m = m_lo + mc;
    const int MT = rpad_rows / 32;
    const int an = n < 0 ? -n : n;
    const int kc0 = (m > an ? m : an) / SG;
    int mts[MTW];
    bool mv[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
        mts[i] = bz * 4 * MTW + w + 4 * i;
        mv[i] = mts[i] < MT;
    }
    if (!mv[0]) return;
    f32x16_t acc[MTW][2];
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[i][t][j] = 0.0f;
    const v4u *Dm = (const v4u *)D + (size_t)mc * kc_tot * rpad * 2;
    const v4u *Am = (const v4u *)A + (size_t)mc * kc_tot * rpad_rows * 2;
    const v4u z4 = {0u, 0u, 0u, 0u};
    for (int kc = kc0; kc < kc_tot; kc += 2) {
        const int kk = kc + half;
        const bool kv = kk < kc_tot;
        v4u bh[2], bl[2], ah[MTW], al[MTW];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const v4u *p = Dm + ((size_t)(kv ? kk : 0) * rpad + ring0 + t * 32 + li) * 2;
            bh[t] = kv ? p[0] : z4;
            bl[t] = kv ? p[1] : z4;
        }
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
            const v4u *p = Am + ((size_t)(kv ? kk : 0) * rpad_rows + (mv[i] ? mts[i] : 0) * 32 + li) * 2;
            ah[i] = (kv && mv[i]) ? p[0] : z4;
            al[i] = (kv && mv[i]) ? p[1] : z4;
        }
        mfma_tiles<FMT, MTW>(acc, mv, ah, al, bh, bl);
    }
    // C layout of a 32x32 tile: lane l, entry j -> row 8(j/4) + 4(l/32) + j%4, column l%32
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
        if (!mv[i]) continue;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int ring = ring0 + t * 32 + li;
            // orders below |n|: only the run that is stable at this ring writes; its
            // continuation (m <= 0) feeds the A slice at m < 0 (components 2,3 at |m|)
            // and the B slice at -m >= 0 (components 0,1 at |m|)
            bool good = false;
            int ms = 0;
            if (an > 0 && ring < nreg) {
                const double ct = cot[ring];
                good = ring_good(n, ct);
                ms = switch_order(n, ct, csc[ring]);
            }
            const bool ext_ok = good && m <= 0 && -m < ms;
            const bool wa = m >= 0 && (good || m >= ms), wa_x = m < 0 && ext_ok;
            const bool wb = m > 0 && (good || m >= ms), wb_x = ext_ok;
            const int am = m < 0 ? -m : m;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int b = mts[i] * 8 + 2 * q + half;
                if (b < B && ring < nreg) {
                    const size_t o = ((size_t)ring * L + am) * 4;
                    const double2 va = make_double2((double)acc[i][t][4 * q + 0], (double)acc[i][t][4 * q + 1]);
                    const double2 vb = make_double2((double)acc[i][t][4 * q + 2], (double)acc[i][t][4 * q + 3]);
                    if (PA && wa) *(double2 *)(PA + (size_t)b * pstride + o) = va;
                    if (PA && wa_x) *(double2 *)(PA + (size_t)b * pstride + o + 2) = va;
                    if (PB && wb) *(double2 *)(PB + (size_t)b * pstride + o + 2) = vb;
                    if (PB && wb_x) *(double2 *)(PB + (size_t)b * pstride + o) = vb;
                }
            }
        }
    }
}

// Forward: columns = 64 degrees l, K = rings.  Output Q[b][l][m][comp] for
// l >= m (degrees below max(m, |n|) carry zero d and give zero).
template <int FMT, int MTW>
__global__ __launch_bounds__(256) void k_mfma_fwd(int gx, int gy, int gz, int L, int rpad, int lp, int n, int m_lo,
                                                  int B, int rpad_rows,
                                                  int nxp, const uint4 *__restrict__ H, const uint4 *__restrict__ D,
                                                  double *__restrict__ QA, double *__restrict__ QB,
                                                  long long qstride, double *__restrict__ QxA,
                                                  double *__restrict__ QxB, long long qxstride)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int half = lane >> 5, li = lane & 31;
    int bx, by, bz;
    if (!xcd_tile(gx, gy, gz, bx, by, bz)) return;
    const int l0 = bx * 64;
    const int mc = by, m = m_lo + mc;
    const int an = n < 0 ? -n : n, am = m < 0 ? -m : m;
    if (l0 + 63 < m) return;
    const int MT = rpad_rows / 32;
    int mts[MTW];
    bool mv[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
        mts[i] = bz * 4 * MTW + w + 4 * i;
        mv[i] = mts[i] < MT;
    }
    if (!mv[0]) return;
    f32x16_t acc[MTW][2];
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[i][t][j] = 0.0f;
    const int kr_tot = rpad / SG;                        // a multiple of 8
    const v4u *Dm = (const v4u *)D + (size_t)mc * kr_tot * lp * 2;
    const v4u *Hm = (const v4u *)H + (size_t)mc * kr_tot * rpad_rows * 2;
    const v4u z4 = {0u, 0u, 0u, 0u};
    for (int kr = 0; kr < kr_tot; kr += 2) {
        const int kk = kr + half;
        v4u bh[2], bl[2], ah[MTW], al[MTW];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const v4u *p = Dm + ((size_t)kk * lp + l0 + t * 32 + li) * 2;
            bh[t] = p[0];
            bl[t] = p[1];
        }
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
            const v4u *p = Hm + ((size_t)kk * rpad_rows + (mv[i] ? mts[i] : 0) * 32 + li) * 2;
            ah[i] = mv[i] ? p[0] : z4;
            al[i] = mv[i] ? p[1] : z4;
        }
        mfma_tiles<FMT, MTW>(acc, mv, ah, al, bh, bl);
    }
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
        if (!mv[i]) continue;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int l = l0 + t * 32 + li;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int b = mts[i] * 8 + 2 * q + half;
                if (b < B && l < L && l >= m) {
                    const double2 va = make_double2((double)acc[i][t][4 * q + 0], (double)acc[i][t][4 * q + 1]);
                    const double2 vb = make_double2((double)acc[i][t][4 * q + 2], (double)acc[i][t][4 * q + 3]);
                    // continuation sums (orders m <= 0 of a run with n != 0): the A slice at
                    // order m < 0 and the B slice at order -m, signed to cancel the finish's
                    // (-1)^{|m| - spin} on negative orders / give d^l_{-m,-n} = (-1)^{m-n} d^l_{m,n}
                    const double sg = ((am + n) & 1) ? -1.0 : 1.0;
                    if (m >= 0) {
                        const size_t o = ((size_t)l * L + m) * 4;
                        if (QA) *(double2 *)(QA + (size_t)b * qstride + o) = va;
                        if (QB && m > 0) *(double2 *)(QB + (size_t)b * qstride + o + 2) = vb;
                    } else if (QxA) {
                        *(double2 *)(QxA + (size_t)b * qxstride + ((size_t)l * nxp + am) * 4 + 2) =
                            make_double2(sg * va.x, sg * va.y);
                    }
                    if (m <= 0 && an > 0 && QxB)
                        *(double2 *)(QxB + (size_t)b * qxstride + ((size_t)l * nxp + am) * 4) =
                            make_double2(sg * vb.x, sg * vb.y);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ launchers
#define S2_LAUNCH_CHECK()                          \
    do {                                           \
        hipError_t e_ = hipGetLastError();         \
        if (e_ != hipSuccess) return e_;           \
    } while (0)

hipError_t launch_zero(hipStream_t st, void *p, size_t bytes)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (unsigned *)p, n);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_kg_table(hipStream_t st, int L, int nx, int lrow, const double *kap, const double *gtab,
                           double2 *kg)
{
    const size_t tot = (size_t)(L + nx) * lrow;
    hipLaunchKernelGGL(k_kg_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, nx, lrow, kap, gtab, kg);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_dgen(hipStream_t st, int layout, int fmt, int nwaves, int nblk, const MfmaGeom &g, int n, int m_hi,
                       int m_lo, const double *cot, const double *csc, const double2 *init,
                       const double2 *kg, const int *lchunk, const int *mtop, double *SX, double *SY, int *SE,
                       uint4 *D)
{
    if (nwaves < 1 || nwaves > DSTAGE_MAX_WAVES || g.rpad % 64 || m_lo <= -g.L || m_hi >= g.L || m_lo > m_hi)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)(g.rpad / 64), (unsigned)nblk), block((unsigned)(64 * nwaves));
#define S2_DGEN(LAY, FMT)                                                                                   \
    hipLaunchKernelGGL((k_dgen<GEN_NCH, LAY, FMT>), grid, block, 0, st, g.L, g.nreg, g.rpad, g.lp, g.kc,    \
                       g.lrow, n, m_hi, m_lo, cot, csc, init, kg, lchunk, mtop, SX, SY, SE, D)
    if (layout == 0 && fmt == S2_CONTRACT_FP32) S2_DGEN(0, S2_CONTRACT_FP32);
    else if (layout == 0) S2_DGEN(0, S2_CONTRACT_SPLIT_BF16);
    else if (fmt == S2_CONTRACT_FP32) S2_DGEN(1, S2_CONTRACT_FP32);
    else S2_DGEN(1, S2_CONTRACT_SPLIT_BF16);
#undef S2_DGEN
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pack_a(hipStream_t st, int fmt, const MfmaGeom &g, int n, int m_lo, int mcn, int B,
                         long long mstride, const double2 *flmA, const double2 *flmB, const double *wA,
                         const double *wB, uint4 *A)
{
    if (g.rows % (4 * PK_B) != 0) return hipErrorInvalidValue;   // whole 8-map tiles of rows
    const dim3 grid((unsigned)g.kc, (unsigned)(g.rows / (4 * PK_B)), (unsigned)((mcn + PK_M - 1) / PK_M)), block(256);
    if (fmt == S2_CONTRACT_FP32)
        hipLaunchKernelGGL(k_pack_a<S2_CONTRACT_FP32>, grid, block, 0, st, g.L, n, m_lo, mcn, g.kc, g.rows, B,
                           mstride, flmA, flmB, wA, wB, A);
    else
        hipLaunchKernelGGL(k_pack_a<S2_CONTRACT_SPLIT_BF16>, grid, block, 0, st, g.L, n, m_lo, mcn, g.kc, g.rows, B,
                           mstride, flmA, flmB, wA, wB, A);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_pack_h(hipStream_t st, int fmt, const MfmaGeom &g, int hstride, int n, const double *cot,
                         const double *csc, int m_lo, int mcn, int B, long long fstride, const double *FA,
                         const double *FB, uint4 *H)
{
    if (g.rows % (4 * PK_B) != 0 || g.rpad % 64 != 0) return hipErrorInvalidValue;   // whole tiles
    const dim3 grid((unsigned)(g.rpad / 64), (unsigned)(g.rows / (4 * PK_B)), (unsigned)mcn), block(256);
    if (fmt == S2_CONTRACT_FP32)
        hipLaunchKernelGGL(k_pack_h<S2_CONTRACT_FP32>, grid, block, 0, st, m_lo, mcn, g.rpad, g.nreg, hstride, g.rows,
                           B, fstride, n, cot, csc, FA, FB, H);
    else
        hipLaunchKernelGGL(k_pack_h<S2_CONTRACT_SPLIT_BF16>, grid, block, 0, st, m_lo, mcn, g.rpad, g.nreg, hstride,
                           g.rows, B, fstride, n, cot, csc, FA, FB, H);
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_mfma_inv(hipStream_t st, int fmt, const MfmaGeom &g, int n, const double *cot, const double *csc,
                           int m_lo, int mcn, int B, const uint4 *A, const uint4 *D, double *PA, double *PB,
                           long long pstride)
{
    const int MT = g.rows / 32;
    const int mtw = MT <= 4 ? 1 : 2;
    // the inverse products keep the plain tile order (ring tile fastest): with the XCD-aware
    // order they took 0.474 -> 0.542 ms per 32-order chunk (FP32, 64 maps at L = 2048),
    // while the forward products gained (0.717 -> 0.585 ms)
    const int gx = g.rpad / 64, gy = mcn, gz = (MT + 4 * mtw - 1) / (4 * mtw);
    const dim3 grid((unsigned)(gx * gy * gz)), block(256);
#define S2_MI(FMT, MTW)                                                                                        \
    hipLaunchKernelGGL((k_mfma_inv<FMT, MTW>), grid, block, 0, st, gx, gy, gz, false, g.L, g.nreg, g.rpad, g.kc, n, m_lo, \
                       B, g.rows, cot, csc, A, D, PA, PB, pstride)
    if (fmt == S2_CONTRACT_FP32) { if (mtw == 1) S2_MI(S2_CONTRACT_FP32, 1); else S2_MI(S2_CONTRACT_FP32, 2); }
    else { if (mtw == 1) S2_MI(S2_CONTRACT_SPLIT_BF16, 1); else S2_MI(S2_CONTRACT_SPLIT_BF16, 2); }
#undef S2_MI
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_mfma_fwd(hipStream_t st, int fmt, const MfmaGeom &g, int n, int nxp, int m_lo, int mcn, int B,
                           const uint4 *H, const uint4 *D, double *QA, double *QB, long long qstride, double *QxA,
                           double *QxB, long long qxstride)
{
    const int MT = g.rows / 32;
    const int mtw = MT <= 4 ? 1 : 2;
    const int gx = g.lp / 64, gy = mcn, gz = (MT + 4 * mtw - 1) / (4 * mtw);
    const dim3 grid((unsigned)((gx * gy * gz + NXCD - 1) / NXCD * NXCD)), block(256);
#define S2_MF(FMT, MTW)                                                                                          \
    hipLaunchKernelGGL((k_mfma_fwd<FMT, MTW>), grid, block, 0, st, gx, gy, gz, g.L, g.rpad, g.lp, n, m_lo, B, g.rows, \
                       nxp, H, D, QA, QB, qstride, QxA, QxB, qxstride)
    if (fmt == S2_CONTRACT_FP32) { if (mtw == 1) S2_MF(S2_CONTRACT_FP32, 1); else S2_MF(S2_CONTRACT_FP32, 2); }
    else { if (mtw == 1) S2_MF(S2_CONTRACT_SPLIT_BF16, 1); else S2_MF(S2_CONTRACT_SPLIT_BF16, 2); }
#undef S2_MF
    S2_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace s2mi
