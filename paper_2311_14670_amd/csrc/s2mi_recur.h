// s2mi_recur.h -- device helpers of the descending-m Wigner recursion shared by
// the fused FP64 sweeps (s2mi_kernels.hip) and the d-tile generator of the
// matrix-core path (s2mi_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace s2mi {

constexpr int RT = 600;   // realise once the scale exponent is above -RT
constexpr int SG = 8;     // degrees (or rings) per register chunk
// Renormalisation period of the recursion (orders; a power of two).  The state grows
// by at most |kappa lambda| + 1 < 2^20 per order for L <= 4096 (|lambda| sin theta <=
// |n| + m + 1 with kappa (|n| + m + 1) <= 181 over every degree below 4096, and
// sin theta >= 1.9e-4 on every grid's swept rings), so between passes a pair scaled
// near 2^-RT stays below 2^-279: far from overflow, and its unscaled contribution
// negligible (see renorm).
constexpr int RN = 16;

__device__ __forceinline__ int ufl(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Tile order of the sweeps and contractions.  Workgroups are dispatched round-robin
// over the 8 XCDs (workgroup i to XCD i mod 8), each with its own L2.  With xcd set, a
// 1-D grid of ceil(gx gy gz / 8) * 8 workgroups is remapped so that every XCD takes one
// contiguous run of the tiles, ordered z fastest, then x, then y: tiles that share an
// operand along x (and every z) then read it through one L2, while each XCD still
// gets tiles of every z.  Without xcd, workgroup i is tile i in x-fastest order.
// Returns false for the padding of the grid.
constexpr int NXCD = 8;
__device__ __forceinline__ bool xcd_tile(int gx, int gy, int gz, int &bx, int &by, int &bz, bool xcd = true)
{
    const int T = gx * gy * gz;
    const int i = (int)blockIdx.x;
    if (!xcd) {
        if (i >= T) return false;
        bx = i % gx;
        const int r = i / gx;
        by = r % gy;
        bz = r / gy;
        return true;
    }
    const int per = (T + NXCD - 1) / NXCD;
    const int j = (i % NXCD) * per + i / NXCD;
    if (j >= T) return false;
    bz = j % gz;
    const int r = j / gz;
    bx = r % gx;
    by = r / gx;
    return true;
}

// State of one recursion slot: the pair (e, ep) and an int E, the slot's values
// being e 2^E and ep 2^E.  Realised (E = 0): e is the value itself.  Not yet realised
// (value below 2^-RT): E < 0 and the pair is kept scaled near 2^-RT, so a sweep can use
// e unscaled in its contraction -- such a slot then contributes at most about
// 2^(321 - RT) times its record (the growth between two passes of the sweeps is below
// 2^320) instead of its exact (equally negligible) value, and no exponent scaling is
// needed per step.  A slot that has not started holds zeros
// with E = 0.

// Exact power-of-two renormalisation of the pair (e, ep) carrying exponent E
// (running renormalisation, Sec. 3.4): a pair whose value is below 2^-RT is rescaled
// so its larger entry is in [2^-RT, 2^(1-RT)), E absorbing the change; a pair whose
// value is at least 2^-RT is realised (E = 0, values unscaled from then on).  Every
// scaling is by a power of two, so the values themselves never change.
__device__ __forceinline__ void renorm(double &e, double &ep, int &E)
{
    const double mx = fmax(fabs(e), fabs(ep));
    // floor(log2 mx) = frexp exponent - 1 (mx is finite: the state grows by a bounded
    // factor between passes); a not-yet-started (zero) state keeps E
    const int k = mx > 0.0 ? __builtin_amdgcn_frexp_exp(mx) - 1 : 0;
    const bool real = (E + k >= -RT);                   // the value's exponent is E + k
    const int sh = real ? E : -k - RT;
    e = ldexp(e, sh);
    ep = ldexp(ep, sh);
    E = real ? 0 : E + k + RT;                           // < 0: E + k < -RT
}

// Stable-direction switch for runs with n != 0.  At a ring the descending
// recursion of d^l_{m,n} grows (is stable) down to about m = n cos(theta); for
// the run with n cos(theta) > 0 the orders m < ms = ceil(|n cos(theta)|) are
// taken instead from the run -n (which is stable down to m = -ms) via
// d^l_{m,n} = (-1)^{m-n} d^l_{-m,-n}.  ring_good: this run is the one with
// n cos(theta) < 0 (ties: n < 0) at the ring; switch_order: ms in [0, |n|].
__device__ __forceinline__ bool ring_good(int n, double ct)
{
    return n != 0 && ((double)n * ct < 0.0 || (ct == 0.0 && n < 0));
}

__device__ __forceinline__ int switch_order(int n, double ct, double cs)
{
    const int an = n < 0 ? -n : n;
    if (an == 0) return 0;
    const int ms = (int)ceil(fabs((double)n * ct / cs) - 1e-9);   // |n cos(theta)|, cos = cot / csc
    return ms < 0 ? 0 : (ms > an ? an : ms);
}

}  // namespace s2mi
