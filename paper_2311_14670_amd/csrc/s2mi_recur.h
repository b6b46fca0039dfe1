// s2mi_recur.h -- device helpers of the descending-m Wigner recursion shared by
// the fused FP64 sweeps (s2mi_kernels.hip) and the d-tile generator of the
// matrix-core path (s2mi_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace s2mi {

constexpr int RT = 600;   // realise once the scale exponent is above -RT
constexpr int SG = 8;     // degrees (or rings) per register chunk

__device__ __forceinline__ int ufl(int x) { return __builtin_amdgcn_readfirstlane(x); }

// exact power-of-two renormalisation of the pair (e, ep) carrying exponent E
// (running renormalisation, Sec. 3.4): while the scale exponent E is below
// -RT the pair is rescaled so its larger entry is in [1, 2); once E + k is
// above -RT it is realised (E = 0) and left unscaled from then on.
__device__ __forceinline__ void renorm(double &e, double &ep, int &E)
{
    const double mx = fmax(fabs(e), fabs(ep));
    // floor(log2 mx) = frexp exponent - 1 (mx is finite: the state grows by a bounded
    // factor between passes); a not-yet-started (zero) state keeps E
    const int k = mx > 0.0 ? __builtin_amdgcn_frexp_exp(mx) - 1 : 0;
    const bool real = (E + k >= -RT);
    const int sh = real ? E : -k;
    e = ldexp(e, sh);
    ep = ldexp(ep, sh);
    E = real ? 0 : E + k;
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
