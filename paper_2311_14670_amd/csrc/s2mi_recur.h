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
    const int k = mx > 0.0 ? ilogb(mx) : 0;          // a not-yet-started (zero) state keeps E
    const bool real = (E + k >= -RT);
    const int sh = real ? E : -k;
    e = ldexp(e, sh);
    ep = ldexp(ep, sh);
    E = real ? 0 : E + k;
}

}  // namespace s2mi
