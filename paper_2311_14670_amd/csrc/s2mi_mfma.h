// s2mi_mfma.h -- host launchers of the matrix-core contraction path (s2mi_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "s2mi.h"
#include "s2mi_internal.h"

namespace s2mi {

// Shapes shared by the generator, the packs and the contractions.
struct MfmaGeom {
    int L;
    int nreg;    // swept rings
    int rpad;    // rings padded to 64 (generator lanes, K of the forward product)
    int lp;      // degrees padded to 64 (columns of the forward product)
    int kc;      // 8-degree chunks, ceil(L/8) (K of the inverse product)
    int lrow;    // row length of the {kappa, g} table, 8 kc
    int rows;    // product rows 4 B padded to 32
};

// zero a byte range (multiple of 4) with a fill kernel
hipError_t launch_zero(hipStream_t st, void *p, size_t bytes);
hipError_t launch_kg_table(hipStream_t st, int L, int nx, int lrow, const double *kap, const double *gtab,
                           double2 *kg);
// layout 0: D[m][l/8][ring][8] (inverse);  layout 1: D[m][ring/8][l][8] (forward)
hipError_t launch_dgen(hipStream_t st, int layout, int fmt, int nwaves, int nblk, const MfmaGeom &g, int n, int m_hi,
                       int m_lo, const double *cot, const double *csc, const double2 *init,
                       const double2 *kg, const int *lchunk, const int *mtop, double *SX, double *SY, int *SE,
                       uint4 *D);
hipError_t launch_pack_a(hipStream_t st, int fmt, const MfmaGeom &g, int n, int m_lo, int mcn, int B,
                         long long mstride, const double2 *flmA, const double2 *flmB, const double *wA,
                         const double *wB, uint4 *A);
hipError_t launch_pack_h(hipStream_t st, int fmt, const MfmaGeom &g, int hstride, int n, const double *cot,
                         const double *csc, int m_lo, int mcn, int B, long long fstride, const double *FA,
                         const double *FB, uint4 *H);
hipError_t launch_mfma_inv(hipStream_t st, int fmt, const MfmaGeom &g, int n, const double *cot, const double *csc,
                           int m_lo, int mcn, int B, const uint4 *A, const uint4 *D, double *PA, double *PB,
                           long long pstride);
hipError_t launch_mfma_fwd(hipStream_t st, int fmt, const MfmaGeom &g, int n, int nxp, int m_lo, int mcn, int B,
                           const uint4 *H, const uint4 *D, double *QA, double *QB, long long qstride, double *QxA,
                           double *QxB, long long qxstride);

}  // namespace s2mi
