// s2mi_kernels.h -- host launchers of the gfx950 kernels (s2mi_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "s2mi_internal.h"

namespace s2mi {

hipError_t launch_pack_inv(hipStream_t st, int L, int nx, int n, int nblk, int slots_per_blk, const int *lslot,
                           const double2 *flmA, const double2 *flmB, const double *wA, const double *wB,
                           const double *kap, const double *gtab, double *C, int side = 0);
hipError_t launch_dstage_inv(hipStream_t st, int nwaves, int nblk, int L, int nx, int nreg, int n, const double *cot,
                             const double *csc, const double2 *init, const double *C, const int *lchunk,
                             const int *mtop, double *partA, double *partB, int side, int nsw,
                             const OrderTiles &ot);
hipError_t launch_init_table(hipStream_t st, int L, int nreg, int n, const double *lsin, const double *lcos,
                             const double *lbin, double2 *init);
hipError_t launch_dstage_fwd(hipStream_t st, int nwaves, int nblk, int G, int L, int nxp, int nreg, int hstride,
                             int lstride, int n, const double *lam, const double2 *init, const double *kap,
                             const double *gtab, const double *HA, const double *HB, const double *HxA,
                             const double *HxB, double *QA, double *QB, double *QxA, double *QxB, int side,
                             int pair, const OrderTiles &ot);
// The recursion state at the order-tile cuts of one run (see OrderTiles): rings
// [0, rp) (zero past nreg), degrees l >= c[k] of each cut k >= 1.
hipError_t launch_order_ckpt(hipStream_t st, int L, int nreg, int n, const double *cot, const double *csc,
                             const double2 *init, const double *kap, const OrderTiles &ot, double *ck);
hipError_t launch_pair_spectra(hipStream_t st, int L, int nreg, int nsw, int hstride, int pstride, const double *H,
                               double *S, double *D);
hipError_t launch_lambda_table(hipStream_t st, int L, int nx, int nreg, int lstride, int n, const double *cot,
                               const double *csc, double *lam);
hipError_t launch_phi_inv(hipStream_t st, int nthreads, size_t lds, int nring, int L, int nreg, int nblk, int spin,
                          const double *part, const int *mtop, const double2 *flm, const double *wl,
                          const int *ring_nphi, const long long *ring_start, const int *ring_shift,
                          const int *ring_fft, const FftArgs *ffts, double2 *map, double2 *fscr);
hipError_t launch_phi_fwd(hipStream_t st, int nthreads, size_t lds, int nring, int hstride, int L, double q,
                          const double2 *map,
                          const int *ring_nphi, const long long *ring_start, const int *ring_shift,
                          const int *ring_fft, const FftArgs *ffts, const double *ringq, double *F,
                          double2 *fscr);
hipError_t launch_mw_filter(hipStream_t st, int nthreads, size_t lds, int L, int ss, int hstride, int spin,
                            const FftArgs *fN, const double *wq, const double *ph, double *F, double2 *hpole,
                            double2 *hpoleN, double2 *fscr, int half, int adj, const FftArgs *fconv);
hipError_t launch_ring_scale(hipStream_t st, int nring, int nphi, const double *w, double2 *map);
hipError_t launch_ring_scale_real(hipStream_t st, int nring, const long long *ring_start, const int *ring_nphi,
                                  const double *w, double *map);
hipError_t launch_hermitian_part(hipStream_t st, int L, const double2 *G, double2 *out);
hipError_t launch_finish_fwd(hipStream_t st, int L, int nblk, int spin, int nB, const double *Q, const double *Qx,
                             int nxp, const double *wl, const double2 *hpole, const double2 *hpoleN,
                             double2 *flm, int half = 0);
// real signals (spin 0): pairs of rings share one complex DFT; maps are real doubles
hipError_t launch_phi_inv_real(hipStream_t st, int nthreads, size_t lds, int npair, int L, int nreg, int nblk,
                               const int *pairs, const double *part, const int *mtop, const double2 *flm,
                               const double *wl, const int *ring_nphi, const long long *ring_start,
                               const int *ring_shift, const int *ring_fft, const FftArgs *ffts, double *map,
                               double2 *fscr);
hipError_t launch_phi_fwd_real(hipStream_t st, int nthreads, size_t lds, int nring, int hstride, int npair, int L,
                               double q, const int *pairs, const double *map, const int *ring_nphi,
                               const long long *ring_start, const int *ring_shift, const int *ring_fft,
                               const FftArgs *ffts, const double *ringq, double *F, double2 *fscr);
hipError_t launch_gamma_dft(hipStream_t st, int N, long long nper, int sign, double q, const double *roots,
                            const double2 *in, double2 *out);
// Debug unitarity sums: out[i][l] = {sum_{m >= 0} (d^l_{m,n}(theta_{rsel[i]}))^2, d^l_{0,n}}.
hipError_t launch_unitarity(hipStream_t st, int L, int n, int nsel, const int *rsel, const double *cot,
                           const double *csc, const double *lsin, const double *lcos, const double *lbin,
                           const double *kap, const double *gtab, double *out);
hipError_t launch_debug_d(hipStream_t st, int L, int nreg, int n, const double *cot, const double *csc,
                          const double *lsin, const double *lcos, const double *lbin, const double *kap,
                          const double *gtab, double *out);
hipError_t launch_bluestein_filter(hipStream_t st, int nfft, const FftArgs *ffts, int nthreads, size_t lds);
hipError_t launch_fadj_gather(hipStream_t st, int L, int ss, int nblk, int spin, const double *part, const int *mtop,
                              const double2 *flm, const double *wl, int hstride, double *F);
hipError_t launch_fadj_scatter(hipStream_t st, int L, int ss, int hstride, double q, const double *F,
                               const double2 *hpole, const double2 *hpoleN, double *out);
hipError_t launch_mask_low(hipStream_t st, int an, int n, int nreg, int hstride, const double *cot, const double *csc,
                           const double *FA, const double *FB, double *HxA, double *HxB);
hipError_t launch_pole_from_F(hipStream_t st, int L, int hstride, int ring, const double *F, double2 *pole);
hipError_t set_kernel_lds_limits(size_t max_dyn);

}  // namespace s2mi
