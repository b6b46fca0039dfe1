/*
 * s2mi.h -- C ABI of the MI355X (gfx950) spin spherical-harmonic and Wigner
 * transform library.
 *
 * Method: Price & McEwen, "Differentiable and accelerated spherical harmonic
 * and Wigner transforms" (arXiv 2311.14670).  The O(L^3) stage -- Wigner-d
 * functions d^l_{m,n}(theta) generated on the fly by the descending-m
 * three-term recursion (Sec. 3.3, Eqs. 25-27) with running renormalisation
 * (Sec. 3.4) and contracted against coefficients (Eq. 33) or ring Fourier
 * modes (Eq. 30) -- runs in hand-written HIP kernels; the per-ring phi-DFT
 * (Eqs. 31-32) runs in the library's own FFT kernels.
 *
 * Conventions
 *   spin harmonics  sY_lm(theta,phi) = (-1)^s sqrt((2l+1)/4pi) e^{i m phi} d^l_{m,-s}(theta)
 *                   (Eqs. 9-10; Condon-Shortley phase, Eq. 1).
 *   bandlimit L     coefficients vanish for l >= L (Sec. 2.4).
 *   coefficients    complex128 (interleaved re, im), dense [l][m + L - 1],
 *                   l < L, |m| < L.  Entries with l < max(|m|, |spin|) are
 *                   ignored on input and written as 0 on output.
 *   MW map          complex128 [t][p], theta_t = (2t+1) pi/(2L-1), t < L
 *                   (t = L-1 is the south pole), phi_p = 2 pi p/(2L-1),
 *                   p < 2L-1 (Sec. 4.2, MW).
 *   HEALPix map     complex128 RING-ordered pixel vector of 12 nside^2
 *                   samples (Sec. 4.2, HEALPix; geometry of Gorski et al.
 *                   2005).  The forward transform is the quadrature of
 *                   Eq. 19 with q = 4 pi / Npix (approximate: no sampling
 *                   theorem).
 *   Wigner (SO(3))  coefficients [n + N - 1][l][m + L - 1] (zero for
 *                   l < max(|m|, |n|)); maps [k][t][p] with
 *                   gamma_k = 2 pi k/(2N-1), MW in (beta, alpha) (Sec. 4.5,
 *                   Eqs. 13-18).
 *   batch           the batch dimension is outermost and contiguous; every
 *                   transform takes 0 <= batch <= max_batch, and batch = 0
 *                   does nothing (no pointer is read or written).
 *
 * Memory and streams
 *   All data pointers passed to transforms are DEVICE pointers owned by the
 *   caller, 16-byte aligned.  Inputs are never modified.  The workspace is a
 *   caller-owned device buffer of at least s2_plan_info().workspace_bytes.
 *   Transforms are enqueued asynchronously on `hip_stream` (a hipStream_t, or
 *   NULL for the default stream) and never synchronise the host; outputs are
 *   undefined until the stream reaches the enqueued work, and undefined if the
 *   call returns an error.  A plan owns its device constants and is immutable
 *   after creation: one plan may be used concurrently on several streams
 *   provided each call has its own workspace.
 *
 * Errors
 *   Every function returns S2_OK (0) or a negative code.  Argument validation
 *   is synchronous, on the host, and happens before any device work is
 *   enqueued.  No C++ exception crosses this interface.  The message of the
 *   last error on the calling thread is available from
 *   s2_last_error_message().
 */
#ifndef S2MI_H
#define S2MI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define S2_OK               0
#define S2_ERR_INVALID_ARG (-1)   /* bad L/spin/N/nside/batch, null or misaligned pointer */
#define S2_ERR_UNSUPPORTED (-2)   /* valid request the library does not implement         */
#define S2_ERR_OOM         (-3)   /* device or host allocation failed                     */
#define S2_ERR_HIP         (-4)   /* HIP runtime or launch error (message kept)           */
#define S2_ERR_CHECK       (-5)   /* a debug check (environment S2MI_DEBUG_CHECKS=1) failed */

typedef struct s2_plan_s *s2_plan_t;

/* Sphere samplings (Sec. 2.5, 4.2).  Maps are complex128 (float64 for the
 * real-signal entry points), batch outermost:
 *   S2_MW       theta_t = (2t+1) pi/(2L-1), t < L (t = L-1: south pole),
 *               phi_p = 2 pi p/(2L-1): [L][2L-1]; exact transforms.
 *   S2_HEALPIX  RING-ordered pixel vector of 12 nside^2 samples (nside given);
 *               forward by the plain quadrature 4 pi/N_pix.
 *   S2_DH       Driscoll & Healy: theta_t = (2t+1) pi/(4L), t < 2L,
 *               phi_p = 2 pi p/(2L-1): [2L][2L-1]; exact transforms (DH weights).
 *   S2_GL       Gauss-Legendre: cos(theta_t) the roots of P_L, theta ascending,
 *               phi_p = 2 pi p/(2L-1): [L][2L-1]; exact transforms (GL weights).
 *   S2_MWSS     MW with symmetric sampling: theta_t = pi t/L, t = 0..L (both poles),
 *               phi_p = 2 pi p/(2L): [L+1][2L]; exact transforms.
 * SO(3) plans (N > 1) need S2_MW; nside is ignored except for S2_HEALPIX. */
typedef enum { S2_MW = 0, S2_HEALPIX = 1, S2_DH = 2, S2_GL = 3, S2_MWSS = 4 } s2_sampling_t;

/* Arithmetic of the l/theta contraction.  The Wigner-d recursion, its
 * renormalisation, the quadrature weights and the phi-DFT are FP64 in every
 * mode; inputs and outputs are always complex128.
 *   S2_FP64                 fused FP64 sweeps, one map at a time.
 *   S2_CONTRACT_FP32        all maps of a call together: per order m the
 *                           contraction is a matrix product on the matrix
 *                           cores with fp32 operands and fp32 accumulation.
 *   S2_CONTRACT_SPLIT_BF16  as above with x = hi + lo (hi = bf16(x),
 *                           lo = bf16(x - hi)) and three products
 *                           hi*hi + hi*lo + lo*hi, fp32 accumulation.
 * The reduced-precision modes trade accuracy (relative errors of order 1e-6
 * and 1e-5) for throughput on large batches. */
typedef enum { S2_FP64 = 0, S2_CONTRACT_FP32 = 1, S2_CONTRACT_SPLIT_BF16 = 2 } s2_precision_t;

typedef struct {
    int L, spin, N, nside, sampling, precision, max_batch;
    int nrings;                 /* isolatitude rings of the sphere sampling          */
    long long nsamples;         /* complex samples per map (SO(3): per gamma slice)  */
    long long ncoeffs;          /* L * (2L-1) per (map, n-slice): dense layout size  */
    size_t workspace_bytes;     /* device workspace one call needs at max_batch      */
    size_t plan_device_bytes;   /* device memory held by the plan                    */
    int swept_rings;            /* rings the inverse sweep's lanes run: nrings without
                                   the poles, or (spin 0, N/S-symmetric samplings,
                                   when that still fills the device; environment
                                   S2MI_RING_PAIRING=0/1 forces off/on) the northern
                                   half, mirror rings following from
                                   d^l_{m,0}(pi - theta) = (-1)^{l+m} d^l_{m,0}(theta) */
    int order_tiles;            /* FP64 sweeps: order ranges run as separate slices of
                                   the grid (1: none), each starting from the Wigner
                                   recursion's state stored at plan creation; chosen
                                   when the sweeps' grids would leave the device
                                   under-filled (environment S2MI_ORDER_TILES=k
                                   forces k, at most 8)                            */
} s2_plan_info_t;

/*
 * Create a plan.  Paper: Sec. 4 (the separable transform of Eqs. 30-33 on an
 * isolatitude sampling) with the Wigner recursion of Sec. 3.
 *   L          bandlimit, 2 <= L <= 4096 (l < L).
 *   spin       |spin| < L (S2 transforms).  Ignored (must be 0) when N > 1.
 *   N          azimuthal band of SO(3) transforms, 1 <= N <= L and N <= 8
 *              (S2_ERR_UNSUPPORTED above); N = 1 for sphere-only plans.  An
 *              SO(3) plan (N > 1) serves so3_*; a plan with N == 1 serves s2_*
 *              (and so3_* with N = 1).
 *   sampling   any s2_sampling_t (HEALPix: nside >= 1; L <= 3*nside+1 is not
 *              enforced, the caller picks L, typically 2*nside).  SO(3) plans
 *              require S2_MW.
 *   max_batch  largest batch any call will pass (sizes the workspace), >= 1.
 *   prec       contraction arithmetic (see s2_precision_t).
 *   hip_stream stream on which the plan's constants are uploaded and its set-up
 *              kernels run (tables of start values, order-tile states, FFT
 *              filters).  The call waits for that stream before it returns (its
 *              host staging buffers are freed then, and a failed set-up kernel is
 *              reported by this call), so the plan is ready on return, on any
 *              stream; work already queued on hip_stream is waited for too.
 * Ownership: *out receives a plan owned by the caller, freed by
 * s2_plan_destroy.  On error *out is set to NULL.
 * Debug check (environment S2MI_DEBUG_CHECKS=1): the plan also evaluates
 * sum_{|m| <= l} (d^l_{m,n}(theta))^2, which is 1 since d^l(theta) is orthogonal,
 * on up to 8 sampled rings for every degree and every pair of runs n, -n, with the
 * start values, tables and stable-direction continuation the transforms use, and
 * fails with S2_ERR_CHECK where |sum - 1| exceeds S2MI_DEBUG_CHECKS_TOL (default
 * 1e-10).
 */
int s2_plan_create(s2_plan_t *out, int L, int spin, int N, s2_sampling_t sampling,
                   int nside, int max_batch, s2_precision_t prec, void *hip_stream);

/* Free a plan and its device memory (synchronises the device first).  NULL is a no-op. */
int s2_plan_destroy(s2_plan_t plan);

/* Sizes of a plan (host only, no device work). */
int s2_plan_info(s2_plan_t plan, s2_plan_info_t *info);

/*
 * Inverse spin SHT (Eq. 4; separable form Eqs. 32-33):
 *   f(theta_t, phi_p) = sum_m e^{i m phi_p} sum_l (-1)^s sqrt((2l+1)/4pi) flm[l][m] d^l_{m,-s}(theta_t)
 *   flm  [batch][L][2L-1] complex128 (device, read)
 *   f    [batch][nsamples] complex128 (device, written)
 */
int s2_inverse(s2_plan_t plan, const void *flm, void *f, int batch, void *workspace,
               void *hip_stream);

/*
 * s2_inverse without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same operation, layouts and results as s2_inverse
 * (the same kernels run; outputs are bitwise equal); the workspace is a fixed
 * device array of S2_NOALLOC_SCRATCH_BYTES inside the library, one per GPU the
 * library runs on, held from its first use on that GPU until the process ends.
 * The call allocates nothing (no hipMalloc / hipFree, no events: stage timing is
 * not recorded) and looks the array's device address up once per device.
 *   flm [batch][L][2L-1] complex128 (device, read), f [batch][nsamples]
 *   complex128 (device, written), 0 <= batch <= max_batch.
 * Plans: FP64 sphere plans (N = 1) whose inverse needs at most
 * S2_NOALLOC_SCRATCH_BYTES of workspace (its records and partial sums: MW
 * L <= 512 at any spin, DH and HEALPix L <= 384); larger plans return
 * S2_ERR_INVALID_ARG with the size they need in the message, matrix-core plans
 * S2_ERR_UNSUPPORTED, SO(3) plans S2_ERR_INVALID_ARG.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different host threads without ordering)
 * race and give undefined results.  Calls ordered on one stream are safe.
 * Nothing in the array needs to start at zero: each call writes every word it
 * later reads.
 */
#define S2_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int s2_inverse_noalloc(s2_plan_t plan, const void *flm, void *f, int batch, void *hip_stream);

/*
 * Forward spin SHT (Eq. 5 discretised as Eqs. 30-31).
 *   MW: exact for band-limited signals (sampling theorem, Sec. 4.2): the ring
 *       DFT extended to the theta-torus and integrated against sin(theta) on
 *       [0, pi].  HEALPix: quadrature of Eq. 19 with q = 4 pi / Npix.
 *   f    [batch][nsamples] complex128 (device, read)
 *   flm  [batch][L][2L-1] complex128 (device, written; zero outside l >= max(|m|,|s|))
 */
int s2_forward(s2_plan_t plan, const void *f, void *flm, int batch, void *workspace,
               void *hip_stream);

/*
 * Real signals (spin-0 plans of any sampling, FP64).  A real map's
 * coefficients obey flm[l][-m] = (-1)^m conj(flm[l][m]) (Sec. 2.1), so the
 * Wigner-d sweeps carry only the orders m >= 0 (half the contraction work) and
 * two rings of equal length share one complex phi-DFT (half the DFT work; the
 * MW / MWSS theta filter runs on one side only).
 *
 * s2_inverse_real: f = Re(inverse SHT of the Hermitian completion of the
 * orders m >= 0 of flm); the orders m < 0 of flm are not read.
 *   flm [batch][L][2L-1] complex128 (device, read), f [batch][nsamples] double
 *   (device, written; the sampling's map layout).
 * s2_forward_real: the forward SHT of a real map, orders m < 0 written by the
 * symmetry above.
 *   f [batch][nsamples] double (device, read), flm [batch][L][2L-1]
 *   complex128 (device, written).
 * Map pointers need 16-byte alignment of the first map only.  Spin != 0 or
 * matrix-core plans: S2_ERR_UNSUPPORTED; SO(3) plans: S2_ERR_INVALID_ARG.
 */
int s2_inverse_real(s2_plan_t plan, const void *flm, void *f, int batch, void *workspace,
                    void *hip_stream);
int s2_forward_real(s2_plan_t plan, const void *f, void *flm, int batch, void *workspace,
                    void *hip_stream);

/*
 * Gradients of the real-signal transforms (Sec. 5, in the convention PyTorch
 * uses for complex inputs: d/dRe + i d/dIm of a real loss).
 * s2_inverse_real_adjoint: for a real map cotangent g, with A the complex
 *   inverse SHT, g_flm = 2 (A^H g) at m > 0, Re (A^H g) at m = 0 and 0 at
 *   m < 0 (orders m > 0 enter the real map twice, order 0 through its real
 *   part, orders m < 0 not at all).
 *   g [batch][nsamples] double (device, read), g_flm [batch][L][2L-1]
 *   complex128 (device, written).
 * s2_forward_real_adjoint: g = Re(F^H g_flm) with F the forward SHT, computed
 *   as F^H of the Hermitian part of g_flm through the real-signal path.
 *   g_flm [batch][L][2L-1] complex128 (device, read), g [batch][nsamples]
 *   double (device, written).
 * Plans and errors as for s2_inverse_real.
 */
int s2_inverse_real_adjoint(s2_plan_t plan, const void *g, void *g_flm, int batch, void *workspace,
                            void *hip_stream);
int s2_forward_real_adjoint(s2_plan_t plan, const void *g_flm, void *g, int batch, void *workspace,
                            void *hip_stream);

/*
 * Hermitian adjoint of the inverse SHT (the VJP of Eqs. 56-58 in the
 * conjugate convention PyTorch uses for complex gradients):
 *   g_flm[l][m] = sum_{t,p} g(theta_t, phi_p) conj(sY_lm(theta_t, phi_p))
 * i.e. an unnormalised forward phi-DFT followed by a forward-type d-stage
 * sweep over the sampling's own rings, with d recomputed on the fly.
 *   g      [batch][nsamples] complex128 (device, read)
 *   g_flm  [batch][L][2L-1] complex128 (device, written)
 */
int s2_inverse_adjoint(s2_plan_t plan, const void *g, void *g_flm, int batch, void *workspace,
                       void *hip_stream);

/*
 * Hermitian adjoint of the forward spin SHT (for gradients through s2_forward;
 * the conjugate convention PyTorch uses for complex tensors):
 *   g = F^H g_flm, with <F f, g_flm> = <f, g> for every map f.
 *   MW: the inverse-type d-stage sweep with the SHT weights (Eqs. 30, 33),
 *       the MW theta filter (which is Hermitian) and the adjoint phi-DFT
 *       (Eq. 31) times 2 pi/(2L-1); the south pole follows Eq. 29.
 *   HEALPix: (4 pi / Npix) times the inverse SHT (the forward is the
 *       quadrature of Eq. 19).
 *   DH, GL: the inverse SHT with the forward's weights, then each ring
 *       scaled by its quadrature weight.
 *   MWSS: as MW with both poles, phi weight 2 pi/(2L), and the adjoint of
 *       its theta filter (dropping the Nyquist frequency makes that filter
 *       non-Hermitian: the adjoint removes the Nyquist component after the
 *       sin(theta) weighting instead of before it).
 *   g_flm  [batch][L][2L-1] complex128 (device, read)
 *   g      [batch][nsamples] complex128 (device, written)
 * FP64 plans only (S2_ERR_UNSUPPORTED otherwise).
 */
int s2_forward_adjoint(s2_plan_t plan, const void *g_flm, void *g, int batch, void *workspace,
                       void *hip_stream);

/*
 * Inverse Wigner transform (Eq. 13 with Eq. 10):
 *   f(alpha_p, beta_t, gamma_k) = sum_n e^{i n gamma_k} sum_m e^{i m alpha_p}
 *                                 sum_l (2l+1)/(8 pi^2) flmn[n][l][m] d^l_{mn}(beta_t)
 *   flmn [batch][2N-1][L][2L-1], f [batch][2N-1][L][2L-1] (MW only).
 */
int so3_inverse(s2_plan_t plan, const void *flmn, void *f, int batch, void *workspace,
                void *hip_stream);

/*
 * Forward Wigner transform (Eq. 14), exact for MW sampling: gamma and alpha
 * DFTs with weights 2pi/(2N-1), 2pi/(2L-1), then per n the exact MW theta
 * integral (spin -n torus extension, Eqs. 15-16) with weight 1.
 */
int so3_forward(s2_plan_t plan, const void *f, void *flmn, int batch, void *workspace,
                void *hip_stream);

/*
 * Hermitian adjoint of the inverse Wigner transform (gradients through
 * so3_inverse, Sec. 5, in the conjugate convention PyTorch uses for complex
 * tensors):
 *   g_flmn[n][l][m] = sum_{t,p,k} g(alpha_p, beta_t, gamma_k) conj(D^l_{mn})
 *                     times (2l+1)/(8 pi^2),
 * computed as the unweighted gamma analysis sum_k g(gamma_k) e^{-i n gamma_k}
 * followed, per n, by the adjoint of the spin -n inverse SHT.
 *   g       [batch][2N-1][L][2L-1] complex128 (device, read)
 *   g_flmn  [batch][2N-1][L][2L-1] complex128 (device, written)
 * MW spin-0 plans, FP64 or matrix-core.
 */
int so3_inverse_adjoint(s2_plan_t plan, const void *g, void *g_flmn, int batch, void *workspace,
                        void *hip_stream);

/*
 * Hermitian adjoint of the forward Wigner transform (gradients through
 * so3_forward): per n the adjoint of the MW forward (inverse-type sweep with
 * the forward's weights, the Hermitian MW theta filter, adjoint phi-DFT times
 * 2 pi/(2L-1)), then the gamma synthesis times 2 pi/(2N-1).
 *   g_flmn  [batch][2N-1][L][2L-1] complex128 (device, read)
 *   g       [batch][2N-1][L][2L-1] complex128 (device, written)
 * MW spin-0 FP64 plans only (S2_ERR_UNSUPPORTED for matrix-core plans).
 */
int so3_forward_adjoint(s2_plan_t plan, const void *g_flmn, void *g, int batch, void *workspace,
                        void *hip_stream);

/*
 * Debug/validation: export the GPU recursion's d^l_{m,n}(theta_r) for one
 * run n (n = -spin or +spin) at rings r = 0 .. nrings-1 (sampling order),
 * for all l < L and 0 <= m <= l, into out[r][m][l] (double, device,
 * written; entries with l < max(m, |n|) are 0).  Used to check the
 * recursion against closed forms and the addition theorem.
 */
int s2_debug_wigner_d(s2_plan_t plan, int n, void *out, void *hip_stream);

/*
 * Stage timing (profiling aid).  When enabled, every kernel launch of the
 * plan's transforms is bracketed by HIP events recorded on the launch stream;
 * s2_plan_read_timing() waits for those events, accumulates the elapsed time
 * and launch count per stage into `out`, and clears the record.  Stages:
 */
#define S2_STAGE_PACK        0   /* inverse coefficient pack            */
#define S2_STAGE_DSTAGE_INV  1   /* inverse Wigner-d sweep (Eq. 33)     */
#define S2_STAGE_PHI_INV     2   /* inverse phi-DFT (Eq. 32)            */
#define S2_STAGE_PHI_FWD     3   /* forward phi-DFT (Eq. 31)            */
#define S2_STAGE_MW_THETA    4   /* MW theta filter (exact quadrature)  */
#define S2_STAGE_DSTAGE_FWD  5   /* forward Wigner-d sweep (Eq. 30)     */
#define S2_STAGE_FINISH      6   /* forward weights and layout          */
#define S2_STAGE_GAMMA       7   /* SO(3) gamma DFT                     */
#define S2_STAGE_DGEN        8   /* d-tile generation (matrix-core path) */
#define S2_STAGE_MFMA        9   /* batched MFMA contraction            */
#define S2_NSTAGES          10
typedef struct { double ms[S2_NSTAGES]; long long launches[S2_NSTAGES]; } s2_timing_t;
int s2_plan_set_timing(s2_plan_t plan, int enable);
int s2_plan_read_timing(s2_plan_t plan, s2_timing_t *out);

/* Human-readable name of an error code (static string). */
const char *s2_error_string(int code);

/* Message of the last error reported on the calling thread ("" if none). */
const char *s2_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* S2MI_H */
