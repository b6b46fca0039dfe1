// s2mi_fft.h -- device DFT engine: one workgroup transforms one sequence held
// in LDS.  Used for the per-ring phi-DFTs (Eqs. 31-32) and the MW theta
// half-sample shifts.
//
// Engine: self-sorting (Stockham) mixed-radix FFT over radices
// {2,3,4,5,7,8,9,11,13}, in place in LDS: every stage reads all its butterfly
// inputs into registers, synchronises, then writes.  Lengths with a larger
// prime factor go through Bluestein's chirp-z identity
//   X_k = conj(c_k) sum_j (x_j conj(c_j)) c_{k-j},  c_j = e^{i pi j^2 / n},
// evaluated as a power-of-two circular convolution.
#pragma once

#include <hip/hip_runtime.h>

#include "s2mi_internal.h"

namespace s2mi {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 cmulc(double2 a, double2 b)   // a * conj(b)
{
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// multiply by sign * i  (sign = -1: -i, +1: +i)
__device__ __forceinline__ double2 cmuli(double2 a, int sign)
{
    return sign < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

__device__ __forceinline__ double2 ldroot(const double *tw, int idx, int sign)
{
    const double2 t = reinterpret_cast<const double2 *>(tw)[idx];
    return sign < 0 ? t : make_double2(t.x, -t.y);
}

// cos(2 pi k / R), sin(2 pi k / R) for the odd radices, k = 0 .. R-1.
template <int R> struct OddRoots;
template <> struct OddRoots<3> {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
};
template <> struct OddRoots<5> {
    static constexpr double c[5] = {1.0, 0.3090169943749474241, -0.8090169943749474241, -0.8090169943749474241,
                                    0.3090169943749474241};
    static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                                    -0.95105651629515357212};
};
template <> struct OddRoots<7> {
    static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624,
                                    -0.90096886790241912624, -0.22252093395631440429, 0.62348980185873353053};
    static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048,
                                    -0.43388373911755812048, -0.97492791218182360702, -0.78183148246802980871};
};
template <> struct OddRoots<11> {
    static constexpr double c[11] = {1.0, 0.84125353283118116886, 0.41541501300188642553, -0.14231483827328514044,
                                     -0.65486073394528506406, -0.95949297361449738989, -0.95949297361449738989,
                                     -0.65486073394528506406, -0.14231483827328514044, 0.41541501300188642553,
                                     0.84125353283118116886};
    static constexpr double s[11] = {0.0, 0.54064081745559758211, 0.90963199535451837141, 0.98982144188093273238,
                                     0.75574957435425828377, 0.28173255684142969771, -0.28173255684142969771,
                                     -0.75574957435425828377, -0.98982144188093273238, -0.90963199535451837141,
                                     -0.54064081745559758211};
};
template <> struct OddRoots<13> {
    static constexpr double c[13] = {1.0, 0.8854560256532098959, 0.56806474673115580251, 0.12053668025532305335,
                                     -0.35460488704253562597, -0.74851074817110109863, -0.97094181742605202716,
                                     -0.97094181742605202716, -0.74851074817110109863, -0.35460488704253562597,
                                     0.12053668025532305335, 0.56806474673115580251, 0.8854560256532098959};
    static constexpr double s[13] = {0.0, 0.46472317204376854566, 0.82298386589365639458, 0.9927088740980539928,
                                     0.93501624268541482344, 0.66312265824079520238, 0.23931566428755776715,
                                     -0.23931566428755776715, -0.66312265824079520238, -0.93501624268541482344,
                                     -0.9927088740980539928, -0.82298386589365639458, -0.46472317204376854566};
};

// Small DFT y_q = sum_r v_r e^{sign 2 pi i r q / R}, stored to out[q * os].
// Odd R: with a_r = v_r + v_{R-r}, b_r = v_r - v_{R-r} (r <= (R-1)/2),
//   y_q, y_{R-q} = v_0 + sum_r a_r cos(2 pi rq/R) +- sign i sum_r b_r sin(2 pi rq/R).
template <int R>
__device__ __forceinline__ void dft_small_store(double2 (&v)[R], int sign, double2 *out, int os)
{
    if constexpr (R == 2) {
        out[0] = cadd(v[0], v[1]);
        out[os] = csub(v[0], v[1]);
    } else if constexpr (R == 4) {
        const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const double2 b0 = cadd(v[1], v[3]), b1 = cmuli(csub(v[1], v[3]), sign);
        out[0] = cadd(a0, b0);
        out[2 * os] = csub(a0, b0);
        out[os] = cadd(a1, b1);
        out[3 * os] = csub(a1, b1);
    } else if constexpr (R == 8) {
        // two radix-4 on even/odd, then combine with e^{sign 2 pi i k/8}
        const double2 e0 = cadd(v[0], v[4]), e1 = csub(v[0], v[4]);
        const double2 e2 = cadd(v[2], v[6]), e3 = cmuli(csub(v[2], v[6]), sign);
        const double2 E0 = cadd(e0, e2), E2 = csub(e0, e2), E1 = cadd(e1, e3), E3 = csub(e1, e3);
        const double2 o0 = cadd(v[1], v[5]), o1 = csub(v[1], v[5]);
        const double2 o2 = cadd(v[3], v[7]), o3 = cmuli(csub(v[3], v[7]), sign);
        const double2 O0 = cadd(o0, o2), O2 = csub(o0, o2), O1 = cadd(o1, o3), O3 = csub(o1, o3);
        const double h = 0.70710678118654752440;
        const double2 t1 = make_double2(h * (O1.x - sign * O1.y), h * (O1.y + sign * O1.x));
        const double2 t2 = cmuli(O2, sign);
        const double2 t3 = make_double2(h * (-O3.x - sign * O3.y), h * (-O3.y + sign * O3.x));
        out[0] = cadd(E0, O0);
        out[4 * os] = csub(E0, O0);
        out[os] = cadd(E1, t1);
        out[5 * os] = csub(E1, t1);
        out[2 * os] = cadd(E2, t2);
        out[6 * os] = csub(E2, t2);
        out[3 * os] = cadd(E3, t3);
        out[7 * os] = csub(E3, t3);
    } else if constexpr (R == 9) {
        // 9 = 3 x 3: with r = 3j + k and q = p + 3s, y_q = sum_k w9^{kp} w3^{ks}
        // (sum_j v_{3j+k} w3^{jp}): three radix-3 DFTs, twiddles, three more
        constexpr double c3 = -0.5, s3 = 0.86602540378443864676;   // cos, sin of 2 pi / 3
        auto dft3 = [sign](double2 a, double2 b, double2 c, double2 &y0, double2 &y1, double2 &y2) {
            const double2 t = cadd(b, c), d = csub(b, c);
            y0 = cadd(a, t);
            const double2 mid = make_double2(fma(c3, t.x, a.x), fma(c3, t.y, a.y));
            const double2 rot = cmuli(make_double2(s3 * d.x, s3 * d.y), sign);   // sign i s3 (b - c)
            y1 = cadd(mid, rot);
            y2 = csub(mid, rot);
        };
        double2 t[3][3];                                  // t[k][p]
#pragma unroll
        for (int k = 0; k < 3; ++k) dft3(v[k], v[3 + k], v[6 + k], t[k][0], t[k][1], t[k][2]);
        const double sg = sign < 0 ? -1.0 : 1.0;          // w9^e = cos(2 pi e / 9) + sign i sin(2 pi e / 9)
        const double2 w1 = make_double2(0.76604444311897803520, sg * 0.64278760968653932632);
        const double2 w2 = make_double2(0.17364817766693034885, sg * 0.98480775301220805937);
        const double2 w4 = make_double2(-0.93969262078590838405, sg * 0.34202014332566873304);
        t[1][1] = cmul(t[1][1], w1);
        t[1][2] = cmul(t[1][2], w2);
        t[2][1] = cmul(t[2][1], w2);
        t[2][2] = cmul(t[2][2], w4);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            double2 y0, y1, y2;
            dft3(t[0][p], t[1][p], t[2][p], y0, y1, y2);
            out[p * os] = y0;
            out[(p + 3) * os] = y1;
            out[(p + 6) * os] = y2;
        }
    } else {
        constexpr int H = (R - 1) / 2;
        double2 y0 = v[0];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            const double2 a = cadd(v[r], v[R - r]), b = csub(v[r], v[R - r]);
            v[r] = a;
            v[R - r] = b;
            y0 = cadd(y0, a);
        }
        out[0] = y0;
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            double2 A = v[0], B = make_double2(0.0, 0.0);
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const double c = OddRoots<R>::c[(r * q) % R], s = OddRoots<R>::s[(r * q) % R];
                A.x = fma(v[r].x, c, A.x);
                A.y = fma(v[r].y, c, A.y);
                B.x = fma(v[R - r].x, s, B.x);
                B.y = fma(v[R - r].y, s, B.y);
            }
            const double2 iB = cmuli(B, sign);
            out[q * os] = cadd(A, iB);
            out[(R - q) * os] = csub(A, iB);
        }
    }
}

// One Stockham stage of radix R; NB butterflies per thread at most.
template <int R, int NB>
__device__ __forceinline__ void fft_stage(double2 *buf, int len, int Ns, const double *tw, int sign)
{
    const int T = blockDim.x, tid = threadIdx.x;
    const int nbf = len / R;
    double2 v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tid + b * T;
        if (j < nbf) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * nbf];
        }
    }
    __syncthreads();
    const int tstep = len / (Ns * R);
    // j / Ns by one high multiply with ceil(2^32 / Ns): exact for j < 2^16, Ns <= 2^13
    // (the error j (ceil(2^32/Ns) - 2^32/Ns) / 2^32 < 2^-19 stays below 1/Ns)
    const unsigned mag = Ns > 1 ? 0xffffffffu / (unsigned)Ns + 1u : 0u;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tid + b * T;
        if (j < nbf) {
            const int jq = Ns > 1 ? (int)__umulhi((unsigned)j, mag) : j;   // j / Ns
            const int k = j - jq * Ns;                                      // j % Ns
            if (Ns > 1) {
                // twiddles w^r, r < R, by repeated multiplication from one table read (the
                // R-1 reads at stride r lanes apart touched a line each; rounding grows
                // like r ulp, r <= 12)
                const double2 w1 = ldroot(tw, k * tstep, sign);
                double2 w = w1;
                v[b][1] = cmul(v[b][1], w);
#pragma unroll
                for (int r = 2; r < R; ++r) {
                    w = cmul(w, w1);
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            const int o = jq * Ns * R + k;
            dft_small_store<R>(v[b], sign, buf + o, Ns);
        }
    }
    __syncthreads();
}

// With blockDim.x >= len/8 (plan-time rule) a thread holds at most 8 values,
// i.e. NB <= ceil(8/R) butterflies; only those variants are instantiated.
template <int R>
__device__ __forceinline__ void fft_stage_nb(double2 *buf, int len, int Ns, const double *tw, int sign)
{
    constexpr int NBMAX = (8 + R - 1) / R;
    const int nb = (len / R + blockDim.x - 1) / blockDim.x;
    if (nb <= 1 || NBMAX == 1) fft_stage<R, 1>(buf, len, Ns, tw, sign);
    else if (nb == 2 || NBMAX == 2) fft_stage<R, (NBMAX >= 2 ? 2 : 1)>(buf, len, Ns, tw, sign);
    else if (nb == 3 || NBMAX == 3) fft_stage<R, (NBMAX >= 3 ? 3 : 1)>(buf, len, Ns, tw, sign);
    else fft_stage<R, (NBMAX >= 4 ? 4 : 1)>(buf, len, Ns, tw, sign);
}

// Unnormalised DFT of length f.len in LDS: X_k = sum_j x_j e^{sign 2 pi i jk/len}.
// Requires blockDim.x * 4 * radix >= len for every stage radix (enforced at plan time).
// f points at a FftArgs in device memory (uniform): its fields are read with
// scalar loads, never copied into a private array.
__device__ __forceinline__ void fft_engine(double2 *buf, const FftArgs *f, int sign)
{
    const int len = f->len, nst = f->nst;
    const double *tw = f->tw;
    int Ns = 1;
    for (int s = 0; s < nst; ++s) {
        const int R = f->rad[s];
        switch (R) {
        case 2: fft_stage_nb<2>(buf, len, Ns, tw, sign); break;
        case 3: fft_stage_nb<3>(buf, len, Ns, tw, sign); break;
        case 4: fft_stage_nb<4>(buf, len, Ns, tw, sign); break;
        case 5: fft_stage_nb<5>(buf, len, Ns, tw, sign); break;
        case 7: fft_stage_nb<7>(buf, len, Ns, tw, sign); break;
        case 8: fft_stage_nb<8>(buf, len, Ns, tw, sign); break;
        case 9: fft_stage_nb<9>(buf, len, Ns, tw, sign); break;
        case 11: fft_stage_nb<11>(buf, len, Ns, tw, sign); break;
        default: fft_stage_nb<13>(buf, len, Ns, tw, sign); break;
        }
        Ns *= R;
    }
}

// Unnormalised DFT of length f.n of buf[0..n) in LDS (buf must hold f.len
// entries).  sign = -1: forward, +1: inverse.  Leaves the result in buf[0..n).
//
// Bluestein (lengths with a prime factor above 13): the inverse is
// conj(DFT(conj(x))); the chirped input u_j = x_j conj(c_j) is convolved with
// the chirp by a forward FFT, a product with the filter spectrum and an inverse
// FFT, then de-chirped.  With f.conv set the chirp is 1 (no products) and the
// result is the cyclic convolution of x (zero past n) with the filter's kernel,
// at t < n.
//
// Split Bluestein (convolution length M = 2H, H = f.len the LDS engine length,
// n < H): u is zero past n < H, so the even spectrum samples U[2k] are
// DFT_H(u)[k] and the odd ones U[2k+1] are DFT_H(u w^j)[k], w = e^{-2 pi i/M}.
// The inverse transform of V = U b~ is needed only at t < n < H, where it is
// IDFT_H(V_even)[t] + conj(w)^t IDFT_H(V_odd)[t].  The halves run one after the
// other in the same LDS buffer; u and the even result wait in scr (2H entries
// of this workgroup's global scratch, each read back only by the thread that
// wrote it).
//
// All forms run as one loop over engine passes, so the engine is inlined once
// per call site.
__device__ __forceinline__ void dft_lds(double2 *buf, const FftArgs *f, int sign, double2 *scr = nullptr)
{
    const int T = blockDim.x, tid = threadIdx.x;
    const int n = f->n, len = f->len;
    const int blue = f->blue, split = blue && f->split;
    const int conv = f->conv;                                // unit chirp: a plain cyclic convolution
    const double2 *ch = reinterpret_cast<const double2 *>(f->chirp);
    const double2 *bf = reinterpret_cast<const double2 *>(f->bflt);
    const double2 *wm = reinterpret_cast<const double2 *>(f->twm);
    const int npass = !blue ? 1 : (split ? 4 : 2);
#pragma unroll 1
    for (int pass = 0; pass < npass; ++pass) {
        if (blue) {
            if (pass == 0) {                                 // chirp (zero-padded to len)
                for (int i = tid; i < len; i += T) {
                    double2 v = make_double2(0.0, 0.0);
                    if (i < n) {
                        double2 x = buf[i];
                        if (sign > 0) x.y = -x.y;
                        v = conv ? x : cmulc(x, ch[i]);
                    }
                    if (split) scr[i] = v;
                    buf[i] = v;
                }
            } else if (pass == 2) {                          // split: odd half input u w^j
                for (int i = tid; i < len; i += T) buf[i] = cmul(scr[i], wm[i]);
            } else {                                         // filter spectrum (split: even / odd samples)
                const int stp = split ? 2 : 1, off = pass == 3 ? 1 : 0;
                for (int i = tid; i < len; i += T) buf[i] = cmul(buf[i], bf[stp * i + off]);
            }
            __syncthreads();
        }
        fft_engine(buf, f, !blue ? sign : ((pass & 1) ? +1 : -1));
        if (split && pass == 1)                              // keep the even half's result
            for (int i = tid; i < len; i += T) scr[len + i] = buf[i];
    }
    if (blue) {                                              // (combine and) de-chirp
        for (int i = tid; i < n; i += T) {
            const double2 v = split ? cadd(scr[len + i], cmulc(buf[i], wm[i])) : buf[i];
            double2 y = conv ? v : cmulc(v, ch[i]);
            if (sign > 0) y.y = -y.y;
            buf[i] = y;
        }
        __syncthreads();
    }
}

}  // namespace s2mi
