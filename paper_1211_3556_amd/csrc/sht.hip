// Harmonic-space half of the split convolution (Sutter, Wandelt & Elsner 2012,
// Sec. 2, eq. 1): the truncated l-space kernel Khat_l, l <= lcut, applied to a
// HEALPix RING map by spherical-harmonic analysis with the pixel quadrature
// and synthesis,
//
//     a_lm = Omega sum_p x_p conj(Y_lm(p)),
//     y_p  = sum_{l <= lcut} Khat_l sum_m a_lm Y_lm(p),
//
// with Y_lm = lambda_lm(cos theta) e^{i m phi} and the orthonormal associated
// Legendre functions lambda_lm.  The paper runs this half on host cores with an
// SHT library while the GPU sums the real-space half; here both halves run on
// the GPU, in five stream-ordered kernels per map, all in FP64:
//
//  1. k_sht_dft_fwd   per ring: F_r(m) = sum_j x_j e^{-i m phi_j}, m <= lcut,
//                     by Goertzel's second-order recurrence (one FMA and one
//                     add per sample and frequency, no phase table); belt
//                     rings whose length is a power of two (and exceeds
//                     2 lcut) take k_sht_fft_fwd instead, a real FFT done as
//                     one LDS-resident complex FFT of half the length;
//  2. k_sht_leg_fwd   per (m, chunk of northern rings): lambda_lm by its
//                     recurrence in l, times the even / odd N-S combinations
//                     of F, reduced over the chunk's rings through LDS into
//                     per-chunk partial a_lm;
//  3. k_sht_mul       a_lm = Omega Khat_l sum over chunks (fixed order);
//  4. k_sht_leg_bwd   per (m, northern ring): G_r(m) = sum_l a_lm lambda_lm,
//                     split into even and odd parts for the ring and its
//                     mirror;
//  5. k_sht_dft_bwd   per ring: y_j = Re sum_m c_m G_r(m) e^{i m phi_j}
//                     (c_0 = 1, c_m = 2) by Clenshaw's recurrence, one pass
//                     for the pixel pair j, n - j; k_sht_fft_bwd is the
//                     inverse real FFT for the rings of k_sht_fft_fwd.
//
// lambda_mm underflows FP64 for large m near the poles, so the recurrence
// carries a power-of-two scale: a value is lam * 2^(512 sc) with sc <= 0, and
// terms are used only once sc reaches 0 (below that they are < 2^-330 times
// the ring's other terms).  Results are deterministic: no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "arkcos_internal.hpp"

namespace arkcos {

// One ring as the transform kernels see it (0-based).
struct ShtRing {
    double z;       // cos theta
    double s;       // sin theta
    double log2s;   // log2 sin theta
    int n;          // pixels
    int first;      // RING index of pixel 0
    int two_o;      // 1: pixel j at phi = (j + 1/2) 2 pi / n, 0: at j 2 pi / n
    int pad;
};
static_assert(sizeof(ShtRing) == 40, "ShtRing layout");

constexpr int kShtThreads = 256;
constexpr int kShtChunk = 4096;     // samples of a ring staged per pass (FP64)
constexpr int kShtMaxFreq = 8;      // frequencies per thread and pass in k_sht_dft_fwd
constexpr int kLegBlock = 8;        // degrees l per LDS reduction in k_sht_leg_fwd
constexpr int kLegCols = 2 * kLegBlock;            // re, im per degree
constexpr int kLegSegs = kShtThreads / kLegCols;   // row segments of a column
constexpr int kLegRings = 2;        // northern rings per lane in k_sht_leg_fwd
constexpr int kLegChunk = kLegRings * kShtThreads;  // rings per k_sht_leg_fwd workgroup
constexpr int kShtPairs = 2;        // pixel pairs per thread in k_sht_dft_bwd
constexpr int kShtFftMaxM = 8192;   // complex FFT length in LDS (128 KB of FP64 pairs)
constexpr double kScaleUp = 0x1p128;     // rescale threshold of a scaled value
constexpr double kScaleStep = 0x1p-512;  // one scale step

// First entry of order m in the (l, m) layout: for each m, l = m .. L.
__host__ __device__ inline long long alm_base(int m, int L)
{
    return (long long)m * (L + 1) - (long long)m * (m - 1) / 2;
}

// lambda_mm of a ring in scaled form: returns the mantissa and sets sc.
__device__ __forceinline__ double lambda_mm_scaled(double mnorm, int m, double log2s, int &sc)
{
    const double e = mnorm + (double)m * log2s;   // log2 |lambda_mm|
    if (e >= -384.0) {
        sc = 0;
        return exp2(e);
    }
    sc = (int)floor((e + 384.0) / 512.0);          // mantissa in [2^-384, 2^128)
    return exp2(e - 512.0 * sc);
}

// One step of the l recurrence, lambda_l = A z lambda_{l-1} - B lambda_{l-2},
// with a rescale while the value is scaled.  Returns the usable value (0 while
// scaled).
__device__ __forceinline__ double lambda_step(double A, double B, double z, double &l1, double &l2,
                                              int &sc)
{
    const double v = fma(A * z, l1, -B * l2);
    l2 = l1;
    l1 = v;
    if (sc < 0) {
        if (fabs(l1) > kScaleUp) {
            l1 *= kScaleStep;
            l2 *= kScaleStep;
            ++sc;
        }
        return sc == 0 ? l1 : 0.0;
    }
    return v;
}

// ------------------------------------------------------------ analysis --
// Goertzel: s_j = x_j + 2 cos(w) s_{j-1} - s_{j-2}; after n samples
// sum_j x_j e^{-i w j} = e^{i w} s_{n-1} - s_{n-2}.  Two samples per step
// update (s1, s2) in place: s2 <- c s1 + x_j - s2, s1 <- c s2 + x_{j+1} - s1.
// Ring lengths are multiples of 4, so every staged count is even.  One launch
// covers frequencies m = m0 + thread + k kShtThreads, k < K.
template <int K>
__global__ __launch_bounds__(kShtThreads) void k_sht_dft_fwd(const ShtRing *__restrict__ rings,
                                                             const int *__restrict__ ring_list,
                                                             const float *__restrict__ x,
                                                             double2 *__restrict__ F, int m0,
                                                             int L, int nrings)
{
    __shared__ double2 sx[kShtChunk / 2];
    const int r = ring_list[blockIdx.x];
    const ShtRing R = rings[r];
    const float *xr = x + R.first;
    double c[K], s1[K], s2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int m = m0 + threadIdx.x + k * kShtThreads;
        c[k] = 2.0 * cospi(2.0 * (double)(m % R.n) / (double)R.n);
        s1[k] = 0.0;
        s2[k] = 0.0;
    }
    for (int j0 = 0; j0 < R.n; j0 += kShtChunk) {
        const int half = min(kShtChunk, R.n - j0) / 2;
        __syncthreads();
        for (int j = threadIdx.x; j < half; j += kShtThreads) {
            const float2 v = *reinterpret_cast<const float2 *>(xr + j0 + 2 * j);
            sx[j] = make_double2((double)v.x, (double)v.y);
        }
        __syncthreads();
        for (int j = 0; j < half; ++j) {
            const double2 v = sx[j];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                s2[k] = fma(c[k], s1[k], v.x - s2[k]);
                s1[k] = fma(c[k], s2[k], v.y - s1[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int m = m0 + threadIdx.x + k * kShtThreads;
        if (m > L) continue;
        double sw, cw;
        sincospi(2.0 * (double)(m % R.n) / (double)R.n, &sw, &cw);
        const double xre = cw * s1[k] - s2[k];
        const double xim = sw * s1[k];
        // times e^{-i m phi_0}, phi_0 = two_o pi / n
        const long long q = ((long long)m * R.two_o) % (2LL * R.n);
        double sp, cp;
        sincospi((double)q / (double)R.n, &sp, &cp);
        F[(size_t)m * nrings + r] = make_double2(cp * xre + sp * xim, cp * xim - sp * xre);
    }
}

// Partial a_lm of one chunk of northern rings (the equator last): ring r and
// its mirror 4N-2-r (0-based) have lambda_lm(pi - theta) = (-1)^(l+m)
// lambda_lm(theta), so they enter through E = F_r + F_mirror (l + m even) and
// O = F_r - F_mirror (l + m odd); the equator enters once, through E.
__global__ __launch_bounds__(kShtThreads) void k_sht_leg_fwd(
    const ShtRing *__restrict__ rings, const double2 *__restrict__ F,
    const double2 *__restrict__ rec, const double *__restrict__ mnorm,
    const int *__restrict__ ring_lo, double *__restrict__ part, int L, int nrings, int nnorth,
    long long nalm)
{
    __shared__ double red[kLegCols][kShtThreads + 1];
    __shared__ double red2[kLegSegs][kLegCols];
    const int m = blockIdx.y;
    const int chunk = blockIdx.x;
    // chunks whose rings all lie below ring_lo[m] contribute nothing (and
    // k_sht_mul skips their partials)
    if ((chunk + 1) * kLegChunk <= ring_lo[m]) return;
    // kLegRings rings per lane: independent recurrences, summed in registers
    // before the block reduction
    double2 E[kLegRings], O[kLegRings];
    double z[kLegRings], l1[kLegRings], l2[kLegRings];
    int sc[kLegRings];
#pragma unroll
    for (int q = 0; q < kLegRings; ++q) {
        const int i = chunk * kLegChunk + q * kShtThreads + threadIdx.x;
        const bool act = i < nnorth;
        const int ii = act ? i : 0;
        const ShtRing R = rings[ii];
        const int mir = nrings - 1 - ii;
        E[q] = make_double2(0.0, 0.0);
        O[q] = E[q];
        if (act) {
            const double2 a = F[(size_t)m * nrings + ii];
            if (mir == ii) {
                E[q] = a;
            } else {
                const double2 b = F[(size_t)m * nrings + mir];
                E[q] = make_double2(a.x + b.x, a.y + b.y);
                O[q] = make_double2(a.x - b.x, a.y - b.y);
            }
        }
        l1[q] = lambda_mm_scaled(mnorm[m], m, R.log2s, sc[q]);
        l2[q] = 0.0;
        z[q] = R.z;
    }
    const long long base = alm_base(m, L);
    for (int l0 = m; l0 <= L; l0 += kLegBlock) {
        double pr[kLegBlock], pim[kLegBlock];
#pragma unroll
        for (int k = 0; k < kLegBlock; ++k) {
            pr[k] = 0.0;
            pim[k] = 0.0;
        }
        bool scaled = false;
#pragma unroll
        for (int q = 0; q < kLegRings; ++q) scaled |= sc[q] < 0;
        if (l0 > m && l0 + kLegBlock - 1 <= L && !__any(scaled)) {
            // a full block with every lane of the wave unscaled: plain steps,
            // the block's coefficients loaded together
            double2 ab[kLegBlock];
#pragma unroll
            for (int k = 0; k < kLegBlock; ++k) ab[k] = rec[base + (l0 + k - m)];
#pragma unroll
            for (int k = 0; k < kLegBlock; ++k) {
                const bool odd = ((l0 + k + m) & 1) != 0;
#pragma unroll
                for (int q = 0; q < kLegRings; ++q) {
                    const double v = fma(ab[k].x * z[q], l1[q], -ab[k].y * l2[q]);
                    l2[q] = l1[q];
                    l1[q] = v;
                    const double2 src = odd ? O[q] : E[q];
                    pr[k] = fma(v, src.x, pr[k]);
                    pim[k] = fma(v, src.y, pim[k]);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kLegBlock; ++k) {
                const int l = l0 + k;
                if (l > L) continue;
                const bool odd = ((l + m) & 1) != 0;
#pragma unroll
                for (int q = 0; q < kLegRings; ++q) {
                    double v;
                    if (l == m) {
                        v = sc[q] == 0 ? l1[q] : 0.0;
                    } else {
                        const double2 ab = rec[base + (l - m)];
                        v = lambda_step(ab.x, ab.y, z[q], l1[q], l2[q], sc[q]);
                    }
                    const double2 src = odd ? O[q] : E[q];
                    pr[k] = fma(v, src.x, pr[k]);
                    pim[k] = fma(v, src.y, pim[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kLegBlock; ++k) {
            red[2 * k][threadIdx.x] = pr[k];
            red[2 * k + 1][threadIdx.x] = pim[k];
        }
        __syncthreads();
        {
            // column col (degree l0 + col/2, re or im) summed over one segment
            // of kShtThreads / kLegSegs lanes
            constexpr int rows = kShtThreads / kLegSegs;
            const int col = threadIdx.x % kLegCols;
            const int seg = threadIdx.x / kLegCols;
            double t = 0.0;
            for (int q = 0; q < rows; ++q) t += red[col][seg * rows + q];
            red2[seg][col] = t;
        }
        __syncthreads();
        if (threadIdx.x < kLegCols) {
            double t = 0.0;
            for (int sgm = 0; sgm < kLegSegs; ++sgm) t += red2[sgm][threadIdx.x];
            const int l = l0 + (threadIdx.x >> 1);
            if (l <= L)
                part[2 * ((size_t)chunk * nalm + base + (l - m)) + (threadIdx.x & 1)] = t;
        }
    }
}

// a_lm = Omega Khat_l sum over the ring chunks, in chunk order.
__global__ __launch_bounds__(kShtThreads) void k_sht_mul(const double2 *__restrict__ part,
                                                         const double *__restrict__ kscale,
                                                         const int *__restrict__ ring_lo,
                                                         double2 *__restrict__ alm, int L,
                                                         int nchunk, long long nalm)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * kShtThreads + threadIdx.x;
    if (l > L) return;
    const long long idx = alm_base(m, L) + (l - m);
    double2 s = make_double2(0.0, 0.0);
    for (int c = ring_lo[m] / kLegChunk; c < nchunk; ++c) {
        const double2 p = part[(size_t)c * nalm + idx];
        s.x += p.x;
        s.y += p.y;
    }
    alm[idx] = make_double2(kscale[l] * s.x, kscale[l] * s.y);
}

// ----------------------------------------------------------- synthesis --
// G_r(m) = sum_l a_lm lambda_lm(theta_r) for northern rings and their mirrors,
// kLegRings rings per lane (independent recurrences sharing the loads of the
// coefficients), in blocks of kLegBlock degrees: plain steps once every lane
// of the wave is unscaled, steps with the rescale check before that.
__global__ __launch_bounds__(kShtThreads) void k_sht_leg_bwd(
    const ShtRing *__restrict__ rings, const double2 *__restrict__ alm,
    const double2 *__restrict__ rec, const double *__restrict__ mnorm,
    const int *__restrict__ ring_lo, double2 *__restrict__ G, int L, int nrings, int nnorth)
{
    const int m = blockIdx.y;
    const int i0 = blockIdx.x * kLegChunk + threadIdx.x;
    if ((blockIdx.x + 1) * kLegChunk <= ring_lo[m]) {   // every term negligible
#pragma unroll
        for (int q = 0; q < kLegRings; ++q) {
            const int i = i0 + q * kShtThreads;
            if (i < nnorth) {
                G[(size_t)m * nrings + i] = make_double2(0.0, 0.0);
                G[(size_t)m * nrings + (nrings - 1 - i)] = make_double2(0.0, 0.0);
            }
        }
        return;
    }
    double z[kLegRings], l1[kLegRings], l2[kLegRings];
    int sc[kLegRings];
    double2 ae[kLegRings], ao[kLegRings];   // l + m even, odd
    const long long base = alm_base(m, L);
    const double2 a_m = alm[base];
#pragma unroll
    for (int q = 0; q < kLegRings; ++q) {
        const int i = min(i0 + q * kShtThreads, nnorth - 1);
        const ShtRing R = rings[i];
        l1[q] = lambda_mm_scaled(mnorm[m], m, R.log2s, sc[q]);
        l2[q] = 0.0;
        z[q] = R.z;
        const double v = sc[q] == 0 ? l1[q] : 0.0;
        ae[q] = make_double2(v * a_m.x, v * a_m.y);
        ao[q] = make_double2(0.0, 0.0);
    }
    // degrees m+1 .. L in blocks of kLegBlock: plain steps when every lane of
    // the wave is unscaled, steps with the rescale check otherwise
    for (int l0 = m + 1; l0 <= L; l0 += kLegBlock) {
        bool scaled = false;
#pragma unroll
        for (int q = 0; q < kLegRings; ++q) scaled |= sc[q] < 0;
        if (l0 + kLegBlock - 1 <= L && !__any(scaled)) {
            double2 rb[kLegBlock], ab[kLegBlock];
#pragma unroll
            for (int k = 0; k < kLegBlock; ++k) {
                rb[k] = rec[base + (l0 + k - m)];
                ab[k] = alm[base + (l0 + k - m)];
            }
#pragma unroll
            for (int k = 0; k < kLegBlock; ++k) {
                const bool odd = ((l0 + k - m) & 1) != 0;
#pragma unroll
                for (int q = 0; q < kLegRings; ++q) {
                    const double v = fma(rb[k].x * z[q], l1[q], -rb[k].y * l2[q]);
                    l2[q] = l1[q];
                    l1[q] = v;
                    double2 &t = odd ? ao[q] : ae[q];
                    t.x = fma(v, ab[k].x, t.x);
                    t.y = fma(v, ab[k].y, t.y);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kLegBlock; ++k) {
                const int l = l0 + k;
                if (l > L) continue;
                const double2 r1 = rec[base + (l - m)];
                const double2 a = alm[base + (l - m)];
                const bool odd = ((l - m) & 1) != 0;
#pragma unroll
                for (int q = 0; q < kLegRings; ++q) {
                    const double v = lambda_step(r1.x, r1.y, z[q], l1[q], l2[q], sc[q]);
                    double2 &t = odd ? ao[q] : ae[q];
                    t.x = fma(v, a.x, t.x);
                    t.y = fma(v, a.y, t.y);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kLegRings; ++q) {
        const int i = i0 + q * kShtThreads;
        if (i >= nnorth) continue;
        const int mir = nrings - 1 - i;
        G[(size_t)m * nrings + i] = make_double2(ae[q].x + ao[q].x, ae[q].y + ao[q].y);
        if (mir != i)
            G[(size_t)m * nrings + mir] = make_double2(ae[q].x - ao[q].x, ae[q].y - ao[q].y);
    }
}

// y_j = Re sum_m H_m e^{i m a_j}, a_j = 2 pi j / n, H_m = c_m G_r(m) e^{i m phi_0}:
// with C = sum Re H_m cos(m a) and S = sum Im H_m sin(m a) (Clenshaw, shared
// coefficient 2 cos a), y_j = C - S and y_{n-j} = C + S.
__global__ __launch_bounds__(kShtThreads) void k_sht_dft_bwd(const ShtRing *__restrict__ rings,
                                                             const int *__restrict__ ring_list,
                                                             const double2 *__restrict__ G,
                                                             float *__restrict__ out, int L,
                                                             int nrings, int accumulate)
{
    extern __shared__ double2 H[];
    const int r = ring_list[blockIdx.x];
    const ShtRing R = rings[r];
    for (int m = threadIdx.x; m <= L; m += kShtThreads) {
        const double2 g = G[(size_t)m * nrings + r];
        const long long q = ((long long)m * R.two_o) % (2LL * R.n);
        double sp, cp;
        sincospi((double)q / (double)R.n, &sp, &cp);
        const double c = m == 0 ? 1.0 : 2.0;
        H[m] = make_double2(c * (g.x * cp - g.y * sp), c * (g.x * sp + g.y * cp));
    }
    __syncthreads();
    float *o = out + R.first;
    const int npairs = R.n / 2 + 1;     // j = 0 .. n/2
    for (int j0 = threadIdx.x * kShtPairs; j0 < npairs; j0 += kShtThreads * kShtPairs) {
        double cc[kShtPairs], b1[kShtPairs], b2[kShtPairs], d1[kShtPairs], d2[kShtPairs];
#pragma unroll
        for (int k = 0; k < kShtPairs; ++k) {
            cc[k] = 2.0 * cospi(2.0 * (double)(j0 + k) / (double)R.n);
            b1[k] = b2[k] = d1[k] = d2[k] = 0.0;
        }
        // b_m = h_m + 2 cos(a) b_{m+1} - b_{m+2} from m = L down, two steps
        // at a time in place (b1 holds the newest term); an odd count starts
        // from b_L = h_L
        int m = L;
        if (((L + 1) & 1) != 0) {
            const double2 h = H[L];
#pragma unroll
            for (int k = 0; k < kShtPairs; ++k) {
                b1[k] = h.x;
                d1[k] = h.y;
            }
            m = L - 1;
        }
        for (; m > 0; m -= 2) {
            const double2 ha = H[m];
            const double2 hb = H[m - 1];
#pragma unroll
            for (int k = 0; k < kShtPairs; ++k) {
                b2[k] = fma(cc[k], b1[k], ha.x - b2[k]);
                b1[k] = fma(cc[k], b2[k], hb.x - b1[k]);
                d2[k] = fma(cc[k], d1[k], ha.y - d2[k]);
                d1[k] = fma(cc[k], d2[k], hb.y - d1[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kShtPairs; ++k) {
            const int j = j0 + k;
            if (j >= npairs) continue;
            double sa, ca;
            sincospi(2.0 * (double)j / (double)R.n, &sa, &ca);
            const double C = b1[k] - b2[k] * ca;     // b_0 - b_1 cos a
            const double S = d2[k] * sa;             // d_1 sin a
            const float y0 = (float)(C - S);
            o[j] = accumulate ? o[j] + y0 : y0;
            const int jm = j == 0 ? 0 : R.n - j;
            if (jm != j) {
                const float y1 = (float)(C + S);
                o[jm] = accumulate ? o[jm] + y1 : y1;
            }
        }
    }
}

// ----------------------------------------------------------- belt FFTs --
// A ring of n = 2M pixels, M a power of two.  The real transform
// X_m = sum_j x_j e^{-2 pi i m j / n} comes from the complex FFT Z of
// z_k = x_{2k} + i x_{2k+1} (length M):
//     X_m = (Z_m + conj Z_{M-m}) / 2 - i e^{-i pi m / M} (Z_m - conj Z_{M-m}) / 2,
// and the inverse from Z_q = (S_q + conj S_{M-q}) + i e^{i pi q / M} (S_q - conj S_{M-q})
// for a Hermitian spectrum S (S_{n-m} = conj S_m, zero above lcut < M), whose
// inverse complex FFT gives z_k = y_{2k} + i y_{2k+1}.  The FFT is radix 2,
// decimation in time, in place in LDS after a bit-reversed load; tw[t] =
// e^{-2 pi i t / M} for t < M/2 and hw[m] = e^{-i pi m / M} for m <= M are
// plan tables.

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// In-place FFT of z (bit-reversed input order), sign -1 (forward) or +1.
__device__ __forceinline__ void fft_lds(double2 *z, const double2 *__restrict__ tw, int M,
                                        int logM, bool inverse)
{
    for (int st = 0; st < logM; ++st) {
        const int h = 1 << st;
        for (int b = threadIdx.x; b < (M >> 1); b += kShtThreads) {
            const int j = b & (h - 1);
            const int k = ((b >> st) << (st + 1)) + j;
            double2 w = tw[j << (logM - 1 - st)];
            if (inverse) w.y = -w.y;
            const double2 a = z[k];
            const double2 t = cmul(w, z[k + h]);
            z[k] = make_double2(a.x + t.x, a.y + t.y);
            z[k + h] = make_double2(a.x - t.x, a.y - t.y);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kShtThreads) void k_sht_fft_fwd(
    const ShtRing *__restrict__ rings, const int *__restrict__ ring_list,
    const double2 *__restrict__ tw, const double2 *__restrict__ hw, const float *__restrict__ x,
    double2 *__restrict__ F, int L, int nrings, int M, int logM)
{
    extern __shared__ double2 z[];
    const int r = ring_list[blockIdx.x];
    const ShtRing R = rings[r];
    const float *xr = x + R.first;
    for (int k = threadIdx.x; k < M; k += kShtThreads) {
        const float2 v = *reinterpret_cast<const float2 *>(xr + 2 * k);
        z[__brev((unsigned)k) >> (32 - logM)] = make_double2((double)v.x, (double)v.y);
    }
    __syncthreads();
    fft_lds(z, tw, M, logM, false);
    for (int m = threadIdx.x; m <= L; m += kShtThreads) {
        const double2 a = z[m & (M - 1)];
        const double2 b = conj2(z[(M - m) & (M - 1)]);
        const double2 e = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
        const double2 d = make_double2(0.5 * (a.x - b.x), 0.5 * (a.y - b.y));
        // X_m = e - i hw[m] d
        const double2 hd = cmul(hw[m], d);
        const double2 X = make_double2(e.x + hd.y, e.y - hd.x);
        // times e^{-i m phi_0}, phi_0 = two_o pi / n
        const long long q = ((long long)m * R.two_o) % (2LL * R.n);
        double sp, cp;
        sincospi((double)q / (double)R.n, &sp, &cp);
        F[(size_t)m * nrings + r] = make_double2(cp * X.x + sp * X.y, cp * X.y - sp * X.x);
    }
}

__global__ __launch_bounds__(kShtThreads) void k_sht_fft_bwd(
    const ShtRing *__restrict__ rings, const int *__restrict__ ring_list,
    const double2 *__restrict__ tw, const double2 *__restrict__ hw, const double2 *__restrict__ G,
    float *__restrict__ out, int L, int nrings, int M, int logM, int accumulate)
{
    extern __shared__ double2 z[];
    const int r = ring_list[blockIdx.x];
    const ShtRing R = rings[r];
    // S_m = G_r(m) e^{i m phi_0} for 1 <= m <= lcut, S_0 = Re G_r(0), else 0
    auto spec = [&](int m) -> double2 {
        if (m > L) return make_double2(0.0, 0.0);
        const double2 g = G[(size_t)m * nrings + r];
        if (m == 0) return make_double2(g.x, 0.0);
        const long long q = ((long long)m * R.two_o) % (2LL * R.n);
        double sp, cp;
        sincospi((double)q / (double)R.n, &sp, &cp);
        return make_double2(g.x * cp - g.y * sp, g.x * sp + g.y * cp);
    };
    for (int qi = threadIdx.x; qi < M; qi += kShtThreads) {
        const double2 a = spec(qi);
        const double2 b = conj2(spec(qi == 0 ? M : M - qi));
        const double2 e = make_double2(a.x + b.x, a.y + b.y);
        const double2 d = make_double2(a.x - b.x, a.y - b.y);
        // Z_q = e + i conj(hw[q]) d
        const double2 hd = cmul(conj2(hw[qi]), d);
        z[__brev((unsigned)qi) >> (32 - logM)] = make_double2(e.x - hd.y, e.y + hd.x);
    }
    __syncthreads();
    fft_lds(z, tw, M, logM, true);
    float *o = out + R.first;
    for (int k = threadIdx.x; k < M; k += kShtThreads) {
        const double2 v = z[k];
        float2 y = make_float2((float)v.x, (float)v.y);
        if (accumulate) {
            const float2 p = *reinterpret_cast<const float2 *>(o + 2 * k);
            y.x = p.x + y.x;
            y.y = p.y + y.y;
        }
        *reinterpret_cast<float2 *>(o + 2 * k) = y;
    }
}

// ---------------------------------------------------------------- host --
struct Harm {
    int nside = 0;
    int nrings = 0;
    int nnorth = 0;     // northern rings and the equator: 2 Nside
    int lcut = 0;
    int max_batch = 1;
    int nchunk = 0;     // ring chunks of kShtThreads rings
    int nchunk_fwd = 0; // ring chunks of the Legendre kernels (kLegChunk rings)
    int device = -1;
    long long npix = 0;
    long long nalm = 0;
    double omega = 0.0;
    std::vector<double> khat;
    ShtRing *d_rings = nullptr;
    double2 *d_rec = nullptr;
    double *d_mnorm = nullptr;
    double *d_kscale = nullptr;
    int *d_ring_lo = nullptr;     // per m: first northern ring whose terms matter
    int *d_dft_rings = nullptr;   // rings of the Goertzel / Clenshaw kernels
    int *d_fft_rings = nullptr;   // rings of the FFT kernels (belt, n = 2^k > 2 lcut)
    double2 *d_tw = nullptr;      // FFT tables tw (M/2) and hw (M + 1)
    double2 *d_hw = nullptr;
    int n_dft = 0, n_fft = 0, fft_m = 0, fft_log = 0;
    double2 *d_F = nullptr;       // F, then G: (lcut+1) x nrings
    double2 *d_part = nullptr;    // nchunk x nalm
    double2 *d_alm = nullptr;
    long long device_bytes = 0;
};

static void harm_free(Harm &h)
{
    if (h.device >= 0) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(h.device);
        (void)hipDeviceSynchronize();
        for (void *p : {(void *)h.d_rings, (void *)h.d_rec, (void *)h.d_mnorm, (void *)h.d_kscale,
                        (void *)h.d_ring_lo, (void *)h.d_dft_rings, (void *)h.d_fft_rings,
                        (void *)h.d_tw, (void *)h.d_hw, (void *)h.d_F, (void *)h.d_part,
                        (void *)h.d_alm})
            if (p) (void)hipFree(p);
        (void)hipSetDevice(cur);
    }
    h.d_rings = nullptr;
    h.d_rec = nullptr;
    h.d_mnorm = nullptr;
    h.d_kscale = nullptr;
    h.d_ring_lo = nullptr;
    h.d_dft_rings = nullptr;
    h.d_fft_rings = nullptr;
    h.d_tw = nullptr;
    h.d_hw = nullptr;
    h.d_F = nullptr;
    h.d_part = nullptr;
    h.d_alm = nullptr;
}

static int harm_alloc(void **p, size_t bytes, long long *total)
{
    if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ARKCOS_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    *total += (long long)bytes;
    return ARKCOS_OK;
}

static int harm_upload_kernel(Harm &h)
{
    std::vector<double> ks(h.lcut + 1);
    for (int l = 0; l <= h.lcut; ++l) ks[l] = h.omega * h.khat[l];
    ARKCOS_HIP_CHECK(hipMemcpy(h.d_kscale, ks.data(), ks.size() * sizeof(double),
                               hipMemcpyHostToDevice));
    return ARKCOS_OK;
}

static int harm_build(Harm &h)
{
    const int L = h.lcut;
    std::vector<ShtRing> rings(h.nrings);
    for (int i = 0; i < h.nrings; ++i) {
        const HostRing g = ring_geometry(h.nside, i + 1);
        rings[i].z = g.z;
        rings[i].s = g.s;
        rings[i].log2s = std::log2(g.s);
        rings[i].n = g.n;
        rings[i].first = (int)g.first;
        rings[i].two_o = g.two_o;
        rings[i].pad = 0;
    }
    // recurrence coefficients A = a_lm, B = a_lm b_lm, and log2 of the
    // lambda_mm normalisation sqrt((2m+1)!!/(4 pi (2m)!!))
    std::vector<double2> rec((size_t)h.nalm);
    std::vector<double> mnorm(L + 1);
    double acc = -std::log2(4.0 * M_PI);
    for (int m = 0; m <= L; ++m) {
        if (m > 0) acc += std::log2((2.0 * m + 1.0) / (2.0 * m));
        mnorm[m] = 0.5 * acc;
        const long long base = alm_base(m, L);
        rec[base] = make_double2(0.0, 0.0);
        for (int l = m + 1; l <= L; ++l) {
            const double dl = l, dm = m;
            const double a = std::sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
            const double b = std::sqrt(((dl - 1.0) * (dl - 1.0) - dm * dm) /
                                       (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
            rec[base + (l - m)] = make_double2(a, a * b);
        }
    }
    // Per order m, the first northern ring (rings run from the pole to the
    // equator, sin theta increasing) on which some lambda_lm, l <= lcut,
    // exceeds 2^-394: below it every term is negligible and the Legendre
    // kernels skip the ring.  For fixed l and m, |lambda_lm| grows with
    // sin theta until the oscillatory range, so the rings that matter are a
    // suffix and a bisection finds its start.
    std::vector<int> ring_lo(L + 1, 0);
    auto matters = [&](int i, int m) {
        const ShtRing &Rg = rings[i];
        double e = mnorm[m] + m * Rg.log2s;      // log2 |lambda_mm|
        if (e > -394.0) return true;
        double scale = std::floor(e);               // |lambda| = v1 2^scale
        double v1 = std::exp2(e - scale);
        double v2 = 0.0;
        const long long base = alm_base(m, L);
        for (int l = m + 1; l <= L; ++l) {
            const double2 ab = rec[base + (l - m)];
            const double v = ab.x * Rg.z * v1 - ab.y * v2;
            v2 = v1;
            v1 = v;
            if (std::fabs(v1) > 0x1p200 || (std::fabs(v1) < 0x1p-200 && v1 != 0.0)) {
                int k = 0;
                std::frexp(v1, &k);
                v1 = std::ldexp(v1, -k);
                v2 = std::ldexp(v2, -k);
                scale += k;
            }
            if (v1 != 0.0 && std::log2(std::fabs(v1)) + scale > -394.0) return true;
        }
        return false;
    };
    for (int m = 0; m <= L; ++m) {
        int lo = 0, hi = h.nnorth - 1;           // first index in [lo, hi] that matters
        if (!matters(hi, m)) {
            ring_lo[m] = hi;
            continue;
        }
        while (lo < hi) {
            const int mid = lo + (hi - lo) / 2;
            if (matters(mid, m)) hi = mid; else lo = mid + 1;
        }
        ring_lo[m] = lo;
    }
    // Belt rings take the FFT when their length n = 4 Nside is a power of two,
    // n/2 fits the LDS (complex FP64) and lcut < n/2; the others Goertzel.
    std::vector<int> dft_rings, fft_rings;
    {
        const int n = 4 * h.nside;
        const bool pow2 = (n & (n - 1)) == 0;
        const int M = n / 2;
        const bool fft = pow2 && M >= 2 && M <= kShtFftMaxM && L < M &&
                         std::getenv("ARKCOS_SHT_NO_FFT") == nullptr;
        for (int i = 0; i < h.nrings; ++i) {
            if (fft && rings[i].n == n) fft_rings.push_back(i); else dft_rings.push_back(i);
        }
        if (fft) {
            h.fft_m = M;
            h.fft_log = 0;
            while ((1 << h.fft_log) < M) ++h.fft_log;
        }
    }
    h.n_dft = (int)dft_rings.size();
    h.n_fft = (int)fft_rings.size();
    ARKCOS_HIP_CHECK(hipGetDevice(&h.device));
    int rc;
    if ((rc = harm_alloc((void **)&h.d_rings, rings.size() * sizeof(ShtRing), &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_rec, rec.size() * sizeof(double2), &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_mnorm, mnorm.size() * sizeof(double), &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_kscale, (L + 1) * sizeof(double), &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_ring_lo, (L + 1) * sizeof(int), &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_dft_rings, dft_rings.size() * sizeof(int), &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_fft_rings, fft_rings.size() * sizeof(int), &h.device_bytes)))
        return rc;
    if (h.n_fft > 0) {
        const int M = h.fft_m;
        std::vector<double2> tw(M / 2 > 0 ? M / 2 : 1), hw(M + 1);
        for (int t = 0; t < M / 2; ++t)
            tw[t] = make_double2(std::cos(2.0 * M_PI * t / M), -std::sin(2.0 * M_PI * t / M));
        for (int m = 0; m <= M; ++m)
            hw[m] = make_double2(std::cos(M_PI * m / M), -std::sin(M_PI * m / M));
        if ((rc = harm_alloc((void **)&h.d_tw, tw.size() * sizeof(double2), &h.device_bytes)))
            return rc;
        if ((rc = harm_alloc((void **)&h.d_hw, hw.size() * sizeof(double2), &h.device_bytes)))
            return rc;
        ARKCOS_HIP_CHECK(hipMemcpy(h.d_tw, tw.data(), tw.size() * sizeof(double2),
                                   hipMemcpyHostToDevice));
        ARKCOS_HIP_CHECK(hipMemcpy(h.d_hw, hw.data(), hw.size() * sizeof(double2),
                                   hipMemcpyHostToDevice));
        const size_t lds = (size_t)M * sizeof(double2);
        ARKCOS_HIP_CHECK(hipFuncSetAttribute((const void *)k_sht_fft_fwd,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        ARKCOS_HIP_CHECK(hipFuncSetAttribute((const void *)k_sht_fft_bwd,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    if (!dft_rings.empty())
        ARKCOS_HIP_CHECK(hipMemcpy(h.d_dft_rings, dft_rings.data(), dft_rings.size() * sizeof(int),
                                   hipMemcpyHostToDevice));
    if (!fft_rings.empty())
        ARKCOS_HIP_CHECK(hipMemcpy(h.d_fft_rings, fft_rings.data(), fft_rings.size() * sizeof(int),
                                   hipMemcpyHostToDevice));
    if ((rc = harm_alloc((void **)&h.d_F, (size_t)(L + 1) * h.nrings * sizeof(double2),
                         &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_part, (size_t)h.nchunk_fwd * h.nalm * sizeof(double2),
                         &h.device_bytes)))
        return rc;
    if ((rc = harm_alloc((void **)&h.d_alm, (size_t)h.nalm * sizeof(double2), &h.device_bytes)))
        return rc;
    ARKCOS_HIP_CHECK(hipMemcpy(h.d_rings, rings.data(), rings.size() * sizeof(ShtRing),
                               hipMemcpyHostToDevice));
    ARKCOS_HIP_CHECK(hipMemcpy(h.d_rec, rec.data(), rec.size() * sizeof(double2),
                               hipMemcpyHostToDevice));
    ARKCOS_HIP_CHECK(hipMemcpy(h.d_mnorm, mnorm.data(), mnorm.size() * sizeof(double),
                               hipMemcpyHostToDevice));
    ARKCOS_HIP_CHECK(hipMemcpy(h.d_ring_lo, ring_lo.data(), ring_lo.size() * sizeof(int),
                               hipMemcpyHostToDevice));
    return harm_upload_kernel(h);
}

// The five kernels for one map.
static int harm_launch(const Harm &h, const float *in, float *out, int accumulate, hipStream_t s)
{
    const int L = h.lcut;
    const size_t fft_lds = (size_t)h.fft_m * sizeof(double2);
    if (h.n_fft > 0)
        hipLaunchKernelGGL(k_sht_fft_fwd, dim3(h.n_fft), dim3(kShtThreads), fft_lds, s, h.d_rings,
                           h.d_fft_rings, h.d_tw, h.d_hw, in, h.d_F, L, h.nrings, h.fft_m,
                           h.fft_log);
    // frequencies per thread, kShtMaxFreq per launch
    for (int m0 = 0, left = (L + kShtThreads) / kShtThreads; h.n_dft > 0 && left > 0;
         m0 += kShtMaxFreq * kShtThreads, left -= kShtMaxFreq) {
        switch (std::min(left, kShtMaxFreq)) {
#define ARKCOS_DFT_CASE(K)                                                                   \
    case K:                                                                                  \
        hipLaunchKernelGGL(k_sht_dft_fwd<K>, dim3(h.n_dft), dim3(kShtThreads), 0, s,        \
                           h.d_rings, h.d_dft_rings, in, h.d_F, m0, L, h.nrings);            \
        break;
            ARKCOS_DFT_CASE(1) ARKCOS_DFT_CASE(2) ARKCOS_DFT_CASE(3) ARKCOS_DFT_CASE(4)
            ARKCOS_DFT_CASE(5) ARKCOS_DFT_CASE(6) ARKCOS_DFT_CASE(7)
            default: ARKCOS_DFT_CASE(8)
#undef ARKCOS_DFT_CASE
        }
    }
    hipLaunchKernelGGL(k_sht_leg_fwd, dim3(h.nchunk_fwd, L + 1), dim3(kShtThreads), 0, s, h.d_rings,
                       h.d_F, h.d_rec, h.d_mnorm, h.d_ring_lo, (double *)h.d_part, L, h.nrings,
                       h.nnorth, h.nalm);
    hipLaunchKernelGGL(k_sht_mul, dim3((L + kShtThreads) / kShtThreads, L + 1), dim3(kShtThreads),
                       0, s, h.d_part, h.d_kscale, h.d_ring_lo, h.d_alm, L, h.nchunk_fwd, h.nalm);
    hipLaunchKernelGGL(k_sht_leg_bwd, dim3(h.nchunk_fwd, L + 1), dim3(kShtThreads), 0, s, h.d_rings,
                       h.d_alm, h.d_rec, h.d_mnorm, h.d_ring_lo, h.d_F, L, h.nrings, h.nnorth);
    if (h.n_dft > 0)
        hipLaunchKernelGGL(k_sht_dft_bwd, dim3(h.n_dft), dim3(kShtThreads),
                           (size_t)(L + 1) * sizeof(double2), s, h.d_rings, h.d_dft_rings, h.d_F,
                           out, L, h.nrings, accumulate);
    if (h.n_fft > 0)
        hipLaunchKernelGGL(k_sht_fft_bwd, dim3(h.n_fft), dim3(kShtThreads), fft_lds, s, h.d_rings,
                           h.d_fft_rings, h.d_tw, h.d_hw, h.d_F, out, L, h.nrings, h.fft_m,
                           h.fft_log, accumulate);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

static bool overlap(const float *a, const float *b, long long n)
{
    return a < b + n && b < a + n;
}

}  // namespace arkcos

using namespace arkcos;

extern "C" {

int arkcos_harm_create(int nside, int lcut, const double *khat, int max_batch,
                       arkcos_harm_t *out)
{
    clear_error();
    if (!out) return fail(ARKCOS_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (nside < 1 || nside > ARKCOS_MAX_NSIDE)
        return fail(ARKCOS_EINVAL, "nside must lie in 1.." + std::to_string(ARKCOS_MAX_NSIDE));
    if (lcut < 0) return fail(ARKCOS_EINVAL, "lcut must be >= 0");
    if (lcut > ARKCOS_MAX_LCUT)
        return fail(ARKCOS_EUNSUPPORTED, "lcut above " + std::to_string(ARKCOS_MAX_LCUT));
    if (!khat) return fail(ARKCOS_EINVAL, "NULL khat");
    if (max_batch < 1) return fail(ARKCOS_EINVAL, "max_batch must be >= 1");
    Harm *h = new (std::nothrow) Harm();
    if (!h) return fail(ARKCOS_ENOMEM, "host allocation failed");
    h->nside = nside;
    h->nrings = 4 * nside - 1;
    h->nnorth = 2 * nside;
    h->lcut = lcut;
    h->max_batch = max_batch;
    h->npix = 12LL * nside * nside;
    h->omega = 4.0 * M_PI / (double)h->npix;
    h->nalm = alm_base(lcut + 1, lcut);
    h->nchunk = (h->nnorth + kShtThreads - 1) / kShtThreads;
    h->nchunk_fwd = (h->nnorth + kLegChunk - 1) / kLegChunk;
    int rc;
    try {
        h->khat.assign(khat, khat + lcut + 1);
        rc = harm_build(*h);
    } catch (const std::bad_alloc &) {
        rc = fail(ARKCOS_ENOMEM, "host allocation failed while building the transform plan");
    }
    if (rc != ARKCOS_OK) {
        harm_free(*h);
        delete h;
        return rc;
    }
    *out = reinterpret_cast<arkcos_harm_t>(h);
    return ARKCOS_OK;
}

int arkcos_harm_destroy(arkcos_harm_t harm)
{
    clear_error();
    if (!harm) return ARKCOS_OK;
    Harm *h = reinterpret_cast<Harm *>(harm);
    harm_free(*h);
    delete h;
    return ARKCOS_OK;
}

int arkcos_harm_set_kernel(arkcos_harm_t harm, const double *khat)
{
    clear_error();
    if (!harm || !khat) return fail(ARKCOS_EINVAL, "NULL pointer");
    Harm *h = reinterpret_cast<Harm *>(harm);
    h->khat.assign(khat, khat + h->lcut + 1);
    int cur = 0;
    ARKCOS_HIP_CHECK(hipGetDevice(&cur));
    ARKCOS_HIP_CHECK(hipSetDevice(h->device));
    int rc = harm_upload_kernel(*h);
    (void)hipSetDevice(cur);
    return rc;
}

int arkcos_harm_get_info(arkcos_harm_t harm, int *nside, int *lcut, long long *nalm,
                         long long *device_bytes)
{
    clear_error();
    if (!harm) return fail(ARKCOS_EINVAL, "NULL transform plan");
    const Harm *h = reinterpret_cast<const Harm *>(harm);
    if (nside) *nside = h->nside;
    if (lcut) *lcut = h->lcut;
    if (nalm) *nalm = h->nalm;
    if (device_bytes) *device_bytes = h->device_bytes;
    return ARKCOS_OK;
}

int arkcos_harm_convolve(arkcos_harm_t harm, const float *d_in, float *d_out, int nbatch,
                         int accumulate, void *stream)
{
    clear_error();
    TraceRange tr("arkcos_harm_convolve");
    if (!harm || !d_in || !d_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    const Harm *h = reinterpret_cast<const Harm *>(harm);
    if (nbatch < 1 || nbatch > h->max_batch)
        return fail(ARKCOS_EINVAL, "nbatch must lie in 1.." + std::to_string(h->max_batch));
    if (accumulate != 0 && accumulate != 1) return fail(ARKCOS_EINVAL, "accumulate must be 0 or 1");
    if (overlap(d_in, d_out, h->npix * nbatch))
        return fail(ARKCOS_EINVAL, "d_in and d_out overlap");
    for (int b = 0; b < nbatch; ++b) {
        int rc = harm_launch(*h, d_in + (size_t)b * h->npix, d_out + (size_t)b * h->npix,
                             accumulate, (hipStream_t)stream);
        if (rc) return rc;
    }
    return ARKCOS_OK;
}

int arkcos_split_convolve(arkcos_plan_t plan, arkcos_harm_t harm, const float *d_in,
                          float *d_out, int nbatch, void *stream)
{
    clear_error();
    TraceRange tr("arkcos_split_convolve");
    if (!plan || !harm) return fail(ARKCOS_EINVAL, "NULL plan");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    const Harm *h = reinterpret_cast<const Harm *>(harm);
    if (P->nside != h->nside)
        return fail(ARKCOS_EINVAL, "the two halves are planned for different Nside");
    int rc = arkcos_convolve(plan, d_in, d_out, nbatch, stream);
    if (rc) return rc;
    return arkcos_harm_convolve(harm, d_in, d_out, nbatch, 1, stream);
}

}  // extern "C"
