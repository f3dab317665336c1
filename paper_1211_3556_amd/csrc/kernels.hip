// gfx950 kernels of the real-space convolution (Sutter, Wandelt & Elsner 2012,
// Sec. 2: the real-space part of the split kernel applied by direct summation
// on the GPU; Sec. 3: radial kernel interpolated from a node table).
//
// Every output ring is gathered by one of two kernels, which write disjoint
// rings:
//
//  * k_circ / k_circ_mfma (circulant rings: belt rings whose whole disc lies
//    in the belt).  All their source rings have 4N pixels, so the weight of
//    (r, j; s, j') depends on j' - j only.  Each (r, s) has one weight row,
//    evaluated once per node table by k_build_weights (angles in FP64,
//    weights rounded once to FP32).
//    The gather is then a correlation: a workgroup owns kGroupRings
//    consecutive output rings and kCircSeg pixels of each and stages one
//    source row and its weights at a time in LDS.  Plans whose rows are short
//    run it on the vector ALUs (per quad of taps two float4 reads of the row
//    and four broadcast reads of the weights feed 64 FMAs); plans with longer
//    rows run it on the matrix cores, as a Toeplitz product per row.
//
//  * k_general (polar caps and belt rings whose disc reaches a cap).  Weights
//    are evaluated per pair in FP32 from exact ring-pair constants: chord from
//    d^2 = A + B sin^2(dphi/2), angle by series, node table in LDS with
//    linear interpolation.  A quarter turn maps pixel j of a ring to
//    j + n/4, the N-S mirror maps ring i to ring 4N - i and the reflection
//    phi -> pi/2 - phi maps a pair to one with the opposite longitude
//    difference, so one weight serves sixteen pairs; source rows are staged
//    in LDS as four arrays of four images each.  With a per-pair kernel
//    evaluation this gather runs on the vector ALUs.
//
// Sums are FP32 within a source-ring row and FP64 across rows.  No atomics
// touch the outputs: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "arkcos_internal.hpp"

namespace arkcos {

// Plan data is read-only while a gather runs.  Reading it through the
// constant address space lets wave-uniform loads (ring and pair records,
// weight rows) become scalar loads.  (The host pass of the compiler, which
// never runs these bodies, sees an ordinary pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using cptr = const __attribute__((address_space(4))) T *;
#else
template <class T>
using cptr = const T *;
#endif
template <class T>
__device__ __forceinline__ cptr<T> cst(const T *p)
{
    return (cptr<T>)(p);
}

// ------------------------------------------------------------ FP32 math --
// sin(x) by its Taylor series through x^13, for |x| <= 2 (truncation below
// 2e-8 relative).  Rows whose candidates stay at small |x| use the
// polynomial of their pair record instead.
__device__ __forceinline__ float sin_series(float x)
{
    const float x2 = x * x;
    float p = 1.0f / 6227020800.0f;           // 1/13!
    p = fmaf(p, x2, -1.0f / 39916800.0f);     // 1/11!
    p = fmaf(p, x2, 1.0f / 362880.0f);        // 1/9!
    p = fmaf(p, x2, -1.0f / 5040.0f);         // 1/7!
    p = fmaf(p, x2, 1.0f / 120.0f);           // 1/5!
    p = fmaf(p, x2, -1.0f / 6.0f);            // 1/3!
    p = fmaf(p, x2, 1.0f);
    return x * p;
}

// asin(y) for 0 <= y <= 0.5 by its Maclaurin series
// asin(y) = sum_k (2k)! / (4^k (k!)^2 (2k+1)) y^(2k+1), k = 0..9.
__device__ __forceinline__ float asin_series(float y)
{
    const float z = y * y;
    float p = 12155.0f / 1245184.0f;
    p = fmaf(p, z, 6435.0f / 557056.0f);
    p = fmaf(p, z, 143.0f / 10240.0f);
    p = fmaf(p, z, 231.0f / 13312.0f);
    p = fmaf(p, z, 63.0f / 2816.0f);
    p = fmaf(p, z, 35.0f / 1152.0f);
    p = fmaf(p, z, 5.0f / 112.0f);
    p = fmaf(p, z, 3.0f / 40.0f);
    p = fmaf(p, z, 1.0f / 6.0f);
    p = fmaf(p, z, 1.0f);
    return y * p;
}

// theta = 2 asin(d/2) from the squared chord d^2.
//  AM 0 (theta_cut <= 0.1 rad): d (1 + d^2/24 + 3 d^4/640), truncation below
//       1e-9 relative for d <= 0.1;
//  AM 1 (theta_cut <= 0.5 rad): d (1 + d^2/24 + 3 d^4/640 + 5 d^6/7168
//       + 35 d^8/294912 + 63 d^10/2883584), below 1e-9 for d^2 <= 0.245;
//  AM 2 (any cut): asin series, with asin(y) = pi/2 - 2 asin(sqrt((1 - y)/2))
//       above y = 1/2 to keep the series argument below 1/2.
// The series have positive coefficients, so the computed angle grows with d
// and a candidate beyond the cut never lands inside it.  The square roots are
// the hardware instruction (1 ulp).
template <int AM>
__device__ __forceinline__ float theta_of(float d2)
{
    if (AM == 2) {
        const float y = fminf(0.5f * __builtin_amdgcn_sqrtf(d2), 1.0f);
        if (y <= 0.5f) return 2.0f * asin_series(y);
        const float w = __builtin_amdgcn_sqrtf(0.5f * (1.0f - y));
        return 2.0f * (1.5707963267948966f - 2.0f * asin_series(w));
    }
    const float d = __builtin_amdgcn_sqrtf(d2);
    float p;
    if (AM == 1) {
        p = 63.0f / 2883584.0f;
        p = fmaf(p, d2, 35.0f / 294912.0f);
        p = fmaf(p, d2, 5.0f / 7168.0f);
        p = fmaf(p, d2, 3.0f / 640.0f);
    } else {
        p = 3.0f / 640.0f;
    }
    p = fmaf(p, d2, 1.0f / 24.0f);
    p = fmaf(p, d2, 1.0f);
    return d * p;
}

// 4 (x mod n) for byte offsets xb = 4x with -n <= x < 2n and nb = 4n: of
// xb, xb + nb and xb - nb read as unsigned, the one in [0, nb) is the
// smallest (the others are at least nb or wrap to above 2^31).
__device__ __forceinline__ unsigned wrap_bytes(int xb, int nb)
{
    return min(min((unsigned)xb, (unsigned)(xb + nb)), (unsigned)(xb - nb));
}

// The same for 0 <= x < 2n.
__device__ __forceinline__ unsigned wrap_bytes_up(unsigned xb, unsigned nb)
{
    return min(xb, xb - nb);
}

// j mod n for -n <= j < 3n.
__device__ __forceinline__ int wrap3(int j, int n)
{
    j = (j < 0) ? j + n : j;
    j = (j >= n) ? j - n : j;
    return (j >= n) ? j - n : j;
}

// Exact longitude numerator m = (2j + 2o_r) n_s - (2j' + 2o_s) n_r; the
// product terms may exceed 2^31 but the difference does not, so wrap-around
// arithmetic modulo 2^32 gives it exactly.  Every factor is below 2^23 in
// magnitude (n <= 4 N_side, |2j' + 2o_s| < 4 n_s), so the 24-bit multiply
// (full rate, low 32 bits of the exact product) serves.
__device__ __forceinline__ unsigned lon_base(int j, int two_o_r, int n_s)
{
    return (unsigned)__mul24(2 * j + two_o_r, n_s);
}
__device__ __forceinline__ int lon_numerator(unsigned mbase, int jq, int two_o_s, int n_r)
{
    return (int)(mbase - (unsigned)__mul24(2 * jq + two_o_s, n_r));
}

__device__ __forceinline__ void load_table(float *lds, const float *table, int ntab)
{
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) lds[i] = table[i];
}

// Work item of a persistent kernel, made wave-uniform.
__device__ __forceinline__ int next_item(unsigned int *counter, int *s_item)
{
    __syncthreads();
    if (threadIdx.x == 0) *s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_item);
}

// Input and output maps of a launch: plan p reads in[p] and writes out[p]
// (nmaps consecutive maps of Npix pixels each).
struct MapIO {
    const float *in[kMaxMaps];
    float *out[kMaxMaps];
};

// ------------------------------------------------------- circulant gather --
// Source pixels each lane prefetches per row: a row spans at most
// kCircSeg + kCircMaxTaps - 1 pixels, and the reads of the last tap quad reach
// kCircSeg + kCircMaxTaps - 1 as well (lane 255, taps padded to 256).
constexpr int kStageRegs = (kCircSeg + kCircMaxTaps + kThreads - 1) / kThreads;
// Weights each lane prefetches per row: kGroupRings per tap.
constexpr int kWeightRegs = kCircMaxTaps * kGroupRings / kThreads;

// A load at a 32-bit byte offset from a wave-uniform base: the base stays in
// scalar registers and no 64-bit address arithmetic is needed per lane.
__device__ __forceinline__ float ld_off(const float *base, unsigned byte_off)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Issue the global loads of one staged row (pixels base .. base+nstage-1 of a
// ring of n pixels, wrapped) into registers.
__device__ __forceinline__ void prefetch_row(const float *src, int base, int nstage, int n,
                                             float v[kStageRegs])
{
    const int xb = 4 * (base + (int)threadIdx.x);
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u) {
        const int e = threadIdx.x + u * kThreads;
        v[u] = (e < nstage) ? ld_off(src, wrap_bytes(xb + 4 * u * kThreads, 4 * n)) : 0.0f;
    }
}

// The same for the row's nw = ntaps * kGroupRings weights.
__device__ __forceinline__ void prefetch_weights(const float *w, int nw, float v[kWeightRegs])
{
#pragma unroll
    for (int u = 0; u < kWeightRegs; ++u) {
        const int e = threadIdx.x + u * kThreads;
        v[u] = (e < nw) ? ld_off(w, 4u * (unsigned)e) : 0.0f;
    }
}

// FP32 partial sums move into the FP64 totals once this many taps (FP32
// terms per output) have accumulated, and at the end of a tile.
constexpr int kCircFlush = 64;

// Weight buffers in LDS: a row's taps (kGroupRings floats each) between two
// zero tap quads, which the matrix-core form reads past both ends of a row.
constexpr int kCircWBuf = (kCircMaxTaps + 8) * kGroupRings;   // floats per weight buffer
constexpr int kCircWRow = 4 * kGroupRings;                     // offset of tap 0
constexpr int kCircWavePix = kCircSeg / (kThreads / 64);       // pixels of one wave
static_assert(kCircWavePix == 256 && kGroupRings == 4, "circulant tile shape");
typedef float circ_v4f __attribute__((ext_vector_type(4)));

// Rows of one circulant tile, double-buffered: the loads of row t+1 (source
// pixels and weights) are in flight while row t is multiplied, and one
// barrier per row separates the buffers.  Returns the tile's FP64 sums in
// acc, in the form's own lane layout (see the two forms below).
template <bool MF>
__device__ __forceinline__ void circ_rows(const DevPlanView &P, const DevTile &T,
                                          const DevGroup &G, int n, const float *in, float *xs,
                                          float *wls, int buf_floats, double acc[4][4])
{
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[q][c] = 0.0;
    // vector form: racc[r][i], ring r at pixel 4 l + i of lane l.
    // matrix form: d[q][c], ring l >> 4 at pixel 256 w + 64 q + 4 (l & 15) + c.
    float racc[4][4];
    circ_v4f d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d[q] = circ_v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 4; ++c) racc[q][c] = 0.0f;
    }
    // matrix form: A[(r,p)][u] = w[r][u - p] sits at float 4 (u - p) + r of
    // the row; B[u][b] = x[4 b + u] at this wave's first N tile
    const int a_lane = kCircWRow + 4 * ((lane >> 4) - (lane & 3)) + ((lane & 15) >> 2);
    const int b_lane = kCircWavePix * wave + 4 * (lane & 15) + (lane >> 4);
    float v[kStageRegs], wv[kWeightRegs];
    if (G.row_begin < G.row_end) {
        const DevRow W = cst(P.rows)[G.row_begin];
        prefetch_row(in + W.first_s, T.j0 + W.k_lo, T.len + W.ntaps - 1, n, v);
        prefetch_weights(P.wts + W.w_off, W.ntaps * kGroupRings, wv);
    }
    int since = 0;   // taps summed in FP32 since the last move into FP64
    int buf = 0;
    for (int row = G.row_begin; row < G.row_end; ++row) {
        const DevRow W = cst(P.rows)[row];
        float *xb = xs + buf * buf_floats;
        float *wb = wls + buf * kCircWBuf;
#pragma unroll
        for (int u = 0; u < kStageRegs; ++u) xb[threadIdx.x + u * kThreads] = v[u];
#pragma unroll
        for (int u = 0; u < kWeightRegs; ++u) wb[kCircWRow + threadIdx.x + u * kThreads] = wv[u];
        __syncthreads();
        if (row + 1 < G.row_end) {
            const DevRow W1 = cst(P.rows)[row + 1];
            prefetch_row(in + W1.first_s, T.j0 + W1.k_lo, T.len + W1.ntaps - 1, n, v);
            prefetch_weights(P.wts + W1.w_off, W1.ntaps * kGroupRings, wv);
        }
        if (MF) {
            // K steps of four u over u = 0 .. ntaps + 2 (taps are zero past ntaps)
            const int nks = (W.ntaps + 6) >> 2;
            const float *ap = wb + a_lane;
            const float *bp = xb + b_lane;
            for (int ks = 0; ks < nks; ++ks) {
                const float a = ap[16 * ks];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    d[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bp[64 * q + 4 * ks], d[q], 0,
                                                                0, 0);
            }
        } else {
            // lane l owns pixels 4l .. 4l+3: taps t0 .. t0+3 need
            // x[4l + t0 .. 4l + t0 + 6], two aligned float4 reads (the buffer is
            // zero past the row's taps, so whole tap quads are read)
            const float4 *w4 = reinterpret_cast<const float4 *>(wb + kCircWRow);
            const float4 *x4 = reinterpret_cast<const float4 *>(xb) + threadIdx.x;
            for (int q = 0; q < W.ntaps; q += 4) {
                const float4 xa = x4[q >> 2];
                const float4 xc = x4[(q >> 2) + 1];
                const float xv[8] = {xa.x, xa.y, xa.z, xa.w, xc.x, xc.y, xc.z, xc.w};
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    const float4 wt = w4[q + tt];
                    const float wr[kGroupRings] = {wt.x, wt.y, wt.z, wt.w};
#pragma unroll
                    for (int i = 0; i < kCircPix; ++i)
#pragma unroll
                        for (int r = 0; r < kGroupRings; ++r)
                            racc[r][i] = fmaf(wr[r], xv[i + tt], racc[r][i]);
                }
            }
        }
        since += W.ntaps;
        if (since >= kCircFlush || row + 1 == G.row_end) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc[q][c] += MF ? (double)d[q][c] : (double)racc[q][c];
                    racc[q][c] = 0.0f;
                }
                d[q] = circ_v4f{0.0f, 0.0f, 0.0f, 0.0f};
            }
            since = 0;
        }
        buf ^= 1;
    }
}

// Persistent circulant gather over tiles (plan, group, segment) x maps, in
// one of two forms, each its own kernel, chosen per plan (circ_form):
//  * vector FMAs: the weights of a tap are read from LDS by every lane at one
//    address (a broadcast), so the FMAs take all operands from vector
//    registers (an FMA with a scalar-register operand issues at about 0.6x
//    the rate on gfx950); lane l owns pixels 4l .. 4l+3 of all four rings.
//  * matrix cores: per row the gather is a Toeplitz product, run as
//    v_mfma_f32_16x16x4f32 (FP32 in and out).  For output pixel 4b + p of
//    ring r (b a block of four pixels, p its phase) and u = p + t,
//      out[r][4b + p] = sum_u w[r][u - p] x[4b + u],
//    so D[(r,p)][b] = sum_u A[(r,p)][u] B[u][b] with A[(r,p)][u] = w[r][u - p]
//    (zero outside the row) and B[u][b] = x[4b + u]: M = 16 rows are four
//    rings times four phases, N = 16 pixel blocks (64 pixels), K steps of
//    four u.  A wave owns 256 pixels as four N tiles, so each A fragment
//    feeds four products.  Lane l holds A[(l & 15)][l >> 4] and
//    B[l >> 4][l & 15] and receives D[4 (l >> 4) + c][l & 15], c = 0..3:
//    ring l >> 4 at four consecutive pixels.  K runs over ntaps + 3 values
//    of u, so short rows waste a larger share of the products: the plan takes
//    this form when its rows average at least kCircMfmaTaps taps.
template <bool MF>
__device__ __forceinline__ void circ_gather(const DevPlanView *__restrict__ views,
                                            const int2 *__restrict__ tile_map, int ntiles,
                                            const MapIO &io, int nmaps, int buf_floats,
                                            unsigned int *counter)
{
    extern __shared__ __align__(16) float xs[];
    float *wls = xs + 2 * buf_floats;      // two weight buffers of kCircWBuf floats
    __shared__ int s_item;
    // the zero tap quads around both weight buffers (rows fill only the middle)
    if ((int)threadIdx.x < kCircWRow) {
        const int e = (int)threadIdx.x;
        wls[e] = 0.0f;
        wls[kCircWBuf - kCircWRow + e] = 0.0f;
        wls[kCircWBuf + e] = 0.0f;
        wls[2 * kCircWBuf - kCircWRow + e] = 0.0f;
    }
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int nitems = ntiles * nmaps;
    for (;;) {
        const int item = next_item(counter, &s_item);
        if (item >= nitems) break;
        const int ti = item / nmaps;
        const int map = item - ti * nmaps;
        const int pi = tile_map ? cst(tile_map)[ti].x : 0;
        const int lt = tile_map ? cst(tile_map)[ti].y : ti;
        const DevPlanView P = cst(views)[pi];
        const DevTile T = cst(P.ctiles)[lt];
        const DevGroup G = cst(P.groups)[T.r];
        const int n = cst(P.rings)[G.r0].n;
        const float *in = io.in[pi] + (size_t)map * P.npix;
        float *out = io.out[pi] + (size_t)map * P.npix;
        double acc[4][4];
        circ_rows<MF>(P, T, G, n, in, xs, wls, buf_floats, acc);
        if (MF) {
            // ring lane >> 4, pixels 256 w + 64 q + 4 (lane & 15) + c (T.len is
            // a multiple of 4)
            const int r = lane >> 4;
            if (r < G.nr) {
                float *o = out + cst(P.rings)[G.r0 + r].first + T.j0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int px = kCircWavePix * wave + 64 * q + 4 * (lane & 15);
                    if (px < T.len) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) o[px + c] = (float)acc[q][c];
                    }
                }
            }
        } else if (4 * (int)threadIdx.x < T.len) {   // T.len is a multiple of 4
#pragma unroll
            for (int r = 0; r < kGroupRings; ++r) {
                if (r < G.nr) {
                    float *o = out + cst(P.rings)[G.r0 + r].first + T.j0 + 4 * threadIdx.x;
#pragma unroll
                    for (int i = 0; i < kCircPix; ++i) o[i] = (float)acc[r][i];
                }
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_circ(
    const DevPlanView *__restrict__ views, const int2 *__restrict__ tile_map, int ntiles, MapIO io,
    int nmaps, int buf_floats, unsigned int *counter)
{
    circ_gather<false>(views, tile_map, ntiles, io, nmaps, buf_floats, counter);
}

// Six waves per SIMD: the compiler then spills a few registers that the row
// loop does not touch, and the matrix pipes see more independent waves (the
// wide-row workloads ran 3-15 % faster than at four waves without spills).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_circ_mfma(
    const DevPlanView *__restrict__ views, const int2 *__restrict__ tile_map, int ntiles, MapIO io,
    int nmaps, int buf_floats, unsigned int *counter)
{
    circ_gather<true>(views, tile_map, ntiles, io, nmaps, buf_floats, counter);
}

// --------------------------------------------------------- general gather --
// Reflection about phi = pi/4 (phi -> pi/2 - phi) maps pixel j of quadrant 0
// of a ring with offset o to jbar = n/4 - 2o - j, and a pair (j, j') to
// (jbar, j'bar) with the opposite longitude difference: the same weight.
// Together with the four quarter turns and the N-S mirror one weight serves
// sixteen pairs.  A general tile holds a segment of up to kGenLanes pixels
// j <= jbar of the first quadrant of 1, 2 or 4 adjacent northern rings (the
// tile shapes are plan parameters); the kGenThreads lanes split into one part
// per ring, 2^lp lanes of a part share each pixel and take every 2^lp-th
// candidate of its window, and one node table in LDS serves all of them.
// Source rows are staged in the chunks the plan lists per tile (GenChunk):
// per source position j', the four quarter turns of x at j' on ring s and on
// its mirror, then the same at j'bar: four float4 arrays of kGenStage entries.

// Largest value of `v` over the wave (wave-uniform result).
__device__ __forceinline__ int wave_max(int v)
{
    // every lane is active and every source lane exists, so each DPP move
    // folds into the max that uses it
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));  // row_mirror
    const int r0 = __builtin_amdgcn_readlane(v, 0);
    const int r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32);
    const int r3 = __builtin_amdgcn_readlane(v, 48);
    return max(max(r0, r1), max(r2, r3));
}

// A wave-uniform value held in a vector register.  On gfx950 a VALU
// instruction with a scalar-register operand issues at about 0.6x the rate of
// one with vector operands only, and an FMA can read one scalar register at
// most; copies made once, outside a loop, avoid both.
__device__ __forceinline__ float vreg(float s)
{
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}
__device__ __forceinline__ int vreg(int s)
{
    int v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// u = theta / h from the squared chord.  For the short series the factor
// 1/h is folded into the coefficients (u_coef = inv_h times those of
// theta_of), which saves one multiply per pair; `lead` is the highest
// coefficient, in a vector register.
struct UCoef {
    float c[6];     // u_coef in vector registers
    float inv_h;
};

template <int AM>
__device__ __forceinline__ UCoef ucoef(const DevPlanView &P)
{
    UCoef u;
#pragma unroll
    for (int k = 0; k < 6; ++k) u.c[k] = (AM == 1 || k < 3) ? vreg(P.u_coef[k]) : 0.0f;
    u.inv_h = vreg(P.inv_h);
    return u;
}

template <int AM>
__device__ __forceinline__ float node_coord(float d2, const UCoef &uc)
{
    if (AM == 2) return theta_of<2>(d2) * uc.inv_h;
    const float d = __builtin_amdgcn_sqrtf(d2);
    float p;
    if (AM == 1) {
        p = fmaf(uc.c[5], d2, uc.c[4]);
        p = fmaf(p, d2, uc.c[3]);
        p = fmaf(p, d2, uc.c[2]);
    } else {
        p = uc.c[2];
    }
    p = fmaf(p, d2, uc.c[1]);
    p = fmaf(p, d2, uc.c[0]);
    return d * p;
}

// One staged position per thread: source position c0 + e of ring s and its
// reflection, four quarter turns each, on ring s (a, c) and its mirror (b, d).
// Threads at or past cn load nothing: positions past the chunk are never
// read.  Loads address their ring by 32-bit byte offsets shared between a
// ring and its mirror (the ring's base stays in scalar registers).
template <int SIDE>
__device__ __forceinline__ void prefetch16(const float *src, const float *srcm, int n_s,
                                           int two_o_s, int c0, int cn, float4 &a, float4 &b,
                                           float4 &c, float4 &d)
{
    const int e = threadIdx.x;
    if (e >= cn) return;
    // byte offsets in the ring: jd of position c0 + e (-n_s < c0 + e < 2 n_s),
    // jr of its reflection qs - 2o_s - jd (-n_s < . < n_s), and their quarter turns
    const int nb = 4 * n_s;
    const unsigned qb = (unsigned)nb >> 2;
    const unsigned jd = wrap_bytes(4 * (c0 + e), nb);
    const int jr0 = (int)qb - 4 * two_o_s - (int)jd;
    const unsigned jr = min((unsigned)jr0, (unsigned)(jr0 + nb));
    unsigned od[4], orf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        od[k] = wrap_bytes_up(jd + k * qb, (unsigned)nb);
        orf[k] = wrap_bytes_up(jr + k * qb, (unsigned)nb);
    }
    // SIDE 1 (2): one-sided tiles read only ring s (its mirror), a and c (b and d)
    if (SIDE != 2) {
        a = make_float4(ld_off(src, od[0]), ld_off(src, od[1]), ld_off(src, od[2]),
                        ld_off(src, od[3]));
        c = make_float4(ld_off(src, orf[0]), ld_off(src, orf[1]), ld_off(src, orf[2]),
                        ld_off(src, orf[3]));
    }
    // loaded for the equator ring too, so that every load of the chunk issues
    // from one branch-free sequence: the general gather never writes the
    // equator's south sums, and the knot gradient gives them zero g
    if (SIDE != 1) {
        b = make_float4(ld_off(srcm, od[0]), ld_off(srcm, od[1]), ld_off(srcm, od[2]),
                        ld_off(srcm, od[3]));
        d = make_float4(ld_off(srcm, orf[0]), ld_off(srcm, orf[1]), ld_off(srcm, orf[2]),
                        ld_off(srcm, orf[3]));
    }
}

// Images of a staged position whose ring lies outside the plan's source rings
// count as zero: ring s (a, c; mask bit 0) and its mirror (b, d; bit 1).
// Wave-uniform.
__device__ __forceinline__ void mask_sources(int mask, float4 &a, float4 &b, float4 &c, float4 &d)
{
    const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (mask & 1) a = c = z;
    if (mask & 2) b = d = z;
}

// Issue the loads of a staged chunk (its record read by scalar loads): all
// four image arrays (SIDE 0) or those of one side (1: ring s, 2: its mirror).
template <int SIDE = 0>
__device__ __forceinline__ void prefetch_chunk(const float *in, const GenChunk &c, float4 &a,
                                               float4 &b, float4 &d2, float4 &d)
{
    prefetch16<SIDE>(in + c.first, in + c.first_m, c.n, c.two_o, c.c0, c.cn, a, b, d2, d);
    mask_sources(c.mask, a, b, d2, d);
}

// Plan constants of the candidate loop, in vector registers.
template <int AM>
struct GenConst {
    float zslot;     // index of the table's zero entries
    float br, bc;    // coarse coordinate from the break of a biased grid, br u0 + bc
    int kb;          // node index of the break
    UCoef ucf;
    __device__ __forceinline__ GenConst(const DevPlanView &P)
        : zslot(vreg((float)P.ntab)), br(vreg(P.bias_r)), bc(vreg(P.bias_c)),
          kb(vreg(P.k_break)), ucf(ucoef<AM>(P)) {}
};

// T candidates jq, jq + step, ... of one lane in the staged chunk; those past
// a1 get the table's zero slot.  T is the wave's largest count.  One
// candidate per iteration: its staged reads issue first and overlap the
// weight arithmetic (unrolled by two, the loop spills at 128 VGPRs).
// BIAS: the plan's node grid is the two-piece biased one.  Beyond the break
// the candidate's node is k_break + v, v = r u0 - r k_break counted from the
// break, so that v keeps FP32's relative precision there (k_break + v in one
// float would round it to ~1e-3 of a coarse node); otherwise u = u0 and the
// map costs nothing.
// SIDE 0: all sixteen images; SIDE 1 (2): only the ring's (the mirror ring's)
// eight, for tiles whose other half lies outside a ring-range plan.
template <bool LONG, int AM, bool INTM, bool BIAS, int SIDE>
__device__ __forceinline__ void gen_candidates16(const DevPair &pp, const GenConst<AM> &gc,
                                                 const float *tab, int m, int dm, int step,
                                                 const float4 *stage, int c0, int cn, int jq,
                                                 int a1, int T, float row[16])
{
    // every uniform operand of the loop in a vector register
    const float zslot = gc.zslot;
    const float A = LONG ? vreg(pp.A) : 0.0f;
    // LONG: d^2 = A + B sin^2 x with x = m xscale and the sine by its series;
    // otherwise the row polynomial in y = (m mscale)^2: u0^2 in angle mode 0,
    // else d^2
    const float B = LONG ? vreg(pp.B) : 0.0f;
    const float xscale = LONG ? vreg(pp.xscale) : 0.0f;
    const float q0 = LONG ? 0.0f : vreg(pp.sq[0]);
    const float q1 = LONG ? 0.0f : vreg(pp.sq[1]);
    const float q2 = LONG ? 0.0f : vreg(pp.sq[2]);
    const float q3 = LONG ? 0.0f : vreg(pp.sq[3]);
    const float q4 = (LONG || AM != 0) ? 0.0f : vreg(pp.sq[4]);
    const UCoef &ucf = gc.ucf;
    // Candidates are addressed by LDS byte address: o steps by 16 step bytes,
    // a lane's candidates end at o_a1 and reads clamp to the chunk's last
    // staged position (the clamped reads carry weight zero).  The staged
    // images are read first, so their latency overlaps the weight arithmetic
    // and the table lookup waits once for both.
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) const v4f lds_float4;
    const int sb = (int)(size_t)(lds_float4 *)stage;
    int o = sb + 16 * (jq - c0);
    const int o_a1 = sb + 16 * (a1 - c0);
    const int o_last = vreg(sb + 16 * (cn - 1));
    const int o_step = vreg(16 * step);
    // The longitude numerator m falls by dm per candidate.  It is kept as an
    // FP32 integer, exact while |m| < 2^24 (the plan checks this per ring and
    // otherwise selects INTM), times a power of two on short rows, so it
    // carries no rounding.
    const float ms = LONG ? 1.0f : pp.mscale;
    float mf = (float)m * ms;
    const float dmf = vreg((float)dm * ms);
    int mi = m;
    const int dmi = vreg(dm);
    // The disc is |m| <= mcut on the exact numerator (mf carries the same
    // power of two on short rows); the FP32 angle only weights the pair.
    const float mcut_f = vreg((float)pp.mcut * ms);
    const unsigned mcut_u = (unsigned)vreg(pp.mcut);
    // the node table by LDS byte address, and its coarse piece's node 0 (the
    // break) in a vector register, so that choosing between them is one select
    typedef __attribute__((address_space(3))) const float lds_float;
    const int tab_b = (int)(size_t)(lds_float *)tab;
    const int tab_cb = BIAS ? vreg(tab_b + 4 * gc.kb) : tab_b;
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
        const bool valid = o <= o_a1;
        const int oc = min(o, o_last);
        lds_float4 *sp = (lds_float4 *)(size_t)oc;
        // SIDE 0: ring and mirror at j' and at the reflection of j'; one-sided:
        // the side's two arrays only (row[0..3] direct, row[4..7] reflected)
        const v4f v0 = sp[(SIDE == 2 ? 1 : 0) * kGenStage];
        const v4f v1 = sp[(SIDE == 0 ? 1 : (SIDE == 1 ? 2 : 3)) * kGenStage];
        const v4f v2 = SIDE == 0 ? sp[2 * kGenStage] : v0;
        const v4f v3 = SIDE == 0 ? sp[3 * kGenStage] : v1;
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the arithmetic
        float u0;
        if (LONG) {
            const float x = (INTM ? (float)mi : mf) * xscale;   // half the longitude difference
            const float sx = sin_series(x);
            u0 = node_coord<AM>(fmaf(B, sx * sx, A), ucf);
        } else if (AM == 0) {
            const float y = mf * mf;
            u0 = __builtin_amdgcn_sqrtf(fmaf(fmaf(fmaf(fmaf(y, q4, q3), y, q2), y, q1), y, q0));
        } else {
            const float y = mf * mf;
            u0 = node_coord<AM>(fmaf(fmaf(fmaf(y, q3, q2), y, q1), y, q0), ucf);
        }
        const float v = BIAS ? fmaf(u0, gc.br, gc.bc) : 0.0f;
        const bool coarse = BIAS && v >= 0.0f;
        const bool inside = INTM ? (unsigned)mi + mcut_u <= 2u * mcut_u : fabsf(mf) <= mcut_f;
        const bool keep = valid && inside;
        const float uc = keep ? (coarse ? v : u0) : zslot;
        const int tb = (keep && coarse) ? tab_cb : tab_b;   // the coarse piece from the break
        const int node = (int)uc;
        const float frac = __builtin_amdgcn_fractf(uc);
        lds_float *kp = (lds_float *)(size_t)(tb + 4 * node);
        const float k0 = kp[0];
        const float k1 = kp[1];
        const float w = fmaf(frac, k1 - k0, k0);
        row[0] = fmaf(w, v0.x, row[0]);
        row[1] = fmaf(w, v0.y, row[1]);
        row[2] = fmaf(w, v0.z, row[2]);
        row[3] = fmaf(w, v0.w, row[3]);
        row[4] = fmaf(w, v1.x, row[4]);
        row[5] = fmaf(w, v1.y, row[5]);
        row[6] = fmaf(w, v1.z, row[6]);
        row[7] = fmaf(w, v1.w, row[7]);
        if (SIDE == 0) {
            row[8] = fmaf(w, v2.x, row[8]);
            row[9] = fmaf(w, v2.y, row[9]);
            row[10] = fmaf(w, v2.z, row[10]);
            row[11] = fmaf(w, v2.w, row[11]);
            row[12] = fmaf(w, v3.x, row[12]);
            row[13] = fmaf(w, v3.y, row[13]);
            row[14] = fmaf(w, v3.z, row[14]);
            row[15] = fmaf(w, v3.w, row[15]);
        }
        o += o_step;
        if (INTM)
            mi -= dmi;
        else
            mf -= dmf;
    }
}

// FP32 partial sums are moved into the FP64 totals once a lane has
// accumulated at least this many candidates since the last move.
constexpr int kGenFlush = 48;

// One general tile (DevTile2) of nr adjacent rings: the lanes form nr equal
// parts of whole waves, part h taking ring q[h] (idle where its len is 0).
// Per staged chunk of a source ring, each part runs the candidates of its
// own ring's row, the sum over the lanes of a pixel follows, and each part
// writes the sixteen images of its pixels.  LONG, AM, INTM and BIAS are fixed
// per tile, so the candidate loop has one form and the row sums stay in place
// across rows.
template <bool LONG, int AM, bool INTM, bool BIAS, int SIDE>
__device__ __forceinline__ void gen_tile2(const DevPlanView &P, const float *tab, float4 *stage,
                                          const DevTile2 *Tp, const float *in, float *out)
{
    constexpr int NI = SIDE == 0 ? 16 : 8;   // images summed per lane
    const int nr = cst(Tp)->nr;
    const int kPart = kGenThreads / nr;   // lanes per ring: 512, 256 or 128
    // wave-uniform (a part is whole waves); made scalar so that every branch
    // on the part is a scalar branch
    const int h = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kPart);
    const int tid = (int)threadIdx.x - h * kPart;
    const GenRing my = cst(Tp->q)[h];
    const int len = my.len;
    const int rn = my.r;                                // an idle part holds a valid ring
    const int rs = P.nrings - 1 - rn;                   // mirror ring
    const bool mirror = rs != rn;
    const DevRing R = cst(P.rings)[rn];
    const int qr = R.n >> 2;
    // 2^lp lanes per pixel: 4 / nr for a full segment, more (up to a wave)
    // for a shorter one, so that every lane works
    int lp = 0;
    while (lp < 6 && (kPart >> (lp + 1)) >= len) ++lp;
    const int nph = 1 << lp;
    const int ph = tid & (nph - 1);
    const int lane_pix = tid >> lp;
    const bool active = lane_pix < len;
    const int j = cst(Tp)->j0 + min(lane_pix, max(len - 1, 0));
    const GenConst<AM> gc(P);

    // the tile's staged chunks: record k + 1 is read (scalar loads, no
    // dependence on earlier loads) while chunk k is used
    const cptr<GenChunk> C = cst(P.gchunks) + cst(Tp)->c_begin;
    const int nch = cst(Tp)->nchunks;
    float4 pa, pb, pc, pd;
    GenChunk ch{};
    if (nch > 0) {   // (a tile whose rows are all empty has no record)
        ch = C[0];
        prefetch_chunk<SIDE>(in, ch, pa, pb, pc, pd);
    }
    double acc[16];
    float row[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        acc[q] = 0.0;
        row[q] = 0.0f;
    }
    int since = 0;
    for (int k = 0; k < nch; ++k) {
        const GenChunk nx = C[min(k + 1, nch - 1)];
        __syncthreads();      // the previous chunk is no longer read
        if ((int)threadIdx.x < ch.cn) {   // the arrays the loop form reads
            if (SIDE != 2) {
                stage[threadIdx.x] = pa;
                stage[2 * kGenStage + threadIdx.x] = pc;
            }
            if (SIDE != 1) {
                stage[kGenStage + threadIdx.x] = pb;
                stage[3 * kGenStage + threadIdx.x] = pd;
            }
        }
        __syncthreads();
        if (k + 1 < nch) prefetch_chunk<SIDE>(in, nx, pa, pb, pc, pd);
        // this part's row of source ring ch.s, if its ring has one
        if (len > 0 && ch.s >= my.s_lo && ch.s <= my.s_hi) {
            const DevPair pp = cst(P.pairs)[my.pb + ch.s - my.s_lo];
            // this lane's candidates inside the chunk: a0 + ph, a0 + ph + nph, ...
            int lo, hi;
            pair_window(pp, ch.n, j, lo, hi);
            const int a0 = max(lo, ch.c0);
            const int a1 = min(hi, ch.c0 + ch.cn - 1);
            const int mine = a1 - a0 - ph >= 0 ? ((a1 - a0 - ph) >> lp) + 1 : 0;
            const int nt = wave_max(mine);
            const int jq0 = a0 + ph;
            const unsigned mbase = lon_base(j, R.two_o, ch.n);
            const int m0 = lon_numerator(mbase, jq0, ch.two_o, R.n);
            const int dm = 2 * nph * R.n;
            gen_candidates16<LONG, AM, INTM, BIAS, SIDE>(pp, gc, tab, m0, dm, nph, stage, ch.c0,
                                                         ch.cn, jq0, a1, nt, row);
            since += nt;
            if (since >= kGenFlush) {   // FP32 partial sums into the FP64 totals
#pragma unroll
                for (int q = 0; q < NI; ++q) {
                    acc[q] += (double)row[q];
                    row[q] = 0.0f;
                }
                since = 0;
            }
        }
        ch = nx;
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) acc[q] += (double)row[q];
    for (int x = 1; x < nph; x <<= 1) {       // the lanes of a pixel, same order in each
#pragma unroll
        for (int q = 0; q < NI; ++q) acc[q] += __shfl_xor(acc[q], x);
    }
    if (SIDE != 0) {   // one side: acc[0..3] at j, acc[4..7] at the reflected pixel
        const bool wr = (SIDE == 1 ? (my.flags & kTileSkipNorth) : (my.flags & kTileSkipSouth)) == 0;
        if (active && wr && (SIDE == 1 || mirror)) {
            float *o = out + cst(P.rings)[SIDE == 1 ? rn : rs].first;
            if (ph == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) o[j + q * qr] = (float)acc[q];
            }
            if (ph == (nph > 1 ? 1 : 0)) {
                const int jb = qr - R.two_o - j;
                if (jb != j && jb != qr) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) o[jb + q * qr] = (float)acc[4 + q];
                }
            }
        }
        return;
    }
    // a ring-range plan leaves rings outside its range untouched
    const bool wn = (my.flags & kTileSkipNorth) == 0;
    const bool ws = mirror && (my.flags & kTileSkipSouth) == 0;
    if (active) {
        float *o = out + R.first;
        float *om = out + cst(P.rings)[rs].first;
        if (ph == 0) {
            if (wn) {
#pragma unroll
                for (int q = 0; q < 4; ++q) o[j + q * qr] = (float)acc[q];
            }
            if (ws) {
#pragma unroll
                for (int q = 0; q < 4; ++q) om[j + q * qr] = (float)acc[4 + q];
            }
        }
        if (ph == (nph > 1 ? 1 : 0)) {   // a second lane, or the only one
            const int jb = qr - R.two_o - j;   // reflected pixel; j itself at a fixed point
            if (jb != j && jb != qr) {
                if (wn) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) o[jb + q * qr] = (float)acc[8 + q];
                }
                if (ws) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) om[jb + q * qr] = (float)acc[12 + q];
                }
            }
        }
    }
}

// The candidate-loop form of a tile: sine series, angle series and numerator
// type from the tile and plan, the node-grid map from BIAS.
template <bool BIAS>
__device__ __forceinline__ void gen_tile_variant(const DevPlanView &P, const float *tab,
                                                 float4 *stage, const DevTile2 *Tp,
                                                 const float *in, float *out)
{
    int fl = 0, skip_all = kTileSkipNorth | kTileSkipSouth;
    for (int k = 0; k < cst(Tp)->nr; ++k) {
        const GenRing q = cst(Tp->q)[k];
        fl |= q.flags;
        if (q.len > 0) skip_all &= q.flags;
    }
    const bool lg = (fl & kTileLongSin) != 0;
    if (fl & kTileIntM) {   // wide windows on large rings (long sine implied)
        switch (P.angle_mode) {
            case 0: gen_tile2<true, 0, true, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            case 1: gen_tile2<true, 1, true, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            default: gen_tile2<true, 2, true, BIAS, 0>(P, tab, stage, Tp, in, out); break;
        }
    } else if (!lg && (skip_all & kTileSkipSouth)) {   // every ring writes its own side only
        switch (P.angle_mode) {
            case 0: gen_tile2<false, 0, false, BIAS, 1>(P, tab, stage, Tp, in, out); break;
            case 1: gen_tile2<false, 1, false, BIAS, 1>(P, tab, stage, Tp, in, out); break;
            default: gen_tile2<false, 2, false, BIAS, 1>(P, tab, stage, Tp, in, out); break;
        }
    } else if (!lg && (skip_all & kTileSkipNorth)) {   // ... its mirror's side only
        switch (P.angle_mode) {
            case 0: gen_tile2<false, 0, false, BIAS, 2>(P, tab, stage, Tp, in, out); break;
            case 1: gen_tile2<false, 1, false, BIAS, 2>(P, tab, stage, Tp, in, out); break;
            default: gen_tile2<false, 2, false, BIAS, 2>(P, tab, stage, Tp, in, out); break;
        }
    } else {
        switch (P.angle_mode * 2 + (lg ? 1 : 0)) {
            case 0: gen_tile2<false, 0, false, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            case 1: gen_tile2<true, 0, false, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            case 2: gen_tile2<false, 1, false, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            case 3: gen_tile2<true, 1, false, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            case 4: gen_tile2<false, 2, false, BIAS, 0>(P, tab, stage, Tp, in, out); break;
            default: gen_tile2<true, 2, false, BIAS, 0>(P, tab, stage, Tp, in, out); break;
        }
    }
}

// Persistent general gather over tiles (plan, north ring, half-quadrant
// segment) x maps.  LDS: the node table of the current plan followed by two
// zero entries (the slot of candidates outside the disc), then the stage.
// The loads of the next chunk are in flight while the current one is used.
__global__ __launch_bounds__(kGenThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_general(const DevPlanView *__restrict__ views, const int2 *__restrict__ tile_map,
               int ntiles, MapIO io, int nmaps, int tab_floats, unsigned int *counter)
{
    extern __shared__ __align__(16) float lds[];
    float *tab = lds;
    float4 *stage = reinterpret_cast<float4 *>(lds + tab_floats);
    __shared__ int s_item;
    const int nitems = ntiles * nmaps;
    int cur = -1;
    for (;;) {
        const int item = next_item(counter, &s_item);
        if (item >= nitems) break;
        const int ti = item / nmaps;
        const int map = item - ti * nmaps;
        const int pi = tile_map ? cst(tile_map)[ti].x : 0;
        const int lt = tile_map ? cst(tile_map)[ti].y : ti;
        const DevPlanView P = cst(views)[pi];
        if (pi != cur) {
            load_table(tab, P.table, P.ntab);
            if (threadIdx.x < 2) tab[P.ntab + threadIdx.x] = 0.0f;
            cur = pi;
        }
        const DevTile2 *Tp = P.gtiles2 + lt;
        const float *in = io.in[pi] + (size_t)map * P.npix;
        float *out = io.out[pi] + (size_t)map * P.npix;
        if (P.biased)
            gen_tile_variant<true>(P, tab, stage, Tp, in, out);
        else
            gen_tile_variant<false>(P, tab, stage, Tp, in, out);
    }
}

__global__ void k_reset_counters(unsigned int *counter)
{
    if (threadIdx.x < 3) counter[threadIdx.x] = 0u;
}

// Omega-scaled FP32 table from device knots.
__global__ void k_set_table(float *table, const float *knots, int ntab, float omega)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntab) table[i] = omega * knots[i];
}

// ---------------------------------------------------------- knot gradient --
// Offset (in floats) of the knot-gradient histogram after an ntab-entry FP32
// table: rounded up to 16 bytes.
__host__ __device__ constexpr int hist_offset_floats(int ntab) { return (ntab + 3) & ~3; }

// The knot-gradient kernels bin into one FP64 histogram per wave, so no two
// waves ever add to the same LDS word: with the static tile assignment below
// every bin receives the same additions in the same order on every run (the
// lanes of one atomic instruction are applied in a fixed hardware order).  At
// the end the wave histograms are added in wave order.
constexpr int kKnotWaves = kThreads / 64;
__host__ __device__ constexpr int hist_stride(int ntab) { return (ntab + 1) & ~1; }

template <int WAVES>
__device__ __forceinline__ void write_partials(const double *hists, int hstride, int ntab,
                                               double *dst)
{
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) {
        double t = hists[i];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) t += hists[w * hstride + i];
        dst[i] = t;
    }
}

// ------------------------------------------------------------ FP64 math --
// Coefficients of the series below, evaluated at compile time:
// asin(y) = sum_k c_k y^(2k+1), c_k = (2k)! / (4^k (k!)^2 (2k+1)), and
// sin(x) = sum_k (-1)^k x^(2k+1) / (2k+1)!.
__host__ __device__ constexpr double asin_coef(int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c *= (2.0 * i - 1.0) / (2.0 * i);
    return c / (2.0 * k + 1.0);
}
__host__ __device__ constexpr double sin_coef(int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c /= -(2.0 * i) * (2.0 * i + 1.0);
    return c;
}

// The knot gradient needs node fractions to ~1e-9 (the hat basis has slope
// 1/h in theta), so these FP64 series keep truncation near 1e-15 relative.

// sin(x) in FP64: through x^11 for |x| <= 0.35 (truncation below 6e-15
// relative), through x^21 for |x| <= 2 (below 2e-16).
template <bool LONG>
__device__ __forceinline__ double sin_d(double x)
{
    constexpr int K = LONG ? 10 : 5;
    const double x2 = x * x;
    double p = sin_coef(K);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) p = fma(p, x2, sin_coef(k));
    return x * p;
}

// asin(y) in FP64 for 0 <= y <= 0.5 (truncation below 2e-15 relative).
__device__ __forceinline__ double asin_d(double y)
{
    constexpr int K = 20;
    const double z = y * y;
    double p = asin_coef(K);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) p = fma(p, z, asin_coef(k));
    return y * p;
}

// sqrt in FP64 from the hardware reciprocal square root and two Newton
// steps (each at least squares the relative error), with sqrt(0) = 0.
__device__ __forceinline__ double sqrt_d(double a)
{
    double r = __builtin_amdgcn_rsq(a);
#pragma unroll
    for (int i = 0; i < 2; ++i) r = r * fma(-0.5 * a, r * r, 1.5);
    return a > 0.0 ? a * r : 0.0;
}

// theta = 2 asin(d/2) in FP64 from the squared chord, in the same three
// regimes as theta_of: d (sum_k c_k (d^2/4)^k) with 5 terms for d <= 0.1 and
// 11 terms for d^2 <= 0.245 (truncation below 2e-15), and the full-range
// asin otherwise.
template <int AM>
__device__ __forceinline__ double theta_d(double d2)
{
    if (AM == 2) {
        const double y = fmin(0.5 * sqrt_d(d2), 1.0);
        if (y <= 0.5) return 2.0 * asin_d(y);
        return 2.0 * (1.5707963267948966192 - 2.0 * asin_d(sqrt_d(0.5 * (1.0 - y))));
    }
    constexpr int K = AM == 0 ? 4 : 10;
    const double z = 0.25 * d2;
    double p = asin_coef(K);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) p = fma(p, z, asin_coef(k));
    return sqrt_d(d2) * p;
}

// FP64 node coordinate map of a plan: u = min(a0 theta, r a0 theta + c)
// (r = 1, c = 0 on a uniform grid, where the min returns a0 theta exactly).
struct NodeMapD {
    double a0, r, c, u_max;
    __device__ __forceinline__ explicit NodeMapD(const DevPlanView &P)
        : a0(P.inv_h_d), r(P.bias_r_d), c(P.bias_c_d), u_max((double)(P.ntab - 1)) {}
};

// Node index and fraction of one pair from the FP64 chord constants; false at
// or beyond the cut.  (The knot gradient needs the fraction to ~1e-9: the hat
// basis has slope 1/h in theta.)
template <bool LONG, int AM>
__device__ __forceinline__ bool pair_node_d(const DevPairD &pd, const NodeMapD &nm, int m,
                                            int &node, double &frac)
{
    const double sx = sin_d<LONG>((double)m * pd.xscale);
    const double u0 = theta_d<AM>(fma(pd.B, sx * sx, pd.A)) * nm.a0;
    const double u = fmin(u0, fma(u0, nm.r, nm.c));
    node = (int)fmin(u, nm.u_max - 1.0);
    frac = u - (double)node;
    return u < nm.u_max;
}

// sqrt in FP64 from the FP32 reciprocal square root (relative error near
// 2^-23) and one Newton step, which squares it (below 1e-13); sqrt(a) = 0
// for a below 1e-30.
__device__ __forceinline__ double sqrt_d_seeded(double a)
{
    const double r0 = (double)__builtin_amdgcn_rsqf((float)a);
    const double r = r0 * fma(-0.5 * a, r0 * r0, 1.5);
    return a > 1e-30 ? a * r : 0.0;
}

// Node index and fraction of a pair of the knot gradient.  Short rows
// evaluate their FP64 row polynomial in y = (m mscale)^2 (truncation below
// 1e-9 relative, so fractions stay within ~1e-7 at 2048 nodes); long rows
// take pair_node_d.
template <bool LONG, int AM>
__device__ __forceinline__ bool pair_node_knot(const DevPairD &pd, const NodeMapD &nm, int m,
                                               int &node, double &frac)
{
    if (LONG) return pair_node_d<true, AM>(pd, nm, m, node, frac);
    const double v = (double)m * pd.mscale;
    const double y = v * v;
    double u0;
    if (AM == 0) {
        const double q = fma(fma(fma(fma(pd.sq[4], y, pd.sq[3]), y, pd.sq[2]), y, pd.sq[1]), y,
                             pd.sq[0]);
        u0 = sqrt_d_seeded(q);
    } else {
        const double d2 = fma(fma(fma(pd.sq[3], y, pd.sq[2]), y, pd.sq[1]), y, pd.sq[0]);
        u0 = theta_d<AM>(d2) * nm.a0;
    }
    const double u = fmin(u0, fma(u0, nm.r, nm.c));
    node = (int)fmin(u, nm.u_max - 1.0);
    frac = u - (double)node;
    return u < nm.u_max;
}

// The knot gradient is sum_p g[p] sum_q hat_k(theta_pq) x[q] over the in-disc
// pairs of all maps.  Both kernels below scatter into per-wave FP64 LDS
// histograms, merged per workgroup into partials[row][ntab] and reduced in a
// fixed order by k_knot_reduce.

// Circulant weight slots (row w_off + tap * kGroupRings + ring): tap k of
// ring r of a group on source ring s is the pair at the exact longitude
// numerator m = n (2o_r - 2o_s - 2k).  FP64 node coordinate u of slot e of
// row W, or -1 outside the ring's window or disc.  It depends on the
// geometry only.
__device__ __forceinline__ double slot_node(const DevPlanView &P, const NodeMapD &nm,
                                            const DevRow &W, const DevGroup &G, int n,
                                            int two_o_s, int e)
{
    const int t = e / kGroupRings;
    const int i = e - t * kGroupRings;
    const int k = W.k_lo + t;
    if (i >= G.nr) return -1.0;
    const DevRing R = P.rings[G.r0 + i];
    const int kk = R.pair_begin + (W.s - P.pairs[R.pair_begin].s);
    if (kk < R.pair_begin || kk >= R.pair_end) return -1.0;
    const DevPair pp = P.pairs[kk];
    int lo, hi;
    pair_window(pp, n, 0, lo, hi);
    if (k < lo || k > hi) return -1.0;
    const DevPairD pd = P.pairs_d[kk];
    const bool lg = (pp.mode & kPairLongSin) != 0;
    const int m = n * (R.two_o - two_o_s - 2 * k);
    int node;
    double frac;
    bool in;
    switch (P.angle_mode * 2 + (lg ? 1 : 0)) {
        case 0: in = pair_node_d<false, 0>(pd, nm, m, node, frac); break;
        case 1: in = pair_node_d<true, 0>(pd, nm, m, node, frac); break;
        case 2: in = pair_node_d<false, 1>(pd, nm, m, node, frac); break;
        case 3: in = pair_node_d<true, 1>(pd, nm, m, node, frac); break;
        case 4: in = pair_node_d<false, 2>(pd, nm, m, node, frac); break;
        default: in = pair_node_d<true, 2>(pd, nm, m, node, frac); break;
    }
    return in ? (double)node + frac : -1.0;
}

// Weight rows of the circulant groups, one workgroup per row: the
// interpolated, Omega-scaled FP32 table at the slot's FP64 node coordinate,
// rounded once (0 outside the window or disc).  The weights are built once
// per table, so the FP64 angle costs nothing in the gather and the
// circulant weights carry no FP32 angle error.
__global__ __launch_bounds__(kThreads) void k_build_weights(DevPlanView P)
{
    const int row = blockIdx.x;
    if (row >= P.nrows) return;
    const DevRow W = P.rows[row];
    const DevGroup G = P.groups[W.g];
    const int n = P.rings[G.r0].n;
    const int two_o_s = P.rings[W.s].two_o;
    const NodeMapD nm(P);
    for (int e = threadIdx.x; e < W.ntaps * kGroupRings; e += blockDim.x) {
        const double u = slot_node(P, nm, W, G, n, two_o_s, e);
        float w = 0.0f;
        if (u >= 0.0) {
            const int node = (int)u;               // u < ntab - 1
            const double frac = u - (double)node;
            const double k0 = P.table[node];
            const double k1 = P.table[node + 1];
            w = (float)fma(frac, k1 - k0, k0);
        }
        P.wts[W.w_off + e] = w;
    }
}

// FP64 node coordinate of every circulant weight slot (knot gradients).
__global__ __launch_bounds__(kThreads) void k_build_knotw(DevPlanView P, double *kw)
{
    const int row = blockIdx.x;
    if (row >= P.nrows) return;
    const DevRow W = P.rows[row];
    const DevGroup G = P.groups[W.g];
    const int n = P.rings[G.r0].n;
    const int two_o_s = P.rings[W.s].two_o;
    const NodeMapD nm(P);
    for (int e = threadIdx.x; e < W.ntaps * kGroupRings; e += blockDim.x)
        kw[W.w_off + e] = slot_node(P, nm, W, G, n, two_o_s, e);
}

// Add c * hat(u) to the histogram (u >= 0: node floor(u), fraction u - node).
__device__ __forceinline__ void hat_scatter(double *hist, double u, float c)
{
    const int node = (int)u;
    const double frac = u - (double)node;
    atomicAdd(&hist[node], (1.0 - frac) * (double)c);
    atomicAdd(&hist[node + 1], frac * (double)c);
}

// ------------------------------------------- circulant rings: correlation --
// On circulant rings theta depends on (r, s, tap) only, so
//   sum_j g_r[j] sum_k hat(u(r, s, k)) x_s[j + k]
//     = sum_k hat(u(r, s, k)) C(r, s, k),   C(r, s, k) = sum_j g_r[j] x_s[j + k]:
// the pair loop becomes a cross-correlation of ring r of g with ring s of x,
// and each distinct (r, s, k) is binned once per tile.  A tile is kKnotSeg
// pixels of the kGroupRings rings of a group; its g is staged once, one array
// per ring.  Each wave takes whole source rows (rows w, w + 4, ...
// of the group for wave w), so a row needs no workgroup barrier: the wave
// stages the row's x in its own LDS strip and forms the row's correlation on
// the matrix cores, 13 taps per pass (the layout is at the loop).  Each C is
// binned with the FP64 node coordinates of k_build_knotw into the wave's own
// histogram.

// staged x of one row (floats): the matrix-core correlation reads up to
// 16 ceil(len/16) + 13 floor((ntaps-1)/13) + 12 < kKnotSeg + kCircMaxTaps + 32
constexpr int kKnotXW = kKnotSeg + kCircMaxTaps + 32;

// Orders a wave's LDS stores before its later LDS loads (the hardware keeps a
// wave's LDS operations in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kThreads) void k_knot_circ(const DevPlanView *__restrict__ views,
                                                        const float *__restrict__ g,
                                                        const float *__restrict__ x, int nmaps,
                                                        double *__restrict__ partials)
{
    extern __shared__ __align__(16) double hists[];
    const DevPlanView P = cst(views)[0];
    const int hstride = hist_stride(P.ntab);
    float *gs = reinterpret_cast<float *>(hists + kKnotWaves * hstride);   // [ring][kKnotSeg]
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    float *xs = gs + kGroupRings * kKnotSeg + wave * kKnotXW;
    for (int i = threadIdx.x; i < kKnotWaves * hstride; i += kThreads) hists[i] = 0.0;
    double *hist = hists + wave * hstride;   // this wave's own bins
    const int nitems = P.nkctiles * nmaps;
    // static assignment: the tiles are dealt round-robin
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int ti = item / nmaps;
        const int map = item - ti * nmaps;
        const DevTile T = cst(P.kctiles)[ti];
        const DevGroup G = cst(P.groups)[T.r];
        const int n = cst(P.rings)[G.r0].n;
        const float *in = x + (size_t)map * P.npix;
        const float *gm = g + (size_t)map * P.npix;
        const int npq = (T.len + 3) >> 2;     // pixel quads of the tile
        int firsts[kGroupRings];              // (uniform) first pixel of each ring of the group
#pragma unroll
        for (int i = 0; i < kGroupRings; ++i)
            firsts[i] = cst(P.rings)[G.r0 + min(i, G.nr - 1)].first + T.j0;
        __syncthreads();   // the previous item no longer reads gs
        // g of the group's rings over the tile, zero past the tile or the group
        for (int p = threadIdx.x; p < kKnotSeg; p += kThreads) {
#pragma unroll
            for (int i = 0; i < kGroupRings; ++i)
                gs[i * kKnotSeg + p] = (p < T.len && i < G.nr) ? gm[firsts[i] + p] : 0.0f;
        }
        __syncthreads();
        // each wave takes every kKnotWaves-th row; the loads of its next row's
        // source pixels are in flight while it works on the current one
        constexpr int kXR = kKnotXW / 64 + 1;
        float v[kXR];
        auto load_row = [&](int row) {
            const DevRow W = cst(P.rows)[row];
            // the row's source pixels j0 + k_lo + e, e < nx (-n < k_lo and the
            // positions stay below 3n, so wrap3 applies)
            const int nx = 4 * (npq + ((W.ntaps + 3) >> 2));
            const float *src = in + W.first_s;
            const int base = T.j0 + W.k_lo;
#pragma unroll
            for (int u = 0; u < kXR; ++u) {
                const int e = lane + 64 * u;
                v[u] = e < nx ? src[wrap3(base + e, n)] : 0.0f;
            }
        };
        if (G.row_begin + wave < G.row_end) load_row(G.row_begin + wave);
        for (int row = G.row_begin + wave; row < G.row_end; row += kKnotWaves) {
            const DevRow W = cst(P.rows)[row];
            wave_lds_order();   // the previous row's reads of xs are done
#pragma unroll
            for (int u = 0; u < kXR; ++u) {
                const int e = lane + 64 * u;
                if (e < kKnotXW) xs[e] = v[u];
            }
            wave_lds_order();
            if (row + kKnotWaves < G.row_end) load_row(row + kKnotWaves);
            // C(r, s, k) on the matrix cores, 13 lags k = u0 .. u0 + 12 per pass:
            //   E[(r,p)][u] = sum_b g_r[4b + p] x[4b + u]  (M = 4 rings x 4 phases,
            //   K = pixel blocks b, four per step, N = 16 values of u = u0 + n),
            //   C(r, s, u0 + n) = sum_p E[(r,p)][u0 + n + p], n <= 12.
            // Lane l holds A[(l & 15)][l >> 4] = g_r[16 ks + 4 (l >> 4) + p] with
            // r = (l & 15) >> 2, p = l & 3, and B[l >> 4][l & 15]; it receives
            // E[(l >> 4, c)][u0 + (l & 15)], c = 0..3, so the sum over p takes
            // element c from lane + c of its 16-lane row.
            const double *kw = cst(P.kw) + W.w_off;
            const int nks = (T.len + 15) >> 4;
            const float *ga = gs + ((lane & 15) >> 2) * kKnotSeg + 4 * (lane >> 4) + (lane & 3);
            const float *xb = xs + 4 * (lane >> 4) + (lane & 15);
            const int r = lane >> 4, nn = lane & 15;
            for (int u0 = 0; u0 < W.ntaps; u0 += 13) {
                const int k = u0 + nn;
                const bool mine = nn < 13 && k < W.ntaps && r < G.nr;
                // this lane's FP64 node coordinate, loaded ahead of the products
                const double u = mine ? kw[4 * k + r] : -1.0;
                // four accumulation chains (K steps modulo 4), so that a
                // product never waits for the one before it
                typedef float v4f __attribute__((ext_vector_type(4)));
                v4f d0 = {0.0f, 0.0f, 0.0f, 0.0f}, d1 = d0, d2 = d0, d3 = d0;
                int ks = 0;
                for (; ks + 3 < nks; ks += 4) {
                    const float a0 = ga[16 * ks], b0 = xb[16 * ks + u0];
                    const float a1 = ga[16 * ks + 16], b1 = xb[16 * ks + 16 + u0];
                    const float a2 = ga[16 * ks + 32], b2 = xb[16 * ks + 32 + u0];
                    const float a3 = ga[16 * ks + 48], b3 = xb[16 * ks + 48 + u0];
                    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, d0, 0, 0, 0);
                    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, d1, 0, 0, 0);
                    d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, d2, 0, 0, 0);
                    d3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, b3, d3, 0, 0, 0);
                }
                for (; ks < nks; ++ks)
                    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[16 * ks], xb[16 * ks + u0], d0, 0,
                                                              0, 0);
                const v4f d = (d0 + d1) + (d2 + d3);
                const float c = d[0] + __shfl_down(d[1], 1, 16) + __shfl_down(d[2], 2, 16) +
                                __shfl_down(d[3], 3, 16);
                if (mine && c != 0.0f && u >= 0.0) hat_scatter(hist, u, c);
            }
        }
    }
    __syncthreads();
    write_partials<kKnotWaves>(hists, hstride, P.ntab, partials + (size_t)blockIdx.x * P.ntab);
}

// ------------------------------------------------- general rings: per pair --
// Candidates T of one lane, as in the general gather: the sixteen products
// g x of a candidate share its FP64 node coordinate.
// A lane visits its cnt candidates starting at candidate `skew` and wrapping
// around: neighbouring pixels, whose candidates at the same step have nearly
// the same separation, then add into different bins of the wave's histogram
// at each step instead of contending for one.
template <bool LONG, int AM>
__device__ __forceinline__ void knot_candidates16(const DevPairD &pd, const NodeMapD &nm,
                                                  int m0, int dm, int lp, const float4 *stage,
                                                  int c0, int cn, int jq0, int cnt, int skew,
                                                  int T, const float gv[16], double *hist)
{
    for (int t = 0; t < T; ++t) {
        int tt = t + skew;
        tt = tt >= cnt ? tt - cnt : tt;
        const int jq = jq0 + (tt << lp);
        const int m = m0 - __mul24(tt, dm);
        const int pos = min(max(jq - c0, 0), cn - 1);
        const float4 v0 = stage[pos];
        const float4 v1 = stage[kGenStage + pos];
        const float4 v2 = stage[2 * kGenStage + pos];
        const float4 v3 = stage[3 * kGenStage + pos];
        float c = gv[0] * v0.x;
        c = fmaf(gv[1], v0.y, c);
        c = fmaf(gv[2], v0.z, c);
        c = fmaf(gv[3], v0.w, c);
        c = fmaf(gv[4], v1.x, c);
        c = fmaf(gv[5], v1.y, c);
        c = fmaf(gv[6], v1.z, c);
        c = fmaf(gv[7], v1.w, c);
        c = fmaf(gv[8], v2.x, c);
        c = fmaf(gv[9], v2.y, c);
        c = fmaf(gv[10], v2.z, c);
        c = fmaf(gv[11], v2.w, c);
        c = fmaf(gv[12], v3.x, c);
        c = fmaf(gv[13], v3.y, c);
        c = fmaf(gv[14], v3.z, c);
        c = fmaf(gv[15], v3.w, c);
        if (t < cnt && c != 0.0f) {
            int node;
            double frac;
            if (pair_node_knot<LONG, AM>(pd, nm, m, node, frac)) {
                atomicAdd(&hist[node], (1.0 - frac) * (double)c);
                atomicAdd(&hist[node + 1], frac * (double)c);
            }
        }
    }
}

// Pairs whose output ring is general, over the general gather's tiles and
// staged chunks (1, 2 or 4 adjacent rings sharing each staged source chunk,
// 2^lp lanes per pixel taking every 2^lp-th candidate).  A lane holds g at the
// sixteen output images of its pixel (zero where a ring-range plan writes no
// output, and for the reflected images at a fixed point of the reflection).
// Workgroups take the items blockIdx.x, blockIdx.x + gridDim.x, ... and bin
// into one histogram per wave.
// One instantiation per angle mode (AM), so that only that mode's FP64 series
// constants occupy registers.
constexpr int kGenWaves = kGenThreads / 64;
template <int AM>
__global__ __launch_bounds__(kGenThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_knot_gen(const DevPlanView *__restrict__ views, const float *__restrict__ g,
                const float *__restrict__ x, int nmaps, double *__restrict__ partials)
{
    extern __shared__ __align__(16) double hists[];
    const DevPlanView P = cst(views)[0];
    const int hstride = hist_stride(P.ntab);
    float4 *stage = reinterpret_cast<float4 *>(hists + kGenWaves * hstride);
    for (int i = threadIdx.x; i < kGenWaves * hstride; i += blockDim.x) hists[i] = 0.0;
    double *hist = hists + (threadIdx.x >> 6) * hstride;   // this wave's own bins
    __syncthreads();
    const NodeMapD nm(P);
    const int nitems = P.ngtiles2 * nmaps;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int ti = item / nmaps;
        const int map = item - ti * nmaps;
        const DevTile2 *Tp = P.gtiles2 + ti;
        const int nr = cst(Tp)->nr;
        const int kPart = kGenThreads / nr;
        const int h = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kPart);
        const int tid = (int)threadIdx.x - h * kPart;
        const GenRing my = cst(Tp->q)[h];
        const int len = my.len;
        const int rn = my.r;
        const int rs = P.nrings - 1 - rn;
        const DevRing R = cst(P.rings)[rn];
        const int qr = R.n >> 2;
        int lp = 0;
        while (lp < 6 && (kPart >> (lp + 1)) >= len) ++lp;
        const int nph = 1 << lp;
        const int ph = tid & (nph - 1);
        const int lane_pix = tid >> lp;
        const bool active = lane_pix < len;
        const int j = cst(Tp)->j0 + min(lane_pix, max(len - 1, 0));
        const int jb = qr - R.two_o - j;
        const bool gn_ok = active && (my.flags & kTileSkipNorth) == 0;
        const bool gs_ok = active && rs != rn && (my.flags & kTileSkipSouth) == 0;
        const bool refl = jb != j && jb != qr;
        const float *in = x + (size_t)map * P.npix;
        const float *gm = g + (size_t)map * P.npix;
        float gv[16];
        {
            const float *gn = gm + R.first;
            const float *gsm = gm + cst(P.rings)[rs].first;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gv[q] = gn_ok ? gn[j + q * qr] : 0.0f;
                gv[4 + q] = gs_ok ? gsm[j + q * qr] : 0.0f;
                gv[8 + q] = (refl && gn_ok) ? gn[jb + q * qr] : 0.0f;
                gv[12 + q] = (refl && gs_ok) ? gsm[jb + q * qr] : 0.0f;
            }
        }
        const cptr<GenChunk> C = cst(P.gchunks) + cst(Tp)->c_begin;
        const int nch = cst(Tp)->nchunks;
        float4 pa, pb, pc, pd4;
        GenChunk ch{};
        if (nch > 0) {
            ch = C[0];
            prefetch_chunk(in, ch, pa, pb, pc, pd4);
        }
        for (int k = 0; k < nch; ++k) {
            const GenChunk nx = C[min(k + 1, nch - 1)];
            __syncthreads();
            if ((int)threadIdx.x < ch.cn) {
                stage[threadIdx.x] = pa;
                stage[kGenStage + threadIdx.x] = pb;
                stage[2 * kGenStage + threadIdx.x] = pc;
                stage[3 * kGenStage + threadIdx.x] = pd4;
            }
            __syncthreads();
            if (k + 1 < nch) prefetch_chunk(in, nx, pa, pb, pc, pd4);
            if (len > 0 && ch.s >= my.s_lo && ch.s <= my.s_hi) {
                const int kk = my.pb + ch.s - my.s_lo;
                const DevPair pp = cst(P.pairs)[kk];
                const DevPairD pd = cst(P.pairs_d)[kk];
                int lo, hi;
                pair_window(pp, ch.n, j, lo, hi);
                const int a0 = max(lo, ch.c0);
                const int a1 = min(hi, ch.c0 + ch.cn - 1);
                const int cnt = a1 - a0 - ph >= 0 ? ((a1 - a0 - ph) >> lp) + 1 : 0;
                const int nt = wave_max(cnt);
                const int jq0 = a0 + ph;
                // start candidate: the pixel's index modulo its count (exact: the
                // quotient of the float division is never within 1/(2 cnt) of an integer)
                const int skew = cnt > 0 ? lane_pix - cnt * (int)(((float)lane_pix + 0.5f) / (float)cnt) : 0;
                const unsigned mbase = lon_base(j, R.two_o, ch.n);
                const int m0 = lon_numerator(mbase, jq0, ch.two_o, R.n);
                const int dm = 2 * nph * R.n;
                if (pp.mode & kPairLongSin)
                    knot_candidates16<true, AM>(pd, nm, m0, dm, lp, stage, ch.c0, ch.cn, jq0,
                                                cnt, skew, nt, gv, hist);
                else
                    knot_candidates16<false, AM>(pd, nm, m0, dm, lp, stage, ch.c0, ch.cn, jq0,
                                                 cnt, skew, nt, gv, hist);
            }
            ch = nx;
        }
    }
    __syncthreads();
    write_partials<kGenWaves>(hists, hstride, P.ntab,
                              partials + ((size_t)P.nkpart_circ + blockIdx.x) * P.ntab);
}
// Fixed-order reduction of the per-workgroup partials, scaled by Omega: a
// block of kReduceWaves waves covers 64 knots, wave w sums rows w, w + kReduceWaves, ...,
// and the wave sums are added in wave order.
constexpr int kReduceWaves = 16;
__global__ __launch_bounds__(64 * kReduceWaves) void k_knot_reduce(
    const double *__restrict__ partials, int nblocks, int ntab, double omega,
    float *__restrict__ gk)
{
    __shared__ double red[kReduceWaves][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (k < ntab)
        for (int b = w; b < nblocks; b += kReduceWaves) s += partials[(size_t)b * ntab + k];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && k < ntab) {
        double t = 0.0;
        for (int i = 0; i < kReduceWaves; ++i) t += red[i][lane];
        gk[k] = (float)(omega * t);
    }
}

// ---------------------------------------------------------------- launch --
int forward_threads() { return kThreads; }
int batch_max_maps() { return kMaxMaps; }

int device_lds_limit(int device, size_t *bytes)
{
    hipDeviceProp_t prop;
    ARKCOS_HIP_CHECK(hipGetDeviceProperties(&prop, device));
    *bytes = prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > 0 &&
        (size_t)prop.maxSharedMemoryPerMultiProcessor < *bytes)
        *bytes = prop.maxSharedMemoryPerMultiProcessor;
    *bytes -= 1024;  // static LDS of the kernels
    return ARKCOS_OK;
}

// Resident workgroups per CU for a kernel with `lds` bytes of dynamic LDS.
template <class K>
static int occupancy(K kernel, size_t lds, int *per_cu, int threads = kThreads)
{
    ARKCOS_HIP_CHECK(hipFuncSetAttribute((const void *)kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ARKCOS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, threads, lds));
    if (*per_cu < 1)
        return fail(ARKCOS_EUNSUPPORTED, "kernel cannot be resident with " +
                                             std::to_string(lds) + " bytes of LDS");
    return ARKCOS_OK;
}

// Two row buffers of kStageRegs * kThreads floats each, then two weight
// buffers of kCircWBuf floats (a row between two zero tap quads).
static int circ_buf_floats() { return kStageRegs * kThreads; }
static size_t circ_lds()
{
    return (size_t)2 * (circ_buf_floats() + kCircWBuf) * sizeof(float);
}
// Node table plus its two zero entries, rounded up to 16 bytes, then four
// float4 arrays of kGenStage staged positions.
static int gen_tab_floats(int ntab) { return (ntab + 2 + 3) & ~3; }
static size_t gen_lds(int ntab)
{
    return (size_t)(gen_tab_floats(ntab) + 16 * kGenStage) * sizeof(float);
}
// FP64 histogram (16-byte aligned), then the staged g and x of a circulant
// knot tile, or the general stage.
static size_t knot_hist_bytes(int ntab)
{
    return (size_t)kKnotWaves * hist_stride(ntab) * sizeof(double);
}
// Per-wave FP64 histograms, the tile's g, and per wave one staged row of x and
// the partial sums of its lanes.
static size_t knot_circ_lds(int ntab)
{
    return knot_hist_bytes(ntab) + (size_t)kGroupRings * kKnotSeg * sizeof(float) +
           (size_t)kKnotWaves * kKnotXW * sizeof(float);
}
static size_t knot_gen_lds(int ntab)
{
    return (size_t)kGenWaves * hist_stride(ntab) * sizeof(double) +
           (size_t)4 * kGenStage * sizeof(float4);
}



int prepare_launches(Plan &p)
{
    ARKCOS_HIP_CHECK(hipDeviceGetAttribute(&p.cus, hipDeviceAttributeMultiprocessorCount,
                                           p.device));
    int rc;
    if ((rc = occupancy(p.circ_form ? k_circ_mfma : k_circ, circ_lds(), &p.occ_circ))) return rc;
    if ((rc = occupancy(k_general, gen_lds(p.desc.ntab), &p.occ_gen, kGenThreads))) return rc;
    p.grid_kc = p.grid_kg = 0;
    if ((p.desc.flags & ARKCOS_PLAN_LEARNABLE) && p.desc.ntab <= ARKCOS_MAX_GRAD_NTAB) {
        if ((rc = occupancy(k_knot_circ, knot_circ_lds(p.desc.ntab), &p.occ_kc))) return rc;
        // (the three angle-mode instantiations have the same resource limits)
        if ((rc = occupancy(k_knot_gen<0>, knot_gen_lds(p.desc.ntab), &p.occ_kg, kGenThreads)))
            return rc;
        // one partial row per resident workgroup of each knot kernel, and no
        // more workgroups than work items
        const long long mb = std::max(1, p.desc.max_batch);
        p.grid_kc = (int)std::min<long long>((long long)p.occ_kc * p.cus,
                                             (long long)p.kctiles.size() * mb);
        p.grid_kg = (int)std::min<long long>((long long)p.occ_kg * p.cus,
                                             (long long)p.gtiles2.size() * mb);
    }
    p.grid = std::max(1, p.grid_kc + p.grid_kg);
    return ARKCOS_OK;
}

int prepare_batch(Batch &b)
{
    ARKCOS_HIP_CHECK(hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount,
                                           b.device));
    int occ_c = 0, occ_m = 0, occ_g = 0, rc;
    if ((rc = occupancy(k_circ, circ_lds(), &occ_c))) return rc;
    if ((rc = occupancy(k_circ_mfma, circ_lds(), &occ_m))) return rc;
    if ((rc = occupancy(k_general, gen_lds(b.max_ntab), &occ_g, kGenThreads))) return rc;
    b.grid_circ = std::max(1, std::min(b.ncirc_valu, occ_c * b.cus));
    b.grid_circ_mfma = std::max(1, std::min((int)b.cmap.size() - b.ncirc_valu, occ_m * b.cus));
    b.grid_gen = std::max(1, std::min((int)b.gmap.size(), occ_g * b.cus));
    return ARKCOS_OK;
}

int launch_set_table(const Plan &p, const float *d_knots, hipStream_t s)
{
    const int ntab = p.desc.ntab;
    hipLaunchKernelGGL(k_set_table, dim3((ntab + 255) / 256), dim3(256), 0, s, p.d_table,
                       d_knots, ntab, (float)p.omega);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

int launch_build_weights(const Plan &p, hipStream_t s)
{
    if (p.rows.empty()) return ARKCOS_OK;
    hipLaunchKernelGGL(k_build_weights, dim3((unsigned)p.rows.size()), dim3(kThreads), 0, s,
                       p.view());
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

// The two gathers of one plan over nbatch maps; they write disjoint rings.
int launch_forward(const Plan &p, const float *in, float *out, int nbatch, hipStream_t s,
                   int parts, unsigned int *counter)
{
    MapIO io{};
    io.in[0] = in;
    io.out[0] = out;
    if (!counter) counter = p.d_counter;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counter);
    const int nct = (parts & ARKCOS_PART_CIRCULANT) ? (int)p.ctiles.size() : 0;
    const int ngt = (parts & ARKCOS_PART_GENERAL) ? (int)p.gtiles2.size() : 0;
    if (nct > 0) {
        const int grid = std::max(1, std::min(nct * nbatch, p.occ_circ * p.cus));
        hipLaunchKernelGGL(p.circ_form ? k_circ_mfma : k_circ, dim3(grid), dim3(kThreads),
                           circ_lds(), s, (const DevPlanView *)p.d_view, (const int2 *)nullptr,
                           nct, io, nbatch, circ_buf_floats(), counter);
    }
    if (ngt > 0) {
        const int grid = std::max(1, std::min(ngt * nbatch, p.occ_gen * p.cus));
        hipLaunchKernelGGL(k_general, dim3(grid), dim3(kGenThreads), gen_lds(p.desc.ntab), s,
                           (const DevPlanView *)p.d_view, (const int2 *)nullptr, ngt, io, nbatch,
                           gen_tab_floats(p.desc.ntab), counter + 1);
    }
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

int launch_build_knotw(const Plan &p, hipStream_t s)
{
    if (p.rows.empty()) return ARKCOS_OK;
    hipLaunchKernelGGL(k_build_knotw, dim3((unsigned)p.rows.size()), dim3(kThreads), 0, s,
                       p.view(), p.d_kw);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

// Circulant rings by correlation, general rings per pair; every partial row
// is written (the grids are the rows reserved at plan creation), then reduced.
static int launch_knot(const Plan &p, const float *g, const float *x, float *gk, int nbatch,
                       hipStream_t s, double *kpart)
{
    const int ntab = p.desc.ntab;
    if (p.grid_kc > 0)
        hipLaunchKernelGGL(k_knot_circ, dim3(p.grid_kc), dim3(kThreads), knot_circ_lds(ntab), s,
                           (const DevPlanView *)p.d_view, g, x, nbatch, kpart);
    if (p.grid_kg > 0) {
        auto kg = p.angle_mode == 0 ? k_knot_gen<0>
                                    : (p.angle_mode == 1 ? k_knot_gen<1> : k_knot_gen<2>);
        hipLaunchKernelGGL(kg, dim3(p.grid_kg), dim3(kGenThreads), knot_gen_lds(ntab), s,
                           (const DevPlanView *)p.d_view, g, x, nbatch, kpart);
    }
    ARKCOS_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_knot_reduce, dim3((ntab + 63) / 64), dim3(64 * kReduceWaves), 0, s,
                       kpart, p.grid_kc + p.grid_kg, ntab, p.omega, gk);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

// Zero the pixels [0, lo) and [hi, npix) of nbatch maps.
__global__ void k_zero_outside(float *x, long long npix, long long lo, long long hi,
                               long long total)
{
    const long long nout = npix - (hi - lo);
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long b = t / nout, i = t - b * nout;
        x[b * npix + (i < lo ? i : i + (hi - lo))] = 0.0f;
    }
}

int launch_backward(const Plan &p, const float *g, const float *x, float *gx, float *gk,
                    int nbatch, hipStream_t s, unsigned int *counter, double *kpart)
{
    // The operator is symmetric, so d/dmap is the same gather applied to g;
    // for a ring range it is the adjoint plan's gather (rings within theta_cut
    // of the range, reading g on the range only), and zero elsewhere.
    if (gx) {
        const Plan &a = p.adj ? *p.adj : p;
        if (p.adj) {
            const long long lo = p.rings[a.desc.ring_first - 1].first;
            const HostRing &last = p.rings[a.desc.ring_last - 1];
            const long long hi = last.first + last.n;
            const long long total = (p.npix - (hi - lo)) * nbatch;
            if (total > 0) {
                const long long blocks = std::min<long long>((total + 255) / 256, 8192);
                hipLaunchKernelGGL(k_zero_outside, dim3((unsigned)blocks), dim3(256), 0, s, gx,
                                   p.npix, lo, hi, total);
            }
        }
        int rc = launch_forward(a, g, gx, nbatch, s, ARKCOS_PART_ALL, counter);
        if (rc) return rc;
    }
    if (gk) return launch_knot(p, g, x, gk, nbatch, s, kpart ? kpart : p.d_kpart);
    return ARKCOS_OK;
}

long long knot_partial_bytes(const Plan &p)
{
    return (long long)(p.grid_kc + p.grid_kg) * p.desc.ntab * (long long)sizeof(double);
}

int launch_batch(const Batch &b, const float *const *in, float *const *out, hipStream_t s,
                 int parts)
{
    if ((int)b.plans.size() > kMaxMaps)
        return fail(ARKCOS_EUNSUPPORTED, "at most " + std::to_string(kMaxMaps) + " maps per batch");
    MapIO io{};
    for (size_t k = 0; k < b.plans.size(); ++k) {
        io.in[k] = in[k];
        io.out[k] = out[k];
    }
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, b.d_counter);
    // the tiles of vector-form plans, then those of matrix-form plans (queue 2)
    const int ncm = (int)b.cmap.size() - b.ncirc_valu;
    if (b.ncirc_valu > 0 && (parts & ARKCOS_PART_CIRCULANT))
        hipLaunchKernelGGL(k_circ, dim3(b.grid_circ), dim3(kThreads), circ_lds(), s,
                           (const DevPlanView *)b.d_views, (const int2 *)b.d_cmap, b.ncirc_valu,
                           io, 1, circ_buf_floats(), b.d_counter);
    if (ncm > 0 && (parts & ARKCOS_PART_CIRCULANT))
        hipLaunchKernelGGL(k_circ_mfma, dim3(b.grid_circ_mfma), dim3(kThreads), circ_lds(), s,
                           (const DevPlanView *)b.d_views, (const int2 *)b.d_cmap + b.ncirc_valu,
                           ncm, io, 1, circ_buf_floats(), b.d_counter + 2);
    if (!b.gmap.empty() && (parts & ARKCOS_PART_GENERAL))
        hipLaunchKernelGGL(k_general, dim3(b.grid_gen), dim3(kGenThreads), gen_lds(b.max_ntab), s,
                           (const DevPlanView *)b.d_views, (const int2 *)b.d_gmap,
                           (int)b.gmap.size(), io, 1, gen_tab_floats(b.max_ntab), b.d_counter + 1);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

}  // namespace arkcos
