// gfx950 kernels of the real-space convolution (Sutter, Wandelt & Elsner 2012,
// Sec. 2: the real-space part of the split kernel applied by direct summation
// on the GPU; Sec. 3: radial kernel interpolated from a node table).
//
// Every output ring is gathered by one of two kernels, which write disjoint
// rings:
//
//  * k_circ (circulant rings: belt rings whose whole disc lies in the belt).
//    All their source rings have 4N pixels, so the weight of (r, j; s, j')
//    depends on j' - j only.  Each (r, s) has one weight row, evaluated once
//    per node table by k_build_weights with exactly the per-pair arithmetic.
//    The gather is then a correlation: a workgroup owns kGroupRings
//    consecutive output rings and kCircSeg pixels of each, stages one source
//    row at a time in LDS, and every LDS read feeds kGroupRings FMAs whose
//    weights are wave-uniform scalar operands.
//
//  * k_general (polar caps and belt rings whose disc reaches a cap).  Weights
//    are evaluated per pair from exact ring-pair constants: chord from
//    d^2 = A + B sin^2(dphi/2), angle by series, node table in LDS with
//    linear interpolation.  A quarter turn maps pixel j of a ring to
//    j + n/4 and the N-S mirror maps ring i to ring 4N - i, so one weight
//    serves eight pairs; source rows are staged in LDS as [pixel][8 images].
//
// Sums are FP32 within a source-ring row and FP64 across rows.  No atomics
// touch the outputs: results are bitwise reproducible.  This is a gather with
// a per-pair kernel evaluation, so it runs on the vector ALUs, not on matrix
// cores.
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
// sin(x) by its Taylor series: LONG through x^13 for |x| <= 2 (truncation
// below 2e-8 relative), otherwise through x^7 for |x| <= 0.35 (below 1e-9).
template <bool LONG>
__device__ __forceinline__ float sin_series(float x)
{
    const float x2 = x * x;
    float p;
    if (LONG) {
        p = 1.0f / 6227020800.0f;             // 1/13!
        p = fmaf(p, x2, -1.0f / 39916800.0f); // 1/11!
        p = fmaf(p, x2, 1.0f / 362880.0f);    // 1/9!
        p = fmaf(p, x2, -1.0f / 5040.0f);     // 1/7!
    } else {
        p = -1.0f / 5040.0f;
    }
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

// Interpolated, Omega-scaled weight of one pair (0 at or beyond theta_cut).
// Branch-free: the node index is clamped into the table and the weight masked.
template <bool LONG, int AM>
__device__ __forceinline__ float pair_weight_t(const DevPair &pp, const float *tab, float inv_h,
                                               float u_max, int m)
{
    const float x = (float)m * pp.xscale;          // half the longitude difference
    const float sx = sin_series<LONG>(x);
    const float d2 = fmaf(pp.B, sx * sx, pp.A);      // squared chord
    const float u = theta_of<AM>(d2) * inv_h;
    const float uc = fminf(u, u_max);
    const int node = min((int)uc, (int)u_max - 1);
    const float frac = uc - (float)node;
    const float k0 = tab[node];
    const float k1 = tab[node + 1];
    const float w = fmaf(frac, k1 - k0, k0);
    return (u < u_max) ? w : 0.0f;
}

// The same weight with the series chosen at run time from the pair and plan.
__device__ __forceinline__ float pair_weight(const DevPlanView &P, const DevPair &pp,
                                             const float *tab, int m)
{
    const bool lg = (pp.mode & kPairLongSin) != 0;
    switch (P.angle_mode) {
        case 0: return lg ? pair_weight_t<true, 0>(pp, tab, P.inv_h, P.u_max, m)
                          : pair_weight_t<false, 0>(pp, tab, P.inv_h, P.u_max, m);
        case 1: return lg ? pair_weight_t<true, 1>(pp, tab, P.inv_h, P.u_max, m)
                          : pair_weight_t<false, 1>(pp, tab, P.inv_h, P.u_max, m);
        default: return lg ? pair_weight_t<true, 2>(pp, tab, P.inv_h, P.u_max, m)
                           : pair_weight_t<false, 2>(pp, tab, P.inv_h, P.u_max, m);
    }
}

__device__ __forceinline__ int wrap_index(int jq, int n)
{
    jq = (jq < 0) ? jq + n : jq;
    return (jq >= n) ? jq - n : jq;
}

// j mod n for -n <= j < 3n.
__device__ __forceinline__ int wrap3(int j, int n)
{
    j = (j < 0) ? j + n : j;
    j = (j >= n) ? j - n : j;
    return (j >= n) ? j - n : j;
}

// Exact longitude numerator m = (2j + 2o_r) n_s - (2j' + 2o_s) n_r; the
// product terms may exceed 2^31 but the difference does not, so unsigned
// wrap-around arithmetic gives it exactly.
__device__ __forceinline__ int lon_numerator(unsigned mbase, int jq, int two_o_s, int n_r)
{
    return (int)(mbase - (unsigned)(2 * jq + two_o_s) * (unsigned)n_r);
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
// Weight rows of the circulant groups, one workgroup per row: tap k of ring r
// is the per-pair weight at the exact longitude numerator
// m = n (2o_r - 2o_s - 2k), zero where k is outside the (r, s) window.
__global__ __launch_bounds__(kThreads) void k_build_weights(DevPlanView P)
{
    const int row = blockIdx.x;
    if (row >= P.nrows) return;
    const DevRow W = P.rows[row];
    const DevGroup G = P.groups[W.g];
    const int n = P.rings[G.r0].n;
    const int two_o_s = P.rings[W.s].two_o;
    for (int e = threadIdx.x; e < W.ntaps * kGroupRings; e += blockDim.x) {
        const int t = e / kGroupRings;
        const int i = e - t * kGroupRings;
        const int k = W.k_lo + t;
        float w = 0.0f;
        if (i < G.nr) {
            const DevRing R = P.rings[G.r0 + i];
            const int kk = R.pair_begin + (W.s - P.pairs[R.pair_begin].s);
            if (kk >= R.pair_begin && kk < R.pair_end) {
                const DevPair pp = P.pairs[kk];
                int lo, hi;
                pair_window(pp, n, 0, lo, hi);
                if (k >= lo && k <= hi)
                    w = pair_weight(P, pp, P.table, n * (R.two_o - two_o_s - 2 * k));
            }
        }
        P.wts[W.w_off + e] = w;
    }
}

// Source pixels each lane prefetches per row: a row spans at most
// kCircSeg + kCircMaxTaps - 1 pixels.
constexpr int kStageRegs = (kCircSeg + kCircMaxTaps + kThreads - 1) / kThreads;

// Issue the global loads of one staged row (pixels base .. base+nstage-1 of a
// ring of n pixels, wrapped) into registers.
__device__ __forceinline__ void prefetch_row(const float *src, int base, int nstage, int n,
                                             float v[kStageRegs])
{
#pragma unroll
    for (int u = 0; u < kStageRegs; ++u) {
        const int e = threadIdx.x + u * kThreads;
        v[u] = (e < nstage) ? src[wrap_index(base + e, n)] : 0.0f;
    }
}

// Persistent circulant gather over tiles (plan, group, segment) x maps.  Rows
// are double-buffered: the loads of row t+1 are in flight while row t is
// multiplied, and one barrier per row separates the buffers.
__global__ __launch_bounds__(kThreads) void k_circ(const DevPlanView *__restrict__ views,
                                                   const int2 *__restrict__ tile_map,
                                                   int ntiles, MapIO io, int nmaps,
                                                   int buf_floats, unsigned int *counter)
{
    extern __shared__ __align__(16) float xs[];
    __shared__ int s_item;
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
        double acc[kGroupRings][kCircPix];
#pragma unroll
        for (int r = 0; r < kGroupRings; ++r)
#pragma unroll
            for (int i = 0; i < kCircPix; ++i) acc[r][i] = 0.0;
        float v[kStageRegs];
        {
            const DevRow W = cst(P.rows)[G.row_begin];
            prefetch_row(in + cst(P.rings)[W.s].first, T.j0 + W.k_lo, T.len + W.ntaps - 1, n, v);
        }
        int buf = 0;
        for (int row = G.row_begin; row < G.row_end; ++row) {
            const DevRow W = cst(P.rows)[row];
            float *xb = xs + buf * buf_floats;
#pragma unroll
            for (int u = 0; u < kStageRegs; ++u) xb[threadIdx.x + u * kThreads] = v[u];
            __syncthreads();
            if (row + 1 < G.row_end) {
                const DevRow W1 = cst(P.rows)[row + 1];
                prefetch_row(in + cst(P.rings)[W1.s].first, T.j0 + W1.k_lo,
                             T.len + W1.ntaps - 1, n, v);
            }
            float racc[kGroupRings][kCircPix];
#pragma unroll
            for (int r = 0; r < kGroupRings; ++r)
#pragma unroll
                for (int i = 0; i < kCircPix; ++i) racc[r][i] = 0.0f;
            cptr<float> w = cst(P.wts + W.w_off);
            const float *x0 = xb + threadIdx.x;
#pragma unroll 2
            for (int t = 0; t < W.ntaps; ++t) {
                float wr[kGroupRings];
#pragma unroll
                for (int r = 0; r < kGroupRings; ++r) wr[r] = w[t * kGroupRings + r];
#pragma unroll
                for (int i = 0; i < kCircPix; ++i) {
                    const float x = x0[i * kThreads + t];
#pragma unroll
                    for (int r = 0; r < kGroupRings; ++r) racc[r][i] = fmaf(wr[r], x, racc[r][i]);
                }
            }
#pragma unroll
            for (int r = 0; r < kGroupRings; ++r)
#pragma unroll
                for (int i = 0; i < kCircPix; ++i) acc[r][i] += (double)racc[r][i];
            buf ^= 1;
        }
        float *out = io.out[pi] + (size_t)map * P.npix;
#pragma unroll
        for (int r = 0; r < kGroupRings; ++r) {
            if (r >= G.nr) break;
            float *o = out + cst(P.rings)[G.r0 + r].first + T.j0;
#pragma unroll
            for (int i = 0; i < kCircPix; ++i) {
                const int jj = threadIdx.x + i * kThreads;
                if (jj < T.len) o[jj] = (float)acc[r][i];
            }
        }
    }
}

// --------------------------------------------------------- general gather --
// Source pixels each lane prefetches per staged chunk.
constexpr int kGenRegs = (kGenChunk + kThreads - 1) / kThreads;

// One staged chunk of one source row of a general tile: row k of the output
// ring's pair list, unwrapped source pixels c0 .. c0+cn-1.
struct GenChunk {
    int k;
    int c0;
    int cn;
};

// Window bounds of a tile's first and last pixel on the row of pair pp.
__device__ __forceinline__ void tile_window(const DevPair &pp, int n_s, const DevTile &T,
                                            int &lo_min, int &hi_max)
{
    int dummy;
    pair_window(pp, n_s, T.j0, lo_min, dummy);
    pair_window(pp, n_s, T.j0 + T.len - 1, dummy, hi_max);
}

// Issue the loads of the 8 images of a chunk: the four quarter turns of ring s
// and of its mirror ring.
__device__ __forceinline__ void prefetch_chunk(const float *src, const float *srcm, bool mirror,
                                               int n_s, int c0, int cn, float4 a[kGenRegs],
                                               float4 b[kGenRegs])
{
    const int qs = n_s >> 2;
#pragma unroll
    for (int u = 0; u < kGenRegs; ++u) {
        const int e = threadIdx.x + u * kThreads;
        a[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        b[u] = a[u];
        if (e < cn) {
            const int i0 = wrap3(c0 + e, n_s);
            const int i1 = wrap3(c0 + e + qs, n_s);
            const int i2 = wrap3(c0 + e + 2 * qs, n_s);
            const int i3 = wrap3(c0 + e + 3 * qs, n_s);
            a[u] = make_float4(src[i0], src[i1], src[i2], src[i3]);
            if (mirror) b[u] = make_float4(srcm[i0], srcm[i1], srcm[i2], srcm[i3]);
        }
    }
}

// Accumulate the candidates a0..a1 of one lane from the staged chunk.
template <bool LONG, int AM>
__device__ __forceinline__ void gen_candidates(const DevPair &pp, const float *tab, float inv_h,
                                               float u_max, unsigned mbase, int two_o_s, int n_r,
                                               const float4 *stage, int c0, int a0, int a1,
                                               float row[8])
{
    for (int jq = a0; jq <= a1; ++jq) {
        const float w = pair_weight_t<LONG, AM>(pp, tab, inv_h, u_max,
                                                lon_numerator(mbase, jq, two_o_s, n_r));
        const float4 v0 = stage[2 * (jq - c0)];
        const float4 v1 = stage[2 * (jq - c0) + 1];
        row[0] = fmaf(w, v0.x, row[0]);
        row[1] = fmaf(w, v0.y, row[1]);
        row[2] = fmaf(w, v0.z, row[2]);
        row[3] = fmaf(w, v0.w, row[3]);
        row[4] = fmaf(w, v1.x, row[4]);
        row[5] = fmaf(w, v1.y, row[5]);
        row[6] = fmaf(w, v1.z, row[6]);
        row[7] = fmaf(w, v1.w, row[7]);
    }
}

// Persistent general gather over tiles (plan, north ring, quadrant segment) x
// maps.  LDS: the node table of the current plan, then one staged chunk as
// [pixel][8] = 4 quarter-turn images of ring s, then 4 of its mirror.  The
// loads of the next chunk are in flight while the current one is multiplied.
__global__ __launch_bounds__(kThreads) void k_general(const DevPlanView *__restrict__ views,
                                                      const int2 *__restrict__ tile_map,
                                                      int ntiles, MapIO io, int nmaps,
                                                      int tab_floats, unsigned int *counter)
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
            cur = pi;
        }
        const DevTile T = cst(P.gtiles)[lt];
        const int rn = T.r;
        const int rs = P.nrings - 1 - rn;           // mirror ring
        const bool mirror = rs != rn;
        const DevRing R = cst(P.rings)[rn];
        const int qr = R.n >> 2;
        const bool active = (int)threadIdx.x < T.len;
        const int j = T.j0 + min((int)threadIdx.x, T.len - 1);
        const float *in = io.in[pi] + (size_t)map * P.npix;

        // first chunk of the first row
        GenChunk ch;
        ch.k = R.pair_begin;
        {
            const DevPair pp = cst(P.pairs)[ch.k];
            int hi_max;
            tile_window(pp, cst(P.rings)[pp.s].n, T, ch.c0, hi_max);
            ch.cn = min(kGenChunk, hi_max - ch.c0 + 1);
        }
        float4 pa[kGenRegs], pb[kGenRegs];
        {
            const DevPair pp = cst(P.pairs)[ch.k];
            const DevRing S = cst(P.rings)[pp.s];
            prefetch_chunk(in + S.first, in + cst(P.rings)[P.nrings - 1 - pp.s].first, mirror,
                           S.n, ch.c0, ch.cn, pa, pb);
        }
        double acc[8];
        float row[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc[q] = 0.0;
            row[q] = 0.0f;
        }
        while (ch.k < R.pair_end) {
            __syncthreads();      // the previous chunk is no longer read
#pragma unroll
            for (int u = 0; u < kGenRegs; ++u) {
                const int e = threadIdx.x + u * kThreads;
                if (e < kGenChunk) {
                    stage[2 * e] = pa[u];
                    stage[2 * e + 1] = pb[u];
                }
            }
            __syncthreads();
            const DevPair pp = cst(P.pairs)[ch.k];
            const DevRing S = cst(P.rings)[pp.s];
            // the next chunk: the rest of this row, else the next row
            GenChunk nx;
            int lo_min, hi_max;
            tile_window(pp, S.n, T, lo_min, hi_max);
            if (ch.c0 + kGenChunk <= hi_max) {
                nx.k = ch.k;
                nx.c0 = ch.c0 + kGenChunk;
                nx.cn = min(kGenChunk, hi_max - nx.c0 + 1);
            } else {
                nx.k = ch.k + 1;
                nx.c0 = 0;
                nx.cn = 0;
                if (nx.k < R.pair_end) {
                    const DevPair pn = cst(P.pairs)[nx.k];
                    int lo2, hi2;
                    tile_window(pn, cst(P.rings)[pn.s].n, T, lo2, hi2);
                    nx.c0 = lo2;
                    nx.cn = min(kGenChunk, hi2 - lo2 + 1);
                }
            }
            if (nx.k < R.pair_end) {
                const DevPair pn = cst(P.pairs)[nx.k];
                const DevRing Sn = cst(P.rings)[pn.s];
                prefetch_chunk(in + Sn.first, in + cst(P.rings)[P.nrings - 1 - pn.s].first, mirror,
                               Sn.n, nx.c0, nx.cn, pa, pb);
            }
            // this lane's candidates inside the chunk
            int lo, hi;
            pair_window(pp, S.n, j, lo, hi);
            const int a0 = max(lo, ch.c0);
            const int a1 = min(hi, ch.c0 + ch.cn - 1);
            const unsigned mbase = (unsigned)(2 * j + R.two_o) * (unsigned)S.n;
            const bool lg = (pp.mode & kPairLongSin) != 0;
            switch (P.angle_mode * 2 + (lg ? 1 : 0)) {
                case 0: gen_candidates<false, 0>(pp, tab, P.inv_h, P.u_max, mbase, S.two_o, R.n, stage, ch.c0, a0, a1, row); break;
                case 1: gen_candidates<true, 0>(pp, tab, P.inv_h, P.u_max, mbase, S.two_o, R.n, stage, ch.c0, a0, a1, row); break;
                case 2: gen_candidates<false, 1>(pp, tab, P.inv_h, P.u_max, mbase, S.two_o, R.n, stage, ch.c0, a0, a1, row); break;
                case 3: gen_candidates<true, 1>(pp, tab, P.inv_h, P.u_max, mbase, S.two_o, R.n, stage, ch.c0, a0, a1, row); break;
                case 4: gen_candidates<false, 2>(pp, tab, P.inv_h, P.u_max, mbase, S.two_o, R.n, stage, ch.c0, a0, a1, row); break;
                default: gen_candidates<true, 2>(pp, tab, P.inv_h, P.u_max, mbase, S.two_o, R.n, stage, ch.c0, a0, a1, row); break;
            }
            if (nx.k != ch.k) {   // row complete: FP32 row sums into the FP64 totals
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    acc[q] += (double)row[q];
                    row[q] = 0.0f;
                }
            }
            ch = nx;
        }
        if (active) {
            float *out = io.out[pi] + (size_t)map * P.npix;
            float *o = out + R.first + j;
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q * qr] = (float)acc[q];
            if (mirror) {
                float *om = out + cst(P.rings)[rs].first + j;
#pragma unroll
                for (int q = 0; q < 4; ++q) om[q * qr] = (float)acc[4 + q];
            }
        }
    }
}

__global__ void k_reset_counters(unsigned int *counter)
{
    if (threadIdx.x < 2) counter[threadIdx.x] = 0u;
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

// sin(x) in FP64: through x^15 for |x| <= 0.35, through x^25 for |x| <= 2
// (truncation below 1e-19 relative).
template <bool LONG>
__device__ __forceinline__ double sin_d(double x)
{
    constexpr int K = LONG ? 12 : 7;
    const double x2 = x * x;
    double p = sin_coef(K);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) p = fma(p, x2, sin_coef(k));
    return x * p;
}

// asin(y) in FP64 for 0 <= y <= 0.5 (truncation below 1e-16 relative).
__device__ __forceinline__ double asin_d(double y)
{
    constexpr int K = 24;
    const double z = y * y;
    double p = asin_coef(K);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) p = fma(p, z, asin_coef(k));
    return y * p;
}

// theta = 2 asin(d/2) in FP64 from the squared chord, in the same three
// regimes as theta_of: d (sum_k c_k (d^2/4)^k) with 8 terms for d <= 0.1 and
// 16 terms for d^2 <= 0.245, and the full-range asin otherwise.
template <int AM>
__device__ __forceinline__ double theta_d(double d2)
{
    if (AM == 2) {
        const double y = fmin(0.5 * sqrt(d2), 1.0);
        if (y <= 0.5) return 2.0 * asin_d(y);
        return 2.0 * (1.5707963267948966192 - 2.0 * asin_d(sqrt(0.5 * (1.0 - y))));
    }
    constexpr int K = AM == 0 ? 8 : 16;
    const double z = 0.25 * d2;
    double p = asin_coef(K);
#pragma unroll
    for (int k = K - 1; k >= 0; --k) p = fma(p, z, asin_coef(k));
    return sqrt(d2) * p;
}

// Node index and fraction of one pair from the FP64 chord constants; false at
// or beyond the cut.  (The knot gradient needs the fraction to ~1e-9: the hat
// basis has slope 1/h in theta.)
template <bool LONG, int AM>
__device__ __forceinline__ bool pair_node_d(const DevPairD &pd, double inv_h, double u_max, int m,
                                            int &node, double &frac)
{
    const double sx = sin_d<LONG>((double)m * pd.xscale);
    const double u = theta_d<AM>(fma(pd.B, sx * sx, pd.A)) * inv_h;
    node = (int)fmin(u, u_max - 1.0);
    frac = u - (double)node;
    return u < u_max;
}

// Scatter the candidates a0..a1 of one lane into the knot histogram: each
// candidate's node and fraction serve the 8 images, whose products g x are
// summed first.
template <bool LONG, int AM>
__device__ __forceinline__ void knot_candidates(const DevPairD &pd, double inv_h, double u_max,
                                                unsigned mbase, int two_o_s, int n_r,
                                                const float4 *stage, int c0, int a0, int a1,
                                                const float gv[8], double *hist)
{
    for (int jq = a0; jq <= a1; ++jq) {
        int node;
        double frac;
        const bool in = pair_node_d<LONG, AM>(pd, inv_h, u_max,
                                               lon_numerator(mbase, jq, two_o_s, n_r), node, frac);
        const float4 v0 = stage[2 * (jq - c0)];
        const float4 v1 = stage[2 * (jq - c0) + 1];
        float c = gv[0] * v0.x;
        c = fmaf(gv[1], v0.y, c);
        c = fmaf(gv[2], v0.z, c);
        c = fmaf(gv[3], v0.w, c);
        c = fmaf(gv[4], v1.x, c);
        c = fmaf(gv[5], v1.y, c);
        c = fmaf(gv[6], v1.z, c);
        c = fmaf(gv[7], v1.w, c);
        if (in && c != 0.0f) {
            atomicAdd(&hist[node], (1.0 - frac) * (double)c);
            atomicAdd(&hist[node + 1], frac * (double)c);
        }
    }
}

// Knot gradient sum_p g[p] sum_q hat_k(theta_pq) x[q] over all pairs of all
// maps.  Tiles cover the first quadrant of every northern ring; a lane holds
// g at the 8 images of its pixel, and the source row is staged as in
// k_general.  Per-workgroup FP64 LDS histograms are written to
// partials[block][ntab] and reduced in a fixed order by k_knot_reduce.
__global__ __launch_bounds__(kThreads) void k_knot(const DevPlanView *__restrict__ views,
                                                   const float *__restrict__ g,
                                                   const float *__restrict__ x, int nmaps,
                                                   unsigned int *counter,
                                                   double *__restrict__ partials)
{
    // 16-byte aligned dynamic LDS: 64-bit LDS atomics need natural alignment.
    extern __shared__ __align__(16) double hist[];
    __shared__ int s_item;
    const DevPlanView P = cst(views)[0];
    float4 *stage = reinterpret_cast<float4 *>(hist + ((P.ntab + 1) & ~1));
    for (int i = threadIdx.x; i < P.ntab; i += blockDim.x) hist[i] = 0.0;
    const double u_max = (double)(P.ntab - 1);
    const int nitems = P.nktiles * nmaps;
    for (;;) {
        const int item = next_item(counter, &s_item);
        if (item >= nitems) break;
        const int ti = item / nmaps;
        const int map = item - ti * nmaps;
        const DevTile T = cst(P.ktiles)[ti];
        const int rn = T.r;
        const int rs = P.nrings - 1 - rn;
        const bool mirror = rs != rn;
        const DevRing R = cst(P.rings)[rn];
        const int qr = R.n >> 2;
        const bool active = (int)threadIdx.x < T.len;
        const int j = T.j0 + min((int)threadIdx.x, T.len - 1);
        const float *in = x + (size_t)map * P.npix;
        const float *gm = g + (size_t)map * P.npix;
        float gv[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            gv[q] = active ? gm[R.first + j + q * qr] : 0.0f;
            gv[4 + q] = (active && mirror) ? gm[cst(P.rings)[rs].first + j + q * qr] : 0.0f;
        }
        for (int k = R.pair_begin; k < R.pair_end; ++k) {
            const DevPair pp = cst(P.pairs)[k];
            const DevPairD pd = cst(P.pairs_d)[k];
            const DevRing S = cst(P.rings)[pp.s];
            const float *src = in + S.first;
            const float *srcm = in + cst(P.rings)[P.nrings - 1 - pp.s].first;
            int lo_min, hi_max, lo, hi;
            tile_window(pp, S.n, T, lo_min, hi_max);
            pair_window(pp, S.n, j, lo, hi);
            const unsigned mbase = (unsigned)(2 * j + R.two_o) * (unsigned)S.n;
            const bool lg = (pp.mode & kPairLongSin) != 0;
            for (int c0 = lo_min; c0 <= hi_max; c0 += kGenChunk) {
                const int cn = min(kGenChunk, hi_max - c0 + 1);
                float4 pa[kGenRegs], pb[kGenRegs];
                prefetch_chunk(src, srcm, mirror, S.n, c0, cn, pa, pb);
                __syncthreads();
#pragma unroll
                for (int u = 0; u < kGenRegs; ++u) {
                    const int e = threadIdx.x + u * kThreads;
                    if (e < kGenChunk) {
                        stage[2 * e] = pa[u];
                        stage[2 * e + 1] = pb[u];
                    }
                }
                __syncthreads();
                const int a0 = max(lo, c0);
                const int a1 = min(hi, c0 + cn - 1);
                switch (P.angle_mode * 2 + (lg ? 1 : 0)) {
                    case 0: knot_candidates<false, 0>(pd, P.inv_h_d, u_max, mbase, S.two_o, R.n, stage, c0, a0, a1, gv, hist); break;
                    case 1: knot_candidates<true, 0>(pd, P.inv_h_d, u_max, mbase, S.two_o, R.n, stage, c0, a0, a1, gv, hist); break;
                    case 2: knot_candidates<false, 1>(pd, P.inv_h_d, u_max, mbase, S.two_o, R.n, stage, c0, a0, a1, gv, hist); break;
                    case 3: knot_candidates<true, 1>(pd, P.inv_h_d, u_max, mbase, S.two_o, R.n, stage, c0, a0, a1, gv, hist); break;
                    case 4: knot_candidates<false, 2>(pd, P.inv_h_d, u_max, mbase, S.two_o, R.n, stage, c0, a0, a1, gv, hist); break;
                    default: knot_candidates<true, 2>(pd, P.inv_h_d, u_max, mbase, S.two_o, R.n, stage, c0, a0, a1, gv, hist); break;
                }
            }
        }
    }
    __syncthreads();
    double *dst = partials + (size_t)blockIdx.x * P.ntab;
    for (int i = threadIdx.x; i < P.ntab; i += blockDim.x) dst[i] = hist[i];
}

// Fixed-order reduction of the per-workgroup partials, scaled by Omega.
__global__ void k_knot_reduce(const double *__restrict__ partials, int nblocks, int ntab,
                              double omega, float *__restrict__ gk)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ntab) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partials[(size_t)b * ntab + k];
    gk[k] = (float)(omega * s);
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
static int occupancy(K kernel, size_t lds, int *per_cu)
{
    ARKCOS_HIP_CHECK(hipFuncSetAttribute((const void *)kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ARKCOS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, kThreads, lds));
    if (*per_cu < 1)
        return fail(ARKCOS_EUNSUPPORTED, "kernel cannot be resident with " +
                                             std::to_string(lds) + " bytes of LDS");
    return ARKCOS_OK;
}

// Two row buffers of kStageRegs * kThreads floats each.
static int circ_buf_floats() { return kStageRegs * kThreads; }
static size_t circ_lds() { return (size_t)2 * circ_buf_floats() * sizeof(float); }
static int gen_tab_floats(int ntab) { return hist_offset_floats(ntab); }
static size_t gen_lds(int ntab)
{
    return (size_t)(gen_tab_floats(ntab) + 8 * kGenChunk) * sizeof(float);
}
static size_t knot_lds(int ntab)
{
    return (size_t)((ntab + 1) & ~1) * sizeof(double) + (size_t)8 * kGenChunk * sizeof(float);
}



int prepare_launches(Plan &p)
{
    ARKCOS_HIP_CHECK(hipDeviceGetAttribute(&p.cus, hipDeviceAttributeMultiprocessorCount,
                                           p.device));
    int rc;
    if ((rc = occupancy(k_circ, circ_lds(), &p.occ_circ))) return rc;
    if ((rc = occupancy(k_general, gen_lds(p.desc.ntab), &p.occ_gen))) return rc;
    int most = 1;
    if ((p.desc.flags & ARKCOS_PLAN_LEARNABLE) && p.desc.ntab <= ARKCOS_MAX_GRAD_NTAB) {
        if ((rc = occupancy(k_knot, knot_lds(p.desc.ntab), &p.occ_knot))) return rc;
        most = p.occ_knot;
    }
    p.grid = most * p.cus;  // rows of the knot-gradient partials
    return ARKCOS_OK;
}

int prepare_batch(Batch &b)
{
    ARKCOS_HIP_CHECK(hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount,
                                           b.device));
    int occ_c = 0, occ_g = 0, rc;
    if ((rc = occupancy(k_circ, circ_lds(), &occ_c))) return rc;
    if ((rc = occupancy(k_general, gen_lds(b.max_ntab), &occ_g))) return rc;
    b.grid_circ = std::max(1, std::min((int)b.cmap.size(), occ_c * b.cus));
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
                   int parts)
{
    MapIO io{};
    io.in[0] = in;
    io.out[0] = out;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, p.d_counter);
    const int nct = (parts & ARKCOS_PART_CIRCULANT) ? (int)p.ctiles.size() : 0;
    const int ngt = (parts & ARKCOS_PART_GENERAL) ? (int)p.gtiles.size() : 0;
    if (nct > 0) {
        const int grid = std::max(1, std::min(nct * nbatch, p.occ_circ * p.cus));
        hipLaunchKernelGGL(k_circ, dim3(grid), dim3(kThreads), circ_lds(), s,
                           (const DevPlanView *)p.d_view, (const int2 *)nullptr, nct, io, nbatch,
                           circ_buf_floats(), p.d_counter);
    }
    if (ngt > 0) {
        const int grid = std::max(1, std::min(ngt * nbatch, p.occ_gen * p.cus));
        hipLaunchKernelGGL(k_general, dim3(grid), dim3(kThreads), gen_lds(p.desc.ntab), s,
                           (const DevPlanView *)p.d_view, (const int2 *)nullptr, ngt, io, nbatch,
                           gen_tab_floats(p.desc.ntab), p.d_counter + 1);
    }
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

static int launch_knot(const Plan &p, const float *g, const float *x, float *gk, int nbatch,
                       hipStream_t s)
{
    const int ntab = p.desc.ntab;
    const int items = (int)p.ktiles.size() * nbatch;
    const int grid = std::max(1, std::min({items, p.occ_knot * p.cus, p.grid}));
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, p.d_counter + 2);
    hipLaunchKernelGGL(k_knot, dim3(grid), dim3(kThreads), knot_lds(ntab), s,
                       (const DevPlanView *)p.d_view, g, x, nbatch, p.d_counter + 2, p.d_kpart);
    ARKCOS_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_knot_reduce, dim3((ntab + 255) / 256), dim3(256), 0, s, p.d_kpart, grid,
                       ntab, p.omega, gk);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

int launch_backward(const Plan &p, const float *g, const float *x, float *gx, float *gk,
                    int nbatch, hipStream_t s)
{
    // The operator is symmetric, so d/dmap is the same gather applied to g.
    if (gx) {
        int rc = launch_forward(p, g, gx, nbatch, s);
        if (rc) return rc;
    }
    if (gk) return launch_knot(p, g, x, gk, nbatch, s);
    return ARKCOS_OK;
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
    if (!b.cmap.empty() && (parts & ARKCOS_PART_CIRCULANT))
        hipLaunchKernelGGL(k_circ, dim3(b.grid_circ), dim3(kThreads), circ_lds(), s,
                           (const DevPlanView *)b.d_views, (const int2 *)b.d_cmap,
                           (int)b.cmap.size(), io, 1, circ_buf_floats(), b.d_counter);
    if (!b.gmap.empty() && (parts & ARKCOS_PART_GENERAL))
        hipLaunchKernelGGL(k_general, dim3(b.grid_gen), dim3(kThreads), gen_lds(b.max_ntab), s,
                           (const DevPlanView *)b.d_views, (const int2 *)b.d_gmap,
                           (int)b.gmap.size(), io, 1, gen_tab_floats(b.max_ntab), b.d_counter + 1);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

}  // namespace arkcos
