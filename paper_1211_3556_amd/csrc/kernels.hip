// gfx950 kernels of the real-space convolution (Sutter, Wandelt & Elsner 2012,
// Sec. 2: the real-space part of the split kernel applied by direct summation
// on the GPU; Sec. 3: radial kernel interpolated from a node table).
//
// Work decomposition: a tile is a run of consecutive pixels of one output
// ring.  Persistent workgroups pull tiles from a queue (longest first), keep
// the node table in LDS and give each lane one output pixel; the lane walks
// the source rings of its ring and the longitude window on each, computes the
// chord from small, exactly known ring-pair constants, converts it to an
// angle, interpolates the table and accumulates (FP32 per source-ring row,
// FP64 across rows).  One weight serves
// every map of the batch.  This is a gather with a per-pair kernel
// evaluation, so it runs on the vector ALUs, not on matrix cores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "arkcos_internal.hpp"

namespace arkcos {

constexpr int kThreads = 256;
constexpr int kMaxBatchMaps = 32;

// ------------------------------------------------------------ FP32 math --
// sin(x) for |x| <= 2 by its Taylor series through x^13 (truncation below
// 2e-8 relative on that range).
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

// theta = 2 asin(d/2) from the squared chord d^2 <= 0.245 (theta <= 0.5 rad):
// theta = d (1 + d^2/24 + 3 d^4/640 + 5 d^6/7168 + 35 d^8/294912
//            + 63 d^10/2883584), truncation below 1e-9 relative.
__device__ __forceinline__ float theta_small(float d2)
{
    const float d = sqrtf(d2);
    float p = 63.0f / 2883584.0f;
    p = fmaf(p, d2, 35.0f / 294912.0f);
    p = fmaf(p, d2, 5.0f / 7168.0f);
    p = fmaf(p, d2, 3.0f / 640.0f);
    p = fmaf(p, d2, 1.0f / 24.0f);
    p = fmaf(p, d2, 1.0f);
    return d * p;
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

// theta = 2 asin(d/2) for any chord 0 <= d <= 2; above y = 1/2 the half-angle
// identity asin(y) = pi/2 - 2 asin(sqrt((1 - y)/2)) keeps the series argument
// below 1/2.
__device__ __forceinline__ float theta_large(float d2)
{
    const float y = fminf(0.5f * sqrtf(d2), 1.0f);
    if (y <= 0.5f) return 2.0f * asin_series(y);
    const float w = sqrtf(0.5f * (1.0f - y));
    return 2.0f * (1.5707963267948966f - 2.0f * asin_series(w));
}

// Interpolated, Omega-scaled weight of one pair (0 at or beyond theta_cut).
// Also returns the node index and fraction for the knot gradient.
__device__ __forceinline__ float pair_weight(const DevPlanView &P, const DevPair &pp,
                                             const float *tab, int m, int &node, float &frac,
                                             bool &inside)
{
    const float x = (float)m * pp.xscale;          // half the longitude difference
    const float sx = sin_series(x);
    const float d2 = fmaf(pp.B, sx * sx, pp.A);      // squared chord
    const float th = P.large_angle ? theta_large(d2) : theta_small(d2);
    const float u = th * P.inv_h;
    inside = u < P.u_max;
    const float uc = inside ? u : 0.0f;
    node = (int)uc;
    frac = uc - (float)node;
    const float k0 = tab[node];
    const float k1 = tab[node + 1];
    return inside ? fmaf(frac, k1 - k0, k0) : 0.0f;
}

// Node index and fraction of one pair from FP64 geometry (same chord, angle
// and table coordinate as pair_weight, through the device math library).
// Returns false at or beyond the cut.
__device__ __forceinline__ bool pair_node_fp64(const DevPlanView &P, const DevPairD &pd, int m,
                                               int &node, double &frac)
{
    const double sx = sin((double)m * pd.xscale);
    const double d2 = fma(pd.B, sx * sx, pd.A);
    const double th = 2.0 * asin(fmin(1.0, 0.5 * sqrt(d2)));
    const double u = th * P.inv_h_d;
    if (!(u < (double)(P.ntab - 1))) return false;
    node = (int)u;
    frac = u - (double)node;
    return true;
}

__device__ __forceinline__ int wrap_index(int jq, int n)
{
    jq = (jq < 0) ? jq + n : jq;
    return (jq >= n) ? jq - n : jq;
}

// Exact longitude numerator m = (2j + 2o_r) n_s - (2j' + 2o_s) n_r; the
// product terms may exceed 2^31 but the difference does not, so unsigned
// wrap-around arithmetic gives it exactly.
__device__ __forceinline__ int lon_numerator(unsigned mbase, int jq, int two_o_s, int n_r)
{
    return (int)(mbase - (unsigned)(2 * jq + two_o_s) * (unsigned)n_r);
}

// Offset (in floats) of the knot-gradient histogram after an ntab-entry FP32
// table: rounded up to 16 bytes.
__host__ __device__ constexpr int hist_offset_floats(int ntab) { return (ntab + 3) & ~3; }

// --------------------------------------------------------------- forward --
// Accumulate the outputs of pixel j of ring R for maps map0 .. map0+NB-1.
// Each source-ring row is summed in FP32 (at most a few hundred terms) and
// the row sums in FP64, which keeps the rounding of long sums (wide discs,
// thousands of pairs) well below the FP32 weight error.
template <int NB>
__device__ __forceinline__ void gather_pixel(const DevPlanView &P, const float *tab,
                                             const DevRing &R, int j,
                                             const float *__restrict__ in, int map0,
                                             int nmaps, float out[NB])
{
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    for (int k = R.pair_begin; k < R.pair_end; ++k) {
        const DevPair pp = P.pairs[k];
        const DevRing S = P.rings[pp.s];
        int lo, hi;
        pair_window(pp, S.n, j, lo, hi);
        const unsigned mbase = (unsigned)(2 * j + R.two_o) * (unsigned)S.n;
        float row[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) row[b] = 0.0f;
        for (int jq = lo; jq <= hi; ++jq) {
            int node;
            float frac;
            bool inside;
            const float w = pair_weight(P, pp, tab, lon_numerator(mbase, jq, S.two_o, R.n),
                                        node, frac, inside);
            const size_t q = (size_t)(S.first + wrap_index(jq, S.n));
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < nmaps) row[b] = fmaf(w, in[(size_t)(map0 + b) * P.npix + q], row[b]);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] += (double)row[b];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) out[b] = (float)acc[b];
}

__device__ __forceinline__ void load_table(float *lds, const float *table, int ntab)
{
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) lds[i] = table[i];
}

// Persistent forward kernel: work item = (tile, group of NB maps), tiles in
// the plan's longest-first order.
template <int NB>
__global__ __launch_bounds__(kThreads) void k_forward(DevPlanView P,
                                                      const float *__restrict__ in,
                                                      float *__restrict__ out, int nbatch,
                                                      unsigned int *counter)
{
    extern __shared__ __align__(16) float lds_tab[];
    __shared__ int s_item;
    load_table(lds_tab, P.table, P.ntab);
    const int ngroups = (nbatch + NB - 1) / NB;
    const int nitems = P.ntiles * ngroups;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= nitems) break;
        const int ti = item / ngroups;
        const int map0 = (item - ti * ngroups) * NB;
        const int nmaps = min(NB, nbatch - map0);
        const DevTile T = P.tiles[ti];
        const DevRing R = P.rings[T.r];
        for (int jj = threadIdx.x; jj < T.len; jj += blockDim.x) {
            const int j = T.j0 + jj;
            float acc[NB];
            gather_pixel<NB>(P, lds_tab, R, j, in, map0, nmaps, acc);
            const size_t p = (size_t)(R.first + j);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b < nmaps) out[(size_t)(map0 + b) * P.npix + p] = acc[b];
        }
    }
}

__global__ void k_reset_counter(unsigned int *counter) { counter[0] = 0u; }

// Omega-scaled FP32 table from device knots.
__global__ void k_set_table(float *table, const float *knots, int ntab, float omega)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntab) table[i] = omega * knots[i];
}

// -------------------------------------------------------------- backward --
// Fused adjoint: gx[q'] over the batch (the same gather applied to g, with the
// forward's FP32 weights, so it is the exact transpose of the forward) and the
// knot gradient sum_b g_b[p] x_b[q] hat_k(theta_pq), with node and fraction
// from FP64 geometry, accumulated per workgroup in an FP64 LDS histogram and
// written to partials[block][ntab].
template <int NB, bool WANT_GX, bool WANT_GK>
__global__ __launch_bounds__(kThreads) void k_backward(DevPlanView P,
                                                       const float *__restrict__ g,
                                                       const float *__restrict__ x,
                                                       float *__restrict__ gx, int nbatch,
                                                       unsigned int *counter,
                                                       double *__restrict__ partials)
{
    // The dynamic LDS base is 16-byte aligned and the FP64 histogram starts at
    // a 16-byte boundary after the table: 64-bit LDS atomics need natural
    // alignment.
    extern __shared__ __align__(16) float lds_tab[];
    double *hist = reinterpret_cast<double *>(lds_tab + hist_offset_floats(P.ntab));
    __shared__ int s_item;
    load_table(lds_tab, P.table, P.ntab);
    if (WANT_GK)
        for (int i = threadIdx.x; i < P.ntab; i += blockDim.x) hist[i] = 0.0;
    const int ngroups = (nbatch + NB - 1) / NB;
    const int nitems = P.ntiles * ngroups;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= nitems) break;
        const int ti = item / ngroups;
        const int map0 = (item - ti * ngroups) * NB;
        const int nmaps = min(NB, nbatch - map0);
        const DevTile T = P.tiles[ti];
        const DevRing R = P.rings[T.r];
        for (int jj = threadIdx.x; jj < T.len; jj += blockDim.x) {
            const int j = T.j0 + jj;
            const size_t p = (size_t)(R.first + j);
            float gp[NB];
            double acc[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                acc[b] = 0.0;
                gp[b] = (WANT_GK && b < nmaps) ? g[(size_t)(map0 + b) * P.npix + p] : 0.0f;
            }
            for (int k = R.pair_begin; k < R.pair_end; ++k) {
                const DevPair pp = P.pairs[k];
                const DevRing S = P.rings[pp.s];
                int lo, hi;
                pair_window(pp, S.n, j, lo, hi);
                const unsigned mbase = (unsigned)(2 * j + R.two_o) * (unsigned)S.n;
                DevPairD pd{};
                if (WANT_GK) pd = P.pairs_d[k];
                float row[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) row[b] = 0.0f;
                for (int jq = lo; jq <= hi; ++jq) {
                    int node;
                    float frac;
                    bool inside;
                    const int m = lon_numerator(mbase, jq, S.two_o, R.n);
                    const float w = WANT_GX ? pair_weight(P, pp, lds_tab, m, node, frac, inside)
                                            : 0.0f;
                    const size_t q = (size_t)(S.first + wrap_index(jq, S.n));
                    float c = 0.0f;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (b < nmaps) {
                            const size_t off = (size_t)(map0 + b) * P.npix;
                            if (WANT_GX) row[b] = fmaf(w, g[off + q], row[b]);
                            if (WANT_GK) c = fmaf(gp[b], x[off + q], c);
                        }
                    }
                    if (WANT_GK) {
                        int nd;
                        double fd;
                        if (pair_node_fp64(P, pd, m, nd, fd)) {
                            atomicAdd(&hist[nd], (1.0 - fd) * (double)c);
                            atomicAdd(&hist[nd + 1], fd * (double)c);
                        }
                    }
                }
                if (WANT_GX) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[b] += (double)row[b];
                }
            }
            if (WANT_GX) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (b < nmaps) gx[(size_t)(map0 + b) * P.npix + p] = (float)acc[b];
            }
        }
    }
    if (WANT_GK) {
        __syncthreads();
        double *dst = partials + (size_t)blockIdx.x * P.ntab;
        for (int i = threadIdx.x; i < P.ntab; i += blockDim.x) dst[i] = hist[i];
    }
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

// --------------------------------------------------------------- batched --
struct BatchArgs {
    const float *in[kMaxBatchMaps];
    float *out[kMaxBatchMaps];
};

// One persistent launch over the tiles of several plans (one map each).  A
// workgroup reloads the LDS table only when the plan of its next tile differs.
__global__ __launch_bounds__(kThreads) void k_batch(const DevPlanView *__restrict__ views,
                                                    const int *__restrict__ tile_plan,
                                                    const int *__restrict__ tile_local,
                                                    int ntiles, BatchArgs args,
                                                    unsigned int *counter)
{
    extern __shared__ __align__(16) float lds_tab[];
    __shared__ int s_item;
    int cur = -1;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= ntiles) break;
        const int pi = tile_plan[item];
        const DevPlanView P = views[pi];
        if (pi != cur) {
            load_table(lds_tab, P.table, P.ntab);
            cur = pi;
            __syncthreads();
        }
        const DevTile T = P.tiles[tile_local[item]];
        const DevRing R = P.rings[T.r];
        const float *in = args.in[pi];
        float *out = args.out[pi];
        for (int jj = threadIdx.x; jj < T.len; jj += blockDim.x) {
            const int j = T.j0 + jj;
            float acc[1];
            gather_pixel<1>(P, lds_tab, R, j, in, 0, 1, acc);
            out[R.first + j] = acc[0];
        }
    }
}

// ---------------------------------------------------------------- launch --
int forward_threads() { return kThreads; }

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

static size_t forward_lds(int ntab) { return (size_t)ntab * sizeof(float); }
static size_t backward_lds(int ntab, bool gk)
{
    return (size_t)hist_offset_floats(ntab) * sizeof(float) +
           (gk ? (size_t)ntab * sizeof(double) : 0);
}

// Variant index of the batch-width templates: NB = 1, 2, 4, 8.
static int nb_index(int nbatch) { return nbatch >= 8 ? 3 : nbatch >= 4 ? 2 : nbatch >= 2 ? 1 : 0; }

template <int NB>
static int prepare_nb(Plan &p, int vi)
{
    int rc = occupancy(k_forward<NB>, forward_lds(p.desc.ntab), &p.occ_fwd[vi]);
    if (rc) return rc;
    if ((p.desc.flags & ARKCOS_PLAN_LEARNABLE) && p.desc.ntab <= ARKCOS_MAX_GRAD_NTAB) {
        if ((rc = occupancy(k_backward<NB, true, true>, backward_lds(p.desc.ntab, true),
                            &p.occ_bwd_gxgk[vi])))
            return rc;
        if ((rc = occupancy(k_backward<NB, false, true>, backward_lds(p.desc.ntab, true),
                            &p.occ_bwd_gk[vi])))
            return rc;
    }
    return ARKCOS_OK;
}

int prepare_launches(Plan &p)
{
    ARKCOS_HIP_CHECK(hipDeviceGetAttribute(&p.cus, hipDeviceAttributeMultiprocessorCount,
                                           p.device));
    int rc;
    if ((rc = prepare_nb<1>(p, 0))) return rc;
    if ((rc = prepare_nb<2>(p, 1))) return rc;
    if ((rc = prepare_nb<4>(p, 2))) return rc;
    if ((rc = prepare_nb<8>(p, 3))) return rc;
    int most = 1;
    for (int v = 0; v < 4; ++v) most = std::max({most, p.occ_bwd_gxgk[v], p.occ_bwd_gk[v]});
    p.grid = most * p.cus;  // rows of the knot-gradient partials
    return ARKCOS_OK;
}

int prepare_batch(Batch &b)
{
    ARKCOS_HIP_CHECK(hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount,
                                           b.device));
    int per_cu = 0;
    int rc = occupancy(k_batch, forward_lds(b.max_ntab), &per_cu);
    if (rc) return rc;
    b.grid = std::max(1, std::min(b.ntiles, per_cu * b.cus));
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

template <int NB>
static int forward_nb(const Plan &p, const float *in, float *out, int nbatch, hipStream_t s)
{
    const size_t lds = forward_lds(p.desc.ntab);
    const int items = (int)p.tiles.size() * ((nbatch + NB - 1) / NB);
    const int grid = std::max(1, std::min(items, p.occ_fwd[nb_index(NB)] * p.cus));
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, p.d_counter);
    hipLaunchKernelGGL(k_forward<NB>, dim3(grid), dim3(kThreads), lds, s, p.view(), in, out,
                       nbatch, p.d_counter);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

int launch_forward(const Plan &p, const float *in, float *out, int nbatch, hipStream_t s)
{
    if (nbatch >= 8) return forward_nb<8>(p, in, out, nbatch, s);
    if (nbatch >= 4) return forward_nb<4>(p, in, out, nbatch, s);
    if (nbatch >= 2) return forward_nb<2>(p, in, out, nbatch, s);
    return forward_nb<1>(p, in, out, nbatch, s);
}

template <int NB, bool GX, bool GK>
static int backward_nb(const Plan &p, const float *g, const float *x, float *gx, float *gk,
                       int nbatch, hipStream_t s)
{
    const int ntab = p.desc.ntab;
    const size_t lds = backward_lds(ntab, GK);
    const int items = (int)p.tiles.size() * ((nbatch + NB - 1) / NB);
    const int occ = GX ? p.occ_bwd_gxgk[nb_index(NB)] : p.occ_bwd_gk[nb_index(NB)];
    const int grid = std::max(1, std::min({items, occ * p.cus, p.grid}));
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, p.d_counter);
    hipLaunchKernelGGL((k_backward<NB, GX, GK>), dim3(grid), dim3(kThreads), lds, s, p.view(),
                       g, x, gx, nbatch, p.d_counter, p.d_kpart);
    ARKCOS_HIP_CHECK(hipGetLastError());
    if (GK) {
        hipLaunchKernelGGL(k_knot_reduce, dim3((ntab + 255) / 256), dim3(256), 0, s, p.d_kpart,
                           grid, ntab, p.omega, gk);
        ARKCOS_HIP_CHECK(hipGetLastError());
    }
    return ARKCOS_OK;
}

template <bool GX, bool GK>
static int backward_dispatch(const Plan &p, const float *g, const float *x, float *gx,
                             float *gk, int nbatch, hipStream_t s)
{
    if (nbatch >= 8) return backward_nb<8, GX, GK>(p, g, x, gx, gk, nbatch, s);
    if (nbatch >= 4) return backward_nb<4, GX, GK>(p, g, x, gx, gk, nbatch, s);
    if (nbatch >= 2) return backward_nb<2, GX, GK>(p, g, x, gx, gk, nbatch, s);
    return backward_nb<1, GX, GK>(p, g, x, gx, gk, nbatch, s);
}

int launch_backward(const Plan &p, const float *g, const float *x, float *gx, float *gk,
                    int nbatch, hipStream_t s)
{
    if (gx && gk) return backward_dispatch<true, true>(p, g, x, gx, gk, nbatch, s);
    if (gk) return backward_dispatch<false, true>(p, g, x, gx, gk, nbatch, s);
    return launch_forward(p, g, gx, nbatch, s);
}

int launch_batch(const Batch &b, const float *const *in, float *const *out, hipStream_t s)
{
    if ((int)b.plans.size() > kMaxBatchMaps)
        return fail(ARKCOS_EUNSUPPORTED, "at most " + std::to_string(kMaxBatchMaps) +
                                             " maps per batch");
    BatchArgs args{};
    for (size_t k = 0; k < b.plans.size(); ++k) {
        args.in[k] = in[k];
        args.out[k] = out[k];
    }
    const size_t lds = forward_lds(b.max_ntab);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, b.d_counter);
    hipLaunchKernelGGL(k_batch, dim3(b.grid), dim3(kThreads), lds, s, b.d_views, b.d_tile_map,
                       b.d_tile_local, b.ntiles, args, b.d_counter);
    ARKCOS_HIP_CHECK(hipGetLastError());
    return ARKCOS_OK;
}

int batch_max_maps() { return kMaxBatchMaps; }

}  // namespace arkcos
