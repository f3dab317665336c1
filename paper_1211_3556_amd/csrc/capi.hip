// C ABI of the compute entry points: argument checks, then stream-ordered
// launches (kernels.hip).  Plan construction lives in plan.hip.
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <numeric>
#include <string>

#include "arkcos_internal.hpp"

using namespace arkcos;

// Workspace of arkcos_convolve_backward_static: the queue counters of the
// gathers in the first 256 bytes, then the knot-gradient partial rows.  One
// copy per device, held for the life of the process.  In host code this name
// is only a handle: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[ARKCOS_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchCounterBytes = 256;

// Device address of `scratch` on each device, looked up once per device with
// that device current.
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

int scratch_address(int device, void **ptr)
{
    if (device < 0 || device >= 64) return fail(ARKCOS_EUNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        ARKCOS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return ARKCOS_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

int check_compute(const Plan *P, int nbatch)
{
    if (P->host_only) return fail(ARKCOS_ESTATE, "host-only plan cannot launch kernels");
    if (!P->knots_set) return fail(ARKCOS_ESTATE, "node table not set");
    if (nbatch < 1 || nbatch > P->desc.max_batch)
        return fail(ARKCOS_EINVAL, "nbatch must lie in 1..max_batch (" +
                                       std::to_string(P->desc.max_batch) + ")");
    return ARKCOS_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

int arkcos_convolve_part(arkcos_plan_t plan, const float *d_in, float *d_out, int nbatch, int part,
                         void *stream)
{
    TraceRange tr("arkcos_convolve");
    clear_error();
    if (!plan || !d_in || !d_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (part < 1 || part > ARKCOS_PART_ALL) return fail(ARKCOS_EINVAL, "unknown part");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    int rc = check_compute(P, nbatch);
    if (rc) return rc;
    const size_t bytes = (size_t)nbatch * (size_t)P->npix * sizeof(float);
    if (overlaps(d_in, bytes, d_out, bytes)) return fail(ARKCOS_EINVAL, "d_in and d_out overlap");
    DeviceGuard g(P->device);
    return launch_forward(*P, d_in, d_out, nbatch, (hipStream_t)stream, part);
}

int arkcos_convolve(arkcos_plan_t plan, const float *d_in, float *d_out, int nbatch,
                    void *stream)
{
    return arkcos_convolve_part(plan, d_in, d_out, nbatch, ARKCOS_PART_ALL, stream);
}

// Argument checks shared by the two backward entry points.
static int check_backward(const Plan *P, const float *d_grad_out, const float *d_in,
                          const float *d_grad_in, const float *d_grad_knots, int nbatch)
{
    if (!d_grad_in && !d_grad_knots)
        return fail(ARKCOS_EINVAL, "at least one of d_grad_in, d_grad_knots must be non-NULL");
    int rc = check_compute(P, nbatch);
    if (rc) return rc;
    const size_t bytes = (size_t)nbatch * (size_t)P->npix * sizeof(float);
    const size_t kbytes = (size_t)P->desc.ntab * sizeof(float);
    if (d_grad_in && overlaps(d_grad_in, bytes, d_grad_out, bytes))
        return fail(ARKCOS_EINVAL, "d_grad_in overlaps d_grad_out");
    if (d_grad_knots) {
        if (!(P->desc.flags & ARKCOS_PLAN_LEARNABLE))
            return fail(ARKCOS_ESTATE, "knot gradients need ARKCOS_PLAN_LEARNABLE");
        if (P->desc.ntab > ARKCOS_MAX_GRAD_NTAB || !P->d_kpart)
            return fail(ARKCOS_EUNSUPPORTED, "knot gradients need ntab <= " +
                                                 std::to_string(ARKCOS_MAX_GRAD_NTAB));
        if (!d_in) return fail(ARKCOS_EINVAL, "knot gradients need d_in");
        if (overlaps(d_grad_knots, kbytes, d_grad_out, bytes) ||
            overlaps(d_grad_knots, kbytes, d_in, bytes))
            return fail(ARKCOS_EINVAL, "d_grad_knots overlaps an input");
        if (d_grad_in && (overlaps(d_grad_in, bytes, d_in, bytes) ||
                          overlaps(d_grad_in, bytes, d_grad_knots, kbytes)))
            return fail(ARKCOS_EINVAL, "d_grad_in overlaps d_in or d_grad_knots");
    }
    return ARKCOS_OK;
}

int arkcos_convolve_backward(arkcos_plan_t plan, const float *d_grad_out, const float *d_in,
                             float *d_grad_in, float *d_grad_knots, int nbatch, void *stream)
{
    TraceRange tr("arkcos_convolve_backward");
    clear_error();
    if (!plan || !d_grad_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    int rc = check_backward(P, d_grad_out, d_in, d_grad_in, d_grad_knots, nbatch);
    if (rc) return rc;
    DeviceGuard g(P->device);
    return launch_backward(*P, d_grad_out, d_in, d_grad_in, d_grad_knots, nbatch,
                           (hipStream_t)stream);
}

int arkcos_convolve_backward_static(arkcos_plan_t plan, const float *d_grad_out,
                                    const float *d_in, float *d_grad_in, float *d_grad_knots,
                                    int nbatch, void *stream)
{
    TraceRange tr("arkcos_convolve_backward_static");
    clear_error();
    if (!plan || !d_grad_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    int rc = check_backward(P, d_grad_out, d_in, d_grad_in, d_grad_knots, nbatch);
    if (rc) return rc;
    const long long need = d_grad_knots ? knot_partial_bytes(*P) : 0;
    if (need > (long long)(ARKCOS_STATIC_SCRATCH_BYTES - kScratchCounterBytes))
        return fail(ARKCOS_EUNSUPPORTED,
                    "knot-gradient partials need " + std::to_string(need) +
                        " bytes, more than the static workspace holds (" +
                        std::to_string(ARKCOS_STATIC_SCRATCH_BYTES - kScratchCounterBytes) + ")");
    DeviceGuard g(P->device);
    void *base = nullptr;
    if ((rc = scratch_address(P->device, &base))) return rc;
    // the counters are reset by a kernel at the start of each gather, and every
    // partial row is written before it is reduced, so nothing is cleared here
    unsigned int *counter = reinterpret_cast<unsigned int *>(base);
    double *kpart = reinterpret_cast<double *>(static_cast<unsigned char *>(base) +
                                               kScratchCounterBytes);
    return launch_backward(*P, d_grad_out, d_in, d_grad_in, d_grad_knots, nbatch,
                           (hipStream_t)stream, counter, kpart);
}

int arkcos_batch_create(const arkcos_plan_t *plans, int nmaps, arkcos_batch_t *out)
{
    clear_error();
    if (!out) return fail(ARKCOS_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (!plans || nmaps < 1) return fail(ARKCOS_EINVAL, "need at least one plan");
    if (nmaps > batch_max_maps())
        return fail(ARKCOS_EUNSUPPORTED, "at most " + std::to_string(batch_max_maps()) +
                                             " maps per batch");
    Batch *B = new (std::nothrow) Batch();
    if (!B) return fail(ARKCOS_ENOMEM, "host allocation failed");
    std::vector<DevPlanView> views;
    std::vector<double> ccost, gcost, mcost;
    std::vector<int2> cmap_m;   // tiles of matrix-form plans
    for (int k = 0; k < nmaps; ++k) {
        Plan *P = reinterpret_cast<Plan *>(plans[k]);
        if (!P) { delete B; return fail(ARKCOS_EINVAL, "NULL plan in batch"); }
        if (P->host_only) { delete B; return fail(ARKCOS_ESTATE, "host-only plan in batch"); }
        if (B->device < 0) B->device = P->device;
        if (P->device != B->device) { delete B; return fail(ARKCOS_EINVAL, "plans on different devices"); }
        B->plans.push_back(P);
        B->max_ntab = std::max(B->max_ntab, P->desc.ntab);
        B->max_taps = std::max(B->max_taps, P->max_taps);
        views.push_back(P->view());
        for (int t = 0; t < (int)P->ctiles.size(); ++t) {
            (P->circ_form ? cmap_m : B->cmap).push_back(make_int2(k, t));
            (P->circ_form ? mcost : ccost).push_back(P->ctile_cost[t]);
        }
        for (int t = 0; t < (int)P->gtiles2.size(); ++t) {
            B->gmap.push_back(make_int2(k, t));
            gcost.push_back(P->gtile2_cost[t]);
        }
    }
    // one queue per kernel over the tiles of every plan, longest first
    auto sort_map = [](std::vector<int2> &m, const std::vector<double> &c) {
        std::vector<size_t> order(m.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return c[a] > c[b]; });
        std::vector<int2> m2(m.size());
        for (size_t i = 0; i < order.size(); ++i) m2[i] = m[order[i]];
        m.swap(m2);
    };
    sort_map(B->cmap, ccost);
    sort_map(cmap_m, mcost);
    B->ncirc_valu = (int)B->cmap.size();
    B->cmap.insert(B->cmap.end(), cmap_m.begin(), cmap_m.end());
    sort_map(B->gmap, gcost);

    DeviceGuard g(B->device);
    auto bail = [&](int rc) {
        (void)hipFree(B->d_cmap);
        (void)hipFree(B->d_gmap);
        (void)hipFree(B->d_views);
        (void)hipFree(B->d_counter);
        delete B;
        return rc;
    };
    const size_t nc = std::max<size_t>(B->cmap.size(), 1), ng = std::max<size_t>(B->gmap.size(), 1);
    if (hipMalloc((void **)&B->d_cmap, sizeof(int2) * nc) != hipSuccess ||
        hipMalloc((void **)&B->d_gmap, sizeof(int2) * ng) != hipSuccess ||
        hipMalloc((void **)&B->d_views, sizeof(DevPlanView) * nmaps) != hipSuccess ||
        hipMalloc((void **)&B->d_counter, sizeof(unsigned int) * 4) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(ARKCOS_ENOMEM, "hipMalloc failed for the batch queues"));
    }
    if ((!B->cmap.empty() && hipMemcpy(B->d_cmap, B->cmap.data(), sizeof(int2) * B->cmap.size(),
                                       hipMemcpyHostToDevice) != hipSuccess) ||
        (!B->gmap.empty() && hipMemcpy(B->d_gmap, B->gmap.data(), sizeof(int2) * B->gmap.size(),
                                       hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(B->d_views, views.data(), sizeof(DevPlanView) * nmaps, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(B->d_counter, 0, sizeof(unsigned int) * 4) != hipSuccess)
        return bail(fail(ARKCOS_EDEVICE, "copy of the batch queues failed"));
    int rc = prepare_batch(*B);
    if (rc) return bail(rc);
    *out = reinterpret_cast<arkcos_batch_t>(B);
    return ARKCOS_OK;
}

int arkcos_batch_convolve(arkcos_batch_t batch, const float *const *d_in, float *const *d_out,
                          void *stream)
{
    return arkcos_batch_convolve_part(batch, d_in, d_out, ARKCOS_PART_ALL, stream);
}

int arkcos_batch_convolve_part(arkcos_batch_t batch, const float *const *d_in,
                               float *const *d_out, int part, void *stream)
{
    clear_error();
    TraceRange tr("arkcos_batch_convolve");
    if (!batch || !d_in || !d_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (part < 1 || part > ARKCOS_PART_ALL) return fail(ARKCOS_EINVAL, "unknown part");
    const Batch *B = reinterpret_cast<const Batch *>(batch);
    const int n = (int)B->plans.size();
    for (int k = 0; k < n; ++k) {
        if (!d_in[k] || !d_out[k]) return fail(ARKCOS_EINVAL, "NULL map pointer");
        if (!B->plans[k]->knots_set) return fail(ARKCOS_ESTATE, "node table not set");
    }
    for (int k = 0; k < n; ++k) {
        const size_t bk = (size_t)B->plans[k]->npix * sizeof(float);
        for (int l = 0; l < n; ++l) {
            const size_t bl = (size_t)B->plans[l]->npix * sizeof(float);
            if (overlaps(d_out[k], bk, d_in[l], bl))
                return fail(ARKCOS_EINVAL, "an output map overlaps an input map");
            if (l != k && overlaps(d_out[k], bk, d_out[l], bl))
                return fail(ARKCOS_EINVAL, "output maps overlap");
        }
    }
    DeviceGuard g(B->device);
    return launch_batch(*B, d_in, d_out, (hipStream_t)stream, part);
}

int arkcos_batch_destroy(arkcos_batch_t batch)
{
    clear_error();
    if (!batch) return ARKCOS_OK;
    Batch *B = reinterpret_cast<Batch *>(batch);
    {
        DeviceGuard g(B->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(B->d_cmap);
        (void)hipFree(B->d_gmap);
        (void)hipFree(B->d_views);
        (void)hipFree(B->d_counter);
    }
    delete B;
    return ARKCOS_OK;
}

}  // extern "C"
