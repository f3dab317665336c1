// Tile autotuning of the general gather: the tuning cache (a text file keyed
// by device arch, Nside and window class), the resolution of a plan's tile
// shapes, and the tuner itself, which times the general gather of one plan
// over candidate tiles on the device.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "arkcos_internal.hpp"

namespace arkcos {

namespace {

std::mutex g_cache_mu;
bool g_cache_set = false;       // arkcos_set_tune_cache was called
std::string g_cache_path;

std::string cache_path()
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_cache_set) return g_cache_path;
    const char *e = getenv("ARKCOS_TUNE_CACHE");
    return e ? std::string(e) : std::string();
}

// gfx name of the current device, or the build target without a device.
std::string device_arch()
{
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::string a(prop.gcnArchName);
        const size_t c = a.find(':');
        if (c != std::string::npos) a.resize(c);
        if (!a.empty()) return a;
    }
    (void)hipGetLastError();
    return "gfx950";
}

int window_class(int nside, double theta_cut)
{
    const double pix = std::sqrt(M_PI / 3.0) / (double)nside;   // sqrt(Omega)
    return (int)std::lround(2.0 * std::log2(theta_cut / pix));
}

// Tuning-cache class of a descriptor: the window class, plus
// ARKCOS_TUNE_RANGE_CLASS for a plan restricted to a ring range.  Such a plan
// tiles only part of the general rings, and its one-sided tiles run the
// eight-image loop, so its best tiles are kept apart from the full sky's.
int tune_class(const arkcos_plan_desc &d)
{
    const bool all = (d.ring_first == 0 && d.ring_last == 0) ||
                     (d.ring_first <= 1 && d.ring_last >= 4 * d.nside - 1);
    return window_class(d.nside, d.theta_cut) + (all ? 0 : ARKCOS_TUNE_RANGE_CLASS);
}

struct CacheEntry {
    arkcos_tiles tiles;
    double ms;
};

// Last entry of the cache file for (arch, nside, class); false if none.
bool cache_lookup(const std::string &path, const std::string &arch, int nside, int cls,
                  CacheEntry *out)
{
    if (path.empty()) return false;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char *hash = strchr(line, '#');
        if (hash) *hash = '\0';
        char a[64];
        int n, c, gp, gq, gpw;
        double ms;
        if (sscanf(line, "%63s %d %d %d %d %d %lf", a, &n, &c, &gp, &gq, &gpw, &ms) != 7) continue;
        if (arch != a || n != nside || c != cls) continue;
        arkcos_tiles t{gp, gq, gpw, 0};
        if (check_tiles(t) != ARKCOS_OK || gp == 0 || gq == 0 || gpw == 0) continue;
        out->tiles = t;
        out->ms = ms;
        found = true;
    }
    fclose(f);
    clear_error();   // a malformed line is skipped, not an error of the caller
    return found;
}

}  // namespace

int check_tiles(const arkcos_tiles &t)
{
    if (t.gen_pixels != 0 && t.gen_pixels != 16 && t.gen_pixels != 32 && t.gen_pixels != 64 &&
        t.gen_pixels != 128)
        return fail(ARKCOS_EINVAL, "tiles.gen_pixels must be 0, 16, 32, 64 or 128");
    auto bad_window = [](int w) { return !(w == 0 || w == -1 || (w >= 1 && w <= 1000000)); };
    if (bad_window(t.gen_quad_window) || bad_window(t.gen_pair_window))
        return fail(ARKCOS_EINVAL, "tile window thresholds must be 0, -1 or 1..1000000");
    if (t.reserved != 0) return fail(ARKCOS_EINVAL, "tiles.reserved must be 0");
    return ARKCOS_OK;
}

int resolve_tiles(const arkcos_plan_desc &d, arkcos_tiles *out, int *source)
{
    int rc = check_tiles(d.tiles);
    if (rc) return rc;
    const arkcos_tiles &t = d.tiles;
    *out = arkcos_tiles{kGenPixelsDefault, kGenQuadWindowDefault, kGenPairWindowDefault, 0};
    *source = 0;
    if (t.gen_pixels == 0 && t.gen_quad_window == 0 && t.gen_pair_window == 0) {
        CacheEntry e;
        if (cache_lookup(cache_path(), device_arch(), d.nside, tune_class(d), &e)) {
            *out = e.tiles;
            *source = 1;
        }
        return ARKCOS_OK;
    }
    if (t.gen_pixels) out->gen_pixels = t.gen_pixels;
    if (t.gen_quad_window) out->gen_quad_window = t.gen_quad_window;
    if (t.gen_pair_window) out->gen_pair_window = t.gen_pair_window;
    *source = 2;
    return ARKCOS_OK;
}

}  // namespace arkcos

using namespace arkcos;

namespace {

// Median time (ms) of `reps` general-gather launches of plan P with tiles t.
int time_tiles(Plan &P, const arkcos_tiles &t, const float *in, float *out, int reps,
               hipStream_t s, hipEvent_t e0, hipEvent_t e1, double *ms)
{
    P.tiles = t;
    build_gen_tiles(P);
    int rc = upload_gen_tiles(P);
    if (rc) return rc;
    if ((rc = launch_forward(P, in, out, 1, s, ARKCOS_PART_GENERAL))) return rc;   // warm-up
    std::vector<double> v;
    for (int k = 0; k < reps; ++k) {
        ARKCOS_HIP_CHECK(hipEventRecord(e0, s));
        if ((rc = launch_forward(P, in, out, 1, s, ARKCOS_PART_GENERAL))) return rc;
        ARKCOS_HIP_CHECK(hipEventRecord(e1, s));
        ARKCOS_HIP_CHECK(hipEventSynchronize(e1));
        float f = 0.0f;
        ARKCOS_HIP_CHECK(hipEventElapsedTime(&f, e0, e1));
        v.push_back(f);
    }
    std::sort(v.begin(), v.end());
    *ms = v[v.size() / 2];
    return ARKCOS_OK;
}

}  // namespace

extern "C" {

int arkcos_set_tune_cache(const char *path)
{
    clear_error();
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache_set = true;
    g_cache_path = path ? std::string(path) : std::string();
    return ARKCOS_OK;
}

int arkcos_tune_key(int nside, double theta_cut, char *arch, int len, int *cls)
{
    clear_error();
    if (nside < 1 || nside > ARKCOS_MAX_NSIDE) return fail(ARKCOS_EINVAL, "nside out of range");
    if (!(theta_cut > 0.0) || theta_cut > M_PI)
        return fail(ARKCOS_EINVAL, "theta_cut must lie in (0, pi]");
    if (arch && len > 0) {
        const std::string a = device_arch();
        snprintf(arch, (size_t)len, "%s", a.c_str());
    }
    if (cls) *cls = window_class(nside, theta_cut);
    return ARKCOS_OK;
}

int arkcos_tune(const arkcos_plan_desc *desc, int reps, const char *cache_file,
                arkcos_tiles *best, double *best_ms, double *default_ms)
{
    clear_error();
    if (!desc) return fail(ARKCOS_EINVAL, "NULL descriptor");
    if (reps < 1) return fail(ARKCOS_EINVAL, "reps must be >= 1");
    int rc = check_tiles(desc->tiles);
    if (rc) return rc;
    arkcos_plan_desc d = *desc;
    std::vector<double> flat;
    if (!d.ktab) {
        flat.assign((size_t)std::max(d.ntab, 2), 1.0);
        d.ktab = flat.data();
    }
    d.flags &= ~ARKCOS_PLAN_HOST_ONLY;
    d.max_batch = 1;
    const arkcos_tiles fixed = desc->tiles;
    arkcos_tiles cur{fixed.gen_pixels ? fixed.gen_pixels : kGenPixelsDefault,
                     fixed.gen_quad_window ? fixed.gen_quad_window : kGenQuadWindowDefault,
                     fixed.gen_pair_window ? fixed.gen_pair_window : kGenPairWindowDefault, 0};
    d.tiles = cur;
    arkcos_plan_t h = nullptr;
    if ((rc = arkcos_plan_create(&d, &h))) return rc;
    Plan &P = *reinterpret_cast<Plan *>(h);
    float *buf = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double t_def = 0.0, t_best = 0.0;
    auto done = [&](int status) {
        if (s) (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        const std::string msg = arkcos_last_error();
        arkcos_plan_destroy(h);
        if (status) fail(status, msg);
        return status;
    };
    if (hipMalloc((void **)&buf, 2 * (size_t)P.npix * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return done(fail(ARKCOS_ENOMEM, "hipMalloc of the tuning maps failed"));
    }
    if (hipMemset(buf, 0x3f, 2 * (size_t)P.npix * sizeof(float)) != hipSuccess ||
        hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        return done(fail(ARKCOS_EDEVICE, "tuning set-up failed"));
    const float *in = buf;
    float *out = buf + P.npix;
    if (!P.gen_ring.empty()) {
        const arkcos_tiles def{kGenPixelsDefault, kGenQuadWindowDefault, kGenPairWindowDefault, 0};
        if ((rc = time_tiles(P, def, in, out, reps, s, e0, e1, &t_def))) return done(rc);
        if ((rc = time_tiles(P, cur, in, out, reps, s, e0, e1, &t_best))) return done(rc);
        const int pix[] = {32, 64, 128};
        const int quad[] = {-1, 32, 64, 96, 128};
        const int pair[] = {-1, 100, 200, 400, 800};
        // coordinate descent over the free fields, two passes
        for (int pass = 0; pass < 2; ++pass) {
            for (int field = 0; field < 3; ++field) {
                const int *cand = field == 0 ? pix : (field == 1 ? quad : pair);
                const int ncand = field == 0 ? 3 : 5;
                const int fixed_v = field == 0 ? fixed.gen_pixels
                                               : (field == 1 ? fixed.gen_quad_window
                                                             : fixed.gen_pair_window);
                if (fixed_v) continue;
                for (int i = 0; i < ncand; ++i) {
                    arkcos_tiles t = cur;
                    int &f = field == 0 ? t.gen_pixels
                                        : (field == 1 ? t.gen_quad_window : t.gen_pair_window);
                    if (f == cand[i]) continue;
                    f = cand[i];
                    double ms = 0.0;
                    if ((rc = time_tiles(P, t, in, out, reps, s, e0, e1, &ms))) return done(rc);
                    if (ms < t_best) {
                        t_best = ms;
                        cur = t;
                    }
                }
            }
        }
    }
    if (best) *best = cur;
    if (best_ms) *best_ms = t_best;
    if (default_ms) *default_ms = t_def;
    if (cache_file) {
        FILE *f = fopen(cache_file, "a");
        if (!f) return done(fail(ARKCOS_EINVAL, std::string("cannot append to ") + cache_file));
        fprintf(f, "%s %d %d %d %d %d %.6f\n", device_arch().c_str(), desc->nside,
                tune_class(*desc), cur.gen_pixels, cur.gen_quad_window,
                cur.gen_pair_window, t_best);
        fclose(f);
    }
    return done(ARKCOS_OK);
}

}  // extern "C"
