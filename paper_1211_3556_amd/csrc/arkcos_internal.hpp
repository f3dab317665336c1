// Internal declarations of libarkcos: plan layout shared by the host plan
// builder and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "arkcos.h"

namespace arkcos {

// ---------------------------------------------------------------- errors --
int fail(int status, const std::string &msg);   // records arkcos_last_error text
void clear_error();

// ------------------------------------------------------- profiler ranges --
// A roctx range named after an entry point, open for the lifetime of the
// object, so that traces (rocprofv3 --marker-trace) show plan builds and
// gathers under the call that issued them.
struct TraceRange {
    explicit TraceRange(const char *name);
    ~TraceRange();
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

#define ARKCOS_HIP_CHECK(call)                                                        \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::arkcos::fail(ARKCOS_EDEVICE, std::string(#call) + ": " +          \
                                                      hipGetErrorString(e_));         \
    } while (0)

// ------------------------------------------------------------ device plan --
// One HEALPix ring as the kernels see it (0-based ring index = ring - 1).
struct DevRing {
    int n;          // pixels in the ring
    int first;      // RING index of pixel 0 (< 12 * 8192^2 < 2^31)
    int two_o;      // 2 * phi offset in pixel units (1: half-pixel offset, 0: none)
    int pair_begin; // first ring-pair entry of this ring as an output ring
    int pair_end;
    int pad0, pad1, pad2;
};

// One (output ring r, source ring s) pair.  The chord between pixel (r, j) and
// pixel (s, j') is
//     d^2 = A + B sin^2(dphi/2),  A = (z_r - z_s)^2 + (sin_r - sin_s)^2
//                                   = 4 sin^2((theta_r - theta_s)/2),
//                                 B = 4 sin_r sin_s,
// with dphi/2 = m * xscale and m = (2j + 2o_r) n_s - (2j' + 2o_s) n_r an exact
// integer.  The longitude window of output pixel j is centred at source index
// c = j * a + b (a = n_s/n_r, b = o_r n_s/n_r - o_s) with half-width w source
// pixels (margin included).  mode bit 0: the window is every pixel of ring s;
// bit 1: |dphi/2| may exceed the short-row limit below, so the row takes the
// long sine series instead of its polynomial.
struct DevPair {
    float A;
    float B;
    float xscale;
    float a;
    float b;
    float w;
    int s;       // 0-based source ring
    int mode;
    // Rows without kPairLongSin: v = m mscale (mscale a power of two that
    // brings xscale / mscale into [1/2, 1), so v is exact in FP32), y = v^2
    // and the polynomial sq[0] + y (sq[1] + y (sq[2] + y (sq[3] + y sq[4]))).
    // In angle mode 0 it is the squared node coordinate u0^2 (the series of
    // (2 asin(d/2))^2 composed with the chord and scaled by the node density);
    // otherwise it is the squared chord d^2, through x^6 (sq[4] = 0).
    float mscale;
    float sq[5];
    // A candidate is inside the disc exactly when |m| <= mcut: the bound on
    // the longitude numerator from the FP64 half-width on the host
    // (|dphi| < dphi_cut with dphi = m pi / (n_r n_s)); 0x7fffffff for a
    // whole row (every pixel of ring s inside).
    int mcut;
    float pad;
};
constexpr int kPairWhole = 1;
constexpr int kPairLongSin = 2;
static_assert(sizeof(DevPair) == 64, "DevPair layout");
// Largest |x| = |dphi / 2| of a short row: the truncated series stay within
// 1e-9 relative there (angle mode 0 through x^8, first omitted term
// 2^9 x^10 / 10!; the squared chord through x^6, next term x^8 / 315).
constexpr double kShortXMaxMode0 = 0.2;
constexpr double kShortXMax = 0.09;

// FP64 copy of the chord constants of a ring pair, used where the node index
// and fraction must be exact to ~1e-9: the circulant weight rows (built once
// per table) and the knot gradient (the hat basis has slope 1/h, so an FP32
// angle moves node fractions by ~1e-7 u).
// The FP64 short-row polynomial (rows without kPairLongSin) is the one of
// DevPair before its rounding to FP32: in y = (m mscale)^2, the squared node
// coordinate in angle mode 0, the squared chord otherwise.
struct DevPairD {
    double A;
    double B;
    double xscale;
    double mscale;
    double sq[5];
    double pad;
};
static_assert(sizeof(DevPairD) == 80, "DevPairD layout");

// One work item: pixels j0 .. j0 + len - 1 of output ring r (or of the rings
// of group r, for the circulant kernel).
struct DevTile {
    int r;
    int j0;
    int len;
    int flags;     // general tiles: kTileLongSin, kTileIntM, kTileSkipNorth, kTileSkipSouth
};
// One ring of a general-gather tile: northern ring r, pixels j0 .. j0 + len - 1
// of its half-quadrant (len may be 0 at the end of a shorter ring), its
// flags, and its rows: source rings s_lo .. s_hi, pair records pb on.
struct GenRing {
    int r;
    int len;
    int flags;     // kTileSkipNorth, kTileSkipSouth; the loop form from all rings
    int pb;
    int s_lo;
    int s_hi;
};
// A general-gather tile of nr = 1, 2 or 4 adjacent northern rings over the
// same half-quadrant segment (adjacent rings cover nearly the same
// longitudes, so one staged chunk of a source ring serves all of them);
// source rings s_first .. s_last are read, staged as the nchunks chunks
// from c_begin on of the plan's chunk list.
constexpr int kGenMaxRings = 4;
struct DevTile2 {
    int nr;
    int j0;
    int s_first;
    int s_last;
    GenRing q[kGenMaxRings];
    int c_begin;
    int nchunks;
    int pad[2];
};
static_assert(sizeof(DevTile2) == 128, "DevTile2 layout");
// One staged chunk of a general tile: unwrapped positions c0 .. c0 + cn - 1
// of source ring s (inside the union of the tile's row windows on s), with
// the geometry of s and of its mirror ring, and which of the two count as
// zero (bit 0: ring s, bit 1: the mirror; outside a plan's source rings).
// Built on the host with the kernels' own window arithmetic, so that the
// kernel reads one record per chunk instead of every ring's pair record.
struct GenChunk {
    int s;
    int c0;
    int cn;
    int n;
    int two_o;
    int first;
    int first_m;
    int mask;
};
static_assert(sizeof(GenChunk) == 32, "GenChunk layout");

constexpr int kTileLongSin = 1;   // some source row needs the long sine series
constexpr int kTileIntM = 2;      // a longitude numerator may reach 2^24: keep it in int32
constexpr int kTileSkipNorth = 4; // the northern ring is outside the plan's ring range
constexpr int kTileSkipSouth = 8; // its mirror ring is outside the plan's ring range

// Rings per group and outputs per lane of the circulant kernel; pixels per
// general tile and source positions one pass of the general kernel stages;
// source pixels one pass of the knot-gradient kernel stages per image.
constexpr int kThreads = 256;
constexpr int kGroupRings = 4;
constexpr int kCircPix = 4;
constexpr int kCircSeg = kThreads * kCircPix;
constexpr int kCircMaxTaps = 256;   // taps of one circulant row (wider rows are split)
// The circulant gather runs on the matrix cores when the plan's rows average
// at least this many taps (a row of t taps costs products for t + 3 there).
constexpr int kCircMfmaTaps = 9;
constexpr int kGenLanes = 128;       // most pixels of one ring per general tile
constexpr int kGenThreads = 512;     // general-gather workgroup (one part of lanes per ring)
// Built-in general-gather tile shapes (arkcos_tiles): pixels per ring, and the
// widest row window (positions) of a ring in a tile of four / of two rings.
constexpr int kGenPixelsDefault = 128;
constexpr int kGenQuadWindowDefault = 64;
constexpr int kGenPairWindowDefault = 200;
constexpr int kGenStage = 248;       // with a 16384-node table two workgroups fit a CU
constexpr int kMaxMaps = 32;
// Circulant knot-gradient tiles: kKnotSeg pixels of a ring group.
constexpr int kKnotSeg = 512;

// A group of up to kGroupRings consecutive belt rings r0 .. r0+nr-1 whose
// source rings all have the ring's own pixel count: the weight of a pair then
// depends only on (r, s, j' - j), so each (r, s) has one weight row.
struct DevGroup {
    int r0;
    int nr;
    int row_begin;
    int row_end;
};

// One source ring s of a group: taps k = k_lo .. k_lo+ntaps-1 (source pixel
// j + k for output pixel j); the weight of tap t for ring r0+i is
// wts[w_off + t * kGroupRings + i] (zero where (r0+i, s, k) is not a candidate).
struct DevRow {
    int s;
    int k_lo;
    int ntaps;
    int w_off;
    int g;
    int first_s;   // RING index of pixel 0 of ring s (no dependent ring lookup per row)
    int pad0, pad1;
};

// Kernel-argument view of a plan (passed by value).
struct DevPlanView {
    const DevRing *rings;
    const DevPair *pairs;
    const float *table;      // ntab FP32 values Omega * K_k
    const DevPairD *pairs_d; // FP64 chord constants of the pairs
    double inv_h_d;          // a0 in FP64 (node coordinate map below)
    double bias_r_d;         // r and c in FP64
    double bias_c_d;
    const DevGroup *groups;  // circulant ring groups
    const DevRow *rows;      // their source rows
    float *wts;              // their weight rows (written by the weight-build kernel)
    const DevTile *ctiles;   // circulant tiles: (group, j0, len)
    const DevTile2 *gtiles2; // the same segments, two adjacent rings per tile (general gather)
    const GenChunk *gchunks; // their staged chunks, tile by tile
    const DevTile *kctiles;  // circulant knot-gradient tiles: (group, j0, len)
    const double *kw;        // FP64 node coordinate per circulant weight slot, or -1
    int nctiles;
    int ngtiles2;
    int nkctiles;
    int nkpart_circ;         // partial rows written by the circulant knot kernel
    int nrows;
    int nrings;
    int ntab;
    int npix;
    int angle_mode;          // angle series: 0 (theta_cut <= 0.1), 1 (<= 0.5), 2 full range
    int circ_mfma;           // circulant gather on the matrix cores (1) or vector FMAs (0)
    // Node coordinate u of an angle (node k at u = k):  u0 = a0 theta, and
    // u = u0 on a uniform grid (a0 = (ntab-1)/theta_cut), u = min(u0, r u0 + c)
    // on the two-piece biased grid (a0 = k_break/theta_break the fine piece's
    // 1/h; r u0 + c the coarse piece's coordinate, which is the smaller one
    // beyond the break).  r = 1 and c = 0 on a uniform grid.  The FP32 gather
    // counts the coarse coordinate from the break instead: u = k_break + v,
    // v = r u0 + bias_c with bias_c = -r k_break (v >= 0 beyond the break).
    int src_lo;              // source rings read (0-based, inclusive): images of rings
    int src_hi;              // outside count as zero (the adjoint of a ring range)
    int biased;
    int k_break;             // node index of the break (0 on a uniform grid)
    float inv_h;             // a0
    float bias_r;
    float bias_c;            // -r k_break
    float u_coef[6];         // a0 times the coefficients of the short angle series
};

// ------------------------------------------------------- shared FP32 math --
// Window of output pixel j of ring r on source ring s, exactly as the kernels
// compute it.  Returns the unwrapped index range [lo, hi]; since
// -1/2 <= c < n_s + 1/2 and w < n_s/2, -n_s < lo and hi < 2 n_s, so one
// conditional add or subtract of n_s wraps any index into the ring.
__host__ __device__ inline void pair_window(const DevPair &p, int n_s, int j, int &lo,
                                            int &hi)
{
    float c = fmaf((float)j, p.a, p.b);
    if (p.mode & kPairWhole) {
        // n_s consecutive pixels centred on c: |dphi| <= pi + pi/n_s
        lo = (int)floorf(c + 0.5f) - (n_s >> 1);
        hi = lo + n_s - 1;
    } else {
        lo = (int)ceilf(c - p.w);
        hi = (int)floorf(c + p.w);
    }
}

// --------------------------------------------------------------- host plan --
struct HostRing {
    double z, s, theta, phi0;
    int n;
    long long first;
    int two_o;
};

// HEALPix RING geometry of ring i (1-based) at resolution N (plan.hip).
HostRing ring_geometry(int N, int i);

struct Plan {
    arkcos_plan_desc desc{};
    int nside = 0;
    int nrings = 0;
    long long npix = 0;
    double omega = 0.0;
    int threads = 0;
    bool host_only = false;
    bool knots_set = false;
    int angle_mode = 0;

    std::vector<HostRing> rings;      // 0-based
    std::vector<DevRing> dev_rings;
    std::vector<DevPair> pairs;
    std::vector<DevPairD> pairs_d;    // same order as pairs
    std::vector<DevGroup> groups;
    std::vector<DevRow> rows;
    std::vector<DevTile> ctiles;      // circulant tiles, longest first
    std::vector<DevTile> gtiles;      // half-quadrant segments of the general rings (host only)
    std::vector<DevTile> kctiles;     // circulant knot-gradient tiles, longest first
    std::vector<double> ctile_cost, gtile_cost, gtile2_cost;
    std::vector<DevTile2> gtiles2;    // general-gather tiles (1, 2 or 4 rings), longest first
    std::vector<GenChunk> gchunks;    // their staged chunks
    arkcos_tiles tiles{};             // resolved general-gather tile shapes
    int tile_source = 0;              // 0 defaults, 1 tuning cache, 2 descriptor
    // the general northern rings in order, for the general-gather tiling:
    // ring, pixels of its half-quadrant, tile flags, widest row window
    std::vector<int> gen_ring, gen_lanes, gen_flags;
    std::vector<double> gen_wmax;
    std::vector<double> ring_cost;    // candidates per output pixel of each ring
    // Source rings read by the gathers (0-based, inclusive; all if src_hi < 0).
    // Only the adjoint sub-plan of a ring-range plan restricts them.
    int src_lo = 0;
    int src_hi = -1;

    // Ring-range plans: the adjoint's plan, whose output rings are every
    // source ring of the range and whose source rings are the range.
    Plan *adj = nullptr;
    long long nweights = 0;
    int max_taps = 0;
    int circ_form = 0;                // circulant gather: 0 vector FMAs, 1 matrix cores
    std::vector<double> ktab;         // current host copy (FP64), if known
    long long candidates = 0;
    bool pairs_counted = false;
    unsigned long long pair_count = 0;
    unsigned long long pair_count_circ = 0;   // pairs of circulant output rings
    std::vector<char> general_ring;           // ring class (1: general)

    // device memory
    int device = -1;
    DevRing *d_rings = nullptr;
    DevPair *d_pairs = nullptr;
    DevPairD *d_pairs_d = nullptr;
    DevGroup *d_groups = nullptr;
    DevRow *d_rows = nullptr;
    float *d_wts = nullptr;
    DevTile *d_ctiles = nullptr;
    DevTile2 *d_gtiles2 = nullptr;
    GenChunk *d_gchunks = nullptr;
    long long gen_tile_bytes = 0;       // device bytes of d_gtiles2 and d_gchunks
    DevTile *d_kctiles = nullptr;
    double *d_kw = nullptr;             // knot node coordinates of the circulant slots
    DevPlanView *d_view = nullptr;      // device copy of view() (a batch of one plan)
    float *d_table = nullptr;
    unsigned int *d_counter = nullptr;  // persistent-queue counter (+ 1 spare)
    double *d_kpart = nullptr;          // knot-gradient partials [grid][ntab] (learnable)
    int grid = 0;                       // rows of d_kpart: grid_kc + grid_kg
    int grid_kc = 0;                    // resident workgroups of the two knot kernels
    int grid_kg = 0;
    int cus = 0;                        // compute units of the device
    int occ_circ = 0;                   // resident workgroups per CU of the two gathers
    int occ_gen = 0;
    int occ_kc = 0;                     // and of the two knot-gradient kernels
    int occ_kg = 0;
    long long device_bytes = 0;

    DevPlanView view() const;
};

struct Batch {
    std::vector<Plan *> plans;
    std::vector<int2> cmap;             // circulant tiles of all plans: (plan, tile), those of
                                        // vector-form plans first, each part longest first
    int ncirc_valu = 0;                 // tiles of vector-form plans at the front of cmap
    std::vector<int2> gmap;             // general tiles of all plans
    int2 *d_cmap = nullptr;
    int2 *d_gmap = nullptr;
    DevPlanView *d_views = nullptr;
    unsigned int *d_counter = nullptr;
    int grid_circ = 0;
    int grid_circ_mfma = 0;
    int grid_gen = 0;
    int cus = 0;
    int max_ntab = 0;
    int max_taps = 0;
    int device = -1;
};

// ----------------------------------------------------------------- launch --
// Implemented in kernels.hip.
int launch_set_table(const Plan &p, const float *d_knots, hipStream_t s);
// `counter` (the gathers' queue counters, three) and `kpart` (knot-gradient partial rows,
// knot_partial_bytes) replace the plan's own workspace when non-NULL.
int launch_forward(const Plan &p, const float *in, float *out, int nbatch, hipStream_t s,
                   int parts = ARKCOS_PART_ALL, unsigned int *counter = nullptr);
int launch_backward(const Plan &p, const float *g, const float *x, float *gx, float *gk,
                    int nbatch, hipStream_t s, unsigned int *counter = nullptr,
                    double *kpart = nullptr);
long long knot_partial_bytes(const Plan &p);
int launch_batch(const Batch &b, const float *const *in, float *const *out, hipStream_t s,
                 int parts = ARKCOS_PART_ALL);
int launch_build_weights(const Plan &p, hipStream_t s);
int launch_build_knotw(const Plan &p, hipStream_t s);
int device_lds_limit(int device, size_t *bytes);
int prepare_launches(Plan &p);   // occupancy of every kernel variant, grid sizes
// General-gather tiles of a built plan from P.tiles (plan.hip).
void build_gen_tiles(Plan &P);
// Replace the device copy of the general-gather tiles (and the plan view).
int upload_gen_tiles(Plan &P);
// Resolve the tile shapes of a descriptor: descriptor fields, else the tuning
// cache, else the defaults (tune.hip); EINVAL on invalid fields.
int resolve_tiles(const arkcos_plan_desc &d, arkcos_tiles *out, int *source);
int check_tiles(const arkcos_tiles &t);
int prepare_batch(Batch &b);
int forward_threads();
int batch_max_maps();

}  // namespace arkcos
