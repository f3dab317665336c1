// Host plan of the real-space convolution: HEALPix ring geometry, the node
// table, per-ring source lists with longitude windows, tiles and exact pair
// counts (Sutter, Wandelt & Elsner 2012, Sec. 2: the real-space part K_theta
// of the split kernel, truncated at theta_cut; Sec. 3: interpolated node
// table).  Everything here runs once per plan, in FP64 on the host.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "arkcos_internal.hpp"

namespace arkcos {

static thread_local std::string g_last_error;

TraceRange::TraceRange(const char *name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

// ARKCOS_LOG=1: one line of plan statistics on stderr per plan built.
static void log_plan(const Plan &P)
{
    const char *v = getenv("ARKCOS_LOG");
    if (!v || std::string(v) != "1") return;
    const int ngen_rings = (int)std::count(P.general_ring.begin(), P.general_ring.end(), 1);
    fprintf(stderr,
            "[arkcos] plan nside %d theta_cut %.6g rad ntab %d%s%s: rings %d circulant / %d "
            "general, ring pairs %zu, circulant tiles %zu, general tiles %zu (%zu staged "
            "chunks; shapes %d/%d/%d from %s), circulant rows %zu (weights %lld, %s), "
            "device bytes %lld\n",
            P.nside, P.desc.theta_cut, P.desc.ntab, P.desc.k_break > 0 ? " biased" : "",
            P.desc.ring_first > 0 ? " ring range" : "", P.nrings - ngen_rings, ngen_rings,
            P.pairs.size(), P.ctiles.size(), P.gtiles2.size(), P.gchunks.size(),
            P.tiles.gen_pixels, P.tiles.gen_quad_window, P.tiles.gen_pair_window,
            P.tile_source == 0 ? "defaults" : (P.tile_source == 1 ? "tuning cache" : "descriptor"),
            P.rows.size(), P.nweights, P.circ_form ? "matrix cores" : "vector FMAs",
            P.device_bytes);
}

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

void clear_error() { g_last_error.clear(); }

// HEALPix RING geometry of ring i (1-based) at resolution N (Gorski et al.
// 2005, the map format of Sec. 2).  Polar rings use the cancellation-free
// sin(theta) = sqrt(a (2 - a)) with a = 1 - |z| = i^2 / (3 N^2).
HostRing ring_geometry(int N, int i)
{
    HostRing g{};
    const double dN = N;
    const long long LN = N;
    if (i < N || i > 3 * N) {
        const int k = (i < N) ? i : 4 * N - i;                 // rings from the nearer pole
        const double a = (double)k * (double)k / (3.0 * dN * dN);
        g.z = (i < N) ? 1.0 - a : a - 1.0;
        g.s = std::sqrt(a * (2.0 - a));
        g.n = 4 * k;
        g.first = (i < N) ? 2LL * k * (k - 1) : 12LL * LN * LN - 2LL * k * (k + 1);
        g.two_o = 1;
    } else {
        g.z = 2.0 * (2.0 * dN - (double)i) / (3.0 * dN);
        g.s = std::sqrt((1.0 - g.z) * (1.0 + g.z));
        g.n = 4 * N;
        g.first = 2LL * LN * (LN - 1) + 4LL * LN * (i - N);
        g.two_o = ((i - N) % 2 == 0) ? 1 : 0;
    }
    g.theta = std::atan2(g.s, g.z);
    g.phi0 = g.two_o * M_PI / (double)g.n;
    return g;
}

// Node coordinates per radian of the first (or only) grid piece: the table
// index of angle theta is u0 = node_density theta on that piece.
static double node_density(const arkcos_plan_desc &d)
{
    if (d.k_break > 0) return d.k_break / d.theta_break;
    return (d.ntab - 1) / d.theta_cut;
}

// Coefficients of a short row's polynomial in y = (m mscale)^2 (the layout is
// described with DevPair).  sin^2 x = sum_k (-1)^(k+1) 2^(2k-1) x^(2k) / (2k)!
// with x^2 = s^2 y; theta^2 = (2 asin(d/2))^2 = sum_n 2 d^(2n) / (n^2 C(2n, n)).
static void short_row_poly(double A, double B, double xscale, int angle_mode, double density,
                           DevPair &p, DevPairD &pd)
{
    int e = 0;
    const double sc = std::frexp(xscale, &e);
    p.mscale = (float)std::ldexp(1.0, e);
    constexpr int K = 4;
    double d[K + 1];   // d^2 = A + B sin^2 x as a polynomial in y
    d[0] = A;
    double term = 1.0;
    for (int k = 1; k <= K; ++k) {
        term *= 4.0 * sc * sc / ((2.0 * k - 1.0) * (2.0 * k));   // 2^(2k) s^(2k) / (2k)!
        d[k] = (k % 2 ? 0.5 : -0.5) * B * term;
    }
    double out[K + 1] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (angle_mode != 0) {
        for (int k = 0; k < K; ++k) out[k] = d[k];
    } else {
        // u0^2 = density^2 sum_n b_n (d^2)^n, truncated at y^K; d^2 < 0.01 on
        // the rows of such a plan, so n <= 6 leaves terms below 1e-13
        double pw[K + 1] = {1.0, 0.0, 0.0, 0.0, 0.0};
        double binom = 1.0;   // C(2n, n)
        for (int n = 1; n <= 6; ++n) {
            double nx[K + 1] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int i = 0; i <= K; ++i)
                for (int j = 0; i + j <= K; ++j) nx[i + j] += pw[i] * d[j];
            for (int i = 0; i <= K; ++i) pw[i] = nx[i];
            binom = binom * (2.0 * n - 1.0) * (2.0 * n) / ((double)n * n);
            const double b = 2.0 / ((double)n * n * binom);
            for (int i = 0; i <= K; ++i) out[i] += b * pw[i];
        }
        for (int i = 0; i <= K; ++i) out[i] *= density * density;
    }
    pd.mscale = std::ldexp(1.0, e);
    for (int i = 0; i <= K; ++i) {
        p.sq[i] = (float)out[i];
        pd.sq[i] = out[i];
    }
}

DevPlanView Plan::view() const
{
    DevPlanView v{};
    v.rings = d_rings;
    v.pairs = d_pairs;
    v.table = d_table;
    v.pairs_d = d_pairs_d;
    v.groups = d_groups;
    v.rows = d_rows;
    v.wts = d_wts;
    v.ctiles = d_ctiles;
    v.gtiles2 = d_gtiles2;
    v.gchunks = d_gchunks;
    v.kctiles = d_kctiles;
    v.kw = d_kw;
    v.nctiles = (int)ctiles.size();
    v.ngtiles2 = (int)gtiles2.size();
    v.nkctiles = (int)kctiles.size();
    v.nkpart_circ = grid_kc;
    v.nrows = (int)rows.size();
    v.nrings = nrings;
    v.ntab = desc.ntab;
    v.npix = (int)npix;
    v.angle_mode = angle_mode;
    v.circ_mfma = circ_form;
    v.src_lo = src_hi >= 0 ? src_lo : 0;
    v.src_hi = src_hi >= 0 ? src_hi : nrings - 1;
    // node coordinate map: u0 = a0 theta, u = min(u0, r u0 + c)
    const bool biased = desc.k_break > 0;
    const double ih = node_density(desc);
    double r = 1.0, c0 = 0.0;
    if (biased) {
        const double a1 = (desc.ntab - 1 - desc.k_break) / (desc.theta_cut - desc.theta_break);
        r = a1 / ih;
        // c >= 0 since the first piece is at least as fine as the second;
        // clamping its rounding keeps u >= 0 (the node index and fraction of
        // a self-pair at theta = 0 must be 0)
        c0 = std::max(0.0, desc.k_break - desc.theta_break * a1);
    }
    v.biased = biased ? 1 : 0;
    v.inv_h_d = ih;
    v.bias_r_d = r;
    v.bias_c_d = c0;
    v.inv_h = (float)ih;
    v.k_break = biased ? desc.k_break : 0;
    v.bias_r = (float)r;
    // the FP32 gather's coarse coordinate from the break, v = r u0 - r k_break,
    // with the product of the FP32 r exact in FP64, so that v = 0 at u0 = k_break
    // to within one rounding
    v.bias_c = (float)(-(double)v.bias_r * (double)v.k_break);
    // theta = d (1 + d^2/24 + 3 d^4/640 + 5 d^6/7168 + 35 d^8/294912 + 63 d^10/2883584)
    const double c[6] = {1.0, 1.0 / 24.0, 3.0 / 640.0, 5.0 / 7168.0, 35.0 / 294912.0,
                         63.0 / 2883584.0};
    for (int k = 0; k < 6; ++k) v.u_coef[k] = (float)(ih * c[k]);
    return v;
}

// Longitude half-width (radians) of the disc on ring s around a pixel of
// ring r, from the haversine identity
//   sin^2(theta/2) = sin^2(dtheta/2) + sin_r sin_s sin^2(dphi/2);
// returns < 0 if the whole ring lies inside, and R < 0 means no pixel.
static double half_width(const HostRing &r, const HostRing &s, double theta_cut, bool *whole)
{
    const double hc = std::sin(0.5 * theta_cut);
    const double hd = std::sin(0.5 * (r.theta - s.theta));
    const double R = (hc * hc - hd * hd) / (r.s * s.s);
    *whole = false;
    if (R >= 1.0) {
        *whole = true;
        return M_PI;
    }
    if (R <= 0.0) return 0.0;
    return 2.0 * std::asin(std::sqrt(R));
}

// Reorder tiles (and their costs) by decreasing cost; ties keep their order.
template <class Tile>
static void sort_by_cost(std::vector<Tile> &tiles, std::vector<double> &cost)
{
    std::vector<size_t> order(tiles.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<Tile> t2(tiles.size());
    std::vector<double> c2(cost.size());
    for (size_t k = 0; k < order.size(); ++k) {
        t2[k] = tiles[order[k]];
        c2[k] = cost[order[k]];
    }
    tiles.swap(t2);
    cost.swap(c2);
}

// Staged chunks of every general tile, in tile order: for each source ring s
// of the tile, the union of its rings' row windows on s (the window of the
// first pixel's lower end to the last pixel's upper end, exactly as the kernel
// bounds a row: the windows move monotonically with the pixel), cut into
// chunks of kGenStage positions.  Rings whose rows all have empty windows
// are not staged.
static void build_gen_chunks(Plan &P)
{
    P.gchunks.clear();
    for (DevTile2 &t : P.gtiles2) {
        t.c_begin = (int)P.gchunks.size();
        for (int s = t.s_first; s <= t.s_last; ++s) {
            int lo_min = 0x7fffffff, hi_max = -0x7fffffff;
            const DevRing &S = P.dev_rings[s];
            for (int k = 0; k < t.nr; ++k) {
                const GenRing &q = t.q[k];
                if (q.len <= 0 || s < q.s_lo || s > q.s_hi) continue;
                const DevPair &pp = P.pairs[q.pb + s - q.s_lo];
                int lo, hi, dummy;
                pair_window(pp, S.n, t.j0, lo, dummy);
                pair_window(pp, S.n, t.j0 + q.len - 1, dummy, hi);
                lo_min = std::min(lo_min, lo);
                hi_max = std::max(hi_max, hi);
            }
            if (lo_min > hi_max) continue;
            const int sm = P.nrings - 1 - s;
            int mask = 0;
            if (P.src_hi >= 0 && (s < P.src_lo || s > P.src_hi)) mask |= 1;
            if (P.src_hi >= 0 && (sm < P.src_lo || sm > P.src_hi)) mask |= 2;
            for (int c0 = lo_min; c0 <= hi_max; c0 += kGenStage) {
                GenChunk c{};
                c.s = s;
                c.c0 = c0;
                c.cn = std::min(kGenStage, hi_max - c0 + 1);
                c.n = S.n;
                c.two_o = S.two_o;
                c.first = S.first;
                c.first_m = P.dev_rings[sm].first;
                c.mask = mask;
                P.gchunks.push_back(c);
            }
        }
        t.nchunks = (int)P.gchunks.size() - t.c_begin;
    }
}

// The general gather's tiles: adjacent general rings with narrow windows in
// groups of four (one lane per pixel at full length) or two (two lanes per
// pixel), each group over the same half-quadrant segments (tiles.gen_pixels
// pixels of each ring), so that a staged source row serves the whole group;
// rings with a very wide window, whose time is the loop's LDS reads, keep a
// tile of their own with more lanes per pixel, whose staged reads share more
// addresses.  Built from the general rings recorded by build_plan, so the
// tuner can re-tile a plan without rebuilding it.
void build_gen_tiles(Plan &P)
{
    const int seg = P.tiles.gen_pixels;
    const double quad_max = P.tiles.gen_quad_window;   // -1: never
    const double pair_max = P.tiles.gen_pair_window;
    const std::vector<int> &gring = P.gen_ring, &glanes = P.gen_lanes, &gflags = P.gen_flags;
    // a row is needed if its source ring or that ring's mirror is read
    int clip_lo = 0, clip_hi = P.nrings - 1;
    if (P.src_hi >= 0) {
        clip_lo = std::min(P.src_lo, P.nrings - 1 - P.src_hi);
        clip_hi = std::max(P.src_hi, P.nrings - 1 - P.src_lo);
    }
    std::vector<int> gwide(gring.size());
    for (size_t g = 0; g < gring.size(); ++g) {
        const double w = P.gen_wmax[g];
        gwide[g] = (pair_max < 0 || w > pair_max) ? 2 : ((quad_max < 0 || w > quad_max) ? 1 : 0);
    }
    P.gtiles2.clear();
    std::vector<double> cost;
    auto run_of = [&](size_t g, int n, int widest) {
        if (g + n > gring.size()) return false;
        for (int i = 0; i < n; ++i) {
            if (gwide[g + i] > widest) return false;
            if (i > 0 && gring[g + i] != gring[g + i - 1] + 1) return false;
        }
        return true;
    };
    for (size_t g = 0; g < gring.size();) {
        const int nr = run_of(g, 4, 0) ? 4 : (run_of(g, 2, 1) ? 2 : 1);
        int lanes = 0;
        for (int i = 0; i < nr; ++i) lanes = std::max(lanes, glanes[g + i]);
        for (int j0 = 0; j0 < lanes; j0 += seg) {
            DevTile2 t{};
            double c = 1.0;
            t.nr = nr;
            t.j0 = j0;
            t.s_first = 0x7fffffff;
            t.s_last = -1;
            for (int h = 0; h < kGenMaxRings; ++h) {
                GenRing &q = t.q[h];
                q.r = h < nr ? gring[g + h] : gring[g];
                q.len = h < nr ? std::max(0, std::min(seg, glanes[g + h] - j0)) : 0;
                q.flags = h < nr ? gflags[g + h] : 0;
                q.s_lo = 0;
                q.s_hi = -1;
                if (q.len > 0) {
                    const DevRing &dr = P.dev_rings[q.r];
                    const int s0 = P.pairs[dr.pair_begin].s;
                    // rows whose ring or mirror ring is read (all rows unless
                    // the source rings are restricted)
                    q.s_lo = std::max(s0, clip_lo);
                    q.s_hi = std::min(P.pairs[dr.pair_end - 1].s, clip_hi);
                    q.pb = dr.pair_begin + (q.s_lo - s0);
                    if (q.s_lo <= q.s_hi) {
                        t.s_first = std::min(t.s_first, q.s_lo);
                        t.s_last = std::max(t.s_last, q.s_hi);
                    }
                    c += P.ring_cost[q.r] * q.len;
                }
            }
            P.gtiles2.push_back(t);
            cost.push_back(c);
        }
        g += nr;
    }
    sort_by_cost(P.gtiles2, cost);
    P.gtile2_cost = cost;
    build_gen_chunks(P);
}

static int build_plan(Plan &P)
{
    const int N = P.nside;
    const double tc = P.desc.theta_cut;
    P.rings.resize(P.nrings);
    P.dev_rings.resize(P.nrings);
    for (int i = 1; i <= P.nrings; ++i) P.rings[i - 1] = ring_geometry(N, i);

    // Source rings of each output ring: a contiguous run, since colatitude
    // grows with the ring index.  A small slack admits rings whose nearest
    // pixel sits on the cut; the per-pair test on the device decides.
    const double slack = 1e-12 + 1e-9 * tc;
    P.pairs.clear();
    P.pairs_d.clear();
    P.candidates = 0;
    std::vector<double> &ring_cost = P.ring_cost;
    ring_cost.assign(P.nrings, 0.0);
    for (int r = 0; r < P.nrings; ++r) {
        const HostRing &R = P.rings[r];
        DevRing &dr = P.dev_rings[r];
        dr.n = R.n;
        dr.first = (int)R.first;
        dr.two_o = R.two_o;
        dr.pair_begin = (int)P.pairs.size();
        int lo = r, hi = r;
        while (lo > 0 && std::fabs(P.rings[lo - 1].theta - R.theta) < tc + slack) --lo;
        while (hi < P.nrings - 1 && std::fabs(P.rings[hi + 1].theta - R.theta) < tc + slack) ++hi;
        double per_pixel = 0.0;
        for (int s = lo; s <= hi; ++s) {
            const HostRing &S = P.rings[s];
            bool whole = false;
            const double dphi = half_width(R, S, tc, &whole);
            DevPair p{};
            DevPairD pd{};
            const double dA = 2.0 * std::sin(0.5 * (R.theta - S.theta));
            pd.A = dA * dA;
            pd.B = 4.0 * R.s * S.s;
            pd.xscale = M_PI / (2.0 * (double)R.n * (double)S.n);
            p.A = (float)pd.A;
            p.B = (float)pd.B;
            p.xscale = (float)pd.xscale;
            short_row_poly(pd.A, pd.B, pd.xscale, P.angle_mode, node_density(P.desc), p, pd);
            p.a = (float)((double)S.n / (double)R.n);
            p.b = (float)(0.5 * R.two_o * (double)S.n / (double)R.n - 0.5 * S.two_o);
            // window half-width in source pixels, widened to cover FP32 rounding
            // of the centre; at most half the ring, so that every pixel of the
            // window lies its shorter way round from the centre.  Membership is
            // the exact test |m| <= mcut, with |m| < X = dphi n_r n_s / pi.
            double w = dphi * S.n / (2.0 * M_PI);
            w = std::min(w * (1.0 + 1e-5) + 0.02, 0.5 * (double)S.n);
            if (whole) {
                p.mode = kPairWhole | kPairLongSin;
                p.w = 0.0f;
                p.mcut = 0x7fffffff;
                per_pixel += S.n;
            } else {
                const double X = dphi * (double)R.n * (double)S.n / M_PI;
                p.mcut = (int)std::ceil(X) - 1;
                // largest |dphi/2| a candidate can have: (w + 1) pixels of ring s
                const double xmax = (w + 1.0) * M_PI / (double)S.n;
                p.mode = xmax > (P.angle_mode == 0 ? kShortXMaxMode0 : kShortXMax) ? kPairLongSin : 0;
                p.w = (float)w;
                per_pixel += std::floor(2.0 * w) + 1.0;
            }
            p.s = s;
            P.pairs.push_back(p);
            P.pairs_d.push_back(pd);
        }
        dr.pair_end = (int)P.pairs.size();
        ring_cost[r] = per_pixel;
        P.candidates += (long long)std::llround(per_pixel * R.n);
    }

    std::vector<double> cost;

    // Ring classes.  A belt ring whose source rings are all belt rings (4N
    // pixels each, windows narrower than a ring) is circulant: the weight of
    // (r, j; s, j') depends on j' - j only.  Every other ring (polar caps and
    // belt rings whose disc reaches a cap) is general.  The classes are kept
    // mirror-symmetric (ring i and ring 4N - i), since the general kernel
    // evaluates each weight for a ring and its mirror image together.
    const int nbelt = 4 * N;
    std::vector<char> general(P.nrings, 1);
    for (int r = 0; r < P.nrings; ++r) {
        if (P.rings[r].n != nbelt || r < N - 1 || r > 3 * N - 1) continue;
        bool circ = true;
        for (int k = P.dev_rings[r].pair_begin; k < P.dev_rings[r].pair_end; ++k) {
            const DevPair &pp = P.pairs[k];
            const bool whole = (pp.mode & kPairWhole) != 0;
            if (whole || P.rings[pp.s].n != nbelt) circ = false;

        }
        general[r] = circ ? 0 : 1;
    }
    for (int r = 0; r < P.nrings; ++r) {
        const int rm = P.nrings - 1 - r;
        const char g = general[r] | general[rm];
        general[r] = general[rm] = g;
    }
    P.general_ring = general;
    // output rings of a ring-range plan (0-based, inclusive); all rings otherwise
    const int out_lo = P.desc.ring_first > 0 ? P.desc.ring_first - 1 : 0;
    const int out_hi = P.desc.ring_first > 0 ? P.desc.ring_last - 1 : P.nrings - 1;
    auto in_range = [&](int r) { return r >= out_lo && r <= out_hi; };

    // Circulant groups of up to kGroupRings consecutive circulant output rings,
    // each with the union of its rings' source rows and tap ranges.
    P.groups.clear();
    P.rows.clear();
    P.nweights = 0;
    P.max_taps = 0;
    for (int r = 0; r < P.nrings;) {
        if (general[r] || !in_range(r)) { ++r; continue; }
        DevGroup G{};
        G.r0 = r;
        G.nr = 0;
        while (r < P.nrings && !general[r] && in_range(r) && G.nr < kGroupRings) { ++G.nr; ++r; }
        G.row_begin = (int)P.rows.size();
        int s_lo = 1 << 30, s_hi = -1;
        for (int i = 0; i < G.nr; ++i) {
            const DevRing &dr = P.dev_rings[G.r0 + i];
            s_lo = std::min(s_lo, P.pairs[dr.pair_begin].s);
            s_hi = std::max(s_hi, P.pairs[dr.pair_end - 1].s);
        }
        for (int sr = s_lo; sr <= s_hi; ++sr) {
            if (P.src_hi >= 0 && (sr < P.src_lo || sr > P.src_hi)) continue;   // not read
            int k_lo = 1 << 30, k_hi = -(1 << 30);
            for (int i = 0; i < G.nr; ++i) {
                const DevRing &dr = P.dev_rings[G.r0 + i];
                const int kk = dr.pair_begin + (sr - P.pairs[dr.pair_begin].s);
                if (kk < dr.pair_begin || kk >= dr.pair_end) continue;
                int lo, hi;
                pair_window(P.pairs[kk], nbelt, 0, lo, hi);
                k_lo = std::min(k_lo, lo);
                k_hi = std::max(k_hi, hi);
            }
            if (k_hi < k_lo) continue;
            // a row wider than one staging pass becomes consecutive rows of at
            // most kCircMaxTaps taps each
            for (int k0 = k_lo; k0 <= k_hi; k0 += kCircMaxTaps) {
                DevRow row{};
                row.s = sr;
                row.first_s = (int)P.rings[sr].first;
                row.k_lo = k0;
                row.ntaps = std::min(kCircMaxTaps, k_hi - k0 + 1);
                row.w_off = (int)std::min<long long>(P.nweights, 0x7fffffffLL);
                row.g = (int)P.groups.size();
                P.nweights += (long long)row.ntaps * kGroupRings;
                P.max_taps = std::max(P.max_taps, row.ntaps);
                P.rows.push_back(row);
            }
        }
        G.row_end = (int)P.rows.size();
        P.groups.push_back(G);
    }
    if (P.nweights > 0x7fffffffLL) return fail(ARKCOS_EUNSUPPORTED, "circulant weight table too large");
    // Matrix cores for rows averaging kCircMfmaTaps taps or more; the test hook
    // ARKCOS_CIRC_FORM=valu or =mfma at plan creation forces either form.
    P.circ_form = !P.rows.empty() &&
                  P.nweights >= (long long)kCircMfmaTaps * kGroupRings * (long long)P.rows.size();
    if (const char *cf = getenv("ARKCOS_CIRC_FORM")) {
        if (std::string(cf) == "valu") P.circ_form = 0;
        if (std::string(cf) == "mfma") P.circ_form = 1;
    }

    // Circulant tiles: kCircSeg consecutive pixels of every ring of a group.
    P.ctiles.clear();
    cost.clear();
    for (int g = 0; g < (int)P.groups.size(); ++g) {
        double taps = 0.0;
        for (int q = P.groups[g].row_begin; q < P.groups[g].row_end; ++q) taps += P.rows[q].ntaps;
        for (int j0 = 0; j0 < nbelt; j0 += kCircSeg) {
            DevTile t{};
            t.r = g;
            t.j0 = j0;
            t.len = std::min(kCircSeg, nbelt - j0);
            P.ctiles.push_back(t);
            cost.push_back(taps * kGroupRings * t.len);
        }
    }
    sort_by_cost(P.ctiles, cost);
    P.ctile_cost = cost;

    // General tiles: up to kGenLanes pixels j <= jbar = n/4 - 2o - j of the
    // first quadrant of a general ring of the northern half (equator
    // included); each pixel yields its four quarter turns, their reflections
    // about phi = pi/4 and the mirror images of all eight.
    P.gtiles.clear();
    cost.clear();
    // test hook: every general tile takes the int32 numerator path
    const char *fim = getenv("ARKCOS_FORCE_INT_NUMERATOR");
    const bool force_int_m = fim && std::string(fim) == "1";
    P.gen_ring.clear();
    P.gen_lanes.clear();
    P.gen_flags.clear();
    P.gen_wmax.clear();
    for (int r = 0; r <= P.nrings - 1 - r; ++r) {
        if (!general[r]) continue;
        const int rm = P.nrings - 1 - r;
        if (!in_range(r) && !in_range(rm)) continue;
        const int quarter = P.rings[r].n / 4;
        const int lanes = (P.rings[r].two_o ? (quarter - 1) / 2 : quarter / 2) + 1;
        // |m| = 2 n_r |c - j'| over the candidates, including those a wave
        // runs past a lane's window (at most 64 lanes per pixel, +4 for the
        // spread of windows across a wave)
        int flags = force_int_m ? (kTileIntM | kTileLongSin) : 0;
        if (!in_range(r)) flags |= kTileSkipNorth;
        if (!in_range(rm)) flags |= kTileSkipSouth;
        for (int k = P.dev_rings[r].pair_begin; k < P.dev_rings[r].pair_end; ++k) {
            const DevPair &pp = P.pairs[k];
            if (pp.mode & kPairLongSin) flags |= kTileLongSin;
            const double W = (pp.mode & kPairWhole) ? 0.5 * P.rings[pp.s].n + 1.0 : pp.w + 1.0;
            if (2.0 * P.rings[r].n * (W + 70.0) >= 16777216.0) flags |= kTileIntM | kTileLongSin;
        }
        for (int j0 = 0; j0 < lanes; j0 += kGenLanes) {
            DevTile t{};
            t.r = r;
            t.j0 = j0;
            t.len = std::min(kGenLanes, lanes - j0);
            t.flags = flags;
            P.gtiles.push_back(t);
            cost.push_back(ring_cost[r] * t.len + 1.0);
        }
        // widest source window of the ring's rows, in source positions
        double wmax = 0.0;
        for (int k = P.dev_rings[r].pair_begin; k < P.dev_rings[r].pair_end; ++k) {
            const DevPair &pp = P.pairs[k];
            wmax = std::max(wmax, (pp.mode & kPairWhole) ? (double)P.rings[pp.s].n : 2.0 * pp.w + 1.0);
        }
        P.gen_ring.push_back(r);
        P.gen_lanes.push_back(lanes);
        P.gen_flags.push_back(flags);
        P.gen_wmax.push_back(wmax);
    }
    sort_by_cost(P.gtiles, cost);
    P.gtile_cost = cost;
    build_gen_tiles(P);

    // Circulant knot-gradient tiles: kKnotSeg consecutive pixels of every
    // ring of a group.
    P.kctiles.clear();
    cost.clear();
    for (int g = 0; g < (int)P.groups.size(); ++g) {
        double taps = 0.0;
        for (int q = P.groups[g].row_begin; q < P.groups[g].row_end; ++q) taps += P.rows[q].ntaps;
        for (int j0 = 0; j0 < nbelt; j0 += kKnotSeg) {
            DevTile t{};
            t.r = g;
            t.j0 = j0;
            t.len = std::min(kKnotSeg, nbelt - j0);
            P.kctiles.push_back(t);
            cost.push_back(taps * t.len + 1.0);
        }
    }
    sort_by_cost(P.kctiles, cost);
    return ARKCOS_OK;
}

// Exact in-disc pair count of one map.  For output pixel j of ring r and
// source ring s the pixels inside the disc are the integers j' in the open
// interval (c - W, c + W), c = ((2j + 2o_r) n_s / n_r - 2o_s) / 2, with
// W = dphi_max n_s / (2 pi).  A rotation by a quarter turn maps pixel j to
// j + n_r/4 and shifts c by n_s/4, so a quarter of each ring is counted.
// Exact in-disc pairs of output rings r0, r0 + step, ... (all, and circulant).
static void count_pairs_rings(const Plan &P, int r0, int step, unsigned long long *all,
                              unsigned long long *circ)
{
    const double tc = P.desc.theta_cut;
    unsigned long long total = 0, circ_total = 0;
    const int out_lo = P.desc.ring_first > 0 ? P.desc.ring_first - 1 : 0;
    const int out_hi = P.desc.ring_first > 0 ? P.desc.ring_last - 1 : P.nrings - 1;
    for (int r = r0; r < P.nrings; r += step) {
        if (r < out_lo || r > out_hi) continue;
        const HostRing &R = P.rings[r];
        const DevRing &dr = P.dev_rings[r];
        unsigned long long ring_total = 0;
        for (int k = dr.pair_begin; k < dr.pair_end; ++k) {
            const HostRing &S = P.rings[P.pairs[k].s];
            bool whole = false;
            const double dphi = half_width(R, S, tc, &whole);
            if (whole) {
                ring_total += (unsigned long long)S.n * (unsigned long long)R.n;
                continue;
            }
            const double W = dphi * S.n / (2.0 * M_PI);
            const int quarter = R.n / 4;
            const bool circulant = (R.n == S.n);
            const int jn = circulant ? 1 : quarter;
            unsigned long long part = 0;
            for (int j = 0; j < jn; ++j) {
                const double c = 0.5 * ((2.0 * j + R.two_o) * (double)S.n / (double)R.n - S.two_o);
                long long cnt = (long long)std::ceil(c + W) - (long long)std::floor(c - W) - 1;
                if (cnt < 0) cnt = 0;
                if (cnt > S.n) cnt = S.n;
                part += (unsigned long long)cnt;
            }
            ring_total += circulant ? part * (unsigned long long)R.n : 4ULL * part;
        }
        total += ring_total;
        if (!P.general_ring[r]) circ_total += ring_total;
    }
    *all = total;
    *circ = circ_total;
}

// The rings are counted on host threads (interleaved, so each thread gets a
// share of the large belt and small polar rings); integer sums, so the
// result does not depend on the thread count.
static unsigned long long count_pairs(const Plan &P, unsigned long long *circ_total)
{
    const int nt = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<unsigned long long> all(nt, 0), circ(nt, 0);
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t)
        pool.emplace_back(count_pairs_rings, std::cref(P), t, nt, &all[t], &circ[t]);
    count_pairs_rings(P, 0, nt, &all[0], &circ[0]);
    for (std::thread &th : pool) th.join();
    unsigned long long total = 0;
    *circ_total = 0;
    for (int t = 0; t < nt; ++t) {
        total += all[t];
        *circ_total += circ[t];
    }
    return total;
}

// Node table by Clenshaw's backward recurrence for sum_l c_l P_l(x) with
// c_l = (2l+1) b_l / (4 pi): with alpha_k = (2k+1) x / (k+1) and
// beta_k = -k / (k+1), y_k = c_k + alpha_k y_{k+1} + beta_{k+1} y_{k+2},
// y_{L+1} = y_{L+2} = 0, and the sum is y_0.
static void tabulate_at(const double *bl, int lmax, const double *theta, int n, double *out)
{
    const double inv4pi = 1.0 / (4.0 * M_PI);
    for (int k = 0; k < n; ++k) {
        const double x = std::cos(theta[k]);
        double y1 = 0.0, y2 = 0.0;  // y_{l+1}, y_{l+2}
        for (int l = lmax; l >= 0; --l) {
            const double alpha = (2.0 * l + 1.0) * x / (l + 1.0);
            const double beta_next = -(l + 1.0) / (l + 2.0);
            const double y = (2.0 * l + 1.0) * bl[l] * inv4pi + alpha * y1 + beta_next * y2;
            y2 = y1;
            y1 = y;
        }
        out[k] = y1;
    }
}

// Node angles of the grid of a plan descriptor (uniform, or two pieces that
// are each uniform: the biased table of Sec. 3).
static void grid_nodes(double tc, int ntab, double tb, int kb, double *out)
{
    if (kb == 0) {
        const double h = tc / (double)(ntab - 1);
        for (int k = 0; k < ntab; ++k) out[k] = k * h;
    } else {
        for (int k = 0; k <= kb; ++k) out[k] = tb * ((double)k / kb);
        for (int k = kb + 1; k < ntab; ++k)
            out[k] = tb + (tc - tb) * ((double)(k - kb) / (ntab - 1 - kb));
        out[kb] = tb;
    }
    out[ntab - 1] = tc;
}

// Validity of a node grid; EINVAL with a message, else ARKCOS_OK.
static int check_grid(double tc, int ntab, double tb, int kb)
{
    if (tb == 0.0 && kb == 0) return ARKCOS_OK;
    if (!(tb > 0.0 && tb < tc))
        return fail(ARKCOS_EINVAL, "theta_break must lie in (0, theta_cut), or be 0 with k_break 0");
    if (kb < 1 || kb > ntab - 2)
        return fail(ARKCOS_EINVAL, "k_break must lie in 1..ntab-2, or be 0 with theta_break 0");
    if (tb / kb > (tc - tb) / (ntab - 1 - kb) * (1.0 + 1e-12))
        return fail(ARKCOS_EINVAL, "the first piece of a biased grid must be at least as fine "
                                   "as the second");
    return ARKCOS_OK;
}

static void free_device(Plan &P)
{
    if (P.device >= 0) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(P.device);
        (void)hipDeviceSynchronize();
        (void)hipFree(P.d_rings);
        (void)hipFree(P.d_pairs);
        (void)hipFree(P.d_pairs_d);
        (void)hipFree(P.d_groups);
        (void)hipFree(P.d_rows);
        (void)hipFree(P.d_wts);
        (void)hipFree(P.d_ctiles);
        (void)hipFree(P.d_gtiles2);
        (void)hipFree(P.d_gchunks);
        (void)hipFree(P.d_kctiles);
        (void)hipFree(P.d_kw);
        (void)hipFree(P.d_view);
        (void)hipFree(P.d_table);
        (void)hipFree(P.d_counter);
        (void)hipFree(P.d_kpart);
        (void)hipSetDevice(cur);
    }
    P.d_rings = nullptr;
    P.d_pairs = nullptr;
    P.d_pairs_d = nullptr;
    P.d_groups = nullptr;
    P.d_rows = nullptr;
    P.d_wts = nullptr;
    P.d_ctiles = nullptr;
    P.d_gtiles2 = nullptr;
    P.d_gchunks = nullptr;
    P.gen_tile_bytes = 0;
    P.d_kctiles = nullptr;
    P.d_kw = nullptr;
    P.d_view = nullptr;
    P.d_table = nullptr;
    P.d_counter = nullptr;
    P.d_kpart = nullptr;
}

template <class T>
static int upload(T **dst, const std::vector<T> &src, long long *bytes)
{
    const size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
    if (hipMalloc((void **)dst, n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ARKCOS_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    *bytes += (long long)n;
    if (!src.empty()) ARKCOS_HIP_CHECK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T),
                                                 hipMemcpyHostToDevice));
    return ARKCOS_OK;
}

int upload_gen_tiles(Plan &P)
{
    (void)hipFree(P.d_gtiles2);
    (void)hipFree(P.d_gchunks);
    P.d_gtiles2 = nullptr;
    P.d_gchunks = nullptr;
    P.device_bytes -= P.gen_tile_bytes;
    P.gen_tile_bytes = 0;
    int rc = upload(&P.d_gtiles2, P.gtiles2, &P.gen_tile_bytes);
    if (!rc) rc = upload(&P.d_gchunks, P.gchunks, &P.gen_tile_bytes);
    P.device_bytes += P.gen_tile_bytes;
    if (rc) return rc;
    const DevPlanView v = P.view();
    ARKCOS_HIP_CHECK(hipMemcpy(P.d_view, &v, sizeof(v), hipMemcpyHostToDevice));
    return ARKCOS_OK;
}

static int write_table_host(Plan &P)
{
    std::vector<float> t(P.desc.ntab);
    for (int k = 0; k < P.desc.ntab; ++k) t[k] = (float)(P.omega * P.ktab[k]);
    ARKCOS_HIP_CHECK(hipMemcpy(P.d_table, t.data(), t.size() * sizeof(float),
                               hipMemcpyHostToDevice));
    int rc = launch_build_weights(P, nullptr);
    if (rc) return rc;
    ARKCOS_HIP_CHECK(hipStreamSynchronize(nullptr));
    return ARKCOS_OK;
}

static int to_device(Plan &P)
{
    if (getenv("ARKCOS_FAULT") && std::string(getenv("ARKCOS_FAULT")) == "alloc")
        return fail(ARKCOS_ENOMEM, "allocation failure forced by ARKCOS_FAULT=alloc");
    ARKCOS_HIP_CHECK(hipGetDevice(&P.device));
    size_t lds = 0;
    int rc = device_lds_limit(P.device, &lds);
    if (rc) return rc;
    if ((size_t)P.desc.ntab * sizeof(float) > lds)
        return fail(ARKCOS_EUNSUPPORTED, "node table of " + std::to_string(P.desc.ntab) +
                                             " FP32 values exceeds the workgroup LDS limit of " +
                                             std::to_string(lds) + " bytes");
    P.device_bytes = 0;
    if ((rc = upload(&P.d_rings, P.dev_rings, &P.device_bytes))) return rc;
    if ((rc = upload(&P.d_pairs, P.pairs, &P.device_bytes))) return rc;
    if ((rc = upload(&P.d_pairs_d, P.pairs_d, &P.device_bytes))) return rc;
    if ((rc = upload(&P.d_groups, P.groups, &P.device_bytes))) return rc;
    if ((rc = upload(&P.d_rows, P.rows, &P.device_bytes))) return rc;
    if ((rc = upload(&P.d_ctiles, P.ctiles, &P.device_bytes))) return rc;
    P.gen_tile_bytes = 0;
    rc = upload(&P.d_gtiles2, P.gtiles2, &P.gen_tile_bytes);
    if (!rc) rc = upload(&P.d_gchunks, P.gchunks, &P.gen_tile_bytes);
    P.device_bytes += P.gen_tile_bytes;
    if (rc) return rc;
    if ((rc = upload(&P.d_wts, std::vector<float>((size_t)std::max<long long>(P.nweights, 1), 0.0f),
                     &P.device_bytes)))
        return rc;
    if ((rc = upload(&P.d_table, std::vector<float>(P.desc.ntab, 0.0f), &P.device_bytes)))
        return rc;
    if ((rc = upload(&P.d_counter, std::vector<unsigned int>(4, 0u), &P.device_bytes))) return rc;
    if ((rc = prepare_launches(P))) return rc;
    if ((P.desc.flags & ARKCOS_PLAN_LEARNABLE) && P.desc.ntab <= ARKCOS_MAX_GRAD_NTAB) {
        std::vector<double> z((size_t)P.grid * P.desc.ntab, 0.0);
        if ((rc = upload(&P.d_kpart, z, &P.device_bytes))) return rc;
        if ((rc = upload(&P.d_kctiles, P.kctiles, &P.device_bytes))) return rc;
        if ((rc = upload(&P.d_kw, std::vector<double>((size_t)std::max<long long>(P.nweights, 1), -1.0),
                         &P.device_bytes)))
            return rc;
        if ((rc = launch_build_knotw(P, nullptr))) return rc;
        ARKCOS_HIP_CHECK(hipStreamSynchronize(nullptr));
    }
    {
        std::vector<DevPlanView> v(1, P.view());
        if ((rc = upload(&P.d_view, v, &P.device_bytes))) return rc;
    }
    if (!P.ktab.empty()) {
        if ((rc = write_table_host(P))) return rc;
        P.knots_set = true;
    }
    return ARKCOS_OK;
}

// Descriptor-derived fields of a plan (before tiles and build).
static void init_plan(Plan &P, const arkcos_plan_desc &d)
{
    P.desc = d;
    P.desc.ktab = nullptr;
    P.nside = d.nside;
    P.nrings = 4 * d.nside - 1;
    P.npix = 12LL * d.nside * d.nside;
    P.omega = 4.0 * M_PI / (double)P.npix;
    P.threads = forward_threads();
    P.host_only = (d.flags & ARKCOS_PLAN_HOST_ONLY) != 0;
    P.angle_mode = d.theta_cut <= 0.1 ? 0 : (d.theta_cut <= 0.5 ? 1 : 2);
    if (d.ktab) P.ktab.assign(d.ktab, d.ktab + d.ntab);
}

static int build_and_upload(Plan &P)
{
    int rc;
    try {
        rc = build_plan(P);
    } catch (const std::bad_alloc &) {
        rc = fail(ARKCOS_ENOMEM, "host allocation failed while building the plan");
    }
    if (rc == ARKCOS_OK && !P.host_only) rc = to_device(P);
    return rc;
}

static void destroy_plan(Plan *P)
{
    if (P->adj) destroy_plan(P->adj);
    free_device(*P);
    delete P;
}

}  // namespace arkcos

using namespace arkcos;

extern "C" {

const char *arkcos_last_error(void) { return arkcos::g_last_error.c_str(); }

const char *arkcos_status_string(int status)
{
    switch (status) {
        case ARKCOS_OK: return "ARKCOS_OK";
        case ARKCOS_EINVAL: return "ARKCOS_EINVAL: invalid argument";
        case ARKCOS_ENOMEM: return "ARKCOS_ENOMEM: out of memory";
        case ARKCOS_EDEVICE: return "ARKCOS_EDEVICE: HIP device error";
        case ARKCOS_EUNSUPPORTED: return "ARKCOS_EUNSUPPORTED: unsupported configuration";
        case ARKCOS_ESTATE: return "ARKCOS_ESTATE: object not in the required state";
        default: return "ARKCOS: unknown status";
    }
}

int arkcos_version(void) { return 10000; }

int arkcos_tabulate_legendre(const double *b_l, int lmax, double theta_cut, int ntab,
                             double *ktab_out)
{
    clear_error();
    if (!b_l || !ktab_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (lmax < 0) return fail(ARKCOS_EINVAL, "lmax must be >= 0");
    if (ntab < 2) return fail(ARKCOS_EINVAL, "ntab must be >= 2");
    if (!(theta_cut > 0.0) || theta_cut > M_PI)
        return fail(ARKCOS_EINVAL, "theta_cut must lie in (0, pi]");
    std::vector<double> th(ntab);
    const double h = theta_cut / (double)(ntab - 1);
    for (int k = 0; k < ntab; ++k) th[k] = k * h;
    tabulate_at(b_l, lmax, th.data(), ntab, ktab_out);
    return ARKCOS_OK;
}

int arkcos_tabulate_legendre_at(const double *b_l, int lmax, const double *theta, int n,
                                double *out)
{
    clear_error();
    if (!b_l || !theta || !out) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (lmax < 0) return fail(ARKCOS_EINVAL, "lmax must be >= 0");
    if (n < 1) return fail(ARKCOS_EINVAL, "n must be >= 1");
    for (int k = 0; k < n; ++k)
        if (!(theta[k] >= 0.0 && theta[k] <= M_PI))
            return fail(ARKCOS_EINVAL, "angles must lie in [0, pi]");
    tabulate_at(b_l, lmax, theta, n, out);
    return ARKCOS_OK;
}

int arkcos_grid_nodes(double theta_cut, int ntab, double theta_break, int k_break,
                      double *theta_out)
{
    clear_error();
    if (!theta_out) return fail(ARKCOS_EINVAL, "NULL pointer");
    if (ntab < 2) return fail(ARKCOS_EINVAL, "ntab must be >= 2");
    if (!(theta_cut > 0.0) || theta_cut > M_PI)
        return fail(ARKCOS_EINVAL, "theta_cut must lie in (0, pi]");
    int rc = check_grid(theta_cut, ntab, theta_break, k_break);
    if (rc) return rc;
    grid_nodes(theta_cut, ntab, theta_break, k_break, theta_out);
    return ARKCOS_OK;
}

int arkcos_ring_info(int nside, int ring, double *z, double *sin_theta, int *npix_ring,
                     long long *first_pixel, double *phi0)
{
    clear_error();
    if (nside < 1 || nside > ARKCOS_MAX_NSIDE)
        return fail(ARKCOS_EINVAL, "nside out of range");
    if (ring < 1 || ring > 4 * nside - 1) return fail(ARKCOS_EINVAL, "ring out of range");
    const HostRing g = ring_geometry(nside, ring);
    if (z) *z = g.z;
    if (sin_theta) *sin_theta = g.s;
    if (npix_ring) *npix_ring = g.n;
    if (first_pixel) *first_pixel = g.first;
    if (phi0) *phi0 = g.phi0;
    return ARKCOS_OK;
}

int arkcos_plan_create(const arkcos_plan_desc *desc, arkcos_plan_t *out)
{
    clear_error();
    TraceRange tr("arkcos_plan_create");
    if (!out) return fail(ARKCOS_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (!desc) return fail(ARKCOS_EINVAL, "NULL descriptor");
    if (desc->nside < 1 || desc->nside > ARKCOS_MAX_NSIDE)
        return fail(ARKCOS_EINVAL, "nside must lie in 1.." + std::to_string(ARKCOS_MAX_NSIDE));
    if (!(desc->theta_cut > 0.0) || desc->theta_cut > M_PI)
        return fail(ARKCOS_EINVAL, "theta_cut must lie in (0, pi]");
    if (desc->ntab < 2) return fail(ARKCOS_EINVAL, "ntab must be >= 2");
    if (desc->max_batch < 1) return fail(ARKCOS_EINVAL, "max_batch must be >= 1");
    if (int rc = check_tiles(desc->tiles)) return rc;
    if (!desc->ktab && !(desc->flags & ARKCOS_PLAN_LEARNABLE))
        return fail(ARKCOS_EINVAL, "ktab may be NULL only for a learnable plan");
    if (desc->flags & ~(ARKCOS_PLAN_HOST_ONLY | ARKCOS_PLAN_LEARNABLE))
        return fail(ARKCOS_EINVAL, "unknown flag bits");
    if (int rc = check_grid(desc->theta_cut, desc->ntab, desc->theta_break, desc->k_break))
        return rc;
    if (!(desc->ring_first == 0 && desc->ring_last == 0) &&
        !(desc->ring_first >= 1 && desc->ring_first <= desc->ring_last &&
          desc->ring_last <= 4 * desc->nside - 1))
        return fail(ARKCOS_EINVAL, "ring range must be 0, 0 or 1 <= ring_first <= ring_last <= "
                                   "4 nside - 1");
    const long long npix = 12LL * desc->nside * desc->nside;
    if ((long long)desc->max_batch * npix > 0x7fffffffLL * 4)
        return fail(ARKCOS_EUNSUPPORTED, "max_batch * Npix too large");

    Plan *P = new (std::nothrow) Plan();
    if (!P) return fail(ARKCOS_ENOMEM, "host allocation failed");
    init_plan(*P, *desc);
    if (int rc = resolve_tiles(*desc, &P->tiles, &P->tile_source)) {
        delete P;
        return rc;
    }
    int rc = build_and_upload(*P);
    if (rc == ARKCOS_OK && desc->ring_first > 0) {
        // The adjoint of a ring range R: output rings are every source ring of
        // R (the rings within theta_cut of it), source rings are R itself,
        // whose images outside R count as zero.  The same gathers then give
        // A^T g for g supported on R, by the symmetry of the operator.
        int e1 = P->nrings, e2 = -1;
        for (int r = desc->ring_first - 1; r <= desc->ring_last - 1; ++r) {
            const DevRing &dr = P->dev_rings[r];
            e1 = std::min(e1, P->pairs[dr.pair_begin].s);
            e2 = std::max(e2, P->pairs[dr.pair_end - 1].s);
        }
        Plan *A = new (std::nothrow) Plan();
        if (!A) {
            rc = fail(ARKCOS_ENOMEM, "host allocation failed");
        } else {
            arkcos_plan_desc ad = *desc;
            ad.ring_first = e1 + 1;
            ad.ring_last = e2 + 1;
            ad.flags &= ~ARKCOS_PLAN_LEARNABLE;   // gathers only
            init_plan(*A, ad);
            A->tiles = P->tiles;
            A->tile_source = P->tile_source;
            A->src_lo = desc->ring_first - 1;
            A->src_hi = desc->ring_last - 1;
            P->adj = A;
            rc = build_and_upload(*A);
        }
    }
    if (rc != ARKCOS_OK) {
        destroy_plan(P);
        return rc;
    }
    log_plan(*P);
    *out = reinterpret_cast<arkcos_plan_t>(P);
    return ARKCOS_OK;
}

int arkcos_plan_destroy(arkcos_plan_t plan)
{
    clear_error();
    if (!plan) return ARKCOS_OK;
    destroy_plan(reinterpret_cast<Plan *>(plan));
    return ARKCOS_OK;
}

int arkcos_plan_get_info(arkcos_plan_t plan, arkcos_plan_info *info)
{
    clear_error();
    if (!plan || !info) return fail(ARKCOS_EINVAL, "NULL pointer");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    info->nside = P->nside;
    info->nrings = P->nrings;
    info->npix = P->npix;
    info->ring_pairs = (long long)P->pairs.size();
    info->tiles = (long long)(P->ctiles.size() + P->gtiles.size());
    info->candidates = P->candidates;
    info->omega = P->omega;
    info->ntab = P->desc.ntab;
    info->tile_shapes = P->tiles;
    info->tile_source = P->tile_source;
    info->flags = P->desc.flags;
    info->threads_per_block = P->threads;
    info->device_bytes = P->device_bytes;
    int circ = 0;
    for (const DevGroup &g : P->groups) circ += g.nr;
    const int nout = P->desc.ring_first > 0 ? P->desc.ring_last - P->desc.ring_first + 1
                                            : P->nrings;
    info->circulant_rings = circ;
    info->general_rings = nout - circ;
    info->ring_first = P->desc.ring_first;
    info->ring_last = P->desc.ring_last;
    info->adjoint_ring_first = P->adj ? P->adj->desc.ring_first : 0;
    info->adjoint_ring_last = P->adj ? P->adj->desc.ring_last : 0;
    info->circulant_tiles = (long long)P->ctiles.size();
    info->general_tiles = (long long)P->gtiles.size();
    info->weights = P->nweights;
    info->circ_form = P->circ_form;
    info->theta_break = P->desc.theta_break;
    info->k_break = P->desc.k_break;
    return ARKCOS_OK;
}

int arkcos_plan_pair_count(arkcos_plan_t plan, unsigned long long *pairs)
{
    clear_error();
    if (!plan || !pairs) return fail(ARKCOS_EINVAL, "NULL pointer");
    Plan *P = reinterpret_cast<Plan *>(plan);
    if (!P->pairs_counted) {
        P->pair_count = count_pairs(*P, &P->pair_count_circ);
        P->pairs_counted = true;
    }
    *pairs = P->pair_count;
    return ARKCOS_OK;
}

int arkcos_plan_pair_count_parts(arkcos_plan_t plan, unsigned long long *circulant,
                                 unsigned long long *general)
{
    clear_error();
    if (!plan) return fail(ARKCOS_EINVAL, "NULL plan");
    unsigned long long total = 0;
    int rc = arkcos_plan_pair_count(plan, &total);
    if (rc) return rc;
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    if (circulant) *circulant = P->pair_count_circ;
    if (general) *general = total - P->pair_count_circ;
    return ARKCOS_OK;
}

int arkcos_plan_window(arkcos_plan_t plan, int ring_out, int ring_src, int j, int *lo, int *hi,
                       int *covered)
{
    clear_error();
    if (!plan || !lo || !hi || !covered) return fail(ARKCOS_EINVAL, "NULL pointer");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    if (ring_out < 1 || ring_out > P->nrings || ring_src < 1 || ring_src > P->nrings)
        return fail(ARKCOS_EINVAL, "ring out of range");
    const DevRing &dr = P->dev_rings[ring_out - 1];
    if (j < 0 || j >= dr.n) return fail(ARKCOS_EINVAL, "pixel index out of range");
    *covered = 0;
    *lo = 1;
    *hi = 0;
    for (int k = dr.pair_begin; k < dr.pair_end; ++k) {
        if (P->pairs[k].s != ring_src - 1) continue;
        pair_window(P->pairs[k], P->dev_rings[ring_src - 1].n, j, *lo, *hi);
        *covered = 1;
    }
    return ARKCOS_OK;
}

int arkcos_plan_gen_tiles(arkcos_plan_t plan, int *out, long long cap, long long *count)
{
    clear_error();
    if (!plan || !count || (cap > 0 && !out)) return fail(ARKCOS_EINVAL, "NULL pointer");
    const Plan *P = reinterpret_cast<const Plan *>(plan);
    long long k = 0;
    for (size_t t = 0; t < P->gtiles2.size(); ++t) {
        const DevTile2 &T = P->gtiles2[t];
        for (int h = 0; h < T.nr; ++h) {
            if (T.q[h].len <= 0) continue;
            if (k < cap) {
                int *o = out + 5 * k;
                o[0] = (int)t;
                o[1] = T.nr;
                o[2] = T.q[h].r + 1;
                o[3] = T.j0;
                o[4] = T.q[h].len;
            }
            ++k;
        }
    }
    *count = k;
    return ARKCOS_OK;
}

int arkcos_plan_set_kernel_host(arkcos_plan_t plan, const double *ktab)
{
    clear_error();
    if (!plan || !ktab) return fail(ARKCOS_EINVAL, "NULL pointer");
    Plan *P = reinterpret_cast<Plan *>(plan);
    if (P->host_only) return fail(ARKCOS_ESTATE, "host-only plan has no device table");
    P->ktab.assign(ktab, ktab + P->desc.ntab);
    if (P->adj) P->adj->ktab = P->ktab;
    int cur = 0;
    ARKCOS_HIP_CHECK(hipGetDevice(&cur));
    ARKCOS_HIP_CHECK(hipSetDevice(P->device));
    int rc = write_table_host(*P);
    if (rc == ARKCOS_OK && P->adj) rc = write_table_host(*P->adj);
    (void)hipSetDevice(cur);
    if (rc == ARKCOS_OK) P->knots_set = true;
    return rc;
}

int arkcos_plan_set_kernel(arkcos_plan_t plan, const float *d_knots, void *stream)
{
    clear_error();
    if (!plan || !d_knots) return fail(ARKCOS_EINVAL, "NULL pointer");
    Plan *P = reinterpret_cast<Plan *>(plan);
    if (P->host_only) return fail(ARKCOS_ESTATE, "host-only plan has no device table");
    if (!(P->desc.flags & ARKCOS_PLAN_LEARNABLE))
        return fail(ARKCOS_ESTATE, "plan was not created with ARKCOS_PLAN_LEARNABLE");
    int rc = launch_set_table(*P, d_knots, (hipStream_t)stream);
    if (rc == ARKCOS_OK) rc = launch_build_weights(*P, (hipStream_t)stream);
    if (rc == ARKCOS_OK && P->adj) rc = launch_set_table(*P->adj, d_knots, (hipStream_t)stream);
    if (rc == ARKCOS_OK && P->adj) rc = launch_build_weights(*P->adj, (hipStream_t)stream);
    if (rc == ARKCOS_OK) {
        P->knots_set = true;
        P->ktab.clear();
    }
    return rc;
}

}  // extern "C"
