/*
 * FP64 CPU oracle for the real-space half of the split spherical convolution.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant generator with the HIP
 * library under paper_1211_3556_amd/.
 *
 * What it computes (Sutter, Wandelt & Elsner 2012, "Accelerating
 * convolutions on the sphere with hybrid GPU/CPU kernel splitting"):
 *
 *   The kernel split of Sec. 2 (eq. 1) writes the approximate kernel as a
 *   truncated harmonic-space part plus the Legendre transform of a
 *   real-space part K_theta that is set to zero beyond theta_cut.  The
 *   real-space part is applied to a pixelised map by direct summation on
 *   the GPU (Sec. 2, the ARKCoS term of eq. 3), with the radial kernel
 *   evaluated by interpolating a table of nodes (Sec. 3, the paragraph on
 *   interpolation of the real-space kernel).  On a HEALPix map (Sec. 2,
 *   Nside 2048) of equal-area pixels that sum is
 *
 *       y[p] = Omega * sum_{q : theta(p,q) < theta_cut} K(theta(p,q)) x[q],
 *       Omega = 4 pi / Npix.
 *
 *   The kernel family of Sec. 3 (eq. 5) with C_l = 1 is a Gaussian beam
 *   b_l; its real-space profile is the Legendre sum
 *       K(theta) = sum_l (2l+1)/(4 pi) b_l P_l(cos theta),
 *   i.e. the inverse of the Legendre transform operator P_{l theta} of eq. 1.
 *
 * Readings where the paper is silent:
 *   - the table has ntab nodes at theta_k = k h, h = theta_cut/(ntab-1),
 *     and K is linear in theta between nodes;
 *   - the biased table of Sec. 3 (half the nodes inside the first 1/16 of the
 *     support) is given as an explicit increasing node list theta_0 = 0 <
 *     ... < theta_{ntab-1} = theta_cut; K is again linear in theta between
 *     consecutive nodes, and the node interval of an angle is found by
 *     bisection over that list;
 *   - the cut is strict: pairs with theta >= theta_cut get K = 0;
 *   - HEALPix RING pixel centres follow Gorski et al. (2005), the pixelisation
 *     the paper names for its data.
 *
 * Everything is FP64, plain loops, one OpenMP "parallel for" over output
 * pixels.  No blocking, no symmetry tricks, no approximation beyond the
 * definition above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* HEALPix RING geometry (Gorski et al. 2005).                               */
/*   rings i = 1 .. 4N-1 from north to south                                 */
/*   north cap  i <  N : z = 1 - i^2/(3N^2), 4i pixels, phi = (j+1/2) pi/(2i) */
/*   belt  N <= i <= 3N: z = 4/3 - 2i/(3N), 4N pixels,                        */
/*                       phi = (j + 1/2 [i-N even]) pi/(2N)                   */
/*   south cap  i > 3N : mirror image of ring 4N-i                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double z;      /* cos(theta) of the ring                                  */
    double s;      /* sin(theta), evaluated without cancellation near poles   */
    double theta;  /* colatitude                                              */
    long   n;      /* pixels in the ring                                     */
    long   first;  /* RING index of the first pixel of the ring              */
    double phi0;   /* longitude of pixel j = 0                                */
    double dphi;   /* 2 pi / n                                                */
} ring_rec;

static void ring_of(long N, long i, ring_rec *r)
{
    const double dN = (double)N;
    const long npix = 12L * N * N;
    if (i < N) {                                   /* north polar cap */
        double a = (double)i * (double)i / (3.0 * dN * dN);   /* 1 - z */
        r->z = 1.0 - a;
        r->s = sqrt(a * (2.0 - a));
        r->n = 4 * i;
        r->first = 2 * i * (i - 1);
        r->phi0 = 0.5 * M_PI / (2.0 * (double)i);
    } else if (i <= 3 * N) {                       /* equatorial belt */
        r->z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * dN);
        r->s = sqrt((1.0 - r->z) * (1.0 + r->z));
        r->n = 4 * N;
        r->first = 2 * N * (N - 1) + 4 * N * (i - N);
        r->phi0 = (((i - N) % 2) == 0) ? 0.5 * M_PI / (2.0 * dN) : 0.0;
    } else {                                       /* south polar cap */
        long k = 4 * N - i;
        double a = (double)k * (double)k / (3.0 * dN * dN);   /* 1 + z */
        r->z = a - 1.0;
        r->s = sqrt(a * (2.0 - a));
        r->n = 4 * k;
        r->first = npix - 2 * k * (k + 1);
        r->phi0 = 0.5 * M_PI / (2.0 * (double)k);
    }
    r->theta = atan2(r->s, r->z);
    r->dphi = 2.0 * M_PI / (double)r->n;
}

static ring_rec *ring_table(long N)
{
    long nr = 4 * N - 1;
    ring_rec *t = (ring_rec *)malloc(sizeof(ring_rec) * (size_t)(nr + 1));
    if (!t) return NULL;
    for (long i = 1; i <= nr; ++i) ring_of(N, i, &t[i]);
    return t;
}

/* ring index (1-based) and in-ring index of a RING-scheme pixel, by
 * bisection on the first-pixel indices of the rings                       */
static long ring_of_pixel(long N, const ring_rec *t, long p, long *j)
{
    long lo = 1, hi = 4 * N - 1;
    while (lo < hi) {                       /* first ring whose end > p */
        long mid = (lo + hi) / 2;
        if (t[mid].first + t[mid].n <= p) lo = mid + 1; else hi = mid;
    }
    *j = p - t[lo].first;
    return lo;
}

static void unit_vector(const ring_rec *r, long j, double v[3])
{
    double phi = r->phi0 + (double)j * r->dphi;
    v[0] = r->s * cos(phi);
    v[1] = r->s * sin(phi);
    v[2] = r->z;
}

/* angular separation from the chord between unit vectors */
static double separation(const double a[3], const double b[3])
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    double half = 0.5 * sqrt(dx * dx + dy * dy + dz * dz);
    if (half > 1.0) half = 1.0;
    return 2.0 * asin(half);
}

/*
 * Linear interpolation of the node table (Sec. 3).  nodes == NULL: uniform
 * nodes theta_k = k theta_cut/(ntab-1).  Otherwise nodes[0..ntab-1] lists the
 * node angles (0 = nodes[0] < ... < nodes[ntab-1] = theta_cut) and the
 * interval [nodes[i], nodes[i+1]) holding theta is found by bisection.
 * Returns the left node i and the fraction t of the way to node i+1.
 */
static void interp_weights(double theta, double theta_cut, long ntab,
                           const double *nodes, long *i, double *t)
{
    if (!nodes) {
        double h = theta_cut / (double)(ntab - 1);
        double u = theta / h;
        long k = (long)floor(u);
        if (k > ntab - 2) k = ntab - 2;
        if (k < 0) k = 0;
        *i = k;
        *t = u - (double)k;
        return;
    }
    long lo = 0, hi = ntab - 1;          /* invariant: nodes[lo] <= theta */
    while (hi - lo > 1) {
        long mid = lo + (hi - lo) / 2;
        if (nodes[mid] <= theta) lo = mid; else hi = mid;
    }
    *i = lo;
    *t = (theta - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
}

/* zero at and beyond theta_cut (the truncation of eq. 1) */
static double kernel_value(double theta, double theta_cut, long ntab,
                           const double *nodes, const double *ktab)
{
    if (!(theta < theta_cut)) return 0.0;
    long i; double t;
    interp_weights(theta, theta_cut, ntab, nodes, &i, &t);
    return (1.0 - t) * ktab[i] + t * ktab[i + 1];
}

/* An explicit node list must start at 0, increase strictly and end at the cut. */
static int bad_nodes(double theta_cut, long ntab, const double *nodes)
{
    if (!nodes) return 0;
    if (nodes[0] != 0.0 || nodes[ntab - 1] != theta_cut) return 1;
    for (long k = 1; k < ntab; ++k)
        if (!(nodes[k] > nodes[k - 1])) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Neighbour enumeration.  For output pixel p, every pixel q with            */
/* theta(p,q) < theta_cut is listed once (with its separation).  Rings are   */
/* admitted when |theta_ring - theta_p| < theta_cut; inside a ring the      */
/* longitude window comes from the spherical law of cosines,                 */
/*   cos dphi_max = (cos theta_cut - z_p z_s) / (s_p s_s),                   */
/* widened by two pixels; the whole ring is taken when the window reaches   */
/* around.  The exact separation test then decides membership.              */
/* ------------------------------------------------------------------------ */
typedef struct { long q; double theta; } orc_nb;
typedef struct { orc_nb *v; long cap; int oom; } orc_list;

static void list_push(orc_list *l, long count, long q, double th)
{
    if (count >= l->cap) {
        long cap = l->cap ? 2 * l->cap : 4096;
        orc_nb *nv = (orc_nb *)realloc(l->v, sizeof(orc_nb) * (size_t)cap);
        if (!nv) { l->oom = 1; return; }
        l->v = nv; l->cap = cap;
    }
    l->v[count].q = q;
    l->v[count].theta = th;
}

static long neighbours(long N, const ring_rec *t, double theta_cut, long p,
                       orc_list *out)
{
    long jp;
    long ip = ring_of_pixel(N, t, p, &jp);
    const ring_rec *rp = &t[ip];
    double vp[3];
    unit_vector(rp, jp, vp);
    double phip = rp->phi0 + (double)jp * rp->dphi;
    long count = 0;
    for (long is = 1; is <= 4 * N - 1; ++is) {
        const ring_rec *rs = &t[is];
        if (!(fabs(rs->theta - rp->theta) < theta_cut + 1e-12)) continue;
        double arg = (cos(theta_cut) - rp->z * rs->z) / (rp->s * rs->s);
        long jlo, jhi, whole = 0;
        if (arg <= -1.0) {
            whole = 1;
        } else {
            if (arg > 1.0) arg = 1.0;
            double half = acos(arg) + 2.0 * rs->dphi;
            if (half >= M_PI) whole = 1;
            else {
                jlo = (long)ceil((phip - half - rs->phi0) / rs->dphi);
                jhi = (long)floor((phip + half - rs->phi0) / rs->dphi);
                if (jhi - jlo + 1 >= rs->n) whole = 1;
            }
        }
        if (whole) { jlo = 0; jhi = rs->n - 1; }
        for (long jj = jlo; jj <= jhi; ++jj) {
            long jq = ((jj % rs->n) + rs->n) % rs->n;
            double vq[3];
            unit_vector(rs, jq, vq);
            double th = separation(vp, vq);
            if (th < theta_cut) {
                list_push(out, count, rs->first + jq, th);
                if (out->oom) return -1;
                ++count;
            }
        }
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (all return 0 on success, negative on bad input).   */
/* ------------------------------------------------------------------------ */

/* Geometry of ring i (1-based). */
int orc_ring(long nside, long i, double *z, double *s, double *theta,
             long *n, long *first, double *phi0)
{
    if (nside < 1 || i < 1 || i > 4 * nside - 1) return -1;
    ring_rec r;
    ring_of(nside, i, &r);
    *z = r.z; *s = r.s; *theta = r.theta; *n = r.n; *first = r.first;
    *phi0 = r.phi0;
    return 0;
}

/* Unit vectors of a list of RING pixels, xyz is 3*npix doubles. */
int orc_pix2vec(long nside, long npix, const long *pix, double *xyz)
{
    if (nside < 1) return -1;
    ring_rec *t = ring_table(nside);
    if (!t) return -2;
    long total = 12L * nside * nside;
    for (long k = 0; k < npix; ++k) {
        if (pix[k] < 0 || pix[k] >= total) { free(t); return -1; }
        long j;
        long i = ring_of_pixel(nside, t, pix[k], &j);
        unit_vector(&t[i], j, xyz + 3 * k);
    }
    free(t);
    return 0;
}

/*
 * Kernel table from a beam: K(theta_k) = sum_{l<=lmax} (2l+1)/(4 pi) b_l
 * P_l(cos theta_k) at theta_k = k theta_cut/(ntab-1), or at theta_k = nodes[k]
 * for an explicit node list.  This is the inverse of
 * the Legendre transform operator of eq. 1 applied to the eq. 5 kernel with
 * C_l = 1.  Legendre polynomials by the three-term recurrence
 *   (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}.
 */
int orc_tabulate(const double *bl, long lmax, double theta_cut, long ntab,
                 const double *nodes, double *ktab)
{
    if (lmax < 0 || ntab < 2 || !(theta_cut > 0.0) || theta_cut > M_PI)
        return -1;
    if (bad_nodes(theta_cut, ntab, nodes)) return -1;
    double h = theta_cut / (double)(ntab - 1);
    #pragma omp parallel for schedule(static)
    for (long k = 0; k < ntab; ++k) {
        double x = cos(nodes ? nodes[k] : (double)k * h);
        double pm1 = 1.0, p = x;          /* P_0, P_1 */
        double sum = bl[0];               /* l = 0 term times 4 pi */
        if (lmax >= 1) sum += 3.0 * bl[1] * x;
        for (long l = 1; l < lmax; ++l) {
            double pn = ((2.0 * l + 1.0) * x * p - (double)l * pm1) / (double)(l + 1);
            pm1 = p; p = pn;
            sum += (2.0 * (l + 1) + 1.0) * bl[l + 1] * p;
        }
        ktab[k] = sum / (4.0 * M_PI);
    }
    return 0;
}

/*
 * Windowed direct sum at a list of output pixels (pix == NULL: all pixels,
 * in RING order).  y has npix_eval entries; pairs_out (nullable) receives
 * the number of in-disc pairs per evaluated pixel.  nodes: NULL for the
 * uniform table, else the ntab node angles.
 */
int orc_convolve(long nside, double theta_cut, long ntab, const double *nodes,
                 const double *ktab, const double *x, long npix_eval,
                 const long *pix, double *y, long *pairs_out)
{
    if (nside < 1 || ntab < 2 || !(theta_cut > 0.0) || theta_cut > M_PI)
        return -1;
    if (bad_nodes(theta_cut, ntab, nodes)) return -1;
    long total = 12L * nside * nside;
    if (!pix) npix_eval = total;
    ring_rec *t = ring_table(nside);
    if (!t) return -2;
    double omega = 4.0 * M_PI / (double)total;
    int bad = 0;
    #pragma omp parallel
    {
        orc_list nb = {NULL, 0, 0};
        #pragma omp for schedule(dynamic, 64)
        for (long k = 0; k < npix_eval; ++k) {
            long p = pix ? pix[k] : k;
            if (p < 0 || p >= total) { bad = 1; continue; }
            long cnt = neighbours(nside, t, theta_cut, p, &nb);
            if (cnt < 0) { bad = 2; continue; }
            double acc = 0.0;
            for (long m = 0; m < cnt; ++m)
                acc += kernel_value(nb.v[m].theta, theta_cut, ntab, nodes, ktab) * x[nb.v[m].q];
            y[k] = omega * acc;
            if (pairs_out) pairs_out[k] = cnt;
        }
        free(nb.v);
    }
    free(t);
    return bad == 2 ? -2 : (bad ? -1 : 0);
}

/*
 * Exhaustive all-pairs sum (every q tested, no windows); for small Nside.
 */
int orc_convolve_exhaustive(long nside, double theta_cut, long ntab,
                            const double *nodes, const double *ktab,
                            const double *x, long npix_eval, const long *pix,
                            double *y, long *pairs_out)
{
    if (nside < 1 || ntab < 2 || !(theta_cut > 0.0) || theta_cut > M_PI)
        return -1;
    if (bad_nodes(theta_cut, ntab, nodes)) return -1;
    long total = 12L * nside * nside;
    if (!pix) npix_eval = total;
    ring_rec *t = ring_table(nside);
    if (!t) return -2;
    double *v = (double *)malloc(sizeof(double) * 3 * (size_t)total);
    if (!v) { free(t); return -2; }
    for (long i = 1; i <= 4 * nside - 1; ++i)
        for (long j = 0; j < t[i].n; ++j)
            unit_vector(&t[i], j, v + 3 * (t[i].first + j));
    double omega = 4.0 * M_PI / (double)total;
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < npix_eval; ++k) {
        long p = pix ? pix[k] : k;
        if (p < 0 || p >= total) { bad = 1; continue; }
        double acc = 0.0;
        long cnt = 0;
        for (long q = 0; q < total; ++q) {
            double th = separation(v + 3 * p, v + 3 * q);
            if (th < theta_cut) {
                acc += kernel_value(th, theta_cut, ntab, nodes, ktab) * x[q];
                ++cnt;
            }
        }
        y[k] = omega * acc;
        if (pairs_out) pairs_out[k] = cnt;
    }
    free(v);
    free(t);
    return bad ? -1 : 0;
}

/*
 * Gradient of a loss with respect to the knots, given g = dL/dy over the
 * whole map:  dL/dK_k = Omega sum_p g[p] sum_q Lambda_k(theta_pq) x[q],
 * with Lambda_k the piecewise-linear hat of node k (weight 1-t to node i and
 * t to node i+1), the derivative of the interpolated kernel with respect to
 * its nodes.  gk has ntab entries.
 */
int orc_knot_grad(long nside, double theta_cut, long ntab, const double *nodes,
                  const double *x, const double *g, double *gk)
{
    if (nside < 1 || ntab < 2 || !(theta_cut > 0.0) || theta_cut > M_PI)
        return -1;
    if (bad_nodes(theta_cut, ntab, nodes)) return -1;
    long total = 12L * nside * nside;
    ring_rec *t = ring_table(nside);
    if (!t) return -2;
    double omega = 4.0 * M_PI / (double)total;
    int nthr = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nthr * (size_t)ntab, sizeof(double));
    if (!part) { free(t); return -2; }
    int bad = 0;
    #pragma omp parallel
    {
        double *mine = part + (size_t)omp_get_thread_num() * (size_t)ntab;
        orc_list nb = {NULL, 0, 0};
        #pragma omp for schedule(dynamic, 64)
        for (long p = 0; p < total; ++p) {
            if (g[p] == 0.0) continue;
            long cnt = neighbours(nside, t, theta_cut, p, &nb);
            if (cnt < 0) { bad = 1; continue; }
            for (long m = 0; m < cnt; ++m) {
                long i; double tt;
                interp_weights(nb.v[m].theta, theta_cut, ntab, nodes, &i, &tt);
                double c = omega * g[p] * x[nb.v[m].q];
                mine[i] += (1.0 - tt) * c;
                mine[i + 1] += tt * c;
            }
        }
        free(nb.v);
    }
    for (long k = 0; k < ntab; ++k) {
        double s = 0.0;
        for (int th = 0; th < nthr; ++th) s += part[(size_t)th * ntab + k];
        gk[k] = s;
    }
    free(part);
    free(t);
    return bad ? -2 : 0;
}

/*
 * The interpolated, truncated kernel itself at n angles (0 at and beyond the
 * cut); nodes as for orc_convolve.
 */
int orc_kernel_eval(double theta_cut, long ntab, const double *nodes,
                    const double *ktab, long n, const double *theta, double *out)
{
    if (ntab < 2 || !(theta_cut > 0.0) || theta_cut > M_PI || n < 0) return -1;
    if (bad_nodes(theta_cut, ntab, nodes)) return -1;
    for (long k = 0; k < n; ++k) {
        if (!(theta[k] >= 0.0)) return -1;
        out[k] = kernel_value(theta[k], theta_cut, ntab, nodes, ktab);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The harmonic-space half of the split (Sec. 2, eq. 1): the truncated      */
/* l-space kernel Khat_l, l <= lcut, applied by spherical-harmonic          */
/* transforms.  With the plain pixel quadrature for the analysis,           */
/*     a_lm = Omega sum_p x_p conj(Y_lm(p)),                                */
/*     y_p  = sum_{l <= lcut} Khat_l sum_{m=-l..l} a_lm Y_lm(p).            */
/* For a real map a_{l,-m} = (-1)^m conj(a_lm), so                          */
/*     y_p = sum_l Khat_l [a_l0 Y_l0(p) + 2 sum_{m>=1} Re(a_lm Y_lm(p))].   */
/* Y_lm(theta, phi) = lambda_lm(cos theta) e^{i m phi} with the orthonormal */
/* associated Legendre functions                                           */
/*     lambda_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m,                 */
/* by the standard recurrences in l at fixed m:                             */
/*     lambda_00 = 1/sqrt(4 pi),                                            */
/*     lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1},          */
/*     lambda_lm = a_lm (cos(theta) lambda_{l-1,m} - b_lm lambda_{l-2,m}),  */
/*     a_lm = sqrt((4l^2-1)/(l^2-m^2)),                                     */
/*     b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).                             */
/* Plain FP64: a lambda_mm below the FP64 range flushes to zero.  For       */
/* lcut <= 1900 no such (theta, m) reaches its oscillatory range            */
/* l ~ m/sin(theta) within l <= lcut (that would need                       */
/* lcut sin(theta) log10(1/sin(theta)) > 308, but the left side is at most  */
/* 0.16 lcut), so the dropped values stay negligible.  The longitude sums   */
/* use libm cos/sin of m phi_j directly.                                    */
/* ------------------------------------------------------------------------ */

/* lambda_lm(theta) for 0 <= m <= l <= L into lam[l*(L+1) + m] */
static void legendre_table(long L, double z, double s, double *lam)
{
    const long W = L + 1;
    double mm = 1.0 / sqrt(4.0 * M_PI);
    for (long m = 0; m <= L; ++m) {
        if (m > 0) mm *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
        lam[m * W + m] = mm;
        double pm2 = 0.0, pm1 = mm;
        for (long l = m + 1; l <= L; ++l) {
            double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            double b = sqrt(((double)(l - 1) * (l - 1) - (double)m * m) /
                            (4.0 * (double)(l - 1) * (l - 1) - 1.0));
            double v = a * (z * pm1 - b * pm2);
            lam[l * W + m] = v;
            pm2 = pm1;
            pm1 = v;
        }
    }
}

int orc_harmonic(long nside, long lcut, const double *khat, const double *x, double *y)
{
    if (nside < 1 || lcut < 0) return -1;
    ring_rec *t = ring_table(nside);
    if (!t) return -2;
    const long nr = 4 * nside - 1, L = lcut, W = L + 1;
    const double omega = 4.0 * M_PI / (12.0 * (double)nside * (double)nside);
    /* per-ring longitude sums F_i(m) = sum_j x_j e^{-i m phi_j} */
    double *fre = (double *)calloc((size_t)nr * W, sizeof(double));
    double *fim = (double *)calloc((size_t)nr * W, sizeof(double));
    double *are = (double *)calloc((size_t)W * W, sizeof(double));
    double *aim = (double *)calloc((size_t)W * W, sizeof(double));
    if (!fre || !fim || !are || !aim) {
        free(fre); free(fim); free(are); free(aim); free(t);
        return -2;
    }
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 1; i <= nr; ++i) {
        const ring_rec *r = &t[i];
        for (long m = 0; m <= L; ++m) {
            double sr = 0.0, si = 0.0;
            for (long j = 0; j < r->n; ++j) {
                double ph = (double)m * (r->phi0 + (double)j * r->dphi);
                double v = x[r->first + j];
                sr += v * cos(ph);
                si -= v * sin(ph);
            }
            fre[(i - 1) * W + m] = sr;
            fim[(i - 1) * W + m] = si;
        }
    }
    /* analysis: a_lm = Omega sum_i lambda_lm(theta_i) F_i(m), ring by ring
       into per-thread partial sums, added in a fixed order */
    int nthr = omp_get_max_threads();
    double *pre = (double *)calloc((size_t)nthr * W * W, sizeof(double));
    double *pim = (double *)calloc((size_t)nthr * W * W, sizeof(double));
    if (!pre || !pim) bad = 1;
    if (!bad) {
        #pragma omp parallel
        {
            double *lam = (double *)malloc(sizeof(double) * (size_t)W * W);
            double *mr = pre + (size_t)omp_get_thread_num() * W * W;
            double *mi = pim + (size_t)omp_get_thread_num() * W * W;
            if (!lam) bad = 1;
            #pragma omp for schedule(static)
            for (long i = 1; i <= nr; ++i) {
                if (!lam) continue;
                legendre_table(L, t[i].z, t[i].s, lam);
                for (long l = 0; l <= L; ++l)
                    for (long m = 0; m <= l; ++m) {
                        mr[l * W + m] += lam[l * W + m] * fre[(i - 1) * W + m];
                        mi[l * W + m] += lam[l * W + m] * fim[(i - 1) * W + m];
                    }
            }
            free(lam);
        }
        for (int th = 0; th < nthr; ++th)
            for (long k = 0; k < W * W; ++k) {
                are[k] += pre[(size_t)th * W * W + k];
                aim[k] += pim[(size_t)th * W * W + k];
            }
        for (long k = 0; k < W * W; ++k) {
            are[k] *= omega;
            aim[k] *= omega;
        }
    }
    free(pre);
    free(pim);
    /* synthesis: G_i(m) = sum_l Khat_l a_lm lambda_lm(theta_i), then
       y_j = Re G_i(0) + 2 sum_{m>=1} Re(G_i(m) e^{i m phi_j}) */
    if (!bad) {
        #pragma omp parallel
        {
            double *lam = (double *)malloc(sizeof(double) * (size_t)W * W);
            double *gr = (double *)malloc(sizeof(double) * (size_t)W);
            double *gi = (double *)malloc(sizeof(double) * (size_t)W);
            if (!lam || !gr || !gi) bad = 1;
            #pragma omp for schedule(dynamic, 1)
            for (long i = 1; i <= nr; ++i) {
                if (!lam || !gr || !gi) continue;
                const ring_rec *r = &t[i];
                legendre_table(L, r->z, r->s, lam);
                for (long m = 0; m <= L; ++m) {
                    double sr = 0.0, si = 0.0;
                    for (long l = m; l <= L; ++l) {
                        sr += khat[l] * are[l * W + m] * lam[l * W + m];
                        si += khat[l] * aim[l * W + m] * lam[l * W + m];
                    }
                    gr[m] = sr;
                    gi[m] = si;
                }
                for (long j = 0; j < r->n; ++j) {
                    double acc = gr[0];
                    for (long m = 1; m <= L; ++m) {
                        double ph = (double)m * (r->phi0 + (double)j * r->dphi);
                        acc += 2.0 * (gr[m] * cos(ph) - gi[m] * sin(ph));
                    }
                    y[r->first + j] = acc;
                }
            }
            free(lam);
            free(gr);
            free(gi);
        }
    }
    free(fre); free(fim); free(are); free(aim); free(t);
    return bad ? -2 : 0;
}

/* The orthonormal lambda_lm(cos theta) of orc_harmonic for one angle,
   0 <= m <= l <= L, into lam[l*(L+1) + m] (entries with m > l untouched). */
int orc_legendre_lm(long L, double theta, double *lam)
{
    if (L < 0) return -1;
    legendre_table(L, cos(theta), sin(theta), lam);
    return 0;
}

/*
 * The RING pixel containing a direction (z = cos theta, phi), from the
 * HEALPix pixel boundaries (Gorski et al. 2005).  With t = phi / (pi/2):
 *   equatorial zone |z| <= 2/3: the boundaries are the lines
 *     N (1/2 + t - 3z/4) = integer  and  N (1/2 + t + 3z/4) = integer;
 *     with a = floor of the first and b = floor of the second, the point is
 *     in ring i = N + a - b (1-based) at in-ring index
 *     floor((a + b - N + [i - N odd] + 1) / 2) mod 4N;
 *   polar caps |z| > 2/3: with r = N sqrt(3 (1 - |z|)) and tq = t - floor(t)
 *     the longitude within the quadrant, the boundaries are the curves
 *     tq r = integer and (1 - tq) r = integer; the ring counted from the
 *     nearest pole is k = floor(tq r) + floor((1 - tq) r) + 1, and the index
 *     floor(t k) mod 4k.
 * At every pixel centre both reduce to the centre's own ring and index.
 */
static long vec2pix_ring(long N, double z, double phi)
{
    const double dN = (double)N;
    double t = phi / (0.5 * M_PI);
    t = fmod(t, 4.0);
    if (t < 0.0) t += 4.0;
    if (fabs(z) <= 2.0 / 3.0) {
        const long a = (long)floor(dN * (0.5 + t - 0.75 * z));
        const long b = (long)floor(dN * (0.5 + t + 0.75 * z));
        const long ir = N + 1 + a - b;              /* 1 .. 2N+1 from ring N */
        const long odd = (ir & 1) ? 0 : 1;           /* ring i = N + ir - 1: [i - N odd] */
        long ip = (a + b - N + odd + 1) / 2;
        ip %= 4 * N;
        if (ip < 0) ip += 4 * N;
        return 2 * N * (N - 1) + 4 * N * (ir - 1) + ip;
    }
    const double tq = t - floor(t);
    const double r = dN * sqrt(3.0 * (1.0 - fabs(z)));
    const long a = (long)floor(tq * r);
    const long b = (long)floor((1.0 - tq) * r);
    long k = a + b + 1;                              /* N only next to |z| = 2/3 */
    if (k > N) k = N;
    if (k < 1) k = 1;
    long ip = (long)floor(t * (double)k);
    ip %= 4 * k;
    if (z > 0.0) return 2 * k * (k - 1) + ip;
    return 12L * N * N - 2 * k * (k + 1) + ip;
}

/* RING pixels of a list of unit vectors (3*n doubles). */
int orc_vec2pix(long nside, long n, const double *xyz, long *pix)
{
    if (nside < 1) return -1;
    for (long k = 0; k < n; ++k) {
        const double *v = xyz + 3 * k;
        const double rr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(rr > 0.0)) return -1;
        pix[k] = vec2pix_ring(nside, v[2] / rr, atan2(v[1], v[0]));
    }
    return 0;
}

/*
 * Rotated copy of a map: for every pixel p of rings ring_first..ring_last
 * (1-based, inclusive), with centre n_p, out[p] = in[q] where q is the pixel
 * containing R^T n_p; a feature at direction c of `in` appears at R c of
 * `out` (rot: row-major 3x3 rotation).  Other pixels of out are untouched.
 */
int orc_rotate_map(long nside, const double *rot, long ring_first, long ring_last,
                   const double *in, double *out)
{
    if (nside < 1 || ring_first < 1 || ring_last < ring_first || ring_last > 4 * nside - 1)
        return -1;
    ring_rec *t = ring_table(nside);
    if (!t) return -2;
    for (long i = ring_first; i <= ring_last; ++i) {
        const ring_rec *r = &t[i];
#pragma omp parallel for schedule(static)
        for (long j = 0; j < r->n; ++j) {
            double v[3], w[3];
            unit_vector(r, j, v);
            for (int c = 0; c < 3; ++c)
                w[c] = rot[0 * 3 + c] * v[0] + rot[1 * 3 + c] * v[1] + rot[2 * 3 + c] * v[2];
            const double rr = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
            out[r->first + j] = in[vec2pix_ring(nside, w[2] / rr, atan2(w[1], w[0]))];
        }
    }
    free(t);
    return 0;
}

/* Number of threads the oracle runs with (for reporting), and a setter. */
int orc_threads(void) { return omp_get_max_threads(); }
int orc_set_threads(int n)
{
    if (n < 1) return -1;
    omp_set_num_threads(n);
    return 0;
}
