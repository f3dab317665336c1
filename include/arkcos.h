/*
 * arkcos -- real-space spherical convolution on MI355X (gfx950).
 *
 * C ABI of the GPU library libarkcos.so.  Every entry point takes plain host
 * or device pointers and sizes; no C++ or framework types cross it.  Device
 * pointers are HIP device memory on the current device; `stream` is a
 * hipStream_t passed as void* (NULL = the default stream).
 *
 * The operation (Sutter, Wandelt & Elsner 2012, Sec. 2, eq. 1 and the
 * ARKCoS term of eq. 3): the real-space part K_theta of a split radial
 * kernel, truncated at theta_cut, applied to a HEALPix RING-ordered map by
 * direct summation,
 *
 *     out[p] = Omega * sum_{q : theta(p,q) < theta_cut} K(theta(p,q)) in[q],
 *     Omega  = 4 pi / Npix,  Npix = 12 Nside^2,
 *
 * where K is linear in theta between ntab nodes on [0, theta_cut] (Sec. 3,
 * interpolation of the real-space kernel), and K = 0 for theta >= theta_cut.
 * The nodes are uniform, theta_k = k theta_cut/(ntab-1), or -- the biased
 * table of Sec. 3 -- uniform on each of two pieces with a finer first piece
 * (see arkcos_plan_desc).  Sums run in FP32 on the device.
 *
 * Conventions for every function:
 *   - returns ARKCOS_OK (0) or a negative status; never aborts or throws;
 *     arkcos_last_error() then holds a per-thread message;
 *   - launches are asynchronous and stream-ordered; device faults surface at
 *     the caller's next synchronisation;
 *   - convolve/backward/batch calls never allocate or synchronise, so they
 *     can be captured in a HIP graph; a plan (and a batch) is used by one
 *     stream at a time, because its workspace (tile counter, gradient
 *     partials) is shared by its calls;
 *   - plan creation and every compute call open a roctx range named after
 *     the entry point (visible in rocprofv3 marker traces);
 *   - with the environment variable ARKCOS_LOG=1, each plan built writes one
 *     line of statistics (ring classes, pairs, tiles, staged chunks, tile
 *     shapes and their source, weights, device bytes) to stderr.
 */
#ifndef ARKCOS_H
#define ARKCOS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arkcos_plan *arkcos_plan_t;    /* opaque; owns host + device plan data */
typedef struct arkcos_batch *arkcos_batch_t;  /* opaque; owns a tile queue over plans  */
typedef struct arkcos_harm *arkcos_harm_t;    /* opaque; harmonic-space half of a split */

enum {
    ARKCOS_OK = 0,
    ARKCOS_EINVAL = -1,       /* bad argument                                 */
    ARKCOS_ENOMEM = -2,       /* host or device allocation failed             */
    ARKCOS_EDEVICE = -3,      /* a HIP call or kernel launch failed           */
    ARKCOS_EUNSUPPORTED = -4, /* valid but not supported (size limits)        */
    ARKCOS_ESTATE = -5        /* object not in a state that allows the call   */
};

/* plan flags */
#define ARKCOS_PLAN_HOST_ONLY 1u  /* build host data only: no device memory, no launches */
#define ARKCOS_PLAN_LEARNABLE 2u  /* knots may be replaced from device memory and
                                     knot gradients may be requested             */

/* Largest supported Nside (ring indices and longitudes stay exact in int32). */
#define ARKCOS_MAX_NSIDE 8192
/* Largest node count for which knot gradients are supported. */
#define ARKCOS_MAX_GRAD_NTAB 2048
/* Largest l_cut of the harmonic-space half (one order's coefficients fit LDS). */
#define ARKCOS_MAX_LCUT 4095
/* Bytes of the per-device static workspace of arkcos_convolve_backward_static
 * (32 MiB: the gathers' queue counters in its first 256 bytes, then the
 * knot-gradient partial rows). */
#define ARKCOS_STATIC_SCRATCH_BYTES (32u << 20)

/*
 * Tile shapes of the general gather (polar caps and belt rings near them).  A
 * tile is a segment of gen_pixels pixels of one northern ring (of the first
 * half-quadrant; each pixel stands for its sixteen symmetric images), or the
 * same segment of two or four adjacent rings, which then share each staged
 * chunk of a source ring.  A ring whose widest source window is at most
 * gen_quad_window positions may go four to a tile, one at most
 * gen_pair_window positions two to a tile; the 512 lanes of a tile are split
 * evenly over its rings and the pixels of each ring.  Each field: 0 = the
 * tuned value from the tuning cache (arkcos_set_tune_cache), else the built-in
 * default (128, 64, 200); otherwise gen_pixels is 16, 32, 64 or 128 and a
 * window threshold is -1 (never) or 1 .. 1000000 positions (else EINVAL).
 * The circulant gather's tiles (4 rings x 1024 pixels) are fixed by its
 * register layout.
 */
typedef struct {
    int gen_pixels;
    int gen_quad_window;
    int gen_pair_window;
    int reserved;         /* must be 0 */
} arkcos_tiles;

typedef struct {
    int nside;            /* HEALPix resolution, 1 .. ARKCOS_MAX_NSIDE (any integer)       */
    double theta_cut;     /* radians, 0 < theta_cut <= pi                                 */
    int ntab;             /* >= 2 nodes on [0, theta_cut] inclusive (node grid below)     */
    const double *ktab;   /* host FP64 node values K(theta_k), length ntab; copied (the
                             caller keeps ownership).  NULL only with ARKCOS_PLAN_LEARNABLE,
                             in which case knots must be set before the first convolve */
    int max_batch;        /* largest nbatch a call may pass (>= 1); sizes the workspace  */
    arkcos_tiles tiles;   /* general-gather tile shapes; all 0 = tuned or default     */
    unsigned flags;       /* ARKCOS_PLAN_* bits                                         */
    /* Node grid.  theta_break = 0 and k_break = 0: uniform nodes
     * theta_k = k theta_cut/(ntab-1).  Otherwise the two-piece table of the
     * biased interpolation of Sec. 3: nodes 0..k_break evenly spaced on
     * [0, theta_break] and nodes k_break..ntab-1 evenly spaced on
     * [theta_break, theta_cut].  Needs 0 < theta_break < theta_cut,
     * 1 <= k_break <= ntab-2 and a first piece at least as fine as the second,
     * theta_break/k_break <= (theta_cut-theta_break)/(ntab-1-k_break)
     * (else EINVAL).  The paper's bias puts half of the nodes in the first
     * 1/16 of the support: theta_break = theta_cut/16, k_break = (ntab-1)/2
     * (integer division).  Kernel tables are values at these nodes
     * (arkcos_grid_nodes, arkcos_tabulate_legendre_at).                      */
    double theta_break;
    int k_break;
    /* Output ring range (partial sky, e.g. a survey patch placed on a polar
     * cap, the use the paper's conclusions (Sec. 4) suggest for small-area maps):
     * ring_first = ring_last = 0 computes every ring; otherwise only output
     * rings ring_first..ring_last (1-based, inclusive, within 1..4 Nside-1,
     * else EINVAL) are written, the other output pixels are left untouched,
     * and the cost scales with the range.  Input pixels are read wherever
     * they lie within theta_cut of the range.  The adjoint of such a plan
     * takes dL/d(out) on the range only (values outside it are ignored): its
     * map gradient is nonzero on the rings within theta_cut of the range
     * (arkcos_plan_info.adjoint_ring_*) and zero elsewhere, and its knot
     * gradient sums over the range's output pixels.  The plan holds a second,
     * internal plan for the adjoint.                                          */
    int ring_first;
    int ring_last;
} arkcos_plan_desc;

typedef struct {
    int nside;
    int nrings;                    /* 4 Nside - 1                                       */
    long long npix;                /* 12 Nside^2                                        */
    long long ring_pairs;          /* (output ring, source ring) pairs in the plan      */
    long long tiles;               /* work items per map: circulant + general tiles     */
    long long candidates;          /* window pixels the kernels visit per map           */
    double omega;                  /* 4 pi / Npix                                       */
    int ntab;
    arkcos_tiles tile_shapes;      /* general-gather tiles in use (every field resolved) */
    int tile_source;               /* where they came from: 0 built-in defaults, 1 the
                                      tuning cache, 2 the descriptor (any field)        */
    unsigned flags;
    int threads_per_block;
    long long device_bytes;        /* device memory the plan holds                      */
    int circulant_rings;           /* output rings gathered with precomputed weight rows */
    int general_rings;             /* output rings gathered with per-pair weights       */
    long long circulant_tiles;     /* work items of the circulant gather per map        */
    long long general_tiles;       /* half-quadrant segments (<= 128 pixels of one ring)
                                      of the general rings; the general gather and its
                                      knot gradient group them into tiles of 1, 2 or 4
                                      rings (arkcos_plan_gen_tiles)                     */
    long long weights;             /* FP32 entries of the circulant weight rows         */
    double theta_break;            /* node grid of the descriptor (0, 0: uniform)       */
    int k_break;
    int ring_first;                /* output ring range of the descriptor (0, 0: all)   */
    int ring_last;
    int adjoint_ring_first;        /* ring-range plans: rings the adjoint writes, every */
    int adjoint_ring_last;         /* ring within theta_cut of the range (0, 0: all)    */
    int circ_form;                 /* circulant gather: 0 vector FMAs, 1 matrix cores
                                      (v_mfma_f32_16x16x4f32), chosen per plan from the
                                      mean width of its weight rows                     */
} arkcos_plan_info;

/* The two gathers of a forward convolution (they write disjoint rings). */
#define ARKCOS_PART_CIRCULANT 1   /* belt rings whose discs stay in the belt */
#define ARKCOS_PART_GENERAL 2     /* polar caps and belt rings near them     */
#define ARKCOS_PART_ALL 3

/* ----------------------------------------------------------------- host -- */

/*
 * Node table of the eq. 5 kernel family (Sec. 3) from its Legendre
 * coefficients: K(theta_k) = sum_{l=0}^{lmax} (2l+1)/(4 pi) b_l P_l(cos theta_k),
 * theta_k = k theta_cut/(ntab-1), k = 0..ntab-1 -- the inverse of the Legendre
 * transform operator P_{l theta} of eq. 1.  Host FP64, three-term recurrence.
 *   b_l      host, lmax+1 doubles (e.g. a Gaussian beam)       [in]
 *   ktab_out host, ntab doubles, caller-allocated               [out]
 * EINVAL on lmax < 0, ntab < 2, theta_cut outside (0, pi], NULL pointers.
 */
int arkcos_tabulate_legendre(const double *b_l, int lmax, double theta_cut, int ntab,
                             double *ktab_out);

/*
 * Node angles of a table (the grid of arkcos_plan_desc: theta_break = 0 and
 * k_break = 0 for uniform nodes, else the two-piece biased grid of Sec. 3).
 *   theta_out  host, ntab doubles, caller-allocated; theta_out[0] = 0 and
 *              theta_out[ntab-1] = theta_cut exactly                   [out]
 * EINVAL on the descriptor errors of arkcos_plan_create for these fields,
 * ntab < 2 or a NULL pointer.
 */
int arkcos_grid_nodes(double theta_cut, int ntab, double theta_break, int k_break,
                      double *theta_out);

/*
 * The eq. 5 kernel profile of arkcos_tabulate_legendre at n arbitrary angles
 * theta[k] in [0, pi] (e.g. the nodes of a biased grid):
 * out[k] = sum_{l=0}^{lmax} (2l+1)/(4 pi) b_l P_l(cos theta[k]).  Host FP64.
 *   b_l   host, lmax+1 doubles                  [in]
 *   theta host, n doubles                       [in]
 *   out   host, n doubles, caller-allocated     [out]
 * EINVAL on lmax < 0, n < 1, an angle outside [0, pi] or NULL pointers.
 */
int arkcos_tabulate_legendre_at(const double *b_l, int lmax, const double *theta, int n,
                                double *out);

/*
 * HEALPix RING geometry of ring `ring` (1 .. 4 Nside - 1), as the library's
 * plan computes it (Gorski et al. 2005; the paper's map format, Sec. 2):
 * z = cos(theta), sin(theta) without cancellation, pixel count, RING index of
 * the first pixel and the longitude of that pixel.  Host only; any out-pointer
 * may be NULL.  EINVAL on nside outside 1..ARKCOS_MAX_NSIDE or ring out of range.
 */
int arkcos_ring_info(int nside, int ring, double *z, double *sin_theta, int *npix_ring,
                     long long *first_pixel, double *phi0);

/* ----------------------------------------------------------------- plan -- */

/*
 * Build a plan for one (Nside, theta_cut, node table): FP64 ring geometry,
 * per output ring the contiguous range of source rings with
 * |theta_r - theta_s| < theta_cut, per ring pair the FP32 chord constants and
 * longitude window, and the tile list (Sec. 2: the part of the kernel that
 * is applied in real space).  Unless ARKCOS_PLAN_HOST_ONLY is set, allocates
 * and fills device memory on the current device (synchronously).
 *   desc  host, read only                                            [in]
 *   out   receives the plan; *out is NULL on failure                 [out]
 * EINVAL on a bad descriptor, ENOMEM, EDEVICE on HIP failures,
 * EUNSUPPORTED if ntab nodes do not fit in the per-workgroup LDS budget.
 */
int arkcos_plan_create(const arkcos_plan_desc *desc, arkcos_plan_t *out);

/* Release a plan and its device memory.  Synchronises the device first.  A NULL
 * plan is accepted. */
int arkcos_plan_destroy(arkcos_plan_t plan);

/* Plan statistics (host only). */
int arkcos_plan_get_info(arkcos_plan_t plan, arkcos_plan_info *info);

/*
 * Exact number of in-disc pairs (theta_pq < theta_cut, self-pairs included) per
 * map, counted in FP64 from the haversine identity ring pair by ring pair (the
 * unit of the throughput metric).  Host only; computed once and cached.
 */
int arkcos_plan_pair_count(arkcos_plan_t plan, unsigned long long *pairs);

/*
 * The same exact count split by the gather that evaluates the pairs: output
 * rings of ARKCOS_PART_CIRCULANT or ARKCOS_PART_GENERAL (either pointer may be
 * NULL).  Host only.
 */
int arkcos_plan_pair_count_parts(arkcos_plan_t plan, unsigned long long *circulant,
                                 unsigned long long *general);

/*
 * Longitude window the device kernels scan for output pixel j of ring
 * `ring_out` on source ring `ring_src` (rings 1-based): unwrapped source
 * indices lo..hi (hi - lo + 1 <= pixels of the source ring; indices are taken
 * modulo the ring length).  *covered = 0 if ring_src is not a source ring of
 * ring_out (lo > hi then).  Evaluated by the same FP32 code the kernels run.
 * Host only; for tests of window completeness.
 */
int arkcos_plan_window(arkcos_plan_t plan, int ring_out, int ring_src, int j, int *lo,
                       int *hi, int *covered);

/*
 * The general gather's tiles, for tests of the tiling: one record of five ints
 * (tile index, rings in the tile, ring (1-based, northern), first pixel, pixel
 * count) per ring of each tile, over pixels j <= n/4 - 2o - j of the ring's
 * first quadrant.  Writes min(cap, total) records to `out` (host, 5 ints each;
 * may be NULL with cap 0) and the total to *count.  Host only.
 */
int arkcos_plan_gen_tiles(arkcos_plan_t plan, int *out, long long cap, long long *count);

/*
 * Replace the node table from host FP64 values (length ntab).  The device copy
 * (FP32, pre-multiplied by Omega) is written with a synchronous copy.
 * ESTATE for a host-only plan.
 */
int arkcos_plan_set_kernel_host(arkcos_plan_t plan, const double *ktab);

/*
 * Replace the node table from device FP32 values d_knots (length ntab), e.g.
 * learnable knots.  Stream-ordered (a small kernel writes Omega * K into the
 * plan's table); d_knots may be reused once the call's work has run.
 * ESTATE unless the plan was created with ARKCOS_PLAN_LEARNABLE.
 */
int arkcos_plan_set_kernel(arkcos_plan_t plan, const float *d_knots, void *stream);

/* ------------------------------------------------------------- compute -- */

/*
 * Forward real-space convolution of nbatch maps (the ARKCoS term, Sec. 2).
 *   d_in   device FP32, nbatch x Npix, RING order, map b at d_in + b*Npix  [in]
 *   d_out  device FP32, same layout, overwritten                          [out]
 * d_in and d_out must not overlap.  1 <= nbatch <= max_batch.
 * EINVAL on bad arguments, ESTATE for a host-only plan or unset knots,
 * EDEVICE if a launch fails.
 */
int arkcos_convolve(arkcos_plan_t plan, const float *d_in, float *d_out, int nbatch,
                    void *stream);

/*
 * One or both gathers of arkcos_convolve (part = ARKCOS_PART_*): the rings of
 * the other gather are left untouched in d_out.  Running both parts, in either
 * order, equals arkcos_convolve bit for bit.  For timing and testing the two
 * kernels separately; arguments and errors as arkcos_convolve, plus EINVAL for
 * an unknown part.
 */
int arkcos_convolve_part(arkcos_plan_t plan, const float *d_in, float *d_out, int nbatch, int part,
                         void *stream);

/*
 * Adjoint of arkcos_convolve for a loss L with d_grad_out = dL/d(out):
 *   d_grad_in    = A^T g, the transposed gather; A is symmetric (theta_pq =
 *                  theta_qp, one Omega), so this is the same sum applied to g;
 *   d_grad_knots = dL/dK_k = Omega sum_p g[p] sum_q Lambda_k(theta_pq) in[q],
 *                  summed over the batch, with Lambda_k the linear hat of node k
 *                  (derivative of the interpolated kernel of Sec. 3 with respect
 *                  to its nodes), with respect to the unscaled knots.
 *   d_grad_out   device FP32, nbatch x Npix                                 [in]
 *   d_in         device FP32, nbatch x Npix (needed only for knot gradients;
 *                may be NULL when d_grad_knots is NULL)                      [in]
 *   d_grad_in    device FP32, nbatch x Npix, overwritten, or NULL            [out]
 *   d_grad_knots device FP32, ntab, overwritten, or NULL                      [out]
 * At least one output must be non-NULL; outputs must not overlap inputs.
 * Knot gradients need ARKCOS_PLAN_LEARNABLE and ntab <= ARKCOS_MAX_GRAD_NTAB
 * (EUNSUPPORTED otherwise).  Both outputs are bitwise reproducible for a
 * plan on a given device: every output pixel of d_grad_in is written by one
 * lane, and the knot gradient is accumulated in FP64 with a static
 * assignment of work to waves, one histogram per wave, and fixed-order
 * merges of the wave and workgroup partials.
 */
int arkcos_convolve_backward(arkcos_plan_t plan, const float *d_grad_out, const float *d_in,
                             float *d_grad_in, float *d_grad_knots, int nbatch, void *stream);

/*
 * arkcos_convolve_backward for callers that cannot allocate device memory at
 * call time or cannot tolerate an allocation in the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Arguments,
 * results and errors are those of arkcos_convolve_backward, and the results
 * are bit for bit the same; the difference is the workspace.  The gathers'
 * queue counters and the knot-gradient partial rows live in a file-scope
 * device array of ARKCOS_STATIC_SCRATCH_BYTES bytes instead of the plan's
 * workspace; each device that runs this call holds its own copy from the
 * library's load until the process ends.  The call itself allocates nothing
 * (no hipMalloc, no allocating library routine); its device address is looked
 * up once per device, on the first call there.  EUNSUPPORTED if the plan's
 * knot-gradient partials (one row of ntab FP64 values per resident workgroup
 * of the two knot kernels, no more than their work items; 16 MiB for
 * ntab = 2048 on a 256-CU device) exceed the array.  Every call on one device shares its array, so
 * calls whose work overlaps on a device race and give wrong results: order
 * them on one stream (or synchronise between streams).  The array keeps the
 * last call's contents; everything a call reads from it is first written by
 * that call.
 */
int arkcos_convolve_backward_static(arkcos_plan_t plan, const float *d_grad_out,
                                    const float *d_in, float *d_grad_in, float *d_grad_knots,
                                    int nbatch, void *stream);

/* ------------------------------------------------------------- batches -- */

/*
 * Group nmaps plans (mixed Nside, theta_cut and node tables) into one work
 * queue that a single persistent launch drains; tiles are ordered
 * longest-first.  The plans must outlive the batch and must not be
 * host-only.  Allocates device memory (synchronously).  Each plan takes one
 * map (nbatch 1) per call.
 */
int arkcos_batch_create(const arkcos_plan_t *plans, int nmaps, arkcos_batch_t *out);

/*
 * Convolve map k of the batch with plan k, k = 0..nmaps-1, in one launch.
 *   d_in   host array of nmaps device pointers (FP32, Npix_k each)  [in]
 *   d_out  host array of nmaps device pointers, overwritten          [out]
 * The pointer arrays are copied into the launch arguments; no allocation.
 */
int arkcos_batch_convolve(arkcos_batch_t batch, const float *const *d_in, float *const *d_out,
                          void *stream);

/*
 * One or both gathers of arkcos_batch_convolve (part = ARKCOS_PART_*), one
 * persistent launch each; the rings of the other gather are left untouched.
 * Both parts, in either order, equal arkcos_batch_convolve bit for bit.
 */
int arkcos_batch_convolve_part(arkcos_batch_t batch, const float *const *d_in,
                               float *const *d_out, int part, void *stream);

/* Release a batch (not its plans).  NULL is accepted. */
int arkcos_batch_destroy(arkcos_batch_t batch);

/* ---------------------------------------------------------- autotuning -- */

/*
 * Tile autotuning.  The best general-gather tiles depend on the device, on
 * Nside and on the disc radius in pixels, which sets the source windows; the
 * tuning cache is a text file with one line per (arch, Nside, window class):
 *     <arch> <nside> <class> <gen_pixels> <gen_quad_window> <gen_pair_window> <ms>
 * ('#' starts a comment; a later line for the same key wins).  The window
 * class is round(2 log2(theta_cut / sqrt(Omega))), Omega = 4 pi / Npix, plus
 * ARKCOS_TUNE_RANGE_CLASS for a descriptor with an output ring range that is
 * not the whole sky (such plans tile part of the general rings only and keep
 * entries of their own).
 *
 * arkcos_set_tune_cache: the cache that plans with all-zero tiles read at
 * creation (copied; NULL or "" = none).  Until it is called the environment
 * variable ARKCOS_TUNE_CACHE names it.  Process-wide.
 */
int arkcos_set_tune_cache(const char *path);

#define ARKCOS_TUNE_RANGE_CLASS 100

/*
 * The cache key of a whole-sky descriptor: arch (the current device's gfx
 * name, or the library's build target gfx950 without a device), Nside and
 * window class (a ring-range descriptor adds ARKCOS_TUNE_RANGE_CLASS).
 *   arch  host buffer of len bytes, NUL-terminated on return (may be NULL)  [out]
 * EINVAL on a bad nside / theta_cut.
 */
int arkcos_tune_key(int nside, double theta_cut, char *arch, int len, int *window_class);

/*
 * Autotune the general-gather tiles of a descriptor on the current device:
 * builds the plan once (with desc->ktab, or a flat table if it is NULL),
 * allocates an input and an output map, and times the general gather (median
 * of reps >= 1 launches after a warm-up) over candidate tiles by coordinate
 * descent: gen_pixels in {32, 64, 128}, gen_quad_window in {-1, 32, 64, 96,
 * 128}, gen_pair_window in {-1, 100, 200, 400, 800}.  Fields of desc->tiles
 * that are non-zero stay fixed.  The best tiles and their time go to *best
 * and *best_ms, the built-in defaults' time to *default_ms (either pointer may
 * be NULL), and, if cache_path is non-NULL, a line is appended to that file.
 * Synchronous; allocates device memory.  Errors as arkcos_plan_create, EDEVICE
 * on timing failures, EINVAL if the cache file cannot be written.
 */
int arkcos_tune(const arkcos_plan_desc *desc, int reps, const char *cache_path,
                arkcos_tiles *best, double *best_ms, double *default_ms);

/* ----------------------------------------------------------- diagnostics -- */

/* Static text for a status code. */
/* ------------------------------------------- harmonic-space half (SHT) -- */

/*
 * The l-space half of the split convolution (Sec. 2, eq. 1, and the
 * l-space cost eq. 4): the truncated harmonic kernel Khat_l, l <= lcut,
 * applied by spherical-harmonic analysis with the pixel quadrature and
 * synthesis on a HEALPix RING map,
 *     a_lm = Omega sum_p in[p] conj(Y_lm(p)),
 *     out[p] = sum_{l <= lcut} Khat_l sum_{m=-l..l} a_lm Y_lm(p),
 * with orthonormal Y_lm.  By the addition theorem this equals the all-pairs
 * sum Omega sum_q K_l(theta_pq) in[q] with the untruncated kernel
 * K_l(theta) = sum_l (2l+1)/(4 pi) Khat_l P_l(cos theta).  The paper applies
 * this half on host cores; here it runs on the GPU in FP64.
 *
 * arkcos_harm_create: Nside 1..ARKCOS_MAX_NSIDE, lcut 0..ARKCOS_MAX_LCUT
 * (EUNSUPPORTED above), khat host FP64 of lcut+1 values (copied), max_batch
 * >= 1.  Allocates device memory on the current device (synchronously):
 * per-ring longitude sums (lcut+1) x (4 Nside - 1) complex FP64, per-chunk
 * partial coefficients, recurrence tables.  EINVAL, ENOMEM, EDEVICE.
 */
int arkcos_harm_create(int nside, int lcut, const double *khat, int max_batch,
                       arkcos_harm_t *out);

/* Release a transform plan (synchronises the device).  NULL is accepted. */
int arkcos_harm_destroy(arkcos_harm_t harm);

/* Replace Khat_l (host FP64, lcut+1 values; synchronous upload). */
int arkcos_harm_set_kernel(arkcos_harm_t harm, const double *khat);

/* Nside, lcut, number of (l, m >= 0) coefficients and device bytes; any
 * out-pointer may be NULL. */
int arkcos_harm_get_info(arkcos_harm_t harm, int *nside, int *lcut, long long *nalm,
                         long long *device_bytes);

/*
 * The l-space half on nbatch maps (same layout as arkcos_convolve).
 *   d_in        device FP32, nbatch x Npix                                [in]
 *   d_out       device FP32, nbatch x Npix: overwritten (accumulate = 0) or
 *               added to (accumulate = 1)                                  [out]
 * d_in and d_out must not overlap.  Stream-ordered, no allocation or
 * synchronisation; a transform plan serves one stream at a time (its
 * workspace is shared by its calls).  EINVAL on bad arguments.
 */
int arkcos_harm_convolve(arkcos_harm_t harm, const float *d_in, float *d_out, int nbatch,
                         int accumulate, void *stream);

/*
 * The full split convolution of Sec. 2 (eq. 1): out = (real-space half of
 * `plan`) + (l-space half of `harm`), i.e. the approximate kernel
 * Ktilde_l = Khat_l + P_{l theta} Khat_theta applied to each map.  The two
 * halves run back to back on `stream`.  The plans must share Nside (EINVAL);
 * other arguments and errors as arkcos_convolve and arkcos_harm_convolve.
 */
int arkcos_split_convolve(arkcos_plan_t plan, arkcos_harm_t harm, const float *d_in,
                          float *d_out, int nbatch, void *stream);

/* ------------------------------------------ polar-cap reorientation -- */
/*
 * The rotation that takes the direction (theta, phi) (colatitude and
 * longitude, radians) to the north pole: R = R_y(-theta) R_z(-phi), written
 * row-major into rot[9] (host).  With it, arkcos_rotate_map moves a survey
 * patch centred on (theta, phi) onto the north polar cap, where a ring-range
 * plan convolves it over the few rings it spans (Sec. 4, Conclusions).
 * EINVAL on NULL or non-finite angles.
 */
int arkcos_rotation_to_pole(double theta, double phi, double *rot);

/*
 * Rotated copy of nbatch RING maps (stride Npix) at nearest-pixel resampling:
 * for every pixel p of output rings ring_first..ring_last (1-based,
 * inclusive; 0, 0 = all), with centre n_p,
 *     d_out[p] = d_in[q],  q the pixel whose boundaries contain R^T n_p,
 * so a feature at direction c of d_in appears at R c of d_out.  Pixels of
 * other rings are not written.  rot: 9 host doubles, row-major, a rotation
 * (|R R^T - I| <= 1e-9 and det R > 0, else EINVAL); copied.  Geometry and
 * point location run in FP64 on the device.  d_in and d_out must not overlap
 * (EINVAL).  Asynchronous on `stream`; allocates nothing.
 */
int arkcos_rotate_map(int nside, const double *rot, const float *d_in, float *d_out, int nbatch,
                      int ring_first, int ring_last, void *stream);

const char *arkcos_status_string(int status);

/* Per-thread detail of the last failing call ("" if none). */
const char *arkcos_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int arkcos_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ARKCOS_H */
