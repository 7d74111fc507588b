/*
 * wost.h -- C interface of the walk-on-stars (WoSt) solver for AMD MI355X.
 *
 * Method: Sawhney, Miller, Gkioulekas and Crane, "Walk on Stars: A Grid-Free
 * Monte Carlo Method for PDEs with Neumann Boundary Conditions", ACM TOG
 * 42(4), 2023.  The library estimates, at given points x of a domain, the
 * solution of the Poisson problem of Sec. 3.2, Eq. (PoissonEquation):
 *
 *     Laplacian(u) = f  in the domain,
 *     u = g             on the Dirichlet boundary,
 *     du/dn = h         on the Neumann boundary, n the unit OUTWARD normal,
 *
 * by averaging independent random walks (the WoSt estimator of Sec. 4.3 and
 * Sec. 4.7, Algorithm 1).  Each walk step queries the boundary geometry
 * (Sec. 5: closest point, closest silhouette point, ray intersection and
 * point sampling) through trees built once per scene.
 *
 * Conventions used by every call:
 *   - Boundaries are meshes: segments in 2D (dim = 2), triangles in 3D
 *     (dim = 3).  A segment (a, b) has outward normal (b_y - a_y, a_x - b_x)
 *     normalised; a triangle (a, b, c) has outward normal (b - a) x (c - a)
 *     normalised.  Meshes need not be watertight (Sec. 5).
 *   - Coordinates and walk state are FP32; per-walk sums are Kahan-
 *     compensated FP32; per-point means and variances are reduced in FP64.
 *   - Random numbers are Philox4x32-10 keyed by the 64-bit seed with
 *     counter (point, walk, step, slot), so results are deterministic in
 *     (scene, points, walks, eps, seed, options) and do not depend on the
 *     launch form, the grid size or the order in which walks run.
 *   - Every function returns a wost_status; no C++ exception crosses this
 *     interface.  After a non-OK status, wost_last_error() returns a
 *     thread-local message.
 *   - Input arrays are borrowed for the duration of the call only.
 *     Output arrays are allocated by the caller.
 *   - Calls that use the same scene must not overlap in time (they share
 *     the scene's device scratch buffers); different scenes may be used
 *     from different threads.
 */
#ifndef WOST_H
#define WOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wost_scene_s* wost_scene;   /* opaque; owned by the library */

typedef enum {
  WOST_OK = 0,
  WOST_ERR_INVALID_ARG = 1,     /* bad argument: see wost_last_error() */
  WOST_ERR_OUT_OF_MEMORY = 2,   /* a device or host allocation failed */
  WOST_ERR_DEVICE = 3,          /* a HIP runtime call or kernel launch failed */
  WOST_ERR_NOT_SUPPORTED = 4,   /* e.g. a scene without Dirichlet boundary */
  WOST_ERR_INTERNAL = 5
} wost_status;

/* Kinds of scalar fields for g, h and f (the paper passes them as
 * callbacks, Sec. 6; a device cannot call host code, so they are given as
 * data the device evaluates). */
typedef enum {
  WOST_FN_ZERO = 0,
  WOST_FN_CONST = 1,       /* coef[0] */
  WOST_FN_POLY2 = 2,       /* 3D: c + x + y + z + xx + yy + zz + xy + yz + zx (10 coefs)
                              2D: c + x + y + xx + yy + xy (6 coefs) */
  WOST_FN_EXPCOS = 3,      /* coef[0] * exp(coef[1] x) * cos(coef[1] y) */
  WOST_FN_PER_CORNER = 4,  /* per_corner[prim][corner], linear over the primitive (g, h only) */
  WOST_FN_EXPLIN = 5       /* coef[0] * exp(coef[1] x + coef[2] y + coef[3] z); solves
                              Laplacian(u) - sigma u = 0 for sigma = |coef[1..3]|^2 */
} wost_fn_kind;

typedef struct {
  int32_t kind;                 /* wost_fn_kind */
  int32_t as_normal_derivative; /* h only: 1 = h(z) = grad(F)(z) . n(prim) for the analytic F
                                   given by (kind, coef); lets an exact u supply g = u and
                                   h = du/dn exactly */
  double coef[10];
  const float* per_corner;      /* host, [n_prims][dim], read during wost_build_scene only */
} wost_fn;

/* Analytic Dirichlet shapes (mixed representations, Sec. 6: a mesh beside
 * implicit surfaces; the paper leaves silhouettes of implicit surfaces open,
 * so shapes carry Dirichlet data only).  Their surfaces are Dirichlet
 * boundary with the scene's g; they take part in the closest-point query
 * only.  p: 2D shapes use the first two coordinates of each point. */
typedef enum {
  WOST_SDF_BALL = 0,      /* centre p[0..2], radius p[6] */
  WOST_SDF_BOX = 1,       /* centre p[0..2], half extents p[3..5] (> 0), rounding radius p[6] (>= 0) */
  WOST_SDF_CAPSULE = 2    /* segment p[0..2] - p[3..5], radius p[6] (> 0) */
} wost_sdf_kind;

typedef struct {
  int32_t kind;     /* wost_sdf_kind */
  int32_t inside;   /* 1: the domain lies inside the shape (BALL, or BOX without rounding);
                       0: outside it */
  double p[8];
} wost_sdf;

typedef struct {
  int32_t dim;                  /* 2 or 3 */
  int64_t n_vertices;
  const float* vertices;        /* host, [n_vertices][dim] */
  int64_t n_prims;
  const int32_t* prims;         /* host, [n_prims][dim] vertex indices */
  const uint8_t* bc;            /* host, [n_prims]: 0 Dirichlet, 1 Neumann, 2 double-sided
                                   Dirichlet, 3 double-sided Neumann (see below) */
  wost_fn g;                    /* on Dirichlet primitives ("+" side of double-sided ones) */
  wost_fn h;                    /* on Neumann primitives ("+" side of double-sided ones) */
  wost_fn f;                    /* in the domain (ZERO, CONST or POLY2) */
  wost_fn g_minus;              /* "-" side of double-sided Dirichlet primitives */
  wost_fn h_minus;              /* "-" side of double-sided Neumann primitives; a normal
                                   derivative here is taken along n- = -n */
  int64_t n_sdf;                /* analytic Dirichlet shapes, 0..256 */
  const wost_sdf* sdf;          /* host, [n_sdf], copied; with shapes, g must be analytic (not
                                   PER_CORNER), and the mesh may be empty (n_prims = 0). The
                                   closest-point query reports shape i as n_prims + i. */
} wost_scene_desc;

/* Double-sided primitives (appendix "Open Domains and Double-Sided
 * Boundaries"): sheets inside the domain, open or closed, that carry boundary
 * data on both sides.  The "+" side of a primitive is the side its normal
 * points away from (the inside of a closed surface with outward normals), the
 * "-" side the one it points into; adjacent primitives of one sheet must be
 * oriented alike.  A walk takes g+ or g- by the side it approached from
 * (x_k - x_{k-1} against n), takes the normal of its own side when it lands
 * on a Neumann sheet, and takes h+ or h- for a Neumann sample by the side of
 * the sample's primitive that its query origin sees.  One-sided primitives
 * (0, 1) use g and h.  Walks of a domain that is not closed by a Dirichlet
 * boundary may wander off; they end at the escape radius (opts.escape_rel). */

/* Solve options; pass NULL for the defaults (each field's "<= 0" value
 * selects its default). */
typedef struct {
  float r_min;        /* minimum star radius (Sec. 4.4.3); default eps */
  int32_t max_steps;  /* walk-length cap; a capped walk returns g at its closest
                         Dirichlet point and is counted; default 65536 */
  float offset_rel;   /* inward offset of query origins on the Neumann boundary
                         (footnote of Sec. 4.4), relative to the scene's
                         half-diagonal L; default 2^-18 */
  float escape_rel;   /* a walk farther than escape_rel * L from the scene centre
                         is stopped and counted as escaped; default 2 */
  int32_t mode;       /* 0 persistent kernel with lane refill whose waves share
                         each tree search among their lanes by work stealing
                         (default), 1 plain launch, one lane per walk,
                         2 persistent kernel with lane refill, each lane
                         searching alone */
  int32_t grid;       /* persistent kernel: blocks; default = resident capacity */
  int32_t refill;     /* persistent kernel: refill a wave when at least this many
                         lanes are idle (1..64); default 1 */
  uint32_t flags;     /* 0, or WOST_SOLVE_COUNT_TRAFFIC */
  int32_t chunk_walks;/* batched form: walks per work-queue chunk; 0 = about four
                         chunks per resident wave, 64..2048 walks */
  int32_t walk_order; /* grouping of walks into waves: 0 point-major (the walks of
                         a point are consecutive), 1 walk-major (walk j of
                         consecutive points) */
  float sigma;        /* screening coefficient: solves Laplacian(u) - sigma u = f
                         (Sec. 3.2, Eq. ScreenedPoissonEquation); 0 (default):
                         Poisson.  Each step's continuation factor
                         Q^{sigma,B} (App. A.2) is applied as Russian
                         roulette; Neumann and source terms use the screened
                         ball Green's function */
  float tikhonov_sigma;  /* Tikhonov switch (Sec. 3.4, pure Neumann problems):
                         from step tikhonov_steps on, sigma + tikhonov_sigma
                         is used; 0 (default): off */
  int32_t tikhonov_steps;
  int32_t claim_walks;   /* 2D persistent kernel: most walks a wave takes from the work
                            queue at once (one atomic per claim; claims shrink near the
                            end of the work); default 128.  3D waves always claim
                            their idle lanes' share */
  int32_t steal_lanes;   /* 3D cooperative searches (mode 0): a wave starts a steal
                            round once at least this many of its lanes are idle
                            (1..64); default 16.  2D waves steal as soon as one lane
                            is idle */
} wost_solve_opts;

/* opts.flags: run the traffic-accounting variant of the walk kernel (plain
 * form, same traversals, plus per-lane fetch counters read back by
 * wost_get_traffic).  Results are identical; it is slower and not timed. */
#define WOST_SOLVE_COUNT_TRAFFIC 1u

/* Counters of the last solve on a scene. */
typedef struct {
  uint64_t steps;     /* executed walk steps: one per closest-point query, the
                         terminating one included */
  uint64_t walks;
  uint64_t capped;
  uint64_t escaped;
  double kernel_ms;   /* device time of the walk kernel */
  int32_t mode;       /* launch form used: 0 persistent (cooperative), 1 plain,
                         2 batched, 3 persistent with per-lane searches */
  int32_t grid_blocks;/* blocks of the walk kernel's grid */
  int32_t graph_captures; /* batched form: graphs this batch context has captured so
                         far (a new call re-captures only when the kinds of its groups
                         or its buffers change); 0 for per-scene solves */
} wost_stats;

/* Tree and primitive fetches of the last solve run with
 * WOST_SOLVE_COUNT_TRAFFIC, per query: Q.1 closest point, Q.2 closest
 * silhouette point (nodes, node cones, elements), Q.3 ray, Q.4 Neumann
 * sample descent, and the visibility ray of the Neumann term.  *_bytes give
 * the bytes one fetch of each kind reads (3D: a Q.1, Q.2, Q.3 or visibility
 * node visit reads one 4-wide record of wide_node_bytes, a Q.2 record's
 * cones included; a Q.4 visit reads a binary node of node_bytes);
 * `bytes` is the
 * algorithmic total (fetches x their sizes, plus per-walk input/output). */
typedef struct {
  uint64_t q1_nodes, q1_prims;
  uint64_t q2_nodes, q2_cones, q2_elems;
  uint64_t q3_nodes, q3_prims;
  uint64_t q4_nodes, q4_prims;
  uint64_t vis_nodes, vis_prims;
  /* wave-level iteration counts (one per wave per loop pass) of the Q.1,
   * Q.2, Q.3 traversal loops and their leaf loops, the Q.4 descent, the
   * visibility traversal and its leaf loop, and of walk steps; with the
   * lane-level counts above they give each loop's SIMT efficiency */
  uint64_t wave_q1, wave_q1_leaf, wave_q2, wave_q2_leaf, wave_q3, wave_q3_leaf, wave_q4;
  uint64_t wave_vis, wave_vis_leaf, wave_steps;
  /* wave-level shader-clock cycles (x16) spent in Q.1, Q.2, Q.3, in the
   * Neumann and source terms (Q.4 and the visibility ray), and in the rest
   * of the loop (RNG, bookkeeping, refill, idle lanes of finished walks) */
  uint64_t cyc_q1, cyc_q2, cyc_q3, cyc_q4, cyc_rest;
  uint32_t node_bytes, cone_bytes, prim_bytes, elem_bytes;
  uint64_t io_bytes;
  uint64_t bytes;
  uint32_t wide_node_bytes;
} wost_traffic;

typedef struct {
  int32_t dim;
  int64_t n_prims, n_dirichlet, n_neumann, n_silhouette_elements;
  int64_t nodes_dirichlet, nodes_neumann, nodes_silhouette;
  int32_t depth_dirichlet, depth_neumann, depth_silhouette;
  int64_t device_bytes;   /* bytes of trees and primitives resident on the device */
  double half_diagonal;   /* L: half the diagonal of the box of the vertices and the shapes */
  double center[3];
  int64_t n_sdf;          /* analytic Dirichlet shapes */
} wost_scene_info;

/* FP32 record of one walk step (parity and diagnostics).  Primitive ids are
 * indices into the scene description's prims array; -1 means none. */
typedef struct {
  float x[3], n[3];   /* position and, when on_neumann, the normal of the walk's side
                         (the outward normal; its negation on the "-" side of a
                         double-sided primitive) */
  int32_t on_neumann, cur;
  float d_dirichlet;  /* Q.1 distance */
  float xbar[3];      /* Q.1 closest point */
  int32_t prim_dirichlet;
  int32_t term;       /* 0 continues, 1 eps-shell, 2 capped, 3 escaped, 4 roulette */
  float g_term;       /* g(xbar) when the walk ends at this step */
  float d_silhouette; /* Q.2 distance within d_dirichlet */
  float r;            /* star radius */
  float v[3];         /* direction */
  int32_t hit, hit_prim;
  float t;            /* distance to the next point along v */
  float p[3];         /* next point */
  int32_t n_prim, valid;  /* Neumann sample: primitive, accepted */
  float z[3];
  float pdf, n_hat;   /* sample pdf, Neumann contribution */
  float s_frac, s_hat;/* source distance fraction, source contribution */
  float acc;          /* walk estimate so far */
  float q;            /* screened continuation factor Q^{sigma,B} (1 for Poisson) */
  int32_t roulette;   /* 1: the walk ended at this step by Russian roulette */
  int32_t side_g;     /* double-sided Dirichlet end: +1 / -1 side of g used; else 0 */
  int32_t side_h;     /* accepted Neumann sample on a double-sided primitive: +1 / -1
                         side of h used; else 0 */
} wost_step_rec;

/* Builds the trees of a scene on the host (binned-SAH bounding volume
 * hierarchies over the Dirichlet and Neumann primitives, a normal-cone
 * hierarchy over the silhouette elements of the Neumann boundary, Sec. 5.1)
 * and uploads them to the current HIP device.
 * Errors: INVALID_ARG for dim not 2/3, empty or out-of-range index arrays,
 * non-finite coordinates, zero-measure primitives, bc values other than 0/1,
 * a PER_CORNER field without data or an unsupported kind for f;
 * (a scene without Dirichlet primitives is accepted; solving it needs
 * opts.sigma > 0 or the Tikhonov switch, else NOT_SUPPORTED at solve time);
 * OUT_OF_MEMORY / DEVICE on allocation or copy failure.
 * On success *out receives a scene owned by the library. */
wost_status wost_build_scene(const wost_scene_desc* desc, wost_scene* out);

/* Releases a scene and its device memory.  NULL is accepted. */
wost_status wost_destroy_scene(wost_scene scene);

/* Sizes of a built scene. */
wost_status wost_get_scene_info(wost_scene scene, wost_scene_info* info);

/* Host-only check: runs the same preprocessing as wost_build_scene without
 * touching any device, validates the trees (every item in exactly one leaf,
 * child boxes contain their items, depth within the traversal stack) and
 * reports their sizes in *info (device_bytes is what an upload would use). */
wost_status wost_check_scene_host(const wost_scene_desc* desc, wost_scene_info* info);

/* Estimates u at n_points points with walks_per_point walks each
 * (Sec. 3.4.1: the mean of independent single-walk estimates).
 * points: host, [n_points][dim] FP32, inside the domain (points outside
 * are not detected; their walks may be counted as escaped).
 * mean_out, var_out: host, [n_points] FP64: the per-point mean and the
 * unbiased sample variance of the walk estimates (0 when walks_per_point
 * is 1); the standard error is sqrt(var / walks_per_point).
 * eps: the eps-shell width of the Dirichlet boundary (Sec. 3.4.2), > 0.
 * Blocks until the results are on the host.
 * Errors: INVALID_ARG for n_points < 0, walks_per_point < 1, eps <= 0 or
 * non-finite, NULL arrays; OUT_OF_MEMORY; DEVICE. */
wost_status wost_solve(wost_scene scene, const float* points, int64_t n_points,
                       int32_t walks_per_point, float eps, uint64_t seed, double* mean_out,
                       double* var_out);

/* Device-pointer form of wost_solve: d_points [n_points][dim] FP32 and
 * d_mean, d_var [n_points] FP64 are device pointers (for instance the data
 * pointers of torch tensors); the work is enqueued on `hip_stream`
 * (a hipStream_t; NULL = the null stream) and the call returns without
 * synchronising.  opts may be NULL.  The scene keeps a device buffer of
 * n_points * walks_per_point FP32 walk estimates between calls.
 * point_base / walk_base offset the RNG counters (point index of point 0,
 * walk index of walk 0), so that a large solve split into pieces draws the
 * same random numbers as the whole. */
wost_status wost_solve_ex(wost_scene scene, const float* d_points, int64_t n_points,
                          int32_t walks_per_point, float eps, uint64_t seed,
                          uint32_t point_base, uint32_t walk_base, const wost_solve_opts* opts,
                          double* d_mean, double* d_var, void* hip_stream);

/* Allocation-free form of wost_solve_ex, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  Same arguments, same kernels and bit-identical
 * results; opts.flags must be 0 (no traffic accounting).  Instead of the
 * scene's own buffers it uses one fixed device array per GPU, held by the
 * library until the process ends: 4 KiB of counters and room for 2^23
 * per-walk estimates (32 MiB).  A solve whose n_points * walks_per_point
 * exceeds 2^23 runs as several launches over consecutive point ranges
 * (each with its points' own random-number ids); walks_per_point above 2^23
 * is rejected with INVALID_ARG.  The call allocates nothing on the device
 * or the host side of HIP (no hipMalloc, no hipFree, no library routine
 * that allocates); the scene's timing events exist from wost_build_scene.
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents (the counters are cleared by a fill kernel at each call):
 * calls that overlap in time on one GPU race, and wost_get_stats /
 * wost_get_walk_events after such a call read the array, so they describe
 * the last no-alloc call on that GPU.  Enqueued on hip_stream; returns
 * without synchronising. */
wost_status wost_solve_ex_noalloc(wost_scene scene, const float* d_points, int64_t n_points,
                                  int32_t walks_per_point, float eps, uint64_t seed, uint32_t point_base,
                                  uint32_t walk_base, const wost_solve_opts* opts, double* d_mean,
                                  double* d_var, void* hip_stream);

/* Evaluation points on the Neumann boundary (Algorithm 1 with its
 * on-boundary flag set at the start, Sec. 4.4.4): as wost_solve_ex, except
 * that prims [n_points] (host int32, the numbering of desc->prims) gives for
 * each point the Neumann primitive it lies on, or -1 for an interior point;
 * on a double-sided Neumann primitive p, the entry p starts the walk on its
 * "+" side and -2 - p on its "-" side.
 * A boundary walk starts on that primitive with its side's normal, so its
 * first step samples the inward hemisphere and weights the Neumann term by
 * 1 / alpha, alpha = 1/2 (the point must lie on the primitive, away from its
 * edges, where the boundary is smooth).  The call waits for the scene's
 * earlier work on hip_stream before staging the primitive list.
 * Errors: as wost_solve_ex; INVALID_ARG for NULL prims with n_points > 0 or
 * an entry that is neither -1, a Neumann primitive, nor -2 - (a double-sided
 * Neumann primitive). */
wost_status wost_solve_boundary_ex(wost_scene scene, const float* d_points, const int32_t* prims,
                                   int64_t n_points, int32_t walks_per_point, float eps,
                                   uint64_t seed, uint32_t point_base, uint32_t walk_base,
                                   const wost_solve_opts* opts, double* d_mean, double* d_var,
                                   void* hip_stream);

/* Autotuner: times short solves of a prefix of the given points (about
 * sample_walks walks per trial; <= 0: 2^20) over the knobs of the persistent
 * cooperative kernel -- refill threshold, grid size, walk order (how walks
 * are grouped into waves), claim size and steal threshold -- by a
 * coordinate search (each knob over its candidates with the others at their
 * best so far, two passes), and writes the fastest into *opts (its other
 * fields are kept; mode is set to 0).  Every candidate produces identical
 * estimates, so tuning never changes results.  The traversal stack depth is
 * not a knob: it is fixed by the deepest tree the builder makes.
 * d_points: device [n_points][dim]; runs on hip_stream and synchronises. */
wost_status wost_autotune(wost_scene scene, const float* d_points, int64_t n_points,
                          int32_t walks_per_point, float eps, uint64_t seed, int64_t sample_walks,
                          wost_solve_opts* opts, void* hip_stream);

/* Counters of the last solve on `scene`; synchronises with it. */
wost_status wost_get_stats(wost_scene scene, wost_stats* out);

/* Walks of the last solve on `scene` that ended at the step cap (kind 2) or
 * beyond the escape radius (kind 3), in the order they ended, at most the
 * first 64 (more are counted in wost_stats but not listed): their RNG point
 * and walk indices and their length in steps, so that they can be re-run
 * step by step with wost_trace_walks.  point_ids, walk_ids, steps, kinds:
 * host arrays of `max` entries; *n_out receives the number written.
 * Synchronises with the solve.  The batched and serving forms keep no list. */
wost_status wost_get_walk_events(wost_scene scene, int32_t max, uint32_t* point_ids, uint32_t* walk_ids,
                                 int32_t* steps, int32_t* kinds, int32_t* n_out);

/* Fetch counters of the last solve on `scene` that ran with
 * WOST_SOLVE_COUNT_TRAFFIC (all zero otherwise); synchronises with it. */
wost_status wost_get_traffic(wost_scene scene, wost_traffic* out);

/* Runs n walks on their own and records up to max_rec steps of each.
 * points [n][dim] FP32 host (start of walk i), point_ids / walk_ids [n]
 * give each walk's RNG counters; prims [n] host (optional, NULL: all
 * interior) the Neumann primitive a start point lies on or -1, as in
 * wost_solve_boundary_ex; recs [n][max_rec] host; n_steps [n] and values
 * [n] host receive the walk length and the walk estimate. */
wost_status wost_trace_walks(wost_scene scene, const float* points, const uint32_t* point_ids,
                             const uint32_t* walk_ids, const int32_t* prims, int64_t n, float eps,
                             uint64_t seed, const wost_solve_opts* opts, int32_t max_rec,
                             wost_step_rec* recs, int32_t* n_steps, float* values);

/* Measurement aid for the roofline of the walk kernels, whose trees stay in
 * L2: the read bandwidth of a streaming kernel in which 4 blocks per CU each
 * read a `bytes`-long device buffer (<= 0: 2 MiB, resident in every XCD's
 * L2 after a warm-up pass; at most 64 MiB, a multiple of 16) `reps` times
 * (<= 0: 16).  *gbs receives the GB/s over the timed launch (HIP events on
 * the null stream).  Allocates and frees its own buffers; synchronises. */
wost_status wost_measure_l2_read(int64_t bytes, int32_t reps, double* gbs);

/* Measures the vector ALU's issue rate: 8 blocks of 256 lanes per compute
 * unit each run 8 independent chains of `iters` (<= 0: 1024) links, after a
 * warm-up launch; kind 0: a link is one FP32 fused multiply-add, kind 1: an
 * integer xor and an add (integer work issues faster than FP32 work, so a
 * walk kernel's mix of both can exceed the FP32 rate).  *glanes receives
 * the VALU lane instructions per second over the timed launch, in units of
 * 10^9 (HIP events on the null stream).  Allocates and frees its own
 * buffer; synchronises. */
wost_status wost_measure_valu(int32_t kind, int32_t iters, double* glanes);

/* Q.1 probe: distance d [n], closest point xbar [n][dim] and primitive id
 * prim [n] of the Dirichlet boundary from points x [n][dim] (host arrays);
 * analytic shape i is reported as n_prims + i, no boundary at all as -1. */
wost_status wost_probe_closest_point(wost_scene scene, const float* x, int64_t n, float* d,
                                     float* xbar, int32_t* prim);

/* Q.2 probe (Algorithms 2-4 semantics; closest rather than first silhouette
 * element): distance from x [n][dim] to the closest silhouette point of the
 * Neumann boundary within rmax [n]; d [n] = rmax[i] when there is none. */
wost_status wost_probe_silhouette(wost_scene scene, const float* x, const float* rmax, int64_t n,
                                  float* d);

/* Q.3 probe: first crossing of o + t v (o, v [n][dim]; v need not be unit,
 * t is in units of |v|) with the Neumann boundary for 0 < t <= tmax [n],
 * ignoring primitive skip [n] (-1 for none).  t [n] (tmax when no hit) and
 * prim [n] (-1 when no hit).  As in the walks, a crossing at
 * -64 offset |v| < t |v| <= 0 (offset = 2^-18 L) of a one-sided primitive
 * that the ray leaves (v . n > 0) counts as a crossing at t = 0 when o lies
 * outside the primitive's plane by less than offset/4: the origin lies on
 * that primitive up to rounding. */
wost_status wost_probe_ray(wost_scene scene, const float* o, const float* v, const float* tmax,
                           const int32_t* skip, int64_t n, float* t, int32_t* prim);

/* Q.4 probe (Algorithms 5-6): one Neumann point sample per ball B(x_i, r_i),
 * x [n][dim], r [n]; RNG counter (i, 0, 0, 1...) under `seed`.  z [n][dim],
 * pdf [n] (0 when no primitive was reached) and prim [n] (-1 then). */
wost_status wost_probe_neumann_sample(wost_scene scene, const float* x, const float* r, int64_t n,
                                      uint64_t seed, float* z, float* pdf, int32_t* prim);

/* The binary Neumann tree that Q.4's random descent walks (Algorithms 5-6),
 * exactly as the device holds it, for checks of the sampler's pdf.
 * nodes: [n_nodes][16] (3D) or [n_nodes][12] (2D) FP32 words per node,
 * node 0 the root: child 0's box (3D: lo xyz, hi xyz; 2D: lo xy, hi xy),
 * child 1's box, the two child codes as int32 bit patterns (>= 0 a node
 * index; < 0 a leaf -(slot * 8 + count) - 1 over leaf slots
 * [slot, slot + count); INT32_MIN no child) and the two children's padded
 * bounding radii.  slot_prim [n_slots]: the primitive id at each leaf slot;
 * slot_measure [n_slots]: its length or area as the sampler weighs it (FP32).
 * Any of nodes, slot_prim, slot_measure may be NULL (the counts are always
 * written), so a first call with NULL arrays sizes them.  Host memory
 * owned by the caller; reads the library's host copy, no device work.
 * Errors: INVALID_ARG for a NULL scene or count pointer. */
wost_status wost_get_neumann_tree(wost_scene scene, int64_t* n_nodes, float* nodes, int64_t* n_slots,
                                  int32_t* slot_prim, float* slot_measure);

/* ---- batched form ---------------------------------------------------------
 * Many (scene, point set) solves of uneven sizes in ONE persistent launch
 * per kernel variant, fed by a device work queue of walk chunks and captured
 * with the per-item reductions into a hipGraph.  Each item draws exactly the
 * random numbers wost_solve_ex would draw for it (same seed, point_base,
 * walk_base), so its mean and variance are bit-identical to the per-scene
 * launch. */
typedef struct wost_batch_s* wost_batch;   /* opaque; owned by the library */

typedef struct {
  wost_scene scene;
  const float* d_points;      /* device, [n_points][dim] FP32 */
  int64_t n_points;
  int32_t walks_per_point;
  float eps;
  uint64_t seed;
  uint32_t point_base, walk_base;
  double* d_mean;             /* device, [n_points] FP64 */
  double* d_var;              /* device, [n_points] FP64 */
} wost_batch_item;

/* Creates an empty batch context (device queue, estimate buffer, graph). */
wost_status wost_batch_create(wost_batch* out);

/* Releases a batch context.  NULL is accepted. */
wost_status wost_batch_destroy(wost_batch batch);

/* Enqueues the items on `hip_stream` (NULL = null stream) and returns.
 * Items sharing dim and data kinds run in one persistent launch; the graph
 * is re-captured only when the items differ from the previous call.
 * opts may be NULL (r_min, max_steps, offset_rel, escape_rel, grid,
 * chunk_walks apply to every item; mode and flags must be 0).
 * Errors: INVALID_ARG for a NULL scene or array, n_points < 0,
 * walks_per_point < 1, eps <= 0; OUT_OF_MEMORY; DEVICE. */
wost_status wost_solve_batch(wost_batch batch, const wost_batch_item* items, int32_t n_items,
                             const wost_solve_opts* opts, void* hip_stream);

/* Counters of the last batched solve (summed over items); synchronises. */
wost_status wost_batch_get_stats(wost_batch batch, wost_stats* out);

/* ---- serving form -----------------------------------------------------------
 * A request loop with continuous batching and progressive refinement
 * (the paper's progressive evaluation, Sec. 1 and Sec. 6).  Requests
 * (scene, points, eps, seed, target standard error) wait in a queue until
 * their device buffers fit the memory budget; every wost_server_step runs
 * ONE refinement round for all admitted requests in one batched launch:
 * more walks per point, merged into per-point FP64 (n, mean, M2) with Chan's
 * pairwise formula in round order.  A round has round_walks walks per point;
 * with adaptive rounds, every round after the first instead takes the walks
 * that the request's largest per-point variance says it still needs for its
 * target (15 % margin, a multiple of 64, at least round_walks, at most
 * max_round_walks), so most requests finish in two or three rounds.  The
 * round sizes of a request depend only on its own results.  A request is done when every
 * point's standard error sqrt(M2 / (n - 1) / n) is <= its target (after at
 * least min_walks walks) or max_walks is reached.  Random numbers are keyed
 * by the request's own seed, point index and walk index, so each result is
 * bit-identical whether the request ran alone or among others.
 * Not thread-safe: one thread drives a server. */
typedef struct wost_server_s* wost_server;   /* opaque; owned by the library */

typedef struct {
  int64_t max_device_bytes;   /* admission budget for request buffers; <= 0: 4 GiB */
  int32_t round_walks;        /* walks per point per round; <= 0: 64 */
  int32_t min_walks;          /* <= 0: round_walks */
  int32_t max_walks;          /* <= 0: 65536 */
  int32_t max_active;         /* admitted requests at once; <= 0: 4096 */
  wost_solve_opts solve;      /* walk options (mode and flags must be 0) */
  int32_t adaptive;           /* 0: every round has round_walks walks; 1: adaptive
                                 rounds (see above) */
  int32_t max_round_walks;    /* adaptive rounds: largest round (walks per point),
                                 also held to round_budget_walks / n_points
                                 (rounded down to 64, at least round_walks);
                                 <= 0: 1024.  The memory budget counts each
                                 request's points at dim * 4 + 32 + 4 * (largest
                                 round) bytes */
  int32_t max_rounds;         /* rounds in flight at once (1..4), each with its own
                                 stream and buffers; <= 0: 2 */
  int32_t wait_us;            /* longest wait of wost_server_step for a round to end
                                 when it has no round to start; <= 0: 2000 */
  int64_t round_budget_walks; /* walks in one round: requests join a round in
                                 admission order while they fit (the first always
                                 does), the others wait for the next; <= 0: 2^24 */
} wost_server_config;

enum { WOST_REQ_QUEUED = 0, WOST_REQ_ACTIVE = 1, WOST_REQ_DONE = 2, WOST_REQ_REJECTED = 3 };

typedef struct {
  int32_t state;              /* WOST_REQ_* */
  int32_t rounds;             /* rounds merged so far */
  int64_t n_points;
  int64_t walks_per_point;    /* walks done per point */
  double max_se;              /* largest per-point standard error so far */
  double t_submit_ms, t_admit_ms, t_done_ms;  /* steady-clock times since server creation */
  int32_t in_flight;          /* 1 while one of its rounds is enqueued or running */
} wost_request_info;

/* Creates a server (cfg may be NULL for the defaults). */
wost_status wost_server_create(const wost_server_config* cfg, wost_server* out);

/* Releases a server and all its requests.  NULL is accepted. */
wost_status wost_server_destroy(wost_server server);

/* Queues a request; points [n_points][dim] host FP32 are copied.  The scene
 * must outlive the request.  *request_id receives its id (>= 0).  A request
 * larger than the whole budget is kept and reported REJECTED.
 * Errors: INVALID_ARG (NULL scene/points, n_points < 1, eps <= 0,
 * target_se <= 0). */
wost_status wost_server_submit(wost_server server, wost_scene scene, const float* points,
                               int64_t n_points, float eps, uint64_t seed, double target_se,
                               int64_t* request_id);

/* One pass of the request loop: merges every round that has finished and
 * retires the converged requests; admits what fits the memory budget;
 * launches one round, on a free round slot (its own stream and buffers),
 * for the admitted requests that have no round in flight, up to the round's
 * walk budget -- so requests that arrive while rounds run start at a later
 * call, and their kernels take the compute units as the running rounds'
 * walks drain.  When it starts nothing it waits at most cfg.wait_us for a
 * round to end; it never blocks longer.  *n_open (optional) receives the
 * number of queued + active requests afterwards. */
wost_status wost_server_step(wost_server server, int32_t* n_open);

/* State of a request; when it is DONE and mean_out / var_out are not NULL,
 * copies its per-point mean and variance (host [n_points] FP64). */
wost_status wost_server_poll(wost_server server, int64_t request_id, wost_request_info* info,
                             double* mean_out, double* var_out);

/* Thread-local description of the last error ("" when none). */
const char* wost_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WOST_H */
