/*
 * bvc.h - C-ABI of the MI355X (gfx950) library for Boundary Value Caching
 * with walk on spheres.
 *
 * Method: Miller, Sawhney, Crane, Gkioulekas, "Boundary Value Caching for Walk
 * on Spheres", ACM TOG 42(4), 2023.  The library implements, for the PDE
 * Lap u = f with Dirichlet data u = g (Eq. 1 with sigma = 0):
 *   - cache points on the offset Dirichlet boundary (Section 3.2) drawn with a
 *     CDF table and stratified uniforms (Section 4, "Sampling");
 *   - walk on spheres from each cache point with the ball gradient estimator
 *     (Section 3.1, Eq. 7) for u-hat and du/dn-hat;
 *   - the Monte Carlo boundary-integral gather of Eqs. 3-6 at evaluation
 *     points (Algorithm 1, UpdateSolution), with its adjoint;
 *   - pointwise walk on spheres for evaluation points within l of the
 *     boundary (Section 3.2).
 *
 * Conventions shared by every entry point
 *   - Status: every function returns 0 (BVC_OK) or a negative BVC_E* code;
 *     bvc_last_error() returns a thread-local message.  Arguments are checked
 *     before any work is enqueued; device faults surface at the next
 *     synchronisation.
 *   - Streams: `stream` is a hipStream_t (NULL = default stream).  Work is
 *     enqueued and the call returns, except where a function says it
 *     synchronises (the ones that return a count to the host).
 *   - Memory: the caller owns all device memory and passes device pointers;
 *     the library allocates no device memory.  A scene keeps host memory only
 *     and is copied into a caller-provided device buffer by bvc_scene_upload.
 *   - Layout: point sets are structure-of-arrays, [dim][n] contiguous
 *     (coordinate a of point k at x[a*n + k]).
 *   - dtype: BVC_F32 or BVC_F64 selects the arithmetic of a call; arrays
 *     typed `void*` hold that type.  Arrays typed `double*` are always FP64.
 *   - Kernels: G_2D = ln r/(2 pi), G_3D = -1/(4 pi r) (Lap G = delta; the
 *     sign of G_3D printed in Appendix A.1 is inconsistent with its own
 *     derivatives and Eq. 2), dG/dn_y, dG/dx, d2G/dx dn_y as in Appendix A.1.
 *   - Random numbers: Philox-4x32-10 (Salmon et al., SC'11) with key = seed
 *     and counter = (block, id, batch, tag); walk step k draws blocks
 *     4k..4k+3; tags 1 cache walk, 2 pointwise walk, 3 cache sampling,
 *     4 source sampling.  Results depend only on (seed, batch, id), never on
 *     the launch shape or schedule.
 */
#ifndef BVC_H
#define BVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BVC_OK 0
#define BVC_EINVAL (-1)      /* invalid argument (null, size, dtype, geometry) */
#define BVC_ENOMEM (-2)      /* host allocation failed */
#define BVC_EDEVICE (-3)     /* HIP runtime error */
#define BVC_EUNSUPPORTED (-4) /* valid but not implemented combination */
#define BVC_ESTATE (-5)      /* object used in the wrong state (e.g. not uploaded) */

#define BVC_F32 0
#define BVC_F64 1
#define BVC_SPLIT_BF16 2 /* bvc_gather_multi only */

/* Field kinds.  A field is boundary data g or a source f given as a built-in
 * parametric family (the paper's callbacks, Section 4 "Setup", cannot cross
 * to the device).  coef is a DEVICE pointer to n_coef doubles.
 *   0 ZERO, 1 CONST param[0],
 *   2 HARMONIC_2D  param[1] Re((x+iy)^k) + param[2] e^x cos y, k = param[0]
 *   3 GAUSS_SUM    sum_k A_k exp(-|x-c_k|^2/(2 s^2)), s = param[0],
 *                  coef = [A_0, c_0(dim), A_1, c_1(dim), ...]
 *   4 GAUSS_POTENTIAL_2D sum_k A_k s^2/2 Ein(|x-c_k|^2/(2 s^2)) + HARMONIC_2D
 *                  with (k, alpha, beta) = param[1..3]; Lap of it = GAUSS_SUM
 *   5 SOLID_HARMONICS_3D sum coef[l^2+l+m] r^l Y_lm (orthonormal real, no
 *                  Condon-Shortley phase), l <= L = param[0]
 *   6 FOURIER_2D   sum_m coef[m] phi_m(theta), theta = atan2(y-param[1],
 *                  x-param[0]); phi_0 = 1, phi_{2j-1} = cos j theta,
 *                  phi_{2j} = sin j theta
 *   7 POINT_SOURCE 2D A ln|x-x0|, 3D A/|x-x0|, A = param[0], x0 = param[1..]
 *   8 EXP_PLANE    A exp(a . x), A = param[0], a = param[1..dim] (solves
 *                  Lap u = |a|^2 u: the screened equation's plane waves)
 *   9 WEDGE_2D     A r^p cos(p phi), r, phi = polar coordinates about
 *                  (param[2], param[3]) with phi in [0, 2 pi); A = param[0],
 *                  p = param[1] (harmonic off the cut phi = 0; with p = 2/3
 *                  it has zero normal derivative on both edges of a 270
 *                  degree corner)
 *  10 QUADRATIC    A |x - x0|^2 + B, A = param[0], B = param[1], x0 =
 *                  param[2..] (Lap = 2 dim A; with a constant source it gives
 *                  closed-form Poisson solutions)
 */
typedef struct {
  int32_t kind;
  int32_t n_coef;
  const double* coef;
  double param[8];
} bvc_field;

typedef struct bvc_scene_s* bvc_scene;

typedef struct {
  int32_t dim;
  int64_t n_verts, n_prims, n_edges;
  int64_t n_nodes;        /* internal BVH nodes */
  int32_t depth;          /* deepest internal level (root = 1) */
  double lo[3], hi[3];    /* bounding box */
  double diagonal;        /* |hi - lo| */
  double boundary_measure; /* total length (2D) or area (3D) */
  size_t device_bytes;    /* size of the buffer bvc_scene_upload needs */
  int32_t uploaded;
} bvc_scene_info;

/* ---------------------------------------------------------------------- */
/* Scene and BVH (Section 4 "Setup": polygonal boundary and an AABB BVH    */
/* for closest-point queries)                                              */
/* ---------------------------------------------------------------------- */
/* Builds the BVH on the host.  verts: host (n_verts, dim) row-major FP64;
 * prims: host (n_prims, dim) int32 vertex indices (2D segments oriented with
 * the domain on the left, i.e. counter-clockwise outer boundary; 3D
 * triangles with outward normals by the right-hand rule).  Rejects NaN or
 * infinite vertices, out-of-range indices and zero-length segments or
 * zero-area triangles.  The returned handle owns host memory only. */
int bvc_scene_create(int32_t dim, const double* verts, int64_t n_verts, const int32_t* prims,
                     int64_t n_prims, bvc_scene* out);
int bvc_scene_get_info(bvc_scene scene, bvc_scene_info* out);
/* Copies the scene (FP64 and FP32 BVH, primitives, sampling tables) into a
 * caller-owned device buffer of at least info.device_bytes bytes, 256-byte
 * aligned.  The buffer must outlive every call that uses the scene.
 * Synchronises the stream (the host staging copy is freed on return). */
int bvc_scene_upload(bvc_scene scene, void* device_buffer, size_t bytes, void* stream);
int bvc_scene_destroy(bvc_scene scene);
/* Host copy of the BVH topology, for tools that count the traversal work a
 * closest-point query needs on this exact tree.  child [n_nodes][2]: >= 0 an
 * internal node, < 0 a leaf ~((start << 3) | (count - 1)) over the leaf-ordered
 * primitives; boxes [n_nodes][4*dim] FP64 child boxes stored in the parent
 * (child 0 lo, child 0 hi, child 1 lo, child 1 hi); order [n_prims]: the
 * original primitive id of each leaf-ordered primitive.  Node 0 is the root.
 * Host pointers, caller-owned, sized from bvc_scene_info; any may be NULL. */
int bvc_scene_export_bvh(bvc_scene scene, int32_t* child, double* boxes, int32_t* order);
/* 3D only: the second bound of each child, slabs [n_nodes][12] FP64 (host,
 * caller-owned): for child c, (n_x, n_y, n_z, smin, smax) at 5c, with n the
 * unit area-weighted mean normal of the child's triangles and [smin, smax]
 * the range of n.y over their vertices, widened by the rounding of n.p
 * (entries 10 and 11 are 0).  Closest-point traversals prune a child when
 * the larger of its box distance and its slab distance exceeds the best
 * distance so far.  BVC_EUNSUPPORTED for 2D scenes. */
int bvc_scene_export_slabs(bvc_scene scene, double* slabs);

/* Total measure of the offset-boundary candidate set at offset l: segment
 * lengths (times `sides`) plus vertex circles (2D); face areas plus edge
 * cylinders plus vertex spheres (3D).  Host-only. */
int bvc_cache_measure(bvc_scene scene, double l, int32_t sides, double* measure);

/* ---------------------------------------------------------------------- */
/* Cache points on the offset Dirichlet boundary (Section 3.2; Section 4)   */
/* ---------------------------------------------------------------------- */
/* Draws n candidates: stratified uniforms u_k = (k + U_k)/n through the CDF
 * of the candidate measure (inward segment/face offsets at distance l,
 * vertex circles or spheres, edge cylinders; sides = 2 adds outward
 * segment offsets in 2D for self-intersecting polygons).  A candidate is
 * accepted when no boundary point is closer than l (up to 1e-9 relative)
 * and it lies inside (2D: nonzero winding number; 3D: pseudonormal sign).
 * Outputs (FP64 device, [dim][n] or [n]): x, unit outward normal of the
 * region {d > l} (towards the closest boundary point), weight w = measure/n,
 * xbar (the closest boundary point, where the control variate c = g(xbar) of
 * the point's walks reads the data), distance R0, accept flag (int32 0/1). */
int bvc_sample_cache(bvc_scene scene, int64_t n, double l, int32_t sides, uint64_t seed,
                     uint32_t batch, double* x, double* nrm, double* w, double* xbar, double* R0,
                     int32_t* accept, void* stream);

/* Cache points on the closed boundary of a region of interest R inside the
 * domain (Section 3.2, "Boundary Specification"; Algorithm 1 with
 * p^dR = 1/|dR|): candidate k sits at arc length (or area) (k + U_k)/n * |dR|
 * along the primitives of `roi` (U_k the first uniform of Philox block 0,
 * id k, tag 6; the second places it inside a triangle), with the primitive's
 * unit outward normal (CCW segments, outward-wound triangles) and weight
 * |dR|/n.  R0 and xbar: distance and closest point on the domain boundary
 * `dom` (where the walks run); accept = 1 when the point lies strictly inside
 * the domain.  Outputs as bvc_sample_cache.  Evaluation points inside R
 * (bvc_classify on `roi` with l = 0) are then gathered from this cache; the
 * estimate vanishes outside R.  The first call for `roi` uploads its sampling
 * table and synchronises. */
int bvc_sample_roi(bvc_scene dom, bvc_scene roi, int64_t n, uint64_t seed, uint32_t batch, double* x,
                   double* nrm, double* w, double* xbar, double* R0, int32_t* accept, void* stream);

/* Cache points for a 2D boundary with a Neumann part (Section 3.2,
 * "Boundary Specification"): samples on the offset Dirichlet boundary (at
 * distance l > eps from the Dirichlet part `dir`, inside the domain whose
 * whole boundary is `full`) and on the Neumann part `neu` where it is farther
 * than l from `dir`; together they bound the region where the cache is
 * gathered.  One stratified draw (Philox block 0, id k, tag 7): candidate k
 * sits at (k + U_k)/n of the concatenated measure of the offset candidates
 * of `dir` (as bvc_sample_cache with sides 1) and the segments of `neu`.
 * Outputs (FP64 device, [2][n] or [n]): x; nrm = towards the closest
 * Dirichlet point on offset points, the segment's outward normal on Neumann
 * points; w = total candidate measure / n; xbar = closest Dirichlet point;
 * R0 = distance to `full` (the first ball of a cache walk); kind (int32 [n]:
 * 0 rejected, 1 accepted offset point (distance l within 1e-9 relative and
 * inside `full`), 2 accepted Neumann point (farther than l)).
 * junction_drop in [0, 1): offset points closer than junction_drop * l to the
 * Neumann part are rejected as well.  0 is the plain sampler (the closed
 * curve of Section 3.2); a positive value removes the pieces of the offset
 * curve next to each Dirichlet / Neumann junction, whose first balls are as
 * small as their distance to the Neumann part (the Eq. 7 estimate's
 * variance grows like (l / R0)^2 there), at the cost of a bias equal to
 * those pieces' share of Green's representation.  The three
 * scenes are CCW segment sets over one boundary; the first call for `dir` at
 * this l and for `neu` uploads their sampling tables and synchronises.
 * Errors: BVC_EUNSUPPORTED in 3D, BVC_EINVAL for an empty part, l <= 0,
 * junction_drop outside [0, 1) or a null output. */
int bvc_sample_mixed(bvc_scene full, bvc_scene dir, bvc_scene neu, int64_t n, double l, double junction_drop,
                     uint64_t seed, uint32_t batch, double* x, double* nrm, double* w, double* xbar, double* R0,
                     int32_t* kind, void* stream);

/* Source samples (Eq. 4): m^dim jittered cells over the box [lo, hi] (host
 * arrays of dim doubles); s_j = |box|/m^dim * f(y_j) * 1[y_j inside and
 * d(y_j) > l].  y: [dim][m^dim] FP64 device, s: [m^dim] FP64 device. */
int bvc_sample_sources(bvc_scene scene, const bvc_field* f, int64_t m, const double* lo,
                       const double* hi, double l, uint64_t seed, uint32_t batch, double* y,
                       double* s, void* stream);

/* Classifies points x ([dim][n] FP64 device): cls = 0 outside, 1 interior
 * (d > l, evaluated by the gather), 2 band (d <= l, evaluated by pointwise
 * walks, Section 3.2).  dist (optional) receives d(x). */
int bvc_classify(bvc_scene scene, int64_t n, const double* x, double l, int32_t* cls,
                 double* dist, void* stream);

/* Classifies 2D points x ([2][n] FP64 device) of a domain with a Neumann
 * part (Section 3.2): cls = 0 outside `full` (nonzero winding number inside),
 * 1 inside and farther than l from the Dirichlet part `dir` (gathered from
 * the mixed cache), 2 inside within l of `dir` (walks on stars).  dist
 * (optional) receives the distance to `dir`.  BVC_EUNSUPPORTED in 3D. */
int bvc_classify_mixed(bvc_scene full, bvc_scene dir, int64_t n, const double* x, double l, int32_t* cls,
                       double* dist, void* stream);

/* Deterministic stream compaction: idx[0..count) = ascending k with
 * flags[k] == want.  scratch: caller-owned device int32 array of at least
 * bvc_compact_scratch_ints(n) entries, 8-byte aligned.  count is written to
 * *count_host; synchronises the stream. */
int64_t bvc_compact_scratch_ints(int64_t n);
int bvc_compact(int64_t n, const int32_t* flags, int32_t want, int32_t* idx, int32_t* scratch,
                int64_t* count_host, void* stream);
/* out[r*ld_out + q] = (dtype_out) in[r*ld_in + idx[q]] for r < rows, q < n_idx
 * (idx NULL = identity).  Used to pack compacted SoA arrays and convert
 * FP64 -> FP32. */
int bvc_take(int32_t dtype_in, int32_t dtype_out, int64_t n_idx, const int32_t* idx,
             int32_t rows, int64_t ld_in, const void* in, int64_t ld_out, void* out, void* stream);
/* bvc_compact without the readback: the count is written to the device
 * int64 *count (zero when n == 0) and nothing synchronises, so that a step
 * can be enqueued (and captured in a HIP graph) before its cache size is
 * known; idx holds the ascending k with flags[k] == want in [0, *count) and
 * is not written beyond. */
int bvc_compact_count(int64_t n, const int32_t* flags, int32_t want, int32_t* idx, int32_t* scratch,
                      int64_t* count, void* stream);
/* bvc_take for the first min(n_cap, *count) entries, count a device int64
 * (entries beyond it are left untouched, and idx is read only below it). */
int bvc_take_count(int32_t dtype_in, int32_t dtype_out, int64_t n_cap, const int64_t* count, const int32_t* idx,
                   int32_t rows, int64_t ld_in, const void* in, int64_t ld_out, void* out, void* stream);
/* out[idx[q]] = in[q] (scatter back; dtype of in and out equal). */
int bvc_scatter(int32_t dtype, int64_t n_idx, const int32_t* idx, int32_t rows, int64_t ld_in,
                const void* in, int64_t ld_out, void* out, void* stream);

/* ---------------------------------------------------------------------- */
/* Walks (Section 3.1, Eq. 7; Algorithm 1 "WalkOnStars" for Dirichlet data) */
/* ---------------------------------------------------------------------- */
typedef struct {
  double eps;              /* epsilon shell: stop when d < eps */
  int32_t max_steps;       /* cap on closest-point queries per walk */
  int32_t n_walks;         /* walks per start point */
  uint64_t seed;
  uint32_t batch;
  int32_t control_variate; /* subtract g(xbar) in the gradient sample */
  int32_t dtype;           /* BVC_F32 or BVC_F64 walk arithmetic */
  int32_t blocks;          /* persistent grid size (0 = automatic) */
  bvc_field g;             /* Dirichlet data */
  bvc_field f;             /* source term (kind 0 for Laplace) */
  void* ev_begin;          /* optional hipEvent_t recorded on the stream right before */
  void* ev_end;            /* and right after the walk kernel (NULL = none), to time
                              the traversal alone; ignored by the batch calls */
  double sigma;            /* screening coefficient of Lap u - sigma u = f (Eq. 1),
                              >= 0.  sigma > 0 (Appendix A.2): every ball of
                              radius R multiplies the estimate by its mean-value
                              factor, 1/I0(sR) in 2D and sR/sinh(sR) in 3D
                              (s = sqrt(sigma)), and the ball gradient weight
                              dim/R0 becomes s/I1(sR0) in 2D and s/i1(sR0) in
                              3D, i1(x) = (x cosh x - sinh x)/x^2.  With a
                              source f each ball's source sample (drawn from
                              the Laplace ball density) is weighted by the
                              ratio of the screened to the Laplace ball
                              Green's function at its radius, and by the
                              factors of the balls before it; the first
                              ball's gradient source sample by the ratio of
                              the centre gradients; these ratios are
                              evaluated in FP64.  Such walks evaluate g at
                              their exit themselves.  Not taken by the batch
                              and clamping calls. */
  double open_center[3];   /* open (unbounded) 3D domains (Appendix B): the centre */
  double open_radius;      /* and radius of a sphere that encloses every vertex of
                              the scene; 0 = a bounded domain.  The domain is the
                              side of the mesh its pseudonormals call inside: for
                              the exterior of a closed solid, give its triangles
                              reversed.  A walk that jumps (jump index k) to
                              r = |x - c| > radius draws the Philox uniforms
                              (u, v) of counter (k, id, batch, tag | 8) and w of
                              (k, id, batch, tag | 16), tag = 1 for cache walks and
                              2 for pointwise walks; it escapes to infinity, where
                              u = 0, when u >= radius / r (the probability that
                              Brownian motion from x never reaches the sphere is
                              1 - radius / r), else it moves to the first point
                              of the sphere it reaches: the sphere's exterior
                              harmonic measure from x, sampled in closed form
                              through the Kelvin transform (polar angle from v,
                              azimuth 2 pi w).  An escaped walk's exit record is
                              NaN and its boundary value 0.  Laplace only (sigma
                              = 0, f = ZERO); taken by the cache, pointwise and
                              tuning walk calls, refused (BVC_EUNSUPPORTED) by
                              the batch, clamping and walk-on-stars calls;
                              BVC_EINVAL when the sphere leaves out a vertex. */
  int32_t side_read;       /* 0: a walk reads g at its closest boundary point and
                              the control variate c at xbar (Section 3.1).  1:
                              the side rule for data that differ on the two
                              sides of a boundary curve (double-sided
                              conditions, Appendix B): an exit reads g at the
                              closest point moved 1e-3 eps towards the walk, and
                              c is read at xbar + 1e-3 (x - xbar), x the start
                              point, so both read the data on the walk's own
                              side.  Refused (BVC_EUNSUPPORTED) by the batch
                              calls. */
  bvc_field h;             /* Neumann data du/dn = h on the Neumann part (Eq. 1);
                              read only by bvc_wost_walks (kind 0: h = 0). */
  const int64_t* n_dev;    /* bvc_cache_walks and bvc_tune_walks only (NULL
                              elsewhere, else BVC_EUNSUPPORTED): device int64 count of cache
                              points, read by the kernels; the call walks the
                              first min(n_cache, *n_dev) points and n_cache is
                              the capacity the arrays are laid out for (record
                              strides n_cache*W).  Lets a step run without
                              reading its cache size back (see
                              bvc_compact_count).  NULL: n_cache points. */
  const int32_t* order;    /* bvc_cache_walks, bvc_pointwise_wos(_noalloc),
                              bvc_tune_walks and bvc_tune_pointwise only (NULL
                              elsewhere, else BVC_EUNSUPPORTED): device int32
                              launch order of the start points, a permutation
                              of [0, count) (count: the n_dev value when given,
                              else the point count), e.g. from
                              bvc_spatial_order.  The walks of point order[0]
                              are started first, then those of order[1], and so
                              on, so that the walks in flight together query
                              nearby parts of the tree and share the caches.
                              Every walk keeps its id, random stream and record
                              slot: the results do not depend on the order.
                              Entries outside [0, count) are skipped (their
                              walks do not run).  NULL: point order. */
} bvc_walk_params;

/* Launch order by position, for the walk params' `order` (a scheduling
 * choice of this library, not part of the method: results do not depend on
 * it).  order[0..count) lists the points 0..count-1 (count = min(n, *n_dev)
 * with a device count, else n) by the Morton index of their cell in a grid of
 * 32^3 (3D) or 256^2 (2D) cells over the scene's bounding box (points outside
 * it, or not finite, fall in the nearest edge cell); the order inside a cell is
 * unspecified (device atomics).  x: device [dim][ld] (ld >= n) of dtype
 * BVC_F32 or BVC_F64; order: device int32 [n] (entries from count on are left
 * unwritten); work: device workspace of at least
 * bvc_spatial_order_workspace_bytes() bytes, 256-byte aligned, overwritten.
 * Allocates nothing; no host synchronisation.  BVC_EINVAL for another dtype,
 * n < 0, n > INT32_MAX, ld < n, a null argument (n > 0) or a short or
 * misaligned workspace; BVC_ESTATE for a scene not uploaded. */
size_t bvc_spatial_order_workspace_bytes(void);
int bvc_spatial_order(bvc_scene scene, int32_t dtype, int64_t n, const void* x, int64_t ld, const int64_t* n_dev,
                      int32_t* order, void* work, size_t work_bytes, void* stream);

/* Walk j of cache point i has id i*W + j (n_cache*W < 2^32).  Each walk takes
 * a first ball B(x_i, R0_i) with no termination test (uniform direction nu;
 * source sample with density |G^B|), then walk on spheres until d < eps (or
 * max_steps queries, counted as capped), reading g at the closest point.
 * U[id]  = g(exit) + in-walk source sums - R0^2/(2 dim) f(y_u)
 * D[id]  = n_i . [(dim/R0) nu (W - c_i) - m(t) R0 yhat f(y_g)]
 * with the first ball's gradient source sample y_g = x_i + t R0 yhat: 2D t
 * from the density (3/2)(1 - t^2), m = 2/3 (the second uniform of Philox
 * block 2 and the first of block 3); 3D t uniform, m = 1 - t^3, yhat uniform
 * on the sphere (blocks 0 and 1 under tag | 128).
 * Inputs x, nrm, xbar: [dim][n_cache] FP64; R0: [n_cache] FP64 (from
 * bvc_sample_cache after compaction).  U, D: [n_cache*W] of params->dtype.
 * Exit records (required; they are also the checkpoint the cache adjoint
 * reads instead of re-walking): rec_exit [dim][n_cache*W] of dtype (the
 * closest boundary point where the walk stopped), rec_w1 [n_cache*W]
 * ((dim/R0)(nu . n_i)); rec_steps int32 [n_cache*W] is optional.  The source
 * term f must be ZERO, CONST, GAUSS_SUM or EXP_PLANE; g is evaluated in FP64
 * at the exit points (FP32 for the closed-form kinds when the walks are FP32).  counters: device uint64[4], zeroed by the call: [0] work
 * queue, [1] total closest-point queries, [2] capped walks, [3] walks. */
int bvc_cache_walks(bvc_scene scene, const bvc_walk_params* params, int64_t n_cache,
                    const double* x, const double* nrm, const double* R0, const double* xbar,
                    void* U, void* D, void* rec_exit, void* rec_w1, int32_t* rec_steps,
                    uint64_t* counters, void* stream);

/* Means over the W walks of each cache point, reduced in FP64 in a fixed
 * order (Eq. 3 needs u-hat and du/dn-hat): uhat, dudn [n] FP64; a = uhat*w,
 * b = dudn*w in `dtype_out` (the gather's cache values). */
int bvc_reduce_walks(int64_t n_cache, int32_t W, int32_t dtype_in, const void* U, const void* D,
                     const double* w, double* uhat, double* dudn, int32_t dtype_out, void* a,
                     void* b, void* stream);
/* The same means for the first min(n_cap, *count) points, count a device
 * int64 (bvc_compact_count); point i's walks are U, D [i*W, i*W + W).
 * Entries at and beyond the count are left untouched.  No host
 * synchronisation. */
int bvc_reduce_walks_count(int64_t n_cap, const int64_t* count, int32_t W, int32_t dtype_in, const void* U,
                           const void* D, const double* w, double* uhat, double* dudn, int32_t dtype_out,
                           void* a, void* b, void* stream);

/* Pointwise walk on spheres at n points x ([dim][n] of params->dtype): the
 * estimator the paper uses within l of the boundary (Section 3.2) and the
 * baseline the cache is compared against.  Walk j of point k has id k*W + j
 * (tag 2); a point already inside the epsilon shell returns g(xbar).
 * U_walk [n*W] and G_walk [dim][n*W] (optional) are per-walk scratch of
 * dtype; u [n] and grad [dim][n] (optional) receive the means.  work: a
 * caller-owned, 256-byte aligned device buffer of at least
 * bvc_pointwise_workspace_bytes(dim, n, W, dtype, grad != NULL) bytes
 * (closest points and exit records). */
size_t bvc_pointwise_workspace_bytes(int32_t dim, int64_t n, int32_t W, int32_t dtype,
                                     int32_t with_grad);
int bvc_pointwise_wos(bvc_scene scene, const bvc_walk_params* params, int64_t n, const void* x,
                      void* U_walk, void* G_walk, void* work, size_t work_bytes, void* u, void* grad,
                      uint64_t* counters, void* stream);

/* Pointwise walk on spheres that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same walks, same Philox streams and the
 * same results, bit for bit, as bvc_pointwise_wos; the per-walk values U_walk
 * and G_walk and the workspace (start radii, closest points, exit records)
 * live in a library-owned device array of BVC_POINTWISE_STATIC_BYTES (32 MiB)
 * on each GPU, held from module load until the process ends, instead of in
 * caller buffers.  The caller still owns x [dim][n], u [n], grad [dim][n]
 * (optional) and counters (device uint64[4]), as for bvc_pointwise_wos.
 * A call needs bvc_pointwise_static_bytes(dim, n, W, dtype, grad != NULL) <=
 * BVC_POINTWISE_STATIC_BYTES: about n W (1 + dim) words of the walk dtype
 * without grad and n W (1 + 3 dim) with it; a larger call returns BVC_EINVAL
 * (nothing is launched) and the caller splits its points over several calls.
 * Every call on one GPU uses that GPU's one array, which keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * GPU (two streams, two host threads) race and must be serialised by the
 * caller.  The first call on each device resolves the array's device address
 * (hipGetSymbolAddress, with that device current); no call makes a HIP
 * allocation or calls a routine that allocates. */
#define BVC_POINTWISE_STATIC_BYTES ((size_t)32 << 20)
size_t bvc_pointwise_static_bytes(int32_t dim, int64_t n, int32_t W, int32_t dtype, int32_t with_grad);
int bvc_pointwise_wos_noalloc(bvc_scene scene, const bvc_walk_params* params, int64_t n, const void* x,
                              void* u, void* grad, uint64_t* counters, void* stream);

/* ---------------------------------------------------------------------- */
/* Gather (Eqs. 3-6; Algorithm 1 splat loops)                              */
/* ---------------------------------------------------------------------- */
typedef struct {
  int64_t n;
  int32_t dtype;
  const void* x;   /* [dim][n] cache points z_i */
  const void* nrm; /* [dim][n] unit outward normals */
  const void* a;   /* [n] u-hat_i / p(z_i) / N */
  const void* b;   /* [n] du/dn-hat_i / p(z_i) / N */
  const int64_t* n_dev; /* NULL, or a device int64 count: the gather sums the
                           first min(n, *n_dev) entries, n being the capacity
                           (leading dimension) of x and nrm.  Taken by
                           bvc_gather_u, bvc_gather_grad and bvc_tune_gather;
                           the adjoint refuses it (BVC_EUNSUPPORTED). */
} bvc_cache_view;

typedef struct {
  int64_t n;
  int32_t dtype;
  const void* y; /* [dim][n] source points */
  const void* s; /* [n] f(y_j) / p(y_j) / M */
} bvc_source_view;

typedef struct {
  int32_t accumulate; /* add into u/grad instead of overwriting */
  double near_tau;    /* FP32 only: pairs with |x - z| < tau use FP64 (0 = off) */
  const double* near_x;  /* FP64 copies for the near field: eval [dim][n_eval] */
  const double* near_cx; /* cache points [dim][n] */
  const double* near_cn; /* cache normals [dim][n] */
  const double* near_a;  /* cache a [n] */
  const double* near_b;  /* cache b [n] */
  double clamp_c;        /* > 0: dG/dn clamped to [-clamp_c, clamp_c] in the
                            potential's boundary term (Eq. 9 in the first
                            integral of Eq. 8); the gradient is not clamped.
                            0 = off */
  double sigma;          /* > 0: screened kernels G = -K0(sr)/(2 pi) in 2D and
                            -exp(-sr)/(4 pi r) in 3D with their derivatives
                            (Appendix A.2; s = sqrt(sigma)); without near field
                            or clamp.  FP32 evaluates K0, K1 to about 5e-7
                            relative, FP64 to about 1e-14.  0 = off */
  int64_t near_lead;     /* near field: > 0 when only the first near_lead
                            evaluation points can have a pair closer than tau
                            (the caller orders them first); the blocks past
                            them skip the near test.  0 = every point;
                            BVC_EINVAL outside [0, n_eval] */
} bvc_gather_params;

/* u_k = sum_i [dG/dn(x_k,z_i) a_i - G(x_k,z_i) b_i] + sum_j G(x_k,y_j) s_j
 * (Eqs. 3-4).  eval_x [dim][n_eval]; u [n_eval]; dtype of cache, sources,
 * eval points and u must agree.  sources may be NULL. */
int bvc_gather_u(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources,
                 int64_t n_eval, const void* eval_x, void* u, const bvc_gather_params* params,
                 void* stream);
/* grad_k = sum_i [d2G/dxdn a_i - dG/dx b_i] + sum_j dG/dx s_j (Eqs. 5-6) into
 * grad [dim][n_eval]; u (optional, may be NULL) receives Eqs. 3-4 from the
 * same pass. */
int bvc_gather_grad(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources,
                    int64_t n_eval, const void* eval_x, void* u, void* grad,
                    const bvc_gather_params* params, void* stream);

/* ---------------------------------------------------------------------- */
/* Walk on stars: mixed Dirichlet / Neumann boundaries (Section 3.1)       */
/* ---------------------------------------------------------------------- */
/* The estimator the cache uses when part of the boundary is Neumann (walk on
 * stars; 2D and 3D, Neumann data h, no source, no screening).  `dir` and
 * `neu` hold the Dirichlet and the Neumann elements of one boundary (2D:
 * counter-clockwise segments; 3D: triangles with outward normals by the
 * right-hand rule; two scenes of one dimension).  Walk j of start point i has
 * id i*W + j (n*W < 2^32).  Each step: star radius R = max(eps, min(d_D,
 * d_S)), d_D the distance to the Dirichlet part and d_S to the closest
 * silhouette of the Neumann part seen from the walk.  2D silhouettes: a
 * corner vertex whose Neumann neighbours are not strictly on opposite sides
 * of the line of sight (within 1e-9 relative in FP64 and 1e-5 in FP32: both
 * on one side, one on it, or both on it at the fold of a thin Neumann curve),
 * and the ends of Neumann runs; a vertex where the boundary continues
 * straight, within 1e-12 relative, is no corner.  3D silhouettes: an edge
 * where the Neumann part ends, and an edge between two triangles that are not
 * coplanar unless the walk lies strictly in front of both planes or strictly
 * behind both (same tolerances).  With Neumann data h (kind != 0) the step
 * adds one sample of its star's Neumann term: every Neumann element within
 * R (1 + 1e-9) (FP32: R (1 + 1e-5)) that the walk does not lie strictly
 * behind is a candidate, of total measure |C| (elements beyond R add 0, so
 * the superset keeps the estimate unbiased and holds the elements that touch
 * the ball at a silhouette in both precisions); one is drawn with probability measure / |C| by an exponential
 * race (key -ln(1 - U) / measure with U the FP64 uniform of Philox block =
 * the element's original id, tag | 32 | (k << 8), k the step; smallest key),
 * z uniform on it (block 4k + 1, tag | 64: 2D a + U1 (b - a), 3D barycentric
 * (1 - s, s (1 - U2), s U2) with s = sqrt(U1)), and the sample is
 * |C| G^B(x, z) h(z), doubled when the walk stands on the Neumann part, when
 * |z - x| < R (else 0); G^B = ln(R/r)/(2 pi) in 2D, (1/r - 1/R)/(4 pi) in 3D.
 * A direction uniform on the circle or sphere (Philox block 4k as walk on
 * spheres), turned into the inward half space on the Neumann part; the walk
 * moves to the nearest crossing within R of a Neumann element it leaves the
 * domain through, else to the sphere; it stops when d_D < eps (or after
 * max_steps, counted as capped) with U = g(closest Dirichlet point) plus its
 * Neumann terms, g and h evaluated in FP64 (FP32 walks: in FP32).
 * mode 0: from offset Dirichlet cache points x with normals nrm, R0 = the
 *   distance to the whole boundary and xbar = the closest Dirichlet point:
 *   a first ball of radius R0 (no test at x), tag 1, and
 *   D = n . (dim/R0) nu (U - c) (Eq. 7, c = g(xbar) with the control variate);
 * mode 1: from interior points, tag 2 (D = 0);
 * mode 3: from points on the Neumann part with outward normals nrm, tag 2.
 * x, nrm, xbar: [dim][n] FP64; R0 [n]; U, D (optional): [n*W] of dtype;
 * steps (optional) int32 [n*W].  workspace: caller-owned, at least
 * bvc_wost_workspace_bytes(neu) bytes (2D: the Neumann run links, corner
 * flags and per-node normal cones that let the silhouette query skip BVH
 * nodes without corners facing the walk; 3D: the triangle across each edge
 * and the flat-edge bits; built on the host at the first call for this
 * Neumann scene, kept with it in pinned host memory, and uploaded by every
 * call on its stream without synchronising).  Calls that overlap on several
 * streams need a workspace each.  counters: uint64[4] as the walks. */
size_t bvc_wost_workspace_bytes(bvc_scene neu);
int bvc_wost_walks(bvc_scene dir, bvc_scene neu, const bvc_walk_params* params, int32_t mode, int64_t n,
                   const double* x, const double* nrm, const double* R0, const double* xbar, void* U, void* D,
                   int32_t* steps, void* workspace, size_t workspace_bytes, uint64_t* counters, void* stream);

/* ---------------------------------------------------------------------- */
/* Bias correction of the clamped gather (Section 3.3, Eq. 8)              */
/* ---------------------------------------------------------------------- */
/* Clamping dG/dn at c (bvc_gather_params.clamp_c) removes the near-boundary
 * artefacts of the gather and adds a bias equal to the second integral of
 * Eq. 8.  This call estimates that integral at points inside the region the
 * cache bounds and adds it to u.  dG/dn(x, z) dz is the signed solid angle
 * dR subtends at x, so a uniform ray direction from x and the ray's
 * crossings z of the offset boundary dR = {z inside : d(z) = l} give
 *   sum_z sign(dG/dn) max(0, 1 - c/|dG/dn(x, z)|) u(z),
 * averaged over n_rays rays per point, with u(z) from one pointwise walk per
 * contributing crossing (|dG/dn| > c; only crossings within
 * bvc_clamp_radius(dim, c) can contribute).  A crossing belongs to dR by the
 * cache sampler's acceptance rule (no boundary point closer than l up to
 * 1e-9 relative, and inside).  Random numbers: ray j of point k takes the
 * Philox pair of block j, id k, batch, tag 5 (2D angle 2 pi ua; 3D
 * z = 1 - 2 ua, azimuth 2 pi ub); the contributing crossings of a ray are
 * ranked h = 0, 1, ... nearest first, at most max_hits are kept, and crossing
 * h walks with id (k n_rays + j) max_hits + h, tag 2, as bvc_pointwise_wos
 * walks (a crossing already closer than eps to the boundary returns g at its
 * closest boundary point).
 * Use a walk seed other than the band walks' so the two sets are independent. */
typedef struct {
  double l;          /* offset distance of the cache boundary */
  int32_t sides;     /* candidate sides, as bvc_sample_cache */
  double c;          /* clamp bound, > 0 */
  int32_t n_rays;    /* rays per point, >= 1 */
  int32_t max_hits;  /* contributing crossings kept per ray, 1..64 */
} bvc_clamp_params;

/* Distance beyond which |dG/dn| <= c: 1/(2 pi c) in 2D, (4 pi c)^(-1/2) in 3D. */
double bvc_clamp_radius(int32_t dim, double c);

/* 2D winding numbers of n points ([2][n] FP64 device) into wind [n] int32:
 * the input bvc_clamp_correction needs to tell inside from outside along a
 * ray (3D scenes use the pseudonormal test and need none). */
int bvc_point_winding(bvc_scene scene, int64_t n, const double* x, int32_t* wind, void* stream);

size_t bvc_clamp_workspace_bytes(int32_t dim, int32_t dtype, int64_t n, int32_t n_rays, int32_t max_hits);

/* x: [dim][n] FP64 device points, each inside the region {d > l};
 * wind: [n] int32 winding numbers (2D; from bvc_point_winding), ignored in
 * 3D; out_index: [n] int64 or NULL: the correction of point k is added to
 * u[out_index[k]] (u[k] when NULL); u: params->dtype (walk precision) device
 * array.  The crossings and weights are computed in FP64, the walks in
 * params->dtype (params->n_walks is ignored: one walk per crossing).
 * workspace: caller-owned, 256-byte aligned, >= bvc_clamp_workspace_bytes
 * bytes.  counters: device uint64[6], zeroed by the call: [0] contributing
 * crossings, [1] rays with more than max_hits of them or more candidates than
 * the ray kernel holds (their extra crossings are dropped), [2] walk queue,
 * [3] closest-point queries of the walks, [4] capped walks, [5] walks.
 * No host synchronisation: the number of contributing crossings stays on the
 * device (in the workspace) and bounds the walk queue there. */
int bvc_clamp_correction(bvc_scene scene, const bvc_walk_params* params, const bvc_clamp_params* cp,
                         int64_t n, const double* x, const int32_t* wind, const int64_t* out_index,
                         void* u, void* workspace, size_t workspace_bytes, uint64_t* counters,
                         void* stream);

/* ---------------------------------------------------------------------- */
/* Autotuning of launch shapes (no passage of the paper: a performance aid) */
/* ---------------------------------------------------------------------- */
/* Times the gather of this problem with 1, 2 and 4 evaluation points per
 * thread (one warm-up and `reps` timed launches each, HIP events on the
 * stream) and keeps the fastest for every later gather of the same class:
 * dim, dtype, gradient or not, near field or not, floor(log2) of n_eval and
 * of the cache size.  The choice is process-wide (guarded by a mutex) and
 * does not change any result: each point's sum runs in the same order for
 * every shape.  Arguments as bvc_gather_grad (grad may be NULL for u only);
 * params->accumulate must be 0.  On return u/grad hold the gather's result
 * and *ppt the choice.  Synchronises the stream. */
int bvc_tune_gather(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources,
                    int64_t n_eval, const void* eval_x, void* u, void* grad,
                    const bvc_gather_params* params, int32_t reps, int32_t* ppt, void* stream);

/* Times the cache walks of this problem over persistent grids of 4, 8 and 16
 * blocks per compute unit and traversal-loop exit thresholds of 0, 8, 16, 32
 * and 48 open lanes, and in 3D with and without the slab bounds in the
 * traversal (default shape: 8 blocks per CU, 32 open lanes in 3D and 0 in 2D,
 * slab bounds on for bounded 3D domains and off for open ones; the other slab
 * setting is tried at the default grid and threshold first, then grids and
 * thresholds with the setting kept; a shape replaces the default only when at
 * least 3% faster) and keeps the choice for every later cache-walk launch of
 * the same class (dim, walk dtype, source term or not, open domain or not,
 * screened or not) whose params->blocks is 0; pointwise walks keep their
 * default shape.  Every shape gives the same walk results (a walk's random
 * numbers depend on its id only, and the slab bounds only prune subtrees that
 * cannot hold a closer primitive).  Arguments as bvc_cache_walks; the outputs
 * hold the walks' results on return; *slabs (optional) receives 1 when the
 * slab bounds are kept.  Synchronises the stream. */
int bvc_tune_walks(bvc_scene scene, const bvc_walk_params* params, int64_t n_cache, const double* x,
                   const double* nrm, const double* R0, const double* xbar, void* U, void* D,
                   void* rec_exit, void* rec_w1, uint64_t* counters, int32_t reps,
                   int32_t* blocks_per_cu, int32_t* open_lanes, int32_t* slabs, void* stream);
/* The same search for the pointwise walks of bvc_pointwise_wos (arguments as
 * there, plus reps and the outputs of bvc_tune_walks): the choice is kept for
 * every later pointwise-walk launch of the class (band points, whose walks
 * start within l of the boundary and take a few steps, favour other shapes
 * than the cache walks).  u and grad hold the means on return.  Synchronises
 * the stream. */
int bvc_tune_pointwise(bvc_scene scene, const bvc_walk_params* params, int64_t n, const void* x, void* U_walk,
                       void* G_walk, void* workspace, size_t workspace_bytes, void* u, void* grad,
                       uint64_t* counters, int32_t reps, int32_t* blocks_per_cu, int32_t* open_lanes,
                       int32_t* slabs, void* stream);

/* Adjoint of the gather for dL/du = r [n_eval]:
 * dL/da_i = sum_k r_k dG/dn(x_k,z_i), dL/db_i = -sum_k r_k G(x_k,z_i),
 * dL/ds_j = sum_k r_k G(x_k,y_j), dL/dx_k = r_k grad u(x_k) (Eq. 5-6).
 * Any output may be NULL. */
int bvc_gather_backward(int32_t dim, const bvc_cache_view* cache,
                        const bvc_source_view* sources, int64_t n_eval, const void* eval_x,
                        const void* dL_du, void* dL_da, void* dL_db, void* dL_ds, void* dL_dx,
                        void* stream);

/* ---------------------------------------------------------------------- */
/* Linearity in the boundary data: basis expansions from exit records       */
/* ---------------------------------------------------------------------- */
/* For an expandable field family (FOURIER_2D, SOLID_HARMONICS_3D; the
 * coefficients of `basis` are ignored, n_coef sets the basis size nb):
 * E[i*nb+m] = (1/W) sum_j phi_m(exit_ij),
 * F[i*nb+m] = (1/W) sum_j w1_ij (phi_m(exit_ij) - cv phi_m(xbar_i)),
 * so that u-hat = E theta and du/dn-hat = F theta for g = sum theta_m phi_m.
 * rec_exit, rec_w1 as written by bvc_cache_walks (dtype); E, F FP64.
 * A NaN exit record (a walk that escaped an open domain) has phi_m = 0 for
 * every m: u = 0 at infinity whatever the data. */
int bvc_basis_means(const bvc_field* basis, int32_t dim, int64_t n_cache, int32_t W,
                    int32_t dtype, const void* rec_exit, const void* rec_w1, const double* xbar,
                    int32_t cv, double* E, double* F, void* stream);
/* Cache adjoint: dL/dtheta_m = sum_i w_i (E_im dL/da_i + F_im dL/db_i)
 * (dL_da, dL_db FP64 [n]; dL_dtheta FP64 [nb]), summed in a fixed order over
 * chunks of 1024 cache points.  scratch: caller-owned FP64 device array of
 * bvc_cache_backward_scratch_doubles(n_cache, nb) entries. */
int64_t bvc_cache_backward_scratch_doubles(int64_t n_cache, int32_t nb);
int bvc_cache_backward(int64_t n_cache, int32_t nb, const double* E, const double* F,
                       const double* w, const double* dL_da, const double* dL_db,
                       double* scratch, double* dL_dtheta, void* stream);
/* Many fields sharing one set of walks: A[i*F+f] = w_i sum_m E_im coef[f*nb+m],
 * B likewise with F (coef FP64 device [n_fields][nb]); A, B of dtype_out. */
int bvc_eval_fields(int64_t n_cache, int32_t nb, int32_t n_fields, const double* E,
                    const double* F, const double* w, const double* coef, int32_t dtype_out,
                    void* A, void* B, void* stream);
/* Multi-RHS gather: U[k*F+f] = sum_i [dG/dn(x_k,z_i) A[i*F+f] - G(x_k,z_i) B[i*F+f]]
 * with the kernel matrix generated on the fly.  FP32 inputs; precision
 * BVC_F32 (FP32 FMA) or BVC_SPLIT_BF16 (three bf16 MFMA products with FP32
 * accumulation).  n_fields is 32 or 64.  cx, cn: [dim][n_cache]; A, B:
 * [n_cache][n_fields]; eval_x: [dim][n_eval]; U: [n_eval][n_fields].
 * workspace: caller-owned, 256-byte aligned device buffer of
 * bvc_gather_multi_workspace_bytes(n_cache, precision) bytes (the split
 * coefficients in the MFMA operand layout; 0 bytes for BVC_F32). */
size_t bvc_gather_multi_workspace_bytes(int64_t n_cache, int32_t precision);
int bvc_gather_multi(int32_t dim, int64_t n_cache, const float* cx, const float* cn,
                     int32_t n_fields, const float* A, const float* B, int64_t n_eval,
                     const float* eval_x, float* U, int32_t precision, void* workspace,
                     size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Many uneven scenes in one launch sequence                                */
/* ---------------------------------------------------------------------- */
/* One scene of a batch: its uploaded scene, FP32 walk parameters, its
 * compacted cache (FP64 arrays as bvc_cache_walks takes them, plus FP32
 * copies of positions and normals for the gather), and its interior
 * evaluation points (FP32 [dim][n_eval]) with the output u [n_eval].  All
 * scenes share dim and either all have a source term or none has. */
typedef struct {
  bvc_scene scene;
  bvc_walk_params walk;
  int64_t n_cache;
  const double* x;
  const double* nrm;
  const double* R0;
  const double* xbar;
  const double* w;
  const float* cx;
  const float* cn;
  int64_t n_eval;
  const float* eval_x;
  float* u;
} bvc_batch_item;

typedef struct bvc_batch_s* bvc_batch;

/* Workspace for a batch: the scene table, per-walk samples and exit records
 * of every scene, cache values, counters (0 on invalid items). */
size_t bvc_batch_workspace_bytes(const bvc_batch_item* items, int32_t n_items);
/* Validates the items and uploads the scene table into the caller's
 * 256-byte aligned workspace (synchronises the stream once).  The handle
 * owns host memory only; the workspace and every array an item points to
 * must outlive it. */
int bvc_batch_plan(const bvc_batch_item* items, int32_t n_items, void* workspace, size_t ws_bytes,
                   void* stream, bvc_batch* out);
/* Enqueues, over the concatenated work of all scenes: counter reset, cache
 * walks (walk j of cache point i of a scene keeps id i*W + j and that
 * scene's seed, so every walk equals the single-scene one), FP64 boundary
 * data at the exits, FP64 cache means, and the gather of u (Eq. 3) at each
 * scene's evaluation points.  Only kernels are enqueued: the call can be
 * captured in a HIP graph and replayed. */
int bvc_batch_launch(bvc_batch batch, void* stream);
/* Device pointer to the batch's uint64[4] counters (as bvc_cache_walks). */
int bvc_batch_counters(bvc_batch batch, uint64_t** dev_counters);
/* Device pointers into the batch's workspace, for inspection once a launch
 * has completed (Eqs. 3 and 7 per scene): the FP32 per-walk samples U and D
 * ([sum over scenes of n_cache*W]; scene s starts at the sum of the earlier
 * scenes' n_cache*W, and walk j of its cache point i sits at i*W + j from
 * there) and the FP32 cache values a = u-hat w and b = du/dn-hat w ([sum of
 * n_cache], scene s from the sum of the earlier scenes' n_cache). */
int bvc_batch_results(bvc_batch batch, float** U, float** D, float** a, float** b);
int bvc_batch_destroy(bvc_batch batch);

const char* bvc_last_error(void);
const char* bvc_version(void);

#ifdef __cplusplus
}
#endif
#endif
