/*
 * Plain FP64 CPU oracle for Boundary Value Caching (BVC) with walk on spheres.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two agree only through the
 * problem definition (the paper) and the random-number convention below, which
 * each side implements on its own.
 *
 * What is computed (paper: Miller, Sawhney, Crane, Gkioulekas, "Boundary Value
 * Caching for Walk on Spheres", ACM TOG 42(4), 2023):
 *   - the PDE  Lap u = f in Omega, u = g on the boundary (Eq. 1, sigma = 0,
 *     Dirichlet only);
 *   - the boundary integral equation (Eq. 2) and its Monte Carlo estimators
 *     (Eqs. 3-6), with the free-space kernels of Appendix A.1;
 *   - walk on spheres with an epsilon shell (Section 3.1), the ball-based
 *     gradient estimator (Eq. 7) for du/dn at cache points;
 *   - cache points on the offset Dirichlet boundary at distance l (Section 3.2)
 *     drawn with a CDF table and stratified uniforms (Section 4, Sampling);
 *   - Algorithm 1 (UpdateSolution): cache walks, splat of boundary and source
 *     samples into evaluation points;
 *   - the clamped double-layer kernel and its bias correction by ray-cast
 *     signed-solid-angle sampling with walks at the crossings (Section 3.3,
 *     Eqs. 8-9).
 *
 * Conventions (fixed readings of the paper, listed in the design notes):
 *   G_2D = ln r / (2 pi),  G_3D = -1 / (4 pi r)   (Lap G = delta; Appendix A.1
 *   prints +1/(4 pi r) for 3D, which contradicts its own derivative formulas).
 *   Arrays are row-major AoS: point k of a (n, dim) array is x[k*dim + a].
 *
 * Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *   key     = (seed & 0xffffffff, seed >> 32)
 *   counter = (block, id, batch, tag)
 *   FP64 uniform from words (w0, w1): ((w0 << 21) | (w1 >> 11)) * 2^-53.
 *   Each block yields two uniforms: ua from (w0, w1), ub from (w2, w3).
 *   Walk step k uses blocks 4k + s, s = 0..3 (see orc_walk for the map).
 *   Tags: 1 cache walk, 2 pointwise walk, 3 cache sampling, 4 source sampling,
 *   5 ray directions of the clamping correction, 6 region-of-interest cache,
 *   7 cache on a boundary with a Neumann part.
 */
#ifndef BVC_ORACLE_H
#define BVC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Field kinds (same numbering as the problem descriptors). */
enum {
  ORC_FIELD_ZERO = 0,
  ORC_FIELD_CONST = 1,
  ORC_FIELD_HARMONIC_2D = 2,
  ORC_FIELD_GAUSS_SUM = 3,
  ORC_FIELD_GAUSS_POTENTIAL_2D = 4,
  ORC_FIELD_SOLID_HARMONICS_3D = 5,
  ORC_FIELD_FOURIER_2D = 6,
  ORC_FIELD_POINT_SOURCE = 7,
  ORC_FIELD_EXP_PLANE = 8,
  ORC_FIELD_WEDGE_2D = 9,
  ORC_FIELD_QUADRATIC = 10 /* A |x - x0|^2 + B: A = param[0], B = param[1], x0 = param[2..] */
};

typedef struct {
  int32_t kind;
  int32_t n_coef;
  const double* coef; /* host */
  double param[8];
} orc_field;

typedef struct orc_scene orc_scene;

/* --- Philox and uniforms ------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_uniform_pair(uint64_t seed, uint32_t block, uint32_t id, uint32_t batch,
                      uint32_t tag, double* ua, double* ub);

/* --- Scene and closest point ------------------------------------------- */
orc_scene* orc_scene_new(int dim, const double* verts, int64_t nv, const int32_t* prims,
                         int64_t np);
void orc_scene_free(orc_scene* s);
/* Closest point on the boundary; ties broken by the smallest primitive id.
 * brute != 0 scans every primitive, otherwise the oracle's own BVH is used. */
void orc_closest(const orc_scene* s, const double* x, int brute, double* dist,
                 double* xbar, int32_t* prim);
void orc_closest_batch(const orc_scene* s, int64_t n, const double* x, int brute,
                       double* dist, double* xbar, int32_t* prim);
/* Inside test: 2D nonzero winding number, 3D pseudonormal sign at the closest
 * feature.  Returns the winding number (2D) or 1/0 (3D). */
int orc_inside(const orc_scene* s, const double* x);
/* Classify points: 0 outside, 1 interior (d > l), 2 band (d <= l). */
void orc_classify(const orc_scene* s, int64_t n, const double* x, double l, int32_t* cls);

/* --- Fields --------------------------------------------------------------- */
double orc_field_eval(const orc_field* fld, int dim, const double* x);
void orc_field_eval_batch(const orc_field* fld, int dim, int64_t n, const double* x,
                          double* out);
/* Basis function m of an expandable field (Fourier / solid harmonics). */
double orc_basis_eval(const orc_field* fld, int dim, int m, const double* x);
double orc_ein(double z);

/* --- Green's functions (Appendix A.1, Lap G = delta) ---------------------- */
/* Outputs: G, dG/dx (dim), dG/dn_y, d2G/dxdn_y (dim); any pointer may be NULL. */
void orc_greens(int dim, const double* x, const double* y, const double* ny, double* G,
                double* dGdx, double* dGdn, double* d2Gdxdn);

/* --- Cache sampling (Section 3.2 offset boundary, Section 4 CDF sampling) -- */
/* Draws n candidates on the offset boundary at distance l; writes per
 * candidate the point, unit outward normal of the region {d > l}, weight
 * (total candidate measure / n), closest boundary point xbar (where the
 * control variate reads g), distance and an accept flag.  sides: 1 = inward
 * offsets only, 2 = both sides (2D).  The region-of-interest and mixed
 * samplers report xbar the same way.
 * Returns the number accepted. */
int64_t orc_sample_cache(const orc_scene* s, int64_t n, double l, int sides, uint64_t seed,
                         uint32_t batch, double* x, double* nrm, double* w, double* xbar,
                         double* R0, int32_t* accept);
double orc_candidate_measure(const orc_scene* s, double l, int sides);

/* Cache points on the closed boundary of a region of interest `roi` inside
 * the domain `dom` (Section 3.2): uniform 1/|dR| with stratified uniforms
 * (tag 6), outward normals of R, weight |dR|/n, distance and closest point on
 * the domain boundary; accepted when strictly inside the domain. */
int64_t orc_sample_roi(const orc_scene* dom, const orc_scene* roi, int64_t n, uint64_t seed, uint32_t batch,
                       double* x, double* nrm, double* w, double* xbar, double* R0, int32_t* accept);

/* Source cache: m*m jittered grid over [lo, hi] (2D); s_j = |box|/M f(y)
 * 1[y in R]. */
void orc_sample_sources(const orc_scene* s, const orc_field* f, int64_t m, const double* lo,
                        const double* hi, double l, uint64_t seed, uint32_t batch, double* y,
                        double* sw);

/* --- Walks (Section 3.1, Eq. 7) ---------------------------------------- */
typedef struct {
  double eps;
  int32_t max_steps;
  int32_t n_walks;
  uint64_t seed;
  uint32_t batch;
  int32_t control_variate; /* subtract g(xbar) in the gradient estimate */
  double sigma;            /* screening coefficient of Lap u - sigma u = f (Eq. 1); 0: Poisson */
  double open_center[3];   /* open (unbounded) 3D domain, Appendix B: a sphere that */
  double open_radius;      /* encloses the whole boundary; 0 = bounded domain */
  int32_t side_read;       /* 0: a walk reads g at its closest boundary point and
                              the control variate at xbar, as Section 3.1 states.
                              1 (double-sided data, Appendix B): both read points
                              are moved off the boundary towards the walk (by
                              1e-3 eps at an exit, by 1e-3 |x - xbar| for the
                              control variate), so that data that differ on the
                              two sides of a boundary curve are read on the
                              walk's own side */
} orc_walk_params;

/* Open 3D domains (Appendix B): from x outside the sphere B(c, Rb), u < Rb/|x-c|
 * reaches the sphere (returns 0 and writes the first point hit, from the
 * uniforms v, w); otherwise the path escapes to infinity (returns 1). */
int orc_sphere_reentry(const double* c, double Rb, const double* x, double u, double v, double w, double* y);

/* One walk.  mode 0: cache walk (tag 1, first ball without termination test);
 * mode 1: pointwise walk (tag 2, returns g(xbar) when R0 < eps).  With
 * p->sigma > 0 (screened) every ball multiplies the estimate by
 * orc_screen_ball_weight and the gradient uses orc_screen_grad_weight instead
 * of dim/R0.  With a source f every ball adds -R^2/(2 dim) f(y) times
 * orc_screen_source_ratio (1 without screening), y from the Laplace ball
 * density, weighted by the factors of the balls before it; the first ball's
 * gradient adds its centre-gradient source sample (see grad_source_point).
 * With p->open_radius > 0 (3D, Laplace, no source) a walk that lands outside
 * the enclosing sphere draws orc_sphere_reentry's uniforms from the Philox
 * counters (jump index, id, batch, tag | 8) and (..., tag | 16); an escaped walk
 * takes u = 0 at infinity and reports a NaN exit point.
 * Outputs U (solution sample), grad (dim; gradient sample), exit point,
 * first-step weight (dim/R0)*(nu . n) (cache mode), steps, capped flag. */
void orc_walk(const orc_scene* s, const orc_field* g, const orc_field* f,
              const orc_walk_params* p, int mode, const double* x, const double* n, double R0,
              const double* xbar, uint32_t id, double* U, double* grad, double* exit_pt,
              double* w1, int32_t* steps, int32_t* capped);

void orc_sample_direction(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch, uint32_t tag,
                          int dim, double* nu);
/* The first ball's gradient source sample (returns t; yhat, y and the weight
 * m(t) as described at grad_source_point). */
double orc_sample_grad_source(uint64_t seed, uint32_t id, uint32_t batch, uint32_t tag, int dim,
                              const double* c, double R, double* yhat, double* y, double* m);
void orc_sample_ball_source(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch, uint32_t tag,
                            int dim, const double* c, double R, double* y);
double orc_grad_radius(double u);

/* Query points of one walk, in the order the walk makes them (Section 3.1):
 * the first-ball point, then every point a jump reaches, up to the query that
 * stops the walk (d < eps or the step cap).  hint[k] is the closest primitive
 * (original id) of query k-1, -1 for the first.  Returns the number written
 * (at most max_q; 0 for a pointwise start inside the epsilon shell). */
int32_t orc_walk_queries(const orc_scene* s, const orc_walk_params* p, int mode, const double* x,
                         double R0, uint32_t id, int32_t max_q, double* q, int32_t* hint);

/* Work of a nearest-first closest-point query on a given BVH (child links and
 * FP64 child boxes stored in the parent, leaves ~((start << 3) | (count - 1))
 * over primitives order[start..]; node 0 is the root): internal nodes expanded
 * and primitive distances evaluated, per query point, with the hint primitive
 * (original id, or -1) evaluated first.  A popped entry whose box is farther
 * than the best distance so far is skipped.  slabs (3D, nullable): a second
 * lower bound per child, (n, smin, smax) at [node][5 c], the distance from n.x
 * to [smin, smax]; a child's bound is the larger of the two. */
void orc_bvh_visits(const orc_scene* s, int64_t n_nodes, const int32_t* child, const double* boxes,
                    const double* slabs, const int32_t* order, int64_t n_q, const double* q,
                    const int32_t* hint, double* nodes, double* prims);

/* All walks of n_cache cache points: U[i*W + j], D[i*W + j] = n_i . grad. */
void orc_cache_walks(const orc_scene* s, const orc_field* g, const orc_field* f,
                     const orc_walk_params* p, int64_t n_cache, const double* x,
                     const double* nrm, const double* R0, const double* xbar, double* U,
                     double* D, double* exit_pt, double* w1, int32_t* steps);
/* Selected walks only (global walk ids). */
void orc_cache_walks_subset(const orc_scene* s, const orc_field* g, const orc_field* f,
                            const orc_walk_params* p, int64_t n_ids, const int64_t* ids,
                            const double* x, const double* nrm, const double* R0,
                            const double* xbar, double* U, double* D, int32_t* steps);
/* Means over walks (in index order): uhat_i, dudn_i. */
void orc_reduce(int64_t n_cache, int32_t W, const double* U, const double* D, double* uhat,
                double* dudn);
/* Pointwise WoS means at n points (W walks each; u and optional gradient). */
void orc_pointwise(const orc_scene* s, const orc_field* g, const orc_field* f,
                   const orc_walk_params* p, int64_t n, const double* x, double* u,
                   double* grad, int64_t* total_steps);

/* --- Gather (Eqs. 3-6) ------------------------------------------------- */
/* u_k = sum_i [dG/dn(x_k,y_i) a_i - G(x_k,y_i) b_i] + sum_j G(x_k,z_j) s_j,
 * grad_k likewise with the x-derivatives.  cond (optional) = sum of |terms|. */
void orc_gather(int dim, int64_t K, const double* ex, int64_t N, const double* cy,
                const double* cn, const double* a, const double* b, int64_t M,
                const double* sy, const double* sw, double* u, double* grad, double* cond);
/* Transposed gather: given r_k = dL/du_k: dL/da_i, dL/db_i, dL/ds_j, and
 * dL/dx_k = r_k grad u(x_k). */
void orc_gather_backward(int dim, int64_t K, const double* ex, const double* r, int64_t N,
                         const double* cy, const double* cn, const double* a, const double* b,
                         int64_t M, const double* sy, const double* sw, double* dLda,
                         double* dLdb, double* dLds, double* dLdx);

/* --- Screened Poisson, sigma > 0 (Eq. 1; Appendix A.2) ----------------- */
/* Modified Bessel functions I0, I1, K0, K1 (x > 0 for K). */
double orc_bessel_i0(double x);
double orc_bessel_i1(double x);
double orc_bessel_k0(double x);
double orc_bessel_k1(double x);
/* Free-space Green's function of Lap - sigma with (Lap - sigma) G = delta:
 * G = -K0(r s)/(2 pi) in 2D, -exp(-r s)/(4 pi r) in 3D (s = sqrt(sigma)), and
 * its derivatives as orc_greens (which is the sigma = 0 case). */
void orc_greens_sigma(int dim, double sigma, const double* x, const double* y, const double* ny,
                      double* G, double* dGdx, double* dGdn, double* d2Gdxdn);
/* Screened ball weights at radius R: the mean-value factor u(c) = P E[u on the
 * sphere] (2D 1/I0(sR), 3D sR/sinh(sR)) and the gradient factor
 * grad u(c) = w E[nu u(c + R nu)] (2D s/I1(sR), 3D s/i1(sR)); sigma = 0 gives
 * 1 and dim/R. */
double orc_screen_ball_weight(int dim, double sigma, double R);
double orc_screen_grad_weight(int dim, double sigma, double R);
/* Screened over Laplace ball Green's function at r = t R (in-ball source term)
 * and the same ratio for the centre gradient of the in-ball source term; 1 at
 * sigma = 0. */
double orc_screen_source_ratio(int dim, double sigma, double R, double t);
double orc_screen_grad_source_ratio(int dim, double sigma, double R, double t);
/* orc_gather with the screened kernels (sigma = 0: orc_gather). */
void orc_gather_sigma(int dim, double sigma, int64_t K, const double* ex, int64_t N, const double* cy,
                      const double* cn, const double* a, const double* b, int64_t M, const double* sy,
                      const double* sw, double* u, double* grad, double* cond);

/* --- Walk on stars, mixed Dirichlet / Neumann boundaries (2D and 3D) ---- */
/* `dir` and `neu` hold the Dirichlet and the Neumann elements of one
 * boundary (2D: counter-clockwise segments; 3D: triangles, outward by the
 * right-hand rule).  Walk j of start point i has id i*W + j.
 * mode 0: from an offset Dirichlet cache point (normal nrm, R0 = distance to
 * the whole boundary, xbar = closest Dirichlet point): first ball of radius
 * R0 with the gradient estimate D = n . (dim/R0) nu (U - g(xbar)) (Eq. 7),
 * tag 1; mode 1: from an interior point, tag 2; mode 3: from a point on the
 * Neumann boundary (nrm = outward normal), tag 2.  Star radius
 * max(eps, min(d_Dirichlet, d_silhouette)) (2D silhouettes: corner vertices
 * seen with both neighbours on one side, run ends; a vertex where the
 * boundary continues straight is no corner; 3D silhouettes: edges where the
 * Neumann part ends and edges between non-coplanar triangles that x does not
 * see both from the front or both from the back); direction uniform (block
 * 4k), turned into the inward half space on the Neumann boundary; the next
 * point is the nearest Neumann crossing within the radius, else the sphere
 * point.  Neumann data h (NULL or kind 0: h = 0): every star adds one sample
 * of its Neumann term (see neumann_term in oracle.c: an element within R
 * drawn by measure with an exponential race, Philox tag | 32 | (k << 8) and
 * block = element index; z uniform on it, block 4k + 1, tag | 64;
 * |C| G^B(x, z) h(z), doubled on the Neumann boundary; candidates within
 * R (1 + 1e-9)).  Stops when
 * d_Dirichlet < eps (or max_steps) with U = g at the closest Dirichlet point
 * plus the walk's Neumann terms.  D may be NULL. */
/* Distance from each x (n x dim) to the closest silhouette of the Neumann
 * elements `neu` as the walk on stars uses it (INFINITY if none). */
void orc_silhouette_distances(const orc_scene* neu, int64_t n, const double* x, double* d);
void orc_wost_walks(const orc_scene* dir, const orc_scene* neu, const orc_field* g, const orc_field* h,
                    const orc_walk_params* p, int mode, int64_t n, const double* x, const double* nrm,
                    const double* R0, const double* xbar, double* U, double* D, int32_t* steps);

/* Cache candidates for a boundary with a Neumann part (2D): the offset
 * Dirichlet boundary (distance l to the Dirichlet part, inside `full`) and
 * the Neumann part beyond distance l, one stratified draw (tag 7); type 0
 * offset / 1 Neumann; R0 = distance to the whole boundary, xbar = closest
 * Dirichlet point.  junction_drop >= 0: offset points closer than
 * junction_drop * l to the Neumann part are rejected too (0 = the plain
 * sampler; a positive value removes the pieces of the offset curve next to a
 * Dirichlet / Neumann junction, a bias traded for the variance of their
 * small first balls).  Returns the number accepted. */
int64_t orc_sample_mixed(const orc_scene* full, const orc_scene* dir, const orc_scene* neu, int64_t n, double l,
                         double junction_drop, uint64_t seed, uint32_t batch, double* x, double* nrm, double* w,
                         double* xbar, double* R0, int32_t* type, int32_t* accept);

/* --- Clamped double-layer kernel and bias correction (Section 3.3) ------ */
/* Distance beyond which |dG/dn| cannot exceed c (INFINITY for c <= 0). */
double orc_clamp_radius(int dim, double c);
/* u only, with dG/dn clamped to [-c, c] (Eq. 9) in the boundary term. */
void orc_gather_clamped(int dim, int64_t K, const double* ex, int64_t N, const double* cy,
                        const double* cn, const double* a, const double* b, int64_t M,
                        const double* sy, const double* sw, double c, double* u);
/* Crossings of the ray x + t w (0 < t <= t_max, |w| = 1) with the offset
 * boundary {z inside : d(z) = l}: returns how many there are and writes the
 * nearest max_hits: t, point z and the unit outward normal of {d > l} at z
 * (pointing to the closest boundary point). */
int32_t orc_offset_hits(const orc_scene* s, double l, int sides, const double* x, const double* w,
                        double t_max, int32_t max_hits, double* t_out, double* z_out, double* n_out);
/* Ray direction j of point k (Philox block j, id k, tag 5). */
void orc_ray_direction(uint64_t seed, uint32_t j, uint32_t k, uint32_t batch, int dim, double* w);
/* Bias correction of the clamped gather (Eq. 8, second integral) at n points:
 * corr[k] = (1/n_rays) sum_j sum_h sign(K) (1 - c/|K|) u(z_jh) over the
 * crossings with |K| > c, ranked h nearest first (at most max_hits per ray),
 * with u from one pointwise walk per crossing (id (k n_rays + j) max_hits + h)
 * or from u_at_hits when not NULL.  stats: contributing crossings, walks,
 * rays with more than max_hits contributing crossings. */
void orc_clamp_correction(const orc_scene* s, const orc_field* g, const orc_field* f,
                          const orc_walk_params* p, double l, int sides, double c, int32_t n_rays,
                          int32_t max_hits, const orc_field* u_at_hits, int64_t n, const double* x,
                          double* corr, int64_t* stats);

/* --- Basis expansion from exit records (linearity in the boundary data) --- */
/* E[i*nb + m] = (1/W) sum_j phi_m(exit_ij),
 * F[i*nb + m] = (1/W) sum_j w1_ij (phi_m(exit_ij) - cv * phi_m(xbar_i)). */
void orc_basis_means(const orc_field* basis, int dim, int64_t n_cache, int32_t W,
                     const double* exit_pt, const double* w1, const double* xbar, int cv,
                     double* E, double* F);

int orc_num_threads(void);
/* Threads of the OpenMP loops from here on (n > 0). */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
