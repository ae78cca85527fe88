// Walk on spheres from cache points and from evaluation points (Section 3.1,
// Eq. 7), the FP64 evaluation of the boundary data at the walks' exit points,
// and the fixed-order reduction of walk samples into means.
//
// The walk kernel is persistent: each wave takes walk ids from a global queue,
// one id per idle lane, so a lane whose walk ended starts the next one at the
// following iteration instead of idling until the longest walk of its wave is
// done.  A walk's random numbers depend only on (seed, batch, id), so results
// do not depend on which lane ran it.  The kernel only traces: it records the
// exit point, the in-walk source sum and the first ball's weights, and a
// second kernel evaluates g in FP64 at the exit points.  Keeping the boundary
// data out of the traversal loop keeps its register footprint small.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>

#include "bessel.hpp"
#include "bvc_device.hpp"

namespace bvc {
namespace {

constexpr int kBlock = 256;
// Walk ids a wave claims from the global queue at a time (at most): one
// atomic per chunk rather than one per refill keeps the queue counter, which
// every XCD shares, off the critical path.  Small launches use smaller chunks
// so that every wave still gets work.
constexpr int kChunkMax = 256;

struct WalkArgs {
  SceneDev S;
  FieldDev f;      // source term: kinds 0, 1, 3, 8
  FieldDev g;      // boundary data (read by the screened source walks at their exit)
  double eps;
  int max_steps;
  int W;
  uint64_t seed;
  uint32_t batch;
  uint64_t total;
  int64_t n_pts;
  const double* x;     // mode 0 and 2 start points [D][n] FP64
  const void* px;      // mode 1 start points [D][n] of T
  const uint32_t* ids; // mode 2: queue position -> walk id (the start point's index)
  const double* nrm;   // mode 0 normals [D][n]
  const double* R0;    // [n] distance of each start point to the boundary
  const double* xbar;  // [D][n] closest boundary points (mode 1 shell exit)
  void* U;             // [total] in-walk source sums plus the first-ball term
  void* Dof;           // mode 0 [total] D offset; mode 1 [D][total] gradient offset
  void* exit;          // [D][total] exit points
  void* w1;            // mode 0 [total] (dim/R0) nu.n; mode 1 [D][total] (dim/R0) nu
  int* steps;          // [total] or null
  uint64_t ld;         // stride of the [D][*] records: total (modes 0, 1), the id range (mode 2)
  unsigned long long* counters;
  unsigned long long chunk;  // walk ids per claim, 1..kChunkMax
  int open_lanes;            // leave the traversal loop at this many open queries
  int slab;                  // 3D: prune the traversal with the slab bounds as well
  double sigma;              // screening coefficient (no source term), 0 = Poisson
  double oc[3];              // open 3D domain: sphere enclosing the boundary,
  double orad;               // 0 = bounded domain
  int side;                  // side rule of double-sided data (reads moved towards the walk)
  const int64_t* n_dev;      // device count of start points (modes 0, 1; <= n_pts) or of queued ids
                             // (mode 2; <= total), or null
  const int32_t* order;      // modes 0, 1: launch order of the start points, or null
};

// Open 3D domains (Appendix B).  A walk that has jumped (jump index k) to
// r = |p - oc| > orad escapes to infinity, where u = 0, with probability
// 1 - orad / r, the chance that Brownian motion from p never reaches the
// sphere (returns true).  Otherwise it moves to the first point of the sphere
// it reaches, drawn from the sphere's exterior harmonic measure: by the Kelvin
// transform, the interior harmonic measure from the image point
// oc + (orad / r)^2 (p - oc), whose distance s to the hit point has density
// proportional to 1 / s^2.  Its inverse CDF at v, with rho = orad / r and
// m = 1 - 2 v, gives the cosine of the polar angle about p - oc as
// (m + rho (m^2 + 3) / 2 + rho^2 m + rho^3 (m^2 - 1) / 2) / (1 + rho m)^2,
// accurate as rho -> 0; the azimuth 2 pi w turns about the orthonormal frame
// of Duff et al. (2017).  FP64 whatever the walk's precision: the step is rare.
template <typename T>
__device__ bool open_step(const WalkArgs& a, uint32_t k, uint32_t id, uint32_t tag, T* p) {
  const double e0 = (double)p[0] - a.oc[0], e1 = (double)p[1] - a.oc[1], e2 = (double)p[2] - a.oc[2];
  const double r2 = e0 * e0 + e1 * e1 + e2 * e2;
  if (!(r2 > a.orad * a.orad)) return false;
  double u, v, w, w2;
  Uniform<double>::pair(a.seed, k, id, a.batch, tag | 8u, u, v);
  Uniform<double>::pair(a.seed, k, id, a.batch, tag | 16u, w, w2);
  const double r = sqrt(r2), rho = a.orad / r;
  if (u >= rho) return true;
  const double ex = e0 / r, ey = e1 / r, ez = e2 / r;
  const double m = 1.0 - 2.0 * v, qd = 1.0 + rho * m;
  double ct = (m + rho * (m * m + 3.0) * 0.5 + rho * rho * m + rho * rho * rho * (m * m - 1.0) * 0.5) / (qd * qd);
  ct = fmin(fmax(ct, -1.0), 1.0);
  const double st = sqrt(1.0 - ct * ct);
  const double sg = ez >= 0.0 ? 1.0 : -1.0;
  const double ha = -1.0 / (sg + ez), hb = ex * ey * ha;
  const double t1[3] = {1.0 + sg * ex * ex * ha, sg * hb, -sg * ex};
  const double t2[3] = {hb, sg + ey * ey * ha, -ey};
  const double e[3] = {ex, ey, ez};
  double sp, cp;
  sincos(2.0 * 3.141592653589793 * w, &sp, &cp);
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = (T)(a.oc[c] + a.orad * (ct * e[c] + st * (cp * t1[c] + sp * t2[c])));
  return false;
}

// In-walk source term in the walk's precision (constants, Gaussian sums and
// exponential planes).
// `scale` is 1/(2 sigma^2), times log2(e) in FP32, where the Gaussian factor
// is taken as a power of two on the hardware exp2.
template <typename T>
__device__ __forceinline__ T source_scale(const FieldDev& F) {
  const double inv = 1.0 / (2.0 * F.param[0] * F.param[0]);
  return sizeof(T) == 4 ? (T)(inv * 1.4426950408889634) : (T)inv;
}

template <typename T, int D>
__device__ __forceinline__ T walk_source(const FieldDev& F, T scale, const T* y) {
  if (F.kind == 1) return (T)F.param[0];
  if (F.kind == 8) {
    // A e^(a.y)
    T e = T(0);
#pragma unroll
    for (int q = 0; q < D; ++q) e = fma((T)F.param[1 + q], y[q], e);
    return (T)F.param[0] * exp(e);
  }
  const int ng = F.n_coef / (1 + D);
  T sum = T(0);
  for (int k = 0; k < ng; ++k) {
    const double* c = F.coef + k * (1 + D);
    T r2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T e = y[a] - (T)c[1 + a];
      r2 = fma(e, e, r2);
    }
    if constexpr (sizeof(T) == 4) sum = fmaf((float)c[0], __builtin_amdgcn_exp2f(-r2 * scale), sum);
    else sum = fma(c[0], exp(-r2 * scale), sum);
  }
  return sum;
}

// Mean-value factor of a screened ball (Lap u = sigma u) in 3D at x = s R:
// x / sinh x.  Below 0.5 the even series of sinh x / x avoids the
// cancellation of exp(x) - exp(-x); above, 2 x e^-x / (1 - e^-2x).
template <typename T>
__device__ __forceinline__ T screen_ball_weight3(T x) {
  if (x < T(0.5)) {
    const T x2 = x * x;
    T p = T(1.0 / 6227020800.0);
    p = fma(p, x2, T(1.0 / 39916800.0));
    p = fma(p, x2, T(1.0 / 362880.0));
    p = fma(p, x2, T(1.0 / 5040.0));
    p = fma(p, x2, T(1.0 / 120.0));
    p = fma(p, x2, T(1.0 / 6.0));
    return T(1) / fma(p, x2, T(1));
  }
  const T e = exp(-x);
  return T(2) * x * e / (T(1) - e * e);
}

// Mean-value factor of a screened ball at x = s R: 1/I0(x) in 2D, x/sinh x in 3D.
template <typename T, int D>
__device__ __forceinline__ T screen_ball_weight(T x) {
  if constexpr (D == 3) return screen_ball_weight3<T>(x);
  else return T(1) / bessel_i0<T>(x);
}

// i1(x) = (x cosh x - sinh x) / x^2, the modified spherical Bessel function
// of order 1, by its series sum_k x^(2k+1) / (2^k k! (2k+3)!!) below 1.
__device__ inline double sph_i1(double x) {
  if (x < 1.0) {
    double term = x / 3.0, sum = term;
    for (int k = 1; k < 14; ++k) {
      term *= x * x / (2.0 * k * (2.0 * k + 3.0));
      sum += term;
    }
    return sum;
  }
  return (x * cosh(x) - sinh(x)) / (x * x);
}

// In-ball source terms of the screened equation (sigma > 0 with a source), in
// FP64 for both walk precisions.  Ball B(c, R), sample at r = t R, s =
// sqrt(sigma).  The walks draw the point from the Laplace ball density and
// weight the sample by the ratio of the screened to the Laplace ball Green's
// function,
//   2D [K0(s r) - K0(s R) I0(s r)/I0(s R)] / ln(R/r),
//   3D R sinh(s (R - r)) / ((R - r) sinh(s R)),
// and the first ball's gradient source sample by the ratio of the centre
// gradients,
//   2D s [K1(s r) - I1(s r) K1(s R)/I1(s R)] / (1/r - r/R^2),
//   3D [e^(-s r)(1 + s r) - e^(-s R)(1 + s R) t^2 i1(s r)/i1(s R)] / (1 - t^3)
// (the free-space kernel's radial derivative minus the order-1 mode of the
// part that cancels it on the sphere).
template <int D>
__device__ inline double screen_source_ratio(double s, double R, double t) {
  const double r = t * R;
  if constexpr (D == 2) {
    double k0r, k1r, k0R, k1R, i0r, i1r, i0R, i1R;
    bessel_k01(s * r, k0r, k1r);
    bessel_k01(s * R, k0R, k1R);
    bessel_i01(s * r, i0r, i1r);
    bessel_i01(s * R, i0R, i1R);
    return (k0r - k0R * i0r / i0R) / -log(t);
  } else {
    const double z = s * R * (1.0 - t);
    const double shz = z < 1e-8 ? 1.0 : sinh(z) / z;
    return s * R * shz / sinh(s * R);
  }
}

template <int D>
__device__ inline double screen_grad_source_ratio(double s, double R, double t) {
  const double r = t * R;
  if constexpr (D == 2) {
    double k0r, k1r, k0R, k1R, i0r, i1r, i0R, i1R;
    bessel_k01(s * r, k0r, k1r);
    bessel_k01(s * R, k0R, k1R);
    bessel_i01(s * r, i0r, i1r);
    bessel_i01(s * R, i0R, i1R);
    return s * (k1r - i1r * k1R / i1R) / (1.0 / r - r / (R * R));
  } else {
    const double num = exp(-s * r) * (1.0 + s * r) - exp(-s * R) * (1.0 + s * R) * t * t * sph_i1(s * r) / sph_i1(s * R);
    return num / (1.0 - t * t * t);
  }
}

// The first ball's factors of a screened walk at x = s R0: the mean-value
// factor P (2D 1/I0(x), 3D x/sinh x) and the ratio of the gradient weight to
// dim/R0 (2D s/I1(x), 3D s/i1(x), times R0/dim).  k_finish applies the same
// expressions.
template <int D>
__device__ inline void screen_first_ball(double s, double r0, double& P, double& ratio) {
  const double x = s * r0;
  if constexpr (D == 3) {
    P = x < 1e-8 ? 1.0 : x / sinh(x);
    ratio = s / sph_i1(x) * r0 / D;
  } else {
    double i0, i1;
    bessel_i01(x, i0, i1);
    P = 1.0 / i0;
    ratio = s / i1 * r0 / D;
  }
}

// Wave-private pool of walk ids [next, end) claimed from a global queue in
// chunks.  All lanes of a wave hold the same pool (every update is computed
// from wave-uniform values), so the pool lives in scalar registers.
struct IdPool {
  unsigned long long next = 0, end = 0;
  bool last = false;  // the queue has handed out its final chunk

  // Gives each lane of `need` the next id (~0 when none is left) and sets
  // `exhausted` once the pool and the queue are both empty.
  __device__ unsigned long long take(uint64_t need, int lane, unsigned long long* queue, unsigned long long chunk,
                                     unsigned long long total, bool& exhausted) {
    const unsigned long long cnt = (unsigned long long)__popcll(need);
    const unsigned long long rank = (unsigned long long)__popcll(need & ((1ull << lane) - 1));
    const unsigned long long avail = end - next;
    unsigned long long lo = 0, hi = 0;
    if (avail < cnt && !last) {
      const int leader = __ffsll((unsigned long long)need) - 1;
      unsigned long long c = 0;
      if (lane == leader) c = atomicAdd(queue, chunk);
      c = __shfl(c, leader);
      lo = c;
      hi = c >= total ? c : std::min<unsigned long long>(c + chunk, total);
      last = c + chunk >= total;
    }
    const unsigned long long used_old = std::min(cnt, avail);
    const unsigned long long used_new = std::min(cnt - used_old, hi - lo);
    unsigned long long my = ~0ull;
    if (rank < avail) my = next + rank;
    else if (rank - avail < hi - lo) my = lo + (rank - avail);
    if (hi > lo) {
      next = lo + used_new;
      end = hi;
    } else {
      next += used_old;
    }
    if (last && next >= end) exhausted = true;
    return my;
  }
};

__host__ __device__ inline unsigned long long chunk_for(uint64_t total, int blocks) {
  const uint64_t waves = (uint64_t)blocks * (kBlock / 64);
  const uint64_t c = total / (2 * waves);  // about two chunks per wave
  return c < 1 ? 1 : (c > (uint64_t)kChunkMax ? (uint64_t)kChunkMax : c);
}

// A walk alternates closest-point queries and sphere jumps.  Queries differ in
// length by orders of magnitude (a point near a curved boundary touches few
// nodes, one deep inside a near-spherical domain touches hundreds), so the
// query is resumable: each iteration advances every open query by one step,
// and the jump of the lanes whose query closed runs once at most `open_lanes`
// lanes of the wave are still querying, so that a long query does not hold
// the other lanes back.  Measured on MI355X: 3D triangle meshes run best with
// the jump phase entered at 32 open lanes (about 1.7x faster than waiting for
// all 64); 2D polylines, whose queries are short and even, run best when the
// wave finishes every query first.  bvc_tune_walks can pick another threshold
// and grid size for a problem class.
//
// The slab bounds of a 3D tree pay where the walks see the surface from its
// concave side (inside a closed surface: C3's cache walks 1.65x faster) and
// cost where they see it from the convex side (outside a closed solid: they
// prune little there, and the exterior walks ran 1.7x slower with them), so
// they are a shape choice too: on for bounded domains, off for open ones,
// and the tuner tries the other setting.
struct WalkShape {
  int blocks_per_cu;
  int open_lanes;
  int slabs;
};
WalkShape default_shape(int dim, bool open = false) {
  return WalkShape{8, dim == 3 ? 32 : 0, dim == 3 && !open ? 1 : 0};
}

// A tuned shape belongs to one kernel instance: dimension, precision, source
// term, start mode, open domain (its own kernel) and screening (another
// per-ball cost).
struct WalkClass {
  int dim, dtype, src, mode, open, screened;
  bool operator<(const WalkClass& o) const {
    if (dim != o.dim) return dim < o.dim;
    if (dtype != o.dtype) return dtype < o.dtype;
    if (src != o.src) return src < o.src;
    if (mode != o.mode) return mode < o.mode;
    if (open != o.open) return open < o.open;
    return screened < o.screened;
  }
};
WalkClass walk_class(int dim, const bvc_walk_params* p, int mode) {
  return WalkClass{dim, p->dtype, p->f.kind != 0 ? 1 : 0, mode, p->open_radius > 0.0 ? 1 : 0, p->sigma > 0.0 ? 1 : 0};
}
std::mutex g_walk_mu;
std::map<WalkClass, WalkShape> g_walk_shape;

WalkShape tuned_shape(const WalkClass& k) {
  std::lock_guard<std::mutex> lock(g_walk_mu);
  auto it = g_walk_shape.find(k);
  return it == g_walk_shape.end() ? default_shape(k.dim, k.open != 0) : it->second;
}

// SS: screened walks with a source term (sigma > 0, f != 0), a kernel of their
// own.  They carry the product of their balls' mean-value factors in thr and
// the source terms (each weighted by the factors of the balls before it) in
// acc_s, evaluate g at their exit themselves, and write U = W + usrc / P0
// (W = acc_s + thr g(exit), usrc the first ball's source term, P0 its
// factor), so that the finish's screened formulas (u = P0 U, D from U with
// the first-ball source term moved into the D offset) apply unchanged.
template <typename T, int D, bool SRC, int MODE, bool OPEN, bool SS = false>
__device__ __forceinline__ void walks_body(const WalkArgs& a, uint32_t* lds) {
  static_assert(!SS || SRC, "a screened source walk has a source");
  uint32_t* stk = lds + threadIdx.x;
  const int stride = blockDim.x;
  const int lane = threadIdx.x & 63;
  const uint32_t tag = MODE == 0 ? 1u : 2u;
  const T eps = (T)a.eps;
  const T src_scale = SRC && a.f.kind == 3 ? source_scale<T>(a.f) : T(0);
  // screened walks without a source term carry the product of their balls'
  // mean-value factors in acc_s, the first ball's excepted
  const bool scr = (!SRC || SS) && a.sigma > 0.0;
  const T s_scr = scr ? (T)sqrt(a.sigma) : T(0);
  const double s64 = SS ? sqrt(a.sigma) : 0.0;
  T thr = T(1);
  const SceneDev& S = a.S;
  T* U = (T*)a.U;
  T* Dof = (T*)a.Dof;
  T* EX = (T*)a.exit;
  T* W1 = (T*)a.w1;

  // Lane state.  A walk is active from its start to its exit; `jump` marks a
  // lane whose next action is a sphere jump from p with radius d (the first
  // ball, k = 0, is centred at the start point with radius R0, so it runs the
  // same jump code as every later ball).
  bool active = false, jump = false, exhausted = false;
  IdPool pool;
  // a device-resident count (start points, or queued ids in mode 2, where W
  // is 1) bounds the ids and sets the claim size (the host sized the grid and
  // records for the capacity)
  uint64_t live = a.total;
  unsigned long long chunk = a.chunk;
  if (a.n_dev) {
    const int64_t c = *a.n_dev;
    const uint64_t t = (uint64_t)(c > 0 ? c : 0) * (uint64_t)a.W;
    if (t < live) live = t;
    chunk = chunk_for(live, (int)gridDim.x);
  }
  uint32_t id = 0;
  int k = 0;
  T p[D];
  T d = T(0), acc_s = T(0), usrc = T(0);
  Query<T, D> qs;
  qs.node = -1;
  qs.pa = qs.pb = qs.pc = 0;
  unsigned long long steps_acc = 0, capped_acc = 0, walks_acc = 0;
#pragma unroll
  for (int q = 0; q < D; ++q) p[q] = T(0);

  while (true) {
    // ---- refill idle lanes with new walks from the wave's chunk of ids
    if (!exhausted) {
      const uint64_t need = __ballot(!active);
      if (need) {
        unsigned long long my = pool.take(need, lane, &a.counters[0], chunk, live, exhausted);
        if (!active) {
          if (my != ~0ull && MODE != 2 && a.order) {
            // launch slot -> walk: slot s runs walk s mod W of point
            // order[s / W]; an entry outside the live points skips the walk
            const uint32_t slot = (uint32_t)my, ps = slot / (uint32_t)a.W;
            const int32_t pi = a.order[ps];
            my = (pi >= 0 && (uint64_t)pi * (uint64_t)a.W < live)
                     ? (unsigned long long)pi * (unsigned long long)a.W + (slot - ps * (uint32_t)a.W)
                     : ~0ull;
          }
          if (my != ~0ull) {
            // mode 2 walks start from the points their ids index (one walk each)
            id = MODE == 2 ? a.ids[my] : (uint32_t)my;
            const int64_t i = MODE == 2 ? (int64_t)id : (int64_t)(id / (uint32_t)a.W);
            const T R0 = (T)a.R0[i];
            if (MODE != 0 && R0 < eps) {
              // the start point already lies in the epsilon shell: its walk
              // returns g at the closest boundary point (with the side rule,
              // approached from the start point's side)
              const double t = a.side && R0 > T(0) ? 1e-3 * a.eps / (double)R0 : 0.0;
#pragma unroll
              for (int q = 0; q < D; ++q) {
                const double xq = MODE != 1 ? a.x[q * a.n_pts + i] : (double)((const T*)a.px)[q * a.n_pts + i];
                const double bq = a.xbar[q * a.n_pts + i];
                EX[(size_t)q * a.ld + id] = (T)fma(t, xq - bq, bq);
              }
              U[id] = T(0);
              if (MODE == 1 && Dof) {
#pragma unroll
                for (int q = 0; q < D; ++q) {
                  Dof[(size_t)q * a.ld + id] = T(0);
                  W1[(size_t)q * a.ld + id] = T(0);
                }
              }
              if (a.steps) a.steps[id] = 0;
              ++walks_acc;
            } else {
#pragma unroll
              for (int q = 0; q < D; ++q)
                p[q] = MODE != 1 ? (T)a.x[q * a.n_pts + i] : ((const T*)a.px)[q * a.n_pts + i];
              d = R0;
              k = 0;
              acc_s = scr && !SS ? T(1) : T(0);
              thr = T(1);
              usrc = T(0);
              active = true;
              jump = true;
            }
          }
        }
      }
    }
    // ---- sphere jump: source sample in the ball, direction, next query
    if (jump) {
      T srcv = T(0);
      const T coef = -d * d * (T(1) / T(2 * D));
      if constexpr (SRC) {
        T y[D];
        const T t = ball_source_point<T, D>(a.seed, (uint32_t)k, id, a.batch, tag, p, d, y);
        srcv = walk_source<T, D>(a.f, src_scale, y);
        if constexpr (SS) srcv *= (T)screen_source_ratio<D>(s64, (double)d, (double)t);
      }
      T nu[D];
      walk_direction<T, D>(a.seed, (uint32_t)k, id, a.batch, tag, nu);
      if (k == 0) {
        // first ball: its source term and the weights of the gradient and
        // normal-derivative estimators (Eq. 7 with the control variate)
        usrc = SRC ? coef * srcv : T(0);
        const int64_t i = (int64_t)(id / (uint32_t)a.W);
        const T wgt = fdiv((T)D, d);
        T gs[D];
#pragma unroll
        for (int q = 0; q < D; ++q) gs[q] = T(0);
        if constexpr (SRC) {
          // gradient source sample (the centre gradient of the in-ball source term)
          T yhat[D], yg[D], m;
          const T tg = grad_source_point<T, D>(a.seed, id, a.batch, tag, p, d, yhat, yg, m);
          T c = -m * d * walk_source<T, D>(a.f, src_scale, yg);
          if constexpr (SS) c *= (T)screen_grad_source_ratio<D>(s64, (double)d, (double)tg);
#pragma unroll
          for (int q = 0; q < D; ++q) gs[q] = c * yhat[q];
        }
        // a screened source walk moves its first-ball source term into U / P0
        // and the D offset (the finish multiplies U by P0 and the gradient
        // weight by the screening ratio)
        T du = usrc;
        if constexpr (SS) {
          double P0, ratio;
          screen_first_ball<D>(s64, (double)d, P0, ratio);
          usrc = (T)((double)usrc / P0);
          du = (T)((double)usrc * ratio);
        }
        if constexpr (MODE == 0) {
          T dn = T(0), ds = T(0);
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const T nq = (T)a.nrm[q * a.n_pts + i];
            dn = fma(nu[q], nq, dn);
            ds = fma(gs[q], nq, ds);
          }
          const T w1 = wgt * dn;
          W1[id] = w1;
          Dof[id] = ds - w1 * du;
        } else if (MODE == 1 && Dof) {
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const T gw = wgt * nu[q];
            W1[(size_t)q * a.ld + id] = gw;
            Dof[(size_t)q * a.ld + id] = gs[q] - gw * du;
          }
        }
      } else if constexpr (SS) {
        acc_s = fma(thr * coef, srcv, acc_s);
        thr *= screen_ball_weight<T, D>(s_scr * d);
      } else if constexpr (SRC) {
        acc_s = fma(coef, srcv, acc_s);
      } else if (scr) {
        acc_s *= screen_ball_weight<T, D>(s_scr * d);
      }
#pragma unroll
      for (int c = 0; c < D; ++c) p[c] = fma(d, nu[c], p[c]);
      bool esc = false;
      if constexpr (OPEN) esc = open_step<T>(a, (uint32_t)k, id, tag, p);
      if (!esc) query_begin<T, D>(S, p, k == 0 ? -1 : qs.bi, qs);
      ++k;
      jump = false;
      if (esc) {
        // escaped to infinity: a NaN exit record, read as u = 0 by the finish
#pragma unroll
        for (int c = 0; c < D; ++c) EX[(size_t)c * a.ld + id] = T(NAN);
        U[id] = acc_s + usrc;
        if (a.steps) a.steps[id] = k;
        steps_acc += (unsigned long long)k;
        ++walks_acc;
        active = false;
      }
    }
    if (!__any(active)) {
      if (exhausted) break;
      continue;
    }
    // ---- expand one node per open query until few queries remain open
    while (true) {
      if (active && query_open(qs)) query_step<T, D>(S, p, qs, stk, stride, a.slab != 0);
      if (__popcll(__ballot(active && query_open(qs))) <= a.open_lanes) break;
    }
    // ---- lanes whose query closed: stop in the shell, or jump next
    if (active && !jump && !query_open(qs)) {
      d = fsqrt(qs.best);
      const bool stop = d < eps;
      const bool cap = !stop && k >= a.max_steps;
      if (stop || cap) {
        // g is read at the closest point; with the side rule it is
        // approached from the walk's side by 1e-3 eps, so that data that
        // differ on the two sides of a boundary curve (double-sided
        // conditions, Appendix B) are read on this side
        const T t = a.side && d > T(0) ? fdiv(T(1e-3) * eps, d) : T(0);
        T ex[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          ex[c] = fma(t, p[c] - qs.bq[c], qs.bq[c]);
          EX[(size_t)c * a.ld + id] = ex[c];
        }
        if constexpr (SS) {
          // g at the exit, as the finish would read it for this precision
          double gq;
          if constexpr (sizeof(T) == 4) {
            float q[D];
#pragma unroll
            for (int c = 0; c < D; ++c) q[c] = ex[c];
            gq = field_value_f32(a.g, D, q);
          } else {
            double q[D];
#pragma unroll
            for (int c = 0; c < D; ++c) q[c] = (double)ex[c];
            gq = field_value(a.g, D, q);
          }
          U[id] = fma(thr, (T)gq, acc_s) + usrc;
        } else {
          U[id] = acc_s + usrc;
        }
        if (a.steps) a.steps[id] = k;
        steps_acc += (unsigned long long)k;
        capped_acc += cap ? 1ull : 0ull;
        ++walks_acc;
        active = false;
      } else {
        jump = true;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    steps_acc += __shfl_xor(steps_acc, off);
    capped_acc += __shfl_xor(capped_acc, off);
    walks_acc += __shfl_xor(walks_acc, off);
  }
  if (lane == 0) {
    atomicAdd(&a.counters[1], steps_acc);
    atomicAdd(&a.counters[2], capped_acc);
    atomicAdd(&a.counters[3], walks_acc);
  }
}

// Walks in bounded domains, and (3D, Laplace, no source) in open domains,
// whose extra step stays out of the bounded kernels.  Register budgets of the
// FP32 kernels, set for latency hiding: 2D held to 64 VGPRs (eight waves per
// SIMD, a few values spill), 3D to 72 (seven waves; eight spill too much).
// FP64 kernels keep their registers.
template <typename T, int D, bool SRC, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (D == 2 ? 8 : 7) : 1)))
void k_walks(WalkArgs a) {
  extern __shared__ uint32_t lds[];
  walks_body<T, D, SRC, MODE, false>(a, lds);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_walks_open(WalkArgs a) {
  extern __shared__ uint32_t lds[];
  walks_body<T, 3, false, MODE, true>(a, lds);
}

// Screened walks with a source term (sigma > 0, f != 0).
template <typename T, int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_walks_ss(WalkArgs a) {
  extern __shared__ uint32_t lds[];
  walks_body<T, D, true, MODE, false, true>(a, lds);
}

// Boundary data at the exit points and the control variate (FP32 walks
// evaluate the closed-form kinds of g in FP32, FP64 walks every kind in
// FP64), combined in FP64.
// With W = g(exit) + S:
// U = W + u_src,  mode 0: D = w1 (W - c) + d_src,  mode 1: grad = gw (W - c) + g_src,
// where c = g(xbar) is the control variate (0 when disabled).  Screened walks
// (sigma > 0, no source) recorded the product of their later balls'
// mean-value factors in U: W = U g(exit), U = P(R0) W with the first ball's
// factor P(x) (1/I0(x) in 2D, x / sinh x in 3D, x = s R0), and the weights
// w1, gw (written as dim / R0 times the direction) rescaled to the screened
// ball gradient weight (s / I1(s R0) in 2D, s / i1(s R0) in 3D); a pointwise
// walk that starts in the epsilon shell keeps g.
// A wave finishes kFinishRun runs of 64 consecutive walks, lane l taking walk
// l of each run, so that every load and store is coalesced; a lane evaluates
// the control variate only when its start point changes.
constexpr int kFinishRun = 8;
constexpr int kShTab = (FieldTables::kMaxL + 1) * (FieldTables::kMaxL + 1) + FieldTables::kMaxL + 1;

// The field evaluators of every kind inline here and would take about 170
// VGPRs (two waves per SIMD); four waves hide the streaming loads better, the
// few spilled values sit on the rarely taken kinds' paths.
template <typename T, int D, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_finish(
    FieldDev g, int cv, uint64_t total, int W, int64_t n_pts, const double* xbar, const T* EX, T* U, T* Dof,
    const T* W1, double sigma, double eps, const double* R0, int side, const double* x64, const T* xT,
    const int64_t* n_dev, int ss) {
  // ids below `live` are finished; `total` stays the records' stride
  uint64_t live = total;
  if (n_dev) {
    const int64_t c = *n_dev;
    const uint64_t t = (uint64_t)(c > 0 ? c : 0) * (uint64_t)W;
    if (t < live) live = t;
  }
  // FP32 walks evaluate solid-harmonic data from an FP32 table of
  // coefficient times normalisation kept in LDS
  __shared__ float sh_tab[kShTab];
  const bool sh32 = sizeof(T) == 4 && g.kind == 5 && (int)g.param[0] <= FieldTables::kMaxL;
  if (sh32) {
    solid_harmonics_table(g.coef, (int)g.param[0], sh_tab);
    __syncthreads();
  }
  const int sh_L = (int)g.param[0];
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t id0 = wave * (64 * kFinishRun) + (threadIdx.x & 63);
  // the lane's exits of all runs evaluated together (solid harmonics, FP32),
  // parked in LDS for the run loop
  __shared__ float g8s[kFinishRun * kBlock];
  if constexpr (sizeof(T) == 4 && D == 3) {
    if (sh32) {
      float q8[kFinishRun][3], g8[kFinishRun];
#pragma unroll
      for (int r = 0; r < kFinishRun; ++r) {
        const uint64_t id = id0 + (uint64_t)r * 64;
#pragma unroll
        for (int e = 0; e < 3; ++e) q8[r][e] = id < live ? (float)EX[(size_t)e * total + id] : 0.0f;
      }
      solid_harmonics_f32_n<kFinishRun>(sh_tab, sh_L, q8, g8);
#pragma unroll
      for (int r = 0; r < kFinishRun; ++r)
        g8s[r * kBlock + threadIdx.x] = isnan(q8[r][0]) ? 0.0f : g8[r];  // NaN: escaped, u = 0
    }
  }
  const bool scr = sigma > 0.0;
  const double s = scr ? sqrt(sigma) : 0.0;
  int64_t i_cv = -1;
  double c = 0.0;
  for (int r = 0; r < kFinishRun; ++r) {
    const uint64_t id = id0 + (uint64_t)r * 64;
    if (id >= live) break;
    const int64_t i = (int64_t)(id / (uint64_t)W);
    if (cv && i != i_cv) {
      // the control variate in the walks' precision: any constant keeps the
      // gradient estimate unbiased; the side rule reads it at xbar moved
      // 1e-3 of the way back to the start point
      double xb[D];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        xb[q] = xbar[q * n_pts + i];
        if (side) {
          const double xs = MODE == 0 ? x64[q * n_pts + i] : (double)xT[q * n_pts + i];
          xb[q] = fma(1e-3, xs - xb[q], xb[q]);
        }
      }
      if constexpr (sizeof(T) == 4) {
        float xf[D];
#pragma unroll
        for (int q = 0; q < D; ++q) xf[q] = (float)xb[q];
        if constexpr (D == 3) c = sh32 ? (double)solid_harmonics_f32(sh_tab, sh_L, xf) : field_value_f32(g, D, xf);
        else c = field_value_f32(g, D, xf);
      } else {
        c = field_value(g, D, xb);
      }
      i_cv = i;
    }
    double gq;
    if constexpr (sizeof(T) == 4) {
      if (D == 3 && sh32) {
        gq = (double)g8s[r * kBlock + threadIdx.x];
      } else {
        float q[D];
#pragma unroll
        for (int e = 0; e < D; ++e) q[e] = EX[(size_t)e * total + id];
        gq = isnan(q[0]) ? 0.0 : field_value_f32(g, D, q);  // NaN: escaped, u = 0 at infinity
      }
    } else {
      double q[D];
#pragma unroll
      for (int e = 0; e < D; ++e) q[e] = (double)EX[(size_t)e * total + id];
      gq = isnan(q[0]) ? 0.0 : field_value(g, D, q);
    }
    const double su = (double)U[id];
    double w_est = gq + su, u_est = gq + su, ratio = 1.0;
    if (scr) {
      const double r0 = R0[i];
      if (MODE == 1 && r0 < eps) {
        w_est = u_est = gq;  // no ball: the walk returned g at the closest point
      } else {
        const double x = s * r0;
        // a screened source walk wrote W + usrc / P0 with g already in it
        w_est = ss ? su : su * gq;
        if constexpr (D == 3) {
          u_est = (x < 1e-8 ? 1.0 : x / sinh(x)) * w_est;
          ratio = s / sph_i1(x) * r0 / D;
        } else {
          double i0, i1;
          bessel_i01(x, i0, i1);
          u_est = w_est / i0;
          ratio = s / i1 * r0 / D;
        }
      }
    }
    U[id] = (T)u_est;
    if constexpr (MODE == 0) {
      Dof[id] = (T)((double)W1[id] * ratio * (w_est - c) + (double)Dof[id]);
    } else if (Dof) {
#pragma unroll
      for (int e = 0; e < D; ++e)
        Dof[(size_t)e * total + id] = (T)((double)W1[(size_t)e * total + id] * ratio * (w_est - c) +
                                          (double)Dof[(size_t)e * total + id]);
    }
  }
}

// Distance and closest point of each evaluation point (pointwise walks).
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_closest_points(SceneDev S, int64_t n, const T* x, double* R0,
                                                            double* xbar) {
  extern __shared__ uint32_t lds[];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  T p[D], q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) p[a] = x[a * n + k];
  int hint = -1;
  const T d2 = closest_point<T, D>(S, p, hint, q, lds + threadIdx.x, blockDim.x);
  R0[k] = (double)fsqrt(d2);
#pragma unroll
  for (int a = 0; a < D; ++a) xbar[a * n + k] = (double)q[a];
}

// Means of W samples per point in FP64, one wave per point, fixed order.
template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_reduce(int64_t n, int W, int rows, int64_t ld, const Ti* U,
                                                    const Ti* G, const double* w, double* uhat, double* ghat,
                                                    To* a, To* b, int64_t ld_g, const int64_t* count) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= (count ? std::min<int64_t>(n, *count) : n)) return;
  double su = 0.0;
  double sg[3] = {0.0, 0.0, 0.0};
  for (int j = lane; j < W; j += 64) {
    su += (double)U[i * W + j];
    for (int r = 0; r < rows; ++r) sg[r] += (double)G[r * ld + i * W + j];
  }
  for (int off = 32; off > 0; off >>= 1) {
    su += __shfl_xor(su, off);
    for (int r = 0; r < rows; ++r) sg[r] += __shfl_xor(sg[r], off);
  }
  if (lane == 0) {
    const double mu = su / W;
    if (uhat) uhat[i] = mu;
    if (a) a[i] = (To)(w ? mu * w[i] : mu);
    for (int r = 0; r < rows; ++r) {
      const double mg = sg[r] / W;
      if (ghat) ghat[r * ld_g + i] = mg;
      if (b) b[r * ld_g + i] = (To)(w ? mg * w[i] : mg);
    }
  }
}

// h: the scene of a call that takes open domains (cache, pointwise and
// tuning walks); null for the calls that refuse them.
int check_walk_params(const bvc_walk_params* p, int dim, const SceneHost* h = nullptr, bool count_ok = false,
                      bool order_ok = false) {
  if (!p) return fail(BVC_EINVAL, "walk params are null");
  if (p->n_dev && !count_ok) return fail(BVC_EUNSUPPORTED, "a device point count is taken by the cache walks only");
  if (p->order && !order_ok)
    return fail(BVC_EUNSUPPORTED, "a launch order is taken by the cache, pointwise and tuning walks only");
  if (!(p->eps > 0) || !std::isfinite(p->eps)) return fail(BVC_EINVAL, "eps must be positive");
  if (p->max_steps < 1) return fail(BVC_EINVAL, "max_steps must be >= 1");
  if (p->n_walks < 1) return fail(BVC_EINVAL, "n_walks must be >= 1");
  if (p->dtype != BVC_F32 && p->dtype != BVC_F64) return fail(BVC_EINVAL, "walk dtype must be F32 or F64");
  int rc = check_field(p->g, dim, "g");
  if (rc) return rc;
  rc = check_field(p->f, dim, "f");
  if (rc) return rc;
  if (p->f.kind != 0 && p->f.kind != 1 && p->f.kind != 3 && p->f.kind != 8)
    return fail(BVC_EUNSUPPORTED, "walk source terms are constants, Gaussian sums or exponential planes");
  if (!(p->sigma >= 0.0) || !std::isfinite(p->sigma)) return fail(BVC_EINVAL, "sigma must be finite and >= 0");
  if (p->side_read != 0 && p->side_read != 1) return fail(BVC_EINVAL, "side_read must be 0 or 1");
  if (p->open_radius != 0.0) {
    if (!h) return fail(BVC_EUNSUPPORTED, "open domains are taken by the cache, pointwise and tuning walks only");
    if (dim != 3) return fail(BVC_EUNSUPPORTED, "open domains are built in 3D");
    if (p->sigma != 0.0 || p->f.kind != 0)
      return fail(BVC_EUNSUPPORTED, "open domains take the Laplace equation without a source");
    const double R = p->open_radius;
    if (!(R > 0.0) || !std::isfinite(R)) return fail(BVC_EINVAL, "open_radius must be positive and finite");
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(p->open_center[c])) return fail(BVC_EINVAL, "open_center must be finite");
    for (size_t v = 0; v + 2 < h->V.size(); v += 3) {
      const double x = h->V[v] - p->open_center[0], y = h->V[v + 1] - p->open_center[1],
                   z = h->V[v + 2] - p->open_center[2];
      if (!(x * x + y * y + z * z < R * R)) return fail(BVC_EINVAL, "the open-domain sphere must enclose every vertex");
    }
  }
  return BVC_OK;
}

template <typename T, int D>
void launch_walks(const WalkArgs& args, int mode, bool src, int blocks, size_t lds, hipStream_t st) {
  if constexpr (D == 3) {
    // open domains: validated as 3D, source-free, modes 0 and 1
    if (args.orad > 0.0) {
      if (mode == 0) hipLaunchKernelGGL((k_walks_open<T, 0>), dim3(blocks), dim3(kBlock), lds, st, args);
      else hipLaunchKernelGGL((k_walks_open<T, 1>), dim3(blocks), dim3(kBlock), lds, st, args);
      return;
    }
  }
  if (src && args.sigma > 0.0) {
    // screened with a source: modes 0 and 1 (the batch and clamping calls
    // refuse screening)
    if (mode == 0) hipLaunchKernelGGL((k_walks_ss<T, D, 0>), dim3(blocks), dim3(kBlock), lds, st, args);
    else hipLaunchKernelGGL((k_walks_ss<T, D, 1>), dim3(blocks), dim3(kBlock), lds, st, args);
    return;
  }
  if (mode == 0) {
    if (src) hipLaunchKernelGGL((k_walks<T, D, true, 0>), dim3(blocks), dim3(kBlock), lds, st, args);
    else hipLaunchKernelGGL((k_walks<T, D, false, 0>), dim3(blocks), dim3(kBlock), lds, st, args);
  } else if (mode == 1) {
    if (src) hipLaunchKernelGGL((k_walks<T, D, true, 1>), dim3(blocks), dim3(kBlock), lds, st, args);
    else hipLaunchKernelGGL((k_walks<T, D, false, 1>), dim3(blocks), dim3(kBlock), lds, st, args);
  } else {
    if (src) hipLaunchKernelGGL((k_walks<T, D, true, 2>), dim3(blocks), dim3(kBlock), lds, st, args);
    else hipLaunchKernelGGL((k_walks<T, D, false, 2>), dim3(blocks), dim3(kBlock), lds, st, args);
  }
}

template <typename T, int D>
void launch_finish(const bvc_walk_params* p, int mode, const WalkArgs& a, hipStream_t st) {
  const uint64_t waves = (a.total + 64 * kFinishRun - 1) / (64 * kFinishRun);
  const int blocks = (int)((waves * 64 + kBlock - 1) / kBlock);
  FieldDev g = to_dev(p->g);
  if (mode == 0)
    hipLaunchKernelGGL((k_finish<T, D, 0>), dim3(blocks), dim3(kBlock), 0, st, g, p->control_variate, a.total,
                       a.W, a.n_pts, a.xbar, (const T*)a.exit, (T*)a.U, (T*)a.Dof, (const T*)a.w1, a.sigma,
                       a.eps, a.R0, a.side, a.x, (const T*)a.px, a.n_dev, (p->f.kind != 0 && a.sigma > 0.0) ? 1 : 0);
  else
    hipLaunchKernelGGL((k_finish<T, D, 1>), dim3(blocks), dim3(kBlock), 0, st, g, p->control_variate, a.total,
                       a.W, a.n_pts, a.xbar, (const T*)a.exit, (T*)a.U, (T*)a.Dof, (const T*)a.w1, a.sigma,
                       a.eps, a.R0, a.side, a.x, (const T*)a.px, a.n_dev, (p->f.kind != 0 && a.sigma > 0.0) ? 1 : 0);
}

size_t stack_bytes(const SceneHost& h) { return (size_t)(h.depth + 1) * kBlock * sizeof(uint32_t); }

// Modes 0 and 1: n start points, W walks each, records of stride n W, then
// the FP64 finish.  Mode 2: n walks whose ids (a.ids) index the start points
// and records (stride a.ld, set by the caller); the caller finishes them.
int run_walks(bvc_scene s, const bvc_walk_params* p, int mode, int64_t n, WalkArgs& a, hipStream_t st,
              const WalkShape* force = nullptr) {
  const SceneHost& h = s->h;
  const uint64_t total = (uint64_t)n * (uint64_t)(mode == 2 ? 1 : p->n_walks);
  a.S = h.view();
  a.f = to_dev(p->f);
  a.g = to_dev(p->g);
  a.eps = p->eps;
  a.sigma = p->sigma;
  for (int c = 0; c < 3; ++c) a.oc[c] = p->open_center[c];
  a.orad = p->open_radius;
  a.side = p->side_read != 0;
  a.max_steps = p->max_steps;
  a.W = mode == 2 ? 1 : p->n_walks;
  a.seed = p->seed;
  a.batch = p->batch;
  a.total = total;
  if (mode == 2) {
    a.n_pts = (int64_t)a.ld;
  } else {
    a.n_pts = n;
    a.ld = total;
  }
  int rc = zero_async(a.counters, 4 * sizeof(unsigned long long), st);
  if (rc || total == 0) return rc;
  const WalkShape shape = force ? *force : tuned_shape(walk_class(h.dim, p, mode));
  a.open_lanes = shape.open_lanes;
  a.slab = shape.slabs;
  int blocks = p->blocks > 0 ? p->blocks : num_cus() * shape.blocks_per_cu;
  const int64_t needed = (int64_t)((total + kBlock - 1) / kBlock);
  blocks = (int)std::max<int64_t>(1, std::min<int64_t>(blocks, needed));
  const size_t lds = stack_bytes(h);
  a.chunk = chunk_for(total, blocks);
  const bool src = p->f.kind != 0;
  const bool f32 = p->dtype == BVC_F32;
  if (p->ev_begin) {
    rc = check_hip(hipEventRecord((hipEvent_t)p->ev_begin, st), "walk begin event");
    if (rc) return rc;
  }
  if (h.dim == 2) {
    if (f32) launch_walks<float, 2>(a, mode, src, blocks, lds, st);
    else launch_walks<double, 2>(a, mode, src, blocks, lds, st);
  } else {
    if (f32) launch_walks<float, 3>(a, mode, src, blocks, lds, st);
    else launch_walks<double, 3>(a, mode, src, blocks, lds, st);
  }
  rc = check_hip(hipGetLastError(), "walk launch");
  if (rc) return rc;
  if (p->ev_end) {
    rc = check_hip(hipEventRecord((hipEvent_t)p->ev_end, st), "walk end event");
    if (rc) return rc;
  }
  if (mode == 2) return BVC_OK;
  if (h.dim == 2) {
    if (f32) launch_finish<float, 2>(p, mode, a, st);
    else launch_finish<double, 2>(p, mode, a, st);
  } else {
    if (f32) launch_finish<float, 3>(p, mode, a, st);
    else launch_finish<double, 3>(p, mode, a, st);
  }
  return check_hip(hipGetLastError(), "walk finish launch");
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// Many scenes in one launch: the walk space of the batch is the
// concatenation of every scene's walk ids; a lane maps its global id to
// (scene, local id) by binary search over the scenes' offsets and then runs
// exactly the walk of the single-scene kernel (same counters, same stream).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int batch_scene_of_walk(const BatchDev& b, uint64_t g) {
  int lo = 0, hi = b.n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.scenes[mid].walk_off <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_batch_zero(unsigned long long* c) {
  if (threadIdx.x < 4) c[threadIdx.x] = 0ull;
}

template <int D, bool SRC>
__global__ __launch_bounds__(kBlock) void k_batch_walks(BatchDev b) {
  extern __shared__ uint32_t lds[];
  uint32_t* stk = lds + threadIdx.x;
  const int stride = blockDim.x;
  const int lane = threadIdx.x & 63;
  bool active = false, exhausted = false;
  uint64_t gid = 0;
  uint32_t id = 0;
  int k = 0, hint = -1, sc = 0;
  float p[D];
  float acc_s = 0.f, usrc = 0.f, eps = 0.f, sscale = 0.f;
  unsigned long long steps_acc = 0, capped_acc = 0, walks_acc = 0;
#pragma unroll
  for (int q = 0; q < D; ++q) p[q] = 0.f;
  IdPool pool;
  while (true) {
    if (!exhausted) {
      const uint64_t need = __ballot(!active);
      if (need) {
        const unsigned long long my = pool.take(need, lane, &b.counters[0], b.chunk, b.total_walks, exhausted);
        if (!active) {
          if (my != ~0ull) {
            gid = my;
            sc = batch_scene_of_walk(b, gid);
            const BatchSceneDev& s = b.scenes[sc];
            id = (uint32_t)(gid - s.walk_off);
            eps = (float)s.eps;
            sscale = SRC && s.f.kind == 3 ? source_scale<float>(s.f) : 0.f;
            const int64_t i = (int64_t)(id / (uint32_t)s.W);
            const float R0 = (float)s.R0[i];
            float x0[D], nu0[D];
#pragma unroll
            for (int q = 0; q < D; ++q) x0[q] = (float)s.x[q * s.n_cache + i];
            walk_direction<float, D>(s.seed, 0, id, s.batch, 1u, nu0);
            float dn = 0.f;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              p[q] = fmaf(R0, nu0[q], x0[q]);
              dn = fmaf(nu0[q], (float)s.nrm[q * s.n_cache + i], dn);
            }
            const float w1 = (float)D / R0 * dn;
            usrc = 0.f;
            float ds = 0.f;
            if constexpr (SRC) {
              float yu[D];
              ball_source_point<float, D>(s.seed, 0, id, s.batch, 1u, x0, R0, yu);
              usrc = -R0 * R0 / (float)(2 * D) * walk_source<float, D>(s.f, sscale, yu);
              float yhat[D], yg[D], m;
              grad_source_point<float, D>(s.seed, id, s.batch, 1u, x0, R0, yhat, yg, m);
              const float c = -m * R0 * walk_source<float, D>(s.f, sscale, yg);
#pragma unroll
              for (int q = 0; q < D; ++q) ds = fmaf(c * yhat[q], (float)s.nrm[q * s.n_cache + i], ds);
            }
            b.w1[gid] = w1;
            b.D[gid] = ds - w1 * usrc;
            acc_s = 0.f;
            k = 1;
            hint = -1;
            active = true;
          }
        }
      }
    }
    if (!__any(active)) {
      if (exhausted) break;
      continue;
    }
    if (active) {
      const BatchSceneDev& s = b.scenes[sc];
      float q[D];
      const float d = fsqrt(closest_point<float, D>(s.S, p, hint, q, stk, stride));
      const bool stop = d < eps;
      const bool cap = !stop && k >= s.max_steps;
      if (stop || cap) {
#pragma unroll
        for (int c = 0; c < D; ++c) b.exit[(size_t)c * b.total_walks + gid] = q[c];
        b.U[gid] = acc_s + usrc;
        steps_acc += (unsigned long long)k;
        capped_acc += cap ? 1ull : 0ull;
        ++walks_acc;
        active = false;
      } else {
        if constexpr (SRC) {
          float y[D];
          ball_source_point<float, D>(s.seed, (uint32_t)k, id, s.batch, 1u, p, d, y);
          acc_s = fmaf(-d * d / (float)(2 * D), walk_source<float, D>(s.f, sscale, y), acc_s);
        }
        float nu[D];
        walk_direction<float, D>(s.seed, (uint32_t)k, id, s.batch, 1u, nu);
#pragma unroll
        for (int c = 0; c < D; ++c) p[c] = fmaf(d, nu[c], p[c]);
        ++k;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    steps_acc += __shfl_xor(steps_acc, off);
    capped_acc += __shfl_xor(capped_acc, off);
    walks_acc += __shfl_xor(walks_acc, off);
  }
  if (lane == 0) {
    atomicAdd(&b.counters[1], steps_acc);
    atomicAdd(&b.counters[2], capped_acc);
    atomicAdd(&b.counters[3], walks_acc);
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_batch_finish(BatchDev b) {
  // same coalesced layout as k_finish
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t id0 = wave * (64 * kFinishRun) + (threadIdx.x & 63);
  int64_t i_cv = -1;
  int sc_cv = -1;
  double c = 0.0;
  for (int r = 0; r < kFinishRun; ++r) {
    const uint64_t gid = id0 + (uint64_t)r * 64;
    if (gid >= b.total_walks) break;
    const int sc = batch_scene_of_walk(b, gid);
    const BatchSceneDev& s = b.scenes[sc];
    const int64_t i = (int64_t)((gid - s.walk_off) / (uint64_t)s.W);
    if (s.cv && (i != i_cv || sc != sc_cv)) {
      float xb[D];
#pragma unroll
      for (int a = 0; a < D; ++a) xb[a] = (float)s.xbar[a * s.n_cache + i];
      c = field_value_f32(s.g, D, xb);
      i_cv = i;
      sc_cv = sc;
    }
    if (!s.cv) c = 0.0;
    float q[D];
#pragma unroll
    for (int a = 0; a < D; ++a) q[a] = b.exit[(size_t)a * b.total_walks + gid];
    const double gq = field_value_f32(s.g, D, q);
    const double su = (double)b.U[gid];
    b.U[gid] = (float)(gq + su);
    b.D[gid] = (float)((double)b.w1[gid] * (gq + su - c) + (double)b.D[gid]);
  }
}

// Cache means per point of the batch (one wave per cache point, FP64).
__global__ __launch_bounds__(kBlock) void k_batch_reduce(BatchDev b) {
  const int lane = threadIdx.x & 63;
  const int64_t gi = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (gi >= b.total_cache) return;
  int lo = 0, hi = b.n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.scenes[mid].cache_off <= gi) lo = mid;
    else hi = mid - 1;
  }
  const BatchSceneDev& s = b.scenes[lo];
  const int64_t i = gi - s.cache_off;
  const uint64_t base = s.walk_off + (uint64_t)i * s.W;
  double su = 0.0, sd = 0.0;
  for (int j = lane; j < s.W; j += 64) {
    su += (double)b.U[base + j];
    sd += (double)b.D[base + j];
  }
  for (int off = 32; off > 0; off >>= 1) {
    su += __shfl_xor(su, off);
    sd += __shfl_xor(sd, off);
  }
  if (lane == 0) {
    b.a[gi] = (float)(su / s.W * s.w[i]);
    b.b[gi] = (float)(sd / s.W * s.w[i]);
  }
}

}  // namespace

int launch_batch_walks(const BatchDev& batch, int max_depth, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_zero, dim3(1), dim3(64), 0, st, batch.counters);
  if (batch.total_walks == 0) return check_hip(hipGetLastError(), "batch walks");
  const size_t lds = (size_t)(max_depth + 1) * kBlock * sizeof(uint32_t);
  const int64_t needed = (int64_t)((batch.total_walks + kBlock - 1) / kBlock);
  blocks = (int)std::max<int64_t>(1, std::min<int64_t>(blocks > 0 ? blocks : num_cus() * 8, needed));
  BatchDev b = batch;
  b.chunk = chunk_for(b.total_walks, blocks);
  if (b.dim == 2) {
    if (b.has_src) hipLaunchKernelGGL((k_batch_walks<2, true>), dim3(blocks), dim3(kBlock), lds, st, b);
    else hipLaunchKernelGGL((k_batch_walks<2, false>), dim3(blocks), dim3(kBlock), lds, st, b);
  } else {
    if (b.has_src) hipLaunchKernelGGL((k_batch_walks<3, true>), dim3(blocks), dim3(kBlock), lds, st, b);
    else hipLaunchKernelGGL((k_batch_walks<3, false>), dim3(blocks), dim3(kBlock), lds, st, b);
  }
  const uint64_t fwaves = (b.total_walks + 64 * kFinishRun - 1) / (64 * kFinishRun);
  const int fblocks = (int)((fwaves * 64 + kBlock - 1) / kBlock);
  if (b.dim == 2) hipLaunchKernelGGL(k_batch_finish<2>, dim3(fblocks), dim3(kBlock), 0, st, b);
  else hipLaunchKernelGGL(k_batch_finish<3>, dim3(fblocks), dim3(kBlock), 0, st, b);
  const int per = kBlock / 64;
  const int rblocks = (int)((b.total_cache + per - 1) / per);
  if (rblocks > 0) hipLaunchKernelGGL(k_batch_reduce, dim3(rblocks), dim3(kBlock), 0, st, b);
  return check_hip(hipGetLastError(), "batch walk launch");
}

namespace {
int cache_walks_entry(bvc_scene s, const bvc_walk_params* p, int64_t n_cache, const double* x, const double* nrm,
                      const double* R0, const double* xbar, void* U, void* D, void* rec_exit, void* rec_w1,
                      int32_t* rec_steps, uint64_t* counters, void* stream, const WalkShape* force) {
  int rc = check_scene(s);
  if (rc) return rc;
  rc = check_walk_params(p, s->h.dim, &s->h, true, true);
  if (rc) return rc;
  if (n_cache < 0) return fail(BVC_EINVAL, "n_cache must be >= 0");
  if ((uint64_t)n_cache * (uint64_t)p->n_walks >= (1ull << 32)) return fail(BVC_EINVAL, "n_cache * W >= 2^32");
  if (!counters) return fail(BVC_EINVAL, "counters is null");
  if (n_cache > 0 && (!x || !nrm || !R0 || !xbar || !U || !D || !rec_exit || !rec_w1))
    return fail(BVC_EINVAL, "null input, output or exit record");
  WalkArgs a{};
  a.x = x;
  a.nrm = nrm;
  a.R0 = R0;
  a.xbar = xbar;
  a.U = U;
  a.Dof = D;
  a.exit = rec_exit;
  a.w1 = rec_w1;
  a.steps = rec_steps;
  a.counters = (unsigned long long*)counters;
  a.n_dev = p->n_dev;
  a.order = p->order;
  return run_walks(s, p, 0, n_cache, a, (hipStream_t)stream, force);
}
}  // namespace
}  // namespace bvc

namespace bvc {
namespace {
struct ClampLayout {
  size_t wind, slot_x, slot_R0, slot_xbar, slot_w, flags, ids, scratch, ex, u, total;
};
ClampLayout clamp_layout(int dim, int dtype, int64_t n, int n_rays, int max_hits) {
  const uint64_t slots = (uint64_t)n * n_rays * max_hits;
  const size_t es = dtype == BVC_F32 ? 4 : 8;
  ClampLayout L{};
  size_t o = 0;
  L.wind = o;
  o += align256((size_t)n * 4);
  L.slot_x = o;
  o += align256((size_t)dim * slots * 8);
  L.slot_R0 = o;
  o += align256(slots * 8);
  L.slot_xbar = o;
  o += align256((size_t)dim * slots * 8);
  L.slot_w = o;
  o += align256(slots * 8);
  L.flags = o;
  o += align256(slots * 4);
  L.ids = o;
  o += align256(slots * 4);
  L.scratch = o;
  o += align256((size_t)bvc_compact_scratch_ints((int64_t)slots) * 4);
  L.ex = o;
  o += align256((size_t)dim * slots * es);
  L.u = o;
  o += align256(slots * es);
  L.total = o;
  return L;
}
}  // namespace

// Scratch of bvc_pointwise_wos_noalloc: start radii, closest points, exit
// records and per-walk values live here instead of in caller buffers.  Each
// GPU holds its own copy of the array from module load until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in symbol): static_scratch() resolves each device's own
// address once, with that device current, and every use goes through it.
static __device__ __align__(256) unsigned char scratch[BVC_POINTWISE_STATIC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(char** out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(BVC_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    rc = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(BVC_EDEVICE, "static scratch address is null or misaligned");
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return BVC_OK;
}

// Times one walk class over its launch shapes with `run` (one launch at a
// forced shape, on `st`): the default shape first, in 3D then the other slab
// setting at the default grid and threshold, then the grids of 4, 8 and 16
// blocks per CU and thresholds of 0, 8, 16, 32 and 48 open lanes with the
// slab setting kept.  A shape replaces the default only when at least 3%
// faster, so that timing noise does not move the choice.
template <typename Run>
int search_shapes(int dim, bool open, int reps, hipStream_t st, const Run& run, WalkShape& best) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = check_hip(hipEventCreate(&e0), "tune event");
  if (!rc) rc = check_hip(hipEventCreate(&e1), "tune event");
  auto time_shape = [&](const WalkShape& sh, float& ms) -> int {
    int r = run(sh);  // warm-up
    if (!r) r = check_hip(hipEventRecord(e0, st), "tune event");
    for (int k = 0; k < reps && !r; ++k) r = run(sh);
    if (!r) r = check_hip(hipEventRecord(e1, st), "tune event");
    if (!r) r = check_hip(hipEventSynchronize(e1), "tune sync");
    ms = 0;
    if (!r) r = check_hip(hipEventElapsedTime(&ms, e0, e1), "tune time");
    return r;
  };
  const WalkShape def = default_shape(dim, open);
  best = def;
  float best_ms = INFINITY;
  if (!rc) rc = time_shape(def, best_ms);
  if (!rc && dim == 3) {
    WalkShape flip = def;
    flip.slabs = 1 - def.slabs;
    float ms = 0;
    rc = time_shape(flip, ms);
    if (!rc && ms < 0.97f * best_ms) {
      best = flip;
      best_ms = ms;
    }
  }
  const WalkShape base = best;
  const float base_ms = best_ms;
  const int bpc[3] = {4, 8, 16};
  const int lanes[5] = {0, 8, 16, 32, 48};
  for (int i = 0; i < 3 && !rc; ++i)
    for (int j = 0; j < 5 && !rc; ++j) {
      if (bpc[i] == base.blocks_per_cu && lanes[j] == base.open_lanes) continue;
      const WalkShape sh{bpc[i], lanes[j], base.slabs};
      float ms = 0;
      rc = time_shape(sh, ms);
      if (!rc && ms < best_ms && ms < 0.97f * base_ms) {
        best_ms = ms;
        best = sh;
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

int pointwise_check(bvc_scene s, const bvc_walk_params* p, int64_t n, const void* x, const void* u,
                    const uint64_t* counters) {
  int rc = check_scene(s);
  if (rc) return rc;
  rc = check_walk_params(p, s->h.dim, &s->h, false, true);
  if (rc) return rc;
  if (n < 0) return fail(BVC_EINVAL, "n must be >= 0");
  if ((uint64_t)n * (uint64_t)p->n_walks >= (1ull << 32)) return fail(BVC_EINVAL, "n * W >= 2^32");
  if (!counters) return fail(BVC_EINVAL, "counters is null");
  if (n > 0 && (!x || !u)) return fail(BVC_EINVAL, "null input/output");
  return BVC_OK;
}

// Closest points of the start points, the walks, and the means.  `work` holds
// the layout of bvc_pointwise_workspace_bytes: R0 [n] FP64, xbar [dim][n]
// FP64, exit records [dim][n W], first-ball weights [dim][n W] (grad only).
int pointwise_run(bvc_scene s, const bvc_walk_params* p, int64_t n, const void* x, void* U_walk, void* G_walk,
                  char* work, void* u, void* grad, uint64_t* counters, hipStream_t st,
                  const WalkShape* force = nullptr) {
  const int dim = s->h.dim;
  const size_t es = p->dtype == BVC_F64 ? 8 : 4;
  const size_t nw = (size_t)n * (size_t)p->n_walks;
  char* w = work;
  double* R0 = (double*)w;
  w += align256((size_t)n * 8);
  double* xbar = (double*)w;
  w += align256((size_t)dim * n * 8);
  void* ex = w;
  w += align256((size_t)dim * nw * es);
  void* gw = grad ? (void*)w : nullptr;
  if (n > 0) {
    const int blocks = (int)((n + kBlock - 1) / kBlock);
    const size_t lds = stack_bytes(s->h);
    SceneDev S = s->h.view();
    if (dim == 2) {
      if (p->dtype == BVC_F32)
        hipLaunchKernelGGL((k_closest_points<float, 2>), dim3(blocks), dim3(kBlock), lds, st, S, n, (const float*)x,
                           R0, xbar);
      else
        hipLaunchKernelGGL((k_closest_points<double, 2>), dim3(blocks), dim3(kBlock), lds, st, S, n,
                           (const double*)x, R0, xbar);
    } else {
      if (p->dtype == BVC_F32)
        hipLaunchKernelGGL((k_closest_points<float, 3>), dim3(blocks), dim3(kBlock), lds, st, S, n, (const float*)x,
                           R0, xbar);
      else
        hipLaunchKernelGGL((k_closest_points<double, 3>), dim3(blocks), dim3(kBlock), lds, st, S, n,
                           (const double*)x, R0, xbar);
    }
  }
  WalkArgs a{};
  a.px = x;
  a.R0 = R0;
  a.xbar = xbar;
  a.U = U_walk;
  a.Dof = grad ? G_walk : nullptr;
  a.exit = ex;
  a.w1 = gw;
  a.counters = (unsigned long long*)counters;
  a.order = p->order;
  int rc = run_walks(s, p, 1, n, a, st, force);
  if (rc || n == 0) return rc;
  const int per = kBlock / 64;
  const int blocks = (int)((n + per - 1) / per);
  const int rows = grad ? dim : 0;
  const int64_t ld = n * (int64_t)p->n_walks;
  if (p->dtype == BVC_F32)
    hipLaunchKernelGGL((k_reduce<float, float>), dim3(blocks), dim3(kBlock), 0, st, n, p->n_walks, rows, ld,
                       (const float*)U_walk, (const float*)G_walk, nullptr, nullptr, nullptr, (float*)u,
                       (float*)grad, n, nullptr);
  else
    hipLaunchKernelGGL((k_reduce<double, double>), dim3(blocks), dim3(kBlock), 0, st, n, p->n_walks, rows, ld,
                       (const double*)U_walk, (const double*)G_walk, nullptr, nullptr, nullptr, (double*)u,
                       (double*)grad, n, nullptr);
  return check_hip(hipGetLastError(), "pointwise reduce launch");
}

int reduce_impl(int64_t n_cache, const int64_t* count, int32_t W, int32_t dti, const void* U, const void* D,
                const double* w, double* uhat, double* dudn, int32_t dto, void* a, void* b, void* stream) {
  if (n_cache < 0 || W < 1) return fail(BVC_EINVAL, "bad sizes");
  if ((dti != BVC_F32 && dti != BVC_F64) || (dto != BVC_F32 && dto != BVC_F64))
    return fail(BVC_EINVAL, "dtype must be F32 or F64");
  if (n_cache == 0) return BVC_OK;
  if (!U || !D) return fail(BVC_EINVAL, "null input");
  if ((a || b) && !w) return fail(BVC_EINVAL, "weights are null");
  hipStream_t st = (hipStream_t)stream;
  const int per = kBlock / 64;
  const int blocks = (int)((n_cache + per - 1) / per);
  const int64_t ld = n_cache * (int64_t)W;
  if (dti == BVC_F32 && dto == BVC_F32)
    hipLaunchKernelGGL((k_reduce<float, float>), dim3(blocks), dim3(kBlock), 0, st, n_cache, W, 1, ld,
                       (const float*)U, (const float*)D, w, uhat, dudn, (float*)a, (float*)b, n_cache, count);
  else if (dti == BVC_F32)
    hipLaunchKernelGGL((k_reduce<float, double>), dim3(blocks), dim3(kBlock), 0, st, n_cache, W, 1, ld,
                       (const float*)U, (const float*)D, w, uhat, dudn, (double*)a, (double*)b, n_cache, count);
  else if (dto == BVC_F32)
    hipLaunchKernelGGL((k_reduce<double, float>), dim3(blocks), dim3(kBlock), 0, st, n_cache, W, 1, ld,
                       (const double*)U, (const double*)D, w, uhat, dudn, (float*)a, (float*)b, n_cache, count);
  else
    hipLaunchKernelGGL((k_reduce<double, double>), dim3(blocks), dim3(kBlock), 0, st, n_cache, W, 1, ld,
                       (const double*)U, (const double*)D, w, uhat, dudn, (double*)a, (double*)b, n_cache, count);
  return check_hip(hipGetLastError(), "reduce launch");
}
}  // namespace
}  // namespace bvc

using namespace bvc;

extern "C" {

double bvc_clamp_radius(int32_t dim, double c) {
  if (!(c > 0.0)) return INFINITY;
  return dim == 2 ? 1.0 / (2.0 * kPi * c) : 1.0 / sqrt(4.0 * kPi * c);
}

int bvc_point_winding(bvc_scene s, int64_t n, const double* x, int32_t* wind, void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  if (s->h.dim != 2) return fail(BVC_EUNSUPPORTED, "winding numbers are for 2D scenes");
  if (n < 0) return fail(BVC_EINVAL, "n must be >= 0");
  if (n > 0 && (!x || !wind)) return fail(BVC_EINVAL, "null argument");
  return launch_point_winding(s->h, n, x, wind, (hipStream_t)stream);
}

size_t bvc_clamp_workspace_bytes(int32_t dim, int32_t dtype, int64_t n, int32_t n_rays, int32_t max_hits) {
  if ((dim != 2 && dim != 3) || n < 0 || n_rays < 1 || max_hits < 1) return 0;
  return clamp_layout(dim, dtype, n, n_rays, max_hits).total;
}

int bvc_clamp_correction(bvc_scene s, const bvc_walk_params* p, const bvc_clamp_params* cp, int64_t n,
                         const double* x, const int32_t* wind, const int64_t* out_index, void* u, void* workspace,
                         size_t workspace_bytes, uint64_t* counters, void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  const int dim = s->h.dim;
  rc = check_walk_params(p, dim);
  if (rc) return rc;
  if (!cp) return fail(BVC_EINVAL, "clamp params are null");
  if (p->sigma > 0.0) return fail(BVC_EUNSUPPORTED, "the clamping correction is built for sigma = 0");
  if (!(cp->l > 0.0) || !std::isfinite(cp->l)) return fail(BVC_EINVAL, "l must be positive");
  if (cp->sides != 1 && !(cp->sides == 2 && dim == 2)) return fail(BVC_EINVAL, "sides must be 1 (or 2 in 2D)");
  if (!(cp->c > 0.0) || !std::isfinite(cp->c)) return fail(BVC_EINVAL, "c must be positive");
  if (cp->n_rays < 1) return fail(BVC_EINVAL, "n_rays must be >= 1");
  if (cp->max_hits < 1 || cp->max_hits > 64) return fail(BVC_EINVAL, "max_hits must be in 1..64");
  if (n < 0) return fail(BVC_EINVAL, "n must be >= 0");
  if (!counters) return fail(BVC_EINVAL, "counters is null");
  const uint64_t slots = (uint64_t)n * cp->n_rays * cp->max_hits;
  if (slots >= (1ull << 31)) return fail(BVC_EINVAL, "n * n_rays * max_hits >= 2^31");
  hipStream_t st = (hipStream_t)stream;
  rc = zero_async(counters, 6 * sizeof(uint64_t), st);
  if (rc || n == 0) return rc;
  if (!x || !u || !workspace) return fail(BVC_EINVAL, "null points, output or workspace");
  if (((uintptr_t)workspace & 255) != 0) return fail(BVC_EINVAL, "workspace must be 256-byte aligned");
  const ClampLayout L = clamp_layout(dim, p->dtype, n, cp->n_rays, cp->max_hits);
  if (workspace_bytes < L.total) return fail(BVC_EINVAL, "workspace too small");
  char* w = (char*)workspace;
  int* wn = (int*)(w + L.wind);
  double* slot_x = (double*)(w + L.slot_x);
  double* slot_R0 = (double*)(w + L.slot_R0);
  double* slot_xbar = (double*)(w + L.slot_xbar);
  double* slot_w = (double*)(w + L.slot_w);
  int* flags = (int*)(w + L.flags);
  int* ids = (int*)(w + L.ids);
  int* scratch = (int*)(w + L.scratch);
  void* EX = w + L.ex;
  void* U = w + L.u;
  if (dim == 2 && !wind) {
    rc = launch_point_winding(s->h, n, x, wn, st);
    if (rc) return rc;
    wind = wn;
  }
  rc = launch_ray_hits(s->h, n, x, wind, cp->l, cp->sides, cp->c, bvc_clamp_radius(dim, cp->c), cp->n_rays,
                       cp->max_hits, p->seed, p->batch, slot_x, slot_R0, slot_xbar, slot_w, flags,
                       (unsigned long long*)counters, st);
  if (rc) return rc;
  // the contributing crossings stay counted on the device (the first 8 bytes
  // of the compaction scratch): the walk launch is sized for every slot and
  // its kernel reads the count, so the call never waits for the GPU
  int64_t* count = (int64_t*)scratch;
  rc = bvc_compact_count((int64_t)slots, flags, 1, ids, scratch, count, stream);
  if (rc) return rc;
  WalkArgs a{};
  a.x = slot_x;
  a.R0 = slot_R0;
  a.xbar = slot_xbar;
  a.ids = (const uint32_t*)ids;
  a.ld = slots;
  a.U = U;
  a.exit = EX;
  a.n_dev = count;
  a.counters = (unsigned long long*)(counters + 2);
  rc = run_walks(s, p, 2, (int64_t)slots, a, st);
  if (rc) return rc;
  return launch_corr_sum(p->g, dim, p->dtype, n, cp->n_rays, cp->max_hits, slot_w, EX, U, out_index, u, st);
}

int bvc_cache_walks(bvc_scene s, const bvc_walk_params* p, int64_t n_cache, const double* x, const double* nrm,
                    const double* R0, const double* xbar, void* U, void* D, void* rec_exit, void* rec_w1,
                    int32_t* rec_steps, uint64_t* counters, void* stream) {
  return cache_walks_entry(s, p, n_cache, x, nrm, R0, xbar, U, D, rec_exit, rec_w1, rec_steps, counters, stream,
                           nullptr);
}

int bvc_tune_walks(bvc_scene s, const bvc_walk_params* p, int64_t n_cache, const double* x, const double* nrm,
                   const double* R0, const double* xbar, void* U, void* D, void* rec_exit, void* rec_w1,
                   uint64_t* counters, int32_t reps, int32_t* blocks_per_cu, int32_t* open_lanes, int32_t* slabs,
                   void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  rc = check_walk_params(p, s->h.dim, &s->h, true, true);
  if (rc) return rc;
  if (reps < 1) return fail(BVC_EINVAL, "reps must be >= 1");
  bvc_walk_params q = *p;
  q.blocks = 0;
  q.ev_begin = nullptr;
  q.ev_end = nullptr;
  WalkShape best{};
  rc = search_shapes(s->h.dim, p->open_radius > 0.0, reps, (hipStream_t)stream,
                     [&](const WalkShape& sh) {
                       return cache_walks_entry(s, &q, n_cache, x, nrm, R0, xbar, U, D, rec_exit, rec_w1, nullptr,
                                                counters, stream, &sh);
                     },
                     best);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lock(g_walk_mu);
    g_walk_shape[walk_class(s->h.dim, p, 0)] = best;
  }
  if (blocks_per_cu) *blocks_per_cu = best.blocks_per_cu;
  if (open_lanes) *open_lanes = best.open_lanes;
  if (slabs) *slabs = best.slabs;
  return BVC_OK;
}

int bvc_tune_pointwise(bvc_scene s, const bvc_walk_params* p, int64_t n, const void* x, void* U_walk, void* G_walk,
                       void* work, size_t work_bytes, void* u, void* grad, uint64_t* counters, int32_t reps,
                       int32_t* blocks_per_cu, int32_t* open_lanes, int32_t* slabs, void* stream) {
  int rc = pointwise_check(s, p, n, x, u, counters);
  if (rc) return rc;
  if (reps < 1) return fail(BVC_EINVAL, "reps must be >= 1");
  if (n > 0 && (!U_walk || !work)) return fail(BVC_EINVAL, "null per-walk scratch or workspace");
  if (grad && !G_walk) return fail(BVC_EINVAL, "grad needs G_walk scratch");
  const size_t need = bvc_pointwise_workspace_bytes(s->h.dim, n, p->n_walks, p->dtype, grad != nullptr);
  if (n > 0 && work_bytes < need) return fail(BVC_EINVAL, "pointwise workspace too small");
  if (((uintptr_t)work & 255) != 0) return fail(BVC_EINVAL, "workspace must be 256-byte aligned");
  bvc_walk_params q = *p;
  q.blocks = 0;
  q.ev_begin = nullptr;
  q.ev_end = nullptr;
  WalkShape best{};
  rc = search_shapes(s->h.dim, p->open_radius > 0.0, reps, (hipStream_t)stream,
                     [&](const WalkShape& sh) {
                       return pointwise_run(s, &q, n, x, U_walk, G_walk, (char*)work, u, grad, counters,
                                            (hipStream_t)stream, &sh);
                     },
                     best);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lock(g_walk_mu);
    g_walk_shape[walk_class(s->h.dim, p, 1)] = best;
  }
  if (blocks_per_cu) *blocks_per_cu = best.blocks_per_cu;
  if (open_lanes) *open_lanes = best.open_lanes;
  if (slabs) *slabs = best.slabs;
  return BVC_OK;
}

size_t bvc_pointwise_workspace_bytes(int32_t dim, int64_t n, int32_t W, int32_t dtype, int32_t with_grad) {
  if (n < 0 || W < 1 || (dim != 2 && dim != 3)) return 0;
  const size_t es = dtype == BVC_F64 ? 8 : 4;
  const size_t nw = (size_t)n * (size_t)W;
  size_t b = align256((size_t)n * 8) + align256((size_t)dim * n * 8) + align256((size_t)dim * nw * es);
  if (with_grad) b += align256((size_t)dim * nw * es);
  return b;
}

int bvc_pointwise_wos(bvc_scene s, const bvc_walk_params* p, int64_t n, const void* x, void* U_walk, void* G_walk,
                      void* work, size_t work_bytes, void* u, void* grad, uint64_t* counters, void* stream) {
  int rc = pointwise_check(s, p, n, x, u, counters);
  if (rc) return rc;
  if (n > 0 && (!U_walk || !work)) return fail(BVC_EINVAL, "null per-walk scratch or workspace");
  if (grad && !G_walk) return fail(BVC_EINVAL, "grad needs G_walk scratch");
  const size_t need = bvc_pointwise_workspace_bytes(s->h.dim, n, p->n_walks, p->dtype, grad != nullptr);
  if (n > 0 && work_bytes < need) return fail(BVC_EINVAL, "pointwise workspace too small");
  if (((uintptr_t)work & 255) != 0) return fail(BVC_EINVAL, "workspace must be 256-byte aligned");
  return pointwise_run(s, p, n, x, U_walk, G_walk, (char*)work, u, grad, counters, (hipStream_t)stream);
}

size_t bvc_pointwise_static_bytes(int32_t dim, int64_t n, int32_t W, int32_t dtype, int32_t with_grad) {
  if (n < 0 || W < 1 || (dim != 2 && dim != 3)) return 0;
  const size_t es = dtype == BVC_F64 ? 8 : 4;
  const size_t nw = (size_t)n * (size_t)W;
  size_t b = bvc_pointwise_workspace_bytes(dim, n, W, dtype, with_grad) + align256(nw * es);
  if (with_grad) b += align256((size_t)dim * nw * es);
  return b;
}

int bvc_pointwise_wos_noalloc(bvc_scene s, const bvc_walk_params* p, int64_t n, const void* x, void* u, void* grad,
                              uint64_t* counters, void* stream) {
  int rc = pointwise_check(s, p, n, x, u, counters);
  if (rc) return rc;
  const size_t need = bvc_pointwise_static_bytes(s->h.dim, n, p->n_walks, p->dtype, grad != nullptr);
  if (need > BVC_POINTWISE_STATIC_BYTES)
    return fail(BVC_EINVAL, "bvc_pointwise_wos_noalloc: " + std::to_string(n) + " points x " +
                                std::to_string(p->n_walks) + " walks need " + std::to_string(need) +
                                " bytes of scratch, more than the library's static " +
                                std::to_string((size_t)BVC_POINTWISE_STATIC_BYTES) +
                                " (use fewer points per call, or bvc_pointwise_wos with a workspace)");
  char* base = nullptr;
  rc = static_scratch(&base);
  if (rc) return rc;
  const int dim = s->h.dim;
  const size_t es = p->dtype == BVC_F64 ? 8 : 4;
  const size_t nw = (size_t)n * (size_t)p->n_walks;
  // layout: the bvc_pointwise_wos workspace, then U_walk [n W], then G_walk [dim][n W]
  char* w = base + bvc_pointwise_workspace_bytes(dim, n, p->n_walks, p->dtype, grad != nullptr);
  void* U_walk = w;
  void* G_walk = grad ? (void*)(w + align256(nw * es)) : nullptr;
  return pointwise_run(s, p, n, x, U_walk, G_walk, base, u, grad, counters, (hipStream_t)stream);
}

int bvc_reduce_walks(int64_t n_cache, int32_t W, int32_t dti, const void* U, const void* D, const double* w,
                     double* uhat, double* dudn, int32_t dto, void* a, void* b, void* stream) {
  return reduce_impl(n_cache, nullptr, W, dti, U, D, w, uhat, dudn, dto, a, b, stream);
}

int bvc_reduce_walks_count(int64_t n_cap, const int64_t* count, int32_t W, int32_t dti, const void* U,
                           const void* D, const double* w, double* uhat, double* dudn, int32_t dto, void* a,
                           void* b, void* stream) {
  if (!count) return fail(BVC_EINVAL, "count is null");
  return reduce_impl(n_cap, count, W, dti, U, D, w, uhat, dudn, dto, a, b, stream);
}

}  // extern "C"
