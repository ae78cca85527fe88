// Walk on stars for mixed Dirichlet / Neumann boundaries in 2D (the WoSt
// estimator of Section 3.1 that the cache relies on when part of the
// boundary is Neumann; homogeneous Neumann data h = 0, no source term).
//
// The Dirichlet and the Neumann segments of one counter-clockwise boundary
// are two scenes with their own BVHs.  From a point x a step takes the star
// radius R = max(eps, min(d_D, d_S)): d_D the distance to the Dirichlet part
// and d_S to the closest silhouette vertex of the Neumann part, so that no
// Neumann segment within R hides another.  A direction is drawn uniformly
// (turned into the inward half circle when the walk stands on the Neumann
// part); the walk moves to the nearest Neumann crossing along it within R,
// else to the sphere.  It stops when d_D < eps and returns g at the closest
// Dirichlet point.  One thread runs one walk; both extra queries traverse the
// Neumann BVH with a stack in LDS (the closest-point query reuses it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "bvc_device.hpp"

namespace bvc {
namespace {

constexpr int kWostBlock = 128;

struct WostArgs {
  SceneDev Sd;  // Dirichlet part
  SceneDev Sn;  // Neumann part
  const int* prev;      // per Neumann segment (original id): start vertex of the segment ending at its start, or -1
  const int* has_next;  // per Neumann segment: 1 when a Neumann segment starts at its end
  FieldDev g;
  double eps;
  int max_steps;
  int W;
  uint64_t seed;
  uint32_t batch;
  int mode;
  int cv;
  int64_t n;
  uint64_t total;
  const double* x;     // [2][n]
  const double* nrm;   // [2][n] (modes 0, 3)
  const double* R0;    // [n] (mode 0): distance to the whole boundary
  const double* xbar;  // [2][n] (mode 0): closest Dirichlet point
  void* U;
  void* D;
  int* steps;
  unsigned long long* counters;
};

// Side of w relative to the line from x through v: +1, -1, or 0 within a
// relative tol of it (a walk on a Neumann segment is on its line only up to
// rounding).
template <typename T>
__device__ __forceinline__ int line_side(const T* x, T vx, T vy, T wx, T wy, T tol) {
  const T ax = vx - x[0], ay = vy - x[1], bx = wx - vx, by = wy - vy;
  const T c = ax * by - ay * bx;
  if (fabs(c) <= tol * sqrt(ax * ax + ay * ay) * sqrt(bx * bx + by * by)) return 0;
  return c > T(0) ? 1 : -1;
}

// Squared distance from p to the closest silhouette vertex of the Neumann
// part: a vertex whose two Neumann neighbours lie strictly on one side of the
// line from p through it, or one on that line and the other off it; the end
// vertex of a Neumann run counts as well.
template <typename T>
__device__ T silhouette_d2(const WostArgs& a, const T* p, uint32_t* stk, int stride) {
  const SceneDev& S = a.Sn;
  const T* pr = SceneArrays<T>::prim(S);
  const T tol = sizeof(T) == 4 ? T(1e-5) : T(1e-9);
  T best = T(INFINITY);
  int sp = 0, node = 0;
  while (true) {
    T lo0[2], hi0[2], lo1[2], hi1[2];
    load_child_boxes<T, 2>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    const T d0 = box_d2<T, 2>(lo0, hi0, p), d1 = box_d2<T, 2>(lo1, hi1, p);
    const int cs[2] = {ch.x, ch.y};
    const T ds[2] = {d0, d1};
    int next = -1;
    for (int s = 0; s < 2; ++s) {
      if (!(ds[s] <= best)) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          const T ax = pr[4 * i], ay = pr[4 * i + 1], bx = pr[4 * i + 2], by = pr[4 * i + 3];
          const int q = S.prim_id[i];
          bool sil = true;
          const int pv = a.prev[q];
          if (pv >= 0) {
            const T ux = (T)S.V[2 * (size_t)pv], uy = (T)S.V[2 * (size_t)pv + 1];
            const int s1 = line_side<T>(p, ax, ay, ux, uy, tol), s2 = line_side<T>(p, ax, ay, bx, by, tol);
            sil = (s1 * s2 > 0) || ((s1 == 0) != (s2 == 0));
          }
          if (sil) best = fmin(best, (ax - p[0]) * (ax - p[0]) + (ay - p[1]) * (ay - p[1]));
          if (!a.has_next[q]) best = fmin(best, (bx - p[0]) * (bx - p[0]) + (by - p[1]) * (by - p[1]));
        }
      } else if (next < 0) {
        next = c;
      } else {
        stk[sp * stride] = (uint32_t)c;
        ++sp;
      }
    }
    if (next < 0 && sp > 0) {
      --sp;
      next = (int)stk[sp * stride];
    }
    if (next < 0) break;
    node = next;
  }
  return best;
}

template <typename T>
__device__ __forceinline__ bool ray_box2(const T* lo, const T* hi, const T* x, const T* w, T t_hi) {
  T t0 = T(0), t1 = t_hi;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (w[q] == T(0)) {
      if (x[q] < lo[q] || x[q] > hi[q]) return false;
      continue;
    }
    const T inv = T(1) / w[q];
    T ta = (lo[q] - x[q]) * inv, tb = (hi[q] - x[q]) * inv;
    if (ta > tb) {
      const T s = ta;
      ta = tb;
      tb = s;
    }
    t0 = fmax(t0, ta);
    t1 = fmin(t1, tb);
  }
  return t0 <= t1;
}

// Nearest crossing of x + t w, lo < t <= hi, with a Neumann segment: t, and
// the leaf-order segment in seg (-1 when none).
template <typename T>
__device__ T neumann_hit(const WostArgs& a, const T* x, const T* w, T lo, T hi, int& seg, uint32_t* stk,
                         int stride) {
  const SceneDev& S = a.Sn;
  const T* pr = SceneArrays<T>::prim(S);
  T best = hi;
  seg = -1;
  int sp = 0, node = 0;
  while (true) {
    T lo0[2], hi0[2], lo1[2], hi1[2];
    load_child_boxes<T, 2>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    const int cs[2] = {ch.x, ch.y};
    const bool hit[2] = {ray_box2<T>(lo0, hi0, x, w, best), ray_box2<T>(lo1, hi1, x, w, best)};
    int next = -1;
    for (int s = 0; s < 2; ++s) {
      if (!hit[s]) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          const T ax = pr[4 * i], ay = pr[4 * i + 1], bx = pr[4 * i + 2], by = pr[4 * i + 3];
          const T e0 = bx - ax, e1 = by - ay;
          const T den = w[0] * e1 - w[1] * e0;
          if (den == T(0)) continue;
          const T r0 = ax - x[0], r1 = ay - x[1];
          const T t = (r0 * e1 - r1 * e0) / den;
          const T u = (r0 * w[1] - r1 * w[0]) / den;
          if (t > lo && u >= T(0) && u <= T(1) && (t < best || (seg < 0 && t <= best))) {
            best = t;
            seg = i;
          }
        }
      } else if (next < 0) {
        next = c;
      } else {
        stk[sp * stride] = (uint32_t)c;
        ++sp;
      }
    }
    if (next < 0 && sp > 0) {
      --sp;
      next = (int)stk[sp * stride];
    }
    if (next < 0) break;
    node = next;
  }
  return best;
}

template <typename T>
__global__ __launch_bounds__(kWostBlock) void k_wost(WostArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t* stk = lds + threadIdx.x;
  const int stride = blockDim.x;
  const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long steps_acc = 0, capped_acc = 0, walks_acc = 0;
  if (id < a.total) {
    const int64_t i = (int64_t)(id / (uint64_t)a.W);
    const uint32_t tag = a.mode == 0 ? 1u : 2u;
    const T eps = (T)a.eps;
    T pos[2] = {(T)a.x[i], (T)a.x[a.n + i]}, nin[2] = {T(0), T(0)}, nu0[2] = {T(0), T(0)};
    bool onb = false;
    int k = 0;
    double R0 = 0.0;
    if (a.mode == 0) {
      R0 = a.R0[i];
      walk_direction<T, 2>(a.seed, 0u, (uint32_t)id, a.batch, tag, nu0);
      pos[0] = (T)(a.x[i] + R0 * (double)nu0[0]);
      pos[1] = (T)(a.x[a.n + i] + R0 * (double)nu0[1]);
      k = 1;
    } else if (a.mode == 3) {
      onb = true;
      nin[0] = -(T)a.nrm[i];
      nin[1] = -(T)a.nrm[a.n + i];
    }
    double W = 0.0;
    bool capped = false;
    for (;; ++k) {
      T q[2];
      int hint = -1;
      const T dD = fsqrt(closest_point<T, 2>(a.Sd, pos, hint, q, stk, stride));
      if (dD < eps || k >= a.max_steps) {
        capped = !(dD < eps);
        const double qd[2] = {(double)q[0], (double)q[1]};
        W = field_value(a.g, 2, qd);
        break;
      }
      const T R = fmax(fmin(dD, fsqrt(silhouette_d2<T>(a, pos, stk, stride))), eps);
      T w[2];
      walk_direction<T, 2>(a.seed, (uint32_t)k, (uint32_t)id, a.batch, tag, w);
      if (onb && w[0] * nin[0] + w[1] * nin[1] < T(0)) {
        w[0] = -w[0];
        w[1] = -w[1];
      }
      int seg;
      const T t = neumann_hit<T>(a, pos, w, T(1e-9) * R, R, seg, stk, stride);
      if (seg >= 0) {
        const T* pr = SceneArrays<T>::prim(a.Sn);
        const T e0 = pr[4 * seg + 2] - pr[4 * seg], e1 = pr[4 * seg + 3] - pr[4 * seg + 1];
        const T len = sqrt(e0 * e0 + e1 * e1);
        pos[0] = fma(t, w[0], pos[0]);
        pos[1] = fma(t, w[1], pos[1]);
        nin[0] = -e1 / len;  // inward normal of a counter-clockwise boundary
        nin[1] = e0 / len;
        onb = true;
      } else {
        pos[0] = fma(R, w[0], pos[0]);
        pos[1] = fma(R, w[1], pos[1]);
        onb = false;
      }
    }
    ((T*)a.U)[id] = (T)W;
    if (a.D) {
      double dv = 0.0;
      if (a.mode == 0) {
        const double xb[2] = {a.xbar[i], a.xbar[a.n + i]};
        const double c = a.cv ? field_value(a.g, 2, xb) : 0.0;
        dv = 2.0 / R0 * ((double)nu0[0] * a.nrm[i] + (double)nu0[1] * a.nrm[a.n + i]) * (W - c);
      }
      ((T*)a.D)[id] = (T)dv;
    }
    if (a.steps) a.steps[id] = k;
    steps_acc = (unsigned long long)k;
    capped_acc = capped ? 1ull : 0ull;
    walks_acc = 1ull;
  }
  for (int off = 32; off > 0; off >>= 1) {
    steps_acc += __shfl_xor(steps_acc, off);
    capped_acc += __shfl_xor(capped_acc, off);
    walks_acc += __shfl_xor(walks_acc, off);
  }
  if ((threadIdx.x & 63) == 0 && walks_acc) {
    atomicAdd(&a.counters[1], steps_acc);
    atomicAdd(&a.counters[2], capped_acc);
    atomicAdd(&a.counters[3], walks_acc);
  }
}

// Neumann run links of a segment set: for each segment (original id) the
// start vertex of the segment ending at its start (-1 if none), and whether
// a segment starts at its end.
void neumann_links(const SceneHost& h, std::vector<int>& prev, std::vector<int>& has_next) {
  std::vector<int> ends_at((size_t)h.nv, -1), starts_at((size_t)h.nv, -1);
  for (int64_t q = 0; q < h.np; ++q) {
    starts_at[(size_t)h.P[2 * q]] = (int)q;
    ends_at[(size_t)h.P[2 * q + 1]] = (int)q;
  }
  prev.assign((size_t)h.np, -1);
  has_next.assign((size_t)h.np, 0);
  for (int64_t q = 0; q < h.np; ++q) {
    const int r = ends_at[(size_t)h.P[2 * q]];
    prev[(size_t)q] = r >= 0 ? h.P[2 * (size_t)r] : -1;
    has_next[(size_t)q] = starts_at[(size_t)h.P[2 * q + 1]] >= 0 ? 1 : 0;
  }
}

}  // namespace
}  // namespace bvc

using namespace bvc;

extern "C" {

size_t bvc_wost_workspace_bytes(bvc_scene neu) {
  if (check_scene(neu)) return 0;
  return (size_t)(2 * neu->h.np) * sizeof(int) + 256;
}

int bvc_wost_walks(bvc_scene dir, bvc_scene neu, const bvc_walk_params* p, int32_t mode, int64_t n, const double* x,
                   const double* nrm, const double* R0, const double* xbar, void* U, void* D, int32_t* steps,
                   void* workspace, size_t workspace_bytes, uint64_t* counters, void* stream) {
  int rc = check_scene(dir);
  if (rc) return rc;
  rc = check_scene(neu);
  if (rc) return rc;
  if (dir->h.dim != 2 || neu->h.dim != 2) return fail(BVC_EUNSUPPORTED, "walk on stars is built for 2D");
  if (!p) return fail(BVC_EINVAL, "walk params are null");
  if (!(p->eps > 0) || p->max_steps < 1 || p->n_walks < 1) return fail(BVC_EINVAL, "bad walk parameters");
  if (p->dtype != BVC_F32 && p->dtype != BVC_F64) return fail(BVC_EINVAL, "walk dtype must be F32 or F64");
  rc = check_field(p->g, 2, "g");
  if (rc) return rc;
  if (p->f.kind != 0 || p->sigma != 0.0)
    return fail(BVC_EUNSUPPORTED, "walk on stars takes no source term and no screening");
  if (mode != 0 && mode != 1 && mode != 3) return fail(BVC_EINVAL, "mode must be 0, 1 or 3");
  if (n < 0 || (uint64_t)n * (uint64_t)p->n_walks >= (1ull << 32)) return fail(BVC_EINVAL, "n * W out of range");
  if (!counters) return fail(BVC_EINVAL, "counters is null");
  hipStream_t st = (hipStream_t)stream;
  rc = zero_async(counters, 4 * sizeof(uint64_t), st);
  if (rc || n == 0) return rc;
  if (!x || !U) return fail(BVC_EINVAL, "null points or output");
  if (mode != 1 && !nrm) return fail(BVC_EINVAL, "modes 0 and 3 need normals");
  if (mode == 0 && (!R0 || !xbar)) return fail(BVC_EINVAL, "mode 0 needs R0 and xbar");
  if (!workspace || workspace_bytes < bvc_wost_workspace_bytes(neu)) return fail(BVC_EINVAL, "workspace too small");
  std::vector<int> prev, has_next;
  neumann_links(neu->h, prev, has_next);
  int* links = (int*)workspace;
  const size_t np = (size_t)neu->h.np;
  rc = check_hip(hipMemcpyAsync(links, prev.data(), np * sizeof(int), hipMemcpyHostToDevice, st), "links upload");
  if (!rc)
    rc = check_hip(hipMemcpyAsync(links + np, has_next.data(), np * sizeof(int), hipMemcpyHostToDevice, st),
                   "links upload");
  if (!rc) rc = check_hip(hipStreamSynchronize(st), "links upload sync");  // the host vectors end here
  if (rc) return rc;
  WostArgs a{};
  a.Sd = dir->h.view();
  a.Sn = neu->h.view();
  a.prev = links;
  a.has_next = links + np;
  a.g = to_dev(p->g);
  a.eps = p->eps;
  a.max_steps = p->max_steps;
  a.W = p->n_walks;
  a.seed = p->seed;
  a.batch = p->batch;
  a.mode = mode;
  a.cv = p->control_variate;
  a.n = n;
  a.total = (uint64_t)n * (uint64_t)p->n_walks;
  a.x = x;
  a.nrm = nrm;
  a.R0 = R0;
  a.xbar = xbar;
  a.U = U;
  a.D = D;
  a.steps = steps;
  a.counters = (unsigned long long*)counters;
  const int depth = std::max(dir->h.depth, neu->h.depth);
  const size_t lds = (size_t)(depth + 2) * kWostBlock * sizeof(uint32_t);
  const int blocks = (int)((a.total + kWostBlock - 1) / kWostBlock);
  if (p->dtype == BVC_F32) hipLaunchKernelGGL(k_wost<float>, dim3(blocks), dim3(kWostBlock), lds, st, a);
  else hipLaunchKernelGGL(k_wost<double>, dim3(blocks), dim3(kWostBlock), lds, st, a);
  return check_hip(hipGetLastError(), "wost launch");
}

}  // extern "C"
