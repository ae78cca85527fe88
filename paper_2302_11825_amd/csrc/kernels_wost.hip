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
constexpr int kHasNext = 1;   // a Neumann segment starts at this segment's end
constexpr int kStraight = 2;  // this segment continues the previous one on a line: its start is no corner

struct WostArgs {
  SceneDev Sd;  // Dirichlet part
  SceneDev Sn;  // Neumann part
  const int* prev;      // per Neumann segment (original id): start vertex of the segment ending at its start, or -1
  const int* flags;     // per Neumann segment: kHasNext | kStraight
  const float4* cones;  // per BVH node and child: normal cone of the child's corner vertices (see wost_tables)
  FieldDev g;
  double eps;
  int max_steps;
  int W;
  uint64_t seed;
  uint32_t batch;
  int mode;
  int cv;
  int side;  // side rule of double-sided data
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

// A child of a BVH node can hold no silhouette vertex for the viewpoint p
// when every direction from p into its box makes an angle with every normal
// of its cone that stays away from a right angle: then all its corner
// vertices see both of their segments from the same side.  cone = (axis,
// sin, cos) of the half-angle (widened on the host); the view cone is the
// box's bounding circle seen from p.
template <typename T>
__device__ __forceinline__ bool cone_culls(const float4 cone, const T* lo, const T* hi, const T* p) {
  const float mx = 0.5f * (float)(lo[0] + hi[0]) - (float)p[0], my = 0.5f * (float)(lo[1] + hi[1]) - (float)p[1];
  const float ex = (float)(hi[0] - lo[0]), ey = (float)(hi[1] - lo[1]);
  const float r2 = 0.25f * (ex * ex + ey * ey);
  const float d2 = mx * mx + my * my;
  if (!(d2 > 1.01f * r2)) return false;  // p inside (or near) the bounding circle
  const float d = sqrtf(d2);
  const float sphi = sqrtf(r2) / d * 1.0001f, cphi = sqrtf(fmaxf(0.0f, 1.0f - sphi * sphi));
  const float cb = cone.w * cphi - cone.z * sphi;  // cos(theta + phi)
  if (!(cb > 0.0f)) return false;
  const float sb = cone.z * cphi + cone.w * sphi;  // sin(theta + phi)
  return fabsf(cone.x * mx + cone.y * my) > sb * d;
}

// Squared distance from p to the closest silhouette vertex of the Neumann
// part within sqrt(bound): a corner vertex whose two Neumann neighbours do
// not lie strictly on opposite sides of the line from p through it (both on
// one side; one on it; both on it, the fold at the tip of a thin Neumann
// curve), and the ends of Neumann runs; a vertex where the boundary continues
// straight is none.  Returns bound when there is none closer (the
// step radius never exceeds the Dirichlet distance, so the search starts
// there).
template <typename T>
__device__ T silhouette_d2(const WostArgs& a, const T* p, T bound, uint32_t* stk, int stride) {
  const SceneDev& S = a.Sn;
  const T* pr = SceneArrays<T>::prim(S);
  const T tol = sizeof(T) == 4 ? T(1e-5) : T(1e-9);
  T best = bound;
  int sp = 0, node = 0;
  while (true) {
    T lo0[2], hi0[2], lo1[2], hi1[2];
    load_child_boxes<T, 2>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    const T d0 = box_d2<T, 2>(lo0, hi0, p), d1 = box_d2<T, 2>(lo1, hi1, p);
    const int cs[2] = {ch.x, ch.y};
    const T ds[2] = {d0, d1};
    const float4 cones[2] = {a.cones[2 * node], a.cones[2 * node + 1]};
    int next = -1;
    for (int s = 0; s < 2; ++s) {
      if (!(ds[s] <= best)) continue;
      const float4 cn = cones[s];
      if (cn.z < -0.5f) continue;  // no corner and no run end below this child
      if (cn.w > -1.5f && cone_culls<T>(cn, s == 0 ? lo0 : lo1, s == 0 ? hi0 : hi1, p)) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          const T ax = pr[4 * i], ay = pr[4 * i + 1], bx = pr[4 * i + 2], by = pr[4 * i + 3];
          const int q = S.prim_id[i];
          const int fl = a.flags[q];
          bool sil = true;
          const int pv = a.prev[q];
          if (fl & kStraight) {
            sil = false;
          } else if (pv >= 0) {
            const T ux = (T)S.V[2 * (size_t)pv], uy = (T)S.V[2 * (size_t)pv + 1];
            const int s1 = line_side<T>(p, ax, ay, ux, uy, tol), s2 = line_side<T>(p, ax, ay, bx, by, tol);
            sil = !(s1 * s2 < 0);  // both on the sight line: a fold (tip of a thin curve)
          }
          if (sil) best = fmin(best, (ax - p[0]) * (ax - p[0]) + (ay - p[1]) * (ay - p[1]));
          if (!(fl & kHasNext)) best = fmin(best, (bx - p[0]) * (bx - p[0]) + (by - p[1]) * (by - p[1]));
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
          // den = |e| w . n_out: only a segment the ray leaves the domain
          // through counts, so that of the two runs of a double-sided
          // Neumann curve (Appendix B) the ray meets the one facing its side
          const T den = w[0] * e1 - w[1] * e0;
          if (!(den > T(0))) continue;
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
      const T d2D = closest_point<T, 2>(a.Sd, pos, hint, q, stk, stride);
      const T dD = fsqrt(d2D);
      if (dD < eps || k >= a.max_steps) {
        capped = !(dD < eps);
        // read g at the closest Dirichlet point (with the side rule,
        // approached from the walk's side)
        const T t = a.side && dD > T(0) ? T(1e-3) * eps / dD : T(0);
        const T qr[2] = {fma(t, pos[0] - q[0], q[0]), fma(t, pos[1] - q[1], q[1])};
        if constexpr (sizeof(T) == 4) {
          W = field_value_f32(a.g, 2, qr);
        } else {
          W = field_value(a.g, 2, qr);
        }
        break;
      }
      const T R = fmax(fmin(dD, fsqrt(silhouette_d2<T>(a, pos, d2D, stk, stride))), eps);
      T w[2];
      walk_direction<T, 2>(a.seed, (uint32_t)k, (uint32_t)id, a.batch, tag, w);
      if (onb && w[0] * nin[0] + w[1] * nin[1] < T(0)) {
        w[0] = -w[0];
        w[1] = -w[1];
      }
      int seg;
      // a walk standing on a Neumann face ignores crossings closer than its
      // position's rounding (in FP32 the other face of a thin Neumann curve
      // lies there); elsewhere every crossing beyond 1e-9 R counts
      const T lo = (sizeof(T) == 4 && onb) ? T(1e-5) * (R + fabs(pos[0]) + fabs(pos[1])) : T(1e-9) * R;
      const T t = neumann_hit<T>(a, pos, w, lo, R, seg, stk, stride);
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
        double xb[2] = {a.xbar[i], a.xbar[a.n + i]};
        if (a.side) {
          xb[0] = fma(1e-3, a.x[i] - xb[0], xb[0]);
          xb[1] = fma(1e-3, a.x[a.n + i] - xb[1], xb[1]);
        }
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

// Host tables of a Neumann segment set.  prev: per segment (original id) the
// start vertex of the segment ending at its start, or -1.  flags: kHasNext
// when a segment starts at its end; kStraight when the segment and the one
// ending at its start continue one line (relative 1e-12), so that their common
// vertex is no corner.  cones: per BVH node and child, the unit normals of
// both segments at every corner vertex below the child (a start vertex that
// is neither straight nor a run start) as (axis, sin, cos) of the half-angle
// widened by 1e-3 rad; sin = -1 when the child holds neither a corner nor a
// run end (never a silhouette), cos = -2 when it holds a run end or its
// normals span a half circle or more (never culled).  A child's segments are
// taken as the leaf-order range its leaves span (a superset, so the cone can
// only be wider than needed).
void wost_tables(const SceneHost& h, std::vector<int>& prev, std::vector<int>& flags, std::vector<float>& cones) {
  std::vector<int> ends_at((size_t)h.nv, -1), starts_at((size_t)h.nv, -1);
  for (int64_t q = 0; q < h.np; ++q) {
    starts_at[(size_t)h.P[2 * q]] = (int)q;
    ends_at[(size_t)h.P[2 * q + 1]] = (int)q;
  }
  prev.assign((size_t)h.np, -1);
  flags.assign((size_t)h.np, 0);
  const double* V = h.V.data();
  auto normal = [&](int from, int to, double* n) {
    const double e0 = V[2 * (size_t)to] - V[2 * (size_t)from], e1 = V[2 * (size_t)to + 1] - V[2 * (size_t)from + 1];
    const double len = std::hypot(e0, e1);
    n[0] = e1 / len;
    n[1] = -e0 / len;
  };
  for (int64_t q = 0; q < h.np; ++q) {
    const int r = ends_at[(size_t)h.P[2 * q]];
    prev[(size_t)q] = r >= 0 ? h.P[2 * (size_t)r] : -1;
    int f = starts_at[(size_t)h.P[2 * q + 1]] >= 0 ? kHasNext : 0;
    if (r >= 0) {
      const double* u = V + 2 * (size_t)prev[(size_t)q];
      const double* a = V + 2 * (size_t)h.P[2 * q];
      const double* b = V + 2 * (size_t)h.P[2 * q + 1];
      const double e0 = a[0] - u[0], e1 = a[1] - u[1], f0 = b[0] - a[0], f1 = b[1] - a[1];
      if (std::fabs(e0 * f1 - e1 * f0) <= 1e-12 * std::hypot(e0, e1) * std::hypot(f0, f1) && e0 * f0 + e1 * f1 > 0)
        f |= kStraight;
    }
    flags[(size_t)q] = f;
  }
  const int nn = (int)h.child.size();
  cones.assign((size_t)nn * 8, 0.0f);
  // leaf-order range below each child, bottom-up (children have larger
  // breadth-first numbers than their parent)
  std::vector<int> rlo(nn, 0), rhi(nn, 0);
  auto child_range = [&](int c, int& lo, int& hi) {
    if (c < 0) {
      lo = leaf_start(c);
      hi = lo + leaf_count(c);
    } else {
      lo = rlo[c];
      hi = rhi[c];
    }
  };
  for (int i = nn - 1; i >= 0; --i) {
    int l0, h0, l1, h1;
    child_range(h.child[i].x, l0, h0);
    child_range(h.child[i].y, l1, h1);
    rlo[i] = std::min(l0, l1);
    rhi[i] = std::max(h0, h1);
  }
  std::vector<double> ns;
  for (int i = 0; i < nn; ++i) {
    for (int s = 0; s < 2; ++s) {
      int lo, hi;
      child_range(s == 0 ? h.child[i].x : h.child[i].y, lo, hi);
      float* out = cones.data() + (size_t)i * 8 + 4 * s;
      bool always = false;
      ns.clear();
      for (int k = lo; k < hi && !always; ++k) {
        const int q = h.prim_id[(size_t)k];
        if (!(flags[(size_t)q] & kHasNext) || prev[(size_t)q] < 0) {
          always = true;
          break;
        }
        if (flags[(size_t)q] & kStraight) continue;
        double n1[2], n2[2];
        normal(prev[(size_t)q], h.P[2 * (size_t)q], n1);
        normal(h.P[2 * (size_t)q], h.P[2 * (size_t)q + 1], n2);
        ns.insert(ns.end(), {n1[0], n1[1], n2[0], n2[1]});
      }
      if (!always && ns.empty()) {
        out[0] = out[1] = 0.0f;
        out[2] = -1.0f;
        out[3] = 1.0f;
        continue;
      }
      double ax = 0, ay = 0;
      for (size_t k = 0; k < ns.size(); k += 2) {
        ax += ns[k];
        ay += ns[k + 1];
      }
      const double al = std::hypot(ax, ay);
      double theta = 4.0;
      if (!always && al > 1e-6 * (double)(ns.size() / 2)) {
        ax /= al;
        ay /= al;
        double cmin = 1.0;
        for (size_t k = 0; k < ns.size(); k += 2) cmin = std::min(cmin, ax * ns[k] + ay * ns[k + 1]);
        theta = std::acos(std::max(-1.0, std::min(1.0, cmin))) + 1e-3;
      }
      if (theta >= 0.5 * kPi) {
        out[0] = out[1] = 0.0f;
        out[2] = 1.0f;
        out[3] = -2.0f;
      } else {
        out[0] = (float)ax;
        out[1] = (float)ay;
        out[2] = (float)std::sin(theta);
        out[3] = (float)std::cos(theta);
      }
    }
  }
}

}  // namespace
}  // namespace bvc

using namespace bvc;

extern "C" {

size_t bvc_wost_workspace_bytes(bvc_scene neu) {
  if (check_scene(neu)) return 0;
  const size_t links = ((size_t)(2 * neu->h.np) * sizeof(int) + 255) / 256 * 256;
  return links + neu->h.child.size() * 8 * sizeof(float) + 256;
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
  if (p->open_radius != 0.0) return fail(BVC_EUNSUPPORTED, "walk on stars is built for bounded domains");
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
  std::vector<int> prev, flags;
  std::vector<float> cones;
  wost_tables(neu->h, prev, flags, cones);
  int* links = (int*)workspace;
  const size_t np = (size_t)neu->h.np;
  float4* cone_dev = (float4*)((char*)workspace + ((2 * np * sizeof(int) + 255) / 256 * 256));
  rc = check_hip(hipMemcpyAsync(links, prev.data(), np * sizeof(int), hipMemcpyHostToDevice, st), "tables upload");
  if (!rc)
    rc = check_hip(hipMemcpyAsync(links + np, flags.data(), np * sizeof(int), hipMemcpyHostToDevice, st),
                   "tables upload");
  if (!rc)
    rc = check_hip(hipMemcpyAsync(cone_dev, cones.data(), cones.size() * sizeof(float), hipMemcpyHostToDevice, st),
                   "tables upload");
  if (!rc) rc = check_hip(hipStreamSynchronize(st), "tables upload sync");  // the host vectors end here
  if (rc) return rc;
  WostArgs a{};
  a.Sd = dir->h.view();
  a.Sn = neu->h.view();
  a.prev = links;
  a.flags = links + np;
  a.cones = cone_dev;
  a.g = to_dev(p->g);
  a.eps = p->eps;
  a.max_steps = p->max_steps;
  a.W = p->n_walks;
  a.seed = p->seed;
  a.batch = p->batch;
  a.mode = mode;
  a.cv = p->control_variate;
  a.side = p->side_read != 0;
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
