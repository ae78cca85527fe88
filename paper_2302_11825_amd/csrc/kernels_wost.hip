// Walk on stars for mixed Dirichlet / Neumann boundaries, 2D and 3D (the
// WoSt estimator of Section 3.1 that the cache relies on when part of the
// boundary is Neumann; Neumann data h, no source term).
//
// The Dirichlet and the Neumann elements of one boundary (2D counter-clockwise
// segments, 3D outward triangles) are two scenes with their own BVHs.  From a
// point x a step takes the star radius R = max(eps, min(d_D, d_S)): d_D the
// distance to the Dirichlet part and d_S to the closest silhouette of the
// Neumann part (2D: corner vertices and run ends; 3D: edges where the Neumann
// part ends and folds between triangles as seen from x), so that no Neumann
// element within R hides another.  With Neumann data h the step adds one
// sample of its star's Neumann term (an element within R drawn by measure,
// a point on it, |C| G^B(x, z) h(z), doubled on the Neumann boundary).  A
// direction is drawn uniformly (turned into the inward half space when the
// walk stands on the Neumann part); the walk moves to the nearest Neumann
// crossing along it within R, else to the sphere.  It stops when d_D < eps
// and returns g at the closest Dirichlet point plus its Neumann terms.  One
// thread runs one walk; the extra queries traverse the Neumann BVH with a
// stack in LDS (the closest-point query reuses it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
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
  const int* prev;      // 2D, per Neumann segment (original id): start vertex of the segment ending at its start, or -1
  const int* flags;     // 2D, per Neumann segment: kHasNext | kStraight
  const float4* cones;  // 2D, per BVH node and child: normal cone of the child's corner vertices (see wost_tables)
  const int* nb;        // 3D, per Neumann triangle (original id) and edge k (vertex k to k + 1): the
                        // triangle across it, or -1 where the Neumann part ends
  const int* flat;      // 3D, per triangle: bit k set when the triangle across edge k is coplanar
  FieldDev g;
  FieldDev h;           // Neumann data (kind 0: h = 0)
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

template <typename T, int D>
__device__ __forceinline__ bool ray_box(const T* lo, const T* hi, const T* x, const T* w, T t_hi) {
  T t0 = T(0), t1 = t_hi;
#pragma unroll
  for (int q = 0; q < D; ++q) {
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
    const bool hit[2] = {ray_box<T, 2>(lo0, hi0, x, w, best), ray_box<T, 2>(lo1, hi1, x, w, best)};
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

// Side of p relative to the plane through v with unit normal n: +1 in front
// (where n points), -1 behind, 0 within a relative tol of the plane.
template <typename T>
__device__ __forceinline__ int plane_side3(const T* p, const T* v, const T* n, T tol) {
  const T d0 = p[0] - v[0], d1 = p[1] - v[1], d2 = p[2] - v[2];
  const T s = n[0] * d0 + n[1] * d1 + n[2] * d2;
  if (fabs(s) <= tol * sqrt(d0 * d0 + d1 * d1 + d2 * d2)) return 0;
  return s > T(0) ? 1 : -1;
}

template <typename T>
__device__ __forceinline__ T segment_d2_3(const T* p, const T* a, const T* b) {
  const T e0 = b[0] - a[0], e1 = b[1] - a[1], e2 = b[2] - a[2];
  const T r0 = p[0] - a[0], r1 = p[1] - a[1], r2 = p[2] - a[2];
  T t = fdiv(r0 * e0 + r1 * e1 + r2 * e2, e0 * e0 + e1 * e1 + e2 * e2);
  t = fmin(fmax(t, T(0)), T(1));
  const T d0 = r0 - t * e0, d1 = r1 - t * e1, d2 = r2 - t * e2;
  return d0 * d0 + d1 * d1 + d2 * d2;
}

template <typename T>
__device__ __forceinline__ void face_normal(const SceneDev& S, int q, T* n) {
#pragma unroll
  for (int c = 0; c < 3; ++c) n[c] = (T)S.fn[3 * (size_t)q + c];
}

// 3D: squared distance from p to the closest silhouette edge of the Neumann
// triangles within sqrt(bound): an edge where the Neumann part ends, or an
// edge between two non-coplanar triangles unless p lies strictly in front
// of both planes or strictly behind both.  Each interior edge is tested from
// the triangle with the larger original id.  Returns bound when none is
// closer.
template <typename T>
__device__ T silhouette_d2_3(const WostArgs& a, const T* p, T bound, uint32_t* stk, int stride) {
  const SceneDev& S = a.Sn;
  const T tol = sizeof(T) == 4 ? T(1e-5) : T(1e-9);
  T best = bound;
  int sp = 0, node = 0;
  while (true) {
    T lo0[3], hi0[3], lo1[3], hi1[3];
    load_child_boxes<T, 3>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    T ds[2] = {box_d2<T, 3>(lo0, hi0, p), box_d2<T, 3>(lo1, hi1, p)};
    slab_bounds<T>(S, node, p, ds[0], ds[1]);
    const int cs[2] = {ch.x, ch.y};
    int next = -1;
    for (int s = 0; s < 2; ++s) {
      if (!(ds[s] <= best)) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          const int q = S.prim_id[i];
          T v[9];
          load_triangle<T>(S, i, v);
          const int fl = a.flat[q];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const int nb = a.nb[3 * q + k];
            if (nb >= 0 && (nb < q || ((fl >> k) & 1))) continue;
            const T* va = v + 3 * k;
            const T* vb = v + 3 * ((k + 1) % 3);
            bool sil = true;
            if (nb >= 0) {
              T n1[3], n2[3];
              face_normal<T>(S, q, n1);
              face_normal<T>(S, nb, n2);
              sil = !(plane_side3<T>(p, va, n1, tol) * plane_side3<T>(p, va, n2, tol) > 0);
            }
            if (sil) best = fmin(best, segment_d2_3<T>(p, va, vb));
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

// 3D: nearest crossing of x + t w, lo < t <= hi, with a Neumann triangle the
// ray leaves the domain through (w . n_out > 0): t, and the leaf-order
// triangle in tri (-1 when none).  The ray's parameters on the triangle by
// Cramer's rule on x + t w = a + u (b - a) + v (c - a).
template <typename T>
__device__ T neumann_hit3(const WostArgs& a, const T* x, const T* w, T lo, T hi, int& tri, uint32_t* stk,
                          int stride) {
  const SceneDev& S = a.Sn;
  T best = hi;
  tri = -1;
  int sp = 0, node = 0;
  while (true) {
    T lo0[3], hi0[3], lo1[3], hi1[3];
    load_child_boxes<T, 3>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    const int cs[2] = {ch.x, ch.y};
    const bool hit[2] = {ray_box<T, 3>(lo0, hi0, x, w, best), ray_box<T, 3>(lo1, hi1, x, w, best)};
    int next = -1;
    for (int s = 0; s < 2; ++s) {
      if (!hit[s]) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          T v[9];
          load_triangle<T>(S, i, v);
          const T e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
          const T e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
          const T n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
          const T den = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
          if (!(den > T(0))) continue;
          const T r[3] = {x[0] - v[0], x[1] - v[1], x[2] - v[2]};
          const T rw[3] = {r[1] * w[2] - r[2] * w[1], r[2] * w[0] - r[0] * w[2], r[0] * w[1] - r[1] * w[0]};
          const T t = -(r[0] * n[0] + r[1] * n[1] + r[2] * n[2]) / den;
          const T u = -(rw[0] * e2[0] + rw[1] * e2[1] + rw[2] * e2[2]) / den;
          const T vv = (rw[0] * e1[0] + rw[1] * e1[1] + rw[2] * e1[2]) / den;
          if (t > lo && u >= T(0) && vv >= T(0) && u + vv <= T(1) && (t < best || (tri < 0 && t <= best))) {
            best = t;
            tri = i;
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

// The Neumann term of one star (Section 3.1: the integral of G^B(x, z) h(z)
// over the Neumann part of the star's boundary, divided by 1/2 when x stands
// on the Neumann part).  Every Neumann element within R (1 + 1e-9) of x (FP32:
// R (1 + 1e-5)) that x does not lie strictly behind is a candidate, a
// superset of the elements that meet the ball (one beyond R draws a point
// outside it and adds 0), so that the elements touching the ball where a
// silhouette sets R, at distance R up to rounding, are in the set in both
// precisions; |C| is their total measure; one is
// drawn with probability measure / |C| by an exponential race (key
// -ln(1 - U) / measure, U the FP64 uniform of Philox block = the element's
// original id, tag | 32 | (k << 8); the smallest key wins whatever order the
// traversal meets the candidates in, keys and measures in FP64 so that the
// choice is the same in both precisions); z is uniform on it (block 4k + 1,
// tag | 64: 2D a + U1 (b - a); 3D barycentric (1 - s, s (1 - U2), s U2),
// s = sqrt(U1)); the sample is |C| G^B(x, z) h(z) / alpha when |z - x| < R,
// else 0, G^B = ln(R / r) / (2 pi) in 2D and (1 / r - 1 / R) / (4 pi) in 3D.
template <typename T, int D>
__device__ double neumann_term(const WostArgs& a, const T* x, T R, bool onb, uint32_t k, uint32_t id,
                               uint32_t tag, uint32_t* stk, int stride) {
  const SceneDev& S = a.Sn;
  const T tol = sizeof(T) == 4 ? T(1e-5) : T(1e-9);
  const T R2 = R * R * (T(1) + T(2) * tol);
  double AC = 0.0, key_best = INFINITY;
  int pick = -1;
  int sp = 0, node = 0;
  while (true) {
    T lo0[D], hi0[D], lo1[D], hi1[D];
    load_child_boxes<T, D>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    T ds[2] = {box_d2<T, D>(lo0, hi0, x), box_d2<T, D>(lo1, hi1, x)};
    if constexpr (D == 3) slab_bounds<T>(S, node, x, ds[0], ds[1]);
    const int cs[2] = {ch.x, ch.y};
    int next = -1;
    for (int s = 0; s < 2; ++s) {
      if (!(ds[s] < R2)) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          T qq[D];
          int reg;
          if (!(prim_d2<T, D>(S, i, x, qq, reg) < R2)) continue;
          const double* v = S.prim64 + (size_t)i * (D == 2 ? 4 : 12);
          double meas;
          if constexpr (D == 2) {
            const T ax = (T)v[0], ay = (T)v[1], bx = (T)v[2], by = (T)v[3];
            const T nx = by - ay, ny = -(bx - ax);  // outward, |e| long
            const T sd = nx * (x[0] - ax) + ny * (x[1] - ay);
            const T dx = x[0] - ax, dy = x[1] - ay;
            if (sd > tol * sqrt(nx * nx + ny * ny) * sqrt(dx * dx + dy * dy)) continue;  // strictly behind
            meas = sqrt((v[2] - v[0]) * (v[2] - v[0]) + (v[3] - v[1]) * (v[3] - v[1]));
          } else {
            T n1[3];
            const int q = S.prim_id[i];
            face_normal<T>(S, q, n1);
            const T va[3] = {(T)v[0], (T)v[1], (T)v[2]};
            if (plane_side3<T>(x, va, n1, tol) > 0) continue;
            const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
            const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
            const double c0 = e1[1] * e2[2] - e1[2] * e2[1], c1 = e1[2] * e2[0] - e1[0] * e2[2],
                         c2 = e1[0] * e2[1] - e1[1] * e2[0];
            meas = 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
          }
          AC += meas;
          double u, unused;
          Uniform<double>::pair(a.seed, (uint32_t)S.prim_id[i], id, a.batch, tag | 32u | (k << 8), u, unused);
          const double key = -log(1.0 - u) / meas;
          if (key < key_best) {
            key_best = key;
            pick = i;
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
  if (pick < 0) return 0.0;
  T u1, u2;
  Uniform<T>::pair(a.seed, 4u * k + 1u, id, a.batch, tag | 64u, u1, u2);
  const T* pr = SceneArrays<T>::prim(S) + (size_t)pick * (D == 2 ? 4 : 12);
  T z[D];
  if constexpr (D == 2) {
#pragma unroll
    for (int q = 0; q < 2; ++q) z[q] = pr[q] + u1 * (pr[2 + q] - pr[q]);
  } else {
    const T sq = sqrt(u1);
#pragma unroll
    for (int q = 0; q < 3; ++q) z[q] = (T(1) - sq) * pr[q] + sq * (T(1) - u2) * pr[3 + q] + sq * u2 * pr[6 + q];
  }
  T r2 = T(0);
#pragma unroll
  for (int q = 0; q < D; ++q) r2 += (z[q] - x[q]) * (z[q] - x[q]);
  const T r = sqrt(r2);
  if (!(r < R) || !(r > T(0))) return 0.0;
  const double G = D == 2 ? log((double)R / (double)r) / (2.0 * kPi) : (1.0 / (double)r - 1.0 / (double)R) / (4.0 * kPi);
  double hz;
  if constexpr (sizeof(T) == 4) {
    hz = field_value_f32(a.h, D, z);
  } else {
    hz = field_value(a.h, D, z);
  }
  return AC * G * hz / (onb ? 0.5 : 1.0);
}

template <typename T, int D>
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
    T pos[D], nin[D], nu0[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      pos[q] = (T)a.x[q * a.n + i];
      nin[q] = T(0);
      nu0[q] = T(0);
    }
    bool onb = false;
    int k = 0;
    double R0 = 0.0, SN = 0.0;
    const bool neumann_data = a.h.kind != 0;
    if (a.mode == 0) {
      R0 = a.R0[i];
      walk_direction<T, D>(a.seed, 0u, (uint32_t)id, a.batch, tag, nu0);
#pragma unroll
      for (int q = 0; q < D; ++q) pos[q] = (T)(a.x[q * a.n + i] + R0 * (double)nu0[q]);
      k = 1;
    } else if (a.mode == 3) {
      onb = true;
#pragma unroll
      for (int q = 0; q < D; ++q) nin[q] = -(T)a.nrm[q * a.n + i];
    }
    double W = 0.0;
    bool capped = false;
    for (;; ++k) {
      T q[D];
      int hint = -1;
      const T d2D = closest_point<T, D>(a.Sd, pos, hint, q, stk, stride);
      const T dD = fsqrt(d2D);
      if (dD < eps || k >= a.max_steps) {
        capped = !(dD < eps);
        // read g at the closest Dirichlet point (with the side rule,
        // approached from the walk's side)
        const T t = a.side && dD > T(0) ? T(1e-3) * eps / dD : T(0);
        T qr[D];
#pragma unroll
        for (int c = 0; c < D; ++c) qr[c] = fma(t, pos[c] - q[c], q[c]);
        if constexpr (sizeof(T) == 4) {
          W = field_value_f32(a.g, D, qr);
        } else {
          W = field_value(a.g, D, qr);
        }
        break;
      }
      T sil;
      if constexpr (D == 2) sil = silhouette_d2<T>(a, pos, d2D, stk, stride);
      else sil = silhouette_d2_3<T>(a, pos, d2D, stk, stride);
      const T R = fmax(fmin(dD, fsqrt(sil)), eps);
      if (neumann_data) SN += neumann_term<T, D>(a, pos, R, onb, (uint32_t)k, (uint32_t)id, tag, stk, stride);
      T w[D];
      walk_direction<T, D>(a.seed, (uint32_t)k, (uint32_t)id, a.batch, tag, w);
      T wn = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) wn += w[c] * nin[c];
      if (onb && wn < T(0)) {
#pragma unroll
        for (int c = 0; c < D; ++c) w[c] = -w[c];
      }
      int el;
      // a walk standing on a Neumann face ignores crossings closer than its
      // position's rounding (in FP32 the other face of a thin Neumann sheet
      // lies there); elsewhere every crossing beyond 1e-9 R counts
      T pabs = R;
#pragma unroll
      for (int c = 0; c < D; ++c) pabs += fabs(pos[c]);
      const T lo = (sizeof(T) == 4 && onb) ? T(1e-5) * pabs : T(1e-9) * R;
      T t;
      if constexpr (D == 2) t = neumann_hit<T>(a, pos, w, lo, R, el, stk, stride);
      else t = neumann_hit3<T>(a, pos, w, lo, R, el, stk, stride);
      if (el >= 0) {
#pragma unroll
        for (int c = 0; c < D; ++c) pos[c] = fma(t, w[c], pos[c]);
        if constexpr (D == 2) {
          const T* pr = SceneArrays<T>::prim(a.Sn);
          const T e0 = pr[4 * el + 2] - pr[4 * el], e1 = pr[4 * el + 3] - pr[4 * el + 1];
          const T len = sqrt(e0 * e0 + e1 * e1);
          nin[0] = -e1 / len;  // inward normal of a counter-clockwise boundary
          nin[1] = e0 / len;
        } else {
          T nf[3];
          face_normal<T>(a.Sn, a.Sn.prim_id[el], nf);
#pragma unroll
          for (int c = 0; c < 3; ++c) nin[c] = -nf[c];
        }
        onb = true;
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c) pos[c] = fma(R, w[c], pos[c]);
        onb = false;
      }
    }
    const double Uw = W + SN;
    ((T*)a.U)[id] = (T)Uw;
    if (a.D) {
      double dv = 0.0;
      if (a.mode == 0) {
        double xb[D], dn = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          xb[c] = a.xbar[c * a.n + i];
          if (a.side) xb[c] = fma(1e-3, a.x[c * a.n + i] - xb[c], xb[c]);
          dn += (double)nu0[c] * a.nrm[c * a.n + i];
        }
        const double cv = a.cv ? field_value(a.g, D, xb) : 0.0;
        dv = (double)D / R0 * dn * (Uw - cv);
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

// Host tables of a 3D Neumann triangle set: per triangle (original id) and
// edge k (vertex k to k + 1 mod 3) the triangle across it (-1 where the
// Neumann part ends) and a flat bit when that triangle is coplanar (unit
// normals with |n1 x n2| <= 1e-12 and n1 . n2 > 0), from the sorted list of
// edges by vertex pair.
void wost_tables3(const SceneHost& h, std::vector<int>& nb, std::vector<int>& flat) {
  const int64_t np = h.np;
  nb.assign((size_t)np * 3, -1);
  flat.assign((size_t)np, 0);
  struct Edge {
    int lo, hi, tri, k;
  };
  std::vector<Edge> E((size_t)np * 3);
  for (int64_t t = 0; t < np; ++t)
    for (int k = 0; k < 3; ++k) {
      const int a = h.P[3 * t + k], b = h.P[3 * t + (k + 1) % 3];
      E[3 * t + k] = Edge{std::min(a, b), std::max(a, b), (int)t, k};
    }
  std::sort(E.begin(), E.end(), [](const Edge& x, const Edge& y) {
    if (x.lo != y.lo) return x.lo < y.lo;
    if (x.hi != y.hi) return x.hi < y.hi;
    if (x.tri != y.tri) return x.tri < y.tri;
    return x.k < y.k;
  });
  for (size_t i = 0; i + 1 < E.size(); ++i) {
    if (E[i].lo != E[i + 1].lo || E[i].hi != E[i + 1].hi) continue;
    const Edge &e = E[i], &f = E[i + 1];
    nb[3 * (size_t)e.tri + e.k] = f.tri;
    nb[3 * (size_t)f.tri + f.k] = e.tri;
    const double* n1 = &h.fn[3 * (size_t)e.tri];
    const double* n2 = &h.fn[3 * (size_t)f.tri];
    const double c0 = n1[1] * n2[2] - n1[2] * n2[1], c1 = n1[2] * n2[0] - n1[0] * n2[2],
                 c2 = n1[0] * n2[1] - n1[1] * n2[0];
    if (std::sqrt(c0 * c0 + c1 * c1 + c2 * c2) <= 1e-12 && n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2] > 0) {
      flat[(size_t)e.tri] |= 1 << e.k;
      flat[(size_t)f.tri] |= 1 << f.k;
    }
    ++i;
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

// The walk-on-stars tables of a Neumann scene in its pinned host buffer
// (built once; later calls find them there).
int wost_host_tables(bvc_scene neu, int dim) {
  std::lock_guard<std::mutex> lock(neu->wost_mu);
  if (neu->wost_tab) return BVC_OK;
  std::vector<int> t0, t1;
  std::vector<float> cones;
  if (dim == 2) wost_tables(neu->h, t0, t1, cones);
  else wost_tables3(neu->h, t0, t1);
  const size_t b0 = (t0.size() + t1.size()) * sizeof(int), b1 = cones.size() * sizeof(float);
  void* tab = nullptr;
  int rc = check_hip(hipHostMalloc(&tab, std::max<size_t>(b0 + b1, 4), hipHostMallocDefault), "pinned tables");
  if (rc) return rc;
  std::memcpy(tab, t0.data(), t0.size() * sizeof(int));
  std::memcpy((int*)tab + t0.size(), t1.data(), t1.size() * sizeof(int));
  if (b1) std::memcpy((char*)tab + b0, cones.data(), b1);
  neu->wost_bytes[0] = b0;
  neu->wost_bytes[1] = b1;
  neu->wost_tab = tab;
  return BVC_OK;
}

}  // namespace
}  // namespace bvc

using namespace bvc;

extern "C" {

size_t bvc_wost_workspace_bytes(bvc_scene neu) {
  if (check_scene(neu)) return 0;
  // 2D: prev and flags per segment, normal cones per node; 3D: neighbours
  // (3 per triangle) and flat bits
  const size_t links = ((size_t)(4 * neu->h.np) * sizeof(int) + 255) / 256 * 256;
  return links + neu->h.child.size() * 8 * sizeof(float) + 256;
}

int bvc_wost_walks(bvc_scene dir, bvc_scene neu, const bvc_walk_params* p, int32_t mode, int64_t n, const double* x,
                   const double* nrm, const double* R0, const double* xbar, void* U, void* D, int32_t* steps,
                   void* workspace, size_t workspace_bytes, uint64_t* counters, void* stream) {
  int rc = check_scene(dir);
  if (rc) return rc;
  rc = check_scene(neu);
  if (rc) return rc;
  const int dim = dir->h.dim;
  if (neu->h.dim != dim) return fail(BVC_EINVAL, "the Dirichlet and Neumann parts must have the same dimension");
  if (!p) return fail(BVC_EINVAL, "walk params are null");
  if (p->n_dev) return fail(BVC_EUNSUPPORTED, "a device point count is taken by the cache walks only");
  if (p->order) return fail(BVC_EUNSUPPORTED, "walks on stars take no launch order");
  if (!(p->eps > 0) || p->max_steps < 1 || p->n_walks < 1) return fail(BVC_EINVAL, "bad walk parameters");
  if (p->dtype != BVC_F32 && p->dtype != BVC_F64) return fail(BVC_EINVAL, "walk dtype must be F32 or F64");
  rc = check_field(p->g, dim, "g");
  if (rc) return rc;
  rc = check_field(p->h, dim, "h");
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
  const size_t np = (size_t)neu->h.np;
  int* links = (int*)workspace;
  float4* cone_dev = (float4*)((char*)workspace + ((4 * np * sizeof(int) + 255) / 256 * 256));
  rc = wost_host_tables(neu, dim);
  if (rc) return rc;
  rc = check_hip(hipMemcpyAsync(links, neu->wost_tab, neu->wost_bytes[0], hipMemcpyHostToDevice, st), "tables upload");
  if (!rc && neu->wost_bytes[1])
    rc = check_hip(hipMemcpyAsync(cone_dev, (const char*)neu->wost_tab + neu->wost_bytes[0], neu->wost_bytes[1],
                                  hipMemcpyHostToDevice, st),
                   "tables upload");
  if (rc) return rc;
  WostArgs a{};
  a.Sd = dir->h.view();
  a.Sn = neu->h.view();
  if (dim == 2) {
    a.prev = links;
    a.flags = links + np;
    a.cones = cone_dev;
  } else {
    a.nb = links;
    a.flat = links + 3 * np;
  }
  a.g = to_dev(p->g);
  a.h = to_dev(p->h);
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
  if (dim == 2) {
    if (p->dtype == BVC_F32) hipLaunchKernelGGL((k_wost<float, 2>), dim3(blocks), dim3(kWostBlock), lds, st, a);
    else hipLaunchKernelGGL((k_wost<double, 2>), dim3(blocks), dim3(kWostBlock), lds, st, a);
  } else {
    if (p->dtype == BVC_F32) hipLaunchKernelGGL((k_wost<float, 3>), dim3(blocks), dim3(kWostBlock), lds, st, a);
    else hipLaunchKernelGGL((k_wost<double, 3>), dim3(blocks), dim3(kWostBlock), lds, st, a);
  }
  return check_hip(hipGetLastError(), "wost launch");
}

}  // extern "C"
