// Bias correction of the clamped gather (Section 3.3, Eq. 8): the crossings
// of random rays with the offset boundary dR = {z inside : d(z) = l}, and the
// weighted sum of the walks started at them.
//
// dG/dn(x, z) dz is the signed solid angle dR subtends at x, so one uniform
// direction w from x and the crossings z of the ray x + t w with dR sample
// the second integral of Eq. 8 without the 1/r^(dim-1) singularity: crossing
// z contributes sign(dG/dn) max(0, 1 - c/|dG/dn(x, z)|) u(z).  Only crossings
// within the clamp radius can contribute.
//
// One thread traces one ray in FP64 over the BVH, with every node box grown
// by l: the offset pieces of a primitive (segment or face offsets at distance
// l, the circle or sphere of a vertex, the cylinder of an edge) lie within l
// of it.  A piece's crossing is a candidate when its |dG/dn| exceeds c; after
// the traversal the candidates are taken nearest first and a candidate
// belongs to dR when no boundary point is closer than l (a closest-point
// query) and it lies inside: in 3D by the pseudonormal sign at its closest
// feature, in 2D by the winding number of the ray's origin plus the signed
// crossings of the boundary segments before the candidate (each found by the
// same traversal).  Every piece is owned by exactly one primitive: a segment
// owns its start vertex's circle, a triangle owns the edges it runs from the
// lower to the higher vertex index; a vertex sphere is met from every
// triangle around the vertex and kept once.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bvc_device.hpp"

namespace bvc {
namespace {

constexpr int kRayBlock = 64;
constexpr int kCand = 16;  // candidates a ray holds (|dG/dn| > c, before the dR test)
constexpr int kCross = 16; // 2D boundary crossings a ray holds

struct RayArgs {
  SceneDev S;
  int64_t n;
  const double* x;     // [D][n]
  const int* wind;     // [n] (2D)
  double l;
  int sides;
  double c;
  double t_max;
  int n_rays;
  int max_hits;
  uint64_t seed;
  uint32_t batch;
  uint64_t slots;      // n * n_rays * max_hits
  double* slot_x;      // [D][slots] crossing points
  double* slot_R0;     // [slots] their distance to the boundary
  double* slot_xbar;   // [D][slots] their closest boundary points
  double* slot_w;      // [slots] weight; 0 marks an empty slot
  int* flags;          // [slots] 1 where a walk is needed
  unsigned long long* counters;  // [0] contributing crossings, [1] rays over capacity
};

template <int D>
__device__ __forceinline__ double dotd(const double* a, const double* b) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) s = fma(a[q], b[q], s);
  return s;
}

// Candidate list of one ray: parameter, unit outward normal of {d > l}, and a
// key that identifies a vertex sphere's root (-1 for other pieces).
template <int D>
struct Cands {
  double t[kCand];
  double nrm[kCand][D];
  int key[kCand];
  int n = 0;
  bool over = false;
};

// |dG/dn(x, x + t w)| for outward normal nv at the crossing: |n.w| / (|S| t^(D-1)).
template <int D>
__device__ __forceinline__ double dgdn_at(double t, double nw) {
  return D == 2 ? nw / (2.0 * kPi * t) : nw / (4.0 * kPi * t * t);
}

template <int D>
__device__ __forceinline__ void add_cand(Cands<D>& C, const RayArgs& a, const double* w, double t, const double* nv,
                                         int key) {
  if (!(t > 0.0 && t <= a.t_max)) return;
  const double k = dgdn_at<D>(t, dotd<D>(nv, w));
  if (!(fabs(k) > a.c)) return;
  if (key >= 0) {
    for (int i = 0; i < C.n; ++i)
      if (C.key[i] == key) return;  // the same vertex sphere met from another triangle
  }
  if (C.n == kCand) {
    C.over = true;
    return;
  }
  C.t[C.n] = t;
#pragma unroll
  for (int q = 0; q < D; ++q) C.nrm[C.n][q] = nv[q];
  C.key[C.n] = key;
  ++C.n;
}

// Roots of |x + t w - c|^2 = l^2 (|w| = 1): circle or sphere of radius l.
template <int D>
__device__ __forceinline__ void round_piece(Cands<D>& C, const RayArgs& a, const double* x, const double* w,
                                            const double* ctr, int key) {
  double qb = 0.0, qc = -a.l * a.l;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const double e = x[q] - ctr[q];
    qb = fma(w[q], e, qb);
    qc = fma(e, e, qc);
  }
  const double disc = qb * qb - qc;
  if (disc < 0.0) return;
  const double sq = sqrt(disc);
  const double ts[2] = {-qb - sq, -qb + sq};
  for (int r = 0; r < 2; ++r) {
    double nv[D];
#pragma unroll
    for (int q = 0; q < D; ++q) nv[q] = (ctr[q] - fma(ts[r], w[q], x[q])) / a.l;
    add_cand<D>(C, a, w, ts[r], nv, key < 0 ? -1 : 2 * key + r);
  }
}

// Segment (2D, leaf order i): its own crossing with the ray (for the winding
// count), its offset segments and the circle of its start vertex.
__device__ __forceinline__ void segment_pieces(Cands<2>& C, double* xt, int* xd, int& nx, bool& xover,
                                               const RayArgs& a, int i, const double* x, const double* w) {
  const double* pr = a.S.prim64 + 4 * (size_t)i;
  const double ax = pr[0], ay = pr[1], bx = pr[2], by = pr[3];
  const double e0 = bx - ax, e1 = by - ay;
  const double den = w[0] * e1 - w[1] * e0;  // cross(w, e)
  if (den != 0.0) {
    const double r0 = ax - x[0], r1 = ay - x[1];
    const double t = (r0 * e1 - r1 * e0) / den;
    const double u = (r0 * w[1] - r1 * w[0]) / den;
    if (t > 0.0 && t <= a.t_max && u >= 0.0 && u < 1.0) {
      if (nx < kCross) {
        xt[nx] = t;
        // entering the left side of a->b (the inside of a counter-clockwise
        // loop) raises the winding number by one
        xd[nx] = den < 0.0 ? 1 : -1;
        ++nx;
      } else {
        xover = true;
      }
    }
    const double len = sqrt(e0 * e0 + e1 * e1);
    const double n0 = e1 / len, n1 = -e0 / len;  // outward normal of a CCW loop
    for (int sd = 0; sd < a.sides; ++sd) {
      const double side = sd == 0 ? 1.0 : -1.0;
      const double p0 = r0 - side * a.l * n0, p1 = r1 - side * a.l * n1;
      const double to = (p0 * e1 - p1 * e0) / den;
      const double uo = (p0 * w[1] - p1 * w[0]) / den;
      if (uo >= 0.0 && uo <= 1.0) {
        const double nv[2] = {side * n0, side * n1};
        add_cand<2>(C, a, w, to, nv, -1);
      }
    }
  }
  const double ctr[2] = {ax, ay};
  round_piece<2>(C, a, x, w, ctr, -1);
}

// Triangle (3D, leaf order i): its inward offset, the cylinders of the edges
// it owns and the spheres of its vertices.
__device__ __forceinline__ void triangle_pieces(Cands<3>& C, const RayArgs& a, int i, const double* x,
                                                const double* w) {
  const int t = a.S.prim_id[i];
  int vid[3];
  double v[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vid[k] = a.S.P[3 * t + k];
#pragma unroll
    for (int q = 0; q < 3; ++q) v[k][q] = a.S.V[3 * (size_t)vid[k] + q];
  }
  double ab[3], ac[3], nn[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    ab[q] = v[1][q] - v[0][q];
    ac[q] = v[2][q] - v[0][q];
  }
  nn[0] = ab[1] * ac[2] - ab[2] * ac[1];
  nn[1] = ab[2] * ac[0] - ab[0] * ac[2];
  nn[2] = ab[0] * ac[1] - ab[1] * ac[0];
  const double ln = sqrt(dotd<3>(nn, nn));
#pragma unroll
  for (int q = 0; q < 3; ++q) nn[q] /= ln;
  {
    // inward offset triangle v0 - l n + s ab + r ac: Cramer's rule on
    // x + t w = v0 - l n + s ab + r ac (Moller and Trumbore's test)
    double pv[3], tv[3], qv[3];
    pv[0] = w[1] * ac[2] - w[2] * ac[1];
    pv[1] = w[2] * ac[0] - w[0] * ac[2];
    pv[2] = w[0] * ac[1] - w[1] * ac[0];
    const double det = dotd<3>(ab, pv);
    if (det != 0.0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) tv[q] = x[q] - (v[0][q] - a.l * nn[q]);
      const double inv = 1.0 / det;
      const double s = dotd<3>(tv, pv) * inv;
      qv[0] = tv[1] * ab[2] - tv[2] * ab[1];
      qv[1] = tv[2] * ab[0] - tv[0] * ab[2];
      qv[2] = tv[0] * ab[1] - tv[1] * ab[0];
      const double r = dotd<3>(w, qv) * inv;
      const double tt = dotd<3>(ac, qv) * inv;
      if (s >= 0.0 && r >= 0.0 && s + r <= 1.0) add_cand<3>(C, a, w, tt, nn, -1);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = k == 2 ? 0 : k + 1;
    if (vid[k] < vid[k1]) {
      // cylinder of radius l around edge v_k -> v_k1, between its end planes
      double e[3], w0[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        e[q] = v[k1][q] - v[k][q];
        w0[q] = x[q] - v[k][q];
      }
      const double L = sqrt(dotd<3>(e, e));
#pragma unroll
      for (int q = 0; q < 3; ++q) e[q] /= L;
      const double we = dotd<3>(w, e), w0e = dotd<3>(w0, e);
      double wp[3], w0p[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        wp[q] = w[q] - we * e[q];
        w0p[q] = w0[q] - w0e * e[q];
      }
      const double qa = dotd<3>(wp, wp);
      if (qa > 0.0) {
        const double qb = dotd<3>(w0p, wp), qc = dotd<3>(w0p, w0p) - a.l * a.l;
        const double disc = qb * qb - qa * qc;
        if (disc >= 0.0) {
          const double sq = sqrt(disc);
          const double ts[2] = {(-qb - sq) / qa, (-qb + sq) / qa};
          for (int r = 0; r < 2; ++r) {
            const double along = (w0e + ts[r] * we) / L;
            if (!(along >= 0.0 && along <= 1.0)) continue;
            double nv[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) nv[q] = -(w0p[q] + ts[r] * wp[q]) / a.l;
            add_cand<3>(C, a, w, ts[r], nv, -1);
          }
        }
      }
    }
    round_piece<3>(C, a, x, w, v[k], vid[k]);
  }
}

// Ray against a box grown by l, for t in [0, t_max].
template <int D>
__device__ __forceinline__ bool ray_box(const double* lo, const double* hi, const double* x, const double* w,
                                        double l, double t_max) {
  double t0 = 0.0, t1 = t_max;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const double a0 = lo[q] - l - x[q], a1 = hi[q] + l - x[q];
    if (w[q] == 0.0) {
      if (a0 > 0.0 || a1 < 0.0) return false;
      continue;
    }
    const double inv = 1.0 / w[q];
    double ta = a0 * inv, tb = a1 * inv;
    if (ta > tb) {
      const double s = ta;
      ta = tb;
      tb = s;
    }
    t0 = fmax(t0, ta);
    t1 = fmin(t1, tb);
  }
  return t0 <= t1;
}

template <int D>
__global__ __launch_bounds__(kRayBlock) void k_ray_hits(RayArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t* stk = lds + threadIdx.x;
  const int stride = blockDim.x;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = g < (uint64_t)a.n * (uint64_t)a.n_rays;
  unsigned long long found = 0, over = 0;
  if (live) {
    const int64_t k = (int64_t)(g / (uint64_t)a.n_rays);
    const int j = (int)(g % (uint64_t)a.n_rays);
    double x[D], w[D];
#pragma unroll
    for (int q = 0; q < D; ++q) x[q] = a.x[q * a.n + k];
    double ua, ub;
    Uniform<double>::pair(a.seed, (uint32_t)j, (uint32_t)k, a.batch, 5, ua, ub);
    if constexpr (D == 2) {
      sincospi(2.0 * ua, &w[1], &w[0]);
    } else {
      const double zz = 1.0 - 2.0 * ua;
      const double rho = sqrt(fmax(0.0, 1.0 - zz * zz));
      double sn, cs;
      sincospi(2.0 * ub, &sn, &cs);
      w[0] = rho * cs;
      w[1] = rho * sn;
      w[2] = zz;
    }
    Cands<D> C;
    double xt[D == 2 ? kCross : 1];
    int xd[D == 2 ? kCross : 1];
    int nx = 0;
    bool xover = false;
    // any-order traversal of the grown boxes
    int sp = 0, node = 0;
    while (true) {
      double lo0[D], hi0[D], lo1[D], hi1[D];
      load_child_boxes<double, D>(a.S, node, lo0, hi0, lo1, hi1);
      const int2 ch = a.S.child[node];
      int next = -1;
      const int cs[2] = {ch.x, ch.y};
      const bool hit[2] = {ray_box<D>(lo0, hi0, x, w, a.l, a.t_max), ray_box<D>(lo1, hi1, x, w, a.l, a.t_max)};
      for (int s = 0; s < 2; ++s) {
        if (!hit[s]) continue;
        const int cc = cs[s];
        if (cc < 0) {
          const int s0 = leaf_start(cc), m = leaf_count(cc);
          for (int i = s0; i < s0 + m; ++i) {
            if constexpr (D == 2) segment_pieces(C, xt, xd, nx, xover, a, i, x, w);
            else triangle_pieces(C, a, i, x, w);
          }
        } else if (next < 0) {
          next = cc;
        } else {
          stk[sp * stride] = (uint32_t)cc;
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
    // candidates nearest first (insertion sort keeps equal t in list order)
    for (int i = 1; i < C.n; ++i) {
      for (int m = i; m > 0 && C.t[m - 1] > C.t[m]; --m) {
        const double tt = C.t[m];
        C.t[m] = C.t[m - 1];
        C.t[m - 1] = tt;
        const int kk = C.key[m];
        C.key[m] = C.key[m - 1];
        C.key[m - 1] = kk;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const double nq = C.nrm[m][q];
          C.nrm[m][q] = C.nrm[m - 1][q];
          C.nrm[m - 1][q] = nq;
        }
      }
    }
    const uint64_t base = ((uint64_t)k * a.n_rays + j) * a.max_hits;
    int h = 0;
    bool more = C.over || xover;
    for (int i = 0; i < C.n; ++i) {
      double z[D];
#pragma unroll
      for (int q = 0; q < D; ++q) z[q] = fma(C.t[i], w[q], x[q]);
      double qz[D];
      int hint = -1;
      const double d = sqrt(closest_point<double, D>(a.S, z, hint, qz, stk, stride));
      if (!(d >= a.l * (1.0 - 1e-9))) continue;
      bool in;
      if constexpr (D == 2) {
        int wn = a.wind[k];
        for (int m = 0; m < nx; ++m)
          if (xt[m] < C.t[i]) wn += xd[m];
        in = wn != 0;
      } else {
        in = inside_3d(a.S, z, a.S.prim_id[hint]);
      }
      if (!in) continue;
      ++found;
      if (h >= a.max_hits) {
        more = true;
        continue;
      }
      const double kv = dgdn_at<D>(C.t[i], dotd<D>(C.nrm[i], w));
      const uint64_t s = base + h;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        a.slot_x[q * a.slots + s] = z[q];
        a.slot_xbar[q * a.slots + s] = qz[q];
      }
      a.slot_R0[s] = d;
      a.slot_w[s] = (kv > 0.0 ? 1.0 : -1.0) * (1.0 - a.c / fabs(kv));
      a.flags[s] = 1;
      ++h;
    }
    for (; h < a.max_hits; ++h) {
      a.slot_w[base + h] = 0.0;
      a.flags[base + h] = 0;
    }
    over = more ? 1ull : 0ull;
  }
  for (int off = 32; off > 0; off >>= 1) {
    found += __shfl_xor(found, off);
    over += __shfl_xor(over, off);
  }
  if ((threadIdx.x & 63) == 0 && (found || over)) {
    atomicAdd(&a.counters[0], found);
    atomicAdd(&a.counters[1], over);
  }
}

__global__ __launch_bounds__(256) void k_point_winding(SceneDev S, int64_t n, const double* x, int* wind) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double p[2] = {x[k], x[n + k]};
  wind[k] = winding_number(S, p);
}

// corr_k = (1/n_rays) sum over the slots of point k of weight * u(z), with
// u(z) = g(exit) + the walk's source terms, in FP64; added to u[out[k]].
// One wave per point: lane l reads slots l, l + 64, ... of the point's
// contiguous run (coalesced), then a shuffle tree sums the lanes.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_corr_sum(FieldDev g, int64_t n, int per, int n_rays, uint64_t slots,
                                                  const double* slot_w, const T* EX, const T* U, const int64_t* out,
                                                  T* u) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (k >= n) return;
  double acc = 0.0;
  for (int m = lane; m < per; m += 64) {
    const uint64_t s = (uint64_t)k * per + m;
    const double wv = slot_w[s];
    if (wv == 0.0) continue;
    double q[D];
#pragma unroll
    for (int e = 0; e < D; ++e) q[e] = (double)EX[(size_t)e * slots + s];
    acc += wv * (field_value(g, D, q) + (double)U[s]);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    const int64_t o = out ? out[k] : k;
    u[o] = (T)((double)u[o] + acc / n_rays);
  }
}

}  // namespace

int launch_ray_hits(const SceneHost& h, int64_t n, const double* x, const int* wind, double l, int sides, double c,
                    double t_max, int n_rays, int max_hits, uint64_t seed, uint32_t batch, double* slot_x,
                    double* slot_R0, double* slot_xbar, double* slot_w, int* flags, unsigned long long* counters,
                    hipStream_t st) {
  RayArgs a{};
  a.S = h.view();
  a.n = n;
  a.x = x;
  a.wind = wind;
  a.l = l;
  a.sides = sides;
  a.c = c;
  a.t_max = t_max;
  a.n_rays = n_rays;
  a.max_hits = max_hits;
  a.seed = seed;
  a.batch = batch;
  a.slots = (uint64_t)n * n_rays * max_hits;
  a.slot_x = slot_x;
  a.slot_R0 = slot_R0;
  a.slot_xbar = slot_xbar;
  a.slot_w = slot_w;
  a.flags = flags;
  a.counters = counters;
  const uint64_t rays = (uint64_t)n * n_rays;
  const int blocks = (int)((rays + kRayBlock - 1) / kRayBlock);
  const size_t lds = (size_t)(h.depth + 2) * kRayBlock * sizeof(uint32_t);
  if (blocks == 0) return BVC_OK;
  if (h.dim == 2) hipLaunchKernelGGL(k_ray_hits<2>, dim3(blocks), dim3(kRayBlock), lds, st, a);
  else hipLaunchKernelGGL(k_ray_hits<3>, dim3(blocks), dim3(kRayBlock), lds, st, a);
  return check_hip(hipGetLastError(), "ray hits launch");
}

int launch_point_winding(const SceneHost& h, int64_t n, const double* x, int* wind, hipStream_t st) {
  if (n == 0) return BVC_OK;
  const int blocks = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_point_winding, dim3(blocks), dim3(256), 0, st, h.view(), n, x, wind);
  return check_hip(hipGetLastError(), "winding launch");
}

int launch_corr_sum(const bvc_field& g, int dim, int dtype, int64_t n, int n_rays, int max_hits,
                    const double* slot_w, const void* EX, const void* U, const int64_t* out, void* u,
                    hipStream_t st) {
  if (n == 0) return BVC_OK;
  const int blocks = (int)((n + 3) / 4);  // four waves (points) per block
  const uint64_t slots = (uint64_t)n * n_rays * max_hits;
  const int per = n_rays * max_hits;
  const FieldDev gd = to_dev(g);
  if (dtype == BVC_F32) {
    if (dim == 2)
      hipLaunchKernelGGL((k_corr_sum<float, 2>), dim3(blocks), dim3(256), 0, st, gd, n, per, n_rays, slots, slot_w,
                         (const float*)EX, (const float*)U, out, (float*)u);
    else
      hipLaunchKernelGGL((k_corr_sum<float, 3>), dim3(blocks), dim3(256), 0, st, gd, n, per, n_rays, slots, slot_w,
                         (const float*)EX, (const float*)U, out, (float*)u);
  } else {
    if (dim == 2)
      hipLaunchKernelGGL((k_corr_sum<double, 2>), dim3(blocks), dim3(256), 0, st, gd, n, per, n_rays, slots,
                         slot_w, (const double*)EX, (const double*)U, out, (double*)u);
    else
      hipLaunchKernelGGL((k_corr_sum<double, 3>), dim3(blocks), dim3(256), 0, st, gd, n, per, n_rays, slots,
                         slot_w, (const double*)EX, (const double*)U, out, (double*)u);
  }
  return check_hip(hipGetLastError(), "correction sum launch");
}

}  // namespace bvc
