// Device building blocks: counter-based random numbers, samplers, closest
// points, BVH traversal, inside tests and the built-in boundary-data fields.
#pragma once

#include <hip/hip_runtime.h>

#include "bvc_internal.hpp"

namespace bvc {

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products whose halves are xored with the other counter
// words and the round key; the key advances by the Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo_a = 0xD2511F53u * c.x;
    const uint32_t hi_a = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo_b = 0xCD9E8D57u * c.z;
    const uint32_t hi_b = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Two uniforms in [0, 1) from the block (block, id, batch, tag): FP64 takes 53
// bits from two words, FP32 the top 24 bits of one word.
template <typename T>
struct Uniform;
template <>
struct Uniform<double> {
  __device__ static void pair(uint64_t seed, uint32_t block, uint32_t id, uint32_t batch,
                              uint32_t tag, double& a, double& b) {
    uint4 w = philox4x32_10(make_uint4(block, id, batch, tag), (uint32_t)seed, (uint32_t)(seed >> 32));
    a = (double)(((uint64_t)w.x << 21) | (w.y >> 11)) * 0x1.0p-53;
    b = (double)(((uint64_t)w.z << 21) | (w.w >> 11)) * 0x1.0p-53;
  }
};
template <>
struct Uniform<float> {
  __device__ static void pair(uint64_t seed, uint32_t block, uint32_t id, uint32_t batch,
                              uint32_t tag, float& a, float& b) {
    uint4 w = philox4x32_10(make_uint4(block, id, batch, tag), (uint32_t)seed, (uint32_t)(seed >> 32));
    a = (float)(w.x >> 8) * 0x1.0p-24f;
    b = (float)(w.z >> 8) * 0x1.0p-24f;
  }
};

// Angles in turns.  FP32 uses the hardware sine and cosine, which take their
// argument in turns (valid for |t| <= 256; t is a uniform in [0, 1) here).
__device__ __forceinline__ void sincos_turns(float t, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}
__device__ __forceinline__ void sincos_turns(double t, double* s, double* c) { sincospi(2.0 * t, s, c); }

// FP32 helpers use the hardware square root and reciprocal (1 ulp), not the
// correctly rounded sequences; FP64 keeps IEEE operations.
template <typename T>
__device__ __forceinline__ T fsqrt(T x) { return sqrt(x); }
template <>
__device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename T>
__device__ __forceinline__ T fdiv(T a, T b) { return a / b; }
template <>
__device__ __forceinline__ float fdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Uniform direction on the unit circle / sphere from block 4k.
template <typename T, int D>
__device__ __forceinline__ void walk_direction(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch,
                                               uint32_t tag, T* nu) {
  T ua, ub;
  Uniform<T>::pair(seed, 4u * k, id, batch, tag, ua, ub);
  if constexpr (D == 2) {
    sincos_turns(ua, &nu[1], &nu[0]);
  } else {
    T z = T(1) - T(2) * ua;
    T rho = fsqrt(fmax(T(0), T(1) - z * z));
    T s, c;
    sincos_turns(ub, &s, &c);
    nu[0] = rho * c;
    nu[1] = rho * s;
    nu[2] = z;
  }
}

// Point of B(c, R) with density proportional to |G^B(c, .)| (blocks 4k+1..3):
// radius fraction sqrt(U1 U2) in 2D, median of three uniforms in 3D.  Returns
// the radius fraction.
template <typename T, int D>
__device__ __forceinline__ T ball_source_point(uint64_t seed, uint32_t k, uint32_t id, uint32_t batch,
                                               uint32_t tag, const T* c, T R, T* y) {
  T u1, u2, u3, u4;
  Uniform<T>::pair(seed, 4u * k + 1u, id, batch, tag, u1, u2);
  Uniform<T>::pair(seed, 4u * k + 2u, id, batch, tag, u3, u4);
  if constexpr (D == 2) {
    T s = fsqrt(u1 * u2);
    T sn, cs;
    sincos_turns(u3, &sn, &cs);
    y[0] = c[0] + R * s * cs;
    y[1] = c[1] + R * s * sn;
    return s;
  } else {
    T s = fmax(fmin(u1, u2), fmin(fmax(u1, u2), u3));
    T u5, u6;
    Uniform<T>::pair(seed, 4u * k + 3u, id, batch, tag, u5, u6);
    T z = T(1) - T(2) * u5;
    T rho = fsqrt(fmax(T(0), T(1) - z * z));
    T sn, cs;
    sincos_turns(u6, &sn, &cs);
    y[0] = c[0] + R * s * rho * cs;
    y[1] = c[1] + R * s * rho * sn;
    y[2] = c[2] + R * s * z;
    return s;
  }
}

// The first ball's gradient source sample (Eq. 7 with a source): the centre
// gradient of the in-ball source term is the mean of -m(t) R yhat f(y), with
// y = c + t R yhat.  2D: t = 2 sin(asin(U)/3) (density (3/2)(1 - t^2)),
// m = 2/3, U the second uniform of block 2 and the angle of yhat the first of
// block 3 (tag); 3D: t uniform (the first uniform of block 1), m = 1 - t^3,
// yhat uniform on the sphere from block 0, both under tag | 128.  Returns t.
template <typename T, int D>
__device__ __forceinline__ T grad_source_point(uint64_t seed, uint32_t id, uint32_t batch, uint32_t tag,
                                               const T* c, T R, T* yhat, T* y, T& m) {
  if constexpr (D == 2) {
    T u1, u2, u3, u4;
    Uniform<T>::pair(seed, 2, id, batch, tag, u1, u2);
    Uniform<T>::pair(seed, 3, id, batch, tag, u3, u4);
    const T t = T(2) * sin(asin(u2) / T(3));
    sincos_turns(u3, &yhat[1], &yhat[0]);
    y[0] = fma(R * t, yhat[0], c[0]);
    y[1] = fma(R * t, yhat[1], c[1]);
    m = T(2) / T(3);
    return t;
  } else {
    T a, b, t, w;
    Uniform<T>::pair(seed, 0, id, batch, tag | 128u, a, b);
    Uniform<T>::pair(seed, 1, id, batch, tag | 128u, t, w);
    const T z = T(1) - T(2) * a;
    const T rho = fsqrt(fmax(T(0), T(1) - z * z));
    T sn, cs;
    sincos_turns(b, &sn, &cs);
    yhat[0] = rho * cs;
    yhat[1] = rho * sn;
    yhat[2] = z;
#pragma unroll
    for (int q = 0; q < 3; ++q) y[q] = fma(R * t, yhat[q], c[q]);
    m = T(1) - t * t * t;
    return t;
  }
}

// ---------------------------------------------------------------------------
// Closest points
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T segment_d2(const T* p, T ax, T ay, T bx, T by, T& cx, T& cy) {
  const T ex = bx - ax, ey = by - ay;
  const T t = fdiv((p[0] - ax) * ex + (p[1] - ay) * ey, ex * ex + ey * ey);
  if (t <= T(0)) {
    cx = ax;
    cy = ay;
  } else if (t >= T(1)) {
    cx = bx;
    cy = by;
  } else {
    cx = ax + t * ex;
    cy = ay + t * ey;
  }
  const T dx = p[0] - cx, dy = p[1] - cy;
  return dx * dx + dy * dy;
}

// Closest point of a triangle by Voronoi regions of its vertices, edges and
// face (Ericson, Real-Time Collision Detection, Sec. 5.1.5).  region: 0 face,
// 1/2/3 vertex a/b/c, 4/5/6 edge ab/bc/ca.  Every region's test is evaluated
// and the first that holds (in the order vertex a, vertex b, edge ab, vertex
// c, edge ca, edge bc, face) picks the barycentric numerators and their
// common denominator, so the wave runs one straight-line sequence with one
// reciprocal whatever region each lane's point lies in.
template <typename T>
__device__ __forceinline__ T triangle_d2(const T* p, const T* a, const T* b, const T* c, T* q, int& region) {
  T ab[3], ac[3], ap[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ab[i] = b[i] - a[i];
    ac[i] = c[i] - a[i];
    ap[i] = p[i] - a[i];
  }
  const T d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
  const T d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
  // dot products of ab and ac with p - b and p - c, from the ones above
  const T abab = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
  const T abac = ab[0] * ac[0] + ab[1] * ac[1] + ab[2] * ac[2];
  const T acac = ac[0] * ac[0] + ac[1] * ac[1] + ac[2] * ac[2];
  const T d3 = d1 - abab, d4 = d2 - abac;  // (p-b).ab, (p-b).ac
  const T d5 = d1 - abac, d6 = d2 - acac;  // (p-c).ab, (p-c).ac
  const T vc = d1 * d4 - d3 * d2;
  const T vb = d5 * d2 - d1 * d6;
  const T va = d3 * d6 - d5 * d4;
  const T e43 = d4 - d3, e56 = d5 - d6;
  const bool in_a = d1 <= T(0) && d2 <= T(0);
  const bool in_b = d3 >= T(0) && d4 <= d3;
  const bool in_ab = vc <= T(0) && d1 >= T(0) && d3 <= T(0);
  const bool in_c = d6 >= T(0) && d5 <= d6;
  const bool in_ca = vb <= T(0) && d2 >= T(0) && d6 <= T(0);
  const bool in_bc = va <= T(0) && e43 >= T(0) && e56 >= T(0);
  // q = a + (nu ab + nv ac) / den (face and edges ab, ca), q = b + nv (c - b)
  // / den (edge bc), q = the vertex itself (vertex regions); the assignments
  // run from the last test to the first so that the first test that holds wins
  int reg = 0;
  T nu = vb, nv = vc, den = va + vb + vc;
  if (in_bc) { reg = 5; nu = T(0); nv = e43; den = e43 + e56; }
  if (in_ca) { reg = 6; nu = T(0); nv = d2; den = d2 - d6; }
  if (in_c) reg = 3;
  if (in_ab) { reg = 4; nu = d1; nv = T(0); den = d1 - d3; }
  if (in_b) reg = 2;
  if (in_a) reg = 1;
  const bool vertex = reg == 1 || reg == 2 || reg == 3;
  if (vertex) { nu = T(0); nv = T(0); den = T(1); }
  const T rden = fdiv(T(1), den);
  const T u = nu * rden, v = nv * rden;
  // vertices are returned exactly when the projection clamps to them
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T qi = a[i] + u * ab[i] + v * ac[i];
    const T qbc = b[i] + v * (c[i] - b[i]);
    qi = reg == 5 ? qbc : qi;
    qi = reg == 1 ? a[i] : qi;
    qi = reg == 2 ? b[i] : qi;
    qi = reg == 3 ? c[i] : qi;
    q[i] = qi;
  }
  region = reg;
  const T dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
  return dx * dx + dy * dy + dz * dz;
}

// The same closest point for a triangle record v = (a, b, c, |b-a|^2,
// (b-a).(c-a), |c-a|^2) whose last three entries the scene builder stored:
// the region tests are those of triangle_d2, and every region's point is
// written as a + U (b - a) + V (c - a) (U, V in {0, 1} at the vertices, U =
// 1 - V on edge bc), so that p - q comes from ap with two FMAs per axis and
// no per-axis selects.  Vertices are then reached through one rounding more
// than the stored coordinates.
template <typename T>
__device__ __forceinline__ T triangle_d2_pre(const T* p, const T* v, T* q, int& region) {
  T ab[3], ac[3], ap[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ab[i] = v[3 + i] - v[i];
    ac[i] = v[6 + i] - v[i];
    ap[i] = p[i] - v[i];
  }
  const T abab = v[9], abac = v[10], acac = v[11];
  const T d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
  const T d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
  const T d3 = d1 - abab, d4 = d2 - abac;  // (p-b).ab, (p-b).ac
  const T d5 = d1 - abac, d6 = d2 - acac;  // (p-c).ab, (p-c).ac
  const T vc = d1 * d4 - d3 * d2;
  const T vb = d5 * d2 - d1 * d6;
  const T va = d3 * d6 - d5 * d4;
  const T e43 = d4 - d3, e56 = d5 - d6;
  const bool in_a = d1 <= T(0) && d2 <= T(0);
  const bool in_b = d3 >= T(0) && d4 <= d3;
  const bool in_ab = vc <= T(0) && d1 >= T(0) && d3 <= T(0);
  const bool in_c = d6 >= T(0) && d5 <= d6;
  const bool in_ca = vb <= T(0) && d2 >= T(0) && d6 <= T(0);
  const bool in_bc = va <= T(0) && e43 >= T(0) && e56 >= T(0);
  // U = nu / den, V = nv / den; the first test that holds wins
  int reg = 0;
  T nu = vb, nv = vc, den = va + vb + vc;
  if (in_bc) { reg = 5; nu = e56; nv = e43; den = e43 + e56; }
  if (in_ca) { reg = 6; nu = T(0); nv = d2; den = d2 - d6; }
  if (in_c) { reg = 3; nu = T(0); nv = T(1); den = T(1); }
  if (in_ab) { reg = 4; nu = d1; nv = T(0); den = d1 - d3; }
  if (in_b) { reg = 2; nu = T(1); nv = T(0); den = T(1); }
  if (in_a) { reg = 1; nu = T(0); nv = T(0); den = T(1); }
  const T rden = fdiv(T(1), den);
  const T U = nu * rden, V = nv * rden;
  region = reg;
  T d2s = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T e = fma(-V, ac[i], fma(-U, ab[i], ap[i]));  // p - q
    q[i] = p[i] - e;
    d2s = fma(e, e, d2s);
  }
  return d2s;
}

template <typename T, int D>
__device__ __forceinline__ T box_d2(const T* lo, const T* hi, const T* p) {
  T d2 = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const T e = fmax(fmax(lo[a] - p[a], p[a] - hi[a]), T(0));
    d2 += e * e;
  }
  return d2;
}

template <typename T>
struct SceneArrays;
template <>
struct SceneArrays<float> {
  __device__ static const float* box(const SceneDev& s) { return s.box32; }
  __device__ static const float* prim(const SceneDev& s) { return s.prim32; }
  __device__ static const float* slab(const SceneDev& s) { return s.slab32; }
};
template <>
struct SceneArrays<double> {
  __device__ static const double* box(const SceneDev& s) { return s.box64; }
  __device__ static const double* prim(const SceneDev& s) { return s.prim64; }
  __device__ static const double* slab(const SceneDev& s) { return s.slab64; }
};

// Raises the box bounds d0, d1 of the two children of a 3D node to their slab
// bounds where those are larger: the squared distance from n.p to the range
// [smin, smax] of n.y over the child's triangles bounds the squared distance
// to any of them from below.
template <typename T>
__device__ __forceinline__ void slab_bounds(const SceneDev& S, int node, const T* p, T& d0, T& d1) {
  const T* b = SceneArrays<T>::slab(S) + (size_t)node * 12;
  T w[10];
  if constexpr (sizeof(T) == 4) {
    const float4 u = reinterpret_cast<const float4*>(b)[0];
    const float4 v = reinterpret_cast<const float4*>(b)[1];
    const float2 x = reinterpret_cast<const float2*>(b)[4];
    w[0] = u.x; w[1] = u.y; w[2] = u.z; w[3] = u.w; w[4] = v.x;
    w[5] = v.y; w[6] = v.z; w[7] = v.w; w[8] = x.x; w[9] = x.y;
  } else {
#pragma unroll
    for (int j = 0; j < 10; ++j) w[j] = b[j];
  }
  const T s0 = w[0] * p[0] + w[1] * p[1] + w[2] * p[2];
  const T s1 = w[5] * p[0] + w[6] * p[1] + w[7] * p[2];
  const T e0 = fmax(fmax(w[3] - s0, s0 - w[4]), T(0));
  const T e1 = fmax(fmax(w[8] - s1, s1 - w[9]), T(0));
  d0 = fmax(d0, e0 * e0);
  d1 = fmax(d1, e1 * e1);
}

// Vertices (a, b, c) of leaf-ordered triangle i.
template <typename T>
__device__ __forceinline__ void load_triangle(const SceneDev& S, int i, T* v) {
  const T* pr = SceneArrays<T>::prim(S);
  if constexpr (sizeof(T) == 4) {
    const float4* r = reinterpret_cast<const float4*>(pr) + 3 * i;
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];
    v[0] = r0.x; v[1] = r0.y; v[2] = r0.z; v[3] = r0.w;
    v[4] = r1.x; v[5] = r1.y; v[6] = r1.z; v[7] = r1.w;
    v[8] = r2.x;
  } else {
    const double2* r = reinterpret_cast<const double2*>(pr) + 6 * i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double2 w = r[j];
      v[2 * j] = w.x;
      v[2 * j + 1] = w.y;
    }
    v[8] = r[4].x;
  }
}

// Triangle record with the three stored dot products of triangle_d2_pre.
template <typename T>
__device__ __forceinline__ void load_triangle_pre(const SceneDev& S, int i, T* v) {
  const T* pr = SceneArrays<T>::prim(S);
  if constexpr (sizeof(T) == 4) {
    const float4* r = reinterpret_cast<const float4*>(pr) + 3 * i;
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];
    v[0] = r0.x; v[1] = r0.y; v[2] = r0.z; v[3] = r0.w;
    v[4] = r1.x; v[5] = r1.y; v[6] = r1.z; v[7] = r1.w;
    v[8] = r2.x; v[9] = r2.y; v[10] = r2.z; v[11] = r2.w;
  } else {
    const double2* r = reinterpret_cast<const double2*>(pr) + 6 * i;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double2 w = r[j];
      v[2 * j] = w.x;
      v[2 * j + 1] = w.y;
    }
  }
}

// Distance^2 and closest point of leaf-ordered primitive i.
template <typename T, int D>
__device__ __forceinline__ T prim_d2(const SceneDev& S, int i, const T* p, T* q, int& region) {
  const T* pr = SceneArrays<T>::prim(S);
  if constexpr (D == 2) {
    region = 0;
    if constexpr (sizeof(T) == 4) {
      const float4 r = reinterpret_cast<const float4*>(pr)[i];
      return segment_d2<T>(p, r.x, r.y, r.z, r.w, q[0], q[1]);
    } else {
      const double2 r0 = reinterpret_cast<const double2*>(pr)[2 * i];
      const double2 r1 = reinterpret_cast<const double2*>(pr)[2 * i + 1];
      return segment_d2<T>(p, r0.x, r0.y, r1.x, r1.y, q[0], q[1]);
    }
  } else {
    T v[12];
    load_triangle_pre<T>(S, i, v);
    return triangle_d2_pre<T>(p, v, q, region);
  }
}

template <typename T, int D>
__device__ __forceinline__ void load_child_boxes(const SceneDev& S, int node, T* lo0, T* hi0, T* lo1, T* hi1) {
  const T* b = SceneArrays<T>::box(S) + (size_t)node * (4 * D);
  if constexpr (sizeof(T) == 4 && D == 2) {
    const float4 u = reinterpret_cast<const float4*>(b)[0];
    const float4 w = reinterpret_cast<const float4*>(b)[1];
    lo0[0] = u.x; lo0[1] = u.y; hi0[0] = u.z; hi0[1] = u.w;
    lo1[0] = w.x; lo1[1] = w.y; hi1[0] = w.z; hi1[1] = w.w;
  } else if constexpr (sizeof(T) == 4 && D == 3) {
    const float4 u = reinterpret_cast<const float4*>(b)[0];
    const float4 v = reinterpret_cast<const float4*>(b)[1];
    const float4 w = reinterpret_cast<const float4*>(b)[2];
    lo0[0] = u.x; lo0[1] = u.y; lo0[2] = u.z; hi0[0] = u.w; hi0[1] = v.x; hi0[2] = v.y;
    lo1[0] = v.z; lo1[1] = v.w; lo1[2] = w.x; hi1[0] = w.y; hi1[1] = w.z; hi1[2] = w.w;
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      lo0[a] = b[a];
      hi0[a] = b[D + a];
      lo1[a] = b[2 * D + a];
      hi1[a] = b[3 * D + a];
    }
  }
}

__device__ __forceinline__ float lower_bound_f32(float d) { return d; }
__device__ __forceinline__ float lower_bound_f32(double d) { return __double2float_rd(d); }

// Traversal stack entry, 32 bits: node index (17 bits) and a lower bound of
// the node's box distance^2 as the 15 non-sign bits of an FP16 number,
// obtained by truncating the FP32 mantissa (round toward zero, which for a
// non-negative value rounds down).  Values below the smallest normal FP16
// become 0 and values beyond the largest become the largest: both still
// bound the true distance from below, so pruning stays exact.
__device__ __forceinline__ uint32_t stack_entry(int node, float d2) {
  const uint32_t bits = __float_as_uint(d2);
  const int e = (int)(bits >> 23) - 127 + 15;
  uint32_t h;
  if (!(d2 > 0.0f) || e <= 0) h = 0;
  else if (e >= 31) h = 0x7BFF;
  else h = ((uint32_t)e << 10) | ((bits >> 13) & 0x3FF);
  return ((uint32_t)node << 15) | h;
}
__device__ __forceinline__ int stack_node(uint32_t s) { return (int)(s >> 15); }
__device__ __forceinline__ float stack_bound(uint32_t s) {
  const uint32_t h = s & 0x7FFF;
  if (h == 0) return 0.0f;
  return __uint_as_float(((((h >> 10) & 0x1F) - 15 + 127) << 23) | ((h & 0x3FF) << 13));
}

// Lower bound of the distance^2 from p to a triangle: distance to its box.
template <typename T>
__device__ __forceinline__ T triangle_box_d2(const T* p, const T* v) {
  T d2 = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T lo = fmin(fmin(v[a], v[3 + a]), v[6 + a]);
    const T hi = fmax(fmax(v[a], v[3 + a]), v[6 + a]);
    const T e = fmax(fmax(lo - p[a], p[a] - hi), T(0));
    d2 += e * e;
  }
  return d2;
}

// Nearest-first closest-point query over the BVH with the traversal stack in
// LDS (one 32-bit entry per level, see stack_entry).  best/bi/bq carry an
// initial candidate (bi < 0: none); the result is the minimum of
// (distance^2, original primitive id).
template <typename T, int D>
__device__ __forceinline__ void bvh_closest(const SceneDev& S, const T* p, T& best, int& bi, T* bq,
                                            uint32_t* stk, int stride) {
  auto consider = [&](int leaf) {
    const int s0 = leaf_start(leaf), n = leaf_count(leaf);
    for (int i = s0; i < s0 + n; ++i) {
      T q[D];
      int reg;
      T d2;
      if constexpr (D == 3) {
        // skip the exact test when the triangle's box is already farther
        T v[12];
        load_triangle_pre<T>(S, i, v);
        if (triangle_box_d2<T>(p, v) > best) continue;
        d2 = triangle_d2_pre<T>(p, v, q, reg);
      } else {
        d2 = prim_d2<T, D>(S, i, p, q, reg);
      }
      bool take = d2 < best;
      if (!take && d2 == best && i != bi) take = bi < 0 || S.prim_id[i] < S.prim_id[bi];
      if (take) {
        best = d2;
        bi = i;
#pragma unroll
        for (int a = 0; a < D; ++a) bq[a] = q[a];
      }
    }
  };
  int sp = 0;
  int node = 0;
  while (true) {
    T lo0[D], hi0[D], lo1[D], hi1[D];
    load_child_boxes<T, D>(S, node, lo0, hi0, lo1, hi1);
    const int2 ch = S.child[node];
    T d0 = box_d2<T, D>(lo0, hi0, p);
    T d1 = box_d2<T, D>(lo1, hi1, p);
    if constexpr (D == 3) slab_bounds<T>(S, node, p, d0, d1);
    int c0 = ch.x, c1 = ch.y;
    if (d1 < d0) {
      const T td = d0;
      d0 = d1;
      d1 = td;
      const int tc = c0;
      c0 = c1;
      c1 = tc;
    }
    int next = -1;
    if (d0 <= best) {
      if (c0 < 0) consider(c0);
      else next = c0;
    }
    if (d1 <= best) {
      if (c1 < 0) {
        consider(c1);
      } else if (next < 0) {
        next = c1;
      } else {
        stk[sp * stride] = stack_entry(c1, lower_bound_f32(d1));
        ++sp;
      }
    }
    while (next < 0 && sp > 0) {
      --sp;
      const uint32_t e = stk[sp * stride];
      if ((T)stack_bound(e) <= best) next = stack_node(e);
    }
    if (next < 0) break;
    node = next;
  }
}

// Resumable form of the same nearest-first query, for wave-interleaved
// traversal.  A step tests at most one primitive and then expands at most one
// node, so every lane of a wave runs the same instructions per step whatever
// mix of nodes and leaves its query meets, and a lane with both a pending
// primitive and an open node advances both in one step.  Leaves reached by an
// expansion wait in three pending slots (leaf encodings, 0 = empty, nearest
// first) and are consumed one primitive per step; a node is expanded only
// when at most one leaf is pending after the step's primitive, so the two
// leaves an expansion can add always fit.  The primitive is tested before the
// node so that the expansion prunes with the updated bound.  The query is
// finished when no node and no leaf remain.
template <typename T, int D>
struct Query {
  int node;       // next internal node to expand, -1 when the stack is empty
  int sp;
  int bi;
  int pa, pb, pc; // pending leaves (pa first)
  T best;
  T bq[D];
};

template <typename T, int D>
__device__ __forceinline__ bool query_open(const Query<T, D>& q) {
  return q.node >= 0 || q.pa != 0;
}

template <typename T, int D>
__device__ __forceinline__ void query_begin(const SceneDev& S, const T* p, int hint, Query<T, D>& q) {
  q.node = 0;
  q.sp = 0;
  q.pa = 0;
  q.pb = 0;
  q.pc = 0;
  q.best = T(INFINITY);
  q.bi = -1;
  if (hint >= 0) {
    int reg;
    q.best = prim_d2<T, D>(S, hint, p, q.bq, reg);
    q.bi = hint;
  }
}

template <typename T, int D>
__device__ __forceinline__ void query_push_leaf(Query<T, D>& q, int leaf) {
  if (q.pa == 0) q.pa = leaf;
  else if (q.pb == 0) q.pb = leaf;
  else q.pc = leaf;
}

template <typename T, int D>
__device__ __forceinline__ void query_step(const SceneDev& S, const T* p, Query<T, D>& q, uint32_t* stk,
                                           int stride, bool slab = true) {
  // ---- one primitive of the first pending leaf
  if (q.pa != 0) {
    const int i = leaf_start(q.pa), n = leaf_count(q.pa);
    bool test = true;
    T qq[D];
    int reg;
    T d2 = T(INFINITY);
    if constexpr (D == 3) {
      T v[12];
      load_triangle_pre<T>(S, i, v);
      // a single-primitive leaf already passed its own box; in longer
      // leaves the triangle's box is a cheap lower bound
      if (n > 1 && triangle_box_d2<T>(p, v) > q.best) test = false;
      if (test) d2 = triangle_d2_pre<T>(p, v, qq, reg);
    } else {
      d2 = prim_d2<T, D>(S, i, p, qq, reg);
    }
    if (test) {
      bool take = d2 < q.best;
      if (!take && d2 == q.best && i != q.bi) take = q.bi < 0 || S.prim_id[i] < S.prim_id[q.bi];
      if (take) {
        q.best = d2;
        q.bi = i;
#pragma unroll
        for (int a = 0; a < D; ++a) q.bq[a] = qq[a];
      }
    }
    if (n > 1) {
      q.pa = encode_leaf(i + 1, n - 1);
    } else {
      q.pa = q.pb;
      q.pb = q.pc;
      q.pc = 0;
    }
  }
  if (q.node < 0 || q.pb != 0) return;
  // ---- expand one node: leaves go to the pending slots, the nearer inner
  // child is expanded next and the farther one is pushed with its bound
  T lo0[D], hi0[D], lo1[D], hi1[D];
  load_child_boxes<T, D>(S, q.node, lo0, hi0, lo1, hi1);
  const int2 ch = S.child[q.node];
  T d0 = box_d2<T, D>(lo0, hi0, p);
  T d1 = box_d2<T, D>(lo1, hi1, p);
  if constexpr (D == 3) {
    if (slab) slab_bounds<T>(S, q.node, p, d0, d1);
  }
  int c0 = ch.x, c1 = ch.y;
  if (d1 < d0) {
    const T td = d0;
    d0 = d1;
    d1 = td;
    const int tc = c0;
    c0 = c1;
    c1 = tc;
  }
  int next = -1;
  if (d0 <= q.best) {
    if (c0 < 0) query_push_leaf(q, c0);
    else next = c0;
  }
  if (d1 <= q.best) {
    if (c1 < 0) {
      query_push_leaf(q, c1);
    } else if (next < 0) {
      next = c1;
    } else {
      stk[q.sp * stride] = stack_entry(c1, lower_bound_f32(d1));
      ++q.sp;
    }
  }
  while (next < 0 && q.sp > 0) {
    --q.sp;
    const uint32_t e = stk[q.sp * stride];
    if ((T)stack_bound(e) <= q.best) next = stack_node(e);
  }
  q.node = next;
}

// Closest point with an optional hint primitive (walk coherence: the
// previous step's closest primitive bounds the new distance from above).
template <typename T, int D>
__device__ __forceinline__ T closest_point(const SceneDev& S, const T* p, int& hint, T* q, uint32_t* stk,
                                           int stride) {
  T best = T(INFINITY);
  int bi = -1;
  if (hint >= 0) {
    int reg;
    best = prim_d2<T, D>(S, hint, p, q, reg);
    bi = hint;
  }
  bvh_closest<T, D>(S, p, best, bi, q, stk, stride);
  hint = bi;
  return best;
}

// ---------------------------------------------------------------------------
// Inside tests (FP64): 2D nonzero winding number by edge crossings, 3D sign
// of the angle-weighted pseudonormal at the closest feature.
// ---------------------------------------------------------------------------
__device__ inline int winding_number(const SceneDev& S, const double* x) {
  int wn = 0;
  for (int p = 0; p < S.np; ++p) {
    const int2 ij = reinterpret_cast<const int2*>(S.P)[p];
    const double2 a = reinterpret_cast<const double2*>(S.V)[ij.x];
    const double2 b = reinterpret_cast<const double2*>(S.V)[ij.y];
    const double cr = (b.x - a.x) * (x[1] - a.y) - (x[0] - a.x) * (b.y - a.y);
    if (a.y <= x[1]) {
      if (b.y > x[1] && cr > 0) ++wn;
    } else if (b.y <= x[1] && cr < 0) {
      --wn;
    }
  }
  return wn;
}

// The same winding number with the BVH: a segment can change it only when
// its y-range holds x[1] (the two comparisons above are exact on the same
// doubles), so children whose FP64 box misses the line y = x[1] are skipped
// and the result equals the full sum.  stk: LDS stack of depth + 1 entries
// at stride `stride`.
__device__ inline int winding_number_bvh(const SceneDev& S, const double* x, uint32_t* stk, int stride) {
  const double* pr = S.prim64;
  const double y = x[1];
  int wn = 0, sp = 0, node = 0;
  while (true) {
    const double* b = S.box64 + (size_t)node * 8;  // child 0: lo(2) hi(2), child 1: lo(2) hi(2)
    const int2 ch = S.child[node];
    const int cs[2] = {ch.x, ch.y};
    int next = -1;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!(b[4 * s + 1] <= y && b[4 * s + 3] >= y)) continue;
      const int c = cs[s];
      if (c < 0) {
        const int s0 = leaf_start(c), m = leaf_count(c);
        for (int i = s0; i < s0 + m; ++i) {
          const double ax = pr[4 * i], ay = pr[4 * i + 1], bx = pr[4 * i + 2], by = pr[4 * i + 3];
          const double cr = (bx - ax) * (y - ay) - (x[0] - ax) * (by - ay);
          if (ay <= y) {
            if (by > y && cr > 0) ++wn;
          } else if (by <= y && cr < 0) {
            --wn;
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
  return wn;
}

// 3D: x is inside when (x - q) . N < 0 for the pseudonormal N of the feature
// of original triangle t that holds the closest point q.
__device__ inline bool inside_3d(const SceneDev& S, const double* x, int t) {
  const double* A = S.V + 3 * (size_t)S.P[3 * t];
  const double* B = S.V + 3 * (size_t)S.P[3 * t + 1];
  const double* C = S.V + 3 * (size_t)S.P[3 * t + 2];
  double q[3];
  int reg;
  triangle_d2<double>(x, A, B, C, q, reg);
  const double* N;
  if (reg == 0) N = S.fn + 3 * (size_t)t;
  else if (reg <= 3) N = S.vpn + 3 * (size_t)S.P[3 * t + (reg - 1)];
  else N = S.epn + 9 * (size_t)t + 3 * (reg - 4);
  return (x[0] - q[0]) * N[0] + (x[1] - q[1]) * N[1] + (x[2] - q[2]) * N[2] < 0.0;
}

// ---------------------------------------------------------------------------
// Built-in fields, evaluated in FP64.
// ---------------------------------------------------------------------------
// Ein(z) = int_0^z (1 - e^-t)/t dt: alternating power series below 4, else
// E1(z) + ln z + gamma with E1 from its continued fraction (modified Lentz).
// Compile-time tables for the boundary-data fields: reciprocals 1/k and the
// normalisations sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) (times sqrt 2 for m > 0) of
// the real solid harmonics up to degree 16, so that the per-walk evaluation
// needs no FP64 division or square root.
constexpr double cx_sqrt(double a) {
  if (!(a > 0.0)) return 0.0;
  double x = a > 1.0 ? a : 1.0;
  for (int i = 0; i < 200; ++i) {
    const double y = 0.5 * (x + a / x);
    if (y >= x) break;  // Newton from above decreases until it stalls
    x = y;
  }
  return x;
}

struct FieldTables {
  static constexpr int kMaxL = 16;
  double inv[81];
  double sh_norm[(kMaxL + 1) * (kMaxL + 1)];
  constexpr FieldTables() : inv(), sh_norm() {
    inv[0] = 0.0;
    for (int k = 1; k < 81; ++k) inv[k] = 1.0 / k;
    for (int l = 0; l <= kMaxL; ++l)
      for (int m = 0; m <= l; ++m) {
        double ratio = 1.0;  // (l-m)!/(l+m)!
        for (int i = l - m + 1; i <= l + m; ++i) ratio /= i;
        double nrm = cx_sqrt((2 * l + 1) / (4.0 * kPi) * ratio);
        if (m > 0) nrm *= 1.4142135623730950488;
        sh_norm[l * l + l + m] = nrm;
      }
  }
};
__device__ constexpr FieldTables kFieldTables{};

__device__ inline double ein(double z) {
  if (z <= 0.0) return 0.0;
  // beyond 40, E1(z) < e^-40/40 is below half an ulp of ln z + gamma
  if (z > 40.0) return log(z) + 0.57721566490153286061;
  if (z < 4.0) {
    double term = z, sum = z;  // term_k = (-1)^{k+1} z^k / k!
    for (int k = 2; k < 80; ++k) {
      const double ik = kFieldTables.inv[k];
      term *= -z * ik;
      const double add = term * ik;
      sum += add;
      if (fabs(add) < 1e-17 * fabs(sum)) break;
    }
    return sum;
  }
  double b = z + 1.0, c = 1e300, d = 1.0 / b, h = d;
  for (int i = 1; i < 400; ++i) {
    const double an = -(double)i * i;
    b += 2.0;
    d = 1.0 / (an * d + b);
    c = b + an / c;
    const double del = c * d;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return h * exp(-z) + log(z) + 0.57721566490153286061;
}

__device__ inline double harmonic2d(double k, double alpha, double beta, const double* x) {
  double re = 1.0, im = 0.0;
  const int kk = (int)k;
  for (int i = 0; i < kk; ++i) {
    const double r2 = re * x[0] - im * x[1];
    im = re * x[1] + im * x[0];
    re = r2;
  }
  return alpha * re + beta * exp(x[0]) * cos(x[1]);
}

// Real solid harmonics r^l Y_lm from the Cartesian recurrences: for each m the
// polynomial Q_l^m(z, r^2) = r^{l-m} P_l^(m)(z/r) obeys
// (l-m) Q_l = (2l-1) z Q_{l-1} - (l+m-1) r^2 Q_{l-2}, Q_m = (2m-1)!!, and
// (x + i y)^m carries the azimuth.  If `only` >= 0, returns basis `only`.
__device__ inline double solid_harmonics(const double* coef, int L, const double* x, int only) {
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  double cm = 1.0, sm = 0.0;  // Re, Im of (x + i y)^m
  double dfact = 1.0;         // (2m-1)!!
  double total = 0.0;
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      const double c2 = cm * x[0] - sm * x[1];
      sm = cm * x[1] + sm * x[0];
      cm = c2;
      dfact *= (2 * m - 1);
    }
    double qm2 = 0.0, qm1 = 0.0;
    for (int l = m; l <= L; ++l) {
      double q;
      if (l == m) q = dfact;
      else if (l == m + 1) q = (2 * m + 1) * x[2] * dfact;
      else q = ((2 * l - 1) * x[2] * qm1 - (l + m - 1) * r2 * qm2) * kFieldTables.inv[l - m];
      qm2 = qm1;
      qm1 = q;
      const double nrm = kFieldTables.sh_norm[l * l + l + m];
      const int ic = l * l + l + m, is = l * l + l - m;
      if (only >= 0) {
        if (only == ic) return nrm * q * cm;
        if (m > 0 && only == is) return nrm * q * sm;
      } else {
        total += coef[ic] * nrm * q * cm;
        if (m > 0) total += coef[is] * nrm * q * sm;
      }
    }
  }
  return only >= 0 ? 0.0 : total;
}

// The same series in FP32 for FP32 walks: tab[l*l + l + m] holds coef times
// the normalisation (rounded once to FP32, see solid_harmonics_table), and the
// recurrences run in FP32 (relative error a few ulp per degree).
__device__ inline float solid_harmonics_f32(const float* tab, int L, const float* x) {
  const float* inv = tab + (L + 1) * (L + 1);
  const float r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  float cm = 1.0f, sm = 0.0f;
  float dfact = 1.0f;
  float total = 0.0f;
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      const float c2 = cm * x[0] - sm * x[1];
      sm = cm * x[1] + sm * x[0];
      cm = c2;
      dfact *= (float)(2 * m - 1);
    }
    float qm2 = 0.0f, qm1 = 0.0f;
    for (int l = m; l <= L; ++l) {
      float q;
      if (l == m) q = dfact;
      else if (l == m + 1) q = (float)(2 * m + 1) * x[2] * dfact;
      else q = ((float)(2 * l - 1) * x[2] * qm1 - (float)(l + m - 1) * r2 * qm2) * inv[l - m];
      qm2 = qm1;
      qm1 = q;
      const float cq = tab[l * l + l + m] * cm;
      total = fmaf(cq, q, total);
      if (m > 0) total = fmaf(tab[l * l + l - m] * sm, q, total);
    }
  }
  return total;
}

// solid_harmonics_f32 at N points at once: each table entry, read once, serves
// the N evaluations, whose recurrences run side by side.
template <int N>
__device__ inline void solid_harmonics_f32_n(const float* tab, int L, const float (*x)[3], float* out) {
  const float* inv = tab + (L + 1) * (L + 1);
  float r2[N], cm[N], sm[N], tot[N], qm1[N], qm2[N];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    r2[n] = x[n][0] * x[n][0] + x[n][1] * x[n][1] + x[n][2] * x[n][2];
    cm[n] = 1.0f;
    sm[n] = 0.0f;
    tot[n] = 0.0f;
  }
  float dfact = 1.0f;
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
#pragma unroll
      for (int n = 0; n < N; ++n) {
        const float c2 = cm[n] * x[n][0] - sm[n] * x[n][1];
        sm[n] = cm[n] * x[n][1] + sm[n] * x[n][0];
        cm[n] = c2;
      }
      dfact *= (float)(2 * m - 1);
    }
    for (int l = m; l <= L; ++l) {
      const float tc = tab[l * l + l + m], ts = tab[l * l + l - m];
      const float a1 = (float)(2 * l - 1), a2 = (float)(l + m - 1), il = inv[l - m];
      const float b1 = (float)(2 * m + 1);
#pragma unroll
      for (int n = 0; n < N; ++n) {
        float q;
        if (l == m) q = dfact;
        else if (l == m + 1) q = b1 * x[n][2] * dfact;
        else q = (a1 * x[n][2] * qm1[n] - a2 * r2[n] * qm2[n]) * il;
        qm2[n] = qm1[n];
        qm1[n] = q;
        tot[n] = fmaf(tc * cm[n], q, tot[n]);
        if (m > 0) tot[n] = fmaf(ts * sm[n], q, tot[n]);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < N; ++n) out[n] = tot[n];
}

// Fills tab[0 .. (L+1)^2 + L] for solid_harmonics_f32 (coefficient times
// normalisation, in FP64, rounded to FP32) and after them the reciprocals
// 1/j, j = 0..L, the threads of the block sharing the entries.
__device__ inline void solid_harmonics_table(const double* coef, int L, float* tab) {
  for (int j = threadIdx.x; j <= L; j += blockDim.x) tab[(L + 1) * (L + 1) + j] = (float)kFieldTables.inv[j];
  for (int k = threadIdx.x; k < (L + 1) * (L + 1); k += blockDim.x) {
    // entry l*l + l + m for |m| <= l; the normalisation depends on |m|
    int l = 0;
    while ((l + 1) * (l + 1) <= k) ++l;
    const int m = k - l * l - l;
    tab[k] = (float)(coef[k] * kFieldTables.sh_norm[l * l + l + (m < 0 ? -m : m)]);
  }
}

__device__ inline double fourier_basis(int b, double th) {
  if (b == 0) return 1.0;
  const int j = (b + 1) / 2;
  double s, c;
  sincos(j * th, &s, &c);
  return (b & 1) ? c : s;
}

__device__ inline double field_value(const FieldDev& F, int dim, const double* x) {
  const double* p = F.param;
  switch (F.kind) {
    case 0:
      return 0.0;
    case 1:
      return p[0];
    case 2:
      return harmonic2d(p[0], p[1], p[2], x);
    case 3: {
      const int ng = F.n_coef / (1 + dim);
      const double inv = 1.0 / (2.0 * p[0] * p[0]);
      double sum = 0.0;
      for (int k = 0; k < ng; ++k) {
        const double* c = F.coef + k * (1 + dim);
        double r2 = 0.0;
        for (int a = 0; a < dim; ++a) r2 += (x[a] - c[1 + a]) * (x[a] - c[1 + a]);
        sum += c[0] * exp(-r2 * inv);
      }
      return sum;
    }
    case 4: {
      const int ng = F.n_coef / 3;
      const double s2 = p[0] * p[0];
      double sum = 0.0;
      for (int k = 0; k < ng; ++k) {
        const double* c = F.coef + 3 * k;
        const double r2 = (x[0] - c[1]) * (x[0] - c[1]) + (x[1] - c[2]) * (x[1] - c[2]);
        sum += c[0] * s2 * 0.5 * ein(r2 / (2.0 * s2));
      }
      return sum + harmonic2d(p[1], p[2], p[3], x);
    }
    case 5:
      return solid_harmonics(F.coef, (int)p[0], x, -1);
    case 6: {
      const double th = atan2(x[1] - p[1], x[0] - p[0]);
      double sum = F.coef[0];
      // cos/sin(j th) by the angle-addition recurrence
      double s1, c1;
      sincos(th, &s1, &c1);
      double cj = 1.0, sj = 0.0;
      for (int b = 1; b < F.n_coef; b += 2) {
        const double cn = cj * c1 - sj * s1;
        sj = sj * c1 + cj * s1;
        cj = cn;
        sum += F.coef[b] * cj;
        if (b + 1 < F.n_coef) sum += F.coef[b + 1] * sj;
      }
      return sum;
    }
    case 7: {
      double r2 = 0.0;
      for (int a = 0; a < dim; ++a) r2 += (x[a] - p[1 + a]) * (x[a] - p[1 + a]);
      return dim == 2 ? p[0] * 0.5 * log(r2) : p[0] * rsqrt(r2);
    }
    case 8: {
      double e = 0.0;
      for (int a = 0; a < dim; ++a) e = fma(p[1 + a], x[a], e);
      return p[0] * exp(e);
    }
    case 9: {
      const double dx = x[0] - p[2], dy = x[1] - p[3];
      double phi = atan2(dy, dx);
      if (phi < 0.0) phi += 2.0 * kPi;
      return p[0] * pow(hypot(dx, dy), p[1]) * cos(p[1] * phi);
    }
    case 10: {
      double r2 = 0.0;
      for (int a = 0; a < dim; ++a) r2 += (x[a] - p[2 + a]) * (x[a] - p[2 + a]);
      return p[0] * r2 + p[1];
    }
  }
  return 0.0;
}

// FP32 evaluation of the closed-form kinds (0-4, 7, 8) for FP32 walks, whose
// Monte Carlo error is orders of magnitude above FP32 rounding; the other
// kinds, and every FP64 walk, use the FP64 field_value.
__device__ inline float ein_f32(float z) {
  if (z <= 0.0f) return 0.0f;
  if (z > 16.0f) return logf(z) + 0.5772156649f;  // E1(z) < e^-16/16, below the FP32 ulp of the rest
  if (z < 4.0f) {
    float term = z, sum = z;
    for (int k = 2; k < 40; ++k) {
      const float ik = (float)kFieldTables.inv[k];
      term *= -z * ik;
      const float add = term * ik;
      sum += add;
      if (fabsf(add) < 1e-8f * fabsf(sum)) break;
    }
    return sum;
  }
  float b = z + 1.0f, c = 1e30f, d = 1.0f / b, h = d;
  for (int i = 1; i < 100; ++i) {
    const float an = -(float)i * (float)i;
    b += 2.0f;
    d = 1.0f / fmaf(an, d, b);
    c = b + an / c;
    const float del = c * d;
    h *= del;
    if (fabsf(del - 1.0f) < 1e-7f) break;
  }
  return h * expf(-z) + logf(z) + 0.5772156649f;
}

__device__ inline float harmonic2d_f32(float k, float alpha, float beta, const float* x) {
  float re = 1.0f, im = 0.0f;
  const int kk = (int)k;
  for (int i = 0; i < kk; ++i) {
    const float r2 = re * x[0] - im * x[1];
    im = re * x[1] + im * x[0];
    re = r2;
  }
  return alpha * re + beta * expf(x[0]) * cosf(x[1]);
}

__device__ inline double field_value_f32(const FieldDev& F, int dim, const float* x) {
  const double* p = F.param;
  switch (F.kind) {
    case 0:
      return 0.0;
    case 1:
      return p[0];
    case 2:
      return (double)harmonic2d_f32((float)p[0], (float)p[1], (float)p[2], x);
    case 3: {
      const int ng = F.n_coef / (1 + dim);
      const float inv = (float)(1.0 / (2.0 * p[0] * p[0]));
      float sum = 0.0f;
      for (int k = 0; k < ng; ++k) {
        const double* c = F.coef + k * (1 + dim);
        float r2 = 0.0f;
        for (int a = 0; a < dim; ++a) {
          const float t = x[a] - (float)c[1 + a];
          r2 = fmaf(t, t, r2);
        }
        sum = fmaf((float)c[0], expf(-r2 * inv), sum);
      }
      return (double)sum;
    }
    case 4: {
      const int ng = F.n_coef / 3;
      const float s2 = (float)(p[0] * p[0]), inv = (float)(1.0 / (2.0 * p[0] * p[0]));
      float sum = 0.0f;
      for (int k = 0; k < ng; ++k) {
        const double* c = F.coef + 3 * k;
        const float dx = x[0] - (float)c[1], dy = x[1] - (float)c[2];
        sum = fmaf((float)c[0] * s2 * 0.5f, ein_f32(fmaf(dx, dx, dy * dy) * inv), sum);
      }
      return (double)(sum + harmonic2d_f32((float)p[1], (float)p[2], (float)p[3], x));
    }
    case 7: {
      float r2 = 0.0f;
      for (int a = 0; a < dim; ++a) {
        const float t = x[a] - (float)p[1 + a];
        r2 = fmaf(t, t, r2);
      }
      return dim == 2 ? p[0] * 0.5 * (double)logf(r2) : p[0] * (double)rsqrtf(r2);
    }
    case 8: {
      float e = 0.0f;
      for (int a = 0; a < dim; ++a) e = fmaf((float)p[1 + a], x[a], e);
      return p[0] * (double)expf(e);
    }
    default: {
      double xd[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < dim; ++a) xd[a] = (double)x[a];
      return field_value(F, dim, xd);
    }
  }
}

__device__ inline double basis_value(const FieldDev& F, int dim, int m, const double* x) {
  switch (F.kind) {
    case 6:
      return fourier_basis(m, atan2(x[1] - F.param[1], x[0] - F.param[0]));
    case 5:
      return solid_harmonics(nullptr, (int)F.param[0], x, m);
    default:
      return 0.0;
  }
}

// Source term in the walk's precision: Gaussian sums stay in T, everything
// else goes through the FP64 evaluator.
template <typename T, int D>
__device__ __forceinline__ T source_value(const FieldDev& F, const T* y) {
  if (F.kind == 3) {
    const int ng = F.n_coef / (1 + D);
    const T inv = T(1) / (T(2) * (T)F.param[0] * (T)F.param[0]);
    T sum = T(0);
    for (int k = 0; k < ng; ++k) {
      const double* c = F.coef + k * (1 + D);
      T r2 = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T e = y[a] - (T)c[1 + a];
        r2 += e * e;
      }
      sum += (T)c[0] * exp(-r2 * inv);
    }
    return sum;
  }
  double yd[D];
#pragma unroll
  for (int a = 0; a < D; ++a) yd[a] = (double)y[a];
  return (T)field_value(F, D, yd);
}

}  // namespace bvc
