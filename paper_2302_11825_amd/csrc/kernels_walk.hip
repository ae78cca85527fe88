// Sampling, classification, compaction and walk-on-spheres kernels with their
// C-ABI entry points.
//
// Walks run in a persistent kernel: each wave takes walk ids from a global
// queue, one id per idle lane, so a lane whose walk ended starts the next one
// at the following iteration instead of idling until the longest walk of its
// wave is done.  A walk's random numbers depend only on (seed, batch, id), so
// results do not depend on which lane ran it.  Each walk writes its own
// sample; cache means are reduced afterwards in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "bvc_device.hpp"

namespace bvc {

int ensure_cdf(SceneHost& S, double l, int sides, hipStream_t stream);
double candidate_measure(const SceneHost& S, double l, int sides);

namespace {

constexpr int kBlock = 256;

inline size_t stack_bytes(const SceneHost& h, int block) {
  return (size_t)(h.depth + 1) * block * sizeof(uint32_t);
}

}  // namespace

int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) n = p.multiProcessorCount;
    if (n <= 0) n = 256;
  }
  return n;
}

namespace {
__global__ void k_zero_words(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}
}  // namespace

int zero_async(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return BVC_OK;
  if (!p || bytes % 4) return fail(BVC_EINVAL, "zero_async needs a non-null pointer and a multiple of 4 bytes");
  const size_t n = bytes / 4;
  const int blocks = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(kBlock), 0, st, (uint32_t*)p, n);
  return check_hip(hipGetLastError(), "zero launch");
}

namespace {

// ---------------------------------------------------------------------------
// Cache sampling
// ---------------------------------------------------------------------------
// A cache point's xbar is its closest boundary point, where the control
// variate c = g(xbar) of its walks reads the data (the walks' side rule for
// double-sided data moves that read point towards the cache point).
__device__ void candidate_point(const SceneDev& S, int e, double r, double v, double l, double* x) {
  if (S.dim == 2) {
    const int ns = S.np * S.sides;
    if (e < ns) {
      const int p = e / S.sides;
      const double side = (e % S.sides == 0) ? 1.0 : -1.0;
      const double* a = S.V + 2 * (size_t)S.P[2 * p];
      const double* b = S.V + 2 * (size_t)S.P[2 * p + 1];
      const double t0 = b[0] - a[0], t1 = b[1] - a[1];
      const double len = sqrt(t0 * t0 + t1 * t1);
      const double n0 = t1 / len, n1 = -t0 / len;  // outward normal of a CCW polygon
      x[0] = (a[0] + r * t0) - side * l * n0;
      x[1] = (a[1] + r * t1) - side * l * n1;
    } else {
      const double* c = S.V + 2 * (size_t)(e - ns);
      double s, cs;
      sincos(2 * kPi * r, &s, &cs);
      x[0] = c[0] + l * cs;
      x[1] = c[1] + l * s;
    }
    return;
  }
  if (e < S.np) {
    const double* A = S.V + 3 * (size_t)S.P[3 * e];
    const double* B = S.V + 3 * (size_t)S.P[3 * e + 1];
    const double* C = S.V + 3 * (size_t)S.P[3 * e + 2];
    const double su = sqrt(r);
    const double b0 = 1 - su, b1 = su * (1 - v), b2 = su * v;
    double ab[3], ac[3];
    for (int a = 0; a < 3; ++a) {
      ab[a] = B[a] - A[a];
      ac[a] = C[a] - A[a];
    }
    const double nn[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2],
                          ab[0] * ac[1] - ab[1] * ac[0]};
    const double len = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    for (int a = 0; a < 3; ++a) x[a] = b0 * A[a] + b1 * B[a] + b2 * C[a] - l * nn[a] / len;
  } else if (e < S.np + S.ne) {
    const int q = e - S.np;
    const double* A = S.V + 3 * (size_t)S.E[2 * q];
    const double* B = S.V + 3 * (size_t)S.E[2 * q + 1];
    double t[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double len = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int a = 0; a < 3; ++a) t[a] /= len;
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (fabs(t[a]) < fabs(t[ax])) ax = a;
    double h[3] = {0, 0, 0};
    h[ax] = 1;
    double e1[3] = {t[1] * h[2] - t[2] * h[1], t[2] * h[0] - t[0] * h[2], t[0] * h[1] - t[1] * h[0]};
    const double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int a = 0; a < 3; ++a) e1[a] /= l1;
    const double e2[3] = {t[1] * e1[2] - t[2] * e1[1], t[2] * e1[0] - t[0] * e1[2],
                          t[0] * e1[1] - t[1] * e1[0]};
    double s, cs;
    sincos(2 * kPi * v, &s, &cs);
    for (int a = 0; a < 3; ++a) x[a] = A[a] + r * (B[a] - A[a]) + l * (cs * e1[a] + s * e2[a]);
  } else {
    const double* c = S.V + 3 * (size_t)(e - S.np - S.ne);
    const double z = 1 - 2 * r;
    const double rho = sqrt(fmax(0.0, 1 - z * z));
    double s, cs;
    sincos(2 * kPi * v, &s, &cs);
    x[0] = c[0] + l * rho * cs;
    x[1] = c[1] + l * rho * s;
    x[2] = c[2] + l * z;
  }
}

template <int D>
__device__ bool inside_point(const SceneDev& S, const double* x, int leaf_prim, uint32_t* stk, int stride) {
  if constexpr (D == 2) return winding_number_bvh(S, x, stk, stride) != 0;
  else return inside_3d(S, x, S.prim_id[leaf_prim]);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sample_cache(SceneDev S, int64_t n, double l, uint64_t seed,
                                                          uint32_t batch, double M, double* x, double* nrm,
                                                          double* w, double* xbar, double* R0, int* acc) {
  extern __shared__ uint32_t lds[];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double ua, ub;
  Uniform<double>::pair(seed, 0, (uint32_t)k, batch, 3, ua, ub);
  const double target = ((double)k + ua) / (double)n * M;
  int lo = 0, hi = S.n_el - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (S.cdf[mid] <= target) lo = mid;
    else hi = mid - 1;
  }
  double r = (target - S.cdf[lo]) / S.meas[lo];
  r = fmin(fmax(r, 0.0), 1.0);
  double xc[D];
  candidate_point(S, lo, r, ub, l, xc);
  double q[D];
  int hint = -1;
  const double d = sqrt(closest_point<double, D>(S, xc, hint, q, lds + threadIdx.x, blockDim.x));
  const bool ok = d >= l * (1 - 1e-9) && inside_point<D>(S, xc, hint, lds + threadIdx.x, blockDim.x);
  acc[k] = ok ? 1 : 0;
  R0[k] = d;
  w[k] = M / (double)n;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    x[a * n + k] = xc[a];
    xbar[a * n + k] = q[a];
    nrm[a * n + k] = (q[a] - xc[a]) / d;
  }
}

// Cache points on the closed boundary of a region of interest R inside the
// domain (Section 3.2, "Boundary Specification"): uniform density 1/|dR|,
// stratified uniforms (k + U_k)/n through the region's primitive measures
// (its sampling table at l = 0 holds the segments or faces; the zero-measure
// vertex and edge entries after them are never reached), the primitive's own
// outward normal, and the distance and closest point on the domain boundary
// where the walks run.  A point is accepted when it lies strictly inside the
// domain.
template <int D>
__global__ __launch_bounds__(kBlock) void k_sample_roi(SceneDev Sd, SceneDev Sr, int64_t n, uint64_t seed,
                                                        uint32_t batch, double M, double* x, double* nrm, double* w,
                                                        double* xbar, double* R0, int* acc) {
  extern __shared__ uint32_t lds[];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double ua, ub;
  Uniform<double>::pair(seed, 0, (uint32_t)k, batch, 6, ua, ub);
  const double target = ((double)k + ua) / (double)n * M;
  int lo = 0, hi = Sr.np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (Sr.cdf[mid] <= target) lo = mid;
    else hi = mid - 1;
  }
  const double r = fmin(fmax((target - Sr.cdf[lo]) / Sr.meas[lo], 0.0), 1.0);
  double xc[D], nc[D];
  if constexpr (D == 2) {
    const double* a = Sr.V + 2 * (size_t)Sr.P[2 * lo];
    const double* b = Sr.V + 2 * (size_t)Sr.P[2 * lo + 1];
    const double t0 = b[0] - a[0], t1 = b[1] - a[1];
    const double len = sqrt(t0 * t0 + t1 * t1);
    xc[0] = a[0] + r * t0;
    xc[1] = a[1] + r * t1;
    nc[0] = t1 / len;  // outward normal of a CCW loop
    nc[1] = -t0 / len;
  } else {
    const double* A = Sr.V + 3 * (size_t)Sr.P[3 * lo];
    const double* Bv = Sr.V + 3 * (size_t)Sr.P[3 * lo + 1];
    const double* C = Sr.V + 3 * (size_t)Sr.P[3 * lo + 2];
    const double su = sqrt(r);
    const double b0 = 1 - su, b1 = su * (1 - ub), b2 = su * ub;
    double ab[3], ac[3];
    for (int q = 0; q < 3; ++q) {
      ab[q] = Bv[q] - A[q];
      ac[q] = C[q] - A[q];
      xc[q] = b0 * A[q] + b1 * Bv[q] + b2 * C[q];
    }
    const double cr[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2],
                          ab[0] * ac[1] - ab[1] * ac[0]};
    const double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int q = 0; q < 3; ++q) nc[q] = cr[q] / len;
  }
  double q[D];
  int hint = -1;
  const double d = sqrt(closest_point<double, D>(Sd, xc, hint, q, lds + threadIdx.x, blockDim.x));
  acc[k] = (d > 0.0 && inside_point<D>(Sd, xc, hint, lds + threadIdx.x, blockDim.x)) ? 1 : 0;
  R0[k] = d;
  w[k] = M / (double)n;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    x[a * n + k] = xc[a];
    nrm[a * n + k] = nc[a];
    xbar[a * n + k] = q[a];
  }
}

// Cache points for a 2D boundary with a Neumann part (Section 3.2, "Boundary
// Specification"): the closed curve made of the offset Dirichlet boundary
// (points at distance l from the Dirichlet part, inside the domain) and the
// Neumann part farther than l from the Dirichlet part.  One stratified draw
// over the Dirichlet offset candidates (segment offsets and vertex circles of
// the Dirichlet scene's table at (l, 1 side)) followed by the Neumann
// segments (their table at l = 0).  Offset points take the normal towards the
// closest Dirichlet point, Neumann points the segment's outward normal.
__global__ __launch_bounds__(kBlock) void k_sample_mixed(SceneDev Sf, SceneDev Sd, SceneDev Sn, int64_t n, double l,
                                                          double jdrop, uint64_t seed, uint32_t batch, double MD,
                                                          double M,
                                                          double* x, double* nrm, double* w, double* xbar,
                                                          double* R0, int* kind) {
  extern __shared__ uint32_t lds[];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double ua, ub;
  Uniform<double>::pair(seed, 0, (uint32_t)k, batch, 7, ua, ub);
  const double target = ((double)k + ua) / (double)n * M;
  double xc[2], nc[2], q[2];
  bool ok;
  int ty;  // 1 offset Dirichlet candidate, 2 Neumann candidate
  int hint = -1;
  if (target < MD) {
    int lo = 0, hi = Sd.n_el - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (Sd.cdf[mid] <= target) lo = mid;
      else hi = mid - 1;
    }
    const double r = fmin(fmax((target - Sd.cdf[lo]) / Sd.meas[lo], 0.0), 1.0);
    candidate_point(Sd, lo, r, ub, l, xc);
    const double d = sqrt(closest_point<double, 2>(Sd, xc, hint, q, lds + threadIdx.x, blockDim.x));
    nc[0] = (q[0] - xc[0]) / d;
    nc[1] = (q[1] - xc[1]) / d;
    ok = fabs(d - l) <= 1e-9 * l && winding_number_bvh(Sf, xc, lds + threadIdx.x, blockDim.x) != 0;
    ty = 1;
  } else {
    const double t2 = target - MD;
    int lo = 0, hi = Sn.np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (Sn.cdf[mid] <= t2) lo = mid;
      else hi = mid - 1;
    }
    const double* a = Sn.V + 2 * (size_t)Sn.P[2 * lo];
    const double* b = Sn.V + 2 * (size_t)Sn.P[2 * lo + 1];
    const double e0 = b[0] - a[0], e1 = b[1] - a[1];
    const double len = sqrt(e0 * e0 + e1 * e1);
    const double r = fmin(fmax((t2 - Sn.cdf[lo]) / len, 0.0), 1.0);
    xc[0] = a[0] + r * e0;
    xc[1] = a[1] + r * e1;
    nc[0] = e1 / len;  // outward normal of a CCW loop
    nc[1] = -e0 / len;
    const double d = sqrt(closest_point<double, 2>(Sd, xc, hint, q, lds + threadIdx.x, blockDim.x));
    ok = d > l;
    ty = 2;
  }
  double qf[2];
  int hf = -1;
  const double dF = sqrt(closest_point<double, 2>(Sf, xc, hf, qf, lds + threadIdx.x, blockDim.x));
  // optional junction drop: an offset point closer than jdrop * l to the
  // Neumann part is rejected (its first ball, no larger than that distance,
  // gives the Eq. 7 estimate a variance growing like (l / R0)^2)
  if (ty == 1 && dF < jdrop * l) ok = false;
  R0[k] = dF;
  kind[k] = ok ? ty : 0;
  w[k] = M / (double)n;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    x[a * n + k] = xc[a];
    nrm[a * n + k] = nc[a];
    xbar[a * n + k] = q[a];
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sample_sources(SceneDev S, FieldDev f, int64_t m, int64_t M, double lo0,
                                                            double lo1, double lo2, double hi0, double hi1,
                                                            double hi2, double l, uint64_t seed, uint32_t batch,
                                                            double* y, double* s) {
  extern __shared__ uint32_t lds[];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double u[4];
  Uniform<double>::pair(seed, 0, (uint32_t)j, batch, 4, u[0], u[1]);
  Uniform<double>::pair(seed, 1, (uint32_t)j, batch, 4, u[2], u[3]);
  const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
  double yj[D];
  int64_t rem = j;
  double vol = 1.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int64_t c = rem % m;
    rem /= m;
    yj[a] = lo[a] + ((double)c + u[a]) / (double)m * (hi[a] - lo[a]);
    vol *= hi[a] - lo[a];
    y[a * M + j] = yj[a];
  }
  double q[D];
  int hint = -1;
  const double d = sqrt(closest_point<double, D>(S, yj, hint, q, lds + threadIdx.x, blockDim.x));
  const bool in = inside_point<D>(S, yj, hint, lds + threadIdx.x, blockDim.x) && d > l;
  s[j] = in ? vol / (double)M * field_value(f, D, yj) : 0.0;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_classify(SceneDev S, int64_t n, const double* x, double l, int* cls,
                                                      double* dist) {
  extern __shared__ uint32_t lds[];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double xk[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xk[a] = x[a * n + k];
  double q[D];
  int hint = -1;
  const double d = sqrt(closest_point<double, D>(S, xk, hint, q, lds + threadIdx.x, blockDim.x));
  const bool in = inside_point<D>(S, xk, hint, lds + threadIdx.x, blockDim.x);
  cls[k] = !in ? 0 : (d > l ? 1 : 2);
  if (dist) dist[k] = d;
}

// Evaluation points of a 2D domain with a Neumann part: inside the whole
// boundary `Sf`, split by the distance to the Dirichlet part `Sd` (Section
// 3.2: the gather applies farther than l, walks on stars within l).
__global__ __launch_bounds__(kBlock) void k_classify_mixed(SceneDev Sf, SceneDev Sd, int64_t n, const double* x,
                                                            double l, int* cls, double* dist) {
  extern __shared__ uint32_t lds[];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double xk[2] = {x[k], x[n + k]};
  double q[2];
  int hint = -1;
  const double d = sqrt(closest_point<double, 2>(Sd, xk, hint, q, lds + threadIdx.x, blockDim.x));
  const bool in = winding_number_bvh(Sf, xk, lds + threadIdx.x, blockDim.x) != 0;
  cls[k] = !in ? 0 : (d > l ? 1 : 2);
  if (dist) dist[k] = d;
}

// ---------------------------------------------------------------------------
// Deterministic compaction: per-block counts, one-block scan, scatter.
// ---------------------------------------------------------------------------
constexpr int kCompactItems = 4;  // items per thread
constexpr int kCompactTile = kBlock * kCompactItems;

__global__ __launch_bounds__(kBlock) void k_compact_count(int64_t n, const int* flags, int want, int* counts) {
  __shared__ int part[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kCompactTile;
  int c = 0;
  for (int i = 0; i < kCompactItems; ++i) {
    const int64_t k = base + (int64_t)i * kBlock + threadIdx.x;
    c += (k < n && flags[k] == want) ? 1 : 0;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int wv = 0; wv < kBlock / 64; ++wv) t += part[wv];
    counts[blockIdx.x] = t;
  }
}

__global__ void k_compact_scan(int nb, int* counts, int64_t* total) {
  // single block: sequential chunks with a block-wide scan per chunk
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? counts[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) counts[i] = carry + buf[threadIdx.x] - v;  // exclusive
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(int64_t n, const int* flags, int want,
                                                             const int* offsets, int* idx) {
  __shared__ int wave_tot[kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int run = offsets[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kCompactTile;
  for (int i = 0; i < kCompactItems; ++i) {
    const int64_t k = base + (int64_t)i * kBlock + threadIdx.x;
    const bool f = k < n && flags[k] == want;
    const uint64_t m = __ballot(f);
    if (lane == 0) wave_tot[wv] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int q = 0; q < wv; ++q) before += wave_tot[q];
    if (f) idx[run + before + __popcll(m & ((1ull << lane) - 1))] = (int)k;
    int tot = 0;
    for (int q = 0; q < kBlock / 64; ++q) tot += wave_tot[q];
    __syncthreads();
    run += tot;
  }
}

template <typename Ti, typename To>
__global__ void k_take(int64_t n_idx, const int64_t* count, const int* idx, int rows, int64_t ld_in, const Ti* in,
                       int64_t ld_out, To* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // a device-resident count bounds the entries (the rest stay untouched)
  const int64_t n = count ? std::min<int64_t>(n_idx, *count) : n_idx;
  if (q >= n) return;
  const int64_t src = idx ? idx[q] : q;
  for (int r = 0; r < rows; ++r) out[r * ld_out + q] = (To)in[r * ld_in + src];
}

template <typename T>
__global__ void k_scatter(int64_t n_idx, const int* idx, int rows, int64_t ld_in, const T* in, int64_t ld_out,
                          T* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_idx) return;
  for (int r = 0; r < rows; ++r) out[r * ld_out + idx[q]] = in[r * ld_in + q];
}

// ---------------------------------------------------------------------------
// Launch order by position: a counting sort of the points by the Morton index
// of their grid cell (32^3 cells in 3D, 256^2 in 2D, 2^15 or 2^16 buckets)
// ---------------------------------------------------------------------------
constexpr int kOrderBuckets = 1 << 16;

struct OrderGrid {
  double lo[3], scale[3];  // cell coordinate = (x - lo) * scale
  int bits;                // per axis
};

template <typename T>
__device__ __forceinline__ uint32_t order_key(const OrderGrid& g, int dim, const T* x, int64_t ld, int64_t i) {
  const double top = (double)((1 << g.bits) - 1);
  uint32_t c[3] = {0u, 0u, 0u};
  for (int a = 0; a < dim; ++a) {
    double t = ((double)x[a * ld + i] - g.lo[a]) * g.scale[a];
    t = t >= 0.0 ? (t <= top ? t : top) : 0.0;  // NaN lands in cell 0
    c[a] = (uint32_t)t;
  }
  uint32_t key = 0u;
  for (int b = 0; b < g.bits; ++b)
    for (int a = 0; a < dim; ++a) key |= ((c[a] >> b) & 1u) << (b * dim + a);
  return key;
}

__device__ __forceinline__ int64_t order_live(int64_t n, const int64_t* n_dev) {
  if (!n_dev) return n;
  const int64_t c = *n_dev;
  return c < 0 ? 0 : (c < n ? c : n);
}

template <typename T>
__global__ void k_order_count(OrderGrid g, int dim, int64_t n, const T* x, int64_t ld, const int64_t* n_dev,
                              uint32_t* hist) {
  const int64_t live = order_live(n, n_dev);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < live; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&hist[order_key(g, dim, x, ld, i)], 1u);
}

// Exclusive prefix sum of the kOrderBuckets counts in place, one block of
// kBlock threads, each owning a contiguous run of buckets.
__global__ __launch_bounds__(kBlock) void k_order_scan(uint32_t* hist) {
  constexpr int kRun = kOrderBuckets / kBlock;
  __shared__ uint32_t part[kBlock];
  const int t = threadIdx.x;
  uint32_t* h = hist + (size_t)t * kRun;
  uint32_t sum = 0u;
  for (int k = 0; k < kRun; ++k) sum += h[k];
  part[t] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the run sums
  for (int off = 1; off < kBlock; off <<= 1) {
    const uint32_t add = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;
  for (int k = 0; k < kRun; ++k) {
    const uint32_t v = h[k];
    h[k] = run;
    run += v;
  }
}

template <typename T>
__global__ void k_order_place(OrderGrid g, int dim, int64_t n, const T* x, int64_t ld, const int64_t* n_dev,
                              uint32_t* next, int32_t* order) {
  const int64_t live = order_live(n, n_dev);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < live; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t pos = atomicAdd(&next[order_key(g, dim, x, ld, i)], 1u);
    order[pos] = (int32_t)i;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Validation helpers (shared with the walk entry points)
// ---------------------------------------------------------------------------
int check_scene(bvc_scene s) {
  if (!s) return fail(BVC_EINVAL, "scene is null");
  if (!s->h.dev) return fail(BVC_ESTATE, "scene is not uploaded");
  return BVC_OK;
}

int check_field(const bvc_field& f, int dim, const char* name) {
  if (f.kind < 0 || f.kind > 10) return fail(BVC_EINVAL, std::string(name) + ": unknown field kind");
  if (f.kind == 9 && dim != 2) return fail(BVC_EINVAL, std::string(name) + ": 2D field used in 3D");
  if (f.n_coef < 0) return fail(BVC_EINVAL, std::string(name) + ": negative coefficient count");
  if (f.n_coef > 0 && !f.coef) return fail(BVC_EINVAL, std::string(name) + ": coefficients are null");
  if ((f.kind == 2 || f.kind == 4 || f.kind == 6) && dim != 2)
    return fail(BVC_EINVAL, std::string(name) + ": 2D field used in 3D");
  if (f.kind == 5 && dim != 3) return fail(BVC_EINVAL, std::string(name) + ": 3D field used in 2D");
  if (f.kind == 3 && (f.n_coef % (1 + dim) != 0 || !(f.param[0] > 0)))
    return fail(BVC_EINVAL, std::string(name) + ": Gaussian sum needs (1+dim)*k coefficients and s > 0");
  if (f.kind == 4 && (f.n_coef % 3 != 0 || !(f.param[0] > 0)))
    return fail(BVC_EINVAL, std::string(name) + ": Gaussian potential needs 3*k coefficients and s > 0");
  if (f.kind == 5) {
    const int L = (int)f.param[0];
    if (L < 0 || L > 16 || f.n_coef != (L + 1) * (L + 1))
      return fail(BVC_EINVAL, std::string(name) + ": solid harmonics need (L+1)^2 coefficients, L <= 16");
  }
  if (f.kind == 6 && f.n_coef < 1) return fail(BVC_EINVAL, std::string(name) + ": Fourier series is empty");
  return BVC_OK;
}

namespace {
int take_impl(int32_t dti, int32_t dto, int64_t n_idx, const int64_t* count, const int32_t* idx, int32_t rows,
              int64_t ld_in, const void* in, int64_t ld_out, void* out, void* stream) {
  if ((dti != BVC_F32 && dti != BVC_F64) || (dto != BVC_F32 && dto != BVC_F64))
    return fail(BVC_EINVAL, "dtype must be F32 or F64");
  if (n_idx < 0 || rows < 0 || ld_in < 0 || ld_out < n_idx) return fail(BVC_EINVAL, "bad sizes");
  if (n_idx == 0 || rows == 0) return BVC_OK;
  if (!in || !out) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)((n_idx + kBlock - 1) / kBlock);
  if (dti == BVC_F64 && dto == BVC_F64)
    hipLaunchKernelGGL((k_take<double, double>), dim3(blocks), dim3(kBlock), 0, st, n_idx, count, idx, rows, ld_in,
                       (const double*)in, ld_out, (double*)out);
  else if (dti == BVC_F64 && dto == BVC_F32)
    hipLaunchKernelGGL((k_take<double, float>), dim3(blocks), dim3(kBlock), 0, st, n_idx, count, idx, rows, ld_in,
                       (const double*)in, ld_out, (float*)out);
  else if (dti == BVC_F32 && dto == BVC_F64)
    hipLaunchKernelGGL((k_take<float, double>), dim3(blocks), dim3(kBlock), 0, st, n_idx, count, idx, rows, ld_in,
                       (const float*)in, ld_out, (double*)out);
  else
    hipLaunchKernelGGL((k_take<float, float>), dim3(blocks), dim3(kBlock), 0, st, n_idx, count, idx, rows, ld_in,
                       (const float*)in, ld_out, (float*)out);
  return check_hip(hipGetLastError(), "take launch");
}
}  // namespace

}  // namespace bvc

using namespace bvc;

extern "C" {

int bvc_sample_cache(bvc_scene s, int64_t n, double l, int32_t sides, uint64_t seed, uint32_t batch,
                     double* x, double* nrm, double* w, double* xbar, double* R0, int32_t* accept,
                     void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (!(l > 0) || !std::isfinite(l)) return fail(BVC_EINVAL, "offset l must be positive");
  if (sides != 1 && sides != 2) return fail(BVC_EINVAL, "sides must be 1 or 2");
  if (sides == 2 && s->h.dim == 3) return fail(BVC_EUNSUPPORTED, "two-sided offsets are 2D only");
  if (n == 0) return BVC_OK;
  if (!x || !nrm || !w || !xbar || !R0 || !accept) return fail(BVC_EINVAL, "null output");
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_cdf(s->h, l, sides, st);
  if (rc) return rc;
  const double M = candidate_measure(s->h, l, sides);
  SceneDev S = s->h.view();
  const int blocks = (int)((n + kBlock - 1) / kBlock);
  const size_t lds = stack_bytes(s->h, kBlock);
  if (S.dim == 2)
    hipLaunchKernelGGL(k_sample_cache<2>, dim3(blocks), dim3(kBlock), lds, st, S, n, l, seed, batch, M, x, nrm, w,
                       xbar, R0, accept);
  else
    hipLaunchKernelGGL(k_sample_cache<3>, dim3(blocks), dim3(kBlock), lds, st, S, n, l, seed, batch, M, x, nrm, w,
                       xbar, R0, accept);
  return check_hip(hipGetLastError(), "sample_cache launch");
}

int bvc_sample_roi(bvc_scene dom, bvc_scene roi, int64_t n, uint64_t seed, uint32_t batch, double* x, double* nrm,
                   double* w, double* xbar, double* R0, int32_t* accept, void* stream) {
  int rc = check_scene(dom);
  if (rc) return rc;
  rc = check_scene(roi);
  if (rc) return rc;
  if (dom->h.dim != roi->h.dim) return fail(BVC_EINVAL, "the region and the domain differ in dimension");
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (n == 0) return BVC_OK;
  if (!x || !nrm || !w || !xbar || !R0 || !accept) return fail(BVC_EINVAL, "null output");
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_cdf(roi->h, 0.0, 1, st);
  if (rc) return rc;
  const double M = candidate_measure(roi->h, 0.0, 1);
  const SceneDev Sd = dom->h.view(), Sr = roi->h.view();
  const int blocks = (int)((n + kBlock - 1) / kBlock);
  const size_t lds = stack_bytes(dom->h, kBlock);
  if (Sd.dim == 2)
    hipLaunchKernelGGL(k_sample_roi<2>, dim3(blocks), dim3(kBlock), lds, st, Sd, Sr, n, seed, batch, M, x, nrm, w,
                       xbar, R0, accept);
  else
    hipLaunchKernelGGL(k_sample_roi<3>, dim3(blocks), dim3(kBlock), lds, st, Sd, Sr, n, seed, batch, M, x, nrm, w,
                       xbar, R0, accept);
  return check_hip(hipGetLastError(), "sample_roi launch");
}

int bvc_sample_mixed(bvc_scene full, bvc_scene dir, bvc_scene neu, int64_t n, double l, double junction_drop,
                     uint64_t seed, uint32_t batch, double* x, double* nrm, double* w, double* xbar, double* R0,
                     int32_t* kind, void* stream) {
  int rc = check_scene(full);
  if (!rc) rc = check_scene(dir);
  if (!rc) rc = check_scene(neu);
  if (rc) return rc;
  if (full->h.dim != 2 || dir->h.dim != 2 || neu->h.dim != 2)
    return fail(BVC_EUNSUPPORTED, "the mixed-boundary cache is 2D only");
  if (dir->h.np == 0 || neu->h.np == 0) return fail(BVC_EINVAL, "the Dirichlet and the Neumann parts must be non-empty");
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (!(l > 0) || !std::isfinite(l)) return fail(BVC_EINVAL, "offset l must be positive");
  if (!(junction_drop >= 0.0) || !(junction_drop < 1.0)) return fail(BVC_EINVAL, "junction_drop must be in [0, 1)");
  if (n == 0) return BVC_OK;
  if (!x || !nrm || !w || !xbar || !R0 || !kind) return fail(BVC_EINVAL, "null output");
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_cdf(dir->h, l, 1, st);
  if (!rc) rc = ensure_cdf(neu->h, 0.0, 1, st);
  if (rc) return rc;
  const double MD = candidate_measure(dir->h, l, 1);
  const double M = MD + candidate_measure(neu->h, 0.0, 1);
  const SceneDev Sf = full->h.view(), Sd = dir->h.view(), Sn = neu->h.view();
  const int blocks = (int)((n + kBlock - 1) / kBlock);
  const size_t lds = std::max(stack_bytes(full->h, kBlock), stack_bytes(dir->h, kBlock));
  hipLaunchKernelGGL(k_sample_mixed, dim3(blocks), dim3(kBlock), lds, st, Sf, Sd, Sn, n, l, junction_drop, seed,
                     batch, MD, M, x, nrm, w, xbar, R0, kind);
  return check_hip(hipGetLastError(), "sample_mixed launch");
}

int bvc_sample_sources(bvc_scene s, const bvc_field* f, int64_t m, const double* lo, const double* hi, double l,
                       uint64_t seed, uint32_t batch, double* y, double* sw, void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  if (!f || !lo || !hi) return fail(BVC_EINVAL, "null argument");
  const int dim = s->h.dim;
  rc = check_field(*f, dim, "f");
  if (rc) return rc;
  if (m < 0) return fail(BVC_EINVAL, "m must be >= 0");
  int64_t M = 1;
  for (int a = 0; a < dim; ++a) {
    M *= m;
    if (!(hi[a] > lo[a])) return fail(BVC_EINVAL, "empty source box");
  }
  if (M >= (int64_t)1 << 31) return fail(BVC_EINVAL, "too many sources");
  if (m == 0) return BVC_OK;
  if (!y || !sw) return fail(BVC_EINVAL, "null output");
  if (!(l >= 0)) return fail(BVC_EINVAL, "l must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  SceneDev S = s->h.view();
  const int blocks = (int)((M + kBlock - 1) / kBlock);
  const size_t lds = stack_bytes(s->h, kBlock);
  const double z0 = dim == 3 ? lo[2] : 0.0, z1 = dim == 3 ? hi[2] : 1.0;
  if (dim == 2)
    hipLaunchKernelGGL(k_sample_sources<2>, dim3(blocks), dim3(kBlock), lds, st, S, to_dev(*f), m, M, lo[0], lo[1],
                       z0, hi[0], hi[1], z1, l, seed, batch, y, sw);
  else
    hipLaunchKernelGGL(k_sample_sources<3>, dim3(blocks), dim3(kBlock), lds, st, S, to_dev(*f), m, M, lo[0], lo[1],
                       z0, hi[0], hi[1], z1, l, seed, batch, y, sw);
  return check_hip(hipGetLastError(), "sample_sources launch");
}

int bvc_classify(bvc_scene s, int64_t n, const double* x, double l, int32_t* cls, double* dist, void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (!(l >= 0)) return fail(BVC_EINVAL, "l must be >= 0");
  if (n == 0) return BVC_OK;
  if (!x || !cls) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  SceneDev S = s->h.view();
  const int blocks = (int)((n + kBlock - 1) / kBlock);
  const size_t lds = stack_bytes(s->h, kBlock);
  if (S.dim == 2)
    hipLaunchKernelGGL(k_classify<2>, dim3(blocks), dim3(kBlock), lds, st, S, n, x, l, cls, dist);
  else
    hipLaunchKernelGGL(k_classify<3>, dim3(blocks), dim3(kBlock), lds, st, S, n, x, l, cls, dist);
  return check_hip(hipGetLastError(), "classify launch");
}

int bvc_classify_mixed(bvc_scene full, bvc_scene dir, int64_t n, const double* x, double l, int32_t* cls,
                       double* dist, void* stream) {
  int rc = check_scene(full);
  if (!rc) rc = check_scene(dir);
  if (rc) return rc;
  if (full->h.dim != 2 || dir->h.dim != 2) return fail(BVC_EUNSUPPORTED, "mixed classification is 2D only");
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (!(l >= 0) || !std::isfinite(l)) return fail(BVC_EINVAL, "l must be finite and >= 0");
  if (n == 0) return BVC_OK;
  if (!x || !cls) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)((n + kBlock - 1) / kBlock);
  const size_t lds = std::max(stack_bytes(full->h, kBlock), stack_bytes(dir->h, kBlock));
  hipLaunchKernelGGL(k_classify_mixed, dim3(blocks), dim3(kBlock), lds, st, full->h.view(), dir->h.view(), n, x, l,
                     cls, dist);
  return check_hip(hipGetLastError(), "classify_mixed launch");
}

int64_t bvc_compact_scratch_ints(int64_t n) { return (n + kCompactTile - 1) / kCompactTile + 4; }

int bvc_compact(int64_t n, const int32_t* flags, int32_t want, int32_t* idx, int32_t* scratch,
                int64_t* count_host, void* stream) {
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (!count_host) return fail(BVC_EINVAL, "count_host is null");
  *count_host = 0;
  if (n == 0) return BVC_OK;
  if (!flags || !idx || !scratch) return fail(BVC_EINVAL, "null argument");
  if (((uintptr_t)scratch & 7) != 0) return fail(BVC_EINVAL, "scratch must be 8-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)((n + kCompactTile - 1) / kCompactTile);
  int* offs = scratch + 2;
  int64_t* tot = (int64_t*)scratch;
  int rc = BVC_OK;
  hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kBlock), 0, st, n, flags, want, offs);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, nb, offs, tot);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kBlock), 0, st, n, flags, want, offs, idx);
  rc = check_hip(hipGetLastError(), "compact launch");
  int64_t h = 0;
  if (!rc) rc = check_hip(hipMemcpyAsync(&h, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st), "compact count");
  if (!rc) rc = check_hip(hipStreamSynchronize(st), "compact sync");
  if (!rc) *count_host = h;
  return rc;
}

int bvc_compact_count(int64_t n, const int32_t* flags, int32_t want, int32_t* idx, int32_t* scratch, int64_t* count,
                      void* stream) {
  if (n < 0 || n >= (int64_t)1 << 31) return fail(BVC_EINVAL, "n out of range");
  if (!count) return fail(BVC_EINVAL, "count is null");
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) return zero_async(count, sizeof(int64_t), st);
  if (!flags || !idx || !scratch) return fail(BVC_EINVAL, "null argument");
  if (((uintptr_t)scratch & 7) != 0) return fail(BVC_EINVAL, "scratch must be 8-byte aligned");
  const int nb = (int)((n + kCompactTile - 1) / kCompactTile);
  int* offs = scratch + 2;
  hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kBlock), 0, st, n, flags, want, offs);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, nb, offs, count);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kBlock), 0, st, n, flags, want, offs, idx);
  return check_hip(hipGetLastError(), "compact launch");
}


int bvc_take(int32_t dti, int32_t dto, int64_t n_idx, const int32_t* idx, int32_t rows, int64_t ld_in,
             const void* in, int64_t ld_out, void* out, void* stream) {
  return take_impl(dti, dto, n_idx, nullptr, idx, rows, ld_in, in, ld_out, out, stream);
}

int bvc_take_count(int32_t dti, int32_t dto, int64_t n_cap, const int64_t* count, const int32_t* idx, int32_t rows,
                   int64_t ld_in, const void* in, int64_t ld_out, void* out, void* stream) {
  if (!count) return fail(BVC_EINVAL, "count is null");
  return take_impl(dti, dto, n_cap, count, idx, rows, ld_in, in, ld_out, out, stream);
}

int bvc_scatter(int32_t dtype, int64_t n_idx, const int32_t* idx, int32_t rows, int64_t ld_in, const void* in,
                int64_t ld_out, void* out, void* stream) {
  if (dtype != BVC_F32 && dtype != BVC_F64) return fail(BVC_EINVAL, "dtype must be F32 or F64");
  if (n_idx < 0 || rows < 0 || ld_in < n_idx || ld_out < 0) return fail(BVC_EINVAL, "bad sizes");
  if (n_idx == 0 || rows == 0) return BVC_OK;
  if (!in || !out || !idx) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const int blocks = (int)((n_idx + kBlock - 1) / kBlock);
  if (dtype == BVC_F64)
    hipLaunchKernelGGL(k_scatter<double>, dim3(blocks), dim3(kBlock), 0, st, n_idx, idx, rows, ld_in,
                       (const double*)in, ld_out, (double*)out);
  else
    hipLaunchKernelGGL(k_scatter<float>, dim3(blocks), dim3(kBlock), 0, st, n_idx, idx, rows, ld_in,
                       (const float*)in, ld_out, (float*)out);
  return check_hip(hipGetLastError(), "scatter launch");
}

size_t bvc_spatial_order_workspace_bytes(void) { return (size_t)kOrderBuckets * sizeof(uint32_t); }

int bvc_spatial_order(bvc_scene s, int32_t dtype, int64_t n, const void* x, int64_t ld, const int64_t* n_dev,
                      int32_t* order, void* work, size_t work_bytes, void* stream) {
  int rc = check_scene(s);
  if (rc) return rc;
  if (dtype != BVC_F32 && dtype != BVC_F64) return fail(BVC_EINVAL, "dtype must be F32 or F64");
  if (n < 0 || ld < n) return fail(BVC_EINVAL, "need 0 <= n <= ld");
  if (n > INT32_MAX) return fail(BVC_EINVAL, "n must fit int32 (order entries)");
  if (n == 0) return BVC_OK;
  if (!x || !order || !work) return fail(BVC_EINVAL, "null argument");
  if (work_bytes < bvc_spatial_order_workspace_bytes()) return fail(BVC_EINVAL, "spatial order workspace too small");
  if (((uintptr_t)work & 255) != 0) return fail(BVC_EINVAL, "spatial order workspace must be 256-byte aligned");
  const SceneHost& h = s->h;
  const int dim = h.dim;
  OrderGrid g{};
  g.bits = dim == 3 ? 5 : 8;
  for (int a = 0; a < dim; ++a) {
    const double ext = h.hi[a] - h.lo[a];
    g.lo[a] = h.lo[a];
    g.scale[a] = ext > 0.0 ? (double)(1 << g.bits) / ext : 0.0;
  }
  hipStream_t st = (hipStream_t)stream;
  uint32_t* hist = (uint32_t*)work;
  rc = zero_async(hist, bvc_spatial_order_workspace_bytes(), st);
  if (rc) return rc;
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  if (dtype == BVC_F64)
    hipLaunchKernelGGL(k_order_count<double>, dim3(blocks), dim3(kBlock), 0, st, g, dim, n, (const double*)x, ld,
                       n_dev, hist);
  else
    hipLaunchKernelGGL(k_order_count<float>, dim3(blocks), dim3(kBlock), 0, st, g, dim, n, (const float*)x, ld,
                       n_dev, hist);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kBlock), 0, st, hist);
  if (dtype == BVC_F64)
    hipLaunchKernelGGL(k_order_place<double>, dim3(blocks), dim3(kBlock), 0, st, g, dim, n, (const double*)x, ld,
                       n_dev, hist, order);
  else
    hipLaunchKernelGGL(k_order_place<float>, dim3(blocks), dim3(kBlock), 0, st, g, dim, n, (const float*)x, ld,
                       n_dev, hist, order);
  return check_hip(hipGetLastError(), "spatial order launch");
}

}  // extern "C"
