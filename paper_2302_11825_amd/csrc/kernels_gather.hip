// Boundary-integral gather (Eqs. 3-6), its adjoint, and the basis expansions
// that make the cache linear in the boundary data.
//
// The gather inverts the loop order of the paper's splat (Algorithm 1): the
// evaluation points are the parallel dimension, held in registers (two per
// thread), and cache entries stream through LDS in tiles that every thread of
// the block reads by broadcast.  No atomics: each point's sum is owned by one
// thread.  Cache entries are pre-scaled once per tile (a n/(2 pi), b/(2 pi),
// ...) so the pair loop is a handful of FMAs, one reciprocal and, in 2D, one
// logarithm.  FP32 partial sums are folded into FP64 after every tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "bessel.hpp"
#include "bvc_device.hpp"

namespace bvc {
namespace {

constexpr int kGBlock = 256;
constexpr int kTile = 256;
constexpr int kPPT = 2;  // evaluation points per thread

// log(r^2) via the hardware log2 in FP32; natural log in FP64.
__device__ __forceinline__ float log_r2(float r2) { return __log2f(r2); }
__device__ __forceinline__ double log_r2(double r2) { return log(r2); }
template <typename T>
__host__ __device__ constexpr T log_scale() {
  return sizeof(T) == 4 ? (T)0.69314718055994530942 : (T)1;  // ln r^2 = ln2 * log2 r^2
}
// FP32: the hardware reciprocal and reciprocal square root (1 ulp), not the
// correctly rounded division sequence.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

template <typename T>
struct GatherArgs {
  int64_t n_eval;
  const T* ex;       // [D][n_eval]
  int64_t n_cache;
  const T* cx;       // [D][n_cache]
  const T* cn;
  const T* ca;
  const T* cb;
  int64_t n_src;
  const T* sy;       // [D][n_src]
  const T* ss;
  T* u;              // [n_eval] or null
  T* g;              // [D][n_eval] or null
  const T* scale;    // multiply outputs by scale[k] (adjoint dL/dx) or null
  int accumulate;
  // FP64 near field (FP32 kernels only): boundary pairs with r^2 < tau2 in
  // FP32 are left out of the FP32 sums and added in FP64 from these copies.
  T tau2;
  const double* nx;   // evaluation points [D][n_eval]
  const double* ncx;  // cache points [D][n_cache]
  const double* ncn;  // cache normals [D][n_cache]
  const double* na;   // [n_cache]
  const double* nb;   // [n_cache]
  // Clamp of dG/dn in the potential's boundary term (Eq. 9), kernels with
  // CLAMP only: clampc in the kernel's precision, clamp64 for the FP64 near
  // field.
  T clampc;
  double clamp64;
  // device count of cache entries (<= n_cache, the arrays' leading
  // dimension), or null for n_cache
  const int64_t* n_dev;
  // near field: the evaluation points that may need it come first (0 = any)
  int64_t near_lead;
};

template <typename T>
__device__ __forceinline__ int64_t cache_count(const GatherArgs<T>& a) {
  return a.n_dev ? std::min<int64_t>(a.n_cache, *a.n_dev) : a.n_cache;
}

// Entry layout in LDS (8 values): 2D boundary {y0, y1, 2 na0, 2 na1, 2 bl, bg,
// na0, na1}, 3D boundary {y0, y1, y2, bl, na0, na1, na2, -}; sources
// {y.., sl, sg} (2D sl doubled like bl).  With CLAMP a ninth array after the
// tile holds each boundary entry's clamp bound in the same scaling as its
// dG/dn term: |a| c (3D), 2 |a| c (2D, whose potential runs doubled).
template <typename T, int D, bool GRAD, bool NEAR = false, int PPT = kPPT, bool CLAMP = false>
__device__ __forceinline__ void gather_block(const GatherArgs<T>& a, int64_t block, T* ent);

// With the near field and near_lead > 0 only the blocks holding one of the
// first near_lead evaluation points run the near test (the caller orders the
// points that can meet a cache point closer than tau first); the others take
// the plain FP32 loop.
template <typename T, int D, bool GRAD, bool NEAR, int PPT, bool CLAMP = false>
__global__ __launch_bounds__(kGBlock) void k_gather(GatherArgs<T> a) {
  __shared__ T ent[kTile * (CLAMP ? 9 : 8)];
  if constexpr (NEAR) {
    if (a.near_lead > 0 && (int64_t)blockIdx.x * (kGBlock * PPT) >= a.near_lead) {
      gather_block<T, D, GRAD, false, PPT, CLAMP>(a, blockIdx.x, ent);
      return;
    }
  }
  gather_block<T, D, GRAD, NEAR, PPT, CLAMP>(a, blockIdx.x, ent);
}

// Clamp of t to [-b, b] (b >= 0): one v_med3 in FP32.
__device__ __forceinline__ float clamp_sym(float t, float b) { return __builtin_amdgcn_fmed3f(t, -b, b); }
__device__ __forceinline__ double clamp_sym(double t, double b) { return fmin(fmax(t, -b), b); }

// FP64 contribution of cache point i to u (and grad u) at evaluation point k,
// from the FP64 copies: u += a dG/dn - b G (Eq. 3), grad from Eq. 5; with
// CLAMP, dG/dn in u is clamped to [-c, c] (Eq. 9).
template <int D, bool GRAD, bool CLAMP = false>
__device__ __forceinline__ void near_pair(const GatherArgs<float>& a, int64_t k, int64_t i, double& tu, double* tg) {
  double d[D];
  double r2 = 0.0, nd = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    d[c] = a.ncx[c * a.n_cache + i] - a.nx[c * a.n_eval + k];
    r2 += d[c] * d[c];
    nd += a.ncn[c * a.n_cache + i] * d[c];
  }
  if (!(r2 > 0.0)) return;  // coincident points carry no finite contribution
  const double av = a.na[i], bv = a.nb[i];
  if constexpr (D == 2) {
    const double k2 = 1.0 / (2.0 * kPi * r2);
    const double kn = CLAMP ? clamp_sym(nd * k2, a.clamp64) : nd * k2;
    tu += av * kn - bv * log(r2) / (4.0 * kPi);
    if constexpr (GRAD) {
      const double q = (2.0 * av * nd / r2 + bv) * k2;
#pragma unroll
      for (int c = 0; c < D; ++c) tg[c] += q * d[c] - av * a.ncn[c * a.n_cache + i] * k2;
    }
  } else {
    const double r = sqrt(r2);
    const double k3 = 1.0 / (4.0 * kPi * r2 * r);
    const double kn = CLAMP ? clamp_sym(nd * k3, a.clamp64) : nd * k3;
    tu += bv / (4.0 * kPi * r) + av * kn;
    if constexpr (GRAD) {
      const double q = (3.0 * av * nd / r2 + bv) * k3;
#pragma unroll
      for (int c = 0; c < D; ++c) tg[c] += q * d[c] - av * a.ncn[c * a.n_cache + i] * k3;
    }
  }
}

// One block's share of the gather: evaluation points
// [block*256*PPT, (block+1)*256*PPT), PPT per thread.  The sum of each point
// runs over the cache in the same order whatever PPT is, so every PPT gives
// bit-identical results and PPT is a pure tuning choice.
template <typename T, int D, bool GRAD, bool NEAR, int PPT, bool CLAMP>
__device__ __forceinline__ void gather_block(const GatherArgs<T>& a, int64_t block, T* ent) {
  static_assert(!NEAR || sizeof(T) == 4, "the near field applies to FP32 gathers");
  const int tid = threadIdx.x;
  const int64_t k0 = block * (kGBlock * PPT) + tid;
  T x[PPT][D];
  bool live[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int64_t k = k0 + p * kGBlock;
    live[p] = k < a.n_eval;
#pragma unroll
    for (int c = 0; c < D; ++c) x[p][c] = live[p] ? a.ex[c * a.n_eval + k] : T(0);
  }
  double tu[PPT], tg[PPT][D];
  T au[PPT], ag[PPT][D];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    tu[p] = 0.0;
    au[p] = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      tg[p][c] = 0.0;
      ag[p][c] = T(0);
    }
  }
  const T inv2pi = (T)(1.0 / (2.0 * kPi)), inv4pi = (T)(1.0 / (4.0 * kPi));
  const T tiny = sizeof(T) == 4 ? (T)1e-18 : (T)1e-200;

  // In 2D the FP32 u accumulators hold twice the potential (the entries carry
  // the factor 2 that the gradient needs), halved when folded into FP64.
  constexpr double kUnfold = D == 2 ? 0.5 : 1.0;
  auto fold = [&]() {
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      tu[p] += kUnfold * (double)au[p];
      au[p] = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        tg[p][c] += (double)ag[p][c];
        ag[p][c] = T(0);
      }
    }
  };

  // ---- boundary samples (Eqs. 3 and 5) ----
  const int64_t nc = cache_count(a);
  for (int64_t t0 = 0; t0 < nc; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, nc - t0);
    if (tid < cnt) {
      const int64_t i = t0 + tid;
      T y[D], nn[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        y[c] = a.cx[c * a.n_cache + i];
        nn[c] = a.cn[c * a.n_cache + i];
      }
      const T av = a.ca[i], bv = a.cb[i];
      T* e = ent + tid * 8;
      if constexpr (CLAMP) ent[kTile * 8 + tid] = (D == 2 ? T(2) : T(1)) * fabs(av) * a.clampc;
      if constexpr (D == 2) {
        // twice the potential terms (see kUnfold), the gradient terms as is
        e[0] = y[0];
        e[1] = y[1];
        e[2] = T(2) * nn[0] * av * inv2pi;
        e[3] = T(2) * nn[1] * av * inv2pi;
        e[4] = -bv * inv2pi * log_scale<T>();  // 2 (-G b) = -(b/2pi) ln r^2
        e[5] = bv * inv2pi;
        e[6] = nn[0] * av * inv2pi;
        e[7] = nn[1] * av * inv2pi;
      } else {
        e[0] = y[0];
        e[1] = y[1];
        e[2] = y[2];
        e[3] = bv * inv4pi;  // -G b = b/(4 pi r)
        e[4] = nn[0] * av * inv4pi;
        e[5] = nn[1] * av * inv4pi;
        e[6] = nn[2] * av * inv4pi;
      }
    }
    __syncthreads();
    bool hit[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) hit[p] = false;
#pragma unroll 4
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 8;
      if constexpr (D == 2) {
        const T y0 = e[0], y1 = e[1], m0 = e[2], m1 = e[3], bl = e[4], bg = e[5];
        const T bt = CLAMP ? ent[kTile * 8 + j] : T(0);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const T dx = y0 - x[p][0], dy = y1 - x[p][1];
          // r^2 + tiny keeps coincident points finite at no extra instruction
          const T r2 = fma(dx, dx, fma(dy, dy, tiny));
          T ri, lr;
          if constexpr (NEAR) {
            // near pairs contribute nothing here; near_sweep adds them in FP64
            const bool nr = r2 < a.tau2;
            hit[p] = hit[p] || nr;
            ri = nr ? T(0) : recip(r2);
            lr = nr ? T(0) : log_r2(r2);
          } else {
            ri = recip(r2);
            lr = log_r2(r2);
          }
          const T t2 = fma(m0, dx, m1 * dy);  // 2 a (n . (y - x)) / (2 pi)
          T q;
          if constexpr (CLAMP) {
            // 2 a clamp(dG/dn) = clamp(2 a dG/dn, -2|a|c, 2|a|c); grad unclamped
            const T tk = t2 * ri;
            au[p] = fma(bl, lr, au[p] + clamp_sym(tk, bt));
            q = tk + bg;
          } else {
            au[p] = fma(bl, lr, fma(t2, ri, au[p]));
            q = fma(t2, ri, bg);
          }
          if constexpr (GRAD) {
            // grad = (q (y - x) - a n / (2 pi)) / r^2,  q = (2 a n.(y-x)/r^2 + b)/(2 pi)
            ag[p][0] = fma(ri, fma(q, dx, -e[6]), ag[p][0]);
            ag[p][1] = fma(ri, fma(q, dy, -e[7]), ag[p][1]);
          }
        }
      } else {
        const T y0 = e[0], y1 = e[1], y2 = e[2], bl = e[3], n0 = e[4], n1 = e[5], n2 = e[6];
        const T bt = CLAMP ? ent[kTile * 8 + j] : T(0);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const T dx = y0 - x[p][0], dy = y1 - x[p][1], dz = y2 - x[p][2];
          const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, tiny)));
          T ri;
          if constexpr (NEAR) {
            const bool nr = r2 < a.tau2;
            hit[p] = hit[p] || nr;
            ri = nr ? T(0) : rsq(r2);
          } else {
            ri = rsq(r2);
          }
          const T ri2 = ri * ri;
          const T t = fma(n0, dx, fma(n1, dy, n2 * dz));
          if constexpr (CLAMP) {
            // b/r + clamp(t/r^3, -|a|c, |a|c)
            au[p] = fma(ri, bl, au[p] + clamp_sym(t * ri2 * ri, bt));
          } else {
            // b/r + t/r^3 = (b + t/r^2)/r
            au[p] = fma(ri, fma(t, ri2, bl), au[p]);
          }
          if constexpr (GRAD) {
            const T ri3 = ri2 * ri;
            const T q = ri3 * fma(T(3) * t, ri2, bl);
            ag[p][0] = fma(-n0, ri3, fma(q, dx, ag[p][0]));
            ag[p][1] = fma(-n1, ri3, fma(q, dy, ag[p][1]));
            ag[p][2] = fma(-n2, ri3, fma(q, dz, ag[p][2]));
          }
        }
      }
    }
    if constexpr (NEAR) {
      // FP64 sweep of the tile for lanes that met a near pair: the same FP32
      // test as above picks exactly the pairs left out of the FP32 sums
      bool any = false;
#pragma unroll
      for (int p = 0; p < PPT; ++p) any = any || (hit[p] && live[p]);
      if (__any(any)) {
        for (int j = 0; j < cnt; ++j) {
          const T* e = ent + j * 8;
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            if (!(hit[p] && live[p])) continue;
            T r2;
            if constexpr (D == 2) {
              const T dx = e[0] - x[p][0], dy = e[1] - x[p][1];
              r2 = fma(dx, dx, fma(dy, dy, tiny));
            } else {
              const T dx = e[0] - x[p][0], dy = e[1] - x[p][1], dz = e[2] - x[p][2];
              r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, tiny)));
            }
            if (r2 < a.tau2) near_pair<D, GRAD, CLAMP>(a, k0 + p * kGBlock, t0 + j, tu[p], tg[p]);
          }
        }
      }
    }
    __syncthreads();
    fold();
  }

  // ---- source samples (Eqs. 4 and 6) ----
  for (int64_t t0 = 0; t0 < a.n_src; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, a.n_src - t0);
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      T* e = ent + tid * 8;
      const T sv = a.ss[j];
#pragma unroll
      for (int c = 0; c < D; ++c) e[c] = a.sy[c * a.n_src + j];
      if constexpr (D == 2) {
        e[2] = sv * inv2pi * log_scale<T>();  // 2 G s = (s/2pi) ln r^2
        e[3] = -sv * inv2pi;                  // dG/dx s = -s (y-x)/(2 pi r^2)
      } else {
        e[3] = -sv * inv4pi;  // G s = -s/(4 pi r); dG/dx s = -s (y-x)/(4 pi r^3)
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 8;
      if constexpr (D == 2) {
        const T y0 = e[0], y1 = e[1], sl = e[2], sg = e[3];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const T dx = y0 - x[p][0], dy = y1 - x[p][1];
          const T r2 = fma(dx, dx, fma(dy, dy, tiny));
          au[p] = fma(sl, log_r2(r2), au[p]);
          if constexpr (GRAD) {
            const T q = sg * recip(r2);
            ag[p][0] += q * dx;
            ag[p][1] += q * dy;
          }
        }
      } else {
        const T y0 = e[0], y1 = e[1], y2 = e[2], sl = e[3];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const T dx = y0 - x[p][0], dy = y1 - x[p][1], dz = y2 - x[p][2];
          const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, tiny)));
          const T ri = rsq(r2);
          au[p] = fma(sl, ri, au[p]);
          if constexpr (GRAD) {
            const T q = sl * ri * ri * ri;
            ag[p][0] += q * dx;
            ag[p][1] += q * dy;
            ag[p][2] += q * dz;
          }
        }
      }
    }
    __syncthreads();
    fold();
  }

#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int64_t k = k0 + p * kGBlock;
    if (!live[p]) continue;
    const double sc = a.scale ? (double)a.scale[k] : 1.0;
    if (a.u) a.u[k] = (T)((a.accumulate ? (double)a.u[k] : 0.0) + sc * tu[p]);
    if (GRAD && a.g) {
#pragma unroll
      for (int c = 0; c < D; ++c)
        a.g[c * a.n_eval + k] = (T)((a.accumulate ? (double)a.g[c * a.n_eval + k] : 0.0) + sc * tg[p][c]);
    }
  }
}

// Screened gather in 3D (Eqs. 3-6 with the kernels of Appendix A.2):
// G = -e/(4 pi r), e = exp(-s r), and with Q = e (1 + s r)
//   a dG/dn - b G = Q t / r^3 + bl e / r,   t = a n.(y-x)/(4 pi), bl = b/(4 pi)
//   grad = Q [(y-x)(3 t/r^2 + bl)/r^3 - a n/(4 pi r^3)] + s^2 e t (y-x)/r^3
// (the Poisson terms times Q plus dG/dn times dQ/dx = s^2 e (y - x)); a
// source term s_j adds G s_j and Q dG0/dx s_j.  One evaluation point per
// thread; the cache and sources stream through LDS tiles as in k_gather.
template <typename T, bool GRAD>
__global__ __launch_bounds__(kGBlock) void k_gather_screened3(GatherArgs<T> a, double sigma) {
  __shared__ T ent[kTile * 8];
  const int tid = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * kGBlock + tid;
  const bool live = k < a.n_eval;
  T x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] = live ? a.ex[c * a.n_eval + k] : T(0);
  const T s = (T)sqrt(sigma), s2 = (T)sigma;
  // e^(-s r) by the hardware exp2 in FP32 (s scaled by log2 e)
  const T sl2 = sizeof(T) == 4 ? (T)(sqrt(sigma) * 1.4426950408889634) : s;
  auto expo = [&](T r) -> T {
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_exp2f(-sl2 * r);
    else return exp(-sl2 * r);
  };
  const T inv4pi = (T)(1.0 / (4.0 * kPi));
  const T tiny = sizeof(T) == 4 ? (T)1e-18 : (T)1e-200;
  double tu = 0.0, tg[3] = {0.0, 0.0, 0.0};
  T au = T(0), ag[3] = {T(0), T(0), T(0)};
  auto fold = [&]() {
    tu += (double)au;
    au = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tg[c] += (double)ag[c];
      ag[c] = T(0);
    }
  };
  const int64_t nc = cache_count(a);
  for (int64_t t0 = 0; t0 < nc; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, nc - t0);
    if (tid < cnt) {
      const int64_t i = t0 + tid;
      T* e = ent + tid * 8;
      const T av = a.ca[i], bv = a.cb[i];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e[c] = a.cx[c * a.n_cache + i];
        e[4 + c] = a.cn[c * a.n_cache + i] * av * inv4pi;
      }
      e[3] = bv * inv4pi;
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 8;
      const T dx = e[0] - x[0], dy = e[1] - x[1], dz = e[2] - x[2];
      const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, tiny)));
      const T ri = rsq(r2);
      const T r = r2 * ri, ri2 = ri * ri, ri3 = ri2 * ri;
      const T ev = expo(r);
      const T Q = ev * fma(s, r, T(1));
      const T t = fma(e[4], dx, fma(e[5], dy, e[6] * dz));
      au = fma(Q * t, ri3, fma(e[3] * ev, ri, au));
      if constexpr (GRAD) {
        const T q = Q * ri3 * fma(T(3) * t, ri2, e[3]) + s2 * ev * t * ri3;
        const T m = Q * ri3;
        ag[0] = fma(q, dx, fma(-m, e[4], ag[0]));
        ag[1] = fma(q, dy, fma(-m, e[5], ag[1]));
        ag[2] = fma(q, dz, fma(-m, e[6], ag[2]));
      }
    }
    __syncthreads();
    fold();
  }
  for (int64_t t0 = 0; t0 < a.n_src; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, a.n_src - t0);
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      T* e = ent + tid * 8;
#pragma unroll
      for (int c = 0; c < 3; ++c) e[c] = a.sy[c * a.n_src + j];
      e[3] = -a.ss[j] * inv4pi;  // G s = -s e/(4 pi r); dG/dx s = Q s (x - y)/(4 pi r^3)
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 8;
      const T dx = e[0] - x[0], dy = e[1] - x[1], dz = e[2] - x[2];
      const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, tiny)));
      const T ri = rsq(r2);
      const T r = r2 * ri;
      const T ev = expo(r);
      au = fma(e[3] * ev, ri, au);
      if constexpr (GRAD) {
        const T q = ev * fma(s, r, T(1)) * e[3] * ri * ri * ri;
        ag[0] = fma(q, dx, ag[0]);
        ag[1] = fma(q, dy, ag[1]);
        ag[2] = fma(q, dz, ag[2]);
      }
    }
    __syncthreads();
    fold();
  }
  if (!live) return;
  const double sc = a.scale ? (double)a.scale[k] : 1.0;
  if (a.u) a.u[k] = (T)((a.accumulate ? (double)a.u[k] : 0.0) + sc * tu);
  if (GRAD && a.g) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      a.g[c * a.n_eval + k] = (T)((a.accumulate ? (double)a.g[c * a.n_eval + k] : 0.0) + sc * tg[c]);
  }
}

// Screened gather in 2D (Eqs. 3-6 with the kernels of Appendix A.2):
// G = -K0(z)/(2 pi), z = s r, and with Q = z K1(z), A = a n/(2 pi),
// B = b/(2 pi), t = A.(y-x):
//   a dG/dn - b G = Q t / r^2 + B K0
//   grad = (y-x) [Q (2 t / r^4 + B / r^2) + s^2 K0 t / r^2] - A Q / r^2
// (the Poisson terms times Q plus dG/dn times dQ/dx = s^2 K0 (y - x)); a
// source term s_j adds G s_j and Q dG0/dx s_j = -Q (y-x) s_j/(2 pi r^2).
// One evaluation point per thread; the cache and sources stream through LDS
// tiles as in k_gather.
template <typename T, bool GRAD>
__global__ __launch_bounds__(kGBlock) void k_gather_screened2(GatherArgs<T> a, double sigma) {
  __shared__ T ent[kTile * 8];
  const int tid = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * kGBlock + tid;
  const bool live = k < a.n_eval;
  T x[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) x[c] = live ? a.ex[c * a.n_eval + k] : T(0);
  const T s = (T)sqrt(sigma), s2 = (T)sigma;
  const T inv2pi = (T)(1.0 / (2.0 * kPi));
  const T tiny = sizeof(T) == 4 ? (T)1e-18 : (T)1e-200;
  double tu = 0.0, tg[2] = {0.0, 0.0};
  T au = T(0), ag[2] = {T(0), T(0)};
  auto fold = [&]() {
    tu += (double)au;
    au = T(0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      tg[c] += (double)ag[c];
      ag[c] = T(0);
    }
  };
  const int64_t nc = cache_count(a);
  for (int64_t t0 = 0; t0 < nc; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, nc - t0);
    if (tid < cnt) {
      const int64_t i = t0 + tid;
      T* e = ent + tid * 8;
      const T av = a.ca[i];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        e[c] = a.cx[c * a.n_cache + i];
        e[3 + c] = a.cn[c * a.n_cache + i] * av * inv2pi;
      }
      e[2] = a.cb[i] * inv2pi;
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 8;
      const T dx = e[0] - x[0], dy = e[1] - x[1];
      const T r2 = fma(dx, dx, fma(dy, dy, tiny));
      const T ri2 = T(1) / r2;
      const T r = sqrt(r2);
      T k0, k1;
      bessel_k01t<T>(s * r, k0, k1);
      const T Q = s * r * k1;
      const T t = fma(e[3], dx, e[4] * dy);
      au = fma(Q * t, ri2, fma(e[2], k0, au));
      if constexpr (GRAD) {
        const T q = Q * ri2 * fma(T(2) * t, ri2, e[2]) + s2 * k0 * t * ri2;
        const T m = Q * ri2;
        ag[0] = fma(q, dx, fma(-m, e[3], ag[0]));
        ag[1] = fma(q, dy, fma(-m, e[4], ag[1]));
      }
    }
    __syncthreads();
    fold();
  }
  for (int64_t t0 = 0; t0 < a.n_src; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, a.n_src - t0);
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      T* e = ent + tid * 8;
#pragma unroll
      for (int c = 0; c < 2; ++c) e[c] = a.sy[c * a.n_src + j];
      e[2] = -a.ss[j] * inv2pi;
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 8;
      const T dx = e[0] - x[0], dy = e[1] - x[1];
      const T r2 = fma(dx, dx, fma(dy, dy, tiny));
      const T r = sqrt(r2);
      T k0, k1;
      bessel_k01t<T>(s * r, k0, k1);
      au = fma(e[2], k0, au);
      if constexpr (GRAD) {
        const T q = e[2] * s * r * k1 / r2;
        ag[0] = fma(q, dx, ag[0]);
        ag[1] = fma(q, dy, ag[1]);
      }
    }
    __syncthreads();
    fold();
  }
  if (!live) return;
  const double sc = a.scale ? (double)a.scale[k] : 1.0;
  if (a.u) a.u[k] = (T)((a.accumulate ? (double)a.u[k] : 0.0) + sc * tu);
  if (GRAD && a.g) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
      a.g[c * a.n_eval + k] = (T)((a.accumulate ? (double)a.g[c * a.n_eval + k] : 0.0) + sc * tg[c]);
  }
}

// Transposed gather: cache (or source) points are the parallel dimension and
// the evaluation points with their residuals r_k stream through LDS.
template <typename T>
struct BackArgs {
  int64_t n_eval;
  const T* ex;
  const T* r;
  int64_t n_pts;
  const T* py;   // [D][n_pts] cache or source points
  const T* pn;   // normals (cache) or null (sources)
  T* out_a;      // cache: dL/da ; sources: dL/ds
  T* out_b;      // cache: dL/db
};

template <typename T, int D, bool CACHE>
__global__ __launch_bounds__(kGBlock) void k_gather_back(BackArgs<T> a) {
  __shared__ T ent[kTile * 4];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * (kGBlock * kPPT) + tid;
  T y[kPPT][D], nn[kPPT][D];
  bool live[kPPT];
#pragma unroll
  for (int p = 0; p < kPPT; ++p) {
    const int64_t i = i0 + p * kGBlock;
    live[p] = i < a.n_pts;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      y[p][c] = live[p] ? a.py[c * a.n_pts + i] : T(0);
      nn[p][c] = (CACHE && live[p]) ? a.pn[c * a.n_pts + i] : T(0);
    }
  }
  double ta[kPPT], tb[kPPT];
  T sa[kPPT], sb[kPPT];
#pragma unroll
  for (int p = 0; p < kPPT; ++p) {
    ta[p] = tb[p] = 0.0;
    sa[p] = sb[p] = T(0);
  }
  const T inv2pi = (T)(1.0 / (2.0 * kPi)), inv4pi = (T)(1.0 / (4.0 * kPi));
  const T tiny = sizeof(T) == 4 ? (T)1e-18 : (T)1e-200;
  for (int64_t t0 = 0; t0 < a.n_eval; t0 += kTile) {
    const int cnt = (int)std::min<int64_t>(kTile, a.n_eval - t0);
    if (tid < cnt) {
      const int64_t k = t0 + tid;
      T* e = ent + tid * 4;
#pragma unroll
      for (int c = 0; c < D; ++c) e[c] = a.ex[c * a.n_eval + k];
      e[3] = a.r[k];
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < cnt; ++j) {
      const T* e = ent + j * 4;
      const T rk = e[3];
#pragma unroll
      for (int p = 0; p < kPPT; ++p) {
        T dx[D], r2 = T(0), t = T(0);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          dx[c] = y[p][c] - e[c];  // y - x
          r2 += dx[c] * dx[c];
          t += nn[p][c] * dx[c];
        }
        r2 = fmax(r2, tiny);
        if constexpr (D == 2) {
          const T lr = log_r2(r2) * log_scale<T>();  // ln r^2
          if constexpr (CACHE) {
            sa[p] += rk * t * recip(r2);  // r dG/dn (times 2 pi)
            sb[p] += rk * lr;             // -r G (times -4 pi)
          } else {
            sa[p] += rk * lr;  // r G (times 4 pi)
          }
        } else {
          const T ri = rsq(r2);
          if constexpr (CACHE) {
            sa[p] += rk * t * ri * ri * ri;  // r dG/dn (times 4 pi)
            sb[p] += rk * ri;                // -r G (times 4 pi)
          } else {
            sa[p] += rk * ri;  // r G (times -4 pi)
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
      ta[p] += (double)sa[p];
      tb[p] += (double)sb[p];
      sa[p] = sb[p] = T(0);
    }
  }
#pragma unroll
  for (int p = 0; p < kPPT; ++p) {
    const int64_t i = i0 + p * kGBlock;
    if (!live[p]) continue;
    if constexpr (D == 2) {
      if constexpr (CACHE) {
        if (a.out_a) a.out_a[i] = (T)(ta[p] / (2.0 * kPi));
        if (a.out_b) a.out_b[i] = (T)(-tb[p] / (4.0 * kPi));
      } else {
        if (a.out_a) a.out_a[i] = (T)(ta[p] / (4.0 * kPi));
      }
    } else {
      if constexpr (CACHE) {
        if (a.out_a) a.out_a[i] = (T)(ta[p] / (4.0 * kPi));
        if (a.out_b) a.out_b[i] = (T)(tb[p] / (4.0 * kPi));
      } else {
        if (a.out_a) a.out_a[i] = (T)(-ta[p] / (4.0 * kPi));
      }
    }
  }
  (void)inv2pi;
  (void)inv4pi;
}

// ---------------------------------------------------------------------------
// Basis expansions from exit records
// ---------------------------------------------------------------------------
// One real solid harmonic r^l Y_lm (orthonormal, no Condon-Shortley phase).
__device__ inline double solid_harmonic_lm(int l, int m, const double* x) {
  const int am = m < 0 ? -m : m;
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  double cm = 1.0, sm = 0.0, dfact = 1.0;
  for (int i = 1; i <= am; ++i) {
    const double c2 = cm * x[0] - sm * x[1];
    sm = cm * x[1] + sm * x[0];
    cm = c2;
    dfact *= (2 * i - 1);
  }
  double q = dfact, q1 = 0.0;
  for (int ll = am + 1; ll <= l; ++ll) {
    const double qn = ll == am + 1 ? (2 * am + 1) * x[2] * dfact
                                   : ((2 * ll - 1) * x[2] * q - (ll + am - 1) * r2 * q1) / (ll - am);
    q1 = q;
    q = qn;
  }
  double ratio = 1.0;
  for (int i = l - am + 1; i <= l + am; ++i) ratio /= i;
  double nrm = sqrt((2 * l + 1) / (4.0 * kPi) * ratio);
  if (m == 0) return nrm * q;
  nrm *= 1.4142135623730950488;
  return m > 0 ? nrm * q * cm : nrm * q * sm;
}

__device__ inline double basis_single(const FieldDev& F, int D, int m, const double* x) {
  if (F.kind == 6) return fourier_basis(m, atan2(x[1] - F.param[1], x[0] - F.param[0]));
  int l = 0;
  while ((l + 1) * (l + 1) <= m) ++l;
  return solid_harmonic_lm(l, m - l * l - l, x);
}

template <typename T, int D>
__global__ void k_basis_means(FieldDev F, int nb, int64_t n_cache, int W, const T* ex, const T* w1,
                              const double* xbar, int cv, double* E, double* Fo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_cache * nb) return;
  const int64_t i = t / nb;
  const int m = (int)(t % nb);
  const int64_t total = n_cache * (int64_t)W;
  double base = 0.0;
  if (cv) {
    double xb[D];
    for (int c = 0; c < D; ++c) xb[c] = xbar[c * n_cache + i];
    base = basis_single(F, D, m, xb);
  }
  double se = 0.0, sf = 0.0;
  for (int j = 0; j < W; ++j) {
    const int64_t id = i * W + j;
    double q[D];
    for (int c = 0; c < D; ++c) q[c] = (double)ex[c * total + id];
    // NaN: the walk escaped an open domain, where u = 0 for any data
    const double phi = isnan(q[0]) ? 0.0 : basis_single(F, D, m, q);
    se += phi;
    sf += (double)w1[id] * (phi - base);
  }
  E[i * nb + m] = se / W;
  Fo[i * nb + m] = sf / W;
}

// Basis means by recurrence chains: one thread per (cache point, chain), and
// a chain's basis values come out of one recurrence per walk.  Sums run
// without the basis normalisation, which multiplies the means at the end.
//
// Real solid harmonics of degree <= L (L <= kMaxChainL): chain 0 is order
// m = 0, chain 2m-1 the cosine and chain 2m the sine part of order m; its
// values are l = m..L, Q_l^m(z, r^2) from the three-term recurrence times
// Re or Im (x + i y)^m.
constexpr int kMaxChainL = 8;

__device__ __forceinline__ void sh_chain_values(int m, int part, int L, double dfact, const double* x,
                                                double* v) {
  double az = 1.0;
  if (m > 0) {
    double cm = 1.0, sm = 0.0;
    for (int i = 0; i < m; ++i) {
      const double c2 = cm * x[0] - sm * x[1];
      sm = cm * x[1] + sm * x[0];
      cm = c2;
    }
    az = part ? sm : cm;
  }
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  double q1 = 0.0, q2 = 0.0;
  // guarded rather than broken off, so that every index is a compile-time
  // constant and the arrays stay in registers
#pragma unroll
  for (int k = 0; k <= kMaxChainL; ++k) {
    double q;
    if (k == 0) q = dfact;
    else if (k == 1) q = (2 * m + 1) * x[2] * dfact;
    else q = ((2 * (m + k) - 1) * x[2] * q1 - (2 * m + k - 1) * r2 * q2) * (1.0 / k);
    q2 = q1;
    q1 = q;
    v[k] = k <= L - m ? q * az : 0.0;
  }
}

template <typename T>
__global__ void k_basis_means_sh(int L, int nb, int64_t n_cache, int W, const T* ex, const T* w1,
                                 const double* xbar, int cv, double* E, double* Fo) {
  const int chains = 2 * L + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_cache * chains) return;
  const int64_t i = t / chains;
  const int c = (int)(t % chains);
  const int m = (c + 1) / 2, part = (c > 0 && c % 2 == 0) ? 1 : 0;
  const int n = L - m + 1;
  double dfact = 1.0;  // (2m - 1)!!
  for (int k = 1; k <= m; ++k) dfact *= (2 * k - 1);
  double base[kMaxChainL + 1], se[kMaxChainL + 1], sf[kMaxChainL + 1], v[kMaxChainL + 1];
#pragma unroll
  for (int k = 0; k <= kMaxChainL; ++k) base[k] = se[k] = sf[k] = v[k] = 0.0;
  if (cv) {
    const double xb[3] = {xbar[i], xbar[n_cache + i], xbar[2 * n_cache + i]};
    sh_chain_values(m, part, L, dfact, xb, base);
  }
  const int64_t total = n_cache * (int64_t)W;
  for (int j = 0; j < W; ++j) {
    const int64_t id = i * W + j;
    const double q[3] = {(double)ex[id], (double)ex[total + id], (double)ex[2 * total + id]};
    if (isnan(q[0])) {
      // escaped an open domain: every basis value is 0 at infinity
#pragma unroll
      for (int k = 0; k <= kMaxChainL; ++k) v[k] = 0.0;
    } else {
      sh_chain_values(m, part, L, dfact, q, v);
    }
    const double w = (double)w1[id];
#pragma unroll
    for (int k = 0; k <= kMaxChainL; ++k) {
      se[k] += v[k];
      sf[k] += w * (v[k] - base[k]);
    }
  }
#pragma unroll
  for (int k = 0; k <= kMaxChainL; ++k) {
    if (k >= n) continue;
    const int l = m + k;
    double ratio = 1.0;  // (l-m)!/(l+m)!
    for (int r = l - m + 1; r <= l + m; ++r) ratio /= r;
    double nrm = sqrt((2 * l + 1) / (4.0 * kPi) * ratio);
    if (m > 0) nrm *= 1.4142135623730950488;
    const int idx = part ? l * l + l - m : l * l + l + m;
    E[i * nb + idx] = nrm * se[k] / W;
    Fo[i * nb + idx] = nrm * sf[k] / W;
  }
}

// Fourier basis in the angle about a centre (2D): basis 0 is 1, basis 2j-1
// cos(j theta), basis 2j sin(j theta).  Chunk c takes frequencies 8c+1..8c+8
// (and basis 0 in chunk 0): the first frequency by powering, then rotations
// by theta.
constexpr int kFourierChunk = 8;

// cos and sin of theta from the unit direction to x, and of j0 theta as
// (cos theta + i sin theta)^j0 by binary powering (no transcendental).
__device__ __forceinline__ void fourier_start(int j0, double cx, double cy, const double* x, double& c1,
                                              double& s1, double& c, double& s) {
  const double dx = x[0] - cx, dy = x[1] - cy;
  const double r2 = dx * dx + dy * dy;
  if (r2 > 0.0) {
    const double ri = 1.0 / sqrt(r2);
    c1 = dx * ri;
    s1 = dy * ri;
  } else {
    c1 = 1.0;  // atan2(0, 0) = 0
    s1 = 0.0;
  }
  double pc = c1, ps = s1;
  c = 1.0;
  s = 0.0;
  for (int e = j0; e > 0; e >>= 1) {
    if (e & 1) {
      const double t = c * pc - s * ps;
      s = s * pc + c * ps;
      c = t;
    }
    const double t = pc * pc - ps * ps;
    ps = 2.0 * pc * ps;
    pc = t;
  }
}

template <typename T>
__global__ void k_basis_means_fourier(int nb, double cx, double cy, int64_t n_cache, int W, const T* ex,
                                      const T* w1, const double* xbar, int cv, double* E, double* Fo) {
  const int chunks = std::max(1, (nb / 2 + kFourierChunk - 1) / kFourierChunk);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_cache * (int64_t)chunks) return;
  const int64_t i = t / chunks;
  const int ch = (int)(t % chunks);
  const int j0 = ch * kFourierChunk + 1;
  double bc[kFourierChunk], bs[kFourierChunk];
  double ec[kFourierChunk], es[kFourierChunk], fc[kFourierChunk], fs[kFourierChunk];
#pragma unroll
  for (int k = 0; k < kFourierChunk; ++k) bc[k] = bs[k] = ec[k] = es[k] = fc[k] = fs[k] = 0.0;
  if (cv) {
    const double xb[2] = {xbar[i], xbar[n_cache + i]};
    double c1, s1, c, s;
    fourier_start(j0, cx, cy, xb, c1, s1, c, s);
#pragma unroll
    for (int k = 0; k < kFourierChunk; ++k) {
      bc[k] = c;
      bs[k] = s;
      const double c2 = c * c1 - s * s1;
      s = s * c1 + c * s1;
      c = c2;
    }
  }
  double e0 = 0.0, f0 = 0.0;
  const int64_t total = n_cache * (int64_t)W;
  for (int j = 0; j < W; ++j) {
    const int64_t id = i * W + j;
    const double q[2] = {(double)ex[id], (double)ex[total + id]};
    const double w = (double)w1[id];
    e0 += 1.0;
    f0 += w * (1.0 - (cv ? 1.0 : 0.0));
    double c1, s1, c, s;
    fourier_start(j0, cx, cy, q, c1, s1, c, s);
#pragma unroll
    for (int k = 0; k < kFourierChunk; ++k) {
      ec[k] += c;
      es[k] += s;
      fc[k] += w * (c - bc[k]);
      fs[k] += w * (s - bs[k]);
      const double c2 = c * c1 - s * s1;
      s = s * c1 + c * s1;
      c = c2;
    }
  }
  if (ch == 0) {
    E[i * nb] = e0 / W;
    Fo[i * nb] = f0 / W;
  }
#pragma unroll
  for (int k = 0; k < kFourierChunk; ++k) {
    const int jj = j0 + k;
    if (2 * jj - 1 < nb) {
      E[i * nb + 2 * jj - 1] = ec[k] / W;
      Fo[i * nb + 2 * jj - 1] = fc[k] / W;
    }
    if (2 * jj < nb) {
      E[i * nb + 2 * jj] = es[k] / W;
      Fo[i * nb + 2 * jj] = fs[k] / W;
    }
  }
}

// dL/dtheta_m = sum_i w_i (E_im gA_i + F_im gB_i): partial sums over chunks
// of cache points, then a fixed-order sum of the chunks.
constexpr int kChunk = 1024;
__global__ void k_cache_back_partial(int64_t n, int nb, const double* E, const double* F, const double* w,
                                     const double* ga, const double* gb, double* part) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (m >= nb) return;
  double s = 0.0;
  const int64_t i1 = std::min<int64_t>(n, (c + 1) * kChunk);
  for (int64_t i = c * kChunk; i < i1; ++i) s += w[i] * (E[i * nb + m] * ga[i] + F[i * nb + m] * gb[i]);
  part[c * nb + m] = s;
}
__global__ void k_cache_back_final(int nb, int64_t chunks, const double* part, double* out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nb) return;
  double s = 0.0;
  for (int64_t c = 0; c < chunks; ++c) s += part[c * nb + m];
  out[m] = s;
}

template <typename To>
__global__ void k_eval_fields(int64_t n, int nb, int nf, const double* E, const double* F, const double* w,
                              const double* coef, To* A, To* B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nf) return;
  const int64_t i = t / nf;
  const int f = (int)(t % nf);
  double sa = 0.0, sb = 0.0;
  for (int m = 0; m < nb; ++m) {
    const double c = coef[(int64_t)f * nb + m];
    sa += E[i * nb + m] * c;
    sb += F[i * nb + m] * c;
  }
  A[i * nf + f] = (To)(sa * w[i]);
  B[i * nf + f] = (To)(sb * w[i]);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int check_view(const bvc_cache_view* c, int dim) {
  if (!c) return fail(BVC_EINVAL, "cache view is null");
  if (c->n < 0) return fail(BVC_EINVAL, "cache size is negative");
  if (c->dtype != BVC_F32 && c->dtype != BVC_F64) return fail(BVC_EINVAL, "cache dtype must be F32 or F64");
  if (c->n > 0 && (!c->x || !c->nrm || !c->a || !c->b)) return fail(BVC_EINVAL, "cache arrays are null");
  (void)dim;
  return BVC_OK;
}

int check_sources(const bvc_source_view* s, int dtype) {
  if (!s) return BVC_OK;
  if (s->n < 0) return fail(BVC_EINVAL, "source count is negative");
  if (s->dtype != dtype) return fail(BVC_EINVAL, "source dtype differs from the cache dtype");
  if (s->n > 0 && (!s->y || !s->s)) return fail(BVC_EINVAL, "source arrays are null");
  return BVC_OK;
}

template <typename T, int D>
void launch_gather(const GatherArgs<T>& a, bool grad, bool near, int ppt, bool clamp, hipStream_t st) {
  if (clamp) ppt = kPPT;  // the clamped kernels come in the default shape only
  const int blocks = (int)((a.n_eval + kGBlock * ppt - 1) / (kGBlock * ppt));
  auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kGBlock), 0, st, a); };
  if (clamp) {
    if constexpr (sizeof(T) == 4) {
      if (near) {
        if (grad) go(k_gather<T, D, true, true, kPPT, true>);
        else go(k_gather<T, D, false, true, kPPT, true>);
        return;
      }
    }
    if (grad) go(k_gather<T, D, true, false, kPPT, true>);
    else go(k_gather<T, D, false, false, kPPT, true>);
    return;
  }
  if constexpr (sizeof(T) == 4) {
    if (near) {
      if (grad) {
        if (ppt == 1) go(k_gather<T, D, true, true, 1>);
        else if (ppt == 4) go(k_gather<T, D, true, true, 4>);
        else go(k_gather<T, D, true, true, 2>);
      } else {
        if (ppt == 1) go(k_gather<T, D, false, true, 1>);
        else if (ppt == 4) go(k_gather<T, D, false, true, 4>);
        else go(k_gather<T, D, false, true, 2>);
      }
      return;
    }
  }
  if (grad) {
    if (ppt == 1) go(k_gather<T, D, true, false, 1>);
    else if (ppt == 4) go(k_gather<T, D, true, false, 4>);
    else go(k_gather<T, D, true, false, 2>);
  } else {
    if (ppt == 1) go(k_gather<T, D, false, false, 1>);
    else if (ppt == 4) go(k_gather<T, D, false, false, 4>);
    else go(k_gather<T, D, false, false, 2>);
  }
}

// ---- tile-shape autotuning ------------------------------------------------
// Evaluation points per thread (PPT) of the gather, chosen per problem class by
// bvc_tune_gather and used by every later gather of that class in the process.
struct GatherClass {
  int dim, dtype, grad, near, log_eval, log_cache;
  bool operator<(const GatherClass& o) const {
    return std::tie(dim, dtype, grad, near, log_eval, log_cache) <
           std::tie(o.dim, o.dtype, o.grad, o.near, o.log_eval, o.log_cache);
  }
};
int ilog2(int64_t n) {
  int l = 0;
  while (n > 1) {
    n >>= 1;
    ++l;
  }
  return l;
}
std::mutex g_tune_mu;
std::map<GatherClass, int> g_gather_ppt;

GatherClass gather_class(int dim, int dtype, bool grad, bool near, int64_t n_eval, int64_t n_cache) {
  return GatherClass{dim, dtype, grad ? 1 : 0, near ? 1 : 0, ilog2(n_eval), ilog2(n_cache)};
}
int tuned_ppt(const GatherClass& k) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_gather_ppt.find(k);
  return it == g_gather_ppt.end() ? kPPT : it->second;
}

template <typename T>
int gather_impl(int dim, const bvc_cache_view* c, const bvc_source_view* s, int64_t n_eval, const void* ex, void* u,
                void* g, const void* scale, int accumulate, hipStream_t st, const bvc_gather_params* near = nullptr,
                int ppt = 0, double clamp_c = 0.0, double sigma = 0.0) {
  if (ppt == 0)
    ppt = tuned_ppt(gather_class(dim, sizeof(T) == 4 ? BVC_F32 : BVC_F64, g != nullptr, near != nullptr, n_eval, c->n));
  GatherArgs<T> a{};
  a.n_eval = n_eval;
  a.ex = (const T*)ex;
  a.n_cache = c->n;
  a.cx = (const T*)c->x;
  a.cn = (const T*)c->nrm;
  a.ca = (const T*)c->a;
  a.cb = (const T*)c->b;
  a.n_src = s ? s->n : 0;
  a.sy = s ? (const T*)s->y : nullptr;
  a.ss = s ? (const T*)s->s : nullptr;
  a.u = (T*)u;
  a.g = (T*)g;
  a.scale = (const T*)scale;
  a.accumulate = accumulate;
  if (near) {
    // tau^2 rounded up to FP32 so that every pair closer than tau in FP32 is near
    float t2 = (float)(near->near_tau * near->near_tau);
    if ((double)t2 < near->near_tau * near->near_tau) t2 = nextafterf(t2, INFINITY);
    a.tau2 = (T)t2;
    a.nx = near->near_x;
    a.ncx = near->near_cx;
    a.ncn = near->near_cn;
    a.na = near->near_a;
    a.nb = near->near_b;
    a.near_lead = near->near_lead;
  }
  a.clampc = (T)clamp_c;
  a.clamp64 = clamp_c;
  a.n_dev = c->n_dev;
  const bool clamp = clamp_c > 0.0;
  if (sigma > 0.0) {
    const int blocks = (int)((n_eval + kGBlock - 1) / kGBlock);
    if (dim == 2) {
      if (g) hipLaunchKernelGGL((k_gather_screened2<T, true>), dim3(blocks), dim3(kGBlock), 0, st, a, sigma);
      else hipLaunchKernelGGL((k_gather_screened2<T, false>), dim3(blocks), dim3(kGBlock), 0, st, a, sigma);
    } else {
      if (g) hipLaunchKernelGGL((k_gather_screened3<T, true>), dim3(blocks), dim3(kGBlock), 0, st, a, sigma);
      else hipLaunchKernelGGL((k_gather_screened3<T, false>), dim3(blocks), dim3(kGBlock), 0, st, a, sigma);
    }
    return check_hip(hipGetLastError(), "screened gather launch");
  }
  if (dim == 2) launch_gather<T, 2>(a, g != nullptr, near != nullptr, ppt, clamp, st);
  else launch_gather<T, 3>(a, g != nullptr, near != nullptr, ppt, clamp, st);
  return check_hip(hipGetLastError(), "gather launch");
}

int gather_entry(int32_t dim, const bvc_cache_view* c, const bvc_source_view* s, int64_t n_eval, const void* ex,
                 void* u, void* g, const bvc_gather_params* prm, void* stream, int ppt = 0) {
  if (dim != 2 && dim != 3) return fail(BVC_EINVAL, "dim must be 2 or 3");
  int rc = check_view(c, dim);
  if (rc) return rc;
  rc = check_sources(s, c->dtype);
  if (rc) return rc;
  if (n_eval < 0) return fail(BVC_EINVAL, "n_eval must be >= 0");
  if (prm && (prm->near_lead < 0 || prm->near_lead > n_eval))
    return fail(BVC_EINVAL, "near_lead must lie in [0, n_eval]");
  if (n_eval == 0) return BVC_OK;
  if (!ex || (!u && !g)) return fail(BVC_EINVAL, "null evaluation points or outputs");
  const int acc = prm ? prm->accumulate : 0;
  hipStream_t st = (hipStream_t)stream;
  const bool near = prm && prm->near_tau > 0.0 && c->dtype == BVC_F32 && c->n > 0;
  if (prm && !(prm->near_tau >= 0.0)) return fail(BVC_EINVAL, "near_tau must be >= 0");
  if (near && (!prm->near_x || !prm->near_cx || !prm->near_cn || !prm->near_a || !prm->near_b))
    return fail(BVC_EINVAL, "near_tau > 0 needs the FP64 copies near_x, near_cx, near_cn, near_a, near_b");
  const double clamp_c = prm ? prm->clamp_c : 0.0;
  if (!(clamp_c >= 0.0) || !std::isfinite(clamp_c)) return fail(BVC_EINVAL, "clamp_c must be finite and >= 0");
  const double sigma = prm ? prm->sigma : 0.0;
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(BVC_EINVAL, "sigma must be finite and >= 0");
  if (sigma > 0.0 && (near || clamp_c > 0.0))
    return fail(BVC_EUNSUPPORTED, "the screened gather takes no near field or clamp");
  if (c->dtype == BVC_F32)
    return gather_impl<float>(dim, c, s, n_eval, ex, u, g, nullptr, acc, st, near ? prm : nullptr, ppt, clamp_c,
                              sigma);
  return gather_impl<double>(dim, c, s, n_eval, ex, u, g, nullptr, acc, st, nullptr, ppt, clamp_c, sigma);
}

template <typename T>
int backward_impl(int dim, const bvc_cache_view* c, const bvc_source_view* s, int64_t n_eval, const void* ex,
                  const void* r, void* da, void* db, void* ds, void* dx, hipStream_t st) {
  if (da || db) {
    BackArgs<T> b{n_eval, (const T*)ex, (const T*)r, c->n, (const T*)c->x, (const T*)c->nrm, (T*)da, (T*)db};
    const int blocks = (int)((c->n + kGBlock * kPPT - 1) / (kGBlock * kPPT));
    if (blocks > 0) {
      if (dim == 2) hipLaunchKernelGGL((k_gather_back<T, 2, true>), dim3(blocks), dim3(kGBlock), 0, st, b);
      else hipLaunchKernelGGL((k_gather_back<T, 3, true>), dim3(blocks), dim3(kGBlock), 0, st, b);
    }
  }
  if (ds && s && s->n > 0) {
    BackArgs<T> b{n_eval, (const T*)ex, (const T*)r, s->n, (const T*)s->y, nullptr, (T*)ds, nullptr};
    const int blocks = (int)((s->n + kGBlock * kPPT - 1) / (kGBlock * kPPT));
    if (dim == 2) hipLaunchKernelGGL((k_gather_back<T, 2, false>), dim3(blocks), dim3(kGBlock), 0, st, b);
    else hipLaunchKernelGGL((k_gather_back<T, 3, false>), dim3(blocks), dim3(kGBlock), 0, st, b);
  }
  if (dx) {
    int rc = gather_impl<T>(dim, c, s, n_eval, ex, nullptr, dx, r, 0, st);
    if (rc) return rc;
  }
  return check_hip(hipGetLastError(), "gather backward launch");
}

// Many scenes in one launch: block t takes tile t of the batch's
// concatenated tile list and gathers it against its own scene's cache.
template <int D>
__global__ __launch_bounds__(kGBlock) void k_batch_gather(BatchDev b) {
  __shared__ float ent[kTile * 8];
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = b.n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.scenes[mid].tile_off <= tile) lo = mid;
    else hi = mid - 1;
  }
  const BatchSceneDev& s = b.scenes[lo];
  GatherArgs<float> a{};
  a.n_eval = s.n_eval;
  a.ex = s.ex;
  a.n_cache = s.n_cache;
  a.cx = s.cx;
  a.cn = s.cn;
  a.ca = b.a + s.cache_off;
  a.cb = b.b + s.cache_off;
  a.n_src = 0;
  a.u = s.u;
  a.g = nullptr;
  a.scale = nullptr;
  a.accumulate = 0;
  gather_block<float, D, false>(a, tile - s.tile_off, ent);
}

}  // namespace

int launch_batch_gather(const BatchDev& b, hipStream_t st) {
  if (b.total_tiles <= 0) return BVC_OK;
  if (b.dim == 2)
    hipLaunchKernelGGL(k_batch_gather<2>, dim3((unsigned)b.total_tiles), dim3(kGBlock), 0, st, b);
  else
    hipLaunchKernelGGL(k_batch_gather<3>, dim3((unsigned)b.total_tiles), dim3(kGBlock), 0, st, b);
  return check_hip(hipGetLastError(), "batch gather launch");
}

}  // namespace bvc

using namespace bvc;

extern "C" {

int bvc_gather_u(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources, int64_t n_eval,
                 const void* eval_x, void* u, const bvc_gather_params* params, void* stream) {
  if (!u) return fail(BVC_EINVAL, "u is null");
  return gather_entry(dim, cache, sources, n_eval, eval_x, u, nullptr, params, stream);
}

int bvc_gather_grad(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources, int64_t n_eval,
                    const void* eval_x, void* u, void* grad, const bvc_gather_params* params, void* stream) {
  if (!grad) return fail(BVC_EINVAL, "grad is null");
  return gather_entry(dim, cache, sources, n_eval, eval_x, u, grad, params, stream);
}

int bvc_tune_gather(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources, int64_t n_eval,
                    const void* eval_x, void* u, void* grad, const bvc_gather_params* params, int32_t reps,
                    int32_t* ppt_out, void* stream) {
  if (reps < 1) return fail(BVC_EINVAL, "reps must be >= 1");
  if (!u && !grad) return fail(BVC_EINVAL, "u and grad are null");
  if (params && params->accumulate) return fail(BVC_EINVAL, "tuning runs the gather repeatedly: accumulate must be 0");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = check_hip(hipEventCreate(&e0), "tune event");
  if (!rc) rc = check_hip(hipEventCreate(&e1), "tune event");
  const int cand[3] = {1, 2, 4};
  float best_ms = INFINITY;
  int best = kPPT;
  for (int ci = 0; ci < 3 && !rc; ++ci) {
    rc = gather_entry(dim, cache, sources, n_eval, eval_x, u, grad, params, stream, cand[ci]);  // warm-up
    if (!rc) rc = check_hip(hipEventRecord(e0, st), "tune event");
    for (int r = 0; r < reps && !rc; ++r)
      rc = gather_entry(dim, cache, sources, n_eval, eval_x, u, grad, params, stream, cand[ci]);
    if (!rc) rc = check_hip(hipEventRecord(e1, st), "tune event");
    if (!rc) rc = check_hip(hipEventSynchronize(e1), "tune sync");
    float ms = 0;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "tune time");
    if (!rc && ms < best_ms) {
      best_ms = ms;
      best = cand[ci];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  const bool near = params && params->near_tau > 0.0 && cache->dtype == BVC_F32 && cache->n > 0;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_gather_ppt[gather_class(dim, cache->dtype, grad != nullptr, near, n_eval, cache->n)] = best;
  }
  if (ppt_out) *ppt_out = best;
  // leave the outputs as a gather with the chosen shape writes them
  return gather_entry(dim, cache, sources, n_eval, eval_x, u, grad, params, stream, best);
}

int bvc_gather_backward(int32_t dim, const bvc_cache_view* cache, const bvc_source_view* sources, int64_t n_eval,
                        const void* eval_x, const void* dL_du, void* dL_da, void* dL_db, void* dL_ds, void* dL_dx,
                        void* stream) {
  if (dim != 2 && dim != 3) return fail(BVC_EINVAL, "dim must be 2 or 3");
  int rc = check_view(cache, dim);
  if (rc) return rc;
  if (cache->n_dev) return fail(BVC_EUNSUPPORTED, "the gather adjoint takes a host cache count");
  rc = check_sources(sources, cache->dtype);
  if (rc) return rc;
  if (n_eval < 0) return fail(BVC_EINVAL, "n_eval must be >= 0");
  if (n_eval > 0 && (!eval_x || !dL_du)) return fail(BVC_EINVAL, "null evaluation points or residuals");
  hipStream_t st = (hipStream_t)stream;
  // with no evaluation points every adjoint is zero
  if (n_eval == 0) {
    const size_t es = cache->dtype == BVC_F32 ? 4 : 8;
    int rc = BVC_OK;
    if (dL_da && cache->n) rc = zero_async(dL_da, cache->n * es, st);
    if (!rc && dL_db && cache->n) rc = zero_async(dL_db, cache->n * es, st);
    if (!rc && dL_ds && sources && sources->n) rc = zero_async(dL_ds, sources->n * es, st);
    return rc;
  }
  if (cache->dtype == BVC_F32)
    return backward_impl<float>(dim, cache, sources, n_eval, eval_x, dL_du, dL_da, dL_db, dL_ds, dL_dx, st);
  return backward_impl<double>(dim, cache, sources, n_eval, eval_x, dL_du, dL_da, dL_db, dL_ds, dL_dx, st);
}

int bvc_basis_means(const bvc_field* basis, int32_t dim, int64_t n_cache, int32_t W, int32_t dtype,
                    const void* rec_exit, const void* rec_w1, const double* xbar, int32_t cv, double* E, double* F,
                    void* stream) {
  if (!basis) return fail(BVC_EINVAL, "basis is null");
  if (!((basis->kind == 6 && dim == 2) || (basis->kind == 5 && dim == 3)))
    return fail(BVC_EINVAL, "basis must be FOURIER_2D (2D) or SOLID_HARMONICS_3D (3D)");
  const int nb = basis->n_coef;
  if (nb < 1) return fail(BVC_EINVAL, "basis size must be >= 1");
  if (basis->kind == 5) {
    const int L = (int)basis->param[0];
    if (nb != (L + 1) * (L + 1)) return fail(BVC_EINVAL, "solid harmonics need (L+1)^2 terms");
  }
  if (n_cache < 0 || W < 1) return fail(BVC_EINVAL, "bad sizes");
  if (dtype != BVC_F32 && dtype != BVC_F64) return fail(BVC_EINVAL, "dtype must be F32 or F64");
  if (n_cache == 0) return BVC_OK;
  if (!rec_exit || !rec_w1 || !E || !F || (cv && !xbar)) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const bool f32 = dtype == BVC_F32;
  if (basis->kind == 6) {
    const int chunks = std::max(1, (nb / 2 + kFourierChunk - 1) / kFourierChunk);
    const int64_t threads = n_cache * (int64_t)chunks;
    const int blocks = (int)((threads + 255) / 256);
    const double cx = basis->param[0], cy = basis->param[1];
    if (f32)
      hipLaunchKernelGGL((k_basis_means_fourier<float>), dim3(blocks), dim3(256), 0, st, nb, cx, cy, n_cache, W,
                         (const float*)rec_exit, (const float*)rec_w1, xbar, cv, E, F);
    else
      hipLaunchKernelGGL((k_basis_means_fourier<double>), dim3(blocks), dim3(256), 0, st, nb, cx, cy, n_cache, W,
                         (const double*)rec_exit, (const double*)rec_w1, xbar, cv, E, F);
  } else if ((int)basis->param[0] <= kMaxChainL) {
    const int L = (int)basis->param[0];
    const int64_t threads = n_cache * (int64_t)(2 * L + 1);
    const int blocks = (int)((threads + 255) / 256);
    if (f32)
      hipLaunchKernelGGL((k_basis_means_sh<float>), dim3(blocks), dim3(256), 0, st, L, nb, n_cache, W,
                         (const float*)rec_exit, (const float*)rec_w1, xbar, cv, E, F);
    else
      hipLaunchKernelGGL((k_basis_means_sh<double>), dim3(blocks), dim3(256), 0, st, L, nb, n_cache, W,
                         (const double*)rec_exit, (const double*)rec_w1, xbar, cv, E, F);
  } else {
    // degrees beyond the chain kernel: one thread per (cache point, basis)
    const int64_t total = n_cache * nb;
    const int blocks = (int)((total + 255) / 256);
    FieldDev Fd = to_dev(*basis);
    if (f32)
      hipLaunchKernelGGL((k_basis_means<float, 3>), dim3(blocks), dim3(256), 0, st, Fd, nb, n_cache, W,
                         (const float*)rec_exit, (const float*)rec_w1, xbar, cv, E, F);
    else
      hipLaunchKernelGGL((k_basis_means<double, 3>), dim3(blocks), dim3(256), 0, st, Fd, nb, n_cache, W,
                         (const double*)rec_exit, (const double*)rec_w1, xbar, cv, E, F);
  }
  return check_hip(hipGetLastError(), "basis means launch");
}

int64_t bvc_cache_backward_scratch_doubles(int64_t n_cache, int32_t nb) {
  return ((n_cache + kChunk - 1) / kChunk) * (int64_t)nb;
}

int bvc_cache_backward(int64_t n_cache, int32_t nb, const double* E, const double* F, const double* w,
                       const double* dL_da, const double* dL_db, double* scratch, double* dL_dtheta,
                       void* stream) {
  if (n_cache < 0 || nb < 1) return fail(BVC_EINVAL, "bad sizes");
  if (!dL_dtheta) return fail(BVC_EINVAL, "dL_dtheta is null");
  hipStream_t st = (hipStream_t)stream;
  if (n_cache == 0) return zero_async(dL_dtheta, nb * sizeof(double), st);
  if (!E || !F || !w || !dL_da || !dL_db || !scratch) return fail(BVC_EINVAL, "null argument");
  const int64_t chunks = (n_cache + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_cache_back_partial, dim3((nb + 63) / 64, (unsigned)chunks), dim3(64), 0, st, n_cache, nb, E, F,
                     w, dL_da, dL_db, scratch);
  hipLaunchKernelGGL(k_cache_back_final, dim3((nb + 63) / 64), dim3(64), 0, st, nb, chunks, scratch, dL_dtheta);
  return check_hip(hipGetLastError(), "cache backward launch");
}

int bvc_eval_fields(int64_t n_cache, int32_t nb, int32_t n_fields, const double* E, const double* F, const double* w,
                    const double* coef, int32_t dtype_out, void* A, void* B, void* stream) {
  if (n_cache < 0 || nb < 1 || n_fields < 1) return fail(BVC_EINVAL, "bad sizes");
  if (dtype_out != BVC_F32 && dtype_out != BVC_F64) return fail(BVC_EINVAL, "dtype must be F32 or F64");
  if (n_cache == 0) return BVC_OK;
  if (!E || !F || !w || !coef || !A || !B) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const int64_t total = n_cache * n_fields;
  const int blocks = (int)((total + 255) / 256);
  if (dtype_out == BVC_F32)
    hipLaunchKernelGGL(k_eval_fields<float>, dim3(blocks), dim3(256), 0, st, n_cache, nb, n_fields, E, F, w, coef,
                       (float*)A, (float*)B);
  else
    hipLaunchKernelGGL(k_eval_fields<double>, dim3(blocks), dim3(256), 0, st, n_cache, nb, n_fields, E, F, w, coef,
                       (double*)A, (double*)B);
  return check_hip(hipGetLastError(), "eval fields launch");
}

}  // extern "C"
