// Multi-RHS gather: many boundary-data fields share one set of walks, so the
// gather becomes U[K x F] = Kmat[K x 2N] * [A; B][2N x F] with the kernel
// matrix Kmat = [dG/dn | -G] generated on the fly (never stored).
//
// BVC_F32: FP32 FMA, one thread per evaluation point and F accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bvc_device.hpp"

namespace bvc {

int gather_multi_mfma(int dim, int64_t n_cache, const float* cx, const float* cn, int nf, const float* A,
                      const float* B, int64_t n_eval, const float* ex, float* U, void* pack, hipStream_t st);
int64_t gather_multi_pack_bytes(int64_t n_cache);

namespace {

constexpr int kMBlock = 128;
constexpr int kMTile = 64;

template <int D, int NF>
__global__ __launch_bounds__(kMBlock) void k_gather_multi_f32(int64_t n_cache, const float* cx, const float* cn,
                                                              const float* A, const float* B, int64_t n_eval,
                                                              const float* ex, float* U) {
  __shared__ float geo[kMTile][8];
  __shared__ float coef[kMTile][2 * NF];
  const int tid = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * kMBlock + tid;
  float x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = k < n_eval ? ex[c * n_eval + k] : 0.f;
  float acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0.f;
  const float c2 = (float)(1.0 / (2.0 * kPi)), c4 = (float)(1.0 / (4.0 * kPi));
  for (int64_t t0 = 0; t0 < n_cache; t0 += kMTile) {
    const int cnt = (int)std::min<int64_t>(kMTile, n_cache - t0);
    for (int q = tid; q < cnt; q += kMBlock) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        geo[q][c] = cx[c * n_cache + t0 + q];
        geo[q][4 + c] = cn[c * n_cache + t0 + q];
      }
    }
    for (int q = tid; q < cnt * NF; q += kMBlock) {
      const int i = q / NF, f = q % NF;
      coef[i][f] = A[(t0 + i) * NF + f];
      coef[i][NF + f] = B[(t0 + i) * NF + f];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      float r2 = 0.f, t = 0.f, dx[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        dx[c] = geo[j][c] - x[c];
        r2 += dx[c] * dx[c];
        t += geo[j][4 + c] * dx[c];
      }
      r2 = fmaxf(r2, 1e-18f);
      float kd, kg;  // dG/dn and -G
      if constexpr (D == 2) {
        kd = c2 * t * __builtin_amdgcn_rcpf(r2);
        kg = -c2 * 0.5f * 0.69314718f * __log2f(r2);
      } else {
        const float ri = __builtin_amdgcn_rsqf(r2);
        kd = c4 * t * ri * ri * ri;
        kg = c4 * ri;
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f] += kd * coef[j][f] + kg * coef[j][NF + f];
    }
    __syncthreads();
  }
  if (k < n_eval) {
#pragma unroll
    for (int f = 0; f < NF; ++f) U[k * NF + f] = acc[f];
  }
}

}  // namespace
}  // namespace bvc

using namespace bvc;

extern "C" size_t bvc_gather_multi_workspace_bytes(int64_t n_cache, int32_t precision) {
  if (n_cache < 0) return 0;
  return precision == BVC_SPLIT_BF16 ? (size_t)gather_multi_pack_bytes(n_cache) : 0;
}

extern "C" int bvc_gather_multi(int32_t dim, int64_t n_cache, const float* cx, const float* cn, int32_t n_fields,
                                const float* A, const float* B, int64_t n_eval, const float* eval_x, float* U,
                                int32_t precision, void* workspace, size_t ws_bytes, void* stream) {
  if (dim != 2 && dim != 3) return fail(BVC_EINVAL, "dim must be 2 or 3");
  if (n_cache < 0 || n_eval < 0) return fail(BVC_EINVAL, "sizes must be >= 0");
  if (n_fields != 32 && n_fields != 64) return fail(BVC_EUNSUPPORTED, "n_fields must be 32 or 64");
  if (precision != BVC_F32 && precision != BVC_SPLIT_BF16) return fail(BVC_EINVAL, "precision must be F32 or SPLIT_BF16");
  if (n_eval == 0) return BVC_OK;
  if (!eval_x || !U || (n_cache > 0 && (!cx || !cn || !A || !B))) return fail(BVC_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (precision == BVC_SPLIT_BF16) {
    if (!workspace || ws_bytes < (size_t)gather_multi_pack_bytes(n_cache))
      return fail(BVC_EINVAL, "split-BF16 workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(BVC_EINVAL, "workspace must be 256-byte aligned");
    return gather_multi_mfma(dim, n_cache, cx, cn, n_fields, A, B, n_eval, eval_x, U, workspace, st);
  }
  const int blocks = (int)((n_eval + kMBlock - 1) / kMBlock);
  if (dim == 2) {
    if (n_fields == 32)
      hipLaunchKernelGGL((k_gather_multi_f32<2, 32>), dim3(blocks), dim3(kMBlock), 0, st, n_cache, cx, cn, A, B, n_eval,
                         eval_x, U);
    else
      hipLaunchKernelGGL((k_gather_multi_f32<2, 64>), dim3(blocks), dim3(kMBlock), 0, st, n_cache, cx, cn, A, B, n_eval,
                         eval_x, U);
  } else {
    if (n_fields == 32)
      hipLaunchKernelGGL((k_gather_multi_f32<3, 32>), dim3(blocks), dim3(kMBlock), 0, st, n_cache, cx, cn, A, B, n_eval,
                         eval_x, U);
    else
      hipLaunchKernelGGL((k_gather_multi_f32<3, 64>), dim3(blocks), dim3(kMBlock), 0, st, n_cache, cx, cn, A, B, n_eval,
                         eval_x, U);
  }
  return check_hip(hipGetLastError(), "gather_multi launch");
}
