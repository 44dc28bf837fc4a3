// Selection, gathering and scattering for the float64 re-evaluation of the
// walkers whose local energy is most exposed to rounding.
//
// Near a node of psi = sum_k P_k (Eq. (4)) the determinant terms cancel,
// and the rounding errors of the reduced-precision network are amplified
// by kappa = max_k |P_k| / |psi| in log|psi| and more strongly in its
// derivatives; a nearly singular orbital matrix amplifies the rounding of
// its own factorisation by its condition number.  The local energy of
// those walkers carries errors many orders above the arithmetic's unit
// roundoff.  The combination kernel writes the log of each walker's error
// scale (kappa, the kinetic-energy magnitude and the conditioning weighted
// by the precision of the determinant arithmetic); the walkers with the
// largest key in each segment of the batch are gathered, evaluated again
// entirely in float64, and their outputs scattered back over the
// reduced-precision ones.
#include <climits>

#include "common.h"
#include "kernels.h"

namespace fn {

// "a comes before b": larger key first, then smaller index
__device__ inline bool before(float ka, int ia, float kb, int ib) { return ka > kb || (ka == kb && ia < ib); }

// one workgroup per segment: bitonic sort of (key, index) pairs in LDS over
// np = next power of two >= segment length, padding keys -inf
__global__ __launch_bounds__(1024) void select_top_kernel(const float* key, int W, int seg_len, int np, int k_seg,
                                                          int32_t* idx) {
  extern __shared__ __attribute__((aligned(16))) char sm[];
  float* Ks = reinterpret_cast<float*>(sm);
  int* Is = reinterpret_cast<int*>(sm + (size_t)np * 4);
  const int seg = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
  const int base = seg * seg_len;
  const int len = min(seg_len, W - base);
  for (int i = tid; i < np; i += bs) {
    if (i < len) {
      float k = key[base + i];
      Ks[i] = k != k ? INFINITY : k;  // NaN ranks first
      Is[i] = base + i;
    } else {
      Ks[i] = -INFINITY;
      Is[i] = INT_MAX;
    }
  }
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < np / 2; i += bs) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride is a power of two
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const float klo = Ks[lo], khi = Ks[hi];
        const int ilo = Is[lo], ihi = Is[hi];
        const bool sw = up ? before(khi, ihi, klo, ilo) : before(klo, ilo, khi, ihi);
        if (sw) {
          Ks[lo] = khi;
          Ks[hi] = klo;
          Is[lo] = ihi;
          Is[hi] = ilo;
        }
      }
      __syncthreads();
    }
  }
  // a segment shorter than k_seg repeats its first walker (same result twice)
  for (int r = tid; r < k_seg; r += bs) idx[(size_t)seg * k_seg + r] = Is[r < len ? r : 0];
}

hipError_t launch_select_top(const float* key, int W, int seg_len, int k_seg, int32_t* idx, hipStream_t s) {
  if (W <= 0 || k_seg <= 0) return hipSuccess;
  if (seg_len <= 0 || seg_len > 8192 || k_seg > seg_len) return hipErrorInvalidValue;
  int np = 1;
  while (np < seg_len) np <<= 1;
  const int n_seg = (W + seg_len - 1) / seg_len;
  const int threads = np / 2 < 1024 ? (np / 2 < 64 ? 64 : np / 2) : 1024;
  hipLaunchKernelGGL(select_top_kernel, dim3(n_seg), dim3(threads), (size_t)np * 8, s, key, W, seg_len, np, k_seg,
                     idx);
  return hipGetLastError();
}

__global__ void gather_walkers_kernel(const float* pos, const int32_t* idx, int R, int n3, float* pos_r) {
  const int64_t total = (int64_t)R * n3;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n3;
    const int c = (int)(e - r * n3);
    pos_r[e] = pos[(int64_t)idx[r] * n3 + c];
  }
}

hipError_t launch_gather_walkers(const float* pos, const int32_t* idx, int R, int n3, float* pos_r, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int64_t total = (int64_t)R * n3;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(gather_walkers_kernel, dim3(grid), dim3(256), 0, s, pos, idx, R, n3, pos_r);
  return hipGetLastError();
}

struct ScatterSet {
  float* out[8];
  const float* src[8];
  int n;
};

__global__ void scatter_results_kernel(const int32_t* idx, int R, ScatterSet set) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int32_t w = idx[r];
  for (int q = 0; q < set.n; ++q) set.out[q][w] = set.src[q][r];
}

hipError_t launch_scatter_results(const int32_t* idx, int R, float* const* outs, const float* const* srcs, int n_out,
                                  hipStream_t s) {
  if (R <= 0) return hipSuccess;
  ScatterSet set;
  set.n = 0;
  for (int q = 0; q < n_out && q < 8; ++q) {
    if (!outs[q]) continue;
    set.out[set.n] = outs[q];
    set.src[set.n] = srcs[q];
    ++set.n;
  }
  if (set.n == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_results_kernel, dim3((R + 255) / 256), dim3(256), 0, s, idx, R, set);
  return hipGetLastError();
}

}  // namespace fn
