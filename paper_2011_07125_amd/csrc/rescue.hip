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
#include "common.h"
#include "kernels.h"

namespace fn {

// Order-preserving image of a key: a larger float gives a larger unsigned
// integer, equal floats (-0 and +0 included) the same one, and NaN (an
// undefined error scale) the largest of all.
__device__ inline uint32_t rank_bits(float k) {
  if (k != k) return 0xffffffffu;
  const uint32_t b = k == 0.0f ? 0u : __float_as_uint(k);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// exclusive prefix sum of one value per thread (blockDim.x = 1024) in LDS
__device__ inline int block_exclusive_scan(int v, int* sc) {
  const int tid = threadIdx.x;
  sc[tid] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int t = tid >= off ? sc[tid - off] : 0;
    __syncthreads();
    sc[tid] += t;
    __syncthreads();
  }
  const int incl = sc[tid];
  __syncthreads();
  return incl - v;
}

// One workgroup per segment of at most 8192 walkers: the k walkers of
// largest key (k_seg in every full segment, k_last in the last one), ties
// broken by the smaller index, written in index order at seg * k_seg.
// The k_seg-th largest key is found by a radix select on its bytes (most
// significant first, one 256-bin histogram per byte); the walkers above it,
// and the first of those equal to it, are then compacted in index order.
__global__ __launch_bounds__(1024) void select_top_kernel(const float* key, int W, int seg_len, int k_seg,
                                                          int k_last, int32_t* idx) {
  __shared__ uint32_t Ks[8192];
  __shared__ int hist[256];
  __shared__ int sc[1024];
  __shared__ int s_pick[2];
  const int seg = blockIdx.x, tid = threadIdx.x;
  const int base = seg * seg_len;
  const int len = min(seg_len, W - base);
  const int k = seg == (int)gridDim.x - 1 ? k_last : k_seg;  // k <= len (host)
  for (int i = tid; i < len; i += 1024) Ks[i] = rank_bits(key[base + i]);
  __syncthreads();
  uint32_t prefix = 0, mask = 0;
  int need = k;  // still to take among the keys that match prefix
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    for (int i = tid; i < len; i += 1024) {
      const uint32_t u = Ks[i];
      if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1);
    }
    __syncthreads();
    if (tid < 64) {
      // the byte value d of the need-th largest key: the first bin from
      // the top whose count reaches need together with the bins above it
      // (bin 0 if none does).  Lane l holds bins 255 - 4 l - j, j < 4; a
      // scan over the wavefront gives the count above each lane's bins.
      int h[4], tot = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) tot += h[j] = hist[255 - 4 * tid - j];
      int inc = tot;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(inc, off, 64);
        if (tid >= off) inc += t;
      }
      int above = inc - tot;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d = 255 - 4 * tid - j;
        if (above < need && (d == 0 || above + h[j] >= need)) {
          s_pick[0] = d;
          s_pick[1] = need - above;
        }
        above += h[j];
      }
    }
    __syncthreads();
    prefix |= (uint32_t)s_pick[0] << shift;
    mask |= 0xffu << shift;
    need = s_pick[1];
    __syncthreads();
  }
  // prefix is the k-th largest key; take every key above it and the
  // first `need` keys equal to it.  Thread t owns indices [t per, (t+1) per).
  const int per = (len + 1023) / 1024;
  const int i0 = tid * per, i1 = min(i0 + per, len);
  int n_gt = 0, n_eq = 0;
  for (int i = i0; i < i1; ++i) {
    const uint32_t u = Ks[i];
    n_gt += u > prefix;
    n_eq += u == prefix;
  }
  int gt = block_exclusive_scan(n_gt, sc);
  int eq = block_exclusive_scan(n_eq, sc);
  int32_t* out = idx + (size_t)seg * k_seg;
  for (int i = i0; i < i1; ++i) {
    const uint32_t u = Ks[i];
    if (u > prefix) {
      out[gt + min(eq, need)] = base + i;
      ++gt;
    } else if (u == prefix) {
      if (eq < need) out[gt + eq] = base + i;
      ++eq;
    }
  }
}

hipError_t launch_select_top(const float* key, int W, int seg_len, int k_seg, int k_last, int32_t* idx,
                             hipStream_t s) {
  if (W <= 0 || k_seg <= 0) return hipSuccess;
  if (seg_len <= 0 || seg_len > 8192 || k_seg > seg_len) return hipErrorInvalidValue;
  const int n_seg = (W + seg_len - 1) / seg_len;
  if (k_last < 1 || k_last > W - (n_seg - 1) * seg_len || k_last > k_seg) return hipErrorInvalidValue;
  hipLaunchKernelGGL(select_top_kernel, dim3(n_seg), dim3(1024), 0, s, key, W, seg_len, k_seg, k_last, idx);
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
