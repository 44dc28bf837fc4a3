// The small kernels of one VMC iteration that are not evaluation passes:
// statistics and clipping of the local energies, running averages of the
// KFAC factors, and the norm-constrained parameter step.
//
// Statistics of the local energies (one workgroup; the batch of one GPU is
// thousands of walkers, read a few times from L2):
//   * mean and population variance in float64 (two passes, fixed order);
//   * the median, the mean of the order statistics (W - 1) / 2 and W / 2,
//     each found by a radix select over an order-preserving 32-bit image of
//     the float32 energies: four 8-bit digit passes, each a 256-bin LDS
//     histogram of the keys that match the digits chosen so far;
//   * the mean absolute deviation from the median and the clipped energies
//     min(max(E, med - s tv), med + s tv), in float64 before rounding;
//   * the gradient cotangents and the KFAC batch weights of the walkers;
// all over the walkers whose local energy is finite.
#include "common.h"
#include "kernels.h"

namespace fn {

constexpr int kStatThreads = 1024;

// float32 -> uint32 with the order of the floats (negative values reversed)
__device__ inline uint32_t order_key(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// sum over the workgroup in a fixed order: per-wave butterfly, then the
// wave partials in index order
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kStatThreads / 64; ++i) t += red[i];
  return t;
}

// the k-th smallest (0-based) of the finite values of e[0..W)
__device__ float select_kth(const float* e, int W, uint32_t k, uint32_t* hist, uint32_t* bc) {
  uint32_t prefix = 0, mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += kStatThreads) hist[b] = 0;
    __syncthreads();
    for (int w = threadIdx.x; w < W; w += kStatThreads) {
      if (!isfinite(e[w])) continue;
      const uint32_t key = order_key(e[w]);
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t cum = 0, sel = 255;
      for (uint32_t b = 0; b < 256; ++b) {
        if (cum + hist[b] > k) {
          sel = b;
          break;
        }
        cum += hist[b];
      }
      bc[0] = sel;
      bc[1] = k - cum;
    }
    __syncthreads();
    prefix |= bc[0] << shift;
    mask |= 255u << shift;
    k = bc[1];
    __syncthreads();
  }
  return key_float(prefix);
}

// Walkers whose local energy is not finite (an exact node, coincident
// particles) are left out of the iteration: every statistic runs over the
// W_f finite energies, the gradient cotangents are
//   cot_w = 2 (E~_w - mean E~) / W_f   (0 for the others)
// and the KFAC batch weights 1 / W_f (0 for the others).  With no finite
// energy every cotangent and weight is 0 and the statistics are NaN.
__global__ __launch_bounds__(kStatThreads) void train_energy_stats_kernel(const float* e, const int32_t* n_acc, int W,
                                                                          int n_steps, double clip_scale,
                                                                          float* e_clip, float* cot, float* wts,
                                                                          double* stats) {
  __shared__ double red[kStatThreads / 64];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t bc[2];
  const int tid = threadIdx.x;
  double s = 0.0, nf = 0.0;
  for (int w = tid; w < W; w += kStatThreads)
    if (isfinite(e[w])) {
      s += (double)e[w];
      nf += 1.0;
    }
  const double Wf = block_sum(nf, red);
  const double mean = block_sum(s, red) / Wf;
  double v = 0.0;
  for (int w = tid; w < W; w += kStatThreads)
    if (isfinite(e[w])) {
      const double d = (double)e[w] - mean;
      v += d * d;
    }
  const double var = block_sum(v, red) / Wf;
  double a = 0.0;
  for (int w = tid; w < W; w += kStatThreads) a += (double)n_acc[w];
  const double acc = block_sum(a, red);
  const uint32_t nfi = (uint32_t)Wf;
  double med = NAN;
  if (nfi > 0) {
    const float lo_k = select_kth(e, W, (nfi - 1) / 2, hist, bc);
    const float hi_k = select_kth(e, W, nfi / 2, hist, bc);
    med = 0.5 * ((double)lo_k + (double)hi_k);
  }
  double t = 0.0;
  for (int w = tid; w < W; w += kStatThreads)
    if (isfinite(e[w])) t += fabs((double)e[w] - med);
  const double tv = block_sum(t, red) / Wf;
  const bool clip = clip_scale > 0.0;
  const double lo = med - clip_scale * tv, hi = med + clip_scale * tv;
  double c = 0.0;
  for (int w = tid; w < W; w += kStatThreads) {
    const double x = (double)e[w];
    const float y = clip && isfinite(e[w]) ? (float)(x < lo ? lo : (x > hi ? hi : x)) : e[w];
    e_clip[w] = y;
    if (isfinite(e[w])) c += (double)y;
  }
  const double cmean = block_sum(c, red) / Wf;
  for (int w = tid; w < W; w += kStatThreads) {
    const bool f = isfinite(e[w]);
    cot[w] = f ? (float)(2.0 * ((double)e_clip[w] - cmean) / Wf) : 0.0f;
    wts[w] = f ? (float)(1.0 / Wf) : 0.0f;
  }
  if (tid == 0) {
    stats[0] = mean;
    stats[1] = var;
    stats[2] = n_steps > 0 ? acc / ((double)W * (double)n_steps) : 0.0;
    stats[3] = med;
    stats[4] = tv;
    stats[5] = cmean;
    stats[8] = (double)W - Wf;
  }
}

hipError_t launch_train_energy_stats(const float* e, const int32_t* n_acc, int W, int n_steps, double clip_scale,
                                     float* e_clip, float* cot, float* wts, double* stats, hipStream_t s) {
  if (W <= 0) return hipSuccess;
  hipLaunchKernelGGL(train_energy_stats_kernel, dim3(1), dim3(kStatThreads), 0, s, e, n_acc, W, n_steps, clip_scale,
                     e_clip, cot, wts, stats);
  return hipGetLastError();
}

// y = a x + b y; y = a x when b = 0 (y is then not read, so it may hold
// anything, NaN included)
__global__ void lincomb_kernel(float* y, const float* x, float a, float b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float ax = a * x[i];
    y[i] = b == 0.0f ? ax : fmaf(b, y[i], ax);
  }
}

hipError_t launch_lincomb(float* y, const float* x, float a, float b, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid), dim3(256), 0, s, y, x, a, b, n);
  return hipGetLastError();
}

// <X, g> in float64: per-block partials in a fixed order, then one block
// sums them and derives the step length lr min(1, sqrt(C / (lr^2 <X, g>)))
constexpr int kDotBlocks = 256, kDotThreads = 256;

__global__ __launch_bounds__(kDotThreads) void dot_partial_kernel(const float* x, const float* g, int64_t n,
                                                                  double* part) {
  __shared__ double sh[kDotThreads];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads)
    v += (double)x[i] * (double)g[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kDotThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kDotBlocks) void step_length_kernel(const double* part, double lr, double norm_constraint,
                                                                 double* stats) {
  __shared__ double sh[kDotBlocks];
  sh[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int off = kDotBlocks / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double q = sh[0];
    double c = lr;
    if (norm_constraint > 0.0 && q > 0.0) c = lr * fmin(1.0, sqrt(norm_constraint / (lr * lr * q)));
    stats[6] = q;
    stats[7] = c;
  }
}

hipError_t launch_step_length(const float* x, const float* g, int64_t n, double lr, double norm_constraint,
                              double* part, double* stats, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks), dim3(kDotThreads), 0, s, x, g, n, part);
  hipLaunchKernelGGL(step_length_kernel, dim3(1), dim3(kDotBlocks), 0, s, part, lr, norm_constraint, stats);
  return hipGetLastError();
}

// theta <- theta - c X, c = stats[7], in float64 before rounding
__global__ void apply_step_kernel(float* theta, const float* x, int64_t n, const double* stats) {
  const double c = stats[7];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    theta[i] = (float)((double)theta[i] - c * (double)x[i]);
}

hipError_t launch_apply_step(float* theta, const float* x, int64_t n, const double* stats, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(apply_step_kernel, dim3(grid), dim3(256), 0, s, theta, x, n, stats);
  return hipGetLastError();
}

}  // namespace fn
