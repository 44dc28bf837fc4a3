// Metropolis random walk on psi^2 (the sampling of Eq. (3)).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), a
// counter-based generator, so every (walker, step, coordinate) draw is
// addressable and a chain is reproducible from (seed, counter) alone.
// Counter scheme (stated in the public header):
//   key = (seed lo, seed hi); s = counter + step
//   normals, walker w, coordinates 4b..4b+3: counter (w, b, s lo, s hi),
//     Box-Muller on word pairs (x0, x1) and (x2, x3)
//   acceptance uniform of walker w: word x0 of counter (w, 2^31, s lo, s hi)
//   uniform from a word x: ((x >> 9) + 0.5) * 2^-23, exact in float32.
#include "common.h"
#include "kernels.h"

namespace fn {

struct PhiloxOut {
  uint32_t x[4];
};

__device__ inline PhiloxOut philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  PhiloxOut o;
  o.x[0] = c0;
  o.x[1] = c1;
  o.x[2] = c2;
  o.x[3] = c3;
  return o;
}

__device__ inline float unit_uniform(uint32_t x) { return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f); }

// the four normals of block b of walker w at step s
__device__ inline void normals4(uint64_t seed, uint64_t s, uint32_t w, uint32_t b, float z[4]) {
  PhiloxOut o = philox4x32_10(w, b, (uint32_t)s, (uint32_t)(s >> 32), (uint32_t)seed, (uint32_t)(seed >> 32));
  const float two_pi = 6.2831853071795864769f;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float u1 = unit_uniform(o.x[2 * p]), u2 = unit_uniform(o.x[2 * p + 1]);
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincosf(two_pi * u2, &sn, &cs);
    z[2 * p] = rad * cs;
    z[2 * p + 1] = rad * sn;
  }
}

__device__ inline float accept_uniform(uint64_t seed, uint64_t s, uint32_t w) {
  PhiloxOut o = philox4x32_10(w, 0x80000000u, (uint32_t)s, (uint32_t)(s >> 32), (uint32_t)seed, (uint32_t)(seed >> 32));
  return unit_uniform(o.x[0]);
}

__global__ void noise_kernel(int W, int n3, int n_steps, uint64_t seed, uint64_t counter, float* noise,
                             float* uniforms) {
  const int nb = (n3 + 3) / 4;
  const int64_t total = (int64_t)n_steps * W * (nb + 1);
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx % (nb + 1));
    const int64_t sw = idx / (nb + 1);
    const int w = (int)(sw % W);
    const int step = (int)(sw / W);
    const uint64_t s = counter + (uint64_t)step;
    if (b == nb) {
      uniforms[sw] = accept_uniform(seed, s, (uint32_t)w);
    } else {
      float z[4];
      normals4(seed, s, (uint32_t)w, (uint32_t)b, z);
      for (int r = 0; r < 4; ++r)
        if (4 * b + r < n3) noise[sw * n3 + 4 * b + r] = z[r];
    }
  }
}

hipError_t launch_mcmc_noise(int W, int n, int n_steps, uint64_t seed, uint64_t counter, float* noise,
                             float* uniforms, hipStream_t s) {
  const int n3 = 3 * n;
  const int64_t total = (int64_t)n_steps * W * ((n3 + 3) / 4 + 1);
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(noise_kernel, dim3(grid), dim3(256), 0, s, W, n3, n_steps, seed, counter, noise, uniforms);
  return hipGetLastError();
}

// prop = pos + width * z   (z supplied for this step, or drawn)
__global__ void propose_kernel(const float* pos, float* prop, int W, int n3, float width, uint64_t seed, uint64_t step,
                               const float* noise, uint32_t w_base) {
  const int nb = (n3 + 3) / 4;
  const int64_t total = (int64_t)W * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx % nb);
    const int64_t w = idx / nb;
    float z[4];
    if (noise) {
      for (int r = 0; r < 4; ++r) z[r] = 4 * b + r < n3 ? noise[w * n3 + 4 * b + r] : 0.0f;
    } else {
      normals4(seed, step, w_base + (uint32_t)w, (uint32_t)b, z);
    }
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * b + r;
      if (q < n3) prop[w * n3 + q] = pos[w * n3 + q] + width * z[r];
    }
  }
}

hipError_t launch_propose_offset(const float* pos, float* prop, int W, int n3, float width, uint64_t seed,
                                 uint64_t step, const float* noise, uint32_t w_base, hipStream_t s) {
  const int64_t total = (int64_t)W * ((n3 + 3) / 4);
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(propose_kernel, dim3(grid), dim3(256), 0, s, pos, prop, W, n3, width, seed, step, noise, w_base);
  return hipGetLastError();
}

// one thread per walker: accept iff psi(x') != 0 and log u < 2 (l' - l)
__global__ void accept_kernel(float* pos, const float* prop, float* logpsi, float* sign, const float* lp_new,
                              const float* sg_new, int32_t* n_acc, int W, int n3, uint64_t seed, uint64_t step,
                              const float* uniforms, int first, uint32_t w_base) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const float u = uniforms ? uniforms[w] : accept_uniform(seed, step, w_base + (uint32_t)w);
  const float lp = lp_new[w], sp = sg_new[w];
  const bool ok = sp != 0.0f && logf(u) < 2.0f * (lp - logpsi[w]);
  if (ok) {
    for (int q = 0; q < n3; ++q) pos[(int64_t)w * n3 + q] = prop[(int64_t)w * n3 + q];
    logpsi[w] = lp;
    sign[w] = sp;
  }
  n_acc[w] = (first ? 0 : n_acc[w]) + (ok ? 1 : 0);
}

hipError_t launch_accept_offset(float* pos, const float* prop, float* logpsi, float* sign, const float* lp_new,
                                const float* sg_new, int32_t* n_acc, int W, int n3, uint64_t seed, uint64_t step,
                                const float* uniforms, int first, uint32_t w_base, hipStream_t s) {
  if (W <= 0) return hipSuccess;
  hipLaunchKernelGGL(accept_kernel, dim3((W + 255) / 256), dim3(256), 0, s, pos, prop, logpsi, sign, lp_new, sg_new,
                     n_acc, W, n3, seed, step, uniforms, first, w_base);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int n, int32_t v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace fn
