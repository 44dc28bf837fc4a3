// Hand-written adjoint of log|psi| with respect to the parameters.
//
// Reverse mode over a value-only forward pass (no tangents are stored; the
// layer values are recomputed by that pass).  With cotangent c_w of
// log|psi_w|:
//   log|psi| = log|sum_k P_k|       -> d/d log|P_k| = rho_k = P_k / psi
//   log|det B| (B[j][i] = phi_i(r_j)) -> d/dB[j][i] = (B^-1)[i][j]
//   phi = u * env                    -> cot u = cot phi * env, cot env = cot phi * u
//   u = h^L_j . w[:, ki] + g[ki]      -> dw, dg, cot h^L_j
//   env = sum_m pi exp(-|s| d)        -> dpi, dsigma
//   h^{l+1} = tanh(pre) (+ h^l)       -> cot pre = cot h^{l+1} sech^2(pre)
//   pre_i = h_i A + hbar B + g_i C + b -> dA, dB, dC, db and the cotangents
//                                        of h_i, hbar (spread over the
//                                        electrons of its spin) and g_i
//                                        (spread over the pair features)
// and the same for the two-electron layers.  Every reduction over walkers,
// electrons or pairs is done in a fixed order (split partial sums reduced
// in order): the gradient is bitwise reproducible.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace fn {

// ---------------------------------------------- determinant / orbital cotangents
// cot_u[(w na + j) * ldu + k na + i] = c_w rho_k Binv[w][k][i][j] env[w][k][j][i]
// (zero in the padding columns), cot_env[w][k][j][i] = c_w rho_k Binv[..][i][j] u[..];
// a walker with c_w = 0 contributes exact zeros (also where rho or Binv is
// not finite, at a node of psi)
template <class R>
__global__ void adj_orbital_cot_kernel(const R* binv, const R* rho, const float* cot, const float* u,
                                       const float* env, int W, int K, int na, int ldu, float* cot_u,
                                       float* cot_env) {
  const int64_t total = (int64_t)W * na * ldu;
  const int nsq = na * na;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % ldu);
    const int64_t row = idx / ldu;
    const int j = (int)(row % na);
    const int64_t w = row / na;
    float cu = 0.0f;
    if (col < K * na) {
      const int k = col / na, i = col % na;
      const int64_t m = w * K + k;
      const R cw = (R)cot[w];
      const R cb = cw == (R)0 ? (R)0 : cw * rho[m] * binv[m * nsq + i * na + j];
      const int64_t e = m * nsq + j * na + i;
      cu = cw == (R)0 ? 0.0f : (float)(cb * (R)env[e]);
      cot_env[e] = cw == (R)0 ? 0.0f : (float)(cb * (R)u[e]);
    }
    cot_u[idx] = cu;
  }
}

hipError_t launch_adj_orbital_cot(bool fp64, const void* binv, const void* rho, const float* cot, const float* u,
                                  const float* env, int W, int K, int na, int ldu, float* cot_u, float* cot_env,
                                  hipStream_t s) {
  const int64_t total = (int64_t)W * na * ldu;
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  if (fp64)
    hipLaunchKernelGGL(adj_orbital_cot_kernel<double>, dim3(grid), dim3(256), 0, s, (const double*)binv,
                       (const double*)rho, cot, u, env, W, K, na, ldu, cot_u, cot_env);
  else
    hipLaunchKernelGGL(adj_orbital_cot_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)binv,
                       (const float*)rho, cot, u, env, W, K, na, ldu, cot_u, cot_env);
  return hipGetLastError();
}

// block reduction of 256 values (fixed order)
__device__ inline float block_sum256(float v, float* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  float r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}

// envelope parameters: one block per (orbital column (k,i), nucleus m)
// and split of the rows (w, j) (blockIdx.y, rps rows each), d = r_j - R_m,
// e = exp(-s):
//   isotropic: s = |sigma| |d|
//     dpi    += sum_{w,j} cot_env e
//     dsigma += sum_{w,j} cot_env pi e (-sign(sigma) |d|)
//   full:      s = |Sigma d| = |u|
//     dpi          += sum_{w,j} cot_env e
//     dSigma[a][b] += sum_{w,j} cot_env pi e (-u_a d_b / s)
// With part, each split writes its sums (dpi first, then the NS dsigma
// entries) to part[split][column m][1 + NS] for env_grad_final_kernel;
// otherwise the one split adds them to dpi and dsigma.
template <bool FULL>
__global__ __launch_bounds__(256) void adj_env_grad_kernel(const float* cot_env, const float* pos, const float* nuc,
                                                           const float* pi, const float* sigma, int W, int K,
                                                           int na, int j0, int n, int N, float* dpi,
                                                           float* dsigma, int64_t rps, float* part) {
  __shared__ float sh[4];
  constexpr int NS = FULL ? 9 : 1;
  const int col = blockIdx.x / N, m = blockIdx.x % N;
  const int k = col / na, i = col % na;
  const float p = pi[col * N + m];
  float M[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) M[q] = sigma[((size_t)col * N + m) * NS + q];
  float api = 0.0f, asg[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) asg[q] = 0.0f;
  const int64_t r_end = std::min<int64_t>((int64_t)W * na, (blockIdx.y + 1) * rps);
  for (int64_t r = blockIdx.y * rps + threadIdx.x; r < r_end; r += 256) {
    const int j = (int)(r % na);
    const int64_t w = r / na;
    const float* x = pos + (w * n + j0 + j) * 3;
    const float dv[3] = {x[0] - nuc[3 * m], x[1] - nuc[3 * m + 1], x[2] - nuc[3 * m + 2]};
    const float c = cot_env[((w * K + k) * na + j) * na + i];
    if constexpr (FULL) {
      float u[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] = M[3 * q] * dv[0] + M[3 * q + 1] * dv[1] + M[3 * q + 2] * dv[2];
      const float sv = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      const float e = expf(-sv);
      api += c * e;
      const float f = -c * p * e / sv;
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int b = 0; b < 3; ++b) asg[3 * q + b] += f * u[q] * dv[b];
    } else {
      const float s = fabsf(M[0]), sgn = M[0] < 0.0f ? -1.0f : 1.0f;
      const float d = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      const float e = expf(-s * d);
      api += c * e;
      asg[0] += c * p * e * (-sgn * d);
    }
  }
  api = block_sum256(api, sh);
#pragma unroll
  for (int q = 0; q < NS; ++q) asg[q] = block_sum256(asg[q], sh);
  if (threadIdx.x == 0) {
    if (part) {
      float* o = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (1 + NS);
      o[0] = api;
#pragma unroll
      for (int q = 0; q < NS; ++q) o[1 + q] = asg[q];
    } else {
      dpi[col * N + m] += api;
#pragma unroll
      for (int q = 0; q < NS; ++q) dsigma[((size_t)col * N + m) * NS + q] += asg[q];
    }
  }
}

// the splits' sums of adj_env_grad_kernel added in split order: one thread
// per (column m, entry q), q = 0 for dpi, 1 + b for dsigma entry b
__global__ void env_grad_final_kernel(const float* part, int splits, int cols, int ns, float* dpi, float* dsigma) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cols * (1 + ns)) return;
  const int cm = t / (1 + ns), q = t - cm * (1 + ns);
  float v = 0.0f;
  for (int sp = 0; sp < splits; ++sp) v += part[(size_t)sp * cols * (1 + ns) + t];
  if (q == 0) dpi[cm] += v;
  else dsigma[(size_t)cm * ns + q - 1] += v;
}

// per walker (one thread per walker, orbital column and nucleus, the sum
// over the walker's electrons j of spin a in order):
//   dpi[w ld + col N + m] += sum_j cot_env e, dsigma likewise
template <bool FULL>
__global__ void adj_env_grad_walker_kernel(const float* cot_env, const float* pos, const float* nuc, const float* pi,
                                           const float* sigma, int W, int K, int na, int j0, int n, int N,
                                           float* dpi, float* dsigma, int64_t ld) {
  constexpr int NS = FULL ? 9 : 1;
  const int64_t total = (int64_t)W * K * na * N;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int cm = (int)(t % ((int64_t)K * na * N));
    const int64_t w = t / ((int64_t)K * na * N);
    const int col = cm / N, m = cm % N;
    const int k = col / na, i = col % na;
    const float p = pi[col * N + m];
    float M[NS], asg[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      M[q] = sigma[((size_t)col * N + m) * NS + q];
      asg[q] = 0.0f;
    }
    float api = 0.0f;
    for (int j = 0; j < na; ++j) {
      const float* x = pos + (w * n + j0 + j) * 3;
      const float dv[3] = {x[0] - nuc[3 * m], x[1] - nuc[3 * m + 1], x[2] - nuc[3 * m + 2]};
      const float c = cot_env[((w * K + k) * na + j) * na + i];
      if constexpr (FULL) {
        float u[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) u[q] = M[3 * q] * dv[0] + M[3 * q + 1] * dv[1] + M[3 * q + 2] * dv[2];
        const float sv = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const float e = expf(-sv);
        api += c * e;
        const float f = -c * p * e / sv;
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int b = 0; b < 3; ++b) asg[3 * q + b] += f * u[q] * dv[b];
      } else {
        const float sa = fabsf(M[0]), sgn = M[0] < 0.0f ? -1.0f : 1.0f;
        const float d = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        const float e = expf(-sa * d);
        api += c * e;
        asg[0] += c * p * e * (-sgn * d);
      }
    }
    dpi[w * ld + col * N + m] += api;
#pragma unroll
    for (int q = 0; q < NS; ++q) dsigma[w * ld + ((int64_t)col * N + m) * NS + q] += asg[q];
  }
}

hipError_t launch_adj_env_grad(const float* cot_env, const float* pos, const float* nuc, const float* pi,
                               const float* sigma, bool full, int W, int K, int na, int j0, int n, int N, float* dpi,
                               float* dsigma, hipStream_t s, int64_t walker_ld, float* part, int64_t part_floats) {
  if (na <= 0 || W <= 0) return hipSuccess;
  if (walker_ld > 0) {
    const int64_t total = (int64_t)W * K * na * N;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    if (full)
      hipLaunchKernelGGL(adj_env_grad_walker_kernel<true>, dim3(grid), dim3(256), 0, s, cot_env, pos, nuc, pi, sigma,
                         W, K, na, j0, n, N, dpi, dsigma, walker_ld);
    else
      hipLaunchKernelGGL(adj_env_grad_walker_kernel<false>, dim3(grid), dim3(256), 0, s, cot_env, pos, nuc, pi, sigma,
                         W, K, na, j0, n, N, dpi, dsigma, walker_ld);
    return hipGetLastError();
  }
  // rows split so that a thread takes at most about eight rows (the loop is
  // bound by the latency of its loads), as many splits as part holds
  const int cols = K * na * N, ns = full ? 9 : 1;
  const int64_t rows = (int64_t)W * na;
  int64_t splits = std::min<int64_t>((rows + 2047) / 2048, 64);
  if (part) splits = std::min<int64_t>(splits, part_floats / ((int64_t)cols * (1 + ns)));
  if (!part || splits < 2) splits = 1;
  const int64_t rps = (rows + splits - 1) / splits;
  float* pp = splits > 1 ? part : nullptr;
  if (full)
    hipLaunchKernelGGL(adj_env_grad_kernel<true>, dim3(cols, (unsigned)splits), dim3(256), 0, s, cot_env, pos, nuc, pi,
                       sigma, W, K, na, j0, n, N, dpi, dsigma, rps, pp);
  else
    hipLaunchKernelGGL(adj_env_grad_kernel<false>, dim3(cols, (unsigned)splits), dim3(256), 0, s, cot_env, pos, nuc,
                       pi, sigma, W, K, na, j0, n, N, dpi, dsigma, rps, pp);
  if (pp)
    hipLaunchKernelGGL(env_grad_final_kernel, dim3((cols * (1 + ns) + 255) / 256), dim3(256), 0, s, pp, (int)splits,
                       cols, ns, dpi, dsigma);
  return hipGetLastError();
}

// ------------------------------------------------------------- X^T Y
// part[split][k][nn] = sum_{r in split} X[map(r)][xcol + k] * Y[r][nn]:
// 64 x 64 output tiles on v_mfma_f32_16x16x4_f32, 16 rows per step through
// double-buffered LDS with the next step's rows loaded into registers
// meanwhile.  The rows are cut into as many splits as bring the launch to
// about ATB_BLOCKS workgroups, so the partials (and their reduction) stay
// small however many rows there are.
constexpr int ATB_BLOCKS = 1024;

int atb_splits(int64_t R, int K1, int N) {
  const int64_t tiles = (int64_t)((K1 + 63) / 64) * ((N + 63) / 64);
  int64_t sp = (ATB_BLOCKS + tiles - 1) / tiles;
  sp = std::min<int64_t>(sp, (R + 63) / 64);
  return (int)std::max<int64_t>(sp, 1);
}
int64_t atb_part_floats(int K1max, int Nmax) {
  return (int64_t)(ATB_BLOCKS + ((K1max + 63) / 64) * ((Nmax + 63) / 64)) * 64 * 64;
}

// VEC: ldx, xcol, ldy multiples of 4 and 16-byte aligned bases (one 16-byte
// load per operand; the last vector of a row is read element by element
// when K1 or N is not a multiple of 4).
// BF: split-bfloat16 products, 32 rows per step.  The rows are the
// reduction index, so an MFMA operand wants eight consecutive rows of one
// column per lane: each lane gathers them from the float32 tile in LDS
// (rows of 66 floats: the four 8-row groups of a read hit distinct banks)
// and splits them into hi and lo parts in registers.
template <bool VEC, bool BF>
__global__ __launch_bounds__(256) void atb_kernel(AtbArgs a, int64_t rows_per_split) {
  constexpr int BR = BF ? 32 : 16, LD = BF ? 64 + 2 : 64 + 4;
  __shared__ float Xs[2][BR][LD];
  __shared__ float Ys[2][BR][LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int tk = blockIdx.x, tn = blockIdx.y;
  if (a.sym) {  // blockIdx.x enumerates the tiles tk <= tn, tn-major
    const int p = blockIdx.x;
    tn = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while (tn * (tn + 1) / 2 > p) --tn;
    while ((tn + 1) * (tn + 2) / 2 <= p) ++tn;
    tk = p - tn * (tn + 1) / 2;
  }
  const int k0 = tk * 64, n0 = tn * 64;
  // per-walker mode: the z index runs over the walkers (segments of seg rows)
  const int64_t n_split = a.dst ? a.R / a.seg : (int64_t)gridDim.z;
  for (int64_t split = blockIdx.z; split < n_split; split += gridDim.z) {
  const int64_t r_begin = split * rows_per_split;
  const int64_t r_end = std::min<int64_t>(r_begin + rows_per_split, a.R);
  floatx4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int lr = tid / 16, lc = (tid % 16) * 4;  // loader: rows lr (+ 16 h), 4 columns
  const bool kin = k0 + lc < a.K1, nin = n0 + lc < a.N;
  float xv[BR / 16][4], yv[BR / 16][4];
  auto load_row = [&](int64_t r, float* xv, float* yv) {
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q] = yv[q] = 0.0f;
    if (r >= r_end) return;
    const int64_t mr = a.xs ? (int64_t)((int)r / a.xs) * a.xa + a.xe + (int)r % a.xs : r;
    const float* xp = a.X + mr * a.ldx + a.xcol + k0 + lc;
    const float* yp = a.Y + r * a.ldy + n0 + lc;
    if constexpr (VEC) {
      if (k0 + lc + 3 < a.K1) {
        const float4 v = *reinterpret_cast<const float4*>(xp);
        xv[0] = v.x, xv[1] = v.y, xv[2] = v.z, xv[3] = v.w;
      } else if (kin) {
        for (int q = 0; q < 4; ++q)
          if (k0 + lc + q < a.K1) xv[q] = xp[q];
      }
      if (n0 + lc + 3 < a.N) {
        const float4 v = *reinterpret_cast<const float4*>(yp);
        yv[0] = v.x, yv[1] = v.y, yv[2] = v.z, yv[3] = v.w;
      } else if (nin) {
        for (int q = 0; q < 4; ++q)
          if (n0 + lc + q < a.N) yv[q] = yp[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (k0 + lc + q < a.K1) xv[q] = xp[q];
        if (n0 + lc + q < a.N) yv[q] = yp[q];
      }
    }
  };
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int h = 0; h < BR / 16; ++h) load_row(r0 + lr + 16 * h, xv[h], yv[h]);
  };
  if (r_begin < r_end) load(r_begin);
  int buf = 0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += BR, buf ^= 1) {
#pragma unroll
    for (int h = 0; h < BR / 16; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Xs[buf][lr + 16 * h][lc + q] = xv[h][q];
        Ys[buf][lr + 16 * h][lc + q] = yv[h][q];
      }
    __syncthreads();
    if (r0 + BR < r_end) load(r0 + BR);
    if constexpr (BF) {
      // lane (kq, c): rows 8 kq .. 8 kq + 7 of column c of each 16-column tile
      const int r8 = (lane >> 4) * 8, c = lane & 15;
      bf16x8 ah[2], al[2], bh[2], bl[2];
      auto frag = [&](const float (*T)[LD], int col, bf16x8* hi, bf16x8* lo) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) split_bf16x2(T[r8 + 2 * p][col], T[r8 + 2 * p + 1][col], &h[p], &l[p]);
        *hi = __builtin_bit_cast(bf16x8, uint4{h[0], h[1], h[2], h[3]});
        *lo = __builtin_bit_cast(bf16x8, uint4{l[0], l[1], l[2], l[3]});
      };
#pragma unroll
      for (int i = 0; i < 2; ++i) frag(Xs[buf], wm * 32 + i * 16 + c, &ah[i], &al[i]);
#pragma unroll
      for (int j = 0; j < 2; ++j) frag(Ys[buf], wn * 32 + j * 16 + c, &bh[j], &bl[j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int rr = ks * 4 + (lane >> 4);
        float af[2], bf[2];
        for (int i = 0; i < 2; ++i) af[i] = Xs[buf][rr][wm * 32 + i * 16 + (lane & 15)];
        for (int j = 0; j < 2; ++j) bf[j] = Ys[buf][rr][wn * 32 + j * 16 + (lane & 15)];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
    // the other buffer is written next step, after this step's barrier
  }
  if (a.dst) {
    // one walker's product: each element has one owner, so += does not race
    float* out = a.dst + split * a.dst_ld;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int q = 0; q < 4; ++q) {
          const int k = k0 + wm * 32 + i * 16 + (lane >> 4) * 4 + q;
          const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
          if (k < a.K1 && nn < a.N) out[(int64_t)k * a.N + nn] += acc[i][j][q];
        }
    // the LDS buffers are rewritten by the next walker's first step
    __syncthreads();
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    continue;
  }
  float* out = a.part + split * a.K1 * a.N;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + wm * 32 + i * 16 + (lane >> 4) * 4 + q;
        const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (k < a.K1 && nn < a.N) out[(int64_t)k * a.N + nn] = acc[i][j][q];
      }
  }
}

hipError_t launch_atb(const AtbArgs& a, hipStream_t s) {
  if (a.R <= 0 || a.K1 <= 0 || a.N <= 0) return hipSuccess;
  if (a.dst && (a.seg <= 0 || a.R % a.seg != 0 || a.sym)) return hipErrorInvalidValue;
  const int sp = a.dst ? (int)std::min<int64_t>(a.R / a.seg, 32768) : atb_splits(a.R, a.K1, a.N);
  // the split form steps over 32 rows (per walker: its segment, padded with zeros)
  const bool bf = a.bf16 != 0;
  const int br = bf ? 32 : 16;
  const int64_t rps = a.dst ? a.seg : ((a.R + sp - 1) / sp + br - 1) / br * br;
  const int tkn = (a.K1 + 63) / 64;
  dim3 grid(a.sym ? tkn * (tkn + 1) / 2 : tkn, a.sym ? 1 : (a.N + 63) / 64, sp);
  const bool vec = a.ldx % 4 == 0 && a.xcol % 4 == 0 && a.ldy % 4 == 0 && ((uintptr_t)a.X % 16) == 0 &&
                   ((uintptr_t)a.Y % 16) == 0;
  if (bf) {
    if (vec) hipLaunchKernelGGL((atb_kernel<true, true>), grid, dim3(256), 0, s, a, rps);
    else hipLaunchKernelGGL((atb_kernel<false, true>), grid, dim3(256), 0, s, a, rps);
  } else {
    if (vec) hipLaunchKernelGGL((atb_kernel<true, false>), grid, dim3(256), 0, s, a, rps);
    else hipLaunchKernelGGL((atb_kernel<false, false>), grid, dim3(256), 0, s, a, rps);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ row sums
// pass 1: part[y][c] = sum_{r in chunk y} src[r * lds + c]
// (four interleaved accumulators, combined in a fixed order); with one
// chunk the sum is added straight into the destination (part = dst)
__device__ inline bool sym_lower(int c, int sym_n) {
  return sym_n > 0 && (c / sym_n) / 64 > (c % sym_n) / 64;
}

__global__ void rowsum_partial_kernel(const float* src, int64_t rows, int cols, int64_t lds, int64_t chunk,
                                      float* part, int sym_n, int add) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols || sym_lower(c, sym_n)) return;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = std::min<int64_t>(r0 + chunk, rows);
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  int64_t r = r0;
  for (; r + 3 < r1; r += 4) {
    a0 += src[r * lds + c];
    a1 += src[(r + 1) * lds + c];
    a2 += src[(r + 2) * lds + c];
    a3 += src[(r + 3) * lds + c];
  }
  for (; r < r1; ++r) a0 += src[r * lds + c];
  const float v = (a0 + a1) + (a2 + a3);
  if (add) part[c] += v;
  else part[(int64_t)blockIdx.y * cols + c] = v;
}
// pass 1 for narrow rows (cols a multiple of 4, at most 256): a thread
// sums one column quad over every rl-th row of its chunk with 16-byte loads
// (rl = 256 / (cols / 4) row lanes per block), and the row lanes are then
// added in order through LDS
__global__ __launch_bounds__(256) void rowsum_narrow_kernel(const float* src, int64_t rows, int cols, int64_t lds,
                                                             int64_t chunk, float* part, int add) {
  __shared__ float4 sh[256];
  const int nq = cols / 4, rl = 256 / nq;
  const int tid = threadIdx.x, q = tid % nq, lane_r = tid / nq;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = std::min<int64_t>(r0 + chunk, rows);
  float4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
  if (lane_r < rl) {
    int64_t r = r0 + lane_r;
    for (; r + rl < r1; r += 2 * rl) {
      const float4 u = *reinterpret_cast<const float4*>(src + r * lds + 4 * q);
      const float4 v = *reinterpret_cast<const float4*>(src + (r + rl) * lds + 4 * q);
      s0.x += u.x, s0.y += u.y, s0.z += u.z, s0.w += u.w;
      s1.x += v.x, s1.y += v.y, s1.z += v.z, s1.w += v.w;
    }
    if (r < r1) {
      const float4 u = *reinterpret_cast<const float4*>(src + r * lds + 4 * q);
      s0.x += u.x, s0.y += u.y, s0.z += u.z, s0.w += u.w;
    }
  }
  sh[tid] = float4{s0.x + s1.x, s0.y + s1.y, s0.z + s1.z, s0.w + s1.w};
  __syncthreads();
  if (lane_r != 0) return;
  float4 t = sh[q];
  for (int k = 1; k < rl; ++k) {
    const float4 u = sh[k * nq + q];
    t.x += u.x, t.y += u.y, t.z += u.z, t.w += u.w;
  }
  float* dst = add ? part + 4 * q : part + (int64_t)blockIdx.y * cols + 4 * q;
  if (add) {
    dst[0] += t.x, dst[1] += t.y, dst[2] += t.z, dst[3] += t.w;
  } else {
    dst[0] = t.x, dst[1] = t.y, dst[2] = t.z, dst[3] = t.w;
  }
}
// pass 2: dst[c] += sum_y part[y][c]; 64 columns x 4 slices of y per block
__global__ __launch_bounds__(256) void rowsum_final_kernel(const float* part, int ny, int cols, float* dst,
                                                            int sym_n) {
  __shared__ float sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), sl = threadIdx.x >> 6;
  const bool skip = c >= cols || sym_lower(c, sym_n);
  float acc = 0.0f;
  if (!skip)
    for (int y = sl; y < ny; y += 4) acc += part[(int64_t)y * cols + c];
  sh[sl][threadIdx.x & 63] = acc;
  __syncthreads();
  if (sl == 0 && !skip) dst[c] += (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

int rowsum_chunks(int64_t rows, int chunk) { return (int)((rows + chunk - 1) / chunk); }

// per walker: dst[q dst_ld + c] += sum of the seg rows of segment q, in row order
__global__ void rowsum_seg_kernel(const float* src, int64_t n_seg, int seg, int cols, int64_t lds, float* dst,
                                  int64_t dst_ld) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  for (int64_t q = blockIdx.y; q < n_seg; q += gridDim.y) {
    const float* p = src + q * seg * lds + c;
    float v = 0.0f;
    for (int r = 0; r < seg; ++r) v += p[(int64_t)r * lds];
    dst[q * dst_ld + c] += v;
  }
}

hipError_t launch_rowsum_seg_add(const float* src, int64_t rows, int seg, int cols, int64_t lds, float* dst,
                                 int64_t dst_ld, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (seg <= 0 || rows % seg != 0) return hipErrorInvalidValue;
  const int64_t n_seg = rows / seg;
  hipLaunchKernelGGL(rowsum_seg_kernel, dim3((cols + 255) / 256, (unsigned)std::min<int64_t>(n_seg, 32768)), dim3(256),
                     0, s, src, n_seg, seg, cols, lds, dst, dst_ld);
  return hipGetLastError();
}

hipError_t launch_rowsum_add(const float* src, int64_t rows, int cols, int64_t lds, float* tmp, float* dst,
                             int chunk, hipStream_t s, int sym_n) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  // at most 128 partial rows (never more than the tmp sizing of
  // rowsum_chunks(rows, chunk) assumes)
  int ny = std::min(rowsum_chunks(rows, chunk), 128);
  const int64_t ch = (rows + ny - 1) / ny;
  ny = (int)((rows + ch - 1) / ch);
  const bool narrow = sym_n == 0 && cols % 4 == 0 && cols <= 256 && lds % 4 == 0 && ((uintptr_t)src % 16) == 0;
  if (ny == 1) {  // one pass, into dst
    if (narrow)
      hipLaunchKernelGGL(rowsum_narrow_kernel, dim3(1, 1), dim3(256), 0, s, src, rows, cols, lds, ch, dst, 1);
    else
      hipLaunchKernelGGL(rowsum_partial_kernel, dim3((cols + 255) / 256, 1), dim3(256), 0, s, src, rows, cols, lds,
                         ch, dst, sym_n, 1);
    return hipGetLastError();
  }
  if (narrow)
    hipLaunchKernelGGL(rowsum_narrow_kernel, dim3(1, ny), dim3(256), 0, s, src, rows, cols, lds, ch, tmp, 0);
  else
    hipLaunchKernelGGL(rowsum_partial_kernel, dim3((cols + 255) / 256, ny), dim3(256), 0, s, src, rows, cols, lds, ch,
                       tmp, sym_n, 0);
  hipLaunchKernelGGL(rowsum_final_kernel, dim3((cols + 63) / 64), dim3(256), 0, s, tmp, ny, cols, dst, sym_n);
  return hipGetLastError();
}

__global__ void sym_mirror_kernel(float* M, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n), c = (int)(e - (int64_t)r * n);
    if (r / 64 > c / 64) M[e] = M[(int64_t)c * n + r];
  }
}

hipError_t launch_sym_mirror(float* M, int n, hipStream_t s) {
  if (n <= 64) return hipSuccess;
  const int64_t total = (int64_t)n * n;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(sym_mirror_kernel, dim3(grid), dim3(256), 0, s, M, n);
  return hipGetLastError();
}

// ----------------------------------------------------------- elementwise
// The cotangent pass of a one-electron layer, one thread per (walker,
// column), the walker's electrons in order:
//   CH[(w n + i)][c] += CMF[w][a(i) cols + c] / n_a   (when cmf is given:
//       the mean-field part of the cotangent of h, from the layer above)
//   CP[(w n + i)][c]  = CH[(w n + i)][c] sech^2(PRE[(w n + i)][c])
//   S[w][c]           = sum_i CP[(w n + i)][c]   (fixed order)
// Rows have cols entries (the layer's input and output widths agree
// whenever cmf is given).
__global__ void adj_cp_sum_kernel(float* ch, const float* pre, const float* cmf, int W, int n, int n_up, int cols,
                                  float* cp, float* S) {
  const int64_t total = (int64_t)W * cols;
  const float na_up = n_up > 0 ? (float)n_up : 1.0f, na_dn = n > n_up ? (float)(n - n_up) : 1.0f;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx % cols);
    const int64_t w = idx / cols;
    const float m_up = cmf ? cmf[w * 2 * cols + c] : 0.0f, m_dn = cmf ? cmf[w * 2 * cols + cols + c] : 0.0f;
    float acc = 0.0f;
    for (int i = 0; i < n; ++i) {
      // products rounded before the sum, as stored (no multiply-add
      // contraction)
#pragma clang fp contract(off)
      const int64_t e = (w * n + i) * cols + c;
      float h = ch[e];
      if (cmf) {
        h += i < n_up ? m_up / na_up : m_dn / na_dn;
        ch[e] = h;
      }
      const float v = h * sech2f(pre[e]);
      cp[e] = v;
      acc += v;
    }
    S[idx] = acc;
  }
}

hipError_t launch_adj_cp_sum(float* ch, const float* pre, const float* cmf, int W, int n, int n_up, int cols,
                             float* cp, float* S, hipStream_t s) {
  const int64_t total = (int64_t)W * cols;
  if (total <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(adj_cp_sum_kernel, dim3(grid), dim3(256), 0, s, ch, pre, cmf, W, n, n_up, cols, cp, S);
  return hipGetLastError();
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// dst[r * ldd + c] = src[r * lds + c]: the value rows of jets (one row in
// every lds floats) into a compact array.  16-byte vectors when the column
// count and both strides allow (every jet width here is a multiple of 32);
// a 64 x 4 block covers 64 vectors of 4 rows, rows advance by the grid.
template <class V>
__global__ __launch_bounds__(256) void copy_rows_kernel(const V* src, int64_t lds, V* dst, int64_t ldd, int64_t rows,
                                                        int vpr) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= vpr) return;
  for (int64_t r = (int64_t)blockIdx.y * 4 + threadIdx.y; r < rows; r += (int64_t)gridDim.y * 4)
    dst[r * ldd + c] = src[r * lds + c];
}

hipError_t launch_copy_rows(const float* src, int64_t lds, float* dst, int64_t ldd, int64_t rows, int cols,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const bool vec = cols % 4 == 0 && lds % 4 == 0 && ldd % 4 == 0 && (uintptr_t)src % 16 == 0 &&
                   (uintptr_t)dst % 16 == 0;
  const int vpr = vec ? cols / 4 : cols;
  const dim3 grid((vpr + 63) / 64, (unsigned)std::min<int64_t>((rows + 3) / 4, 16384));
  if (vec)
    hipLaunchKernelGGL(copy_rows_kernel<float4>, grid, dim3(64, 4), 0, s, (const float4*)src, lds / 4, (float4*)dst,
                       ldd / 4, rows, vpr);
  else
    hipLaunchKernelGGL(copy_rows_kernel<float>, grid, dim3(64, 4), 0, s, src, lds, dst, ldd, rows, vpr);
  return hipGetLastError();
}

__global__ void copy_f32_kernel(const float* src, float* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(copy_f32_kernel, dim3(grid), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// ------------------------------------------------- two-electron backward
// One block per group of E electrons i of walker w, all n partners j: the
// R = E n pair rows r = (i - i0) n + j.  For l = L-2 .. 0, with Ct the
// cotangent of h^{l+1}_ij:
//   pre = h^l_ij W_l + c_l ; cp = Ct sech^2(pre)
//   part_W[k][o] = sum_r h^l_r[k] cp_r[o] ; part_c[o] = sum_r cp_r[o]
//   Ct <- cp W_l^T (+ Ct when widths match) + (1/n_a) cot g^{a(j),l}_i
// starting from Ct = (1/n_a) cot g^{a(j),L-1}_i.  The three contractions
// run on v_mfma_f32_16x16x4_f32 over the pair rows in LDS (rows padded to
// 16, features to DM, zeros in the padding); the parameter partials of the
// block go to part[block][...] in the layout of the W_l, c_l blocks.
template <int DM>
__global__ __launch_bounds__(256) void adj_two_electron_kernel(Adj2eArgs a, int E, int ngrp) {
  extern __shared__ __attribute__((aligned(16))) float sh[];
  constexpr int LD = DM + 1;  // row stride of the LDS arrays
  const int n = a.n, d2 = a.d2, L = a.L, nu = a.n_up;
  const int RP = round_up(E * n, 16);
  float* Hs = sh;            // [RP][LD] h^l_ij
  float* Ct = Hs + RP * LD;  // [RP][LD] cotangent of h^{l+1}_ij
  float* Cp = Ct + RP * LD;  // [RP][LD] Ct sech^2(pre)
  float* Ws = Cp + RP * LD;  // [DM][LD] W_l
  float* cs = Ws + DM * LD;  // [DM]     c_l
  float* red = cs + DM;      // [256 / DM][DM] column-sum partials
  int* rowi = reinterpret_cast<int*>(red + 256);  // [RP] electron of pair row r (within the walker)
  int* rowa = rowi + RP;                          // [RP] spin of the partner of pair row r
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int blk = blockIdx.x;
  const int64_t w = blk / ngrp;
  const int i0 = (blk % ngrp) * E;
  const int Rb = min(E, n - i0) * n;  // live pair rows
  float* part = a.part + (int64_t)blk * a.ldp;
  const float cw = a.kfac ? a.sc[w] * a.sc[w] : 0.0f;
  const int TMr = RP / 16, TNd = DM / 16;
  // pair row r = (electron i0 + r / n, partner r % n): one division per row, here
  for (int r = tid; r < RP; r += 256) {
    const int e = r / n;
    rowi[r] = i0 + e;
    rowa[r] = r - e * n < nu ? 0 : 1;
  }
  const float inv_u = nu > 0 ? 1.0f / (float)nu : 0.0f, inv_d = n - nu > 0 ? 1.0f / (float)(n - nu) : 0.0f;
  __syncthreads();

  // mean-field cotangent (1/n_a) cot g^{a(j),l}_i of row r, feature k < ein
  auto mf_cot = [&](int l, int ein, int r, int k) {
    const int al = rowa[r];
    return a.CG[l][(w * n + rowi[r]) * a.ldcg[l] + al * ein + k] * (al == 0 ? inv_u : inv_d);
  };
  {
    const int l = L - 1, ein = l == 0 ? 4 : d2;
    for (int idx = tid; idx < RP * DM; idx += 256) {
      const int r = idx / DM, k = idx % DM;
      Ct[r * LD + k] = (r < Rb && k < ein) ? mf_cot(l, ein, r, k) : 0.0f;
    }
  }
  for (int l = L - 2; l >= 0; --l) {
    const int ein = l == 0 ? 4 : d2;
    const int ke = round_up(ein, 4), kd = round_up(d2, 4);
    __syncthreads();
    for (int idx = tid; idx < RP * DM; idx += 256) {
      const int r = idx / DM, k = idx % DM;
      float v = 0.0f;
      if (r < Rb && k < ein) v = a.h2[l][((w * n + i0) * n + r) * ein + k];
      Hs[r * LD + k] = v;
    }
    for (int idx = tid; idx < DM * DM; idx += 256) {
      const int k = idx / DM, o = idx % DM;
      Ws[k * LD + o] = (k < ein && o < d2) ? a.params[a.w_off[l] + k * d2 + o] : 0.0f;
    }
    for (int o = tid; o < DM; o += 256) cs[o] = o < d2 ? a.params[a.c_off[l] + o] : 0.0f;
    __syncthreads();
    // cp = Ct sech^2(H W + c)   [RP x DM]
    for (int t = wave; t < TMr * TNd; t += 4) {
      const int tm = t / TNd, tn = t % TNd;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < ke; ks += 4)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Hs[(tm * 16 + lr) * LD + ks + lk], Ws[(ks + lk) * LD + tn * 16 + lr],
                                                   acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = tm * 16 + 4 * lk + q, col = tn * 16 + lr;
        Cp[row * LD + col] = Ct[row * LD + col] * sech2f(acc[q] + cs[col]);
      }
    }
    __syncthreads();
    // parameter partials: H^T cp [ein x d2], column sums of cp [d2]
    const int TMk = round_up(ein, 16) / 16;
    for (int t = wave; t < TMk * TNd; t += 4) {
      const int tm = t / TNd, tn = t % TNd;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < RP; ks += 4)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Hs[(ks + lk) * LD + tm * 16 + lr], Cp[(ks + lk) * LD + tn * 16 + lr],
                                                   acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = tm * 16 + 4 * lk + q, o = tn * 16 + lr;
        if (k < ein && o < d2) part[a.p_off[l] + k * d2 + o] = acc[q];
      }
    }
    // column sums of cp: 256 / DM row-chunks per column, then the chunks
    // in fixed order
    {
      constexpr int NCH = 256 / DM;
      const int o = tid % DM, ch = tid / DM;
      float sum = 0.0f;
      for (int r = ch; r < RP; r += NCH) sum += Cp[r * LD + o];
      red[ch * DM + o] = sum;
      __syncthreads();
      if (tid < d2) {
        float tot = 0.0f;
#pragma unroll
        for (int c = 0; c < NCH; ++c) tot += red[c * DM + tid];
        part[a.p_off[l] + ein * d2 + tid] = tot;
      }
    }
    if (a.kfac) {
      // KFAC statistics of this layer: c_w [H 1]^T [H 1] and cp^T cp over
      // the pair rows (cp already carries sqrt(c_w) through the cotangent)
      float* kA = part + a.k_off[l];
      float* kG = kA + (ein + 1) * (ein + 1);
      for (int t = wave; t < TMk * TMk; t += 4) {
        const int tm = t / TMk, tn = t % TMk;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < RP; ks += 4)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Hs[(ks + lk) * LD + tm * 16 + lr], Hs[(ks + lk) * LD + tn * 16 + lr],
                                                     acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = tm * 16 + 4 * lk + q, o = tn * 16 + lr;
          if (k < ein && o < ein) kA[k * (ein + 1) + o] = cw * acc[q];
        }
      }
      for (int t = wave; t < TNd * TNd; t += 4) {
        const int tm = t / TNd, tn = t % TNd;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < RP; ks += 4)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Cp[(ks + lk) * LD + tm * 16 + lr], Cp[(ks + lk) * LD + tn * 16 + lr],
                                                     acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = tm * 16 + 4 * lk + q, o = tn * 16 + lr;
          if (k < d2 && o < d2) kG[k * d2 + o] = acc[q];
        }
      }
      // the bias row and column: c_w sum_rows h, and c_w times the row count
      {
        constexpr int NCH = 256 / DM;
        const int o = tid % DM, ch = tid / DM;
        float sum = 0.0f;
        for (int r = ch; r < RP; r += NCH) sum += Hs[r * LD + o];
        __syncthreads();
        red[ch * DM + o] = sum;
        __syncthreads();
        if (tid < ein) {
          float tot = 0.0f;
#pragma unroll
          for (int c = 0; c < NCH; ++c) tot += red[c * DM + tid];
          kA[tid * (ein + 1) + ein] = cw * tot;
          kA[ein * (ein + 1) + tid] = cw * tot;
        }
        if (tid == 0) kA[ein * (ein + 1) + ein] = cw * (float)Rb;
      }
    }
    // Ct <- cp W^T (+ Ct when widths match) + mean-field cotangent of layer l
    // (each element read and written by one lane: in place)
    const bool res = ein == d2;
    const int TNk = round_up(ein, 16) / 16;
    for (int t = wave; t < TMr * TNk; t += 4) {
      const int tm = t / TNk, tn = t % TNk;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < kd; ks += 4)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Cp[(tm * 16 + lr) * LD + ks + lk], Ws[(tn * 16 + lr) * LD + ks + lk],
                                                   acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = tm * 16 + 4 * lk + q, k = tn * 16 + lr;
        float v = 0.0f;
        if (row < Rb && k < ein) v = acc[q] + (res ? Ct[row * LD + k] : 0.0f) + mf_cot(l, ein, row, k);
        Ct[row * LD + k] = v;
      }
    }
  }
}

// electrons per block of the two-electron backward: pair rows E n <= 64
// (about 31 KiB of LDS for two-electron widths up to 32, so that five
// blocks share a compute unit; 128 rows allowed three and took 25% longer)
// and the LDS arrays within 64 KiB
static int adj2e_dm(int d2) { return d2 <= 16 ? 16 : d2 <= 32 ? 32 : 64; }
static int adj2e_group(int n, int d2) {
  const int dm = adj2e_dm(d2), ld = dm + 1;
  // LDS: three [rows][ld] arrays, W and c, 256 column-sum partials and two
  // int tables of at most 128 rows
  const int rows_cap = std::min(64, (65536 / 4 - dm * ld - dm - 256 - 2 * 128) / (3 * ld) / 16 * 16);
  return std::max(1, std::min(n, rows_cap / n));
}

int adj_two_electron_rows(int W, int n, int d2) {
  const int E = adj2e_group(n, d2);
  return W * ((n + E - 1) / E);
}

template <int DM>
static hipError_t run_adj2e(const Adj2eArgs& a, hipStream_t s) {
  const int E = adj2e_group(a.n, a.d2), ngrp = (a.n + E - 1) / E;
  const int RP = round_up(E * a.n, 16);
  const size_t shmem = ((size_t)3 * RP * (DM + 1) + (size_t)DM * (DM + 1) + DM + 256 + 2 * RP) * sizeof(float);
  if (shmem > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL((adj_two_electron_kernel<DM>), dim3((unsigned)((int64_t)a.W * ngrp)), dim3(256), shmem, s, a, E,
                     ngrp);
  return hipGetLastError();
}

hipError_t launch_adj_two_electron(const Adj2eArgs& a, hipStream_t s) {
  if (a.W <= 0 || a.L < 2) return hipSuccess;
  if (a.d2 > 64) return hipErrorInvalidValue;
  const int dm = adj2e_dm(a.d2);
  return dm == 16 ? run_adj2e<16>(a, s) : dm == 32 ? run_adj2e<32>(a, s) : run_adj2e<64>(a, s);
}

// hi and lo bfloat16 planes of a float32 vector (the split of the
// split-bfloat16 products, element by element)
__global__ void split_planes_kernel(const float* x, int64_t n, uint16_t* hi, uint16_t* lo) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    split_bf16(x[i], hi + i, lo + i);
}

hipError_t launch_split_planes(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(split_planes_kernel, dim3(grid), dim3(256), 0, s, x, n, hi, lo);
  return hipGetLastError();
}

// ---------------------------------------------------------- KFAC inputs
__global__ void kfac_sqrt_weights_kernel(const float* c, int Wc, float* sc) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < Wc) sc[w] = sqrtf(fmaxf(c[w], 0.0f));
}

hipError_t launch_kfac_sqrt_weights(const float* c, int Wc, float* sc, hipStream_t s) {
  if (Wc <= 0) return hipSuccess;
  hipLaunchKernelGGL(kfac_sqrt_weights_kernel, dim3((Wc + 255) / 256), dim3(256), 0, s, c, Wc, sc);
  return hipGetLastError();
}

// one workgroup per row r = w n + i
__global__ __launch_bounds__(256) void kfac_aug_layer_kernel(const float* H, int ldh, int din, const float* Hbar,
                                                             int dinp, const float* G, int ldg, int ein,
                                                             const float* sc, int n, int ldo, float* out) {
  const int64_t r = blockIdx.x;
  const int w = (int)(r / n);
  const float s = sc[w];
  const float* h = H + r * ldh;
  const float* hb = Hbar + (int64_t)w * 2 * dinp;
  const float* g = G + r * ldg;
  float* o = out + r * ldo;
  for (int c = threadIdx.x; c < ldo; c += blockDim.x) {
    float v = 0.0f;
    if (c < din) v = h[c];
    else if (c < 2 * din) v = hb[c - din];
    else if (c < 3 * din) v = hb[dinp + c - 2 * din];
    else if (c < 3 * din + 2 * ein) v = g[c - 3 * din];
    else if (c == 3 * din + 2 * ein) v = 1.0f;
    o[c] = s * v;
  }
}

hipError_t launch_kfac_aug_layer(const float* H, int ldh, int din, const float* Hbar, int dinp, const float* G,
                                 int ldg, int ein, const float* sc, int Wc, int n, int ldo, float* out, hipStream_t s) {
  const int64_t R = (int64_t)Wc * n;
  if (R <= 0) return hipSuccess;
  if (ldo < 3 * din + 2 * ein + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kfac_aug_layer_kernel, dim3((unsigned)R), dim3(256), 0, s, H, ldh, din, Hbar, dinp, G, ldg, ein,
                     sc, n, ldo, out);
  return hipGetLastError();
}

// one workgroup per row r = w n_a + j
__global__ __launch_bounds__(256) void kfac_aug_orbital_kernel(const float* H, int ldh, int d1, const float* sc, int n,
                                                               int j0, int na, int ldo, float* out) {
  const int64_t r = blockIdx.x;
  const int w = (int)(r / na), j = (int)(r - (int64_t)w * na);
  const float s = sc[w];
  const float* h = H + ((int64_t)w * n + j0 + j) * ldh;
  float* o = out + r * ldo;
  for (int c = threadIdx.x; c < ldo; c += blockDim.x) o[c] = c < d1 ? s * h[c] : (c == d1 ? s : 0.0f);
}

hipError_t launch_kfac_aug_orbital(const float* H, int ldh, int d1, const float* sc, int Wc, int n, int j0, int na,
                                   int ldo, float* out, hipStream_t s) {
  const int64_t R = (int64_t)Wc * na;
  if (R <= 0) return hipSuccess;
  if (ldo < d1 + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kfac_aug_orbital_kernel, dim3((unsigned)R), dim3(256), 0, s, H, ldh, d1, sc, n, j0, na, ldo, out);
  return hipGetLastError();
}

// ----------------------------------------- energy statistics and cotangent
// cot[w] = (e[w] - mean) / W_total for the walkers of one chunk
__global__ void cot_from_stats_kernel(const float* e, int Wc, const double* stats, int W_total, float* cot) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < Wc) cot[w] = (float)(((double)e[w] - stats[0]) / (double)W_total);
}

hipError_t launch_cot_from_stats(const float* e, int Wc, const double* stats, int W_total, float* cot, hipStream_t s) {
  if (Wc <= 0) return hipSuccess;
  hipLaunchKernelGGL(cot_from_stats_kernel, dim3((Wc + 255) / 256), dim3(256), 0, s, e, Wc, stats, W_total, cot);
  return hipGetLastError();
}

// one block: mean and population variance of e_loc in float64 (two passes,
// fixed order)
__global__ __launch_bounds__(256) void energy_stats_kernel(const float* e, int W, double* stats, float* cot) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int w = tid; w < W; w += 256) s += (double)e[w];
  sh[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  const double mean = sh[0] / (double)W;
  __syncthreads();
  double v = 0.0;
  for (int w = tid; w < W; w += 256) {
    const double d = (double)e[w] - mean;
    v += d * d;
  }
  sh[tid] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    stats[0] = mean;
    stats[1] = sh[0] / (double)W;
  }
  if (cot)
    for (int w = tid; w < W; w += 256) cot[w] = (float)(((double)e[w] - mean) / (double)W);
}

hipError_t launch_energy_stats(const float* e, int W, double* stats, float* cot, hipStream_t s) {
  if (W <= 0) return hipSuccess;
  hipLaunchKernelGGL(energy_stats_kernel, dim3(1), dim3(256), 0, s, e, W, stats, cot);
  return hipGetLastError();
}

}  // namespace fn
