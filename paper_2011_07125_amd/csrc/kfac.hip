// The KFAC step direction (Martens and Grosse 2015, the optimiser the
// paper's introduction names): for every dense layer with Kronecker factors
// A (inputs + 1) and G (outputs) and gradient block M = [weights; bias],
//   X = (A + pi s I)^-1 M (G + s / pi I)^-1,   s = sqrt(lambda),
//   pi = sqrt((tr A / dim A) / (tr G / dim G))   (factored Tikhonov damping).
//
// Everything is float64.  The damped factors are Cholesky-factored as one
// batch of matrices in 32 x 32 tiles (diagonal tile in LDS, the panel below
// it row by row, the trailing tiles pairwise over the whole GPU), then
// X = L_A^-T L_A^-1 M, transposed, and the same two triangular solves with
// L_G give X^T.  Matrices are row-major; only lower triangles are read as
// factors.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace fn {

constexpr int TB = 32;

// the value of v in lane l of the wavefront (l uniform)
__device__ inline double readlane_f64(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l), hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One TB x TB tile product on the float64 matrix cores, for a 256-thread
// workgroup: wave w forms the 16 x 16 output block (w / 2, w % 2) of
//   C[r][c] = sum_k X(r, k) Y(k, c)
// with 8 steps of v_mfma_f64_16x16x4 (k = 4 s + lane / 16).  The result of
// element q of the lane is row 16 (w / 2) + lane / 16 + 4 q, column
// 16 (w % 2) + lane % 16, handed to put(row, col, value).
template <class FX, class FY, class FP>
__device__ inline void tile_mm_f64(int tid, FX X, FY Y, FP put) {
  const int lane = tid & 63, w = tid >> 6;
  const int r0 = (w >> 1) * 16, c0 = (w & 1) * 16, lr = lane & 15, lk = lane >> 4;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < TB / 4; ++s)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X(r0 + lr, 4 * s + lk), Y(4 * s + lk, c0 + lr), acc, 0, 0, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) put(r0 + lk + 4 * q, c0 + lr, acc[q]);
}

// ------------------------------------------------------------- set-up
// per dense layer b (blockIdx.x): damped copies of A and G, and M, in
// float64; blockIdx.y takes PREP_ROWS rows of each.  Every workgroup forms
// the two traces of its layer itself (dim_A + dim_G diagonal loads), so the
// copies need no second launch.
constexpr int PREP_ROWS = 8;

__global__ __launch_bounds__(256) void kfac_prep_kernel(KfacPrepArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int nA = a.dA[b], nG = a.dG[b];
  const int r0 = blockIdx.y * PREP_ROWS;
  if (r0 >= nA && r0 >= nG) return;
  const float* A = a.factors + a.offA[b];
  const float* G = a.factors + a.offG[b];
  __shared__ double red[2][256];
  double ta = 0.0, tg = 0.0;
  for (int i = tid; i < nA; i += 256) ta += (double)A[(size_t)i * nA + i];
  for (int i = tid; i < nG; i += 256) tg += (double)G[(size_t)i * nG + i];
  red[0][tid] = ta;
  red[1][tid] = tg;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  ta = red[0][0] / nA;
  tg = red[1][0] / nG;
  const double pi = (ta > 0.0 && tg > 0.0) ? sqrt(ta / tg) : 1.0;
  const double dA = pi * a.sqrt_damping, dG = a.sqrt_damping / pi;
  double* LA = a.S + a.offLA[b];
  double* LG = a.S + a.offLG[b];
  double* Y = a.S + a.offY[b];
  const float* M = a.grad + a.offP[b];
  for (int r = r0; r < r0 + PREP_ROWS; ++r) {
    if (r < nA) {
      const size_t o = (size_t)r * nA;
      for (int c = tid; c < nA; c += 256) LA[o + c] = (double)A[o + c] + (r == c ? dA : 0.0);
      const size_t om = (size_t)r * nG;
      for (int c = tid; c < nG; c += 256) Y[om + c] = (double)M[om + c];
    }
    if (r < nG) {
      const size_t o = (size_t)r * nG;
      for (int c = tid; c < nG; c += 256) LG[o + c] = (double)G[o + c] + (r == c ? dG : 0.0);
    }
  }
}

// ------------------------------------------------------------ Cholesky
// Right-looking blocked Cholesky in TB x TB tiles.  Step kb factors the
// diagonal tile in LDS and also stores the inverse of its triangular factor
// (bt.offI), so that the panel below it and every step of the triangular
// solves are small matrix products instead of serial substitutions.

// the factored tile (rows and columns past n padded with identity) and the
// inverse of its lower-triangular factor
__global__ __launch_bounds__(256) void chol_diag_kernel(SpdBatch bt, double* S, int kb) {
  const int mat = blockIdx.x, tid = threadIdx.x;
  const int n = bt.n[mat], t0 = kb * TB;
  if (t0 >= n) return;
  const int tb = min(TB, n - t0);
  double* A = S + bt.off[mat];
  double* I = S + bt.offI[mat] + (size_t)kb * TB * TB;
  __shared__ double D[TB][TB + 1], V[TB][TB + 1], RD[TB];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    D[r][c] = (r < tb && c < tb) ? A[(size_t)(t0 + r) * n + t0 + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // the factorisation in one wavefront: lane i < TB holds row i in
  // registers; column j's pivot and entries reach every lane by readlane
  // (uniform lane indices), so no barrier is needed.  Lanes past TB work on
  // zero rows and store nothing.
  if (tid < 64) {
    const int i = tid;
    double a[TB];
#pragma unroll
    for (int k = 0; k < TB; ++k) a[k] = i < TB ? D[i][k] : 0.0;
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const double d = sqrt(readlane_f64(a[j], j)), rd = 1.0 / d;
      a[j] = i == j ? d : (i > j ? a[j] * rd : a[j]);
#pragma unroll
      for (int k = j + 1; k < TB; ++k) {
        const double lkj = readlane_f64(a[j], k);
        a[k] = i >= k ? a[k] - a[j] * lkj : a[k];
      }
    }
    if (i < TB) {
#pragma unroll
      for (int k = 0; k < TB; ++k) D[i][k] = a[k];
      // the reciprocals of the diagonal, off the substitution's critical path
#pragma unroll
      for (int k = 0; k < TB; ++k)
        if (k == i) RD[i] = 1.0 / a[k];
    }
  }
  __syncthreads();
  // V = D^-1 (lower triangular) by forward substitution, column c by the
  // eight lanes 8 c .. 8 c + 7: row r of the column is
  //   (delta_rc - sum_{c <= k < r} D[r][k] V[k][c]) / D[r][r],
  // each lane summing k = c + g, c + g + 8, ... and keeping its own V[k][c]
  {
    const int c = tid >> 3, g = tid & 7;
    double vk[TB / 8];
#pragma unroll
    for (int q = 0; q < TB / 8; ++q) vk[q] = 0.0;
    for (int r = 0; r < TB; ++r) {
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < TB / 8; ++q) {
        const int k = c + g + 8 * q;
        if (k < r) part += D[r][k] * vk[q];
      }
      part += __shfl_xor(part, 1, 8);
      part += __shfl_xor(part, 2, 8);
      part += __shfl_xor(part, 4, 8);
      const double x = r < c ? 0.0 : ((r == c ? 1.0 : 0.0) - part) * RD[r];
#pragma unroll
      for (int q = 0; q < TB / 8; ++q)
        if (r == c + g + 8 * q) vk[q] = x;
      if (g == 0) V[r][c] = x;
    }
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (r < tb && c <= r) A[(size_t)(t0 + r) * n + t0 + c] = D[r][c];
    I[e] = V[r][c];
  }
}

// tiles (ib, kb), ib > kb: L[ib][kb] = A[ib][kb] D^-T
__global__ __launch_bounds__(256) void chol_panel_kernel(SpdBatch bt, double* S, int kb) {
  const int mat = blockIdx.x, ib = blockIdx.y, tid = threadIdx.x;
  const int n = bt.n[mat], nt = (n + TB - 1) / TB;
  if (ib <= kb || ib >= nt) return;
  const int t0 = kb * TB, r0 = ib * TB, rb = min(TB, n - r0);
  double* A = S + bt.off[mat];
  const double* I = S + bt.offI[mat] + (size_t)kb * TB * TB;
  __shared__ double V[TB][TB + 1], P[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    V[r][c] = I[e];
    P[r][c] = r < rb ? A[(size_t)(r0 + r) * n + t0 + c] : 0.0;  // kb < ib: the tile's columns are whole
  }
  __syncthreads();
  tile_mm_f64(
      tid, [&](int r, int k) { return P[r][k]; }, [&](int k, int c) { return V[c][k]; },
      [&](int r, int c, double v) {
        if (r < rb) A[(size_t)(r0 + r) * n + t0 + c] = v;
      });
}

// trailing tiles (ib, jb), kb < jb <= ib: A[ib][jb] -= L[ib][kb] L[jb][kb]^T;
// blockIdx.y enumerates the pairs (ii, jj), jj <= ii, of the tiles after kb
__global__ __launch_bounds__(256) void chol_update_kernel(SpdBatch bt, double* S, int kb) {
  const int mat = blockIdx.x, tid = threadIdx.x;
  const int n = bt.n[mat], nt = (n + TB - 1) / TB;
  const int rem = nt - kb - 1;
  const int p = blockIdx.y;
  if (rem <= 0 || p >= rem * (rem + 1) / 2) return;
  int ii = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (ii * (ii + 1) / 2 > p) --ii;
  while ((ii + 1) * (ii + 2) / 2 <= p) ++ii;
  const int jj = p - ii * (ii + 1) / 2;
  const int ib = kb + 1 + ii, jb = kb + 1 + jj;
  const int t0 = kb * TB, r0 = ib * TB, c0 = jb * TB;
  const int rb = min(TB, n - r0), cb = min(TB, n - c0);
  double* A = S + bt.off[mat];
  __shared__ double Pi[TB][TB + 1], Pj[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    Pi[r][c] = r < rb ? A[(size_t)(r0 + r) * n + t0 + c] : 0.0;
    Pj[r][c] = r < cb ? A[(size_t)(c0 + r) * n + t0 + c] : 0.0;
  }
  __syncthreads();
  tile_mm_f64(
      tid, [&](int r, int k) { return Pi[r][k]; }, [&](int k, int c) { return Pj[c][k]; },
      [&](int r, int c, double v) {
        if (r < rb && c < cb) A[(size_t)(r0 + r) * n + c0 + c] -= v;
      });
}

// ------------------------------------------------------------ triangular solves
// B [n][m] row-major, solved in place for L L^T X = B in two sweeps over the
// row blocks, one launch per block step; bt.offZ is an n x m scratch.
//   forward, step kb:  Z_kb = D_kb^-1 B_kb (written to the scratch by the
//     workgroup of row block kb); every row block ib > kb forms Z_kb itself
//     and updates B_ib -= L[ib][kb] Z_kb in place;
//   backward, step kb: X_kb = D_kb^-T Z_kb (written to B by row block kb);
//     every row block ib < kb forms X_kb itself and updates
//     Z_ib -= L[kb][ib]^T X_kb in place.
// Within a launch every workgroup reads only block kb of the sweep's input,
// which no workgroup of that launch writes.
__global__ __launch_bounds__(256) void trsm_step_kernel(SpdBatch bt, double* S, int kb, int upper) {
  const int mat = blockIdx.x, ib = blockIdx.y, ct = blockIdx.z, tid = threadIdx.x;
  const int n = bt.n[mat], m = bt.m[mat], nt = (n + TB - 1) / TB;
  if (kb >= nt || ib >= nt || ct * TB >= m || (upper ? ib > kb : ib < kb)) return;
  const int t0 = kb * TB, r0 = ib * TB, c0 = ct * TB;
  const int tb = min(TB, n - t0), rb = min(TB, n - r0), cb = min(TB, m - c0);
  const double* L = S + bt.off[mat];
  const double* I = S + bt.offI[mat] + (size_t)kb * TB * TB;
  double* src = S + (upper ? bt.offZ[mat] : bt.offB[mat]);  // this sweep's input (updated in place)
  double* dst = S + (upper ? bt.offB[mat] : bt.offZ[mat]);  // this sweep's output
  __shared__ double V[TB][TB + 1], Bk[TB][TB + 1], Zk[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    // V[r][k]: the coefficient of Bk[k] in row r of the block's solution
    V[r][c] = upper ? I[c * TB + r] : I[e];
    Bk[r][c] = (r < tb && c < cb) ? src[(size_t)(t0 + r) * m + c0 + c] : 0.0;
  }
  __syncthreads();
  tile_mm_f64(
      tid, [&](int r, int k) { return V[r][k]; }, [&](int k, int c) { return Bk[k][c]; },
      [&](int r, int c, double v) { Zk[r][c] = v; });
  __syncthreads();
  if (ib == kb) {
    for (int e = tid; e < TB * TB; e += 256) {
      const int r = e / TB, c = e % TB;
      if (r < tb && c < cb) dst[(size_t)(t0 + r) * m + c0 + c] = Zk[r][c];
    }
    return;
  }
  // T[r][k]: the coefficient of Zk[k] in row r of block ib
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (!upper) V[r][c] = (r < rb && c < tb) ? L[(size_t)(r0 + r) * n + t0 + c] : 0.0;
    else V[r][c] = (r < rb && c < tb) ? L[(size_t)(t0 + c) * n + r0 + r] : 0.0;
  }
  __syncthreads();
  tile_mm_f64(
      tid, [&](int r, int k) { return V[r][k]; }, [&](int k, int c) { return Zk[k][c]; },
      [&](int r, int c, double v) {
        if (r < rb && c < cb) src[(size_t)(r0 + r) * m + c0 + c] -= v;
      });
}

// ------------------------------------------------------------ transposes
// Y_b [nA][nG] -> Yt_b [nG][nA]; blockIdx.x the layer, y / z 32 x 32 tiles
__global__ __launch_bounds__(256) void kfac_transpose_kernel(KfacPrepArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int nA = a.dA[b], nG = a.dG[b];
  const int r0 = blockIdx.y * TB, c0 = blockIdx.z * TB;
  if (r0 >= nA || c0 >= nG) return;
  const double* Y = a.S + a.offY[b];
  double* Yt = a.S + a.offYt[b];
  __shared__ double T[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (r0 + r < nA && c0 + c < nG) T[r][c] = Y[(size_t)(r0 + r) * nG + c0 + c];
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 256) {
    const int c = e / TB, r = e % TB;
    if (r0 + r < nA && c0 + c < nG) Yt[(size_t)(c0 + c) * nA + r0 + r] = T[r][c];
  }
}

// update[offP + r nG + c] = Xt[c][r] (float)
__global__ __launch_bounds__(256) void kfac_write_kernel(KfacPrepArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int nA = a.dA[b], nG = a.dG[b];
  const int r0 = blockIdx.y * TB, c0 = blockIdx.z * TB;
  if (r0 >= nA || c0 >= nG) return;
  const double* Xt = a.S + a.offYt[b];
  float* U = a.update + a.offP[b];
  __shared__ double T[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int c = e / TB, r = e % TB;
    if (r0 + r < nA && c0 + c < nG) T[c][r] = Xt[(size_t)(c0 + c) * nA + r0 + r];
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (r0 + r < nA && c0 + c < nG) U[(size_t)(r0 + r) * nG + c0 + c] = (float)T[c][r];
  }
}

// ------------------------------------------------------------ drivers
static int max_tiles(const SpdBatch& bt) {
  int t = 0;
  for (int i = 0; i < bt.nm; ++i) t = std::max(t, (bt.n[i] + TB - 1) / TB);
  return t;
}

hipError_t launch_spd_cholesky(const SpdBatch& bt, double* S, hipStream_t s) {
  if (bt.nm <= 0) return hipSuccess;
  if (bt.nm > KFAC_MAX_MATS) return hipErrorInvalidValue;
  const int nt = max_tiles(bt);
  for (int kb = 0; kb < nt; ++kb) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(bt.nm), dim3(256), 0, s, bt, S, kb);
    if (kb + 1 < nt) {
      hipLaunchKernelGGL(chol_panel_kernel, dim3(bt.nm, nt), dim3(256), 0, s, bt, S, kb);
      const int rem = nt - kb - 1;
      hipLaunchKernelGGL(chol_update_kernel, dim3(bt.nm, rem * (rem + 1) / 2), dim3(256), 0, s, bt, S, kb);
    }
  }
  return hipGetLastError();
}

hipError_t launch_spd_solve(const SpdBatch& bt, double* S, hipStream_t s) {
  if (bt.nm <= 0) return hipSuccess;
  if (bt.nm > KFAC_MAX_MATS) return hipErrorInvalidValue;
  const int nt = max_tiles(bt);
  int ct = 0;
  for (int i = 0; i < bt.nm; ++i) ct = std::max(ct, (bt.m[i] + TB - 1) / TB);
  for (int kb = 0; kb < nt; ++kb)
    hipLaunchKernelGGL(trsm_step_kernel, dim3(bt.nm, nt, ct), dim3(256), 0, s, bt, S, kb, 0);
  for (int kb = nt - 1; kb >= 0; --kb)
    hipLaunchKernelGGL(trsm_step_kernel, dim3(bt.nm, nt, ct), dim3(256), 0, s, bt, S, kb, 1);
  return hipGetLastError();
}

hipError_t launch_kfac_prep(const KfacPrepArgs& a, hipStream_t s) {
  if (a.nb <= 0) return hipSuccess;
  int rows = 0;
  for (int b = 0; b < a.nb; ++b) rows = std::max(rows, std::max(a.dA[b], a.dG[b]));
  hipLaunchKernelGGL(kfac_prep_kernel, dim3(a.nb, (rows + PREP_ROWS - 1) / PREP_ROWS), dim3(256), 0, s, a);
  return hipGetLastError();
}

static void tile_grid(const KfacPrepArgs& a, int* ty, int* tz) {
  int mA = 0, mG = 0;
  for (int b = 0; b < a.nb; ++b) {
    mA = std::max(mA, a.dA[b]);
    mG = std::max(mG, a.dG[b]);
  }
  *ty = (mA + TB - 1) / TB;
  *tz = (mG + TB - 1) / TB;
}

hipError_t launch_kfac_transpose(const KfacPrepArgs& a, hipStream_t s) {
  if (a.nb <= 0) return hipSuccess;
  int ty, tz;
  tile_grid(a, &ty, &tz);
  hipLaunchKernelGGL(kfac_transpose_kernel, dim3(a.nb, ty, tz), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_kfac_write(const KfacPrepArgs& a, hipStream_t s) {
  if (a.nb <= 0) return hipSuccess;
  int ty, tz;
  tile_grid(a, &ty, &tz);
  hipLaunchKernelGGL(kfac_write_kernel, dim3(a.nb, ty, tz), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fn
