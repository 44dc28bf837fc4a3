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

// ------------------------------------------------------------- set-up
// per dense layer b: damped copies of A and G, and M, in float64
__global__ __launch_bounds__(256) void kfac_prep_kernel(KfacPrepArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int nA = a.dA[b], nG = a.dG[b];
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
  for (int64_t e = tid; e < (int64_t)nA * nA; e += 256) {
    const int64_t r = e / nA, c = e - r * nA;
    LA[e] = (double)A[e] + (r == c ? dA : 0.0);
  }
  for (int64_t e = tid; e < (int64_t)nG * nG; e += 256) {
    const int64_t r = e / nG, c = e - r * nG;
    LG[e] = (double)G[e] + (r == c ? dG : 0.0);
  }
  const float* M = a.grad + a.offP[b];
  for (int64_t e = tid; e < (int64_t)nA * nG; e += 256) Y[e] = (double)M[e];
}

// ------------------------------------------------------------ Cholesky
// the factored tile in LDS; rows and columns past n padded with identity
__global__ __launch_bounds__(256) void chol_diag_kernel(SpdBatch bt, double* S, int kb) {
  const int mat = blockIdx.x, tid = threadIdx.x;
  const int n = bt.n[mat], t0 = kb * TB;
  if (t0 >= n) return;
  const int tb = min(TB, n - t0);
  double* A = S + bt.off[mat];
  __shared__ double D[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    D[r][c] = (r < tb && c < tb) ? A[(size_t)(t0 + r) * n + t0 + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < tb; ++j) {
    if (tid == 0) D[j][j] = sqrt(D[j][j]);
    __syncthreads();
    for (int i = j + 1 + tid; i < tb; i += 256) D[i][j] /= D[j][j];
    __syncthreads();
    for (int e = tid; e < TB * TB; e += 256) {
      const int i = e / TB, k = e % TB;
      if (k > j && k <= i && i < tb) D[i][k] -= D[i][j] * D[k][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (r < tb && c <= r) A[(size_t)(t0 + r) * n + t0 + c] = D[r][c];
  }
}

// tiles (ib, kb), ib > kb: rows of A[ib][kb] D^-T, one row per thread
__global__ __launch_bounds__(64) void chol_panel_kernel(SpdBatch bt, double* S, int kb) {
  const int mat = blockIdx.x, ib = blockIdx.y, tid = threadIdx.x;
  const int n = bt.n[mat], nt = (n + TB - 1) / TB;
  if (ib <= kb || ib >= nt) return;
  const int t0 = kb * TB, r0 = ib * TB, rb = min(TB, n - r0);
  double* A = S + bt.off[mat];
  __shared__ double D[TB][TB + 1], P[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 64) {
    const int r = e / TB, c = e % TB;
    D[r][c] = A[(size_t)(t0 + r) * n + t0 + c];  // kb < ib: the diagonal tile is whole
    P[r][c] = r < rb ? A[(size_t)(r0 + r) * n + t0 + c] : 0.0;
  }
  __syncthreads();
  if (tid < rb) {
    for (int j = 0; j < TB; ++j) {
      double s = P[tid][j];
      for (int k = 0; k < j; ++k) s -= P[tid][k] * D[j][k];
      P[tid][j] = s / D[j][j];
    }
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 64) {
    const int r = e / TB, c = e % TB;
    if (r < rb) A[(size_t)(r0 + r) * n + t0 + c] = P[r][c];
  }
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
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (r >= rb || c >= cb) continue;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < TB; ++k) s += Pi[r][k] * Pj[c][k];
    A[(size_t)(r0 + r) * n + c0 + c] -= s;
  }
}

// ------------------------------------------------------------ triangular solves
// B [n][m] row-major in place: forward L Z = B (upper = 0) or backward
// L^T Z = B (upper = 1), step kb: the diagonal block, one column per thread
__global__ __launch_bounds__(64) void trsm_diag_kernel(SpdBatch bt, double* S, int kb, int upper) {
  const int mat = blockIdx.x, ct = blockIdx.y, tid = threadIdx.x;
  const int n = bt.n[mat], m = bt.m[mat], t0 = kb * TB;
  if (t0 >= n || ct * TB >= m) return;
  const int tb = min(TB, n - t0), c0 = ct * TB, cb = min(TB, m - c0);
  const double* L = S + bt.off[mat];
  double* B = S + bt.offB[mat];
  __shared__ double D[TB][TB + 1], Z[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 64) {
    const int r = e / TB, c = e % TB;
    D[r][c] = (r < tb && c < tb && c <= r) ? L[(size_t)(t0 + r) * n + t0 + c] : 0.0;
    Z[r][c] = (r < tb && c < cb) ? B[(size_t)(t0 + r) * m + c0 + c] : 0.0;
  }
  __syncthreads();
  if (tid < cb) {
    if (!upper) {
      for (int r = 0; r < tb; ++r) {
        double s = Z[r][tid];
        for (int k = 0; k < r; ++k) s -= D[r][k] * Z[k][tid];
        Z[r][tid] = s / D[r][r];
      }
    } else {
      for (int r = tb - 1; r >= 0; --r) {
        double s = Z[r][tid];
        for (int k = r + 1; k < tb; ++k) s -= D[k][r] * Z[k][tid];
        Z[r][tid] = s / D[r][r];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 64) {
    const int r = e / TB, c = e % TB;
    if (r < tb && c < cb) B[(size_t)(t0 + r) * m + c0 + c] = Z[r][c];
  }
}

// the other row blocks after step kb: forward B[ib] -= L[ib][kb] Z[kb]
// (ib > kb); backward B[ib] -= L[kb][ib]^T Z[kb] (ib < kb)
__global__ __launch_bounds__(256) void trsm_update_kernel(SpdBatch bt, double* S, int kb, int upper) {
  const int mat = blockIdx.x, ib = blockIdx.y, ct = blockIdx.z, tid = threadIdx.x;
  const int n = bt.n[mat], m = bt.m[mat], nt = (n + TB - 1) / TB;
  if (ib >= nt || kb >= nt || ct * TB >= m || (upper ? ib >= kb : ib <= kb)) return;
  const int t0 = kb * TB, r0 = ib * TB, c0 = ct * TB;
  const int tb = min(TB, n - t0), rb = min(TB, n - r0), cb = min(TB, m - c0);
  const double* L = S + bt.off[mat];
  double* B = S + bt.offB[mat];
  __shared__ double T[TB][TB + 1], Z[TB][TB + 1];
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    // T[r][k]: the coefficient of Z[kb][k] in row r of block ib
    if (!upper) T[r][c] = (r < rb && c < tb) ? L[(size_t)(r0 + r) * n + t0 + c] : 0.0;
    else T[r][c] = (r < rb && c < tb) ? L[(size_t)(t0 + c) * n + r0 + r] : 0.0;
    Z[r][c] = (r < tb && c < cb) ? B[(size_t)(t0 + r) * m + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e / TB, c = e % TB;
    if (r >= rb || c >= cb) continue;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < TB; ++k) s += T[r][k] * Z[k][c];
    B[(size_t)(r0 + r) * m + c0 + c] -= s;
  }
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
      hipLaunchKernelGGL(chol_panel_kernel, dim3(bt.nm, nt), dim3(64), 0, s, bt, S, kb);
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
  for (int kb = 0; kb < nt; ++kb) {
    hipLaunchKernelGGL(trsm_diag_kernel, dim3(bt.nm, ct), dim3(64), 0, s, bt, S, kb, 0);
    if (kb + 1 < nt) hipLaunchKernelGGL(trsm_update_kernel, dim3(bt.nm, nt, ct), dim3(256), 0, s, bt, S, kb, 0);
  }
  for (int kb = nt - 1; kb >= 0; --kb) {
    hipLaunchKernelGGL(trsm_diag_kernel, dim3(bt.nm, ct), dim3(64), 0, s, bt, S, kb, 1);
    if (kb > 0) hipLaunchKernelGGL(trsm_update_kernel, dim3(bt.nm, nt, ct), dim3(256), 0, s, bt, S, kb, 1);
  }
  return hipGetLastError();
}

hipError_t launch_kfac_prep(const KfacPrepArgs& a, hipStream_t s) {
  if (a.nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(kfac_prep_kernel, dim3(a.nb), dim3(256), 0, s, a);
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
