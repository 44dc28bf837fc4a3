// Determinants of Eq. (4) and the local energy.
//
// One wavefront per (walker, determinant k, spin a) orbital matrix B with
// B[j][i] = phi^{ka}_i(r_j) (the transpose of A^{ka}; same determinant):
// LU with partial pivoting in LDS -> sign and log|det B|, B^-1, and in jet
// mode the contractions with the jets of B:
//   d_c = tr(B^-1 dB/dx_c)                 (d log|det| / dx_c)
//   q   = sum_c tr((B^-1 dB/dx_c)^2)
//   lap = tr(B^-1 lap(B))
// so that lap log|det| = lap - q, and in jet mode the condition number
// cond_1(A) = ||B||_inf ||B^-1||_inf of the orbital matrix A = B^T (row sums
// of B taken before the factorisation).  R = double in the bf16 form, float
// in the fp32 form.
//
// The combination (one wavefront per walker) forms psi = sum_k s_k e^{l_k}
// as a signed log-sum-exp, rho_k = P_k / psi, and
//   lap(psi)/psi = sum_k rho_k [sum_a (lap_a - q_a) + sum_c (d_c^up + d_c^down)^2]
//   E_kin = -lap(psi)/(2 psi)
// plus the Coulomb potential of Eq. (2) by wavefront reductions (float64).
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace fn {

constexpr int MAXNA = 32;

// PT: type of the orbital jets (float, or double with R = double)
template <class R, class PT>
__global__ __launch_bounds__(64) void det_kernel(const PT* phi, int K, int na, int T, int n3, R* D, int dstride,
                                                 R* ainv) {
  __shared__ R LU[MAXNA * MAXNA];
  __shared__ R Bi[MAXNA * MAXNA];
  __shared__ R Ys[64 + MAXNA * MAXNA];
  __shared__ int piv[MAXNA];
  __shared__ int s_p;
  __shared__ R s_part[64];
  const int lane = threadIdx.x;
  const int64_t mat = blockIdx.x;  // = w * K + k
  const int nsq = na * na;
  const PT* P = phi + mat * (int64_t)T * nsq;
  R* out = D + mat * dstride;

  for (int e = lane; e < nsq; e += 64) LU[e] = (R)P[e];
  __syncthreads();
  R nb = 0;  // ||B||_inf
  if (T > 1) {
    for (int r = lane; r < na; r += 64) {
      R rs = 0;
      for (int k = 0; k < na; ++k) rs += fabs(LU[r * na + k]);
      nb = rs;
    }
    nb = wave_max(nb);
  }
  bool singular = false;
  for (int c = 0; c < na; ++c) {
    if (lane == 0) {
      int p = c;
      R best = fabs(LU[c * na + c]);
      for (int r = c + 1; r < na; ++r) {
        R m = fabs(LU[r * na + c]);
        if (m > best) {
          best = m;
          p = r;
        }
      }
      s_p = best == (R)0 ? -1 : p;
      piv[c] = p;
    }
    __syncthreads();
    const int p = s_p;
    if (p < 0) {
      singular = true;
      break;
    }
    if (p != c)
      for (int k = lane; k < na; k += 64) {
        R t = LU[c * na + k];
        LU[c * na + k] = LU[p * na + k];
        LU[p * na + k] = t;
      }
    __syncthreads();
    const R inv_p = (R)1 / LU[c * na + c];
    for (int r = c + 1 + lane; r < na; r += 64) {
      const R f = LU[r * na + c] * inv_p;
      LU[r * na + c] = f;
      for (int k = c + 1; k < na; ++k) LU[r * na + k] -= f * LU[c * na + k];
    }
    __syncthreads();
  }
  if (singular) {
    for (int e = lane; e < dstride; e += 64) out[e] = (R)0;
    if (lane == 0) {
      out[1] = -INFINITY;
      if (T > 1) out[4 + n3] = INFINITY;
    }
    if (ainv)
      for (int e = lane; e < nsq; e += 64) ainv[mat * nsq + e] = (R)0;
    return;
  }
  if (lane == 0) {
    R sg = 1, la = 0;
    for (int c = 0; c < na; ++c) {
      if (piv[c] != c) sg = -sg;
      R u = LU[c * na + c];
      if (u < 0) sg = -sg;
      la += log(fabs(u));
    }
    out[0] = sg;
    out[1] = la;
  }
  const bool need_inv = ainv != nullptr || T > 1;
  if (!need_inv) return;
  // B^-1 column by column: lane c solves L U x = P e_c (in the Bi column)
  for (int c = lane; c < na; c += 64) {
    for (int r = 0; r < na; ++r) Bi[r * na + c] = r == c ? (R)1 : (R)0;
    for (int k = 0; k < na; ++k)
      if (piv[k] != k) {
        R t = Bi[k * na + c];
        Bi[k * na + c] = Bi[piv[k] * na + c];
        Bi[piv[k] * na + c] = t;
      }
    for (int r = 0; r < na; ++r) {
      R acc = Bi[r * na + c];
      for (int k = 0; k < r; ++k) acc -= LU[r * na + k] * Bi[k * na + c];
      Bi[r * na + c] = acc;
    }
    for (int r = na - 1; r >= 0; --r) {
      R acc = Bi[r * na + c];
      for (int k = r + 1; k < na; ++k) acc -= LU[r * na + k] * Bi[k * na + c];
      Bi[r * na + c] = acc / LU[r * na + r];
    }
  }
  __syncthreads();
  if (ainv)
    for (int e = lane; e < nsq; e += 64) ainv[mat * nsq + e] = Bi[e];
  if (T <= 1) return;
  {
    R ni = 0;  // ||B^-1||_inf
    for (int r = lane; r < na; r += 64) {
      R rs = 0;
      for (int k = 0; k < na; ++k) rs += fabs(Bi[r * na + k]);
      ni = rs;
    }
    ni = wave_max(ni);
    if (lane == 0) out[4 + n3] = nb * ni;
  }

  // jet contractions; "tangent" index tt in [0, n3] where tt == n3 is the
  // Laplacian row (trace only)
  const int G = nsq <= 64 ? 64 / nsq : 1;
  R q_acc = 0;
  for (int t0 = 0; t0 <= n3; t0 += G) {
    const int ng = (t0 + G <= n3 + 1) ? G : (n3 + 1 - t0);
    R dpart = 0, qpart = 0;
    // Y = B^-1 M_t
    for (int e = lane; e < ng * nsq; e += 64) {
      const int gi = e / nsq, ab = e % nsq, ar = ab / na, b = ab % na;
      const int tt = t0 + gi;
      const int row = tt < n3 ? 1 + tt : T - 1;
      const PT* M = P + (int64_t)row * nsq;
      R acc = 0;
      for (int c = 0; c < na; ++c) acc += Bi[ar * na + c] * (R)M[c * na + b];
      Ys[e] = acc;
    }
    __syncthreads();
    for (int e = lane; e < ng * nsq; e += 64) {
      const int gi = e / nsq, ab = e % nsq, ar = ab / na, b = ab % na;
      const R y = Ys[e];
      R dp = ar == b ? y : (R)0;
      R qp = y * Ys[gi * nsq + b * na + ar];
      if (G == 1) {
        dpart += dp;
        qpart += qp;
      } else {
        // one element per lane: stash for the per-tangent sums below
        Ys[64 + e] = qp;  // region beyond 64 is free when nsq <= 64... guarded below
        (void)dp;
      }
    }
    if (G == 1) {
      dpart = wave_sum(dpart);
      qpart = wave_sum(qpart);
      if (lane == 0) {
        if (t0 < n3) {
          out[2 + t0] = dpart;
          q_acc += qpart;
        } else {
          out[3 + n3] = dpart;
        }
      }
    } else {
      __syncthreads();
      if (lane < ng) {
        const int tt = t0 + lane;
        R dsum = 0, qsum = 0;
        for (int ab = 0; ab < nsq; ++ab) {
          const int ar = ab / na, b = ab % na;
          if (ar == b) dsum += Ys[lane * nsq + ab];
          qsum += Ys[64 + lane * nsq + ab];
        }
        if (tt < n3) {
          out[2 + tt] = dsum;
          q_acc += qsum;
        } else {
          out[3 + n3] = dsum;
        }
      }
    }
    __syncthreads();
  }
  s_part[lane] = q_acc;
  __syncthreads();
  if (lane == 0) {
    R q = 0;
    for (int l = 0; l < 64; ++l) q += s_part[l];
    out[2 + n3] = q;
  }
}

// Matrices of 7..16 rows: one 256-thread workgroup per matrix.  The
// factorisation and B^-1 are as in det_kernel (rows in parallel); the
// contractions, which carry almost all of the arithmetic (n_a^3 per
// tangent, 3n + 1 tangents), are organised so that every jet element is
// read from HBM once:
//  * the tangent matrices M_t are staged into LDS MID_G at a time (rows
//    1 .. T-1 of the matrix's jets are contiguous: one coalesced copy);
//  * thread (slot, a, b) keeps row a of B^-1 in registers and forms
//    Y_t[a][b] = sum_c B^-1[a][c] M_t[c][b] for the tangents t of its slot;
//  * tr(Y_t^2) = sum_ab Y_t[a][b] Y_t[b][a] is accumulated per thread over
//    all tangents and reduced once at the end; tr(Y_t) is summed per
//    tangent by one thread.
constexpr int MID_NT = 256, MID_G = 8;

template <class R>
__device__ inline R block_reduce(R v, R* red, bool is_max) {
  v = is_max ? wave_max(v) : wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  R t = red[0];
  for (int i = 1; i < MID_NT / 64; ++i) t = is_max ? (red[i] > t ? red[i] : t) : t + red[i];
  return t;
}

template <class R, class PT, int NA>
__global__ __launch_bounds__(MID_NT) void det_mid_kernel(const PT* phi, int T, int n3, R* D, int dstride, R* ainv) {
  constexpr int NSQ = NA * NA;
  constexpr int S = MID_NT / NSQ;  // tangent slots
  __shared__ R LU[NSQ];
  __shared__ R Bi[NSQ];
  __shared__ PT Ms[MID_G * NSQ];
  __shared__ R Ys[MID_G * NSQ];
  __shared__ R red[MID_NT / 64];
  __shared__ int piv[NA];
  __shared__ int s_p;
  const int tid = threadIdx.x;
  const int64_t mat = blockIdx.x;
  const PT* P = phi + mat * (int64_t)T * NSQ;
  R* out = D + mat * dstride;

  for (int e = tid; e < NSQ; e += MID_NT) LU[e] = (R)P[e];
  __syncthreads();
  R nb = 0;  // ||B||_inf
  if (T > 1) {
    R rs = 0;
    if (tid < NA)
      for (int k = 0; k < NA; ++k) rs += fabs(LU[tid * NA + k]);
    nb = block_reduce(rs, red, true);
  }
  bool singular = false;
  for (int c = 0; c < NA; ++c) {
    if (tid == 0) {
      int p = c;
      R best = fabs(LU[c * NA + c]);
      for (int r = c + 1; r < NA; ++r) {
        const R m = fabs(LU[r * NA + c]);
        if (m > best) {
          best = m;
          p = r;
        }
      }
      s_p = best == (R)0 ? -1 : p;
      piv[c] = p;
    }
    __syncthreads();
    const int p = s_p;
    if (p < 0) {
      singular = true;
      break;
    }
    if (p != c && tid < NA) {
      const R t = LU[c * NA + tid];
      LU[c * NA + tid] = LU[p * NA + tid];
      LU[p * NA + tid] = t;
    }
    __syncthreads();
    const R inv_p = (R)1 / LU[c * NA + c];
    const int r = c + 1 + tid;
    if (r < NA) {
      const R f = LU[r * NA + c] * inv_p;
      LU[r * NA + c] = f;
      for (int k = c + 1; k < NA; ++k) LU[r * NA + k] -= f * LU[c * NA + k];
    }
    __syncthreads();
  }
  if (singular) {
    for (int e = tid; e < dstride; e += MID_NT) out[e] = (R)0;
    __syncthreads();
    if (tid == 0) {
      out[1] = -INFINITY;
      if (T > 1) out[4 + n3] = INFINITY;
    }
    if (ainv)
      for (int e = tid; e < NSQ; e += MID_NT) ainv[mat * NSQ + e] = (R)0;
    return;
  }
  if (tid == 0) {
    R sg = 1, la = 0;
    for (int c = 0; c < NA; ++c) {
      if (piv[c] != c) sg = -sg;
      const R u = LU[c * NA + c];
      if (u < 0) sg = -sg;
      la += log(fabs(u));
    }
    out[0] = sg;
    out[1] = la;
  }
  if (ainv == nullptr && T <= 1) return;
  // B^-1 column by column: thread c solves L U x = P e_c
  if (tid < NA) {
    const int c = tid;
    for (int r = 0; r < NA; ++r) Bi[r * NA + c] = r == c ? (R)1 : (R)0;
    for (int k = 0; k < NA; ++k)
      if (piv[k] != k) {
        const R t = Bi[k * NA + c];
        Bi[k * NA + c] = Bi[piv[k] * NA + c];
        Bi[piv[k] * NA + c] = t;
      }
    for (int r = 0; r < NA; ++r) {
      R acc = Bi[r * NA + c];
      for (int k = 0; k < r; ++k) acc -= LU[r * NA + k] * Bi[k * NA + c];
      Bi[r * NA + c] = acc;
    }
    for (int r = NA - 1; r >= 0; --r) {
      R acc = Bi[r * NA + c];
      for (int k = r + 1; k < NA; ++k) acc -= LU[r * NA + k] * Bi[k * NA + c];
      Bi[r * NA + c] = acc / LU[r * NA + r];
    }
  }
  __syncthreads();
  if (ainv)
    for (int e = tid; e < NSQ; e += MID_NT) ainv[mat * NSQ + e] = Bi[e];
  if (T <= 1) return;
  {
    R rs = 0;  // ||B^-1||_inf
    if (tid < NA)
      for (int k = 0; k < NA; ++k) rs += fabs(Bi[tid * NA + k]);
    const R ni = block_reduce(rs, red, true);
    if (tid == 0) out[4 + n3] = nb * ni;
  }
  const int slot = tid / NSQ, ab = tid - slot * NSQ, a = ab / NA, b = ab - a * NA;
  const bool act = slot < S;
  R brow[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c) brow[c] = act ? Bi[a * NA + c] : (R)0;
  R q_acc = 0;
  const int nt = n3 + 1;  // the 3n tangent rows and the Laplacian row, rows 1 .. T-1
  for (int t0 = 0; t0 < nt; t0 += MID_G) {
    const int ng = nt - t0 < MID_G ? nt - t0 : MID_G;
    const PT* src = P + (int64_t)(1 + t0) * NSQ;
    for (int e = tid; e < ng * NSQ; e += MID_NT) Ms[e] = src[e];
    __syncthreads();
    if (act)
      for (int g = slot; g < ng; g += S) {
        R y = 0;
#pragma unroll
        for (int c = 0; c < NA; ++c) y += brow[c] * (R)Ms[g * NSQ + c * NA + b];
        Ys[g * NSQ + ab] = y;
      }
    __syncthreads();
    if (act)
      for (int g = slot; g < ng; g += S)
        if (t0 + g < n3) q_acc += Ys[g * NSQ + ab] * Ys[g * NSQ + b * NA + a];
    if (tid < ng) {
      R d = 0;
      for (int i = 0; i < NA; ++i) d += Ys[tid * NSQ + i * NA + i];
      const int tt = t0 + tid;
      out[tt < n3 ? 2 + tt : 3 + n3] = d;
    }
    __syncthreads();
  }
  const R q = block_reduce(q_acc, red, false);
  if (tid == 0) out[2 + n3] = q;
}

// Value-only determinants (sign and log|det|, no inverse) of 7..16-row
// matrices, as the Metropolis and log|psi| passes need them: four matrices
// per wavefront, sixteen lanes each, lane r of a group holding row r of its
// matrix in registers.  Partial pivoting by a shuffle reduction over the
// group (ties to the lower row, as in the LU of det_mid_kernel), the row
// exchange and the pivot-row broadcast by shuffles; no LDS, no barriers.
template <class R, class PT, int NA>
__global__ __launch_bounds__(256) void det_value_kernel(const PT* phi, int64_t M, R* D, int dstride) {
  const int lane = threadIdx.x & 63, r = lane & 15, base = lane & ~15;
  const int64_t mat = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;  // uniform over the 16 lanes
  const bool valid = mat < M;
  const PT* P = phi + (valid ? mat : 0) * (int64_t)(NA * NA);
  R a[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) a[k] = (valid && r < NA) ? (R)P[r * NA + k] : (R)0;
  R sg = 1, la = 0;
  bool singular = false;
#pragma unroll
  for (int c = 0; c < NA; ++c) {
    R v = (r >= c && r < NA) ? fabs(a[c]) : (R)-1;
    int idx = r;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      const R ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = idx;  // the same in every lane of the group
    if (v == (R)0) singular = true;
    // exchange rows c and p (columns c .. NA-1; the rest is not needed)
    const int src = base + (r == c ? p : (r == p ? c : r));
#pragma unroll
    for (int k = c; k < NA; ++k) a[k] = __shfl(a[k], src, 64);
    R u[NA];
#pragma unroll
    for (int k = c; k < NA; ++k) u[k] = __shfl(a[k], base + c, 64);
    const R piv = singular ? (R)1 : u[c];
    if (p != c) sg = -sg;
    if (piv < 0) sg = -sg;
    la += log(fabs(piv));
    const R inv_p = (R)1 / piv;  // the factorisation's own arithmetic (det_mid_kernel)
    const R f = (r > c && r < NA) ? a[c] * inv_p : (R)0;
#pragma unroll
    for (int k = c + 1; k < NA; ++k) a[k] -= f * u[k];
  }
  if (valid && r == 0) {
    R* out = D + mat * dstride;
    if (singular) {
      for (int e = 0; e < dstride; ++e) out[e] = (R)0;
      out[1] = -INFINITY;
    } else {
      out[0] = sg;
      out[1] = la;
    }
  }
}

template <class R, class PT>
static hipError_t run_det_value(int na, const PT* phi, int64_t M, R* D, int dstride, hipStream_t s) {
  const int grid = (int)((M * 16 + 255) / 256);
#define FN_VAL(N)                                                                                       \
  case N:                                                                                              \
    hipLaunchKernelGGL((det_value_kernel<R, PT, N>), dim3(grid), dim3(256), 0, s, phi, M, D, dstride); \
    break;
  switch (na) {
    FN_VAL(7) FN_VAL(8) FN_VAL(9) FN_VAL(10) FN_VAL(11) FN_VAL(12) FN_VAL(13) FN_VAL(14) FN_VAL(15) FN_VAL(16)
    default: return hipErrorInvalidValue;
  }
#undef FN_VAL
  return hipGetLastError();
}

template <class R, class PT>
static hipError_t run_det_mid(int na, const PT* phi, int grid, int T, int n3, R* D, int dstride, R* ainv,
                              hipStream_t s) {
#define FN_MID(N)                                                                                           \
  case N:                                                                                                  \
    hipLaunchKernelGGL((det_mid_kernel<R, PT, N>), dim3(grid), dim3(MID_NT), 0, s, phi, T, n3, D, dstride, ainv); \
    break;
  switch (na) {
    FN_MID(7) FN_MID(8) FN_MID(9) FN_MID(10) FN_MID(11) FN_MID(12) FN_MID(13) FN_MID(14) FN_MID(15) FN_MID(16)
    default: return hipErrorInvalidValue;
  }
#undef FN_MID
  return hipGetLastError();
}

// Small matrices (n_a <= 6): P threads per matrix (consecutive lanes of one
// wavefront), everything in registers.  The orbital jets are stored
// matrix-index fastest, phi[(t n_a^2 + e) M + mat] with M = W K, so that
// consecutive threads read consecutive addresses.  Each of the P threads
// factors the matrix (the same instructions, so the same bits): Gauss-Jordan
// elimination with partial pivoting on [B | I] gives B^-1, the pivots give
// sign and log|det B|.  The tangent rows are dealt out over the P threads
// (thread p takes t = p, p + P, ...); each writes its d_t, and the terms of
// q = sum_t tr((B^-1 M_t)^2) go through LDS so that the first thread adds
// them in t order, as one thread alone would.
constexpr int DET_SMALL_MAX_TAN = 3 * MAXNA;  // tangent rows of the LDS terms (3n, n <= 32)

template <class R, int NA, class PT, int P>
__global__ __launch_bounds__(64) void det_small_kernel(const PT* phi, int64_t M, int T, int n3, R* D, int dstride,
                                                       R* ainv) {
  constexpr int NSQ = NA * NA, MPB = 64 / P;  // matrices per block (one wavefront)
  __shared__ R qs[P > 1 ? MPB : 1][P > 1 ? DET_SMALL_MAX_TAN : 1];
  const int lm = threadIdx.x / P, p = threadIdx.x % P;
  const int64_t mat = (int64_t)blockIdx.x * MPB + lm;
  const bool valid = mat < M;
  if (P == 1 && !valid) return;
  // lanes past the last matrix factor the last one and store nothing
  const int64_t mr = valid ? mat : M - 1;
  R* out = D + mr * dstride;
  R B[NA][NA], X[NA][NA];
#pragma unroll
  for (int j = 0; j < NA; ++j)
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      B[j][i] = (R)phi[(int64_t)(j * NA + i) * M + mr];
      X[j][i] = j == i ? (R)1 : (R)0;
    }
  R nb = 0;  // ||B||_inf
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    R rs = 0;
#pragma unroll
    for (int i = 0; i < NA; ++i) rs += fabs(B[j][i]);
    nb = fmax(nb, rs);
  }
  R sg = 1, la = 0;
  bool singular = false;
#pragma unroll
  for (int c = 0; c < NA; ++c) {
    // pivot row p >= c with the largest |B[p][c]|; exchange rows c and p
    R best = fabs(B[c][c]);
    int pr = c;
#pragma unroll
    for (int r = c + 1; r < NA; ++r)
      if (fabs(B[r][c]) > best) {
        best = fabs(B[r][c]);
        pr = r;
      }
    if (best == (R)0) singular = true;
#pragma unroll
    for (int r = c + 1; r < NA; ++r)
      if (r == pr) {
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          R t = B[c][k];
          B[c][k] = B[r][k];
          B[r][k] = t;
          t = X[c][k];
          X[c][k] = X[r][k];
          X[r][k] = t;
        }
      }
    if (pr != c) sg = -sg;
    const R piv = singular ? (R)1 : B[c][c];
    if (piv < 0) sg = -sg;
    la += log(fabs(piv));
    const R ip = (R)1 / piv;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      B[c][k] *= ip;
      X[c][k] *= ip;
    }
#pragma unroll
    for (int r = 0; r < NA; ++r)
      if (r != c) {
        const R f = B[r][c];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          B[r][k] -= f * B[c][k];
          X[r][k] -= f * X[c][k];
        }
      }
  }
  const bool lead = valid && p == 0;
  const bool store = valid && !singular;
  if (lead) {
    if (singular) {
      for (int e = 0; e < dstride; ++e) out[e] = (R)0;
      out[1] = -INFINITY;
      if (T > 1) out[4 + n3] = INFINITY;
      if (ainv)
        for (int e = 0; e < NSQ; ++e) ainv[mat * NSQ + e] = (R)0;
    } else {
      out[0] = sg;
      out[1] = la;
      if (ainv) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NA; ++b) ainv[mat * NSQ + a * NA + b] = X[a][b];
      }
    }
  }
  if (T <= 1) return;  // uniform over the launch
  if (lead && !singular) {
    R ni = 0;  // ||B^-1||_inf
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      R rs = 0;
#pragma unroll
      for (int b = 0; b < NA; ++b) rs += fabs(X[a][b]);
      ni = fmax(ni, rs);
    }
    out[4 + n3] = nb * ni;
  }
  // d_t = tr(B^-1 M_t), q = sum_t tr((B^-1 M_t)^2), lap = tr(B^-1 lap B).
  // The next tangent matrix is loaded while this one is multiplied; every
  // step issues the same loads (the last one reloads its own matrix), so
  // that the wait before a step is only for the loads of the step before.
  auto load_t = [&](int tt, PT (&dst)[NA][NA]) {
    const int row = tt < n3 ? 1 + tt : T - 1;
    const PT* Pm = phi + (int64_t)row * NSQ * M + mr;
#pragma unroll
    for (int c = 0; c < NA; ++c)
#pragma unroll
      for (int b = 0; b < NA; ++b) dst[c][b] = Pm[(int64_t)(c * NA + b) * M];
  };
  R q = 0;
  PT nxt[NA][NA];
  if (p <= n3) load_t(p, nxt);
  for (int tt = p; tt <= n3; tt += P) {
    R Mt[NA][NA];
#pragma unroll
    for (int c = 0; c < NA; ++c)
#pragma unroll
      for (int b = 0; b < NA; ++b) Mt[c][b] = (R)nxt[c][b];
    load_t(min(tt + P, n3), nxt);
    R Y[NA][NA];
    R d = 0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NA; ++b) {
        R acc = 0;
#pragma unroll
        for (int c = 0; c < NA; ++c) acc += X[a][c] * Mt[c][b];
        Y[a][b] = acc;
      }
#pragma unroll
    for (int a = 0; a < NA; ++a) d += Y[a][a];
    if (tt < n3) {
      if (store) out[2 + tt] = d;
      R qq = 0;
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NA; ++b) qq += Y[a][b] * Y[b][a];
      if constexpr (P > 1) qs[lm][tt] = qq;
      else q += qq;
    } else if (store) {
      out[3 + n3] = d;
    }
  }
  if constexpr (P > 1) {
    __syncthreads();
    if (lead && !singular)
      for (int tt = 0; tt < n3; ++tt) q += qs[lm][tt];
  }
  if (lead && !singular) out[2 + n3] = q;
}

template <class R, class PT, int P>
static hipError_t run_det_small_p(int na, const PT* phi, int64_t M, int T, int n3, R* D, int dstride, R* ainv,
                                  hipStream_t s) {
  // one wavefront per block, so that the few thousand matrices of a
  // float64 re-evaluation still spread over the compute units
  const int grid = (int)((M + 64 / P - 1) / (64 / P));
  switch (na) {
    case 1: hipLaunchKernelGGL((det_small_kernel<R, 1, PT, P>), dim3(grid), dim3(64), 0, s, phi, M, T, n3, D, dstride, ainv); break;
    case 2: hipLaunchKernelGGL((det_small_kernel<R, 2, PT, P>), dim3(grid), dim3(64), 0, s, phi, M, T, n3, D, dstride, ainv); break;
    case 3: hipLaunchKernelGGL((det_small_kernel<R, 3, PT, P>), dim3(grid), dim3(64), 0, s, phi, M, T, n3, D, dstride, ainv); break;
    case 4: hipLaunchKernelGGL((det_small_kernel<R, 4, PT, P>), dim3(grid), dim3(64), 0, s, phi, M, T, n3, D, dstride, ainv); break;
    case 5: hipLaunchKernelGGL((det_small_kernel<R, 5, PT, P>), dim3(grid), dim3(64), 0, s, phi, M, T, n3, D, dstride, ainv); break;
    case 6: hipLaunchKernelGGL((det_small_kernel<R, 6, PT, P>), dim3(grid), dim3(64), 0, s, phi, M, T, n3, D, dstride, ainv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// threads per matrix: one for the value passes and for batches that give
// every SIMD a wavefront (32768 matrices or more: the extra factorisations
// and loads of more threads cost more than they save, 61 -> 81 us for the
// 65536 matrices of a Ne-like spin at four per matrix); with tangents and
// fewer matrices, up to eight, so that the few wavefronts of a small batch
// (the float64 re-evaluation: 29 -> 12 us for 1968 matrices at eight) take
// fewer serial steps
template <class R, class PT>
static hipError_t run_det_small(int na, const PT* phi, int64_t M, int T, int n3, R* D, int dstride, R* ainv,
                                hipStream_t s) {
  if (T <= 1 || n3 > DET_SMALL_MAX_TAN || M >= 32768)
    return run_det_small_p<R, PT, 1>(na, phi, M, T, n3, D, dstride, ainv, s);
  if (M >= 16384) return run_det_small_p<R, PT, 2>(na, phi, M, T, n3, D, dstride, ainv, s);
  if (M >= 8192) return run_det_small_p<R, PT, 4>(na, phi, M, T, n3, D, dstride, ainv, s);
  return run_det_small_p<R, PT, 8>(na, phi, M, T, n3, D, dstride, ainv, s);
}

bool det_uses_small(int na) { return na <= DET_SMALL_MAX; }

hipError_t launch_det(bool fp64, const void* phi, bool phi64, int W, int K, int na, int T, int n3, void* D,
                      int dstride, void* ainv, hipStream_t s) {
  if (na <= 0 || W <= 0) return hipSuccess;
  if (na > MAXNA || (phi64 && !fp64)) return hipErrorInvalidValue;
  const float* pf = (const float*)phi;
  const double* pd = (const double*)phi;
  if (det_uses_small(na)) {
    const int64_t M = (int64_t)W * K;
    if (phi64) return run_det_small<double, double>(na, pd, M, T, n3, (double*)D, dstride, (double*)ainv, s);
    return fp64 ? run_det_small<double, float>(na, pf, M, T, n3, (double*)D, dstride, (double*)ainv, s)
                : run_det_small<float, float>(na, pf, M, T, n3, (float*)D, dstride, (float*)ainv, s);
  }
  const int grid = W * K;
  // 7..16 rows with the jet rows in their standard order (the Laplacian
  // row directly after the 3n tangent rows)
  if (na <= DET_MID_MAX && T <= 1 && ainv == nullptr) {
    const int64_t M = (int64_t)W * K;
    if (phi64) return run_det_value<double, double>(na, pd, M, (double*)D, dstride, s);
    return fp64 ? run_det_value<double, float>(na, pf, M, (double*)D, dstride, s)
                : run_det_value<float, float>(na, pf, M, (float*)D, dstride, s);
  }
  if (na <= DET_MID_MAX && (T <= 1 || T == n3 + 2)) {
    if (phi64) return run_det_mid<double, double>(na, pd, grid, T, n3, (double*)D, dstride, (double*)ainv, s);
    return fp64 ? run_det_mid<double, float>(na, pf, grid, T, n3, (double*)D, dstride, (double*)ainv, s)
                : run_det_mid<float, float>(na, pf, grid, T, n3, (float*)D, dstride, (float*)ainv, s);
  }
  if (phi64)
    hipLaunchKernelGGL((det_kernel<double, double>), dim3(grid), dim3(64), 0, s, pd, K, na, T, n3, (double*)D, dstride,
                       (double*)ainv);
  else if (fp64)
    hipLaunchKernelGGL((det_kernel<double, float>), dim3(grid), dim3(64), 0, s, pf, K, na, T, n3, (double*)D, dstride,
                       (double*)ainv);
  else
    hipLaunchKernelGGL((det_kernel<float, float>), dim3(grid), dim3(64), 0, s, pf, K, na, T, n3, (float*)D, dstride,
                       (float*)ainv);
  return hipGetLastError();
}

// ------------------------------------------------------------- combination
template <class R>
__global__ __launch_bounds__(64) void combine_kernel(CombineArgs a) {
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int K = a.K, n3 = a.n3;
  const R* Du = (const R*)a.D[0];
  const R* Dd = (const R*)a.D[1];
  const bool hu = a.na[0] > 0, hd = a.na[1] > 0;
  const int ds = a.dstride;

  // determinant terms: lane k
  R sk = 0, lk = -INFINITY;
  if (lane < K) {
    R su = hu ? Du[(w * K + lane) * ds] : (R)1, sd = hd ? Dd[(w * K + lane) * ds] : (R)1;
    R lu = hu ? Du[(w * K + lane) * ds + 1] : (R)0, ld = hd ? Dd[(w * K + lane) * ds + 1] : (R)0;
    sk = su * sd;
    lk = sk != (R)0 ? lu + ld : (R)-INFINITY;
  }
  const R m = wave_max(lk);
  R ex = (lane < K && sk != (R)0) ? sk * exp(lk - m) : (R)0;
  const R S = wave_sum(ex);
  const bool node = !(m > (R)-INFINITY) || S == (R)0;
  const R logabs = node ? (R)-INFINITY : m + log(fabs(S));
  const R sgn = node ? (R)0 : (S > 0 ? (R)1 : (R)-1);
  const R rho = node ? (R)0 : ex / S;
  if (a.rho && lane < K) ((R*)a.rho)[w * K + lane] = rho;


  // largest condition number over the walker's orbital matrices
  R cmax = 0;
  if (a.jet && lane < K) {
    if (hu) cmax = Du[(w * K + lane) * ds + 4 + n3];
    if (hd) cmax = fmax(cmax, Dd[(w * K + lane) * ds + 4 + n3]);
  }
  if (a.jet) cmax = wave_max(cmax);

  double ekin = 0.0;
  if (a.jet) {
    // sum_k rho_k sum_a (lap_a - q_a)
    R part = 0;
    if (lane < K) {
      R t = 0;
      if (hu) t += Du[(w * K + lane) * ds + 3 + n3] - Du[(w * K + lane) * ds + 2 + n3];
      if (hd) t += Dd[(w * K + lane) * ds + 3 + n3] - Dd[(w * K + lane) * ds + 2 + n3];
      part = rho * t;
    }
    // sum_c sum_k rho_k (d_kc^up + d_kc^down)^2, lanes over coordinates
    __shared__ R s_rho[64];
    s_rho[lane] = rho;
    __syncthreads();
    R sq = 0;
    for (int c = lane; c < n3; c += 64) {
      for (int k = 0; k < K; ++k) {
        R dsum = 0;
        if (hu) dsum += Du[(w * K + k) * ds + 2 + c];
        if (hd) dsum += Dd[(w * K + k) * ds + 2 + c];
        sq += s_rho[k] * dsum * dsum;
      }
    }
    const R lap_over_psi = wave_sum(part) + wave_sum(sq);
    ekin = node ? NAN : -0.5 * (double)lap_over_psi;
  }

  // Coulomb potential of Eq. (2), float64
  double v = 0.0;
  if (a.jet || a.e_pot) {
    const float* x = a.pos + w * (int64_t)a.n * 3;
    const int n = a.n, N = a.N;
    const int npair = n * (n - 1) / 2;
    for (int p = lane; p < npair; p += 64) {
      // p -> (i, j), i < j
      int i = 0, rem = p;
      while (rem >= n - 1 - i) {
        rem -= n - 1 - i;
        ++i;
      }
      const int j = i + 1 + rem;
      double dx = (double)x[3 * i] - x[3 * j], dy = (double)x[3 * i + 1] - x[3 * j + 1],
             dz = (double)x[3 * i + 2] - x[3 * j + 2];
      v += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    }
    for (int p = lane; p < n * N; p += 64) {
      const int i = p / N, I = p % N;
      double dx = (double)x[3 * i] - a.nuc[3 * I], dy = (double)x[3 * i + 1] - a.nuc[3 * I + 1],
             dz = (double)x[3 * i + 2] - a.nuc[3 * I + 2];
      v -= (double)a.Z[I] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    for (int p = lane; p < N * N; p += 64) {
      const int I = p / N, J = p % N;
      if (I < J) {
        double dx = (double)a.nuc[3 * I] - a.nuc[3 * J], dy = (double)a.nuc[3 * I + 1] - a.nuc[3 * J + 1],
               dz = (double)a.nuc[3 * I + 2] - a.nuc[3 * J + 2];
        v += (double)a.Z[I] * a.Z[J] / sqrt(dx * dx + dy * dy + dz * dz);
      }
    }
    v = wave_sum(v);
  }
  if (lane == 0) {
    // rescue key: the log of the scale of the walker's rounding error in E_L,
    //   kappa max(1, |E_L|, |E_kin|) (1 + (u_det / u_orb) cond),
    // kappa = max_k |P_k| / |psi| (determinant-sum cancellation), E_kin the
    // only term computed through the network, cond the largest condition
    // number of its orbital matrices, weighted by the ratio of the unit
    // roundoff of the determinant arithmetic to that of the orbitals
    if (a.rescue_key) {
      const double el = fmax(1.0, fmax(fabs(ekin + v), fabs(ekin)));
      a.rescue_key[w] =
          node ? INFINITY : (float)((double)(m - logabs) + log(el) + log1p((double)a.cond_weight * (double)cmax));
    }
    a.sign[w] = (float)sgn;
    a.logpsi[w] = (float)logabs;
    if (a.jet) {
      a.e_loc[w] = (float)(ekin + v);
      if (a.e_kin) a.e_kin[w] = (float)ekin;
      if (a.e_pot) a.e_pot[w] = (float)v;
    }
  }
}

hipError_t launch_combine(bool fp64, const CombineArgs& a, hipStream_t s) {
  if (a.W <= 0) return hipSuccess;
  if (a.K > 64) return hipErrorInvalidValue;
  if (fp64) hipLaunchKernelGGL(combine_kernel<double>, dim3(a.W), dim3(64), 0, s, a);
  else hipLaunchKernelGGL(combine_kernel<float>, dim3(a.W), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace fn
