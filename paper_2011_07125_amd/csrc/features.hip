// Input features, the two-electron stream and the mean fields.
//
// Jets: every activation of an electron is carried as T = 3n+2 rows: the
// value, its derivatives with respect to each of the 3n electron
// coordinates (row 1 + 3j + c for coordinate c of electron j) and its
// Laplacian over all 3n coordinates (row T-1).  Rows T..Tp-1 are zero
// padding.  In value mode T = Tp = 1.
//
// Two-electron activations h_ij depend on r_i and r_j only, so their jets
// are carried sparsely as 8 rows (value, d/dr_i, d/dr_j, Laplacian) and
// never leave the chip: one workgroup runs all two-electron layers of its
// electrons in registers and LDS and writes only the dense jets of the
// spin-resolved means g^a_i that the one-electron layers consume.
#include "common.h"
#include "kernels.h"

namespace fn {

// ------------------------------------------------------------ weight packing
struct PackPlan {
  int n_items;
  // dst_off, N, ldb, k0, len0, src0, k1, len1, src1, src_ld, transpose
  int64_t it[32][11];
};

// packed[n][k] = params[src + (k - k0) * src_ld + n] (transpose) or
// params[src + n * src_ld + (k - k0)] for k in one of the two
// segments, 0 elsewhere; float32, split into bfloat16 hi and lo planes, or
// float64
template <int PMODE>
__global__ void pack_weights_kernel(const float* params, void* dst, int64_t plane, PackPlan plan) {
  const int item = blockIdx.y;
  if (item >= plan.n_items) return;
  const int64_t* p = plan.it[item];
  const int64_t N = p[1], ldb = p[2], total = N * ldb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t n = idx / ldb, k = idx % ldb;
    float v = 0.0f;
    if (k >= p[3] && k < p[3] + p[4]) v = params[p[5] + (p[10] ? (k - p[3]) * p[9] + n : n * p[9] + (k - p[3]))];
    else if (k >= p[6] && k < p[6] + p[7]) v = params[p[8] + (p[10] ? (k - p[6]) * p[9] + n : n * p[9] + (k - p[6]))];
    if constexpr (PMODE == MODE_BF16X3) {
      uint16_t* d = reinterpret_cast<uint16_t*>(dst);
      const uint16_t h = f32_to_bf16_bits(v);
      d[p[0] + idx] = h;
      d[plane + p[0] + idx] = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
    } else if constexpr (PMODE == MODE_F64) {
      reinterpret_cast<double*>(dst)[p[0] + idx] = (double)v;
    } else {
      reinterpret_cast<float*>(dst)[p[0] + idx] = v;
    }
  }
}

hipError_t launch_pack_weights(int mode, const float* params, void* dst, int64_t plane, const int64_t* plan,
                               int n_items, hipStream_t s) {
  if (n_items > 32) return hipErrorInvalidValue;
  PackPlan pp;
  pp.n_items = n_items;
  for (int i = 0; i < n_items; ++i)
    for (int j = 0; j < 11; ++j) pp.it[i][j] = plan[i * 11 + j];
  dim3 grid(64, n_items);
  if (mode == MODE_BF16X3) hipLaunchKernelGGL(pack_weights_kernel<MODE_BF16X3>, grid, dim3(256), 0, s, params, dst, plane, pp);
  else if (mode == MODE_F64) hipLaunchKernelGGL(pack_weights_kernel<MODE_F64>, grid, dim3(256), 0, s, params, dst, plane, pp);
  else hipLaunchKernelGGL(pack_weights_kernel<MODE_F32>, grid, dim3(256), 0, s, params, dst, plane, pp);
  return hipGetLastError();
}

// ------------------------------------------------------- one-electron input
// H0[(g Tp + t) ldh + f], g = w n + i: the jets of
//   h_i = concat_I (r_i - R_I, |r_i - R_I|)
// d/dr_i of (r_i - R_I)_c = e_c; of |r_i - R_I| = (r_i - R_I)/|r_i - R_I|;
// Laplacian of |r_i - R_I| = 2 / |r_i - R_I|.  S: float or double
// (arithmetic and storage).  Also the spin means the first layer's mean
// field reads, Hbar[(w Tp + t)][a ldh + f] = mean_{j of spin a} H0[...]:
// the sums take j in order from zero and are scaled as the separate
// mean-field pass scales them (by 1/n_a in float32, divided by n_a in
// float64), so they are the means of the stored values.
//
// Item k of walker w is jet row t = k / nv and nucleus I = k % nv (nv =
// ldh / 4): its four features for every electron of the walker in turn,
// stored as one vector each.  A block handles several walkers when one
// walker has fewer items than threads (the value pass has one row).
template <class S>
__global__ __launch_bounds__(256) void features_kernel(const float* pos, const float* nuc, int W, int n, int n_up,
                                                       int N, int T, int Tp, S* H0, int ldh, S* Hbar,
                                                       float* h0_val, float* hbar_val) {
  const int nv = ldh / 4, items = Tp * nv;
  const int wpb = items >= (int)blockDim.x ? 1 : (int)blockDim.x / items;  // walkers per block step
  for (int w0 = blockIdx.x * wpb; w0 < W; w0 += gridDim.x * wpb) {
    for (int q = threadIdx.x; q < wpb * items; q += blockDim.x) {
      const int e = q / items, k = q - e * items;
      const int w = w0 + e;
      if (w >= W) break;  // e grows with q
      const int t = k / nv, I = k - t * nv;
      S su[4] = {0, 0, 0, 0}, sd[4] = {0, 0, 0, 0};
      for (int j = 0; j < n; ++j) {
        const int64_t g = (int64_t)w * n + j;
        S v[4] = {0, 0, 0, 0};
        if (I < N && t < T) {
          const float* r = pos + g * 3;
          const S d0 = (S)r[0] - (S)nuc[3 * I], d1 = (S)r[1] - (S)nuc[3 * I + 1], d2 = (S)r[2] - (S)nuc[3 * I + 2];
          const S dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
          const S dc[3] = {d0, d1, d2};
          if (t == 0) {
            v[0] = d0;
            v[1] = d1;
            v[2] = d2;
            v[3] = dist;
          } else if (t == T - 1) {
            v[3] = (S)2 / dist;
          } else {
            const int jt = (t - 1) / 3, c = (t - 1) - 3 * jt;
            if (jt == j) {
              v[c] = (S)1;
              v[3] = dc[c] / dist;
            }
          }
        }
        S* dst = H0 + (g * Tp + t) * ldh + 4 * I;
        if (h0_val && t == 0)
          *reinterpret_cast<float4*>(h0_val + g * ldh + 4 * I) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        if constexpr (sizeof(S) == 4) {
          *reinterpret_cast<float4*>(dst) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        } else {
          reinterpret_cast<double2*>(dst)[0] = double2{(double)v[0], (double)v[1]};
          reinterpret_cast<double2*>(dst)[1] = double2{(double)v[2], (double)v[3]};
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (j < n_up) su[c] += v[c];
          else sd[c] += v[c];
        }
      }
      S mu[4], md[4];
      const int nd = n - n_up;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (sizeof(S) == 4) {
          mu[c] = su[c] * (n_up > 0 ? 1.0f / (float)n_up : 0.0f);
          md[c] = sd[c] * (nd > 0 ? 1.0f / (float)nd : 0.0f);
        } else {
          mu[c] = n_up > 0 ? su[c] / (S)n_up : (S)0;
          md[c] = nd > 0 ? sd[c] / (S)nd : (S)0;
        }
      }
      S* hb = Hbar + ((int64_t)w * Tp + t) * 2 * ldh + 4 * I;
      if (hbar_val && t == 0) {
        float* o = hbar_val + (int64_t)w * 2 * ldh + 4 * I;
        *reinterpret_cast<float4*>(o) = float4{(float)mu[0], (float)mu[1], (float)mu[2], (float)mu[3]};
        *reinterpret_cast<float4*>(o + ldh) = float4{(float)md[0], (float)md[1], (float)md[2], (float)md[3]};
      }
      if constexpr (sizeof(S) == 4) {
        *reinterpret_cast<float4*>(hb) = float4{mu[0], mu[1], mu[2], mu[3]};
        *reinterpret_cast<float4*>(hb + ldh) = float4{md[0], md[1], md[2], md[3]};
      } else {
        reinterpret_cast<double2*>(hb)[0] = double2{mu[0], mu[1]};
        reinterpret_cast<double2*>(hb)[1] = double2{mu[2], mu[3]};
        reinterpret_cast<double2*>(hb + ldh)[0] = double2{md[0], md[1]};
        reinterpret_cast<double2*>(hb + ldh)[1] = double2{md[2], md[3]};
      }
    }
  }
}

hipError_t launch_features(bool f64, const float* pos, const float* nuc, int W, int n, int n_up, int N, int T, int Tp,
                           void* H0, int ldh, void* Hbar, hipStream_t s, float* h0_val, float* hbar_val) {
  if ((int64_t)W * n <= 0) return hipSuccess;
  // rows of 16-byte-aligned vectors (buffers are 256-byte aligned)
  if ((int64_t)W * n >= (1LL << 31) || ldh % 4 != 0 || ldh < 4 * N || n_up < 0 || n_up > n)
    return hipErrorInvalidValue;
  const int items = Tp * (ldh / 4), wpb = items >= 256 ? 1 : 256 / items;
  const int grid = (int)std::min<int64_t>((W + wpb - 1) / wpb, 16384);
  if (f64)
    hipLaunchKernelGGL(features_kernel<double>, dim3(grid), dim3(256), 0, s, pos, nuc, W, n, n_up, N, T, Tp,
                       (double*)H0, ldh, (double*)Hbar, h0_val, hbar_val);
  else
    hipLaunchKernelGGL(features_kernel<float>, dim3(grid), dim3(256), 0, s, pos, nuc, W, n, n_up, N, T, Tp,
                       (float*)H0, ldh, (float*)Hbar, h0_val, hbar_val);
  return hipGetLastError();
}

// ------------------------------------------------------ two-electron stream
struct TwoElecDev {
  const float* pos;
  const float* params;
  int64_t w_off[8], c_off[8];
  int W, n, n_up, L, d2, T, Tp, R2, ipb;
  void* G[8];
  int ldg[8];
  float* h2_out[8];
  float* g_val_out[8];
};

// slot s of the block: electron ii = s / (n R2), partner j = (s / R2) % n,
// sparse jet row q = s % R2 (value, d/dr_i x3, d/dr_j x3, Laplacian).
// D2 is the two-electron width rounded up to a compiled size; the extra
// features carry zero weights and stay zero.  The slot rows of Ps have the
// odd stride D2 + 1, so the 64 slots of a wavefront reading one feature hit
// distinct LDS banks.
template <int D2> constexpr int two_e_ps_stride() { return D2 + 1; }
// LDS rows of the slots, padded to whole 16-row matrix tiles
__host__ __device__ inline int two_e_rows(int slots) { return (slots + 15) / 16 * 16; }
inline size_t two_e_ws_offset(int slots, int ps) { return ((size_t)two_e_rows(slots) * ps + 3) / 4 * 4; }
// shared rows of a g jet (value, d/dr_i x3, Laplacian in jet mode; the value
// in value mode) and the LDS elements of their partner sums
__host__ __device__ inline int two_e_shared_rows(int R2) { return R2 == 8 ? 5 : 1; }
inline size_t two_e_sums_elems(int ipb, int R2, int D2) { return (size_t)ipb * two_e_shared_rows(R2) * 2 * D2; }

// S: float or double (arithmetic, LDS and the stored jets of g^a_i)
template <class S, int D2>
__global__ __launch_bounds__(256) void two_electron_kernel(TwoElecDev a) {
  extern __shared__ __attribute__((aligned(16))) char sh_raw[];
  S* sh = reinterpret_cast<S*>(sh_raw);
  constexpr int PS = two_e_ps_stride<D2>();
  const int n = a.n, R2 = a.R2, d2 = a.d2;
  S* Ps = sh;                                                          // [rows][PS]
  S* Ws = sh + ((size_t)two_e_rows(a.ipb * n * R2) * PS + 3) / 4 * 4;  // [D2][D2] then c[D2], 16-byte aligned
  S* Ss = Ws + D2 * D2 + D2;  // [ipb][shared rows][2 ein]: partner sums of the shared g rows
  const int tid = threadIdx.x;
  const int slots = a.ipb * n * R2;
  // electrons of the block: gbase .. gbase + ipb - 1 (W n < 2^31), the
  // first being electron i0 of walker w0
  const int gbase = blockIdx.x * a.ipb;
  const int n_groups = a.W * n;
  const int w0 = gbase / n, i0 = gbase - w0 * n;

  // slot s: electron ii of the block, partner j, sparse jet row q (R2 is 8
  // in jet mode, 1 in value mode)
  const int s = tid;
  const int q = R2 == 8 ? (s & 7) : 0, pr = R2 == 8 ? (s >> 3) : s;
  const int ii = pr / n, j = pr - ii * n;
  const bool live = s < slots && gbase + ii < n_groups;
  const int iw = (i0 + ii) / n;  // walkers past w0
  const int i = i0 + ii - iw * n;
  const int64_t w = (int64_t)w0 + iw;

  // input pair features (r_i - r_j, |r_i - r_j|) and their sparse jets;
  // rows of no live slot are zero
  if (!live && s < two_e_rows(slots)) {
#pragma unroll
    for (int k = 0; k < D2; ++k) Ps[(size_t)s * PS + k] = (S)0;
  }
  if (live) {
    S in[4] = {0, 0, 0, 0};
    if (i != j) {
      const float* ri = a.pos + (w * n + i) * 3;
      const float* rj = a.pos + (w * n + j) * 3;
      const S dd[3] = {(S)ri[0] - (S)rj[0], (S)ri[1] - (S)rj[1], (S)ri[2] - (S)rj[2]};
      const S dist = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      if (q == 0) {
        in[0] = dd[0]; in[1] = dd[1]; in[2] = dd[2]; in[3] = dist;
      } else if (q <= 6) {
        const int c = (q - 1) % 3;
        const S sgn = q <= 3 ? (S)1 : (S)-1;  // d/dr_i or d/dr_j
        in[0] = c == 0 ? sgn : (S)0;
        in[1] = c == 1 ? sgn : (S)0;
        in[2] = c == 2 ? sgn : (S)0;
        in[3] = sgn * dd[c] / dist;
      } else {
        in[3] = (S)4 / dist;  // Laplacian over r_i and r_j of |r_i - r_j|
      }
    }
#pragma unroll
    for (int k = 0; k < D2; ++k) Ps[(size_t)s * PS + k] = k < 4 ? in[k] : (S)0;
  }

  int ein = 4;
  const int n_up = a.n_up, n_dn = n - a.n_up;
  for (int l = 0; l < a.L; ++l) {
    __syncthreads();
    // dense jets of g^a_i = mean_{j in a} h_ij from the pair activations in
    // LDS.  Row t of the jet is a shared row (the value, d/dr_i, the
    // Laplacian: sums over the partners of spin a) or the d/dr_j row of one
    // partner j (that pair's row alone, zero in the other spin's columns).
    {
      S* G = reinterpret_cast<S*>(a.G[l]);
      const int ldg = a.ldg[l];
      float* const gv = a.g_val_out[l];  // row 0 of the jets, compactly (optional)
      const int T = a.T, Tp = a.Tp;
      const int nq = two_e_shared_rows(R2), ncol = 2 * ein;
      const S inv_up = n_up > 0 ? (S)1 / (S)n_up : (S)0, inv_dn = n_dn > 0 ? (S)1 / (S)n_dn : (S)0;
      // phase 1: partner sums, one (electron, shared row, column) per item,
      // four partners per step (independent LDS reads in flight).  The item
      // (eq = e nq + qq, c) advances by the block size with a carry: no
      // division inside the loop.
      {
        int c = tid % ncol, eq = tid / ncol;
        const int dc = blockDim.x % ncol, deq = blockDim.x / ncol;
        while (eq < a.ipb * nq) {
          const int e = nq == 1 ? eq : (eq * 52429) >> 18;  // eq / 5, exact for eq < 2^14
          const int qq = eq - e * nq;
          const int al = c >= ein, o = c - al * ein;
          const int j0 = al == 0 ? 0 : n_up, na = al == 0 ? n_up : n_dn;
          const int qs = qq == 4 ? 7 : qq;  // sparse jet row: value, d/dr_i x3, Laplacian
          const S* base = Ps + ((size_t)(e * n + j0) * R2 + qs) * PS + o;
          const size_t step = (size_t)R2 * PS;
          S s0 = 0, s1 = 0, s2 = 0, s3 = 0;
          int jj = 0;
          for (; jj + 3 < na; jj += 4) {
            s0 += base[jj * step];
            s1 += base[(jj + 1) * step];
            s2 += base[(jj + 2) * step];
            s3 += base[(jj + 3) * step];
          }
          for (; jj < na; ++jj) s0 += base[jj * step];
          Ss[(size_t)eq * ncol + c] = ((s0 + s1) + (s2 + s3)) * (al == 0 ? inv_up : inv_dn);
          c += dc;
          eq += deq;
          if (c >= ncol) {
            c -= ncol;
            ++eq;
          }
        }
      }
      __syncthreads();
      // phase 2: four columns of one (electron e, jet row t) per item, one
      // 16-byte store (ldg is a multiple of 32).
      const int nc4 = ldg / 4;
      if (ein % 4 == 0 && blockDim.x % nc4 == 0 && Tp % (blockDim.x / nc4) == 0) {
        // every thread keeps one column quad c0 (in one spin half: ncol =
        // 2 ein) and the jet rows t = tid / nc4 + k blockDim / nc4 of every
        // electron of the block, so that everything but the electron is
        // worked out once per row (the jet passes: the same items as below,
        // in another order)
        const int c0 = (tid % nc4) * 4, rstep = blockDim.x / nc4;
        const int al = c0 >= ein ? 1 : 0;
        const bool colv = c0 < ncol;
        const S sc = al == 0 ? inv_up : inv_dn;
        const int e_end = min(a.ipb, n_groups - gbase);
        for (int t = tid / nc4; t < Tp; t += rstep) {
          const bool live = t < T && colv;
          const int jt = t >= 1 ? ((t - 1) * 43691) >> 17 : -1;  // (t - 1) / 3, exact for t < 2^16
          const int cc = t - 1 - 3 * jt;
          const bool row_shared = t == 0 || t == T - 1;
          const int qq = t == 0 ? 0 : t == T - 1 ? 4 : 1 + cc;
          // partner row of jt: only the quads of jt's spin half are nonzero
          const bool own_half = (al == 0) == (jt < n_up);
          const S* ssrc = Ss + (size_t)qq * ncol + c0;
          const int jp = jt < 0 ? 0 : jt < n ? jt : n - 1;  // the address of a row that reads it
          const S* psrc = Ps + ((size_t)jp * R2 + 4 + cc) * PS + (c0 - al * ein);
          S* dst = G + ((int64_t)gbase * Tp + t) * ldg + c0;
          int ie = i0;
          for (int e = 0; e < e_end; ++e) {
            S v[4] = {0, 0, 0, 0};
            if (live) {
              if (row_shared || jt == ie) {
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = ssrc[(size_t)e * nq * ncol + k];
              } else if (own_half) {
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = psrc[(size_t)e * n * R2 * PS + k] * sc;
              }
            }
            S* d = dst + (int64_t)e * Tp * ldg;
            if (gv && t == 0)
              *reinterpret_cast<float4*>(gv + (int64_t)(gbase + e) * ldg + c0) =
                  float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            if constexpr (sizeof(S) == 4) {
              *reinterpret_cast<float4*>(d) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            } else {
              reinterpret_cast<double2*>(d)[0] = double2{(double)v[0], (double)v[1]};
              reinterpret_cast<double2*>(d)[1] = double2{(double)v[2], (double)v[3]};
            }
            ie = ie + 1 == n ? 0 : ie + 1;
          }
        }
      } else {
        // general case: (e, t, c4) and the electron's index ie within its
        // walker advance with carries
        int c4 = tid % nc4, row = tid / nc4;
        const int dc4 = blockDim.x % nc4, drow = blockDim.x / nc4;
        int e = row / Tp, t = row - e * Tp;
        int ie = (i0 + e) % n;
        while (e < a.ipb) {
          const int c0 = c4 * 4;
          if (gbase + e < n_groups) {
            S v[4] = {0, 0, 0, 0};
            if (t < T && c0 < ncol) {
              const int jt = t >= 1 ? ((t - 1) * 43691) >> 17 : -1;  // (t - 1) / 3, exact for t < 2^16
              const int cc = t - 1 - 3 * jt;
              const bool shared = t == 0 || t == T - 1 || jt == ie;
              const int qq = t == 0 ? 0 : t == T - 1 ? 4 : 1 + cc;
              const bool jt_up = jt < n_up;
              if (ein % 4 == 0) {
                // the four columns lie in one spin half (ncol = 2 ein)
                const int al = c0 >= ein;
                if (shared) {
                  const S* src = Ss + (size_t)(e * nq + qq) * ncol + c0;
#pragma unroll
                  for (int k = 0; k < 4; ++k) v[k] = src[k];
                } else if ((al == 0) == jt_up) {
                  const S* src = Ps + ((size_t)(e * n + jt) * R2 + 4 + cc) * PS + (c0 - al * ein);
                  const S sc = al == 0 ? inv_up : inv_dn;
#pragma unroll
                  for (int k = 0; k < 4; ++k) v[k] = src[k] * sc;
                }
              } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  const int c = c0 + k;
                  if (c >= ncol) continue;
                  const int al = c >= ein;
                  if (shared) v[k] = Ss[(size_t)(e * nq + qq) * ncol + c];
                  else if ((al == 0) == jt_up)
                    v[k] = Ps[((size_t)(e * n + jt) * R2 + 4 + cc) * PS + (c - al * ein)] * (al == 0 ? inv_up : inv_dn);
                }
              }
            }
            S* dst = G + ((int64_t)(gbase + e) * Tp + t) * ldg + c0;
            if (gv && t == 0)
              *reinterpret_cast<float4*>(gv + (int64_t)(gbase + e) * ldg + c0) =
                  float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            if constexpr (sizeof(S) == 4) {
              *reinterpret_cast<float4*>(dst) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            } else {
              reinterpret_cast<double2*>(dst)[0] = double2{(double)v[0], (double)v[1]};
              reinterpret_cast<double2*>(dst)[1] = double2{(double)v[2], (double)v[3]};
            }
          }
          c4 += dc4;
          int adv = drow;
          if (c4 >= nc4) {
            c4 -= nc4;
            ++adv;
          }
          t += adv;
          while (t >= Tp) {
            t -= Tp;
            ++e;
            ie = ie + 1 == n ? 0 : ie + 1;
          }
        }
      }
      if (a.h2_out[l]) {
        // the values of the block's pair activations are one contiguous run
        // of the output ([electron][partner][ein] with pair = e n +
        // partner; in jet mode the value is the pair's sparse row 0); pair
        // and feature by shifts when ein is a power of two
        const int nval = (min(a.ipb, n_groups - gbase)) * n * ein;
        float* dst = a.h2_out[l] + (int64_t)gbase * n * ein;
        const bool pow2 = (ein & (ein - 1)) == 0;
        const int sh = __builtin_ctz(ein);
        for (int idx = tid; idx < nval; idx += blockDim.x) {
          const int pr = pow2 ? idx >> sh : idx / ein, o = idx - pr * ein;
          dst[idx] = (float)Ps[(size_t)pr * R2 * PS + o];
        }
      }
    }
    if (l + 1 == a.L) break;
    // two-electron layer l: h' = tanh(h W_l + c_l) (+ h when widths match)
    for (int k = tid; k < D2 * D2 + D2; k += blockDim.x) {
      S v = 0;
      if (k < D2 * D2) {
        const int kr = k / D2, o = k % D2;
        if (kr < ein && o < d2) v = (S)a.params[a.w_off[l] + kr * d2 + o];
      } else if (k - D2 * D2 < d2) {
        v = (S)a.params[a.c_off[l] + (k - D2 * D2)];
      }
      Ws[k] = v;
    }
    __syncthreads();
    if constexpr (sizeof(S) == 4 && D2 >= 16) {
      // float32: the layer product [rows x ein] x [ein x D2] on MFMA.  Each
      // wave owns whole 16-row tiles (two pairs x 8 sparse jet rows, or 16
      // value rows) and updates them in place after its own reads.  In the
      // accumulator layout item r of lane (kq, c) is row 4 kq + r: jet row
      // q = 4 (kq & 1) + r of pair kq >> 1, column c.
      const int lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
      const int n_rt = two_e_rows(slots) / 16;
      const bool res = ein == d2;
      const S* cb = Ws + D2 * D2;
      for (int tm = wave; tm < n_rt; tm += 4) {
        floatx4 acc[D2 / 16];
#pragma unroll
        for (int tn = 0; tn < D2 / 16; ++tn) acc[tn] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < ein; ks += 4) {
          const float av = Ps[(size_t)(tm * 16 + lr) * PS + ks + lk];
#pragma unroll
          for (int tn = 0; tn < D2 / 16; ++tn)
            acc[tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Ws[(ks + lk) * D2 + tn * 16 + lr], acc[tn], 0, 0, 0);
        }
#pragma unroll
        for (int tn = 0; tn < D2 / 16; ++tn) {
          const int col = tn * 16 + lr;
          float o4[4];
          if (R2 == 8) {
            const float u0 = __shfl(acc[tn][0], lane & ~16, 64) + cb[col];
            float sq = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int q = 4 * (lk & 1) + r;
              if (q >= 1 && q <= 6) sq += acc[tn][r] * acc[tn][r];
            }
            const float s2 = sq + __shfl_xor(sq, 16, 64);
            float y, dy;
            tanh_sech2(u0, &y, &dy);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int q = 4 * (lk & 1) + r;
              o4[r] = q == 0 ? y : q <= 6 ? dy * acc[tn][r] : dy * acc[tn][r] - 2.0f * y * dy * s2;
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              float y, dy;
              tanh_sech2(acc[tn][r] + cb[col], &y, &dy);
              o4[r] = y;
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t e = (size_t)(tm * 16 + 4 * lk + r) * PS + col;
            float v = o4[r];
            if (res) v += Ps[e];
            Ps[e] = col < d2 ? v : 0.0f;
          }
        }
      }
      ein = d2;
    } else if constexpr (sizeof(S) == 8 && D2 >= 16) {
      // float64: the same product on v_mfma_f64_16x16x4f64, whose item r of
      // lane (kq, c) is row kq + 4 r: jet row q = kq + 4 (r & 1) of pair
      // r >> 1 (the value row of pair p is item 2 p of lane group 0)
      const int lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
      const int n_rt = two_e_rows(slots) / 16;
      const bool res = ein == d2;
      const S* cb = Ws + D2 * D2;
      for (int tm = wave; tm < n_rt; tm += 4) {
        doublex4 acc[D2 / 16];
#pragma unroll
        for (int tn = 0; tn < D2 / 16; ++tn) acc[tn] = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int ks = 0; ks < ein; ks += 4) {
          const double av = Ps[(size_t)(tm * 16 + lr) * PS + ks + lk];
#pragma unroll
          for (int tn = 0; tn < D2 / 16; ++tn)
            acc[tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ws[(ks + lk) * D2 + tn * 16 + lr], acc[tn], 0, 0, 0);
        }
#pragma unroll
        for (int tn = 0; tn < D2 / 16; ++tn) {
          const int col = tn * 16 + lr;
          double o4[4];
          if (R2 == 8) {
#pragma unroll
            for (int pp = 0; pp < 2; ++pp) {
              const double u0 = __shfl(acc[tn][2 * pp], lr, 64) + cb[col];
              double sq = 0.0;
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int q = lk + 4 * h;
                if (q >= 1 && q <= 6) sq += acc[tn][2 * pp + h] * acc[tn][2 * pp + h];
              }
              sq += __shfl_xor(sq, 16, 64);
              sq += __shfl_xor(sq, 32, 64);
              double y, dy;
              tanh_sech2(u0, &y, &dy);
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int q = lk + 4 * h, r = 2 * pp + h;
                o4[r] = q == 0 ? y : q <= 6 ? dy * acc[tn][r] : dy * acc[tn][r] - 2.0 * y * dy * sq;
              }
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double y, dy;
              tanh_sech2(acc[tn][r] + cb[col], &y, &dy);
              o4[r] = y;
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t e = (size_t)(tm * 16 + lk + 4 * r) * PS + col;
            double v = o4[r];
            if (res) v += Ps[e];
            Ps[e] = col < d2 ? v : 0.0;
          }
        }
      }
      ein = d2;
    } else {
      S u[D2];
#pragma unroll
      for (int o = 0; o < D2; ++o) u[o] = q == 0 ? Ws[D2 * D2 + o] : (S)0;
      if (live) {
        for (int k = 0; k < ein; ++k) {
          const S x = Ps[(size_t)s * PS + k];
          if constexpr (sizeof(S) == 4) {
            const float4* wr = reinterpret_cast<const float4*>(Ws + k * D2);
#pragma unroll
            for (int o4 = 0; o4 < D2 / 4; ++o4) {
              const float4 wv = wr[o4];
              u[4 * o4] += x * wv.x;
              u[4 * o4 + 1] += x * wv.y;
              u[4 * o4 + 2] += x * wv.z;
              u[4 * o4 + 3] += x * wv.w;
            }
          } else {
            const S* wr = Ws + k * D2;
#pragma unroll
            for (int o = 0; o < D2; ++o) u[o] += x * wr[o];
          }
        }
      }
      const bool res = ein == d2;
      // the tanh chain rule of one output column: y = tanh u0 and
      // dy = sech^2 u0 of the value row, s2 the sum of the squared tangents
      auto chain = [&](int o, S y, S dy, S s2) {
        const S uo = u[o];
        S outv;
        if (q == 0) outv = y;
        else if (q <= 6) outv = dy * uo;
        else outv = dy * uo - (S)2 * y * dy * s2;
        if (res && live) outv += Ps[(size_t)s * PS + o];
        u[o] = o < d2 ? outv : (S)0;
      };
      if constexpr (D2 % 8 == 0) {
        if (R2 == 8) {
          // jet rows: the eight lanes of a pair share u0 per column, so
          // lane q evaluates the activation of column ob + q once and the
          // pair exchanges the results by shuffles
          const int pb = tid & ~7;
#pragma unroll
          for (int ob = 0; ob < D2; ob += 8) {
            S u0q = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const S v = __shfl(u[ob + j], pb, 64);
              if (q == j) u0q = v;
            }
            S yq, dyq;
            tanh_sech2(u0q, &yq, &dyq);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int o = ob + j;
              const S uo = u[o];
              S sq = (q >= 1 && q <= 6) ? uo * uo : (S)0;
              sq += __shfl_xor(sq, 1, 64);
              sq += __shfl_xor(sq, 2, 64);
              sq += __shfl_xor(sq, 4, 64);
              chain(o, __shfl(yq, pb + j, 64), __shfl(dyq, pb + j, 64), sq);
            }
          }
        }
      }
      if (D2 % 8 != 0 || R2 != 8) {
#pragma unroll
        for (int o = 0; o < D2; ++o) {
          const S uo = u[o];
          S y, dy, s2 = 0;
          if (R2 == 8) {
            const S u0 = __shfl(uo, tid & ~7, 64);
            S sq = (q >= 1 && q <= 6) ? uo * uo : (S)0;
            sq += __shfl_xor(sq, 1, 64);
            sq += __shfl_xor(sq, 2, 64);
            sq += __shfl_xor(sq, 4, 64);
            s2 = sq;
            tanh_sech2(u0, &y, &dy);
          } else {
            tanh_sech2(uo, &y, &dy);
          }
          chain(o, y, dy, s2);
        }
      }
      ein = d2;
      __syncthreads();
      if (live) {
#pragma unroll
        for (int o = 0; o < D2; ++o) Ps[(size_t)s * PS + o] = u[o];
      }
    }
  }
}

template <class S, int D2>
static hipError_t run_two_e(const TwoElecDev& d, int grid, hipStream_t s) {
  const size_t shmem = (two_e_ws_offset(d.ipb * d.n * d.R2, two_e_ps_stride<D2>()) + (size_t)D2 * D2 + D2 +
                        two_e_sums_elems(d.ipb, d.R2, D2)) *
                       sizeof(S);
  if (shmem > 65536) {
    // once per instantiation (a local static is initialised once, thread-safely)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&two_electron_kernel<S, D2>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((two_electron_kernel<S, D2>), dim3(grid), dim3(256), shmem, s, d);
  return hipGetLastError();
}

template <class S>
static hipError_t pick_two_e(const TwoElecDev& d, int grid, hipStream_t s) {
  if (d.d2 <= 4) return run_two_e<S, 4>(d, grid, s);
  if (d.d2 <= 8) return run_two_e<S, 8>(d, grid, s);
  if (d.d2 <= 16) return run_two_e<S, 16>(d, grid, s);
  if (d.d2 <= 32) return run_two_e<S, 32>(d, grid, s);
  return run_two_e<S, 64>(d, grid, s);
}

// electrons per block of the two-electron stream: at most 256 slots and at
// most 64 KiB of LDS, or one electron in up to 160 KiB (the LDS of a CU)
// when one does not fit in 64 KiB; 0 if it does not fit at all
int two_electron_per_block(int n, int d2, int T, int scalar_bytes) {
  const int R2 = T > 1 ? 8 : 1;
  const int D2p = d2 <= 4 ? 4 : d2 <= 8 ? 8 : d2 <= 16 ? 16 : d2 <= 32 ? 32 : 64;
  auto elems = [&](int ipb) {
    return (int)(two_e_rows(ipb * n * R2) * (D2p + 1) + 4 + D2p * D2p + D2p + two_e_sums_elems(ipb, R2, D2p));
  };
  int ipb = 256 / (n * R2);
  // value passes: at most 160 slots, so more and smaller workgroups share
  // the compute units (the Ne-like value pass: 25 -> 16 electrons per
  // workgroup, 0.122 -> 0.098 ms)
  if (R2 == 1) ipb = std::min(ipb, std::max(1, 160 / n));
  while (ipb > 1 && elems(ipb) * scalar_bytes > 65536) --ipb;
  if (ipb >= 1 && elems(ipb) * scalar_bytes <= 65536) return ipb;
  return (ipb >= 1 && elems(1) * scalar_bytes <= 160 * 1024) ? 1 : 0;
}

hipError_t launch_two_electron(bool f64, const TwoElecArgs& a, hipStream_t s) {
  TwoElecDev d;
  d.pos = a.pos;
  d.params = a.params;
  for (int l = 0; l < 8; ++l) {
    d.w_off[l] = l + 1 < a.L ? a.w_off[l] : 0;
    d.c_off[l] = l + 1 < a.L ? a.c_off[l] : 0;
    d.G[l] = l < a.L ? a.G[l] : nullptr;
    d.ldg[l] = l < a.L ? a.ldg[l] : 0;
    d.h2_out[l] = l < a.L ? a.h2_out[l] : nullptr;
    d.g_val_out[l] = l < a.L ? a.g_val_out[l] : nullptr;
  }
  d.W = a.W; d.n = a.n; d.n_up = a.n_up; d.L = a.L; d.d2 = a.d2; d.T = a.T; d.Tp = a.Tp;
  d.R2 = a.T > 1 ? 8 : 1;
  if (a.d2 > 64 || a.n * d.R2 > 256 || a.L > 8 || (int64_t)a.W * a.n >= (1LL << 31)) return hipErrorInvalidValue;
  d.ipb = two_electron_per_block(a.n, a.d2, a.T, f64 ? 8 : 4);
  if (d.ipb < 1) return hipErrorInvalidValue;
  const int64_t groups = (int64_t)a.W * a.n;
  const int grid = (int)((groups + d.ipb - 1) / d.ipb);
  if (grid <= 0) return hipSuccess;
  return f64 ? pick_two_e<double>(d, grid, s) : pick_two_e<float>(d, grid, s);
}

// ------------------------------------------------------------ mean fields
// Hbar[(w Tp + t)][a din_p + f] = mean_{j of spin a} H[((w n + j) Tp + t)][f]
template <class S>
__global__ void meanfield_kernel(const S* H, int ldh, int W, int n, int n_up, int Tp, int din_p, S* Hbar) {
  const int64_t total = (int64_t)W * Tp * 2 * din_p;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx % (2 * din_p));
    const int64_t row = idx / (2 * din_p);
    const int t = (int)(row % Tp);
    const int64_t w = row / Tp;
    const int al = c / din_p, f = c % din_p;
    const int j0 = al == 0 ? 0 : n_up, na = al == 0 ? n_up : n - n_up;
    S acc = 0;
    for (int j = j0; j < j0 + na; ++j) acc += H[((w * n + j) * Tp + t) * (int64_t)ldh + f];
    Hbar[idx] = na > 0 ? acc / (S)na : (S)0;
  }
}

// float32 version: one thread per 4 consecutive features of one (walker,
// jet row), both spins, 16-byte loads (din_p and ldh multiples of 4).  A
// thread's loads are issued eight at a time before any is added, so that
// eight are in flight per thread; the sums still take j in order.  I is the
// item index type (32-bit when the item count allows).
template <class I>
__global__ void meanfield4_kernel(const float* H, int ldh, int W, int n, int n_up, int Tp, int din_p, float* Hbar) {
  const I q4 = (I)(din_p / 4);
  const I total = (I)W * (I)Tp * q4;
  const float iu = n_up > 0 ? 1.0f / (float)n_up : 0.0f;
  const float id = n - n_up > 0 ? 1.0f / (float)(n - n_up) : 0.0f;
  const int64_t js = (int64_t)Tp * ldh;  // electron stride
  for (I idx = (I)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (I)gridDim.x * blockDim.x) {
    const int f = (int)(idx % q4) * 4;
    const I row = idx / q4;  // w Tp + t
    const int t = (int)(row % (I)Tp);
    const int64_t w = (int64_t)(row / (I)Tp);
    const float* src = H + (w * n * Tp + t) * (int64_t)ldh + f;
    float4 su = {0.f, 0.f, 0.f, 0.f}, sd = {0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < n; j0 += 8) {
      float4 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        v[k] = j0 + k < n ? *reinterpret_cast<const float4*>(src + (j0 + k) * js) : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (j0 + k >= n) break;
        float4& s = j0 + k < n_up ? su : sd;
        s.x += v[k].x;
        s.y += v[k].y;
        s.z += v[k].z;
        s.w += v[k].w;
      }
    }
    float* o = Hbar + (int64_t)row * 2 * din_p + f;
    *reinterpret_cast<float4*>(o) = float4{su.x * iu, su.y * iu, su.z * iu, su.w * iu};
    *reinterpret_cast<float4*>(o + din_p) = float4{sd.x * id, sd.y * id, sd.z * id, sd.w * id};
  }
}

// float64 version: one thread per 2 consecutive features of one (walker,
// jet row), both spins, 16-byte loads (din_p and ldh even), the sums in j
// order divided by n_a as meanfield_kernel does
__global__ void meanfield2_kernel(const double* H, int ldh, int W, int n, int n_up, int Tp, int din_p, double* Hbar) {
  const int q2 = din_p / 2;
  const int64_t total = (int64_t)W * Tp * q2;
  const int64_t js = (int64_t)Tp * ldh;  // electron stride
  const int nd = n - n_up;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(idx % q2) * 2;
    const int64_t row = idx / q2;  // w Tp + t
    const int t = (int)(row % Tp);
    const int64_t w = row / Tp;
    const double* src = H + (w * n * Tp + t) * (int64_t)ldh + f;
    double2 su = {0.0, 0.0}, sd = {0.0, 0.0};
    for (int j = 0; j < n; ++j) {
      const double2 v = *reinterpret_cast<const double2*>(src + j * js);
      if (j < n_up) {
        su.x += v.x;
        su.y += v.y;
      } else {
        sd.x += v.x;
        sd.y += v.y;
      }
    }
    double* o = Hbar + row * 2 * din_p + f;
    *reinterpret_cast<double2*>(o) = n_up > 0 ? double2{su.x / (double)n_up, su.y / (double)n_up} : double2{0.0, 0.0};
    *reinterpret_cast<double2*>(o + din_p) = nd > 0 ? double2{sd.x / (double)nd, sd.y / (double)nd} : double2{0.0, 0.0};
  }
}

hipError_t launch_meanfield(bool f64, const void* H, int ldh, int W, int n, int n_up, int Tp, int din_p, void* Hbar,
                            hipStream_t s) {
  int64_t total = (int64_t)W * Tp * 2 * din_p;
  int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  if (grid <= 0) return hipSuccess;
  if (f64) {
    if (din_p % 2 == 0 && ldh % 2 == 0) {
      const int64_t t2 = (int64_t)W * Tp * (din_p / 2);
      hipLaunchKernelGGL(meanfield2_kernel, dim3((unsigned)std::min<int64_t>((t2 + 255) / 256, 65536)), dim3(256), 0, s,
                         (const double*)H, ldh, W, n, n_up, Tp, din_p, (double*)Hbar);
    } else {
      hipLaunchKernelGGL(meanfield_kernel<double>, dim3(grid), dim3(256), 0, s, (const double*)H, ldh, W, n, n_up, Tp,
                         din_p, (double*)Hbar);
    }
    return hipGetLastError();
  }
  if (din_p % 4 == 0 && ldh % 4 == 0) {
    const int64_t t4 = (int64_t)W * Tp * (din_p / 4);
    const dim3 grid4((unsigned)std::min<int64_t>((t4 + 255) / 256, 1 << 20));
    if (t4 + (int64_t)grid4.x * 256 < (1LL << 32))
      hipLaunchKernelGGL(meanfield4_kernel<uint32_t>, grid4, dim3(256), 0, s, (const float*)H, ldh, W, n, n_up, Tp, din_p,
                         (float*)Hbar);
    else
      hipLaunchKernelGGL(meanfield4_kernel<int64_t>, grid4, dim3(256), 0, s, (const float*)H, ldh, W, n, n_up, Tp, din_p,
                         (float*)Hbar);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(meanfield_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)H, ldh, W, n, n_up, Tp, din_p,
                     (float*)Hbar);
  return hipGetLastError();
}

}  // namespace fn
