// Jet GEMM on CDNA4 matrix cores with fused epilogues.
//
// The one-electron layers of the permutation-equivariant network, the
// projection of the mean field and the orbital projection of Eq. (5) are
// all products  rows x K  by  K x N  where every row is one jet row (value,
// one of the 3n tangents, or the Laplacian) of one electron of one walker.
// The 3n+2 jet rows of an electron are what make these products dense;
// a workgroup tile always holds whole electrons so that the epilogue can
// apply the chain rule of tanh (which needs the sum over tangent rows of
// the squared pre-activation) or the product rule with the envelope
// without leaving the tile.
//
// Tile: BM rows (whole electrons) x BN columns, 256 threads as 2 x 2
// wavefronts of 64, each wavefront a grid of 16x16 MFMA tiles.  Three
// arithmetic modes:
//   MODE_F32:   v_mfma_f32_16x16x4_f32 on float32 operands, K step 32
//   MODE_BF16X3: each operand split x = hi + lo into two bfloat16 (16
//               significand bits in all) and x y ~ hi_x hi_y + hi_x lo_y +
//               lo_x hi_y by three v_mfma_f32_16x16x32_bf16 into one
//               float32 accumulator; the activations are split while being
//               staged into LDS, the weights are pre-split by the packer
//   MODE_F64:   v_mfma_f64_16x16x4_f64 on float64 operands, K step 16, with
//               float64 activations and a float64 epilogue (the float64
//               re-evaluation of ill-conditioned walkers)
// Global -> register -> LDS double buffering: the next K tile is fetched
// while the current one is multiplied.
#include "common.h"
#include "kernels.h"

namespace fn {

template <int MODE> struct ModeT {
  using S = float;  // activations, accumulators and epilogue
  using Acc = floatx4;
  static constexpr int BK = 32;
  static constexpr int LDS_K = MODE == MODE_F32 ? BK + 4 : BK + 8;  // staged row stride (elements)
  static constexpr int ESZ = MODE == MODE_F32 ? 4 : 2;
  static constexpr int PLANES = MODE == MODE_F32 ? 1 : 2;
  static constexpr int VPR_A = BK / 4;                               // 16-byte vectors per A tile row
  static constexpr int VPR_B = MODE == MODE_F32 ? BK / 4 : BK / 8;   // 16-byte vectors per B tile row
  static constexpr int LDC_PAD = 4;
};
template <> struct ModeT<MODE_BF16X6> {
  using S = float;
  using Acc = floatx4;
  static constexpr int BK = 32;
  static constexpr int LDS_K = BK + 8;  // staged row stride (bfloat16 elements)
  static constexpr int ESZ = 2;
  static constexpr int PLANES = 3;
  static constexpr int VPR_A = BK / 4;  // A and B both read as float32, split while staged
  static constexpr int VPR_B = BK / 4;
  static constexpr int LDC_PAD = 4;
};
template <> struct ModeT<MODE_F64> {
  using S = double;
  using Acc = doublex4;
  static constexpr int BK = 16;
  static constexpr int LDS_K = BK + 1;
  static constexpr int ESZ = 8;
  static constexpr int PLANES = 1;
  static constexpr int VPR_A = BK / 2;
  static constexpr int VPR_B = BK / 2;
  static constexpr int LDC_PAD = 1;
};

template <int MODE, int BM, int BN>
struct Smem {
  using M = ModeT<MODE>;
  static constexpr int BK = M::BK;
  static constexpr int LDS_K = M::LDS_K;
  static constexpr int A_PLANE = BM * LDS_K * M::ESZ;
  static constexpr int B_PLANE = BN * LDS_K * M::ESZ;
  static constexpr int AB_BYTES = M::PLANES * (A_PLANE + B_PLANE);
  static constexpr int LDC = BN + M::LDC_PAD;
  static constexpr int C_BYTES = BM * LDC * (int)sizeof(typename M::S);
  static constexpr int BYTES = AB_BYTES > C_BYTES ? AB_BYTES : C_BYTES;
};

__device__ inline uint32_t pack2(uint16_t a, uint16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

template <int MODE, int BM, int BN, int EPI>
__global__ __launch_bounds__(256) void jet_gemm_kernel(JetGemmArgs a, int n_mtiles, int n_ntiles) {
  using SM = Smem<MODE, BM, BN>;
  using MT = ModeT<MODE>;
  using S = typename MT::S;
  constexpr int BK = SM::BK;
  constexpr int LDS_K = SM::LDS_K;
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int VPR_A = MT::VPR_A, VPR_B = MT::VPR_B;
  constexpr int NVA = (BM * VPR_A + 255) / 256;
  constexpr int NVB = (BN * VPR_B + 255) / 256;
  __shared__ __attribute__((aligned(16))) char smem[SM::BYTES];
  S* Cs = reinterpret_cast<S*>(smem);

  // XCD-aware tile order: the n_ntiles column tiles of one row tile are
  // given block ids that differ by multiples of 8, so they land on the same
  // XCD and share its L2 for the A tile.
  const int bid = blockIdx.x;
  const int n_t = (bid / 8) % n_ntiles;
  const int m_t = (bid / (8 * n_ntiles)) * 8 + (bid % 8);
  if (m_t >= n_mtiles) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int rows_per = a.rows_per;
  const int E = BM / rows_per;
  const int g0 = m_t * E;
  const int n0 = n_t * BN;
  const int K = a.ka0 + a.ka1;
  const int nkt = K / BK;

  // memory rows of this thread's A vectors (fixed over the K loop)
  long rowoff[NVA];
#pragma unroll
  for (int i = 0; i < NVA; ++i) {
    int v = tid + i * 256;
    rowoff[i] = -1;
    if (v < BM * VPR_A) {
      int r = v / VPR_A;
      int e = r / rows_per, t = r % rows_per;
      int g = g0 + e;
      if (g < a.n_groups) {
        long mg = (long)(g / a.n_sub) * a.n_all + a.e_off + (g % a.n_sub);
        rowoff[i] = mg * rows_per + t;
      }
    }
  }

  // A and B elements: S (float32 or float64); the split form reads bfloat16 B
  constexpr int EA = 16 / (int)sizeof(S);  // A elements per 16-byte vector
  uint4 ra[NVA], rb[NVB], rbl[MODE == MODE_BF16X3 ? NVB : 1];
  auto load = [&](int kt) {
    const int kb = kt * BK;
    const S* src;
    int lda, kk;
    if (kb < a.ka0) {
      src = (const S*)a.a0;
      lda = a.lda0;
      kk = kb;
    } else {
      src = (const S*)a.a1;
      lda = a.lda1;
      kk = kb - a.ka0;
    }
#pragma unroll
    for (int i = 0; i < NVA; ++i) {
      int v = tid + i * 256;
      uint4 z = {0, 0, 0, 0};
      if (v < BM * VPR_A && rowoff[i] >= 0) {
        int kv = (v % VPR_A) * EA;
        z = *reinterpret_cast<const uint4*>(src + (size_t)rowoff[i] * lda + kk + kv);
      }
      ra[i] = z;
    }
#pragma unroll
    for (int i = 0; i < NVB; ++i) {
      int v = tid + i * 256;
      uint4 z = {0, 0, 0, 0}, zl = {0, 0, 0, 0};
      if (v < BN * VPR_B) {
        int nn = v / VPR_B, col = n0 + nn;
        if (col < a.N) {
          if constexpr (MODE == MODE_BF16X3) {
            int kv = (v % VPR_B) * 8;
            z = *reinterpret_cast<const uint4*>((const uint16_t*)a.bt + (size_t)col * a.ldb + kb + kv);
            zl = *reinterpret_cast<const uint4*>((const uint16_t*)a.bt_lo + (size_t)col * a.ldb + kb + kv);
          } else {
            int kv = (v % VPR_B) * EA;
            z = *reinterpret_cast<const uint4*>((const S*)a.bt + (size_t)col * a.ldb + kb + kv);
          }
        }
      }
      rb[i] = z;
      if constexpr (MODE == MODE_BF16X3) rbl[i] = zl;
    }
  };
  auto store = [&]() {
    if constexpr (MODE == MODE_F32) {
      float* As = reinterpret_cast<float*>(smem);
      float* Bs = reinterpret_cast<float*>(smem + SM::A_PLANE);
#pragma unroll
      for (int i = 0; i < NVA; ++i) {
        int v = tid + i * 256;
        if (v < BM * VPR_A) *reinterpret_cast<uint4*>(As + (v / VPR_A) * LDS_K + (v % VPR_A) * 4) = ra[i];
      }
#pragma unroll
      for (int i = 0; i < NVB; ++i) {
        int v = tid + i * 256;
        if (v < BN * VPR_B) *reinterpret_cast<uint4*>(Bs + (v / VPR_B) * LDS_K + (v % VPR_B) * 4) = rb[i];
      }
    } else if constexpr (MODE == MODE_F64) {
      // odd row stride: 8-byte stores
      double* As = reinterpret_cast<double*>(smem);
      double* Bs = reinterpret_cast<double*>(smem + SM::A_PLANE);
#pragma unroll
      for (int i = 0; i < NVA; ++i) {
        int v = tid + i * 256;
        if (v < BM * VPR_A) {
          double* d = As + (v / VPR_A) * LDS_K + (v % VPR_A) * 2;
          d[0] = __builtin_bit_cast(double, uint2{ra[i].x, ra[i].y});
          d[1] = __builtin_bit_cast(double, uint2{ra[i].z, ra[i].w});
        }
      }
#pragma unroll
      for (int i = 0; i < NVB; ++i) {
        int v = tid + i * 256;
        if (v < BN * VPR_B) {
          double* d = Bs + (v / VPR_B) * LDS_K + (v % VPR_B) * 2;
          d[0] = __builtin_bit_cast(double, uint2{rb[i].x, rb[i].y});
          d[1] = __builtin_bit_cast(double, uint2{rb[i].z, rb[i].w});
        }
      }
    } else if constexpr (MODE == MODE_BF16X6) {
      // three bfloat16 planes of A, then three of B, rows of LDS_K elements
      uint16_t* Ap = reinterpret_cast<uint16_t*>(smem);
      uint16_t* Bp = reinterpret_cast<uint16_t*>(smem + 3 * SM::A_PLANE);
      constexpr int AP = SM::A_PLANE / 2, BP = SM::B_PLANE / 2;  // plane strides (elements)
#pragma unroll
      for (int i = 0; i < NVA; ++i) {
        int v = tid + i * 256;
        if (v < BM * VPR_A) {
          uint32_t h0, m0, l0, h1, m1, l1;
          split3_bf16x2(__builtin_bit_cast(float, ra[i].x), __builtin_bit_cast(float, ra[i].y), &h0, &m0, &l0);
          split3_bf16x2(__builtin_bit_cast(float, ra[i].z), __builtin_bit_cast(float, ra[i].w), &h1, &m1, &l1);
          const int off = (v / VPR_A) * LDS_K + (v % VPR_A) * 4;
          *reinterpret_cast<uint2*>(Ap + off) = uint2{h0, h1};
          *reinterpret_cast<uint2*>(Ap + AP + off) = uint2{m0, m1};
          *reinterpret_cast<uint2*>(Ap + 2 * AP + off) = uint2{l0, l1};
        }
      }
#pragma unroll
      for (int i = 0; i < NVB; ++i) {
        int v = tid + i * 256;
        if (v < BN * VPR_B) {
          uint32_t h0, m0, l0, h1, m1, l1;
          split3_bf16x2(__builtin_bit_cast(float, rb[i].x), __builtin_bit_cast(float, rb[i].y), &h0, &m0, &l0);
          split3_bf16x2(__builtin_bit_cast(float, rb[i].z), __builtin_bit_cast(float, rb[i].w), &h1, &m1, &l1);
          const int off = (v / VPR_B) * LDS_K + (v % VPR_B) * 4;
          *reinterpret_cast<uint2*>(Bp + off) = uint2{h0, h1};
          *reinterpret_cast<uint2*>(Bp + BP + off) = uint2{m0, m1};
          *reinterpret_cast<uint2*>(Bp + 2 * BP + off) = uint2{l0, l1};
        }
      }
    } else {
      uint16_t* Ah = reinterpret_cast<uint16_t*>(smem);
      uint16_t* Al = reinterpret_cast<uint16_t*>(smem + SM::A_PLANE);
      uint16_t* Bh = reinterpret_cast<uint16_t*>(smem + 2 * SM::A_PLANE);
      uint16_t* Bl = reinterpret_cast<uint16_t*>(smem + 2 * SM::A_PLANE + SM::B_PLANE);
#pragma unroll
      for (int i = 0; i < NVA; ++i) {
        int v = tid + i * 256;
        if (v < BM * VPR_A) {
          const float x[4] = {__builtin_bit_cast(float, ra[i].x), __builtin_bit_cast(float, ra[i].y),
                              __builtin_bit_cast(float, ra[i].z), __builtin_bit_cast(float, ra[i].w)};
          uint16_t h[4], l[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) split_bf16(x[q], &h[q], &l[q]);
          const int off = (v / VPR_A) * LDS_K + (v % VPR_A) * 4;
          *reinterpret_cast<uint2*>(Ah + off) = uint2{pack2(h[0], h[1]), pack2(h[2], h[3])};
          *reinterpret_cast<uint2*>(Al + off) = uint2{pack2(l[0], l[1]), pack2(l[2], l[3])};
        }
      }
#pragma unroll
      for (int i = 0; i < NVB; ++i) {
        int v = tid + i * 256;
        if (v < BN * VPR_B) {
          const int off = (v / VPR_B) * LDS_K + (v % VPR_B) * 8;
          *reinterpret_cast<uint4*>(Bh + off) = rb[i];
          *reinterpret_cast<uint4*>(Bl + off) = rbl[i];
        }
      }
    }
  };

  typename MT::Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = typename MT::Acc{0, 0, 0, 0};

  const int arow = wm * (BM / 2) + (lane & 15);
  const int brow = wn * (BN / 2) + (lane & 15);
  const int kq = lane >> 4;

  if (nkt > 0) load(0);
  for (int kt = 0; kt < nkt; ++kt) {
    __syncthreads();
    store();
    __syncthreads();
    if (kt + 1 < nkt) load(kt + 1);
    if constexpr (MODE == MODE_F32 || MODE == MODE_F64) {
      const S* As = reinterpret_cast<const S*>(smem);
      const S* Bs = reinterpret_cast<const S*>(smem + SM::A_PLANE);
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        S af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = As[(arow + i * 16) * LDS_K + ks * 4 + kq];
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = Bs[(brow + j * 16) * LDS_K + ks * 4 + kq];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            if constexpr (MODE == MODE_F64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bfr[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
          }
      }
    } else if constexpr (MODE == MODE_BF16X6) {
      const uint16_t* Ap = reinterpret_cast<const uint16_t*>(smem);
      const uint16_t* Bp = reinterpret_cast<const uint16_t*>(smem + 3 * SM::A_PLANE);
      constexpr int AP = SM::A_PLANE / 2, BP = SM::B_PLANE / 2;
      bf16x8 a1[TM], a2[TM], a3[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = (arow + i * 16) * LDS_K + kq * 8;
        a1[i] = *reinterpret_cast<const bf16x8*>(Ap + o);
        a2[i] = *reinterpret_cast<const bf16x8*>(Ap + AP + o);
        a3[i] = *reinterpret_cast<const bf16x8*>(Ap + 2 * AP + o);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = (brow + j * 16) * LDS_K + kq * 8;
        const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(Bp + o);
        const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(Bp + BP + o);
        const bf16x8 b3 = *reinterpret_cast<const bf16x8*>(Bp + 2 * BP + o);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          // the products of order 2^-16, then 2^-8, then the leading one
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[i], b1, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[i], b2, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], b3, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[i], b1, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], b2, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[i], b1, acc[i][j], 0, 0, 0);
        }
      }
    } else {
      const uint16_t* Ah = reinterpret_cast<const uint16_t*>(smem);
      const uint16_t* Al = reinterpret_cast<const uint16_t*>(smem + SM::A_PLANE);
      const uint16_t* Bh = reinterpret_cast<const uint16_t*>(smem + 2 * SM::A_PLANE);
      const uint16_t* Bl = reinterpret_cast<const uint16_t*>(smem + 2 * SM::A_PLANE + SM::B_PLANE);
      bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ah[i] = *reinterpret_cast<const bf16x8*>(Ah + (arow + i * 16) * LDS_K + kq * 8);
        al[i] = *reinterpret_cast<const bf16x8*>(Al + (arow + i * 16) * LDS_K + kq * 8);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        bh[j] = *reinterpret_cast<const bf16x8*>(Bh + (brow + j * 16) * LDS_K + kq * 8);
        bl[j] = *reinterpret_cast<const bf16x8*>(Bl + (brow + j * 16) * LDS_K + kq * 8);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          // small cross terms first, then the leading term
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
  }
  __syncthreads();
  // accumulators -> LDS tile [BM][BN]; the layer epilogue first adds the
  // per-walker mean-field term P (every jet row) and the bias (value row),
  // all loads issued together from the accumulator layout.  Item r of lane
  // (kq, c) holds row 4 kq + r of its 16x16 tile for the float32 and
  // bfloat16 instructions, row kq + 4 r for the float64 one; column c.
  constexpr int LDC = SM::LDC;
  const int T = a.T;
  S bj[TN];
  if constexpr (EPI == EPI_TANHJET) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int gc = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
      bj[j] = gc < a.N ? (S)a.bias[gc] : (S)0;
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    // the P loads of the 16-row tile are issued together (rows and columns
    // clamped into range, masked afterwards)
    S pv[4][TN];
    if constexpr (EPI == EPI_TANHJET) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * (BM / 2) + i * 16 + (MODE == MODE_F64 ? kq + 4 * r : kq * 4 + r);
        const int e = row / rows_per, t = row % rows_per;
        const int g = min(g0 + e, a.n_groups - 1);
        const S* Prow = (const S*)a.P + ((size_t)(g / a.n_all) * rows_per + min(t, T - 1)) * a.ldp;
#pragma unroll
        for (int j = 0; j < TN; ++j) pv[r][j] = Prow[min(n0 + wn * (BN / 2) + j * 16 + (lane & 15), a.N - 1)];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = wm * (BM / 2) + i * 16 + (MODE == MODE_F64 ? kq + 4 * r : kq * 4 + r);
      bool live = false, bias_row = false;
      if constexpr (EPI == EPI_TANHJET) {
        const int e = row / rows_per, t = row % rows_per;
        live = g0 + e < a.n_groups && t < T;
        bias_row = t == 0;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = wn * (BN / 2) + j * 16 + (lane & 15);
        S v = acc[i][j][r];
        if constexpr (EPI == EPI_TANHJET) {
          if (live && n0 + col < a.N) {
            v += pv[r][j];
            if (bias_row) v += bj[j];
          }
        }
        Cs[row * LDC + col] = v;
      }
    }
  }
  __syncthreads();
  if constexpr (EPI == EPI_PLAIN) {
    for (int p = tid; p < BM * BN; p += 256) {
      int r = p / BN, col = p % BN;
      int e = r / rows_per, t = r % rows_per;
      int g = g0 + e, gc = n0 + col;
      if (g < a.n_groups && gc < a.N) {
        const long og = a.c_nsub ? (long)(g / a.c_nsub) * a.c_nall + a.c_eoff + (g % a.c_nsub) : (long)g;
        S* dst = (S*)a.c + ((size_t)og * rows_per + t) * a.ldc + gc;
        const S v = Cs[r * LDC + col];
        *dst = a.c_accum ? *dst + v : v;
      }
    }
  } else if constexpr (EPI == EPI_TANHJET) {
    // chain rule of tanh on each (electron, feature) jet, in place in LDS:
    //   y = tanh(u0), d_c y = sech^2(u0) d_c u,
    //   lap y = sech^2(u0) lap u - 2 tanh(u0) sech^2(u0) sum_c (d_c u)^2
    for (int p = tid; p < E * BN; p += 256) {
      const int e = p / BN, col = p % BN;
      const int g = g0 + e, gc = n0 + col;
      if (g >= a.n_groups || gc >= a.N) continue;
      S* Cr = Cs + (e * rows_per) * LDC + col;
      const S u0 = Cr[0];
      S y, dy;
      tanh_sech2(u0, &y, &dy);
      if (a.pre_out) a.pre_out[(size_t)g * a.N + gc] = (float)u0;
      Cr[0] = y;
      if (T > 1) {
        S s2 = 0;
        for (int t = 1; t < T - 1; ++t) {
          const S u = Cr[t * LDC];
          s2 += u * u;
        }
        for (int t = 1; t < T - 1; ++t) Cr[t * LDC] *= dy;
        Cr[(T - 1) * LDC] = dy * Cr[(T - 1) * LDC] - (S)2 * y * dy * s2;
        for (int t = T; t < rows_per; ++t) Cr[t * LDC] = 0;
      }
    }
    __syncthreads();
    // coalesced write-out of whole rows, residual added on the way
    S* out = reinterpret_cast<S*>(a.out);
    const S* res = reinterpret_cast<const S*>(a.a0);
    if constexpr (MODE == MODE_F64) {
      for (int p = tid; p < BM * BN; p += 256) {
        const int r = p / BN, c = p % BN;
        const int e = r / rows_per, t = r % rows_per;
        const int g = g0 + e, gc = n0 + c;
        if (g >= a.n_groups || gc >= a.N) continue;
        const size_t orow = (size_t)g * rows_per + t;
        S v = Cs[r * LDC + c];
        if (a.res) v += res[orow * a.lda0 + gc];
        out[orow * a.ldo + gc] = v;
      }
    } else {
      constexpr int V4 = BN / 4;
      for (int p = tid; p < BM * V4; p += 256) {
        const int r = p / V4, c4 = (p % V4) * 4;
        const int e = r / rows_per, t = r % rows_per;
        const int g = g0 + e, gc = n0 + c4;
        if (g >= a.n_groups || gc >= a.N) continue;
        const size_t orow = (size_t)g * rows_per + t;
        float4 v = *reinterpret_cast<const float4*>(Cs + r * LDC + c4);
        if (a.res) {
          const float4 rr = *reinterpret_cast<const float4*>(res + orow * a.lda0 + gc);
          v.x += rr.x;
          v.y += rr.y;
          v.z += rr.z;
          v.w += rr.w;
        }
        *reinterpret_cast<float4*>(out + orow * a.ldo + gc) = v;
        if (a.val_out && t == 0) *reinterpret_cast<float4*>(a.val_out + (size_t)g * a.N + gc) = v;
      }
    }
  } else {  // EPI_ORBITAL
    const int na = a.n_sub;
    const int nsq = na * na;
    const int Kd = a.N / na;
    S* phi = reinterpret_cast<S*>(a.phi);
    // items (electron e, orbital i, determinant k) of the tile's columns
    // gc = k n_a + i.  With the matrix-index-fastest layout (phi_M > 0) k
    // runs fastest, so consecutive lanes store consecutive matrices of one
    // (jet row, electron, orbital); otherwise i runs fastest (consecutive
    // orbitals are adjacent in memory).
    const int k_lo = n0 / na, nk = min(Kd, (n0 + BN - 1) / na + 1) - k_lo;
    const int per_e = na * nk;
    for (int p = tid; p < E * per_e; p += 256) {
      const int e = p / per_e, r = p - e * per_e;
      int i, k;
      if (a.phi_M) {
        i = r / nk;
        k = k_lo + (r - i * nk);
      } else {
        const int kk = r / na;
        i = r - kk * na;
        k = k_lo + kk;
      }
      const int gc = k * na + i, col = gc - n0;
      const int g = g0 + e;
      if (g >= a.n_groups || col < 0 || col >= BN || gc >= a.N) continue;
      const int w = g / na, jj = g % na;
      const int j = a.e_off + jj;  // electron index
      const float* rj = a.pos + ((size_t)w * a.n_elec + j) * 3;
      const S x0 = rj[0], x1 = rj[1], x2 = rj[2];
      // envelope sum_m pi exp(-s_m) and its gradient and Laplacian with
      // respect to r_j, d = r_j - R_m:
      //   isotropic: s = |sigma| |d|, grad s = |sigma| d / |d|,
      //              lap s = 2 |sigma| / |d|
      //   full:      s = |u|, u = Sigma d, grad s = Sigma^T u / s,
      //              lap s = (tr(Sigma^T Sigma) - |grad s|^2) / s
      //   grad e = -e grad s, lap e = e (|grad s|^2 - lap s)
      S e0 = 0, ex = 0, ey = 0, ez = 0, le = 0;
      for (int m = 0; m < a.n_nuc; ++m) {
        const S dx = x0 - (S)a.nuc[3 * m], dyv = x1 - (S)a.nuc[3 * m + 1], dz = x2 - (S)a.nuc[3 * m + 2];
        const S pim = (S)a.pi[(size_t)gc * a.n_nuc + m];
        if (a.env_full) {
          const float* Sg = a.sigma + ((size_t)gc * a.n_nuc + m) * 9;
          S M[9];
#pragma unroll
          for (int q = 0; q < 9; ++q) M[q] = (S)Sg[q];
          const S u0 = M[0] * dx + M[1] * dyv + M[2] * dz;
          const S u1 = M[3] * dx + M[4] * dyv + M[5] * dz;
          const S u2 = M[6] * dx + M[7] * dyv + M[8] * dz;
          const S sv = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
          const S inv_s = (S)1 / sv;
          const S g0 = (M[0] * u0 + M[3] * u1 + M[6] * u2) * inv_s;
          const S g1 = (M[1] * u0 + M[4] * u1 + M[7] * u2) * inv_s;
          const S g2 = (M[2] * u0 + M[5] * u1 + M[8] * u2) * inv_s;
          S tr = 0;
#pragma unroll
          for (int q = 0; q < 9; ++q) tr += M[q] * M[q];
          const S gg = g0 * g0 + g1 * g1 + g2 * g2;
          const S v = pim * exp(-sv);
          e0 += v;
          ex -= v * g0;
          ey -= v * g1;
          ez -= v * g2;
          le += v * (gg - (tr - gg) * inv_s);
        } else {
          const S d = sqrt(dx * dx + dyv * dyv + dz * dz);
          const S sg = fabs((S)a.sigma[(size_t)gc * a.n_nuc + m]);
          const S v = pim * exp(-sg * d);
          const S inv_d = (S)1 / d;
          e0 += v;
          ex -= sg * v * dx * inv_d;
          ey -= sg * v * dyv * inv_d;
          ez -= sg * v * dz * inv_d;
          le += v * (sg * sg - (S)2 * sg * inv_d);
        }
      }
      const S* Cr = Cs + (e * rows_per) * LDC + col;
      const S u0 = Cr[0] + (S)a.g_orb[gc];
      const int64_t mat = (int64_t)w * Kd + k;
      const size_t ts = a.phi_M ? (size_t)nsq * a.phi_M : (size_t)nsq;  // stride between jet rows
      S* ph = a.phi_M ? phi + (size_t)(jj * na + i) * a.phi_M + mat : phi + (size_t)mat * T * nsq + jj * na + i;
      ph[0] = u0 * e0;
      if (a.u_out) {
        size_t o = ((size_t)(w * Kd + k) * na + jj) * na + i;
        a.u_out[o] = (float)u0;
        a.env_out[o] = (float)e0;
      }
      if (T > 1) {
        const int tj = 1 + 3 * j;
        for (int t = 1; t < T - 1; ++t) ph[(size_t)t * ts] = Cr[t * LDC] * e0;
        const S ux = Cr[tj * LDC], uy = Cr[(tj + 1) * LDC], uz = Cr[(tj + 2) * LDC];
        ph[(size_t)tj * ts] += u0 * ex;
        ph[(size_t)(tj + 1) * ts] += u0 * ey;
        ph[(size_t)(tj + 2) * ts] += u0 * ez;
        const S lu = Cr[(T - 1) * LDC];
        ph[(size_t)(T - 1) * ts] = lu * e0 + u0 * le + (S)2 * (ux * ex + uy * ey + uz * ez);
      }
    }
  }
}

template <int MODE, int BM, int BN, int EPI>
static hipError_t run(const JetGemmArgs& a, hipStream_t s) {
  const int E = BM / a.rows_per;
  const int n_mtiles = (a.n_groups + E - 1) / E;
  const int n_ntiles = (a.N + BN - 1) / BN;
  const int grid = ((n_mtiles + 7) / 8) * 8 * n_ntiles;
  hipLaunchKernelGGL((jet_gemm_kernel<MODE, BM, BN, EPI>), dim3(grid), dim3(256), 0, s, a, n_mtiles, n_ntiles);
  return hipGetLastError();
}

template <int MODE, int EPI>
static hipError_t pick(const JetGemmArgs& a, hipStream_t s) {
  const bool bm96 = a.rows_per == 96;
  if (!bm96 && (128 % a.rows_per) != 0) return hipErrorInvalidValue;
  if constexpr (MODE == MODE_F64) {
    // float64 tiles sized for the LDS epilogue tile (at most 50 KiB)
    if (bm96) return run<MODE, 96, 64, EPI>(a, s);
    if (a.rows_per == 128) return run<MODE, 128, 32, EPI>(a, s);
    return run<MODE, 64, 64, EPI>(a, s);
  } else {
    // column tile: the one of 128, 96, 64 that wastes the fewest columns
    // (the wider on ties); e.g. 96 for the 80 orbital columns of 16
    // determinants of 5 electrons
    const int w128 = (a.N + 127) / 128 * 128 - a.N;
    const int w96 = (a.N + 95) / 96 * 96 - a.N;
    const int w64 = (a.N + 63) / 64 * 64 - a.N;
    const int bn = a.N <= 64 ? 64 : (w128 <= w96 && w128 <= w64) ? 128 : (w96 <= w64 ? 96 : 64);
    if (a.rows_per == 1) {
      // value pass (one row per electron): row tiles of 128, 64 or 32 rows,
      // the largest that still gives the launch about 1024 workgroups
      const int64_t nt = (a.N + bn - 1) / bn;
      const int bm = (int64_t)(a.n_groups + 127) / 128 * nt >= 1024 ? 128
                     : (int64_t)(a.n_groups + 63) / 64 * nt >= 1024 ? 64 : 32;
      if (bm == 64) {
        if (bn == 128) return run<MODE, 64, 128, EPI>(a, s);
        if (bn == 96) return run<MODE, 64, 96, EPI>(a, s);
        return run<MODE, 64, 64, EPI>(a, s);
      }
      if (bm == 32) {
        if (bn == 128) return run<MODE, 32, 128, EPI>(a, s);
        if (bn == 96) return run<MODE, 32, 96, EPI>(a, s);
        return run<MODE, 32, 64, EPI>(a, s);
      }
    }
    if (bm96) {
      if (bn == 128) return run<MODE, 96, 128, EPI>(a, s);
      if (bn == 96) return run<MODE, 96, 96, EPI>(a, s);
      return run<MODE, 96, 64, EPI>(a, s);
    }
    // orbital products of 32-row jets: row tiles of three electrons (more
    // workgroups per CU than four-electron tiles; the Ne-like orbital stage
    // 0.58 -> 0.51 ms in the six-product form, 0.67 -> 0.65 ms in fp32)
    if (EPI == EPI_ORBITAL && a.rows_per == 32 && bn == 96) return run<MODE, 96, 96, EPI>(a, s);
    if (bn == 128) return run<MODE, 128, 128, EPI>(a, s);
    if (bn == 96) return run<MODE, 128, 96, EPI>(a, s);
    return run<MODE, 128, 64, EPI>(a, s);
  }
}

template <int MODE>
static hipError_t pick_epi(int epi, const JetGemmArgs& a, hipStream_t s) {
  if (epi == EPI_PLAIN) return pick<MODE, EPI_PLAIN>(a, s);
  if (epi == EPI_TANHJET) return pick<MODE, EPI_TANHJET>(a, s);
  return pick<MODE, EPI_ORBITAL>(a, s);
}

hipError_t launch_jet_gemm(int mode, int epi, const JetGemmArgs& a, hipStream_t s) {
  if (a.n_groups <= 0) return hipSuccess;
  if ((a.ka0 % 32) || (a.ka1 % 32)) return hipErrorInvalidValue;
  if (a.mf_out && (mode == MODE_F64 || epi != EPI_TANHJET || !layer_mf_supported(a))) return hipErrorInvalidValue;
  if (mode == MODE_F64) return pick_epi<MODE_F64>(epi, a, s);
  // the one-electron layers take the full-width streaming kernel when their
  // shape allows it
  if (epi == EPI_TANHJET && layer_gemm_supported(a)) return launch_layer_gemm(mode, a, s);
  if (epi == EPI_PLAIN && layer_plain_supported(a)) return launch_layer_plain(mode, a, s);
  if (mode == MODE_BF16X3) return pick_epi<MODE_BF16X3>(epi, a, s);
  if (mode == MODE_BF16X6) return epi == EPI_ORBITAL ? pick<MODE_BF16X6, EPI_ORBITAL>(a, s) : hipErrorInvalidValue;
  return pick_epi<MODE_F32>(epi, a, s);
}

}  // namespace fn
