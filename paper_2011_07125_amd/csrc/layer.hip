// One-electron layer GEMM with the tanh-jet epilogue, sized for the tall,
// skinny products of the jet algebra: rows = walkers x electrons x jet rows
// (millions), K = d1 + 2 d2, N = d1.
//
// Per layer the arithmetic intensity is K N / (2 (K + N)) flop per byte of
// float32 activations (about 50 for K = 320, N = 256), far below the ridge
// of the bfloat16 matrix cores, so the kernel is organised around HBM
// streaming rather than MFMA reuse:
//  * a 512-thread workgroup owns BM rows (whole electrons, and a whole
//    number of waves per electron) x BN = 128 columns; the column tiles of
//    one row tile are issued back to back on the same XCD, so the repeated
//    read of the activations is served by that XCD's L2;
//  * for small atoms (equal spin groups of at most five electrons, 32 jet
//    rows) a workgroup instead owns one spin group of one walker, one wave
//    row per electron, and also writes the group's mean of its output rows:
//    the mean field the next layer reads (Sec. 3) is formed from the tile in
//    LDS instead of by a separate pass that reads every layer output again;
//  * in the split-bfloat16 form each activation element is split into hi/lo
//    parts once, by the thread that stages it into LDS (hardware
//    round-to-nearest-even conversion); the bfloat16 tiles are stored without
//    padding under an XOR swizzle of 16-byte chunks (conflict-free fragment
//    reads), so two stages take 64 KiB and two workgroups share a CU;
//  * the epilogue does not stage the tile in LDS: per column, the jet rows of
//    one electron sit in the accumulators of the wave's four lane groups (and
//    of the electron's other waves when the jet is taller than a wave's
//    rows).  The sum of squared tangents is reduced with cross-lane shuffles
//    and a 4 KiB cross-wave exchange in fixed order, the tanh chain rule is
//    applied in registers, and results go straight to HBM with the residual added;
//  * every global access is a raw buffer operation whose wave-uniform part
//    (tile or electron base, jet row, K step) sits in scalar registers and
//    whose per-lane part is one 32-bit offset computed once: the loops carry
//    no 64-bit address arithmetic and no per-element branches, and rows past
//    the last electron get an offset beyond the buffer range, which the
//    hardware reads as zero.
#include "common.h"
#include "kernels.h"

namespace fn {

template <int MODE, int BM, int BN, int WM, int WN>
struct LayerCfg {
  static constexpr int NT = 64 * WM * WN, BK = 32;
  static constexpr int WROWS = BM / WM, WCOLS = BN / WN;
  static constexpr int TM = WROWS / 16, TN = WCOLS / 16;
  static constexpr int LDA = MODE == MODE_F32 ? BK + 4 : BK;  // elements per staged row
  static constexpr int LDB = LDA;
  static constexpr int A_BYTES = MODE == MODE_F32 ? BM * LDA * 4 : 2 * BM * LDA * 2;
  static constexpr int B_BYTES = MODE == MODE_F32 ? BN * LDB * 4 : 2 * BN * LDB * 2;
  static constexpr int STAGE = A_BYTES + B_BYTES;
  static constexpr int RED_BYTES = 2 * WM * BN * 4;
  static constexpr int BYTES = 2 * STAGE > RED_BYTES ? 2 * STAGE : RED_BYTES;
  static constexpr int NA = BM * BK / 4;  // float4 per A tile
  static constexpr int NVA = (NA + NT - 1) / NT;
  static constexpr int NB = MODE == MODE_F32 ? BN * BK / 4 : BN * BK / 8;  // 16-byte vectors per B plane
  static constexpr int NVB = (NB + NT - 1) / NT;
  static_assert(NT <= 1024 && WROWS % 16 == 0 && WCOLS % 16 == 0, "tile shape");
  static_assert(BN % 128 == 0, "N is a multiple of 128");
};

__device__ inline uint32_t pk2(uint16_t a, uint16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// raw buffer over the 2^31 - 1 bytes from p (word 3: the gfx9 data format
// for untyped 32-bit access); loads at offsets of 2^31 or more return zero
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7fffffff, 0x00020000);
}
constexpr int kOutOfRange = (int)0x80000000;
__device__ inline float ldf(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline void stf(float x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, soff, 0);
}

// element offset of 16-byte chunk c (0..3) of row r in an unpadded bfloat16
// tile of 32-element rows: chunks are permuted by (r >> 1) & 3, so eight
// consecutive rows read at one chunk index cover all banks once
__device__ inline int swz(int r, int c) { return r * 32 + ((c ^ ((r >> 1) & 3)) << 3); }

// KIND_JET: the tanh layer's jet pass (rows_per jet rows per electron);
// KIND_VALUE: its value pass (one row per electron); KIND_PLAIN: the plain
// product c (=, or += with c_accum) over contiguous rows (rows_per = 1)
// KIND_JET_MF: the jet pass over tiles of one spin group each (WM
// electrons of 32 jet rows, one wave row per electron) that also writes the
// group's mean of the output rows (mf_out)
constexpr int KIND_VALUE = 0, KIND_JET = 1, KIND_PLAIN = 2, KIND_JET_MF = 3;

template <int MODE, int BM, int BN, int WM, int WN, int KIND>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(WM * WN >= 8 ? 4 : 2, 8))) void
layer_gemm_kernel(
    JetGemmArgs a, int n_mtiles, int n_ntiles) {
  constexpr bool JET = KIND == KIND_JET || KIND == KIND_JET_MF;
  using C = LayerCfg<MODE, BM, BN, WM, WN>;
  constexpr int BK = C::BK, LDA = C::LDA, LDB = C::LDB, TM = C::TM, TN = C::TN, WROWS = C::WROWS;
  extern __shared__ __attribute__((aligned(16))) char smem[];

  const int bid = blockIdx.x;
  const int n_t = (bid / 8) % n_ntiles;
  const int m_t = (bid / (8 * n_ntiles)) * 8 + (bid % 8);
  if (m_t >= n_mtiles) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int rows_per = JET ? a.rows_per : 1;
  const int E = BM / rows_per;  // electrons per row tile
  const int g0 = m_t * E;
  const int n0 = n_t * BN;
  const int nkt = (a.ka0 + a.ka1) / BK;

  // A loader: 8 float4 per 32-wide tile row, at byte offsets from the
  // tile's first row (row numbers grow with the electron index)
  const int q0 = g0 / a.n_sub, m0 = g0 - q0 * a.n_sub;
  const long row0 = ((long)q0 * a.n_all + a.e_off + m0) * rows_per;
  int voff0[C::NVA], voff1[C::NVA];
#pragma unroll
  for (int i = 0; i < C::NVA; ++i) {
    const int v = tid + i * C::NT;
    const int r = v / (BK / 4);
    const int e = r / rows_per, t = r - e * rows_per;
    const int g = g0 + e;
    // electron g = g0 + e: g / n_sub = q0 + qe, g % n_sub = me (32-bit)
    const int qe = (m0 + e) / a.n_sub, me = m0 + e - qe * a.n_sub;
    const long rr = ((long)qe * a.n_all + (me - m0)) * rows_per + t;
    const int c4 = (v % (BK / 4)) * 4;
    const bool ok = v < C::NA && g < a.n_groups;
    voff0[i] = ok ? (int)((rr * a.lda0 + c4) * 4) : kOutOfRange;
    voff1[i] = ok ? (int)((rr * a.lda1 + c4) * 4) : kOutOfRange;
  }
  const __amdgpu_buffer_rsrc_t rA0 = rsrc((const float*)a.a0 + row0 * a.lda0);
  const __amdgpu_buffer_rsrc_t rA1 = rsrc(a.ka1 > 0 ? (const float*)a.a1 + row0 * a.lda1 : (const float*)a.a0);
  // B loader: columns n0 .. n0 + BN - 1 all exist (N is a multiple of BN)
  constexpr int ESZ = MODE == MODE_F32 ? 4 : 2;
  constexpr int VPR = MODE == MODE_F32 ? BK / 4 : BK / 8;  // 16-byte vectors per B row
  int voffB[C::NVB];
#pragma unroll
  for (int i = 0; i < C::NVB; ++i) {
    const int v = tid + i * C::NT;
    voffB[i] = C::NB % C::NT == 0 || v < C::NB ? ((v / VPR) * a.ldb + (v % VPR) * (16 / ESZ)) * ESZ : kOutOfRange;
  }
  const __amdgpu_buffer_rsrc_t rB = rsrc((const char*)a.bt + (size_t)n0 * a.ldb * ESZ);
  const __amdgpu_buffer_rsrc_t rBl =
      rsrc(MODE == MODE_F32 ? (const char*)a.bt : (const char*)a.bt_lo + (size_t)n0 * a.ldb * ESZ);

  // two register stages in the split-bfloat16 jet pass: the loads of K
  // steps kt+2 and kt+3 are in flight while step kt is multiplied
  struct Regs {
    u32x4 ra[C::NVA];
    u32x4 rb[C::NVB], rbl[MODE == MODE_F32 ? 1 : C::NVB];
  };
  Regs R0, R1;

  // K-step order: the segment-1 steps, the segment-0 steps outside this
  // tile's residual columns, then the residual columns [n0, n0 + BN) of
  // segment 0 last, so that the epilogue's residual loads find them in L2
  const int nk0 = a.ka0 / BK;
  const int r0 = a.res ? n0 / BK : nk0;
  const int nres = a.res ? (n0 + BN <= a.ka0 ? BN / BK : 0) : 0;
  const int n1 = nkt - nk0, nout = nk0 - nres;
  auto ktile = [&](int kt) {
    if (kt < n1) return nk0 + kt;
    kt -= n1;
    if (kt < nout) return kt < r0 ? kt : kt + nres;
    return r0 + (kt - nout);
  };
  auto gload = [&](int kt_step, Regs& R) {
    const int kb = ktile(kt_step) * BK;
    if (kb < a.ka0) {
#pragma unroll
      for (int i = 0; i < C::NVA; ++i) R.ra[i] = __builtin_amdgcn_raw_buffer_load_b128(rA0, voff0[i], kb * 4, 0);
    } else {
#pragma unroll
      for (int i = 0; i < C::NVA; ++i)
        R.ra[i] = __builtin_amdgcn_raw_buffer_load_b128(rA1, voff1[i], (kb - a.ka0) * 4, 0);
    }
#pragma unroll
    for (int i = 0; i < C::NVB; ++i) {
      R.rb[i] = __builtin_amdgcn_raw_buffer_load_b128(rB, voffB[i], kb * ESZ, 0);
      if constexpr (MODE != MODE_F32) R.rbl[i] = __builtin_amdgcn_raw_buffer_load_b128(rBl, voffB[i], kb * ESZ, 0);
    }
  };
  auto sstore = [&](const Regs& R, int buf) {
    const u32x4* ra = R.ra;
    const u32x4* rb = R.rb;
    const u32x4* rbl = R.rbl;
    char* st = smem + buf * C::STAGE;
    if constexpr (MODE == MODE_F32) {
      float* As = reinterpret_cast<float*>(st);
      float* Bs = reinterpret_cast<float*>(st + C::A_BYTES);
#pragma unroll
      for (int i = 0; i < C::NVA; ++i) {
        const int v = tid + i * C::NT;
        if (C::NA % C::NT == 0 || v < C::NA)
          *reinterpret_cast<u32x4*>(As + (v / (BK / 4)) * LDA + (v % (BK / 4)) * 4) = ra[i];
      }
#pragma unroll
      for (int i = 0; i < C::NVB; ++i) {
        const int v = tid + i * C::NT;
        if (C::NB % C::NT == 0 || v < C::NB)
          *reinterpret_cast<u32x4*>(Bs + (v / (BK / 4)) * LDB + (v % (BK / 4)) * 4) = rb[i];
      }
    } else {
      uint16_t* Ah = reinterpret_cast<uint16_t*>(st);
      uint16_t* Al = Ah + BM * LDA;
      uint16_t* Bh = reinterpret_cast<uint16_t*>(st + C::A_BYTES);
      uint16_t* Bl = Bh + BN * LDB;
#pragma unroll
      for (int i = 0; i < C::NVA; ++i) {
        const int v = tid + i * C::NT;
        if (C::NA % C::NT == 0 || v < C::NA) {
          const int q = v % (BK / 4);
          const int off = swz(v / (BK / 4), q >> 1) + (q & 1) * 4;
          uint32_t h0, h1, l0, l1;
          split_bf16x2(__uint_as_float(ra[i].x), __uint_as_float(ra[i].y), &h0, &l0);
          split_bf16x2(__uint_as_float(ra[i].z), __uint_as_float(ra[i].w), &h1, &l1);
          *reinterpret_cast<uint2*>(Ah + off) = uint2{h0, h1};
          *reinterpret_cast<uint2*>(Al + off) = uint2{l0, l1};
        }
      }
#pragma unroll
      for (int i = 0; i < C::NVB; ++i) {
        const int v = tid + i * C::NT;
        if (C::NB % C::NT == 0 || v < C::NB) {
          const int off = swz(v / (BK / 8), v % (BK / 8));
          *reinterpret_cast<u32x4*>(Bh + off) = rb[i];
          *reinterpret_cast<u32x4*>(Bl + off) = rbl[i];
        }
      }
    }
  };

  floatx4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int arow = wm * WROWS + (lane & 15);
  const int bcol = wn * C::WCOLS + (lane & 15);
  const int kq = lane >> 4;

  auto compute = [&](int buf) {
    const char* st = smem + buf * C::STAGE;
    if constexpr (MODE == MODE_F32) {
      const float* As = reinterpret_cast<const float*>(st);
      const float* Bs = reinterpret_cast<const float*>(st + C::A_BYTES);
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        float af[TM], bf[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = As[(arow + i * 16) * LDA + ks * 4 + kq];
#pragma unroll
        for (int j = 0; j < TN; ++j) bf[j] = Bs[(bcol + j * 16) * LDB + ks * 4 + kq];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else {
      const uint16_t* Ah = reinterpret_cast<const uint16_t*>(st);
      const uint16_t* Al = Ah + BM * LDA;
      const uint16_t* Bh = reinterpret_cast<const uint16_t*>(st + C::A_BYTES);
      const uint16_t* Bl = Bh + BN * LDB;
      bf16x8 ah[TM], al[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ah[i] = *reinterpret_cast<const bf16x8*>(Ah + swz(arow + i * 16, kq));
        al[i] = *reinterpret_cast<const bf16x8*>(Al + swz(arow + i * 16, kq));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(Bh + swz(bcol + j * 16, kq));
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(Bl + swz(bcol + j * 16, kq));
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
        }
      }
    }
  };

  if constexpr (JET && MODE != MODE_F32) {
    if (nkt > 0) {
      gload(0, R0);
      sstore(R0, 0);
    }
    if (nkt > 1) gload(1, R1);
    if (nkt > 2) gload(2, R0);
    __syncthreads();
    // unrolled by two so that the register stage of each step is static:
    // step s sits in LDS buffer s & 1; its registers were R(s & 1)
    for (int kt = 0; kt < nkt; kt += 2) {
      compute(0);
      if (kt + 1 < nkt) {
        sstore(R1, 1);
        if (kt + 3 < nkt) gload(kt + 3, R1);
      }
      __syncthreads();
      if (kt + 1 >= nkt) break;
      compute(1);
      if (kt + 2 < nkt) {
        sstore(R0, 0);
        if (kt + 4 < nkt) gload(kt + 4, R0);
      }
      __syncthreads();
    }
  } else {
    // value pass (short K loop, wide epilogue) and float32 operands (eight
    // MFMA k-steps per K step hide the loads): one register stage
    if (nkt > 0) {
      gload(0, R0);
      sstore(R0, 0);
    }
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
      if (kt + 1 < nkt) gload(kt + 1, R0);
      compute(kt & 1);
      if (kt + 1 < nkt) sstore(R0, (kt + 1) & 1);
      __syncthreads();
    }
  }

  // ---------------------------------------------------------------- epilogue
  // accumulator (i, j, r) of lane (kq, c) is tile row wm WROWS + 16 i + 4 kq + r,
  // tile column wn WCOLS + 16 j + c
  const int T = a.T;
  // output and residual never overlap (ping-pong activation buffers)
  float* __restrict__ out = reinterpret_cast<float*>(a.out);
  const float* __restrict__ res = reinterpret_cast<const float*>(a.a0);
  int gcol[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) gcol[j] = n0 + wn * C::WCOLS + j * 16 + (lane & 15);

  if constexpr (KIND == KIND_PLAIN) {
    // row g0 + 16 i + 4 kq + r of the wave: the lane offset carries 4 kq
    // rows and the column, the scalar offset 16 i + r rows, the immediate
    // 16 j columns; rows past the last one are out of range (dropped)
    const __amdgpu_buffer_rsrc_t rC = rsrc((float*)a.c + (size_t)g0 * a.ldc + n0 + wn * C::WCOLS);
    const int wr = wm * WROWS + kq * 4;
    const int voC = ((wr * a.ldc) + (lane & 15)) * 4;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      float old[4][TN];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int so = (i * 16 + r) * a.ldc * 4;
        const int vo = g0 + wr + i * 16 + r < a.n_groups ? voC : kOutOfRange;
#pragma unroll
        for (int j = 0; j < TN; ++j) old[r][j] = a.c_accum ? ldf(rC, vo + j * 64, so) : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int so = (i * 16 + r) * a.ldc * 4;
        const int vo = g0 + wr + i * 16 + r < a.n_groups ? voC : kOutOfRange;
#pragma unroll
        for (int j = 0; j < TN; ++j) stf(acc[i][j][r] + old[r][j], rC, vo + j * 64, so);
      }
    }
    return;
  }

  if constexpr (KIND == KIND_VALUE) {
    // value pass: every row is an electron.  Per 16-row tile the mean-field
    // and residual loads are issued together, then the results are stored.
    const float* __restrict__ Pv = (const float*)a.P;
    float* __restrict__ pre = a.pre_out;
    float bj[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) bj[j] = a.bias[gcol[j]];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      float pv[4][TN], rv[4][TN];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int g = g0 + wm * WROWS + i * 16 + kq * 4 + r;
        const bool ok = g < a.n_groups;
        const float* Prow = Pv + (size_t)(ok ? g / a.n_all : 0) * a.ldp;
        const float* rrow = res + (size_t)(ok ? g : 0) * a.lda0;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          pv[r][j] = ok ? Prow[gcol[j]] : 0.0f;
          rv[r][j] = (ok && a.res) ? rrow[gcol[j]] : 0.0f;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int g = g0 + wm * WROWS + i * 16 + kq * 4 + r;
        if (g >= a.n_groups) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int gc = gcol[j];
          const float u0 = acc[i][j][r] + pv[r][j] + bj[j];
          float y, dy;
          tanh_sech2f(u0, &y, &dy);
          if (pre) pre[(size_t)g * a.N + gc] = u0;
          out[(size_t)g * a.ldo + gc] = y + rv[r][j];
        }
      }
    }
    return;
  }

  // jet mode: the rows of this wave lie in one electron (rows_per % WROWS == 0).
  // Lane (kq, c) holds rows t = tw0 + 16 i + 4 kq + r of columns
  // wn WCOLS + 16 j + c: the (i, r) part of a row and the whole column base
  // are wave-uniform (scalar offsets and buffer bases), 4 kq rows and c
  // columns are the lane's own offset, and 16 j columns an immediate.
  const int wrow0 = wm * WROWS;
  const int e_loc = wrow0 / rows_per;
  const int tw0 = wrow0 - e_loc * rows_per;  // jet row of the wave's first row
  const int g = g0 + e_loc;
  const bool gval = g < a.n_groups;
  const int cw = n0 + wn * C::WCOLS;  // first column of the wave
  const size_t obase = (size_t)(gval ? g : 0) * rows_per;
  // the mean-field term has rows_per rows per walker (rows past T unused)
  const __amdgpu_buffer_rsrc_t rP =
      rsrc((const float*)a.P + (size_t)(gval ? g / a.n_all : 0) * rows_per * a.ldp + cw);
  const __amdgpu_buffer_rsrc_t rR = rsrc(res + obase * a.lda0 + cw);
  const __amdgpu_buffer_rsrc_t rO = rsrc(out + obase * a.ldo + cw);
  const int c = lane & 15;
  const int voP = (kq * 4 * a.ldp + c) * 4, voR = (kq * 4 * a.lda0 + c) * 4, voO = (kq * 4 * a.ldo + c) * 4;

  // pre-activation u = acc + P (the bias enters the value row below);
  // partial sums of the squared tangent rows 1 .. T-2.  Per 16-row tile all
  // P loads are issued together before any is used.
  float s2[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) s2[j] = 0.0f;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    float pv[4][TN];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int so = (tw0 + i * 16 + r) * a.ldp * 4;
#pragma unroll
      for (int j = 0; j < TN; ++j) pv[r][j] = ldf(rP, voP + j * 64, so);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = tw0 + i * 16 + kq * 4 + r;
      const bool live = t < a.T, tangent = (i + r > 0 || t >= 1) && t <= a.T - 2;  // t >= 16 i + r
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const float v = acc[i][j][r] + (live ? pv[r][j] : 0.0f);
        acc[i][j][r] = v;
        const float q = tangent ? v : 0.0f;
        s2[j] = fmaf(q, q, s2[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    s2[j] += __shfl_xor(s2[j], 16, 64);
    s2[j] += __shfl_xor(s2[j], 32, 64);
  }
  // cross-wave exchange (stage buffers are free after the main loop's last barrier)
  float* red = reinterpret_cast<float*>(smem);  // [WM][BN] partial sums
  float* val = red + WM * BN;                   // [WM][BN] value rows
  const int cl = wn * C::WCOLS + c;
  if (kq == 0) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      red[wm * BN + cl + j * 16] = s2[j];
      if (tw0 == 0) val[wm * BN + cl + j * 16] = acc[0][j][0];
    }
  }
  __syncthreads();
  const int wfirst = wm - tw0 / WROWS, wper = rows_per / WROWS;
  float y[TN], dy[TN], lapc[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    float ss = 0.0f;
    for (int w = wfirst; w < wfirst + wper; ++w) ss += red[w * BN + cl + j * 16];
    const float u0 = val[wfirst * BN + cl + j * 16] + a.bias[cw + c + j * 16];
    tanh_sech2f(u0, &y[j], &dy[j]);
    lapc[j] = -2.0f * y[j] * dy[j] * ss;
    if (a.pre_out && tw0 == 0 && kq == 0 && gval) a.pre_out[(size_t)g * a.N + cw + c + j * 16] = u0;
  }
  // spin-group tiles: every electron of the tile exists (the host checks
  // it); the output tile is staged in LDS, over the exchange buffer once
  // every wave has read it, in rows padded by 4 floats so that the four
  // 4-row lane groups of a store hit different banks
  constexpr int MF_LD = BN + 4;
  float* mfs = reinterpret_cast<float*>(smem);  // [BM][MF_LD]
  if constexpr (KIND == KIND_JET_MF) __syncthreads();
  else if (!gval) return;
  // per 16-row tile: all residual loads first, then the stores.  Row t
  // becomes y (t = 0), sech^2 u0 times its tangent (0 < t < T - 1), the
  // same plus the curvature term (t = T - 1), or zero (padding, t >= T),
  // plus the residual.
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    float rv[4][TN];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int so = (tw0 + i * 16 + r) * a.lda0 * 4;
#pragma unroll
      for (int j = 0; j < TN; ++j) rv[r][j] = a.res ? ldf(rR, voR + j * 64, so) : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = tw0 + i * 16 + kq * 4 + r;
      const bool live = t < a.T, last = t == a.T - 1;
      const bool first = i + r == 0 && t == 0, deriv = (i + r > 0 || t >= 1) && live;  // t >= 16 i + r
      const int so = (tw0 + i * 16 + r) * a.ldo * 4;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const float br = (first ? y[j] : (last ? lapc[j] : 0.0f)) + (live ? rv[r][j] : 0.0f);
        const float o = deriv ? fmaf(dy[j], acc[i][j][r], br) : br;  // selected: pad rows may hold anything
        stf(o, rO, voO + j * 64, so);
        if (first && a.val_out) a.val_out[(size_t)g * a.N + cw + c + j * 16] = o;
        if constexpr (KIND == KIND_JET_MF) mfs[(wrow0 + i * 16 + kq * 4 + r) * MF_LD + cl + j * 16] = o;
      }
    }
  }
  if constexpr (KIND == KIND_JET_MF) {
    // the group's mean of each output row: electrons in order, then times
    // 1 / WM (the summation order and scaling of the separate mean-field
    // pass, so both give the same bits)
    __syncthreads();
    const int wk = m_t >> 1, al = m_t & 1;  // tile m_t: spin group al of walker wk
    const float inv = 1.0f / (float)WM;
    float* dst = a.mf_out + (size_t)wk * rows_per * a.mf_ld + al * a.mf_half + n0;
    for (int q = tid; q < rows_per * (BN / 4); q += C::NT) {
      const int t = q / (BN / 4), c4 = (q % (BN / 4)) * 4;
      float4 sm = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < WM; ++e) {
        const float4 v = *reinterpret_cast<const float4*>(mfs + (e * rows_per + t) * MF_LD + c4);
        sm.x += v.x;
        sm.y += v.y;
        sm.z += v.z;
        sm.w += v.w;
      }
      *reinterpret_cast<float4*>(dst + (size_t)t * a.mf_ld + c4) = float4{sm.x * inv, sm.y * inv, sm.z * inv, sm.w * inv};
    }
  }
}

template <int MODE, int BM, int BN, int WM, int WN, int KIND>
static hipError_t run_layer(const JetGemmArgs& a, hipStream_t s) {
  using C = LayerCfg<MODE, BM, BN, WM, WN>;
  // the spin-group tiles stage their output tile in LDS
  constexpr int BYTES = KIND == KIND_JET_MF && BM * (BN + 4) * 4 > C::BYTES ? BM * (BN + 4) * 4 : C::BYTES;
  const int E = KIND == KIND_JET || KIND == KIND_JET_MF ? BM / a.rows_per : BM;
  const int n_mtiles = (a.n_groups + E - 1) / E;
  const int n_ntiles = (a.N + BN - 1) / BN;
  const int grid = ((n_mtiles + 7) / 8) * 8 * n_ntiles;
  // once per instantiation (a local static is initialised once, thread-safely)
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&layer_gemm_kernel<MODE, BM, BN, WM, WN, KIND>),
      hipFuncAttributeMaxDynamicSharedMemorySize, BYTES);
  if (attr != hipSuccess) return hipErrorInvalidValue;
  hipLaunchKernelGGL((layer_gemm_kernel<MODE, BM, BN, WM, WN, KIND>), dim3(grid), dim3(C::NT), BYTES, s, a,
                     n_mtiles, n_ntiles);
  return hipGetLastError();
}

// tile shapes: a row tile holds whole electrons and each wave's rows lie in
// one electron (value mode: one row per electron)
template <int MODE>
static hipError_t pick_layer(const JetGemmArgs& a, hipStream_t s) {
  if (a.rows_per == 1) {
    // value pass: 64-row tiles when 128-row tiles give the launch fewer
    // than about 1024 workgroups
    const int64_t nt = (a.N + 127) / 128;
    if ((int64_t)(a.n_groups + 127) / 128 * nt < 1024) return run_layer<MODE, 64, 128, 4, 2, KIND_VALUE>(a, s);
    return run_layer<MODE, 128, 128, 4, 2, KIND_VALUE>(a, s);
  }
  if (a.mf_out) {
    // one spin group of mf_na electrons per tile, one wave row per electron
    switch (a.mf_na) {
      case 1: return run_layer<MODE, 32, 128, 1, 2, KIND_JET_MF>(a, s);
      case 2: return run_layer<MODE, 64, 128, 2, 2, KIND_JET_MF>(a, s);
      case 3: return run_layer<MODE, 96, 128, 3, 2, KIND_JET_MF>(a, s);
      case 4: return run_layer<MODE, 128, 128, 4, 2, KIND_JET_MF>(a, s);
      case 5: return run_layer<MODE, 160, 128, 5, 2, KIND_JET_MF>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.rows_per == 96) return run_layer<MODE, 96, 128, 2, 4, KIND_JET>(a, s);
  if (a.rows_per == 32 || a.rows_per == 64 || a.rows_per == 128)
    return run_layer<MODE, 128, 128, 4, 2, KIND_JET>(a, s);
  return hipErrorInvalidValue;
}

// plain products whose A rows and output rows are both contiguous (no
// electron subsets), flattened to one row per (group, jet row)
bool layer_plain_supported(const JetGemmArgs& a) {
  const bool flat_a = a.rows_per == 1 || (a.n_sub == a.n_all && a.e_off == 0);
  return flat_a && a.c_nsub == 0 && a.N % 128 == 0 && a.ka0 % 32 == 0 && a.ka1 % 32 == 0 &&
         (int64_t)a.n_groups * a.rows_per < (1LL << 31) && a.ldc >= a.N;
}

hipError_t launch_layer_plain(int mode, const JetGemmArgs& a, hipStream_t s) {
  if (a.n_groups <= 0) return hipSuccess;
  if (!layer_plain_supported(a)) return hipErrorInvalidValue;
  JetGemmArgs f = a;
  if (a.rows_per > 1) {
    f.n_groups = a.n_groups * a.rows_per;
    f.n_sub = f.n_all = 1;
    f.e_off = 0;
  }
  f.rows_per = 1;
  f.T = 1;
  // 64-row tiles when 128-row tiles give the launch fewer than about 1024
  // workgroups (the per-walker products of the value passes: 0.068 -> 0.058
  // ms for the Ne-like mean-field products of one pass; the jet pass's keep
  // 128 rows, 0.46 against 0.59 ms)
  if ((int64_t)(f.n_groups + 127) / 128 * ((f.N + 127) / 128) < 1024)
    return mode == MODE_BF16X3 ? run_layer<MODE_BF16X3, 64, 128, 4, 2, KIND_PLAIN>(f, s)
                               : run_layer<MODE_F32, 64, 128, 4, 2, KIND_PLAIN>(f, s);
  return mode == MODE_BF16X3 ? run_layer<MODE_BF16X3, 128, 128, 4, 2, KIND_PLAIN>(f, s)
                             : run_layer<MODE_F32, 128, 128, 4, 2, KIND_PLAIN>(f, s);
}

bool layer_gemm_supported(const JetGemmArgs& a) {
  const int rp = a.rows_per;
  const bool tall = rp == 32 || rp == 64 || rp == 96 || rp == 128;
  return (rp == 1 ? a.T == 1 : tall && a.T <= rp) && a.N % 128 == 0 && a.ka0 % 32 == 0 && a.ka1 % 32 == 0;
}

bool layer_mf_supported(const JetGemmArgs& a) {
  return layer_gemm_supported(a) && a.rows_per == 32 && a.mf_na >= 1 && a.mf_na <= 5 && a.n_all == 2 * a.mf_na &&
         a.n_sub == a.n_all && a.e_off == 0 && a.n_groups % a.n_all == 0 && a.mf_ld % 4 == 0 && a.mf_half % 4 == 0 &&
         a.mf_half >= a.N && a.mf_ld >= 2 * a.mf_half;
}

hipError_t launch_layer_gemm(int mode, const JetGemmArgs& a, hipStream_t s) {
  if (a.n_groups <= 0) return hipSuccess;
  if (!layer_gemm_supported(a) || (a.mf_out && !layer_mf_supported(a))) return hipErrorInvalidValue;
  return mode == MODE_BF16X3 ? pick_layer<MODE_BF16X3>(a, s) : pick_layer<MODE_F32>(a, s);
}

}  // namespace fn
