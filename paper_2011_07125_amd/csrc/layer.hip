// One-electron layer GEMM with the tanh-jet epilogue, sized for the tall,
// skinny products of the jet algebra: rows = walkers x electrons x jet rows
// (millions), K = d1 + 2 d2, N = d1.
//
// Per layer the arithmetic intensity is K N / (2 (K + N)) flop per byte of
// float32 activations (about 50 for K = 320, N = 256), far below the ridge
// of the bfloat16 matrix cores, so the kernel is organised around HBM
// streaming rather than MFMA reuse:
//  * a workgroup (512 threads for 128-row tiles) owns BM rows (whole
//    electrons, and a whole number of waves per electron) x BN = 128
//    columns; the column tiles of one row tile are issued back to back on
//    the same XCD, so the repeated read of the activations is served by
//    that XCD's L2;
//  * for small atoms (equal spin groups of at most five electrons, 32 jet
//    rows) a tile is instead one spin group of one walker, one wave row per
//    electron, and the tile's mean of its output rows is written too: the
//    mean field the next layer reads (Sec. 3) is formed from the tile in LDS
//    instead of by a separate pass that reads every layer output again.
//    These workgroups (one per CU) loop over tiles, and the loads of the
//    next tile's first K steps are in flight during each epilogue;
//  * in the split-bfloat16 form each activation element is split into hi/lo
//    parts once, by the thread that stages it into LDS (hardware
//    round-to-nearest-even conversion); the bfloat16 tiles are stored without
//    padding under an XOR swizzle of 16-byte chunks (conflict-free fragment
//    reads), so two stages take 64 KiB and two workgroups share a CU.  The
//    loads run two K steps ahead in registers; every step issues the same
//    loads (selects, out-of-range offsets past the end), so that the
//    compiler's wait counts leave them in flight;
//  * the epilogue does not stage the tile in LDS (but for the copy the
//    spin-group tiles sum into the means): per column, the jet rows of
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
#include <algorithm>

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
// a wave-uniform pointer the compiler cannot prove uniform (else a buffer
// access through it becomes a loop over the lanes' distinct values)
__device__ inline const void* uniform(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  // the builtin returns a signed int: widen through uint32_t (no sign extension)
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const void*>((hi << 32) | lo);
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

// waves per SIMD the register budget is sized for: two 8-wave workgroups
// per CU, or small workgroups; the looping spin-group tiles run one
// workgroup per CU (their LDS), so their waves share the four SIMDs
constexpr int layer_waves_per_eu(int waves, bool one_per_cu) {
  return one_per_cu ? (waves + 3) / 4 : (waves >= 8 ? 4 : 2);
}

// the split-bfloat16 spin-group tiles loop over tiles (blockIdx.x, then
// every gridDim.x-th one): the loads of the next tile's first K steps are in
// flight while this tile's epilogue runs.  Other kinds and float32 operands
// take one tile per workgroup.
template <int MODE, int KIND>
constexpr bool layer_loops() { return KIND == KIND_JET_MF && MODE != MODE_F32; }

template <int MODE, int BM, int BN, int WM, int WN, int KIND>
__global__ __launch_bounds__(64 * WM * WN)
__attribute__((amdgpu_waves_per_eu(layer_waves_per_eu(WM * WN, layer_loops<MODE, KIND>()), 8))) void
layer_gemm_kernel(JetGemmArgs a, int n_mtiles, int n_ntiles) {
  constexpr bool JET = KIND == KIND_JET || KIND == KIND_JET_MF;
  constexpr bool LOOP = layer_loops<MODE, KIND>();
  using C = LayerCfg<MODE, BM, BN, WM, WN>;
  constexpr int BK = C::BK, LDA = C::LDA, LDB = C::LDB, TM = C::TM, TN = C::TN, WROWS = C::WROWS;
  // the epilogue's LDS: after the stage buffers when the next tile's first
  // step is staged during the epilogue, else over them
  constexpr int EPI = LOOP ? 2 * C::STAGE : 0;
  extern __shared__ __attribute__((aligned(16))) char smem[];

  // tile t (row tile m, column tile n): the column tiles of a row tile are
  // 8 tiles apart, so that they run on the same XCD; the last 8 row tiles
  // may include padding (m >= n_mtiles)
  const int n_tiles = (n_mtiles + 7) / 8 * 8 * n_ntiles;
  auto tile_m = [&](int t) { return (t / (8 * n_ntiles)) * 8 + (t % 8); };
  auto tile_n = [&](int t) { return (t / 8) % n_ntiles; };
  const int t0 = blockIdx.x;
  if (!LOOP && tile_m(t0) >= n_mtiles) return;
  // K steps go in pairs across tiles (two register stages): with an odd
  // count each workgroup takes one tile (the host launches one per tile)
  const int nkt = (a.ka0 + a.ka1) / BK;
  const int tstep = LOOP && nkt % 2 == 0 ? gridDim.x : n_tiles;  // n_tiles: no second tile
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int rows_per = JET ? a.rows_per : 1;
  const int E = BM / rows_per;  // electrons per row tile
  // first jet row of row tile m (row numbers grow with the electron index)
  auto tile_row0 = [&](int m) {
    const int g0 = m * E;
    const int q0 = g0 / a.n_sub, m0 = g0 - q0 * a.n_sub;
    return ((long)q0 * a.n_all + a.e_off + m0) * rows_per;
  };

  // A loader: 8 float4 per 32-wide tile row, at byte offsets from the
  // tile's first row, computed for the first tile.  The spin-group tiles
  // (whole groups of consecutive electrons, all present) share them.
  const int g0 = LOOP ? 0 : tile_m(t0) * E;
  const int q0 = g0 / a.n_sub, m0 = g0 - q0 * a.n_sub;
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
  // B loader: columns n0 .. n0 + BN - 1 all exist (N is a multiple of BN)
  constexpr int ESZ = MODE == MODE_F32 ? 4 : 2;
  constexpr int VPR = MODE == MODE_F32 ? BK / 4 : BK / 8;  // 16-byte vectors per B row
  int voffB[C::NVB];
#pragma unroll
  for (int i = 0; i < C::NVB; ++i) {
    const int v = tid + i * C::NT;
    voffB[i] = C::NB % C::NT == 0 || v < C::NB ? ((v / VPR) * a.ldb + (v % VPR) * (16 / ESZ)) * ESZ : kOutOfRange;
  }

  // register stages of the loads: NS in the split-bfloat16 jet pass (the
  // loads of K steps k+1 .. k+NS are in flight while step k is multiplied),
  // one elsewhere
  struct Regs {
    u32x4 ra[C::NVA];
    u32x4 rb[C::NVB], rbl[MODE == MODE_F32 ? 1 : C::NVB];
  };

  // K-step order: the segment-1 steps, the segment-0 steps outside the
  // tile's residual columns, then the residual columns [n0, n0 + BN) of
  // segment 0 last, so that the epilogue's residual loads find them in L2
  const int nk0 = a.ka0 / BK, n1 = nkt - nk0;
  auto ktile = [&](int kt, int n0) {
    const int r0 = a.res ? n0 / BK : nk0;
    const int nres = a.res ? (n0 + BN <= a.ka0 ? BN / BK : 0) : 0;
    const int k = kt - n1, nout = nk0 - nres;
    const int t = k >= nout ? r0 + (k - nout) : (k >= r0 ? k + nres : k);
    return kt < n1 ? nk0 + kt : t;
  };
  // the loads are issued in K-step order over the workgroup's tiles; the
  // cursor holds the next one's tile (iteration c_lt: live, column base,
  // first row) and K step
  int c_lt = 0, c_lk = 0, c_n0 = 0;
  bool c_live = false;
  long c_row0 = 0;
  auto set_tile = [&](int lt) {
    const int t = t0 + lt * tstep;
    c_live = t < n_tiles && tile_m(t) < n_mtiles;
    const int tt = c_live ? t : t0;
    c_n0 = tile_n(tt) * BN;
    c_row0 = LOOP || lt == 0 ? tile_row0(tile_m(tt)) : c_row0;
  };
  // every call issues the same loads, whatever the step: the segment is
  // picked by selects, and a step of a tile that does not exist reads out
  // of range (zeros, no memory access).  With the same number of loads on
  // every path the compiler's wait counts keep the later stages in flight
  // instead of draining them at each LDS store.
  set_tile(0);
  // the first tile's bases (a single-tile workgroup's only ones)
  auto a0_base = [&](long row0) { return (const float*)a.a0 + row0 * a.lda0; };
  auto a1_base = [&](long row0) {
    return a.ka1 > 0 ? (const float*)a.a1 + row0 * a.lda1 : (const float*)a.a0;
  };
  auto b_base = [&](const void* bt, int n0) { return uniform((const char*)bt + (size_t)n0 * a.ldb * ESZ); };
  const float* const pA0f = a0_base(c_row0);
  const float* const pA1f = a1_base(c_row0);
  const __amdgpu_buffer_rsrc_t rBf = rsrc(b_base(a.bt, c_n0));
  const __amdgpu_buffer_rsrc_t rBlf = rsrc(MODE == MODE_F32 ? a.bt : b_base(a.bt_lo, c_n0));
  const int n0f = c_n0;
  auto gload = [&](Regs& R) {
    // single-tile workgroups: the steps past the last one are dead
    const bool live = LOOP ? c_live : c_lk < nkt;
    const int kb = ktile(LOOP || live ? c_lk : 0, LOOP ? c_n0 : n0f) * BK;
    const bool s0 = kb < a.ka0;
    const float* pa = LOOP ? (s0 ? a0_base(c_row0) : a1_base(c_row0)) : (s0 ? pA0f : pA1f);
    const __amdgpu_buffer_rsrc_t rA = rsrc(uniform(pa));
    const int soA = (s0 ? kb : kb - a.ka0) * 4;
    const int dead = live ? 0 : kOutOfRange;  // or-ed into the lane offsets
#pragma unroll
    for (int i = 0; i < C::NVA; ++i)
      R.ra[i] = __builtin_amdgcn_raw_buffer_load_b128(rA, (s0 ? voff0[i] : voff1[i]) | dead, soA, 0);
    const __amdgpu_buffer_rsrc_t rB = LOOP ? rsrc(b_base(a.bt, c_n0)) : rBf;
    const __amdgpu_buffer_rsrc_t rBl = LOOP ? rsrc(MODE == MODE_F32 ? a.bt : b_base(a.bt_lo, c_n0)) : rBlf;
#pragma unroll
    for (int i = 0; i < C::NVB; ++i) {
      R.rb[i] = __builtin_amdgcn_raw_buffer_load_b128(rB, voffB[i] | dead, kb * ESZ, 0);
      if constexpr (MODE != MODE_F32) R.rbl[i] = __builtin_amdgcn_raw_buffer_load_b128(rBl, voffB[i] | dead, kb * ESZ, 0);
    }
    if constexpr (LOOP) {
      if (++c_lk == nkt) {
        c_lk = 0;
        set_tile(++c_lt);
      }
    } else {
      ++c_lk;
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
  auto zero_acc = [&]() {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  };
  zero_acc();
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

  // ---------------------------------------------------------------- epilogue
  auto epilogue = [&](int t) {
    const int m_t = tile_m(t), g0 = m_t * E, n0 = tile_n(t) * BN;
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
    // cross-wave exchange (stage buffers are free after the main loop's last
    // barrier), unless one wave holds the electron's whole jet: then its
    // sums are complete and its value row is in lane group 0 (the same sums,
    // so the same bits)
    float* red = reinterpret_cast<float*>(smem + EPI);  // [WM][BN] partial sums
    float* val = red + WM * BN;                   // [WM][BN] value rows
    const int cl = wn * C::WCOLS + c;
    const int wfirst = wm - tw0 / WROWS, wper = rows_per / WROWS;
    const bool whole = wper == 1;
    if (!whole) {
      if (kq == 0) {
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          red[wm * BN + cl + j * 16] = s2[j];
          if (tw0 == 0) val[wm * BN + cl + j * 16] = acc[0][j][0];
        }
      }
      __syncthreads();
    }
    float y[TN], dy[TN], lapc[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      float ss = 0.0f;
      if (whole) ss += s2[j];
      else
        for (int w = wfirst; w < wfirst + wper; ++w) ss += red[w * BN + cl + j * 16];
      const float vrow = whole ? __shfl(acc[0][j][0], c, 64) : val[wfirst * BN + cl + j * 16];
      const float u0 = vrow + a.bias[cw + c + j * 16];
      tanh_sech2f(u0, &y[j], &dy[j]);
      lapc[j] = -2.0f * y[j] * dy[j] * ss;
      if (a.pre_out && tw0 == 0 && kq == 0 && gval) a.pre_out[(size_t)g * a.N + cw + c + j * 16] = u0;
    }
    // spin-group tiles: every electron of the tile exists (the host checks
    // it); the output tile is staged in LDS, over the exchange buffer once
    // every wave has read it, unpadded: column c of row R sits at
    // c ^ 16 ((R >> 2) & 3), so that the four 4-row lane groups of a store
    // hit different banks (and a 160-row tile takes 80 KiB, two per CU)
    float* mfs = reinterpret_cast<float*>(smem + EPI);  // [BM][BN], swizzled
    if constexpr (KIND == KIND_JET_MF) {
      if (!whole) __syncthreads();
    }
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
          if constexpr (KIND == KIND_JET_MF) mfs[(wrow0 + i * 16 + kq * 4 + r) * BN + ((cl + j * 16) ^ (kq << 4))] = o;
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
          const float4 v = *reinterpret_cast<const float4*>(mfs + (e * rows_per + t) * BN + (c4 ^ ((t & 12) << 2)));
          sm.x += v.x;
          sm.y += v.y;
          sm.z += v.z;
          sm.w += v.w;
        }
        *reinterpret_cast<float4*>(dst + (size_t)t * a.mf_ld + c4) = float4{sm.x * inv, sm.y * inv, sm.z * inv, sm.w * inv};
      }
    }
  };

  if constexpr (JET && MODE != MODE_F32) {
    constexpr int NS = 2;
    static_assert(NS % 2 == 0, "a group of NS steps starts in LDS buffer 0");
    Regs R[NS];
    if (nkt > 0) {
      gload(R[0]);
      sstore(R[0], 0);
    }
#pragma unroll
    for (int u = 1; u <= NS; ++u) gload(R[u % NS]);
    __syncthreads();
    // groups of NS steps, unrolled so that the register stage of each step
    // is static (step k sits in LDS buffer k & 1, its registers were
    // R[k % NS]); no exit inside a group, so that every path round the loop
    // issues the same loads.  A workgroup loops over tiles only when
    // nkt % NS == 0, so that the next tile's steps continue the pattern.
    // Stores of a stage of no tile write zeros into a buffer that is not
    // read again.
    auto ksteps = [&]() {
      int kt = 0;
      for (; kt + NS <= nkt; kt += NS) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
          compute(u & 1);
          sstore(R[(u + 1) % NS], (u + 1) & 1);
          gload(R[(u + 1) % NS]);
          __syncthreads();
          // keep the next step's conversions after its loads' wait
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int u = 0; u + 1 < NS; ++u) {
        if (kt + u < nkt) {
          compute(u & 1);
          sstore(R[(u + 1) % NS], (u + 1) & 1);
          __syncthreads();
        }
      }
    };
    if constexpr (LOOP) {
      for (int t = t0; t < n_tiles; t += tstep) {
        ksteps();
        if (tile_m(t) < n_mtiles) epilogue(t);
        zero_acc();
      }
    } else {
      ksteps();
      epilogue(t0);
    }
  } else {
    Regs R0;
    // value pass (short K loop, wide epilogue) and float32 operands (eight
    // MFMA k-steps per K step hide the loads): one register stage
    if (nkt > 0) {
      gload(R0);
      sstore(R0, 0);
    }
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
      if (kt + 1 < nkt) gload(R0);
      compute(kt & 1);
      if (kt + 1 < nkt) sstore(R0, (kt + 1) & 1);
      __syncthreads();
    }
    epilogue(t0);
  }
}

template <int MODE, int BM, int BN, int WM, int WN, int KIND>
static hipError_t run_layer(const JetGemmArgs& a, hipStream_t s) {
  using C = LayerCfg<MODE, BM, BN, WM, WN>;
  constexpr bool LOOP = layer_loops<MODE, KIND>();
  // the spin-group tiles stage their output tile in LDS: after the stage
  // buffers when looping (they hold the next tile's first step meanwhile),
  // else over them
  constexpr int EPI_BYTES = BM * BN * 4 > C::RED_BYTES ? BM * BN * 4 : C::RED_BYTES;
  constexpr int BYTES = LOOP                    ? 2 * C::STAGE + EPI_BYTES
                        : KIND == KIND_JET_MF ? (EPI_BYTES > C::BYTES ? EPI_BYTES : C::BYTES)
                                              : C::BYTES;
  const int E = KIND == KIND_JET || KIND == KIND_JET_MF ? BM / a.rows_per : BM;
  const int n_mtiles = (a.n_groups + E - 1) / E;
  const int n_ntiles = (a.N + BN - 1) / BN;
  const int n_tiles = ((n_mtiles + 7) / 8) * 8 * n_ntiles;
  auto kern = &layer_gemm_kernel<MODE, BM, BN, WM, WN, KIND>;
  // once per instantiation (a local static is initialised once, thread-safely)
  static const hipError_t attr =
      hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, BYTES);
  if (attr != hipSuccess) return hipErrorInvalidValue;
  int grid = n_tiles;
  if (LOOP && (a.ka0 + a.ka1) / C::BK % 2 == 0) {
    // as many workgroups as are resident at once, in multiples of 8 (one
    // per XCD), each looping over tiles (the kernel's condition)
    static const int per_cu = [&]() {
      int n = 0;
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, C::NT, BYTES) == hipSuccess && n > 0 ? n : 1;
    }();
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return hipErrorInvalidValue;
    const int resident = std::max(8, n_cu * per_cu / 8 * 8);
    grid = std::min(n_tiles, resident);
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::NT), BYTES, s, a, n_mtiles, n_ntiles);
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
  return (rp == 1 ? a.T == 1 : tall && a.T <= rp) && a.N % 128 == 0 && a.ka0 > 0 && a.ka0 % 32 == 0 &&
         a.ka1 % 32 == 0;
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
