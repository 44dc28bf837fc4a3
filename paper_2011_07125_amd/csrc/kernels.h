// Internal launch interface between the host orchestration (abi.cpp) and
// the HIP kernels of libferminet.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fn {

enum { EPI_PLAIN = 0, EPI_TANHJET = 1, EPI_ORBITAL = 2 };
// GEMM arithmetic: float32 MFMA, three bfloat16 MFMA passes on operands
// split into hi + lo parts, or float64 MFMA on float64 operands (then every
// activation, mean-field term, orbital jet and epilogue is float64 too);
// MODE_BF16X6 (orbital products of the jet GEMM only): float32 operands
// split into three bfloat16 parts each (all 24 significand bits) and the
// six products of parts whose orders sum to at most 2^-16, by six bfloat16
// MFMAs into a float32 accumulator: float32 accuracy at about 3/8 of the
// matrix-core time of float32 MFMA
enum { MODE_F32 = 0, MODE_BF16X3 = 1, MODE_F64 = 2, MODE_BF16X6 = 3 };

// One MFMA GEMM over rows grouped by "electron" (rows_per rows each: the
// value row, the 3n tangent rows and the Laplacian row of a jet, padded),
// with a fused epilogue.  Group g of the GEMM reads memory group
//   mg = (g / n_sub) * n_all + e_off + (g % n_sub),  row mg * rows_per + t.
struct JetGemmArgs {
  const void* a0; int lda0; int ka0;  // A segment 0 (ka0 multiple of 32; elements)
  const void* a1; int lda1; int ka1;  // A segment 1 (ka1 multiple of 32, may be 0)
  const void* bt; int ldb;            // packed weights [N][ldb], k contiguous, ldb >= ka0 + ka1 (mode's type)
  const void* bt_lo;                  // MODE_BF16X3: lo plane of the weights (bt holds the hi plane)
  int n_groups, rows_per, T;
  int n_sub, n_all, e_off;
  int N;
  // EPI_PLAIN: c[(og * rows_per + t) * ldc + col] (= or += when c_accum) with
  //   og = g, or (g / c_nsub) * c_nall + c_eoff + g % c_nsub when c_nsub > 0
  void* c; int ldc;                   // float32 (float64 in MODE_F64)
  int c_nsub, c_nall, c_eoff, c_accum;
  // EPI_TANHJET: out[(g * rows_per + t) * ldo + col] (activation type), with
  //   P[((g / n_all) * rows_per + t) * ldp + col] added to every row, bias on
  //   the value row, residual from segment 0 when res != 0; pre_out[g * N + col]
  //   receives the pre-activation of the value row when not NULL
  void* out; int ldo;
  const void* P; int ldp;             // float32 (float64 in MODE_F64)
  const float* bias;
  int res;
  float* pre_out;
  float* val_out;  // optional (float32 modes): the value row of out, compact: val_out[g * N + col]
  // optional (float32 modes, layer_mf_supported): the spin means of out,
  //   mf_out[((g / n_all) * rows_per + t) * mf_ld + a * mf_half + col] =
  //   mean over the mf_na electrons of spin a of the walker of out's row t
  //   (n_all = 2 mf_na electrons per walker, spin up first)
  float* mf_out; int mf_ld; int mf_half; int mf_na;
  // EPI_ORBITAL: phi[((w * K + k) * T + t) * n_sub^2 + j * n_sub + i] with
  //   w = g / n_sub, j = g % n_sub, col = k * n_sub + i
  //   or, when phi_M > 0 (matrix index fastest, for the small-matrix
  //   determinant kernel): phi[((t n_sub + j) n_sub + i) * phi_M + w * K + k]
  void* phi;                          // float32 (float64 in MODE_F64)
  int64_t phi_M;
  const float* pos; const float* nuc; int n_nuc; int n_elec;
  const float* g_orb; const float* pi; const float* sigma;
  int env_full;  // sigma holds 3x3 matrices [col][m][3][3] (full covariance envelope)
  float* u_out; float* env_out;  // value mode, optional: [w][K][j][i]
};

hipError_t launch_jet_gemm(int mode, int epi, const JetGemmArgs& a, hipStream_t s);
// full-width streaming kernel for the EPI_TANHJET layers (layer.hip), and
// the same kernel with a plain epilogue for EPI_PLAIN products over
// contiguous rows
bool layer_gemm_supported(const JetGemmArgs& a);
// the jet layer can also write the spin means of its output (mf_out): equal
// spin groups of at most 5 electrons, 32 jet rows, all electrons in the rows
bool layer_mf_supported(const JetGemmArgs& a);
hipError_t launch_layer_gemm(int mode, const JetGemmArgs& a, hipStream_t s);
bool layer_plain_supported(const JetGemmArgs& a);
hipError_t launch_layer_plain(int mode, const JetGemmArgs& a, hipStream_t s);

// ---- features and two-electron stream (features.hip)
// mode MODE_F32 / MODE_F64: float32 / float64 weights; MODE_BF16X3:
// bfloat16 hi planes at dst and lo planes at dst + plane (elements)
hipError_t launch_pack_weights(int mode, const float* params, void* dst, int64_t plane, const int64_t* plan,
                               int n_items, hipStream_t s);
// f64: float64 arithmetic and storage (otherwise float32).  The input
// jets H0 [W n][Tp][ldh] and their spin means Hbar [W Tp][2 ldh] (the first
// n_up electrons of a walker are spin up)
// h0_val, hbar_val (optional, float32): row 0 (the values) of H0 and of
// Hbar, [W n][ldh] and [W][2 ldh]
hipError_t launch_features(bool f64, const float* pos, const float* nuc, int W, int n, int n_up, int N, int T,
                           int Tp, void* H0, int ldh, void* Hbar, hipStream_t s, float* h0_val = nullptr,
                           float* hbar_val = nullptr);
struct TwoElecArgs {
  const float* pos;   // [W][n][3]
  const float* params;
  const int64_t* w_off;  // HOST array: offsets of W_l in params, l = 0..L-2
  const int64_t* c_off;  // HOST array: offsets of c_l
  int W, n, n_up, L, d2, T, Tp;
  void* G[8];         // G^l [(w n + i) Tp + t][ldg_l] (float32, or float64 with f64)
  int ldg[8];
  float* h2_out[8];   // optional, float32: the values h^l_ij [w][i][j][ein_l] (both modes)
  float* g_val_out[8];  // optional, float32: row 0 (the values) of G^l, [w n + i][ldg_l]
};
hipError_t launch_two_electron(bool f64, const TwoElecArgs& a, hipStream_t s);
// electrons per workgroup of the two-electron stream (0: does not fit in LDS)
int two_electron_per_block(int n, int d2, int T, int scalar_bytes);
hipError_t launch_meanfield(bool f64, const void* H, int ldh, int W, int n, int n_up, int Tp, int din_p, void* Hbar,
                            hipStream_t s);

// ---- determinants and combination (det.hip)
// D_a[(w K + k) * dstride + ...]: sign, log|det|, d_c (3n), q, lap, cond_1(A)  (jet mode)
//                                  sign, log|det|                      (value mode)
// matrices up to this size take the one-thread-per-matrix kernel, which
// expects the matrix-index-fastest layout of the orbital jets (phi_M = W K)
constexpr int DET_SMALL_MAX = 6, DET_MID_MAX = 16;
bool det_uses_small(int na);
// phi64: the orbital jets are float64 (requires fp64)
hipError_t launch_det(bool fp64, const void* phi, bool phi64, int W, int K, int na, int T, int n3, void* D,
                      int dstride, void* ainv, hipStream_t s);
struct CombineArgs {
  const void* D[2]; int dstride; int na[2];
  int W, K, n, n3, N, jet;
  const float* pos; const float* nuc; const float* Z;
  float* sign; float* logpsi; float* e_loc; float* e_kin; float* e_pot;
  void* rho;  // optional [W][K]: rho_k = P_k / psi (value mode, adjoint)
  float* rescue_key;  // optional [W] (jet mode): log(kappa max(1, |E_L|, |E_kin|) (1 + cond_weight cond))
                      // with kappa = max_k |P_k| / |psi| and cond the largest cond_1 of the
                      // walker's orbital matrices (+inf at a node, NaN propagates)
  float cond_weight;  // unit roundoff of the determinant arithmetic over that of the orbitals
};
hipError_t launch_combine(bool fp64, const CombineArgs& a, hipStream_t s);

// ---- float64 re-evaluation of selected walkers (rescue.hip)
// idx[seg * k_seg + r], r < k: the k walkers of segment seg (walkers
// seg * seg_len ..) with the largest key, in increasing index order (NaN keys
// count as +inf, ties to the smaller index); k = k_seg in every full segment
// and k_last in the last one; seg_len <= 8192
hipError_t launch_select_top(const float* key, int W, int seg_len, int k_seg, int k_last, int32_t* idx,
                             hipStream_t s);
hipError_t launch_gather_walkers(const float* pos, const int32_t* idx, int R, int n3, float* pos_r, hipStream_t s);
// out[idx[r]] = src[r] for each non-NULL (out, src) pair
hipError_t launch_scatter_results(const int32_t* idx, int R, float* const* outs, const float* const* srcs, int n_out,
                                  hipStream_t s);

// ---- Metropolis (mcmc.hip)
hipError_t launch_mcmc_noise(int W, int n, int n_steps, uint64_t seed, uint64_t counter, float* noise,
                             float* uniforms, hipStream_t s);
// walkers of a chunk draw with their index in the whole batch (w_base + w)
hipError_t launch_propose_offset(const float* pos, float* prop, int W, int n3, float width, uint64_t seed,
                                 uint64_t step, const float* noise, uint32_t w_base, hipStream_t s);
hipError_t launch_accept_offset(float* pos, const float* prop, float* logpsi, float* sign, const float* lp_new,
                                const float* sg_new, int32_t* n_acc, int W, int n3, uint64_t seed, uint64_t step,
                                const float* uniforms, int first, uint32_t w_base, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);

// ---- adjoint (adjoint.hip)
// part[split][k][nn] = sum over the rows r of the split of
//   X[mr * ldx + xcol + k] * Y[r * ldy + nn],  k < K1, nn < N,
// mr = r, or (r / xs) * xa + xe + r % xs when xs > 0
struct AtbArgs {
  const float* X; int64_t ldx; int xcol; int xs, xa, xe;
  const float* Y; int64_t ldy;
  int64_t R; int K1, N;
  float* part;
  // sym: X and Y are the same columns (K1 == N); only the output tiles on
  // and above the diagonal (64 x 64) are formed
  int sym;
  // per-walker mode (dst != NULL): the rows are cut into R / seg segments of
  // seg rows (one walker each) and segment q adds its product into
  // dst + q * dst_ld (part and sym unused)
  float* dst = nullptr;
  int64_t dst_ld = 0;
  int seg = 0;
  // split-bfloat16 products (the bf16 form): each operand x = hi + lo in
  // bfloat16, x y ~ hi hi + hi lo + lo hi on v_mfma_f32_16x16x32_bf16
  int bf16 = 0;
};
int atb_splits(int64_t R, int K1, int N);   // partials written by launch_atb
int64_t atb_part_floats(int K1max, int Nmax);  // bound on splits * K1 * N over K1 <= K1max, N <= Nmax
hipError_t launch_atb(const AtbArgs& a, hipStream_t s);
int rowsum_chunks(int64_t rows, int chunk);
// dst[c] += sum_r src[r * lds + c] in a fixed order (tmp: rowsum_chunks(rows, chunk) * cols floats)
// sym_n > 0: cols = sym_n^2 (an atb partial of a symmetric product); the
// columns in 64 x 64 tiles below the diagonal are neither read nor written
hipError_t launch_split_planes(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t s);
hipError_t launch_rowsum_add(const float* src, int64_t rows, int cols, int64_t lds, float* tmp, float* dst,
                             int chunk, hipStream_t s, int sym_n = 0);
// per walker: dst[q * dst_ld + c] += sum_{r < seg} src[(q seg + r) * lds + c]
// for the R / seg segments q (one walker each)
hipError_t launch_rowsum_seg_add(const float* src, int64_t rows, int seg, int cols, int64_t lds, float* dst,
                                 int64_t dst_ld, hipStream_t s);
// M[r][c] = M[c][r] for the 64 x 64 tiles below the diagonal of an n x n matrix
hipError_t launch_sym_mirror(float* M, int n, hipStream_t s);
hipError_t launch_adj_orbital_cot(bool fp64, const void* binv, const void* rho, const float* cot, const float* u,
                                  const float* env, int W, int K, int na, int ldu, float* cot_u, float* cot_env,
                                  hipStream_t s);
// dpi, dsigma += the envelope-parameter gradient summed over the W walkers,
// or (walker_ld > 0) per walker at dpi + w walker_ld, dsigma + w walker_ld.
// part (part_floats floats, or NULL): scratch for the partial sums of the
// walker rows' splits
hipError_t launch_adj_env_grad(const float* cot_env, const float* pos, const float* nuc, const float* pi,
                               const float* sigma, bool full, int W, int K, int na, int j0, int n, int N, float* dpi,
                               float* dsigma, hipStream_t s, int64_t walker_ld = 0, float* part = nullptr,
                               int64_t part_floats = 0);
// the cotangent pass of a one-electron layer (W walkers of n electrons,
// rows of cols): CH += the mean-field cotangent CMF [W][2 cols] / n_a (when
// cmf is not NULL), CP = CH sech^2(PRE), S[w] = sum over the walker's
// electrons of CP
hipError_t launch_adj_cp_sum(float* ch, const float* pre, const float* cmf, int W, int n, int n_up, int cols,
                             float* cp, float* S, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
// dst[r * ldd + c] = src[r * lds + c] for r < rows, c < cols
hipError_t launch_copy_rows(const float* src, int64_t lds, float* dst, int64_t ldd, int64_t rows, int cols,
                            hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s);
struct Adj2eArgs {
  const float* params;
  int64_t w_off[8], c_off[8];  // offsets of W_l, c_l in params
  int64_t p_off[8];            // offsets of W_l within the partial row
  int64_t p2;                  // floats per partial row (all two-electron parameters)
  const float* h2[8];          // h^l_ij values [w n + i][n][ein_l], l < L-1
  const float* CG[8];          // cot g^l_i [w n + i][ldcg_l] (columns a ein_l + o)
  int ldcg[8];
  int W, n, n_up, L, d2;
  float* part;                 // [adj_two_electron_rows(W, n, d2)][ldp]
  int64_t ldp;                 // floats per partial row (>= p2)
  // KFAC statistics (kfac != 0): per partial row, for each layer l < L-1,
  // the (ein_l + 1)^2 block sum_pairs c_w a~ a~^T (a~ = [h_ij; 1]) at column
  // k_off[l], then the d2^2 block sum_pairs cp cp^T; sc[w] = sqrt(c_w)
  int kfac;
  int64_t k_off[8];
  const float* sc;
};
hipError_t launch_adj_two_electron(const Adj2eArgs& a, hipStream_t s);
// rows of parameter partials the two-electron backward writes (<= W n)
int adj_two_electron_rows(int W, int n, int d2);
hipError_t launch_energy_stats(const float* e, int W, double* stats, float* cot, hipStream_t s);
// KFAC statistics: sc[w] = sqrt(max(c_w, 0)); the inputs a~ of a dense
// layer materialised row by row and scaled by sc[w]:
//   one-electron layer: out[w n + i] = sc[w] [h_i (din), hbar^up_w (din),
//     hbar^down_w (din), g_i (2 ein), 1, 0 ...]   (ldo columns)
//   orbitals of one spin: out[w n_a + j] = sc[w] [h^L_{j0 + j} (d1), 1, 0 ...]
hipError_t launch_kfac_sqrt_weights(const float* c, int Wc, float* sc, hipStream_t s);
hipError_t launch_kfac_aug_layer(const float* H, int ldh, int din, const float* Hbar, int dinp, const float* G,
                                 int ldg, int ein, const float* sc, int Wc, int n, int ldo, float* out, hipStream_t s);
hipError_t launch_kfac_aug_orbital(const float* H, int ldh, int d1, const float* sc, int Wc, int n, int j0, int na,
                                   int ldo, float* out, hipStream_t s);

// ---- KFAC step direction (kfac.hip), float64
constexpr int KFAC_MAX_BLOCKS = 32, KFAC_MAX_MATS = 64;
struct KfacPrepArgs {
  int nb;                                           // dense layers
  int64_t offA[KFAC_MAX_BLOCKS], offG[KFAC_MAX_BLOCKS];  // in the factors (floats)
  int64_t offP[KFAC_MAX_BLOCKS];                    // [weights; bias] in the parameter layout
  int64_t offLA[KFAC_MAX_BLOCKS], offLG[KFAC_MAX_BLOCKS], offY[KFAC_MAX_BLOCKS], offYt[KFAC_MAX_BLOCKS];  // in S
  int64_t offIA[KFAC_MAX_BLOCKS], offIG[KFAC_MAX_BLOCKS];  // inverse diagonal tiles of the factors, in S
  int dA[KFAC_MAX_BLOCKS], dG[KFAC_MAX_BLOCKS];
  const float* factors;
  const float* grad;
  float* update;
  double* S;
  double sqrt_damping;
};
// matrices mat: n x n at S + off (row-major); the inverses of the
// triangular factor's diagonal tiles (ceil(n / 32) tiles of 32 x 32) at
// S + offI; right-hand sides n x m at S + offB with an n x m scratch at S + offZ
struct SpdBatch {
  int nm;
  int n[KFAC_MAX_MATS], m[KFAC_MAX_MATS];
  int64_t off[KFAC_MAX_MATS], offI[KFAC_MAX_MATS], offB[KFAC_MAX_MATS], offZ[KFAC_MAX_MATS];
};
hipError_t launch_kfac_prep(const KfacPrepArgs& a, hipStream_t s);       // damped factors, M
hipError_t launch_spd_cholesky(const SpdBatch& bt, double* S, hipStream_t s);  // in place, lower
hipError_t launch_spd_solve(const SpdBatch& bt, double* S, hipStream_t s);     // B <- (L L^T)^-1 B
hipError_t launch_kfac_transpose(const KfacPrepArgs& a, hipStream_t s);  // Y -> Yt
hipError_t launch_kfac_write(const KfacPrepArgs& a, hipStream_t s);      // Yt^T -> update
hipError_t launch_cot_from_stats(const float* e, int Wc, const double* stats, int W_total, float* cot, hipStream_t s);

// ---- one VMC iteration (train.hip)
// Over the W_f walkers with a finite E: stats[0..5] = mean E, variance E,
// acceptance (sum n_acc / (W n_steps), all walkers), median, mean
// |E - median|, mean of the clipped energies; stats[8] = W - W_f; e_clip =
// E clipped to median +- clip_scale * that deviation (E itself if
// clip_scale <= 0 or E is not finite); cot = 2 (e_clip - mean e_clip) / W_f
// and wts = 1 / W_f for finite E, both 0 otherwise
hipError_t launch_train_energy_stats(const float* e, const int32_t* n_acc, int W, int n_steps, double clip_scale,
                                     float* e_clip, float* cot, float* wts, double* stats, hipStream_t s);
// y = a x + b y (y = a x when b = 0)
hipError_t launch_lincomb(float* y, const float* x, float a, float b, int64_t n, hipStream_t s);
// stats[6] = <x, g>, stats[7] = lr min(1, sqrt(C / (lr^2 <x, g>))) (lr when
// C <= 0 or <x, g> <= 0); part: 256 doubles of scratch
hipError_t launch_step_length(const float* x, const float* g, int64_t n, double lr, double norm_constraint,
                              double* part, double* stats, hipStream_t s);
// theta -= stats[7] x
hipError_t launch_apply_step(float* theta, const float* x, int64_t n, const double* stats, hipStream_t s);

}  // namespace fn
