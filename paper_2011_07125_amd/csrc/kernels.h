// Internal launch interface between the host orchestration (abi.cpp) and
// the HIP kernels of libferminet.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fn {

enum { EPI_PLAIN = 0, EPI_TANHJET = 1, EPI_ORBITAL = 2 };
// GEMM arithmetic: float32 MFMA, or three bfloat16 MFMA passes on operands
// split into hi + lo parts
enum { MODE_F32 = 0, MODE_BF16X3 = 1 };

// One MFMA GEMM over rows grouped by "electron" (rows_per rows each: the
// value row, the 3n tangent rows and the Laplacian row of a jet, padded),
// with a fused epilogue.  Group g of the GEMM reads memory group
//   mg = (g / n_sub) * n_all + e_off + (g % n_sub),  row mg * rows_per + t.
struct JetGemmArgs {
  const void* a0; int lda0; int ka0;  // A segment 0 (ka0 multiple of 32; elements)
  const void* a1; int lda1; int ka1;  // A segment 1 (ka1 multiple of 32, may be 0)
  const void* bt; int ldb;            // packed weights [N][ldb], k contiguous, ldb >= ka0 + ka1
  const void* bt_lo;                  // MODE_BF16X3: lo plane of the weights (bt holds the hi plane)
  int n_groups, rows_per, T;
  int n_sub, n_all, e_off;
  int N;
  // EPI_PLAIN: c[(og * rows_per + t) * ldc + col] (= or += when c_accum) with
  //   og = g, or (g / c_nsub) * c_nall + c_eoff + g % c_nsub when c_nsub > 0
  float* c; int ldc;
  int c_nsub, c_nall, c_eoff, c_accum;
  // EPI_TANHJET: out[(g * rows_per + t) * ldo + col] (activation type), with
  //   P[((g / n_all) * rows_per + t) * ldp + col] added to every row, bias on
  //   the value row, residual from segment 0 when res != 0; pre_out[g * N + col]
  //   receives the pre-activation of the value row when not NULL
  void* out; int ldo;
  const float* P; int ldp;
  const float* bias;
  int res;
  float* pre_out;
  // EPI_ORBITAL: phi[((w * K + k) * T + t) * n_sub^2 + j * n_sub + i] with
  //   w = g / n_sub, j = g % n_sub, col = k * n_sub + i
  //   or, when phi_M > 0 (matrix index fastest, for the small-matrix
  //   determinant kernel): phi[((t n_sub + j) n_sub + i) * phi_M + w * K + k]
  float* phi;
  int64_t phi_M;
  const float* pos; const float* nuc; int n_nuc; int n_elec;
  const float* g_orb; const float* pi; const float* sigma;
  float* u_out; float* env_out;  // value mode, optional: [w][K][j][i]
};

hipError_t launch_jet_gemm(int mode, int epi, const JetGemmArgs& a, hipStream_t s);
// full-width streaming kernel for the EPI_TANHJET layers (layer.hip)
bool layer_gemm_supported(const JetGemmArgs& a);
hipError_t launch_layer_gemm(int mode, const JetGemmArgs& a, hipStream_t s);

// ---- features and two-electron stream (features.hip)
// split: write bfloat16 hi planes at dst and lo planes at dst + plane (elements)
hipError_t launch_pack_weights(bool split, const float* params, void* dst, int64_t plane, const int64_t* plan,
                               int n_items, hipStream_t s);
hipError_t launch_features(bool bf16, const float* pos, const float* nuc, int W, int n, int N, int T, int Tp,
                           void* H0, int ldh, hipStream_t s);
struct TwoElecArgs {
  const float* pos;   // [W][n][3]
  const float* params;
  const int64_t* w_off;  // HOST array: offsets of W_l in params, l = 0..L-2
  const int64_t* c_off;  // HOST array: offsets of c_l
  int W, n, n_up, L, d2, T, Tp;
  void* G[8];         // G^l [(w n + i) Tp + t][ldg_l] (activation type)
  int ldg[8];
  float* h2_out[8];   // value mode, optional: h^l_ij [w][i][j][ein_l]
};
hipError_t launch_two_electron(bool bf16, const TwoElecArgs& a, hipStream_t s);
hipError_t launch_meanfield(bool bf16, const void* H, int ldh, int W, int n, int n_up, int Tp, int din_p, void* Hbar,
                            hipStream_t s);

// ---- determinants and combination (det.hip)
// D_a[(w K + k) * dstride + ...]: sign, log|det|, d_c (3n), q, lap  (jet mode)
//                                  sign, log|det|                      (value mode)
// matrices up to this size take the one-thread-per-matrix kernel, which
// expects the matrix-index-fastest layout of the orbital jets (phi_M = W K)
constexpr int DET_SMALL_MAX = 6;
bool det_uses_small(int na);
hipError_t launch_det(bool fp64, const float* phi, int W, int K, int na, int T, int n3, void* D, int dstride,
                      void* ainv, hipStream_t s);
struct CombineArgs {
  const void* D[2]; int dstride; int na[2];
  int W, K, n, n3, N, jet;
  const float* pos; const float* nuc; const float* Z;
  float* sign; float* logpsi; float* e_loc; float* e_kin; float* e_pot;
  void* rho;  // optional [W][K]: rho_k = P_k / psi (value mode, adjoint)
};
hipError_t launch_combine(bool fp64, const CombineArgs& a, hipStream_t s);

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
};
int atb_splits(int64_t R);
hipError_t launch_atb(const AtbArgs& a, hipStream_t s);
int rowsum_chunks(int64_t rows, int chunk);
// dst[c] += sum_r src[r * lds + c] in a fixed order (tmp: rowsum_chunks(rows, chunk) * cols floats)
hipError_t launch_rowsum_add(const float* src, int64_t rows, int cols, int64_t lds, float* tmp, float* dst,
                             int chunk, hipStream_t s);
hipError_t launch_adj_orbital_cot(bool fp64, const void* binv, const void* rho, const float* cot, const float* u,
                                  const float* env, int W, int K, int na, int ldu, float* cot_u, float* cot_env,
                                  hipStream_t s);
hipError_t launch_adj_env_grad(const float* cot_env, const float* pos, const float* nuc, const float* pi,
                               const float* sigma, int W, int K, int na, int j0, int n, int N, float* dpi,
                               float* dsigma, hipStream_t s);
hipError_t launch_adj_cp(const float* ch, const float* pre, int64_t total, float* cp, hipStream_t s);
hipError_t launch_adj_walker_sum(const float* cp, int W, int n, int cols, float* S, hipStream_t s);
hipError_t launch_adj_scatter_mf(const float* cmf, int W, int n, int n_up, int din, int half, float* ch, int ldh,
                                 hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
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
  float* part;                 // [W n][p2]
};
hipError_t launch_adj_two_electron(const Adj2eArgs& a, hipStream_t s);
hipError_t launch_energy_stats(const float* e, int W, double* stats, float* cot, hipStream_t s);
hipError_t launch_cot_from_stats(const float* e, int Wc, const double* stats, int W_total, float* cot, hipStream_t s);

}  // namespace fn
