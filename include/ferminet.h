/* ferminet.h -- C ABI of libferminet.so, the MI355X (gfx950) hot path of
 * FermiNet variational Monte Carlo.
 *
 * The library evaluates, batched over walkers, the FermiNet wavefunction of
 * Eqs. (4)-(5) of "Better, Faster Fermionic Neural Networks" (Spencer, Pfau,
 * Botev, Foulkes) with the two simplifications of its Section 3 (no
 * determinant weights omega_k; isotropic envelope exponents), its local
 * energy psi^-1 H psi for the Hamiltonian of Eq. (2), the gradient of
 * log|psi| with respect to the parameters (the quantity the energy
 * minimisation of Eq. (3) and KFAC consume), and Metropolis steps that
 * sample psi^2 (Eq. (3)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers unless marked HOST.  The caller
 *    owns every buffer, including the workspace; the library allocates no
 *    memory and keeps no state between calls.  Calls are asynchronous on
 *    the given stream (NULL = the default stream).  Calls that share one
 *    workspace must not overlap.
 *  - Arguments are validated on the host before anything is enqueued: on
 *    any status other than FN_OK nothing has been launched and no output
 *    has been touched.  FN_ERR_HIP reports a failed launch (outputs then
 *    undefined).
 *  - Atomic units: positions in bohr, energies in Hartree.
 *  - pos        [W][n][3] float32, electron positions, electrons of spin up
 *               first (indices 0..n_up-1), then spin down.
 *  - spins      HOST [n] int32, 0 = up, 1 = down.  Must equal n_up zeros
 *               followed by n_down ones (FN_ERR_SPINS otherwise).
 *  - nuc_pos    [N][3] float32 nuclear positions (fixed, Born-Oppenheimer).
 *  - nuc_charge [N] float32 nuclear charges Z_I.
 *  - params     [P] float32, the flat parameter vector in the layout below.
 *  - Numerical edge cases are not errors: an exact node (psi = 0) gives
 *    sign 0, log|psi| = -inf and a NaN local energy; an electron exactly on
 *    a nucleus or on another electron gives IEEE infinities.
 *
 * The network (permutation-equivariant one- and two-electron streams of the
 * original FermiNet, whose layer equations the paper does not restate):
 *    h^0_i  = concat_I (r_i - R_I, |r_i - R_I|)            (width 4N)
 *    h^0_ij = (r_i - r_j, |r_i - r_j|), zero at i == j    (width 4)
 *    for l = 0..L-1:
 *      hbar^a   = mean_{j of spin a} h^l_j      (zero vector if no such j)
 *      g^a_i    = mean_{j of spin a} h^l_ij     (includes j == i)
 *      f_i      = [h^l_i, hbar^up, hbar^down, g^up_i, g^down_i]
 *      h^{l+1}_i  = tanh(f_i V_l + b_l)   (+ h^l_i when the widths match)
 *      h^{l+1}_ij = tanh(h^l_ij W_l + c_l) (+ h^l_ij when the widths match),
 *                   for l = 0..L-2 only
 *    orbitals (Eq. (5), isotropic envelope, Section 3), for spin a,
 *    determinant k, orbital i, electron j of spin a:
 *      phi^{ka}_i(r_j) = (h^L_j . w_a[:, k n_a + i] + g_a[k n_a + i])
 *                        * sum_m pi_a[k n_a + i][m] exp(-|sigma_a[k n_a + i][m]| |r_j - R_m|)
 *    psi = sum_k det[phi^{k,up}_i(r_j)] det[phi^{k,down}_i(r_j)]   (Eq. (4))
 *
 * Flat parameter layout (row-major, [in][out] so that y = x W + b):
 *    for l in 0..L-1:  V_l [3 din_l + 2 ein_l][d1], then b_l [d1]
 *    for l in 0..L-2:  W_l [ein_l][d2],             then c_l [d2]
 *    for a in up, down: w_a [d1][K n_a], then g_a [K n_a]
 *    for a in up, down: pi_a [K n_a][N]
 *    for a in up, down: sigma_a [K n_a][N] (isotropic envelope), or
 *                       Sigma_a [K n_a][N][3][3] (full covariance, row-major)
 *    din_0 = 4N, ein_0 = 4; din_l = d1, ein_l = d2 for l > 0.
 *    The rows of V_l are ordered as f_i: [h_i | hbar^up | hbar^down |
 *    g^up_i | g^down_i].
 */
#ifndef FERMINET_H_
#define FERMINET_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FN_OK = 0,
  FN_ERR_NULL = 1,        /* a required pointer is NULL */
  FN_ERR_CONFIG = 2,      /* shapes out of range (see fn_config) */
  FN_ERR_SPINS = 3,       /* spins not n_up zeros followed by n_down ones */
  FN_ERR_WORKSPACE = 4,   /* workspace too small for one walker, or misaligned */
  FN_ERR_UNSUPPORTED = 5, /* valid request this build does not implement */
  FN_ERR_HIP = 6,         /* a HIP launch failed */
  FN_ERR_ARG = 7          /* other invalid scalar argument (W < 0, n_steps < 0, ...) */
} fn_status;

typedef enum {
  /* every stage in float32 (layer GEMMs on FP32 MFMA) */
  FN_PREC_FP32 = 0,
  /* one-electron layer GEMMs and their mean-field terms with
   * split-bfloat16 operands (hi and lo parts, three bfloat16 MFMA
   * products, float32 accumulation); the two-electron layers and the
   * orbital GEMM in float32 (the orbital product's rounding dominated the
   * local-energy error of the form); tanh, envelope and jet epilogues in
   * float32; LU, log-determinant, A^-1 contractions and the determinant
   * combination in float64.  The parameter gradient's cotangent products
   * through the one-electron and orbital layers use split-bfloat16
   * operands too; its reductions over walkers are float32 */
  FN_PREC_BF16 = 1,
  /* float32 network and orbitals, float64 determinants and combination */
  FN_PREC_FP32_FP64DET = 2,
  /* every stage in float64 (layer and orbital GEMMs on FP64 MFMA); inputs
   * are still the float32 arrays below, widened exactly.  Not available
   * for the parameter gradient (FN_ERR_UNSUPPORTED). */
  FN_PREC_FP64 = 3
} fn_precision;

typedef enum {
  /* exp(-|sigma_im| |r_j - R_m|): one exponent per orbital and nucleus,
   * the simplification of Section 3 */
  FN_ENV_ISOTROPIC = 0,
  /* exp(-|Sigma_im (r_j - R_m)|) with a 3x3 matrix Sigma_im (row-major,
   * applied to the column vector r_j - R_m): Eq. (5) as written */
  FN_ENV_FULL = 1
} fn_envelope;

/* Shapes.  Limits of this build: 1 <= n_elec <= 32 with any split
 * 0 <= n_up, n_down (n_up + n_down = n_elec), 1 <= n_nuc <= 32,
 * 1 <= n_layers <= 8, width1 in [32, 1024] and a multiple of 32,
 * 1 <= width2 <= 64, 1 <= n_det <= 64, and the two-electron stream of one
 * electron (8 sparse jet rows per pair) must fit in the 160 KiB of LDS of a compute unit
 * (FN_ERR_CONFIG otherwise). */
typedef struct {
  int32_t n_elec;    /* n = n_up + n_down */
  int32_t n_up;
  int32_t n_down;
  int32_t n_nuc;     /* N */
  int32_t n_layers;  /* L, one-electron layers (L-1 two-electron layers) */
  int32_t width1;    /* d1, one-electron stream width */
  int32_t width2;    /* d2, two-electron stream width */
  int32_t n_det;     /* K, determinants */
  int32_t precision; /* fn_precision */
  int32_t envelope;  /* fn_envelope */
  /* Local energy in the reduced-precision forms: the fraction f in [0, 1]
   * of walkers re-evaluated entirely in float64 (0: none; ignored by
   * FN_PREC_FP64 and by the other entry points).  Within each chunk of
   * the batch, in segments of at most 8192 walkers, the ceil(f * segment)
   * walkers with the largest error scale
   *   kappa max(1, |E_L|, |E_kin|) (1 + (u_det / u_orb) cond),
   * where kappa = max_k |P_k| / |psi| is the determinant-sum cancellation
   * (P_k = det^up_k det^down_k, Eq. (4); infinite at a node), E_L and E_kin
   * the reduced-precision local and kinetic energy, cond the largest
   * condition number cond_1 of the walker's orbital matrices, and
   * u_det / u_orb the unit roundoff of the determinant arithmetic over that
   * of the orbitals (2^-29 with the float64 determinants of float32
   * orbitals of FN_PREC_BF16 and FN_PREC_FP32_FP64DET, 1 in FN_PREC_FP32;
   * equal scales go to the smaller walker index, an undefined one first),
   * are gathered, evaluated again as FN_PREC_FP64 would, and
   * their sign, log|psi|, e_loc, e_kin and e_pot replace the
   * reduced-precision values.  Rounding errors of E_L are amplified by
   * kappa near a node of the determinant sum and, in the factorisation, by
   * the conditioning of the orbital matrices; only the kinetic term passes
   * through the network.  The scale ranks the walkers by their share of
   * the batch-mean error; the re-evaluation removes the dominant part of it
   * at a fixed cost. */
  float rescue_fraction;
} fn_config;

typedef struct {
  char name[16];  /* "V0", "b0", "W0", "c0", "w_orb0", "g_orb0", "pi0", "sigma1", ... */
  int64_t offset; /* in floats, from the start of params */
  int64_t rows;   /* first dimension (1 for vectors) */
  int64_t cols;   /* second dimension */
} fn_param_block;

typedef enum {
  FN_ENTRY_LOGPSI = 0,
  FN_ENTRY_LOCAL_ENERGY = 1,
  FN_ENTRY_GRAD_LOGPSI = 2,
  FN_ENTRY_MCMC = 3,
  FN_ENTRY_KFAC = 4,
  FN_ENTRY_KFAC_PRECONDITION = 5, /* chunk_walkers is ignored */
  FN_ENTRY_TRAIN = 6,             /* chunk_walkers is the batch size W (see vmc_train_step) */
  FN_ENTRY_LOCAL_ENERGY_GRADIENT = 7 /* vmc_local_energy_gradient in one pass of chunk_walkers */
} fn_entry;

/* Settings of one VMC iteration (vmc_train_step). */
typedef struct {
  int32_t mcmc_steps;    /* Metropolis steps before the evaluation, >= 0 */
  float mcmc_width;      /* proposal standard deviation (bohr) */
  uint64_t seed;         /* Philox key of the moves, as in vmc_mcmc_step */
  uint64_t counter;      /* step counter of the first move, as in vmc_mcmc_step */
  float learning_rate;   /* lr > 0 */
  float damping;         /* lambda > 0 of the KFAC direction */
  float norm_constraint; /* C of the step length; <= 0: no constraint */
  float factor_decay;    /* running average of the KFAC factors, in [0, 1]; 0 takes the batch's */
  float clip_scale;      /* s of the energy clipping; <= 0: no clipping */
  int32_t reserved;
} fn_train_options;

/* One dense layer's Kronecker factors in the output of ferminet_kfac_factors. */
typedef struct {
  char name[16];     /* "layer0".., "pair0".., "orbital0", "orbital1" */
  int64_t offset_A;  /* in floats: A, dim_A x dim_A row-major */
  int64_t offset_G;  /* in floats: G, dim_G x dim_G row-major */
  int32_t dim_A;     /* inputs + 1 (the bias input) */
  int32_t dim_G;     /* outputs */
  int32_t positions; /* positions per walker the layer is applied at */
  int32_t reserved;
} fn_kfac_block;

/* Human-readable text of a status code (static storage). */
const char* ferminet_status_string(int32_t status);

/* Number of float32 parameters P of the layout above, or -1 if cfg is
 * invalid. */
int64_t ferminet_param_count(const fn_config* cfg);

/* The parameter blocks in layout order.  Writes at most cap entries to out
 * (HOST) and the number of blocks to *n_out (HOST).  FN_ERR_ARG if cap is
 * too small (then *n_out holds the required count). */
fn_status ferminet_param_layout(const fn_config* cfg, fn_param_block* out, int32_t cap, int32_t* n_out);

/* Workspace bytes (*bytes, HOST) that let the given entry point process
 * chunk_walkers walkers in one pass.  Any workspace of at least
 * ferminet_workspace_bytes(cfg, 1, entry) bytes works: larger batches are
 * then processed in chunks of as many walkers as fit.  The workspace must
 * be 256-byte aligned. */
fn_status ferminet_workspace_bytes(const fn_config* cfg, int32_t chunk_walkers, int32_t entry, size_t* bytes);

/* sign(psi) and log|psi| of Eq. (4) for W walkers.
 *   sign   [W] float32 out: +1, -1, or 0 at an exact node
 *   logpsi [W] float32 out */
fn_status ferminet_logpsi(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                          const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                          float* logpsi, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ferminet_logpsi for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or sampling loops, harnesses that
 * forbid hipMalloc): the same computation, the same outputs bit for bit,
 * with the workspace taken from a 64 MiB device array inside the library
 * instead of a caller's buffer.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); the array is set up on the
 * call's first use on a device and held by that device until the process
 * ends.  The batch is processed in chunks of as many walkers as the 64 MiB
 * hold (about 1600 walkers of the Ne-like network); a network whose
 * one-walker workspace (ferminet_workspace_bytes(cfg, 1, FN_ENTRY_LOGPSI))
 * exceeds 64 MiB is rejected with FN_ERR_WORKSPACE before anything is
 * enqueued.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  FN_ERR_HIP if the
 * array's device address cannot be obtained.  Other arguments and errors
 * as ferminet_logpsi. */
fn_status ferminet_logpsi_noalloc(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                  const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                  float* logpsi, hipStream_t stream);

/* Local energy E_L = psi^-1 H psi with H of Eq. (2) for W walkers: the
 * kinetic part -1/2 sum_c [d^2_c log|psi| + (d_c log|psi|)^2] over all 3n
 * electron coordinates, from forward-mode jets (value, 3n tangents and
 * Laplacian) carried through every layer; the potential part from the
 * electron-electron, electron-nucleus and nucleus-nucleus Coulomb sums.
 * With cfg->rescue_fraction > 0 the walkers of largest error scale are
 * re-evaluated in float64 (see fn_config); the workspace then also holds
 * the float64 buffers of those walkers.
 *   sign, logpsi [W] out (as ferminet_logpsi)
 *   e_loc [W] out; e_kin, e_pot [W] out, each may be NULL */
fn_status ferminet_local_energy(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                float* logpsi, float* e_loc, float* e_kin, float* e_pot, void* workspace,
                                size_t workspace_bytes, hipStream_t stream);

/* Parameter gradient of log|psi| (Eq. (4)) from a hand-written adjoint
 * (values recomputed, no tangents stored): the derivative that the
 * gradient estimator of the energy of Eq. (3) and the KFAC statistics
 * consume.
 *   cotangent [W] float32 in, or NULL;
 *   grad, with a cotangent: [P] float32 out, in the parameter layout,
 *       grad[p] = sum_w cotangent[w] * d log|psi_w| / d theta_p;
 *   grad, with cotangent NULL: [W][P] float32 out, row w holding
 *       d log|psi_w| / d theta of walker w (W * P floats; the caller sizes
 *       it, e.g. 4096 x 688832 floats = 11.3 GB for the Ne-like network).
 * Each walker's sums run in a fixed order, so both forms are reproducible
 * run to run.  FN_ERR_NULL if grad is NULL; FN_ERR_UNSUPPORTED in the
 * FN_PREC_FP64 form.  With W = 0 the [P] form writes zeros and the [W][P]
 * form writes nothing. */
fn_status ferminet_grad_logpsi(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                               const float* nuc_pos, const float* nuc_charge, const float* params,
                               const float* cotangent, float* grad, void* workspace, size_t workspace_bytes,
                               hipStream_t stream);

/* VMC energy gradient estimator for Eq. (3), as the mean over the batch:
 *   grad[p] = (1/W) sum_w (E_L,w - mean E_L) d log|psi_w| / d theta_p
 * (the gradient of the energy itself is twice this).  e_stats (2 doubles,
 * device) receives the batch mean and the population variance of e_loc,
 * computed in float64.  Uses the FN_ENTRY_GRAD_LOGPSI workspace. */
fn_status vmc_energy_gradient(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                              const float* nuc_pos, const float* nuc_charge, const float* params,
                              const float* e_loc, double* e_stats, float* grad, void* workspace,
                              size_t workspace_bytes, hipStream_t stream);

/* Statistics of the Kronecker-factored approximate curvature (KFAC,
 * Martens and Grosse 2015), the optimiser the paper's introduction names,
 * for every dense layer of the network.  A layer with inputs a and
 * pre-activations z = a W + b applied at positions r of walker w (the n
 * electrons for the one-electron layers, whose input is
 * f_i = [h_i, hbar^up, hbar^down, g^up_i, g^down_i]; the n^2 electron pairs
 * (i n + j) for the two-electron layers; the n_a electrons of one spin for
 * the orbital layer of that spin, whose input is h^L_j) contributes
 *   A = sum_w c_w sum_r a~ a~^T,   a~ = [a; 1]
 *   G = sum_w c_w sum_r g g^T,     g = d log|psi_w| / d z_{w,r}
 * so that sum_w c_w sum_r a~ g^T is the gradient of sum_w c_w log|psi_w|
 * with respect to [W; b] (the weight block followed by its bias in the
 * parameter layout).  The envelope parameters (pi, sigma) are not dense
 * layers and have no factors.
 *   weights  [W] float32 in: c_w (negative values count as 0)
 *   factors  float32 out, ferminet_kfac_layout's total floats: each
 *            block's A then G (overwritten, not accumulated)
 * Runs the hand-written adjoint with cotangents sqrt(c_w), in the fp32 or
 * split-bf16 form (FN_ERR_UNSUPPORTED for FN_PREC_FP64).  Uses the
 * FN_ENTRY_KFAC workspace. */
fn_status ferminet_kfac_factors(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                const float* nuc_pos, const float* nuc_charge, const float* params,
                                const float* weights, float* factors, void* workspace, size_t workspace_bytes,
                                hipStream_t stream);

/* The blocks of ferminet_kfac_factors in output order: the one-electron
 * layers, the two-electron layers, then the orbital layers of the spins
 * that have electrons.  Writes at most cap entries to out (HOST), the
 * block count to *n_out and the total floats to *total (HOST); FN_ERR_ARG
 * if cap is too small. */
fn_status ferminet_kfac_layout(const fn_config* cfg, fn_kfac_block* out, int32_t cap, int32_t* n_out,
                               int64_t* total);

/* The KFAC step direction (Martens and Grosse 2015, factored Tikhonov
 * damping) from the factors of ferminet_kfac_factors: for every dense layer
 * with gradient block M = [W; b] ((dim_A) x (dim_G) floats at the weight
 * block's offset in the parameter layout, the bias row last),
 *   X = (A + pi s I)^-1 M (G + s / pi I)^-1,  s = sqrt(damping),
 *   pi = sqrt((tr A / dim_A) / (tr G / dim_G))  (1 if a trace is not positive)
 * computed in float64 (Cholesky factors of the damped factors, triangular
 * solves); the envelope parameters (pi, sigma), which belong to no dense
 * layer, keep their gradient.
 *   factors  [total] float32 in (ferminet_kfac_layout)
 *   grad     [P] float32 in; update [P] float32 out (may not alias grad)
 *   damping  lambda > 0 and finite, else FN_ERR_ARG
 * The factors must be positive semi-definite (as ferminet_kfac_factors
 * returns them); the damping then makes every Cholesky pivot positive.
 * Uses the FN_ENTRY_KFAC_PRECONDITION workspace. */
fn_status ferminet_kfac_precondition(const fn_config* cfg, const float* factors, const float* grad, float damping,
                                     float* update, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ferminet_local_energy followed by vmc_energy_gradient on its energies,
 * in one pass: the energy of Eq. (2) per walker and the gradient estimator
 * of Eq. (3),
 *   grad[p] = (1/W) sum_w (E_L,w - mean E_L) d log|psi_w| / d theta_p,
 * with e_stats (2 doubles, device) the batch mean and population variance
 * of e_loc.  The reverse pass reads the values of the local energy's own
 * jet pass (row 0 of every jet) instead of evaluating the network once
 * more.  Outputs and their precision as the two calls; cfg->rescue_fraction
 * as in ferminet_local_energy.  The single pass needs
 * ferminet_workspace_bytes(cfg, W, FN_ENTRY_LOCAL_ENERGY_GRADIENT); a smaller
 * workspace runs the two calls in turn (each in chunks).  W = 0 gives
 * FN_ERR_ARG, the FN_PREC_FP64 form FN_ERR_UNSUPPORTED. */
fn_status vmc_local_energy_gradient(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                    const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                    float* logpsi, float* e_loc, float* e_kin, float* e_pot, double* e_stats,
                                    float* grad, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* One iteration of the variational optimisation of E[E_L] under psi^2
 * (Eq. (3)) with KFAC (Martens and Grosse 2015), the optimiser the paper
 * names; the paper gives no settings, so they are arguments.  Walkers whose
 * local energy is not finite (an exact node of psi or coincident particles)
 * are left out of steps 3 and 4: W_f below counts the others, and the
 * statistics, the median and the clipping run over them only.  In order, on
 * the stream:
 *   1. log|psi| of the walkers under the current parameters, then
 *      options->mcmc_steps Metropolis moves (vmc_mcmc_step; noise and
 *      uniforms as there, both NULL or both given);
 *   2. the local energies e_loc [W] (float32 out; ferminet_local_energy in
 *      cfg's form, with cfg's float64 re-evaluation fraction);
 *   3. E~ = e_loc clipped to median +- s * mean|e_loc - median| (the median
 *      of an even count is the mean of the two middle values; no clipping
 *      for s <= 0) and the energy gradient
 *        g = 2 sum_w (E~_w - mean E~) / W_f d log|psi_w| / d theta;
 *   4. the KFAC factors of the batch (weights 1/W_f) and the running average
 *        factors <- decay factors + (1 - decay) batch factors
 *      (factors: [total] float32 in/out in ferminet_kfac_layout's layout;
 *      with decay = 0 its input is not read);
 *   5. the damped direction X (ferminet_kfac_precondition) and the step
 *        params <- params - lr c X,  c = min(1, sqrt(C / (lr^2 <X, g>)))
 *      (c = 1 for C <= 0 or <X, g> <= 0), params [P] float32 in/out.
 *   stats  [9] float64 DEVICE out: mean and population variance of e_loc,
 *          acceptance rate (accepted moves / (W mcmc_steps); 0 without
 *          moves), median, mean |e_loc - median|, mean E~, <X, g>, lr c,
 *          and the number of walkers left out (W - W_f).  With W_f = 0 the
 *          energy statistics are NaN, the gradient and the batch factors
 *          are zero and the parameters do not change.
 * W >= 1 (else FN_ERR_ARG); FN_ERR_UNSUPPORTED for FN_PREC_FP64.  Options
 * outside their ranges or not finite give FN_ERR_ARG.  The workspace holds
 * per-walker and per-parameter buffers for the whole batch followed by the
 * passes' own workspace: ferminet_workspace_bytes(cfg, W, FN_ENTRY_TRAIN)
 * runs every pass in one chunk; less works down to the passes' one-walker
 * chunks (FN_ERR_WORKSPACE otherwise, checked before anything is
 * enqueued). */
fn_status vmc_train_step(const fn_config* cfg, int32_t W, float* pos, const int32_t* spins, const float* nuc_pos,
                         const float* nuc_charge, float* params, float* factors, const fn_train_options* options,
                         const float* noise, const float* uniforms, float* e_loc, double* stats, void* workspace,
                         size_t workspace_bytes, hipStream_t stream);

/* n_steps Metropolis random-walk steps sampling psi^2 (Eq. (3)), all
 * electrons moved at once:
 *   x' = x + step_width * z,  z ~ N(0, I_{3n});
 *   accept iff log(u) < 2 (log|psi(x')| - log|psi(x)|), u ~ U(0,1),
 *   and psi(x') != 0.
 *   pos [W][n][3], logpsi [W], sign [W]  in/out: the current state; logpsi
 *       and sign must be those of pos on entry (ferminet_logpsi).
 *   n_accepted [W] int32 out: accepted moves of each walker in this call.
 *   noise [n_steps][W][3n], uniforms [n_steps][W]: supplied draws; both
 *       NULL draws them from Philox4x32-10 (Salmon et al., SC'11) as
 *       vmc_mcmc_noise documents, with step index counter + s. */
fn_status vmc_mcmc_step(const fn_config* cfg, int32_t W, float* pos, const int32_t* spins, const float* nuc_pos,
                        const float* nuc_charge, const float* params, float* logpsi, float* sign, int32_t n_steps,
                        float step_width, uint64_t seed, uint64_t counter, const float* noise,
                        const float* uniforms, int32_t* n_accepted, void* workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* The draws vmc_mcmc_step makes internally, for replay and testing.
 *   key     = (seed & 0xffffffff, seed >> 32); s = counter + step
 *   normals of walker w, coordinates 4b..4b+3: Philox4x32-10 of counter
 *           (w, b, s & 0xffffffff, s >> 32) gives words x0..x3;
 *           u_k = ((x_k >> 9) + 0.5) * 2^-23; Box-Muller on (u0, u1) and
 *           (u2, u3): z = sqrt(-2 ln u_a) (cos, sin)(2 pi u_b)
 *   uniform of walker w: word x0 of counter (w, 0x80000000, s lo, s hi),
 *           mapped the same way.
 *   noise [n_steps][W][3n] float32 out, uniforms [n_steps][W] float32 out */
fn_status vmc_mcmc_noise(int32_t W, int32_t n_elec, int32_t n_steps, uint64_t seed, uint64_t counter, float* noise,
                         float* uniforms, hipStream_t stream);

/* ---- diagnostics: per-stage device time ----
 * ferminet_stage_timing(1) makes every later launch record a pair of HIP
 * events on its stream (process-wide; it adds a small host overhead);
 * ferminet_stage_timing(0) stops it.  Either call discards pending records.
 * ferminet_stage_times waits for the recorded events, writes per-stage
 * totals in milliseconds and launch counts to total_ms[cap] and count[cap]
 * (HOST), clears the records and returns the number of stages (-1 if cap is
 * too small or a pointer is NULL).  ferminet_stage_name gives the stage
 * names (static storage). */
fn_status ferminet_stage_timing(int32_t enable);
int32_t ferminet_stage_times(double* total_ms, int32_t* count, int32_t cap);
const char* ferminet_stage_name(int32_t stage);

/* ---- execution options (process-wide) ----
 * FN_OPT_FUSED_MEANFIELD (default 1): where the layer shape allows it
 * (equal spin groups of at most 5 electrons, jets of at most 32 rows,
 * float32 and split-bf16 forms) the jet layer kernel also forms the spin
 * means of its output that the next layer reads (the mean field of Sec. 3),
 * instead of a separate pass over the layer output; 0 always runs the
 * separate pass.  Both give the same bits.  ferminet_set_option sets value
 * (0 or 1) for later calls and returns FN_ERR_ARG for an unknown option or
 * value; set it while no call is running. */
typedef enum { FN_OPT_FUSED_MEANFIELD = 1 } fn_option;
fn_status ferminet_set_option(int32_t option, int32_t value);

#ifdef __cplusplus
}
#endif

#endif /* FERMINET_H_ */
