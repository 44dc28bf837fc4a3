// Host side of libferminet: argument validation, the workspace plan, walker
// chunking and the launch sequence of every entry point of ferminet.h.
// Everything here is bookkeeping; all arithmetic of the method runs in the
// HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/ferminet.h"
#include "common.h"
#include "kernels.h"

namespace fn {

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
  fn_config cfg;
  int n, nu, nd, N, L, d1, d2, K, n3;
  bool bf16, fp64, f64;
  bool env_full;  // full-covariance envelope (3x3 Sigma per orbital and nucleus)
  int mode;       // GEMM arithmetic (MODE_*)
  float rescue;   // fraction of each chunk re-evaluated in float64 (local energy)
  size_t act;     // bytes per activation element
  int din[8], ein[8], dinp[8], gwp[8];
  int64_t offV[8], offb[8], offW2[8], offc2[8], offw[2], offg[2], offpi[2], offsg[2], P;
  // packed weights (elements, activation type)
  int64_t pk_main[8], pk_mf[8], pk_orb[2], pk_total;
  int ld_main[8], ld_mf[8];
  int na(int a) const { return a == 0 ? nu : nd; }
};

static fn_status make_plan(const fn_config* c, Plan& p) {
  if (!c) return FN_ERR_NULL;
  p.cfg = *c;
  p.n = c->n_elec;
  p.nu = c->n_up;
  p.nd = c->n_down;
  p.N = c->n_nuc;
  p.L = c->n_layers;
  p.d1 = c->width1;
  p.d2 = c->width2;
  p.K = c->n_det;
  if (p.nu < 0 || p.nd < 0 || p.nu + p.nd != p.n || p.n < 1 || p.n > 32 || p.nu > 32 || p.nd > 32) return FN_ERR_CONFIG;
  if (p.N < 1 || p.N > 32 || p.L < 1 || p.L > 8 || p.K < 1 || p.K > 64) return FN_ERR_CONFIG;
  if (p.d1 < 32 || p.d1 > 1024 || p.d1 % 32 != 0 || p.d2 < 1 || p.d2 > 64) return FN_ERR_CONFIG;
  if (c->precision != FN_PREC_FP32 && c->precision != FN_PREC_BF16 && c->precision != FN_PREC_FP32_FP64DET &&
      c->precision != FN_PREC_FP64)
    return FN_ERR_CONFIG;
  if (!(c->rescue_fraction >= 0.0f && c->rescue_fraction <= 1.0f)) return FN_ERR_CONFIG;
  if (c->envelope != FN_ENV_ISOTROPIC && c->envelope != FN_ENV_FULL) return FN_ERR_CONFIG;
  p.env_full = c->envelope == FN_ENV_FULL;
  p.bf16 = c->precision == FN_PREC_BF16;
  p.f64 = c->precision == FN_PREC_FP64;
  p.fp64 = c->precision != FN_PREC_FP32;
  p.mode = p.f64 ? MODE_F64 : p.bf16 ? MODE_BF16X3 : MODE_F32;
  p.rescue = p.f64 ? 0.0f : c->rescue_fraction;
  // activations are float32 in HBM, float64 in the float64 form
  p.act = p.f64 ? 8 : 4;
  // the two-electron stream keeps one electron's 8-row pair jets in LDS
  // (also in float64 when walkers are re-evaluated)
  if (two_electron_per_block(p.n, p.d2, 3 * p.n + 2, (int)p.act) < 1) return FN_ERR_CONFIG;
  if (p.rescue > 0.0f && two_electron_per_block(p.n, p.d2, 3 * p.n + 2, 8) < 1) return FN_ERR_CONFIG;
  p.n3 = 3 * p.n;
  int64_t off = 0;
  for (int l = 0; l < p.L; ++l) {
    p.din[l] = l == 0 ? 4 * p.N : p.d1;
    p.ein[l] = l == 0 ? 4 : p.d2;
    p.dinp[l] = round_up(p.din[l], 32);
    p.gwp[l] = round_up(2 * p.ein[l], 32);
    p.offV[l] = off;
    off += (int64_t)(3 * p.din[l] + 2 * p.ein[l]) * p.d1;
    p.offb[l] = off;
    off += p.d1;
  }
  for (int l = 0; l + 1 < p.L; ++l) {
    p.offW2[l] = off;
    off += (int64_t)p.ein[l] * p.d2;
    p.offc2[l] = off;
    off += p.d2;
  }
  for (int a = 0; a < 2; ++a) {
    p.offw[a] = off;
    off += (int64_t)p.d1 * p.K * p.na(a);
    p.offg[a] = off;
    off += (int64_t)p.K * p.na(a);
  }
  for (int a = 0; a < 2; ++a) {
    p.offpi[a] = off;
    off += (int64_t)p.K * p.na(a) * p.N;
  }
  for (int a = 0; a < 2; ++a) {
    p.offsg[a] = off;
    off += (int64_t)p.K * p.na(a) * p.N * (p.env_full ? 9 : 1);
  }
  p.P = off;
  // packed weights, each block 256-byte aligned
  int64_t pk = 0;
  const int64_t al = 256 / (int64_t)p.act;
  for (int l = 0; l < p.L; ++l) {
    p.ld_main[l] = p.dinp[l] + p.gwp[l];
    p.pk_main[l] = pk;
    pk += (int64_t)p.d1 * p.ld_main[l];
    pk = (pk + al - 1) / al * al;
    p.ld_mf[l] = 2 * p.dinp[l];
    p.pk_mf[l] = pk;
    pk += (int64_t)p.d1 * p.ld_mf[l];
    pk = (pk + al - 1) / al * al;
  }
  for (int a = 0; a < 2; ++a) {
    p.pk_orb[a] = pk;
    pk += (int64_t)p.K * p.na(a) * p.d1;
    pk = (pk + al - 1) / al * al;
  }
  p.pk_total = pk;
  return FN_OK;
}

// the packing plan: [dst_off, N, ldb, k0, len0, src0, k1, len1, src1, src_ld, transpose]
static int pack_plan(const Plan& p, std::vector<int64_t>& it) {
  it.clear();
  auto add = [&](int64_t dst, int64_t N, int64_t ldb, int64_t k0, int64_t l0, int64_t s0, int64_t k1, int64_t l1,
                 int64_t s1, int64_t sld) {
    int64_t v[11] = {dst, N, ldb, k0, l0, s0, k1, l1, s1, sld, 1};
    it.insert(it.end(), v, v + 11);
  };
  for (int l = 0; l < p.L; ++l) {
    const int din = p.din[l], ein = p.ein[l];
    // [h_i | g^up_i | g^down_i] rows of V_l
    add(p.pk_main[l], p.d1, p.ld_main[l], 0, din, p.offV[l], p.dinp[l], 2 * ein, p.offV[l] + (int64_t)3 * din * p.d1,
        p.d1);
    // [hbar^up | hbar^down] rows of V_l
    add(p.pk_mf[l], p.d1, p.ld_mf[l], 0, din, p.offV[l] + (int64_t)din * p.d1, p.dinp[l], din,
        p.offV[l] + (int64_t)2 * din * p.d1, p.d1);
  }
  for (int a = 0; a < 2; ++a)
    if (p.na(a) > 0) add(p.pk_orb[a], (int64_t)p.K * p.na(a), p.d1, 0, p.d1, p.offw[a], 0, 0, 0, (int64_t)p.K * p.na(a));
  return (int)(it.size() / 11);
}

// ----------------------------------------------------------- workspace
// bytes of the packed weights: the blocks in the arithmetic's type (two
// bfloat16 planes in the split form) and, in the split form, float32 copies
// of the orbital blocks at the same element offsets
static size_t pk_bytes(const Plan& p) { return (size_t)p.pk_total * p.act + (p.bf16 ? (size_t)p.pk_total * 4 : 0); }

enum Mode { VALUE = 0, JET = 1 };
enum Stage {
  ST_PACK, ST_FEATURES, ST_TWO_E, ST_MEANFIELD, ST_GEMM_MF, ST_GEMM_LAYER, ST_GEMM_ORB, ST_DET, ST_COMBINE,
  ST_PROPOSE, ST_ACCEPT, ST_ADJ_FWD, ST_ADJ_DET, ST_ADJ_ORB, ST_ADJ_LAYERS, ST_ADJ_TWO_E, ST_ADJ_REDUCE,
  ST_GEMM_LAYER_VALUE, ST_RESCUE, ST_KFAC, ST_TRAIN, ST_GEMM_LAYER_MF, ST_COUNT
};

struct Bufs {
  void* pk;
  void* H0;
  void* G[8];
  void* Ha;
  void* Hb;
  void* Hbar;
  void* Pm;      // mean-field terms (activation type)
  void* phi[2];  // orbital jets (activation type)
  void* D[2];
  float* rkey;   // rescue key per walker (local energy with re-evaluation), else NULL
  float* prop;
  float* lp_new;
  float* sg_new;
  int T, Tp, dstride;
};

struct Carver {
  char* base;
  size_t used;
  void* take(size_t bytes) {
    void* p = base ? base + used : nullptr;
    used += align256(bytes);
    return p;
  }
};

// per-chunk forward buffers; returns bytes used from the carver
static void carve_forward(const Plan& p, Mode m, int64_t Wc, Carver& cv, Bufs& b, bool mcmc) {
  b.T = m == JET ? 3 * p.n + 2 : 1;
  b.Tp = m == JET ? round_up(b.T, 32) : 1;
  b.dstride = m == JET ? p.n3 + 5 : 2;
  const int64_t rows = Wc * p.n * b.Tp;
  b.H0 = cv.take((size_t)rows * p.dinp[0] * p.act);
  for (int l = 0; l < p.L; ++l) b.G[l] = cv.take((size_t)rows * p.gwp[l] * p.act);
  b.Ha = cv.take((size_t)rows * p.d1 * p.act);
  b.Hb = cv.take((size_t)rows * p.d1 * p.act);
  int dmax = 0;
  for (int l = 0; l < p.L; ++l) dmax = std::max(dmax, p.dinp[l]);
  b.Hbar = cv.take((size_t)Wc * b.Tp * 2 * dmax * p.act);
  b.Pm = cv.take((size_t)Wc * b.Tp * p.d1 * p.act);
  const size_t rb = p.fp64 ? 8 : 4;
  for (int a = 0; a < 2; ++a) {
    b.phi[a] = cv.take((size_t)Wc * p.K * b.T * p.na(a) * p.na(a) * p.act);
    b.D[a] = cv.take((size_t)Wc * p.K * b.dstride * rb);
  }
  b.rkey = (m == JET && p.rescue > 0.0f) ? (float*)cv.take((size_t)Wc * 4) : nullptr;
  if (mcmc) {
    b.prop = (float*)cv.take((size_t)Wc * p.n3 * 4);
    b.lp_new = (float*)cv.take((size_t)Wc * 4);
    b.sg_new = (float*)cv.take((size_t)Wc * 4);
  } else {
    b.prop = b.lp_new = b.sg_new = nullptr;
  }
}

// ------------------------------------------------------ adjoint buffers
struct AdjBufs {
  float* H[9];      // values of h^l, l = 0..L ([Wc n][dinp_0] then [Wc n][d1])
  float* PRE[9];    // pre-activations of layer l output, l = 1..L
  float* G[8];      // g^l values [Wc n][gwp_l]
  float* Hbar[8];   // [Wc][2 dinp_l]
  float* h2[8];     // pair values h^l_ij, l < L-1: [Wc n][n][ein_l]
  float* Pm;        // [Wc][d1]
  float* phi[2];
  float* u[2];
  float* env[2];
  void* binv[2];
  void* D[2];
  void* rho;
  float* sign;
  float* logpsi;
  float* CH;  // cotangents of a layer's output, then of its input (in place)
  float* CP;
  float* S;
  float* CMF;
  float* CG[8];
  float* cot_u[2];
  float* cot_env[2];
  float* part;
  int64_t part_n;  // floats of part
  float* tmp;
  float* part2;
  float* wo[2];     // orbital weights w_a, columns padded to ldu (float32)
  uint16_t* pw = nullptr;  // split form: bfloat16 hi plane of the parameters, then the lo plane at pw_lo
  int64_t pw_lo = 0;
  uint16_t* wo_pl[2] = {nullptr, nullptr};  // split form: hi then lo plane of wo[a] (d1 ldu each)
  float* cot;       // [Wc]
  int ldu;
  int64_t p2;       // two-electron parameters in all
  // KFAC statistics (FN_ENTRY_KFAC only)
  float* Faug;      // [R][ldf] scaled inputs a~ of one dense layer
  int ldf;
  float* sc;        // [Wc] sqrt(c_w)
  int64_t kcols;    // KFAC columns of a two-electron partial row
  int64_t ldp2;     // floats per two-electron partial row (p2 + kcols)
};

static constexpr int kRowChunk = 64;

// ------------------------------------------------------------ KFAC layout
// the dense layers: one-electron layers, two-electron layers, orbitals of
// each spin that has electrons; each block's A then G in the output
struct KfacBlk {
  char name[16];
  int kind, layer, dA, dG, npos;
  int64_t offA, offG;
};
static std::vector<KfacBlk> kfac_blocks(const Plan& p, int64_t* total) {
  std::vector<KfacBlk> v;
  int64_t off = 0;
  auto add = [&](const char* nm, int kind, int layer, int dA, int dG, int npos) {
    KfacBlk k;
    memset(&k, 0, sizeof(k));
    snprintf(k.name, sizeof(k.name), "%s", nm);
    k.kind = kind;
    k.layer = layer;
    k.dA = dA;
    k.dG = dG;
    k.npos = npos;
    k.offA = off;
    off += (int64_t)dA * dA;
    k.offG = off;
    off += (int64_t)dG * dG;
    v.push_back(k);
  };
  char nm[16];
  for (int l = 0; l < p.L; ++l) {
    snprintf(nm, sizeof(nm), "layer%d", l);
    add(nm, 0, l, 3 * p.din[l] + 2 * p.ein[l] + 1, p.d1, p.n);
  }
  for (int l = 0; l + 1 < p.L; ++l) {
    snprintf(nm, sizeof(nm), "pair%d", l);
    add(nm, 1, l, p.ein[l] + 1, p.d2, p.n * p.n);
  }
  for (int a = 0; a < 2; ++a)
    if (p.na(a) > 0) {
      snprintf(nm, sizeof(nm), "orbital%d", a);
      add(nm, 2, a, p.d1 + 1, p.K * p.na(a), p.na(a));
    }
  if (total) *total = off;
  return v;
}

static void carve_adjoint(const Plan& p, int64_t Wc, Carver& cv, AdjBufs& b, bool kfac = false) {
  const int64_t R = Wc * p.n;
  const size_t rb = p.fp64 ? 8 : 4;
  int dmax = 0;
  for (int l = 0; l < p.L; ++l) dmax = std::max(dmax, p.dinp[l]);
  b.ldu = round_up(p.K * std::max(p.nu, p.nd), 32);
  for (int l = 0; l <= p.L; ++l) b.H[l] = (float*)cv.take((size_t)R * (l == 0 ? p.dinp[0] : p.d1) * 4);
  for (int l = 1; l <= p.L; ++l) b.PRE[l] = (float*)cv.take((size_t)R * p.d1 * 4);
  b.PRE[0] = nullptr;
  for (int l = 0; l < p.L; ++l) {
    b.G[l] = (float*)cv.take((size_t)R * p.gwp[l] * 4);
    b.Hbar[l] = (float*)cv.take((size_t)Wc * 2 * p.dinp[l] * 4);
    b.CG[l] = (float*)cv.take((size_t)R * p.gwp[l] * 4);
    b.h2[l] = l + 1 < p.L ? (float*)cv.take((size_t)R * p.n * p.ein[l] * 4) : nullptr;
  }
  b.Pm = (float*)cv.take((size_t)Wc * p.d1 * 4);
  for (int a = 0; a < 2; ++a) {
    const size_t m = (size_t)Wc * p.K * p.na(a) * p.na(a);
    b.phi[a] = (float*)cv.take(m * 4);
    b.u[a] = (float*)cv.take(m * 4);
    b.env[a] = (float*)cv.take(m * 4);
    b.binv[a] = cv.take(m * rb);
    b.D[a] = cv.take((size_t)Wc * p.K * 2 * rb);
    b.cot_u[a] = (float*)cv.take((size_t)Wc * p.na(a) * b.ldu * 4);
    b.cot_env[a] = (float*)cv.take(m * 4);
    b.wo[a] = (float*)cv.take((size_t)p.d1 * b.ldu * 4);
  }
  b.rho = cv.take((size_t)Wc * p.K * rb);
  b.sign = (float*)cv.take((size_t)Wc * 4);
  b.logpsi = (float*)cv.take((size_t)Wc * 4);
  b.CH = (float*)cv.take((size_t)R * p.d1 * 4);
  b.CP = (float*)cv.take((size_t)R * p.d1 * 4);
  if (p.bf16) {
    b.pw_lo = (p.P + 7) / 8 * 8;  // 16-byte aligned lo plane
    b.pw = (uint16_t*)cv.take((size_t)b.pw_lo * 2 * 2);
    for (int a = 0; a < 2; ++a) b.wo_pl[a] = (uint16_t*)cv.take((size_t)p.d1 * b.ldu * 2 * 2);
  }
  b.S = (float*)cv.take((size_t)Wc * p.d1 * 4);
  b.CMF = (float*)cv.take((size_t)Wc * 2 * dmax * 4);
  // X^T Y partials: splits(R) * K1 * N with K1 <= max(d1, 2 dinp, 2 ein)
  // (2 dinp: the mean-field weights of both spins in one product),
  // N <= max(d1, K n_a)
  int64_t k1max = std::max<int64_t>(p.d1, std::max(2 * dmax, 2 * std::max(4, p.d2)));
  int64_t nmax = std::max<int64_t>(p.d1, (int64_t)p.K * std::max(p.nu, p.nd));
  b.kcols = 0;
  b.ldf = 0;
  if (kfac) {
    // A = a~^T a~ and G = g^T g of every dense layer; two-electron blocks
    // as extra columns of the pair partials
    for (const KfacBlk& k : kfac_blocks(p, nullptr)) {
      k1max = std::max<int64_t>(k1max, std::max(k.dA, k.dG));
      nmax = std::max<int64_t>(nmax, std::max(k.dA, k.dG));
      if (k.kind == 1) b.kcols += (int64_t)k.dA * k.dA + (int64_t)k.dG * k.dG;
      if (k.kind != 1) b.ldf = std::max(b.ldf, round_up(k.dA, 4));
    }
  }
  const int64_t part_n = atb_part_floats((int)k1max, (int)nmax);
  b.part = (float*)cv.take((size_t)part_n * 4);
  b.part_n = part_n;
  b.p2 = 0;
  for (int l = 0; l + 1 < p.L; ++l) b.p2 += (int64_t)p.ein[l] * p.d2 + p.d2;
  b.ldp2 = b.p2 + b.kcols;
  b.part2 = (float*)cv.take((size_t)R * std::max<int64_t>(b.ldp2, 1) * 4);
  b.Faug = kfac ? (float*)cv.take((size_t)R * b.ldf * 4) : nullptr;
  b.sc = kfac ? (float*)cv.take((size_t)Wc * 4) : nullptr;
  // row-sum partials: column sums over R rows (d1, p2, KFAC or ldu columns)
  // and the reduction of the X^T Y partials over their splits
  const int64_t t1 = (int64_t)rowsum_chunks(R, kRowChunk) *
                     std::max<int64_t>(std::max<int64_t>(p.d1, std::max(b.p2, b.kcols)), b.ldu);
  const int64_t t2 = (int64_t)rowsum_chunks(atb_part_floats((int)k1max, (int)nmax) / 4096, kRowChunk) * k1max * nmax;
  b.tmp = (float*)cv.take((size_t)std::max(t1, t2) * 4);
  b.cot = (float*)cv.take((size_t)Wc * 4);
}

// ---------------------------------------- float64 re-evaluation buffers
// Per chunk of Wc walkers: segments of at most 8192 walkers; each segment
// of len walkers re-evaluates its ceil(f len) walkers of largest error
// scale.  Every segment but the last is full (k_seg each); the last takes
// k_last.  R = (segments - 1) k_seg + k_last in all.
struct RescueDims {
  int seg_len, k_seg, k_last;
  int64_t R;
};
static int rescue_count(float f, int64_t len) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(len, (int64_t)std::ceil((double)f * (double)len)));
}
static RescueDims rescue_dims(const Plan& p, int64_t Wc) {
  RescueDims d{0, 0, 0, 0};
  if (p.rescue <= 0.0f || Wc < 1) return d;
  d.seg_len = (int)std::min<int64_t>(Wc, 8192);
  const int64_t n_seg = (Wc + d.seg_len - 1) / d.seg_len;
  d.k_seg = rescue_count(p.rescue, d.seg_len);
  d.k_last = rescue_count(p.rescue, Wc - (n_seg - 1) * d.seg_len);
  d.R = (n_seg - 1) * d.k_seg + d.k_last;
  return d;
}

struct RescueBufs {
  Plan p64;
  void* pk64;
  Bufs b;
  int32_t* idx;
  float* pos_r;
  float* out[5];  // sign, logpsi, e_loc, e_kin, e_pot of the re-evaluated walkers
};

static void carve_rescue(const Plan& p, int64_t Wc, Carver& cv, RescueBufs& r) {
  const RescueDims d = rescue_dims(p, Wc);
  fn_config c = p.cfg;
  c.precision = FN_PREC_FP64;
  make_plan(&c, r.p64);
  r.pk64 = cv.take((size_t)r.p64.pk_total * r.p64.act);
  carve_forward(r.p64, JET, d.R, cv, r.b, false);
  r.idx = (int32_t*)cv.take((size_t)d.R * 4);
  r.pos_r = (float*)cv.take((size_t)d.R * p.n3 * 4);
  for (int q = 0; q < 5; ++q) r.out[q] = (float*)cv.take((size_t)d.R * 4);
}

// float64 scratch of the KFAC step direction: per dense layer the damped
// factors and two copies of its gradient block
static void carve_kfac_solve(const Plan& p, Carver& cv, KfacPrepArgs& a) {
  const std::vector<KfacBlk> kb = kfac_blocks(p, nullptr);
  a.nb = (int)kb.size();
  char* base = cv.base;
  auto take = [&](int64_t doubles) { return (int64_t)(((char*)cv.take((size_t)doubles * 8) - base) / 8); };
  for (int b = 0; b < a.nb; ++b) {
    const KfacBlk& k = kb[b];
    a.dA[b] = k.dA;
    a.dG[b] = k.dG;
    a.offA[b] = k.offA;
    a.offG[b] = k.offG;
    a.offP[b] = k.kind == 0 ? p.offV[k.layer] : k.kind == 1 ? p.offW2[k.layer] : p.offw[k.layer];
    a.offLA[b] = take((int64_t)k.dA * k.dA);
    a.offLG[b] = take((int64_t)k.dG * k.dG);
    a.offY[b] = take((int64_t)k.dA * k.dG);
    a.offYt[b] = take((int64_t)k.dA * k.dG);
    a.offIA[b] = take((int64_t)(k.dA + 31) / 32 * 32 * 32);
    a.offIG[b] = take((int64_t)(k.dG + 31) / 32 * 32 * 32);
  }
}

// buffers of one VMC iteration that live across its passes (the batch of W
// walkers; the passes take their own workspace after these)
struct TrainBufs {
  float *sign, *logpsi, *e_clip, *wts, *cot;
  int32_t* n_acc;
  double* part;
  float *grad, *dir, *fb;
};

static void carve_train(const Plan& p, int64_t W, Carver& cv, TrainBufs& t) {
  t.sign = (float*)cv.take(W * 4);
  t.logpsi = (float*)cv.take(W * 4);
  t.e_clip = (float*)cv.take(W * 4);
  t.wts = (float*)cv.take(W * 4);
  t.cot = (float*)cv.take(W * 4);
  t.n_acc = (int32_t*)cv.take(W * 4);
  t.part = (double*)cv.take(256 * 8);
  t.grad = (float*)cv.take(p.P * 4);
  t.dir = (float*)cv.take(p.P * 4);
  int64_t total = 0;
  kfac_blocks(p, &total);
  t.fb = (float*)cv.take(total * 4);
}

// One pass over a batch of Wc walkers: the packed weights, the jet pass,
// its float64 re-evaluation and the reverse pass's buffers (with the KFAC
// statistics' buffers when kfac), which the jet pass fills with its values.
struct OnePass {
  Bufs b;
  RescueBufs r;
  AdjBufs ab;
};
static void carve_one_pass(const Plan& p, int64_t Wc, Carver& cv, OnePass& o, bool kfac) {
  o.b.pk = cv.take(pk_bytes(p));
  carve_forward(p, JET, Wc, cv, o.b, false);
  if (p.rescue > 0.0f) {
    carve_rescue(p, Wc, cv, o.r);
    o.r.b.pk = o.r.pk64;
  }
  carve_adjoint(p, Wc, cv, o.ab, kfac);
}
static size_t one_pass_bytes(const Plan& p, int64_t Wc, bool kfac) {
  Carver cv{nullptr, 0};
  OnePass o;
  carve_one_pass(p, Wc, cv, o, kfac);
  return cv.used;
}

static size_t chunk_bytes(const Plan& p, int entry, int64_t Wc) {
  Carver cv{nullptr, 0};
  if (entry == FN_ENTRY_TRAIN) {
    TrainBufs t;
    carve_train(p, Wc, cv, t);
    size_t pass = chunk_bytes(p, FN_ENTRY_KFAC_PRECONDITION, 1);
    for (int e = FN_ENTRY_LOGPSI; e <= FN_ENTRY_KFAC; ++e) pass = std::max(pass, chunk_bytes(p, e, Wc));
    // the local energy, gradient and KFAC statistics of the batch in one pass
    pass = std::max(pass, one_pass_bytes(p, Wc, true));
    return cv.used + pass;
  }
  if (entry == FN_ENTRY_KFAC_PRECONDITION) {
    KfacPrepArgs a;
    Carver c0{(char*)nullptr, 0};
    carve_kfac_solve(p, c0, a);
    return c0.used;
  }
  Bufs b;
  cv.take(pk_bytes(p));
  if (entry == FN_ENTRY_LOCAL_ENERGY_GRADIENT) return one_pass_bytes(p, Wc, false);
  if (entry == FN_ENTRY_GRAD_LOGPSI || entry == FN_ENTRY_KFAC) {
    AdjBufs ab;
    carve_adjoint(p, Wc, cv, ab, entry == FN_ENTRY_KFAC);
    return cv.used;
  }
  carve_forward(p, entry == FN_ENTRY_LOCAL_ENERGY ? JET : VALUE, Wc, cv, b, entry == FN_ENTRY_MCMC);
  if (entry == FN_ENTRY_LOCAL_ENERGY && p.rescue > 0.0f) {
    RescueBufs r;
    carve_rescue(p, Wc, cv, r);
  }
  return cv.used;
}

static int64_t max_chunk(const Plan& p, int entry, size_t ws_bytes, int64_t W) {
  const size_t b1 = chunk_bytes(p, entry, 1);
  if (ws_bytes < b1) return 0;
  if (ws_bytes >= chunk_bytes(p, entry, W)) return W;
  // bytes grow monotonically with the chunk: bisect
  int64_t lo = 1, hi = W;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (chunk_bytes(p, entry, mid) <= ws_bytes) lo = mid;
    else hi = mid;
  }
  return lo;
}

#define FN_HIP(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return FN_ERR_HIP; \
  } while (0)

// ------------------------------------------------------- stage timing
// Diagnostics only (off by default): when enabled, every launch is
// bracketed by two HIP events on the caller's stream, so per-stage device
// time can be read back after the work has run.
static const char* kStageNames[ST_COUNT] = {
    "pack_weights", "features",  "two_electron", "meanfield",    "gemm_meanfield", "gemm_layer",
    "gemm_orbital", "det",       "combine",      "mcmc_propose", "mcmc_accept",    "adj_forward",
    "adj_det",      "adj_orbital", "adj_layers", "adj_two_electron", "adj_reduce",     "gemm_layer_value",
    "rescue_fp64",  "kfac_precondition", "train_step", "gemm_layer_mf"};
static std::mutex g_time_mu;
static std::atomic<bool> g_timing{false};
struct StageRec {
  int stage;
  hipEvent_t a, b;
};
static std::vector<StageRec> g_recs;

struct StageScope {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageScope(int st, hipStream_t str) : stage(st), s(str) {
    if (g_timing && hipEventCreate(&a) == hipSuccess) hipEventRecord(a, s);
  }
  ~StageScope() {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(g_time_mu);
    g_recs.push_back({stage, a, b});
  }
};

#define FN_T(stage, x)                            \
  do {                                            \
    StageScope _sc(stage, s);                     \
    if ((x) != hipSuccess) return FN_ERR_HIP;     \
  } while (0)

static fn_status pack(const Plan& p, const float* params, void* dst, hipStream_t s) {
  std::vector<int64_t> it;
  int n = pack_plan(p, it);
  FN_T(ST_PACK, launch_pack_weights(p.mode, params, dst, p.pk_total, it.data(), n, s));
  if (p.bf16) {  // float32 copies of the orbital blocks (the last items of the plan)
    const int first = n - (p.nu > 0) - (p.nd > 0);
    FN_T(ST_PACK, launch_pack_weights(MODE_F32, params, (char*)dst + (size_t)p.pk_total * 4, p.pk_total,
                                      it.data() + (size_t)first * 11, n - first, s));
  }
  return FN_OK;
}

// packed weight block at element offset off: float32, or the bfloat16 hi
// plane (lo = false) / lo plane (lo = true) in the split form
static const void* wt(const Bufs& b, const Plan& p, int64_t off, bool lo) {
  if (!p.bf16) return lo ? nullptr : (const char*)b.pk + off * p.act;
  return (const char*)b.pk + (off + (lo ? p.pk_total : 0)) * 2;
}

// the orbital layer's weights and the arithmetic of its product: in the
// split-bfloat16 form the orbital GEMM runs with float32 accuracy, its
// float32 operands (a float32 copy of the orbital weights is packed after
// the two bfloat16 planes) split into three bfloat16 parts each (the
// rounding of a two-part product, amplified by the cancellation in its dot
// products and by the conditioning of the orbital matrices, dominated the
// local-energy error of the form)
static const void* wt_orb(const Bufs& b, const Plan& p, int a) {
  if (!p.bf16) return wt(b, p, p.pk_orb[a], false);
  return (const char*)b.pk + ((size_t)p.pk_total * 4 + (size_t)p.pk_orb[a] * 4);
}
static int orb_mode(const Plan& p) { return p.mode == MODE_BF16X3 ? MODE_BF16X6 : p.mode; }

// FN_OPT_FUSED_MEANFIELD
static std::atomic<bool> g_fused_meanfield{true};

// forward pass over one chunk of Wc walkers.  jet: local energy; value:
// sign and log|psi| only.  Launches are timed under their own stages, or
// all under stage_all when it is not negative.
// cap (jet mode): the values of the pass (row 0 of every jet), written
// into the adjoint's buffers as its own value-only pass would write them
static fn_status forward(const Plan& p, Mode m, int64_t Wc, const float* pos, const float* nuc, const float* Z,
                         const float* params, const Bufs& b, float* sign, float* logpsi, float* e_loc,
                         float* e_kin, float* e_pot, hipStream_t s, int stage_all = -1,
                         const AdjBufs* cap = nullptr) {
  const int T = b.T, Tp = b.Tp;
  const int64_t R = Wc * p.n;
  auto SG = [stage_all](int st) { return stage_all >= 0 ? stage_all : st; };
  // the input jets and, for the first layer, their spin means
  // (and their value rows for the reverse pass, when it reads this pass)
  FN_T(SG(ST_FEATURES), launch_features(p.f64, pos, nuc, (int)Wc, p.n, p.nu, p.N, T, Tp, b.H0, p.dinp[0], b.Hbar, s,
                                        cap ? cap->H[0] : nullptr, cap ? cap->Hbar[0] : nullptr));
  TwoElecArgs te;
  memset(&te, 0, sizeof(te));
  te.pos = pos;
  te.params = params;
  te.w_off = p.offW2;
  te.c_off = p.offc2;
  te.W = (int)Wc;
  te.n = p.n;
  te.n_up = p.nu;
  te.L = p.L;
  te.d2 = p.d2;
  te.T = T;
  te.Tp = Tp;
  for (int l = 0; l < p.L; ++l) {
    te.G[l] = b.G[l];
    te.ldg[l] = p.gwp[l];
    te.h2_out[l] = cap ? cap->h2[l] : nullptr;
    te.g_val_out[l] = cap ? cap->G[l] : nullptr;
  }
  FN_T(SG(ST_TWO_E), launch_two_electron(p.f64, te, s));
  const void* Hin = b.H0;
  void* Hout = b.Ha;
  bool hbar_ready = true;  // the previous kernel wrote the spin means of Hin
  for (int l = 0; l < p.L; ++l) {
    if (!hbar_ready)
      FN_T(SG(ST_MEANFIELD), launch_meanfield(p.f64, Hin, p.dinp[l], (int)Wc, p.n, p.nu, Tp, p.dinp[l], b.Hbar, s));
    if (cap && l > 0)  // the features kernel wrote the first layer's
      FN_T(SG(ST_MEANFIELD), launch_copy_rows((const float*)b.Hbar, (int64_t)Tp * 2 * p.dinp[l], cap->Hbar[l],
                                              2 * p.dinp[l], Wc, 2 * p.dinp[l], s));
    JetGemmArgs g;
    memset(&g, 0, sizeof(g));
    g.a0 = b.Hbar;
    g.lda0 = 2 * p.dinp[l];
    g.ka0 = 2 * p.dinp[l];
    g.bt = wt(b, p, p.pk_mf[l], false);
    g.bt_lo = wt(b, p, p.pk_mf[l], true);
    g.ldb = p.ld_mf[l];
    g.n_groups = (int)Wc;
    g.rows_per = Tp;
    g.T = T;
    g.n_sub = 1;
    g.n_all = 1;
    g.N = p.d1;
    g.c = b.Pm;
    g.ldc = p.d1;
    FN_T(SG(ST_GEMM_MF), launch_jet_gemm(p.mode, EPI_PLAIN, g, s));
    JetGemmArgs h;
    memset(&h, 0, sizeof(h));
    h.a0 = Hin;
    h.lda0 = p.dinp[l];
    h.ka0 = p.dinp[l];
    h.a1 = b.G[l];
    h.lda1 = p.gwp[l];
    h.ka1 = p.gwp[l];
    h.bt = wt(b, p, p.pk_main[l], false);
    h.bt_lo = wt(b, p, p.pk_main[l], true);
    h.ldb = p.ld_main[l];
    h.n_groups = (int)(Wc * p.n);
    h.rows_per = Tp;
    h.T = T;
    h.n_sub = p.n;
    h.n_all = p.n;
    h.N = p.d1;
    h.out = Hout;
    h.ldo = p.d1;
    h.P = b.Pm;
    h.ldp = p.d1;
    h.bias = params + p.offb[l];
    h.res = p.din[l] == p.d1;
    h.pre_out = cap ? cap->PRE[l + 1] : nullptr;
    h.val_out = cap ? cap->H[l + 1] : nullptr;
    // the spin means of this layer's output, for the next layer, from the
    // layer kernel itself where its shape allows
    hbar_ready = false;
    if (l + 1 < p.L && !p.f64 && g_fused_meanfield.load()) {
      h.mf_out = (float*)b.Hbar;
      h.mf_ld = 2 * p.dinp[l + 1];
      h.mf_half = p.dinp[l + 1];
      h.mf_na = p.nu;
      hbar_ready = layer_mf_supported(h);
      if (!hbar_ready) h.mf_out = nullptr;
    }
    FN_T(SG(m == JET ? (hbar_ready ? ST_GEMM_LAYER_MF : ST_GEMM_LAYER) : ST_GEMM_LAYER_VALUE),
         launch_jet_gemm(p.mode, EPI_TANHJET, h, s));
    Hin = Hout;
    Hout = Hout == b.Ha ? b.Hb : b.Ha;
  }
  for (int a = 0; a < 2; ++a) {
    const int na = p.na(a);
    if (na == 0) continue;
    JetGemmArgs o;
    memset(&o, 0, sizeof(o));
    o.a0 = Hin;
    o.lda0 = p.d1;
    o.ka0 = p.d1;
    o.bt = wt_orb(b, p, a);
    o.bt_lo = nullptr;
    o.ldb = p.d1;
    o.n_groups = (int)(Wc * na);
    o.rows_per = Tp;
    o.T = T;
    o.n_sub = na;
    o.n_all = p.n;
    o.e_off = a == 0 ? 0 : p.nu;
    o.N = p.K * na;
    o.phi = b.phi[a];
    o.phi_M = det_uses_small(na) ? Wc * p.K : 0;
    o.pos = pos;
    o.nuc = nuc;
    o.n_nuc = p.N;
    o.n_elec = p.n;
    o.g_orb = params + p.offg[a];
    o.pi = params + p.offpi[a];
    o.sigma = params + p.offsg[a];
    o.env_full = p.env_full;
    o.u_out = cap ? cap->u[a] : nullptr;
    o.env_out = cap ? cap->env[a] : nullptr;
    FN_T(SG(ST_GEMM_ORB), launch_jet_gemm(orb_mode(p), EPI_ORBITAL, o, s));
    FN_T(SG(ST_DET), launch_det(p.fp64, b.phi[a], p.f64, (int)Wc, p.K, na, T, p.n3, b.D[a], b.dstride,
                                cap ? cap->binv[a] : nullptr, s));
  }
  CombineArgs cb;
  memset(&cb, 0, sizeof(cb));
  cb.D[0] = b.D[0];
  cb.D[1] = b.D[1];
  cb.dstride = b.dstride;
  cb.na[0] = p.nu;
  cb.na[1] = p.nd;
  cb.W = (int)Wc;
  cb.K = p.K;
  cb.n = p.n;
  cb.n3 = p.n3;
  cb.N = p.N;
  cb.jet = m == JET;
  cb.pos = pos;
  cb.nuc = nuc;
  cb.Z = Z;
  cb.sign = sign;
  cb.logpsi = logpsi;
  cb.e_loc = e_loc;
  cb.e_kin = e_kin;
  cb.e_pot = e_pot;
  cb.rescue_key = m == JET ? b.rkey : nullptr;
  cb.rho = cap ? cap->rho : nullptr;
  // orbitals: split bfloat16 (16 significand bits) or float32; determinants:
  // float64 or float32
  // unit roundoff of the determinant arithmetic over that of the orbital
  // product (float32 in every form but the float64 one)
  cb.cond_weight = (float)(std::ldexp(1.0, p.fp64 ? -53 : -24) / std::ldexp(1.0, -24));
  FN_T(SG(ST_COMBINE), launch_combine(p.fp64, cb, s));
  return FN_OK;
}

static fn_status check_common(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                              const float* nuc_pos, const float* nuc_charge, const float* params, void* ws,
                              Plan& p) {
  fn_status st = make_plan(cfg, p);
  if (st != FN_OK) return st;
  if (W < 0) return FN_ERR_ARG;
  if (!spins) return FN_ERR_NULL;
  for (int i = 0; i < p.n; ++i)
    if (spins[i] != (i < p.nu ? 0 : 1)) return FN_ERR_SPINS;
  if (W > 0 && (!pos || !nuc_pos || !nuc_charge || !params || !ws)) return FN_ERR_NULL;
  if (((uintptr_t)ws) & 255) return FN_ERR_WORKSPACE;
  return FN_OK;
}

// value-only forward pass of one chunk that keeps what the adjoint needs
static fn_status forward_store(const Plan& p, int64_t Wc, const float* pos, const float* nuc, const float* Z,
                               const float* params, const void* pk, const AdjBufs& b, hipStream_t s) {
  Bufs fb;
  fb.pk = const_cast<void*>(pk);
  FN_T(ST_ADJ_FWD, launch_features(false, pos, nuc, (int)Wc, p.n, p.nu, p.N, 1, 1, b.H[0], p.dinp[0], b.Hbar[0], s));
  TwoElecArgs te;
  memset(&te, 0, sizeof(te));
  te.pos = pos;
  te.params = params;
  te.w_off = p.offW2;
  te.c_off = p.offc2;
  te.W = (int)Wc;
  te.n = p.n;
  te.n_up = p.nu;
  te.L = p.L;
  te.d2 = p.d2;
  te.T = 1;
  te.Tp = 1;
  for (int l = 0; l < p.L; ++l) {
    te.G[l] = b.G[l];
    te.ldg[l] = p.gwp[l];
    te.h2_out[l] = b.h2[l];
  }
  FN_T(ST_ADJ_FWD, launch_two_electron(false, te, s));
  const int mode = p.bf16 ? MODE_BF16X3 : MODE_F32;
  for (int l = 0; l < p.L; ++l) {
    const int ldh = l == 0 ? p.dinp[0] : p.d1;
    if (l > 0)  // the features kernel wrote the first layer's
      FN_T(ST_ADJ_FWD, launch_meanfield(false, b.H[l], ldh, (int)Wc, p.n, p.nu, 1, p.dinp[l], b.Hbar[l], s));
    JetGemmArgs g;
    memset(&g, 0, sizeof(g));
    g.a0 = b.Hbar[l];
    g.lda0 = 2 * p.dinp[l];
    g.ka0 = 2 * p.dinp[l];
    g.bt = wt(fb, p, p.pk_mf[l], false);
    g.bt_lo = wt(fb, p, p.pk_mf[l], true);
    g.ldb = p.ld_mf[l];
    g.n_groups = (int)Wc;
    g.rows_per = 1;
    g.T = 1;
    g.n_sub = 1;
    g.n_all = 1;
    g.N = p.d1;
    g.c = b.Pm;
    g.ldc = p.d1;
    FN_T(ST_ADJ_FWD, launch_jet_gemm(mode, EPI_PLAIN, g, s));
    JetGemmArgs h;
    memset(&h, 0, sizeof(h));
    h.a0 = b.H[l];
    h.lda0 = ldh;
    h.ka0 = p.dinp[l];
    h.a1 = b.G[l];
    h.lda1 = p.gwp[l];
    h.ka1 = p.gwp[l];
    h.bt = wt(fb, p, p.pk_main[l], false);
    h.bt_lo = wt(fb, p, p.pk_main[l], true);
    h.ldb = p.ld_main[l];
    h.n_groups = (int)(Wc * p.n);
    h.rows_per = 1;
    h.T = 1;
    h.n_sub = p.n;
    h.n_all = p.n;
    h.N = p.d1;
    h.out = b.H[l + 1];
    h.ldo = p.d1;
    h.P = b.Pm;
    h.ldp = p.d1;
    h.bias = params + p.offb[l];
    h.res = p.din[l] == p.d1;
    h.pre_out = b.PRE[l + 1];
    FN_T(ST_ADJ_FWD, launch_jet_gemm(mode, EPI_TANHJET, h, s));
  }
  for (int a = 0; a < 2; ++a) {
    const int na = p.na(a);
    if (na == 0) continue;
    JetGemmArgs o;
    memset(&o, 0, sizeof(o));
    o.a0 = b.H[p.L];
    o.lda0 = p.d1;
    o.ka0 = p.d1;
    o.bt = wt_orb(fb, p, a);
    o.bt_lo = nullptr;
    o.ldb = p.d1;
    o.n_groups = (int)(Wc * na);
    o.rows_per = 1;
    o.T = 1;
    o.n_sub = na;
    o.n_all = p.n;
    o.e_off = a == 0 ? 0 : p.nu;
    o.N = p.K * na;
    o.phi = b.phi[a];
    o.phi_M = det_uses_small(na) ? Wc * p.K : 0;
    o.pos = pos;
    o.nuc = nuc;
    o.n_nuc = p.N;
    o.n_elec = p.n;
    o.g_orb = params + p.offg[a];
    o.pi = params + p.offpi[a];
    o.sigma = params + p.offsg[a];
    o.env_full = p.env_full;
    o.u_out = b.u[a];
    o.env_out = b.env[a];
    FN_T(ST_ADJ_FWD, launch_jet_gemm(orb_mode(p), EPI_ORBITAL, o, s));
    FN_T(ST_ADJ_DET, launch_det(p.fp64, b.phi[a], false, (int)Wc, p.K, na, 1, p.n3, b.D[a], 2, b.binv[a], s));
  }
  CombineArgs cb;
  memset(&cb, 0, sizeof(cb));
  cb.D[0] = b.D[0];
  cb.D[1] = b.D[1];
  cb.dstride = 2;
  cb.na[0] = p.nu;
  cb.na[1] = p.nd;
  cb.W = (int)Wc;
  cb.K = p.K;
  cb.n = p.n;
  cb.n3 = p.n3;
  cb.N = p.N;
  cb.jet = 0;
  cb.pos = pos;
  cb.nuc = nuc;
  cb.Z = Z;
  cb.sign = b.sign;
  cb.logpsi = b.logpsi;
  cb.rho = b.rho;
  FN_T(ST_ADJ_DET, launch_combine(p.fp64, cb, s));
  return FN_OK;
}

// X^T Y over R rows added into grad[off ...] (K1 x N block, row-major)
// sym: X and Y are the same columns (K1 == N) and dst is symmetric: only its
// 64 x 64 tiles on and above the diagonal are accumulated (launch_sym_mirror
// completes it once every chunk is in)
// gld > 0: per walker instead, seg rows per walker, walker q's product
// added at dst + q gld
static fn_status atb_add(const AdjBufs& b, const float* X, int64_t ldx, int xcol, int xs, int xa, int xe,
                         const float* Y, int64_t ldy, int64_t R, int K1, int N, float* dst, hipStream_t s,
                         bool sym = false, int64_t gld = 0, int seg = 0) {
  AtbArgs a;
  a.X = X;
  a.ldx = ldx;
  a.xcol = xcol;
  a.xs = xs;
  a.xa = xa;
  a.xe = xe;
  a.Y = Y;
  a.ldy = ldy;
  a.R = R;
  a.K1 = K1;
  a.N = N;
  a.part = b.part;
  a.sym = sym ? 1 : 0;
  // the split form's sums over rows on split-bfloat16 products (per-walker
  // products keep float32: a walker's few rows would pad a 32-row step)
  a.bf16 = b.pw != nullptr && gld == 0 ? 1 : 0;
  if (gld > 0) {
    a.dst = dst;
    a.dst_ld = gld;
    a.seg = seg;
    FN_T(ST_ADJ_REDUCE, launch_atb(a, s));
    return FN_OK;
  }
  FN_T(ST_ADJ_REDUCE, launch_atb(a, s));
  const int64_t cols = (int64_t)K1 * N;
  FN_T(ST_ADJ_REDUCE, launch_rowsum_add(b.part, atb_splits(R, K1, N), (int)cols, cols, b.tmp, dst, kRowChunk, s,
                                        sym ? N : 0));
  return FN_OK;
}

// C [rows][K] times (rows of params) [N][ld] transposed: out[r][n] (=/+=) sum_k C[r][k] Wt[n][k]
static fn_status gemm_cwt(const float* C, int ldc_in, int K, int64_t rows, const float* Wt, int ldw, int N,
                          float* out, int ldo, int accum, int o_nsub, int o_nall, int o_eoff, int stage,
                          hipStream_t s, const uint16_t* whi = nullptr, const uint16_t* wlo = nullptr) {
  JetGemmArgs g;
  memset(&g, 0, sizeof(g));
  g.a0 = C;
  g.lda0 = ldc_in;
  g.ka0 = K;
  g.bt = Wt;
  g.ldb = ldw;
  g.n_groups = (int)rows;
  g.rows_per = 1;
  g.T = 1;
  g.n_sub = 1;
  g.n_all = 1;
  g.N = N;
  g.c = out;
  g.ldc = ldo;
  g.c_nsub = o_nsub;
  g.c_nall = o_nall;
  g.c_eoff = o_eoff;
  g.c_accum = accum;
  // the split form multiplies by the bfloat16 planes of the weights where
  // their rows are 16-byte aligned
  const bool split = whi && wlo && ldw % 8 == 0 && (uintptr_t)whi % 16 == 0 && (uintptr_t)wlo % 16 == 0;
  if (split) {
    g.bt = whi;
    g.bt_lo = wlo;
  }
  FN_T(stage, launch_jet_gemm(split ? MODE_BF16X3 : MODE_F32, EPI_PLAIN, g, s));
  return FN_OK;
}

// reverse pass of one chunk with walker cotangents cot[Wc]; adds into grad
// (when not NULL) and, with kout, the KFAC factors of the chunk into kout
// (the cotangents then being sqrt(c_w), held in b.sc).  gld > 0: grad holds
// one gradient per walker of the chunk, walker q's at grad + q gld.
static fn_status backward(const Plan& p, int64_t Wc, const float* pos, const float* nuc, const float* params,
                          const float* cot, const AdjBufs& b, float* grad, hipStream_t s, float* kout = nullptr,
                          int64_t gld = 0) {
  const int64_t R = Wc * p.n;
  fn_status st;
  // the cotangent of the current layer's output, updated in place into
  // that of its input
  float* CHc = b.CH;
  std::vector<KfacBlk> kb;
  if (kout) kb = kfac_blocks(p, nullptr);
  auto kblk = [&](int kind, int layer) -> const KfacBlk* {
    for (const KfacBlk& k : kb)
      if (k.kind == kind && k.layer == layer) return &k;
    return nullptr;
  };
  // determinants -> orbitals -> envelope
  for (int a = 0; a < 2; ++a) {
    const int na = p.na(a);
    if (na == 0) continue;
    const int j0 = a == 0 ? 0 : p.nu;
    FN_T(ST_ADJ_ORB, launch_adj_orbital_cot(p.fp64, b.binv[a], b.rho, cot, b.u[a], b.env[a], (int)Wc, p.K, na, b.ldu,
                                            b.cot_u[a], b.cot_env[a], s));
    if (grad) {
      FN_T(ST_ADJ_ORB, launch_adj_env_grad(b.cot_env[a], pos, nuc, params + p.offpi[a], params + p.offsg[a],
                                           p.env_full, (int)Wc, p.K, na, j0, p.n, p.N, grad + p.offpi[a],
                                           grad + p.offsg[a], s, gld, b.part, b.part_n));
      if (gld > 0)
        FN_T(ST_ADJ_REDUCE, launch_rowsum_seg_add(b.cot_u[a], Wc * na, na, p.K * na, b.ldu, grad + p.offg[a], gld, s));
      else
        FN_T(ST_ADJ_REDUCE,
             launch_rowsum_add(b.cot_u[a], Wc * na, p.K * na, b.ldu, b.tmp, grad + p.offg[a], kRowChunk, s));
      st = atb_add(b, b.H[p.L], p.d1, 0, na, p.n, j0, b.cot_u[a], b.ldu, Wc * na, p.d1, p.K * na, grad + p.offw[a], s,
                   false, gld, na);
      if (st != FN_OK) return st;
    }
    if (kout) {
      // orbital layer of spin a: G = cot_u^T cot_u, A = a~^T a~ with a~ = sqrt(c_w) [h^L_j, 1]
      const KfacBlk* k = kblk(2, a);
      st = atb_add(b, b.cot_u[a], b.ldu, 0, 0, 0, 0, b.cot_u[a], b.ldu, Wc * na, k->dG, k->dG, kout + k->offG, s,
                   true);
      if (st != FN_OK) return st;
      FN_T(ST_ADJ_REDUCE, launch_kfac_aug_orbital(b.H[p.L], p.d1, p.d1, b.sc, (int)Wc, p.n, j0, na, b.ldf, b.Faug, s));
      st = atb_add(b, b.Faug, b.ldf, 0, 0, 0, 0, b.Faug, b.ldf, Wc * na, k->dA, k->dA, kout + k->offA, s, true);
      if (st != FN_OK) return st;
    }
    // cot h^L of the electrons of spin a
    const uint16_t* wh = b.wo_pl[a];
    st = gemm_cwt(b.cot_u[a], b.ldu, b.ldu, Wc * na, b.wo[a], b.ldu, p.d1, CHc, p.d1, 0, na, p.n, j0, ST_ADJ_ORB, s, wh,
                  wh ? wh + (int64_t)p.d1 * b.ldu : nullptr);
    if (st != FN_OK) return st;
  }
  // one-electron layers, last to first.  The mean-field part of a layer's
  // input cotangent (CMF, per walker) is added to CH by the next layer's
  // cotangent pass, which reads CH anyway.
  const float* cmf_pending = nullptr;
  for (int l = p.L - 1; l >= 0; --l) {
    const int din = p.din[l], ein = p.ein[l];
    const float* V = params + p.offV[l];
    FN_T(ST_ADJ_LAYERS,
         launch_adj_cp_sum(CHc, b.PRE[l + 1], cmf_pending, (int)Wc, p.n, p.nu, p.d1, b.CP, b.S, s));
    const int ldh = l == 0 ? p.dinp[0] : p.d1;
    if (grad) {
      // bias: sum over the electrons of CP, from its per-walker sums S
      if (gld > 0)
        FN_T(ST_ADJ_REDUCE, launch_rowsum_seg_add(b.S, Wc, 1, p.d1, p.d1, grad + p.offb[l], gld, s));
      else
        FN_T(ST_ADJ_REDUCE, launch_rowsum_add(b.S, Wc, p.d1, p.d1, b.tmp, grad + p.offb[l], kRowChunk, s));
      // dA = sum h_i^T cp_i
      st = atb_add(b, b.H[l], ldh, 0, 0, 0, 0, b.CP, p.d1, R, din, p.d1, grad + p.offV[l], s, false, gld, p.n);
      if (st != FN_OK) return st;
      // dB^a = sum_w hbar^a_w^T S_w; one product for both spins where
      // their column blocks of Hbar are adjacent (no padding), as the two
      // blocks of dB are in the parameters
      const int nsp = p.dinp[l] == din ? 1 : 2;
      for (int a = 0; a < nsp; ++a) {
        st = atb_add(b, b.Hbar[l], 2 * p.dinp[l], a * p.dinp[l], 0, 0, 0, b.S, p.d1, Wc, din * (3 - nsp), p.d1,
                     grad + p.offV[l] + (int64_t)(din + a * din) * p.d1, s, false, gld, 1);
        if (st != FN_OK) return st;
      }
      // dC = sum g_i^T cp_i (columns a ein + o)
      st = atb_add(b, b.G[l], p.gwp[l], 0, 0, 0, 0, b.CP, p.d1, R, 2 * ein, p.d1,
                   grad + p.offV[l] + (int64_t)3 * din * p.d1, s, false, gld, p.n);
      if (st != FN_OK) return st;
    }
    if (kout) {
      // one-electron layer l: G = cp^T cp, A = a~^T a~ with
      // a~ = sqrt(c_w) [h_i, hbar^up, hbar^down, g^up_i, g^down_i, 1]
      const KfacBlk* k = kblk(0, l);
      st = atb_add(b, b.CP, p.d1, 0, 0, 0, 0, b.CP, p.d1, R, k->dG, k->dG, kout + k->offG, s, true);
      if (st != FN_OK) return st;
      FN_T(ST_ADJ_REDUCE, launch_kfac_aug_layer(b.H[l], ldh, din, b.Hbar[l], p.dinp[l], b.G[l], p.gwp[l], ein, b.sc,
                                                (int)Wc, p.n, b.ldf, b.Faug, s));
      st = atb_add(b, b.Faug, b.ldf, 0, 0, 0, 0, b.Faug, b.ldf, R, k->dA, k->dA, kout + k->offA, s, true);
      if (st != FN_OK) return st;
    }
    // cot g^l_i = cp_i [C^up; C^down]^T  (for the two-electron stream)
    // the weights' bfloat16 planes at element offset o of the parameters (split form)
    auto hi = [&](int64_t o) { return b.pw ? b.pw + p.offV[l] + o : nullptr; };
    auto lo = [&](int64_t o) { return b.pw ? b.pw + b.pw_lo + p.offV[l] + o : nullptr; };
    st = gemm_cwt(b.CP, p.d1, p.d1, R, V + (int64_t)3 * din * p.d1, p.d1, 2 * ein, b.CG[l], p.gwp[l], 0, 0, 0, 0,
                  ST_ADJ_LAYERS, s, hi((int64_t)3 * din * p.d1), lo((int64_t)3 * din * p.d1));
    if (st != FN_OK) return st;
    if (l == 0) break;  // the input features carry no parameters
    // cot h^l_i = cp_i A^T + cot h^{l+1}_i + cot hbar^{a(i)} / n_a: the
    // first two terms in place (for l > 0, h^l is the output of layer
    // l - 1, so din = d1 and the residual is always there), the last one
    // with the next cotangent pass
    st = gemm_cwt(b.CP, p.d1, p.d1, R, V, p.d1, din, CHc, p.d1, 1, 0, 0, 0, ST_ADJ_LAYERS, s, hi(0), lo(0));
    if (st != FN_OK) return st;
    st = gemm_cwt(b.S, p.d1, p.d1, Wc, V + (int64_t)din * p.d1, p.d1, 2 * din, b.CMF, 2 * din, 0, 0, 0, 0,
                  ST_ADJ_LAYERS, s, hi((int64_t)din * p.d1), lo((int64_t)din * p.d1));
    if (st != FN_OK) return st;
    cmf_pending = b.CMF;
  }
  // two-electron stream
  if (p.L >= 2) {
    Adj2eArgs a2;
    memset(&a2, 0, sizeof(a2));
    a2.params = params;
    int64_t po = 0;
    for (int l = 0; l < p.L; ++l) {
      if (l + 1 < p.L) {
        a2.w_off[l] = p.offW2[l];
        a2.c_off[l] = p.offc2[l];
        a2.p_off[l] = po;
        po += (int64_t)p.ein[l] * p.d2 + p.d2;
        a2.h2[l] = b.h2[l];
      }
      a2.CG[l] = b.CG[l];
      a2.ldcg[l] = p.gwp[l];
    }
    a2.p2 = b.p2;
    a2.ldp = b.ldp2;
    a2.W = (int)Wc;
    a2.n = p.n;
    a2.n_up = p.nu;
    a2.L = p.L;
    a2.d2 = p.d2;
    a2.part = b.part2;
    const KfacBlk* k0 = kout ? kblk(1, 0) : nullptr;
    if (k0) {
      // the pair blocks are contiguous in the output, A then G per layer,
      // as the KFAC columns of the partial rows
      a2.kfac = 1;
      a2.sc = b.sc;
      for (int l = 0; l + 1 < p.L; ++l) a2.k_off[l] = b.p2 + (kblk(1, l)->offA - k0->offA);
    }
    FN_T(ST_ADJ_TWO_E, launch_adj_two_electron(a2, s));
    const int rows2 = adj_two_electron_rows((int)Wc, p.n, p.d2);
    if (grad && gld > 0)
      FN_T(ST_ADJ_REDUCE, launch_rowsum_seg_add(b.part2, rows2, (int)(rows2 / Wc), (int)b.p2, b.ldp2,
                                                grad + p.offW2[0], gld, s));
    else if (grad)
      FN_T(ST_ADJ_REDUCE,
           launch_rowsum_add(b.part2, rows2, (int)b.p2, b.ldp2, b.tmp, grad + p.offW2[0], kRowChunk, s));
    if (k0)
      FN_T(ST_ADJ_REDUCE, launch_rowsum_add(b.part2 + b.p2, rows2, (int)b.kcols, b.ldp2, b.tmp, kout + k0->offA,
                                            kRowChunk, s));
  }
  return FN_OK;
}

// the reverse pass's own copies of the weights: the bfloat16 planes of the
// parameters (split form) and the orbital weights with zero-padded columns
static fn_status adjoint_weights(const Plan& p, const AdjBufs& b, const float* params, hipStream_t s) {
  // split form: the bfloat16 planes of the parameters for the reverse
  // pass's cotangent products
  if (b.pw) FN_T(ST_PACK, launch_split_planes(params, p.P, b.pw, b.pw + b.pw_lo, s));
  // orbital weights with zero-padded columns, float32, rows as stored
  std::vector<int64_t> it;
  for (int a = 0; a < 2; ++a) {
    if (p.na(a) == 0) continue;
    const int64_t off = (int64_t)((char*)b.wo[a] - (char*)b.wo[0]) / 4;
    int64_t v[11] = {off, p.d1, b.ldu, 0, (int64_t)p.K * p.na(a), p.offw[a], 0, 0, 0, (int64_t)p.K * p.na(a), 0};
    it.insert(it.end(), v, v + 11);
  }
  if (!it.empty()) FN_T(ST_PACK, launch_pack_weights(false, params, b.wo[0], 0, it.data(), (int)(it.size() / 11), s));
  for (int a = 0; a < 2; ++a)
    if (b.wo_pl[a] && p.na(a) > 0) {
      const int64_t m = (int64_t)p.d1 * b.ldu;
      FN_T(ST_PACK, launch_split_planes(b.wo[a], m, b.wo_pl[a], b.wo_pl[a] + m, s));
    }
  return FN_OK;
}

// the whole adjoint over all chunks: grad = sum_w cot[w] d log|psi_w| / d theta.
// cot_all: per-walker cotangents [W], or nullptr with e_loc/stats for the
// VMC estimator ((E_L - mean) / W, computed chunk by chunk on the device).
// kfac_w (with kout): the KFAC statistics with walker weights kfac_w
// instead of a gradient (grad, cot_all, e_loc and stats unused)
static fn_status run_adjoint(const Plan& p, int32_t W, const float* pos, const float* nuc_pos, const float* nuc_charge,
                             const float* params, const float* cot_all, const float* e_loc, const double* stats,
                             float* grad, void* ws, size_t ws_bytes, hipStream_t s, const float* kfac_w = nullptr,
                             float* kout = nullptr, bool per_walker = false) {
  // the adjoint runs in float32 / split bfloat16 only
  if (p.f64) return FN_ERR_UNSUPPORTED;
  const bool kfac = kout != nullptr;
  const int entry = kfac ? FN_ENTRY_KFAC : FN_ENTRY_GRAD_LOGPSI;
  const int64_t chunk = max_chunk(p, entry, ws_bytes, W);
  if (chunk < 1) return FN_ERR_WORKSPACE;
  Carver cv{(char*)ws, 0};
  void* pk = cv.take(pk_bytes(p));
  AdjBufs b;
  carve_adjoint(p, chunk, cv, b, kfac);
  fn_status st = pack(p, params, pk, s);
  if (st != FN_OK) return st;
  st = adjoint_weights(p, b, params, s);
  if (st != FN_OK) return st;
  if (kfac) {
    int64_t total = 0;
    kfac_blocks(p, &total);
    FN_T(ST_ADJ_REDUCE, launch_fill_f32(kout, total, 0.0f, s));
  } else {
    FN_T(ST_ADJ_REDUCE, launch_fill_f32(grad, per_walker ? (int64_t)W * p.P : p.P, 0.0f, s));
  }
  for (int64_t w0 = 0; w0 < W; w0 += chunk) {
    const int64_t wc = std::min<int64_t>(chunk, W - w0);
    const float* x = pos + w0 * p.n3;
    st = forward_store(p, wc, x, nuc_pos, nuc_charge, params, pk, b, s);
    if (st != FN_OK) return st;
    if (kfac) {
      // cotangents sqrt(c_w): every pre-activation cotangent then carries sqrt(c_w)
      FN_T(ST_ADJ_REDUCE, launch_kfac_sqrt_weights(kfac_w + w0, (int)wc, b.sc, s));
      st = backward(p, wc, x, nuc_pos, params, b.sc, b, nullptr, s, kout);
    } else if (per_walker) {
      // d log|psi_w| / d theta of every walker: unit cotangents, one
      // gradient row [P] per walker
      FN_T(ST_ADJ_REDUCE, launch_fill_f32(b.cot, wc, 1.0f, s));
      st = backward(p, wc, x, nuc_pos, params, b.cot, b, grad + w0 * p.P, s, nullptr, p.P);
    } else {
      const float* cot = cot_all ? cot_all + w0 : b.cot;
      if (!cot_all) FN_T(ST_ADJ_REDUCE, launch_cot_from_stats(e_loc + w0, (int)wc, stats, W, b.cot, s));
      st = backward(p, wc, x, nuc_pos, params, cot, b, grad, s);
    }
    if (st != FN_OK) return st;
  }
  if (kfac)  // the symmetric products formed only their upper tiles
    for (const KfacBlk& k : kfac_blocks(p, nullptr))
      if (k.kind != 1) {
        FN_T(ST_ADJ_REDUCE, launch_sym_mirror(kout + k.offA, k.dA, s));
        FN_T(ST_ADJ_REDUCE, launch_sym_mirror(kout + k.offG, k.dG, s));
      }
  return FN_OK;
}

}  // namespace fn

using namespace fn;

extern "C" {

const char* ferminet_status_string(int32_t st) {
  switch (st) {
    case FN_OK: return "ok";
    case FN_ERR_NULL: return "a required pointer is NULL";
    case FN_ERR_CONFIG: return "configuration out of range";
    case FN_ERR_SPINS: return "spins must be n_up zeros followed by n_down ones";
    case FN_ERR_WORKSPACE: return "workspace too small for one walker, or not 256-byte aligned";
    case FN_ERR_UNSUPPORTED: return "not supported by this build";
    case FN_ERR_HIP: return "HIP launch failed";
    case FN_ERR_ARG: return "invalid argument";
    default: return "unknown status";
  }
}

int64_t ferminet_param_count(const fn_config* cfg) {
  Plan p;
  if (make_plan(cfg, p) != FN_OK) return -1;
  return p.P;
}

fn_status ferminet_param_layout(const fn_config* cfg, fn_param_block* out, int32_t cap, int32_t* n_out) {
  Plan p;
  fn_status st = make_plan(cfg, p);
  if (st != FN_OK) return st;
  if (!n_out || (cap > 0 && !out)) return FN_ERR_NULL;
  std::vector<fn_param_block> v;
  auto add = [&](const char* name, int64_t off, int64_t r, int64_t c) {
    fn_param_block b;
    memset(&b, 0, sizeof(b));
    snprintf(b.name, sizeof(b.name), "%s", name);
    b.offset = off;
    b.rows = r;
    b.cols = c;
    v.push_back(b);
  };
  char nm[16];
  for (int l = 0; l < p.L; ++l) {
    snprintf(nm, 16, "V%d", l);
    add(nm, p.offV[l], 3 * p.din[l] + 2 * p.ein[l], p.d1);
    snprintf(nm, 16, "b%d", l);
    add(nm, p.offb[l], 1, p.d1);
  }
  for (int l = 0; l + 1 < p.L; ++l) {
    snprintf(nm, 16, "W%d", l);
    add(nm, p.offW2[l], p.ein[l], p.d2);
    snprintf(nm, 16, "c%d", l);
    add(nm, p.offc2[l], 1, p.d2);
  }
  for (int a = 0; a < 2; ++a) {
    snprintf(nm, 16, "w_orb%d", a);
    add(nm, p.offw[a], p.d1, (int64_t)p.K * p.na(a));
    snprintf(nm, 16, "g_orb%d", a);
    add(nm, p.offg[a], 1, (int64_t)p.K * p.na(a));
  }
  for (int a = 0; a < 2; ++a) {
    snprintf(nm, 16, "pi%d", a);
    add(nm, p.offpi[a], (int64_t)p.K * p.na(a), p.N);
  }
  for (int a = 0; a < 2; ++a) {
    snprintf(nm, 16, "sigma%d", a);
    add(nm, p.offsg[a], (int64_t)p.K * p.na(a), (int64_t)p.N * (p.env_full ? 9 : 1));
  }
  *n_out = (int32_t)v.size();
  if (cap < (int32_t)v.size()) return FN_ERR_ARG;
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i];
  return FN_OK;
}

fn_status ferminet_workspace_bytes(const fn_config* cfg, int32_t chunk_walkers, int32_t entry, size_t* bytes) {
  Plan p;
  fn_status st = make_plan(cfg, p);
  if (st != FN_OK) return st;
  if (!bytes) return FN_ERR_NULL;
  if (chunk_walkers < 1 || entry < 0 || entry > FN_ENTRY_LOCAL_ENERGY_GRADIENT) return FN_ERR_ARG;
  *bytes = chunk_bytes(p, entry, chunk_walkers);
  return FN_OK;
}

// float64 re-evaluation of the walkers of largest error scale of one chunk
static fn_status reevaluate(const Plan& p, const RescueBufs& r, const Bufs& b, int64_t wc, const float* x,
                            const float* nuc_pos, const float* nuc_charge, const float* params, float* const* outs,
                            hipStream_t s);

// the jet pass of a one-pass layout over all W walkers (its values kept in
// o.ab for the reverse pass) and the float64 re-evaluation; outs: sign,
// logpsi, e_loc, e_kin, e_pot (the last two may be NULL)
static fn_status one_pass_forward(const Plan& p, int64_t W, const float* pos, const float* nuc_pos,
                                  const float* nuc_charge, const float* params, const OnePass& o, float* const* outs,
                                  hipStream_t s) {
  fn_status st = pack(p, params, o.b.pk, s);
  if (st != FN_OK) return st;
  const bool rescue = p.rescue > 0.0f;
  if (rescue) {
    st = pack(o.r.p64, params, o.r.pk64, s);
    if (st != FN_OK) return st;
  }
  st = adjoint_weights(p, o.ab, params, s);
  if (st != FN_OK) return st;
  st = forward(p, JET, W, pos, nuc_pos, nuc_charge, params, o.b, outs[0], outs[1], outs[2], outs[3], outs[4], s, -1,
               &o.ab);
  if (st != FN_OK) return st;
  if (rescue) return reevaluate(p, o.r, o.b, W, pos, nuc_pos, nuc_charge, params, outs, s);
  return FN_OK;
}

// float64 re-evaluation of the walkers of largest error scale of one chunk
// of wc walkers at positions x: their five outputs replace those of outs
static fn_status reevaluate(const Plan& p, const RescueBufs& r, const Bufs& b, int64_t wc, const float* x,
                            const float* nuc_pos, const float* nuc_charge, const float* params, float* const* outs,
                            hipStream_t s) {
  const RescueDims d = rescue_dims(p, wc);
  FN_T(ST_RESCUE, launch_select_top(b.rkey, (int)wc, d.seg_len, d.k_seg, d.k_last, r.idx, s));
  FN_T(ST_RESCUE, launch_gather_walkers(x, r.idx, (int)d.R, p.n3, r.pos_r, s));
  fn_status st = forward(r.p64, JET, d.R, r.pos_r, nuc_pos, nuc_charge, params, r.b, r.out[0], r.out[1], r.out[2],
                         r.out[3], r.out[4], s, ST_RESCUE);
  if (st != FN_OK) return st;
  const float* srcs[5] = {r.out[0], r.out[1], r.out[2], r.out[3], r.out[4]};
  FN_T(ST_RESCUE, launch_scatter_results(r.idx, (int)d.R, outs, srcs, 5, s));
  return FN_OK;
}

static fn_status run_forward_entry(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                   const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                   float* logpsi, float* e_loc, float* e_kin, float* e_pot, void* ws,
                                   size_t ws_bytes, hipStream_t s, bool jet) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, ws, p);
  if (st != FN_OK) return st;
  if (W > 0 && (!sign || !logpsi || (jet && !e_loc))) return FN_ERR_NULL;
  if (W == 0) return FN_OK;
  const int entry = jet ? FN_ENTRY_LOCAL_ENERGY : FN_ENTRY_LOGPSI;
  const int64_t chunk = max_chunk(p, entry, ws_bytes, W);
  if (chunk < 1) return FN_ERR_WORKSPACE;
  Carver cv{(char*)ws, 0};
  Bufs b;
  b.pk = cv.take(pk_bytes(p));
  carve_forward(p, jet ? JET : VALUE, chunk, cv, b, false);
  const bool rescue = jet && p.rescue > 0.0f;
  RescueBufs r;
  if (rescue) {
    carve_rescue(p, chunk, cv, r);
    r.b.pk = r.pk64;
  }
  st = pack(p, params, b.pk, s);
  if (st != FN_OK) return st;
  if (rescue) {
    st = pack(r.p64, params, r.pk64, s);
    if (st != FN_OK) return st;
  }
  for (int64_t w0 = 0; w0 < W; w0 += chunk) {
    const int64_t wc = std::min<int64_t>(chunk, W - w0);
    const float* x = pos + w0 * p.n3;
    float* outs[5] = {sign + w0, logpsi + w0, jet ? e_loc + w0 : nullptr, e_kin ? e_kin + w0 : nullptr,
                      e_pot ? e_pot + w0 : nullptr};
    st = forward(p, jet ? JET : VALUE, wc, x, nuc_pos, nuc_charge, params, b, outs[0], outs[1], outs[2], outs[3],
                 outs[4], s);
    if (st != FN_OK) return st;
    if (!rescue) continue;
    st = reevaluate(p, r, b, wc, x, nuc_pos, nuc_charge, params, outs, s);
    if (st != FN_OK) return st;
  }
  return FN_OK;
}

}  // extern "C"

namespace fn {

// ------------------------------------------- value pass without allocation
// The workspace of ferminet_logpsi_noalloc: a file-scope device array that
// every GPU the library runs on holds until the process ends.  Host code
// never uses the array's name as an address: its device address is looked
// up once per device (hipGetSymbolAddress, with that device current, on
// the entry point's first call there) and that pointer is what the
// launches receive.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices] = {};

static fn_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return FN_ERR_HIP;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FN_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FN_OK;
}

}  // namespace fn

extern "C" {

fn_status ferminet_logpsi_noalloc(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                  const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                  float* logpsi, hipStream_t stream) {
  void* ws = nullptr;
  const fn_status st = scratch_of_current_device(&ws);
  if (st != FN_OK) return st;
  // the value pass writes every workspace element it reads: nothing has to
  // start at zero
  return run_forward_entry(cfg, W, pos, spins, nuc_pos, nuc_charge, params, sign, logpsi, nullptr, nullptr, nullptr,
                           ws, kScratchBytes, stream, false);
}

fn_status ferminet_logpsi(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                          const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                          float* logpsi, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  return run_forward_entry(cfg, W, pos, spins, nuc_pos, nuc_charge, params, sign, logpsi, nullptr, nullptr, nullptr,
                           workspace, workspace_bytes, stream, false);
}

fn_status ferminet_local_energy(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                float* logpsi, float* e_loc, float* e_kin, float* e_pot, void* workspace,
                                size_t workspace_bytes, hipStream_t stream) {
  return run_forward_entry(cfg, W, pos, spins, nuc_pos, nuc_charge, params, sign, logpsi, e_loc, e_kin, e_pot,
                           workspace, workspace_bytes, stream, true);
}

fn_status vmc_mcmc_noise(int32_t W, int32_t n_elec, int32_t n_steps, uint64_t seed, uint64_t counter, float* noise,
                         float* uniforms, hipStream_t stream) {
  if (W < 0 || n_elec < 1 || n_steps < 0) return FN_ERR_ARG;
  if (W == 0 || n_steps == 0) return FN_OK;
  if (!noise || !uniforms) return FN_ERR_NULL;
  if (launch_mcmc_noise(W, n_elec, n_steps, seed, counter, noise, uniforms, stream) != hipSuccess) return FN_ERR_HIP;
  return FN_OK;
}

fn_status vmc_mcmc_step(const fn_config* cfg, int32_t W, float* pos, const int32_t* spins, const float* nuc_pos,
                        const float* nuc_charge, const float* params, float* logpsi, float* sign, int32_t n_steps,
                        float step_width, uint64_t seed, uint64_t counter, const float* noise,
                        const float* uniforms, int32_t* n_accepted, void* workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (n_steps < 0) return FN_ERR_ARG;
  if ((noise == nullptr) != (uniforms == nullptr)) return FN_ERR_ARG;
  if (W > 0 && (!logpsi || !sign || !n_accepted)) return FN_ERR_NULL;
  if (W == 0) return FN_OK;
  const int64_t chunk = max_chunk(p, FN_ENTRY_MCMC, workspace_bytes, W);
  if (chunk < 1) return FN_ERR_WORKSPACE;
  if (n_steps == 0) {
    if (launch_fill_i32(n_accepted, W, 0, stream) != hipSuccess) return FN_ERR_HIP;
    return FN_OK;
  }
  Carver cv{(char*)workspace, 0};
  Bufs b;
  b.pk = cv.take(pk_bytes(p));
  carve_forward(p, VALUE, chunk, cv, b, true);
  st = pack(p, params, b.pk, stream);
  if (st != FN_OK) return st;
  for (int64_t w0 = 0; w0 < W; w0 += chunk) {
    const int64_t wc = std::min<int64_t>(chunk, W - w0);
    float* x = pos + w0 * p.n3;
    for (int step = 0; step < n_steps; ++step) {
      const uint64_t sidx = counter + (uint64_t)step;
      // the counter scheme addresses walkers by their index in the whole
      // batch; the chunk's walkers are drawn with their global indices
      const float* nz = noise ? noise + ((int64_t)step * W + w0) * p.n3 : nullptr;
      const float* un = uniforms ? uniforms + (int64_t)step * W + w0 : nullptr;
      const hipStream_t s = stream;
      FN_T(ST_PROPOSE,
           launch_propose_offset(x, b.prop, (int)wc, p.n3, step_width, seed, sidx, nz, (uint32_t)w0, s));
      st = forward(p, VALUE, wc, b.prop, nuc_pos, nuc_charge, params, b, b.sg_new, b.lp_new, nullptr, nullptr,
                   nullptr, s);
      if (st != FN_OK) return st;
      FN_T(ST_ACCEPT, launch_accept_offset(x, b.prop, logpsi + w0, sign + w0, b.lp_new, b.sg_new, n_accepted + w0,
                                           (int)wc, p.n3, seed, sidx, un, step == 0, (uint32_t)w0, s));
    }
  }
  return FN_OK;
}

fn_status ferminet_grad_logpsi(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                               const float* nuc_pos, const float* nuc_charge, const float* params,
                               const float* cotangent, float* grad, void* workspace, size_t workspace_bytes,
                               hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (!grad) return FN_ERR_NULL;
  if (W == 0) {
    if (cotangent) {
      const hipStream_t s = stream;
      FN_T(ST_ADJ_REDUCE, launch_fill_f32(grad, p.P, 0.0f, s));
    }
    return FN_OK;
  }
  return run_adjoint(p, W, pos, nuc_pos, nuc_charge, params, cotangent, nullptr, nullptr, grad, workspace,
                     workspace_bytes, stream, nullptr, nullptr, cotangent == nullptr);
}

fn_status ferminet_kfac_factors(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                const float* nuc_pos, const float* nuc_charge, const float* params,
                                const float* weights, float* factors, void* workspace, size_t workspace_bytes,
                                hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (!weights || !factors) return FN_ERR_NULL;
  if (p.f64) return FN_ERR_UNSUPPORTED;
  if (W == 0) {
    int64_t total = 0;
    kfac_blocks(p, &total);
    const hipStream_t s = stream;
    FN_T(ST_ADJ_REDUCE, launch_fill_f32(factors, total, 0.0f, s));
    return FN_OK;
  }
  return run_adjoint(p, W, pos, nuc_pos, nuc_charge, params, nullptr, nullptr, nullptr, nullptr, workspace,
                     workspace_bytes, stream, weights, factors);
}

fn_status ferminet_kfac_precondition(const fn_config* cfg, const float* factors, const float* grad, float damping,
                                     float* update, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  Plan p;
  fn_status st = make_plan(cfg, p);
  if (st != FN_OK) return st;
  if (!factors || !grad || !update || !workspace) return FN_ERR_NULL;
  if (!(damping > 0.0f) || !std::isfinite(damping)) return FN_ERR_ARG;
  if (update == grad) return FN_ERR_ARG;
  if (((uintptr_t)workspace & 255) != 0) return FN_ERR_WORKSPACE;
  KfacPrepArgs a;
  memset(&a, 0, sizeof(a));
  Carver cv{(char*)workspace, 0};
  carve_kfac_solve(p, cv, a);
  if (a.nb > KFAC_MAX_BLOCKS) return FN_ERR_UNSUPPORTED;
  if (workspace_bytes < cv.used) return FN_ERR_WORKSPACE;
  // every dense layer's bias row directly follows its weights
  for (int l = 0; l < p.L; ++l)
    if (p.offb[l] != p.offV[l] + (int64_t)(3 * p.din[l] + 2 * p.ein[l]) * p.d1) return FN_ERR_CONFIG;
  a.factors = factors;
  a.grad = grad;
  a.update = update;
  a.S = (double*)workspace;
  a.sqrt_damping = std::sqrt((double)damping);
  const hipStream_t s = stream;
  FN_T(ST_KFAC, launch_copy_f32(grad, update, p.P, s));
  FN_T(ST_KFAC, launch_kfac_prep(a, s));
  SpdBatch ch;
  memset(&ch, 0, sizeof(ch));
  for (int b = 0; b < a.nb; ++b) {
    ch.n[ch.nm] = a.dA[b];
    ch.offI[ch.nm] = a.offIA[b];
    ch.off[ch.nm++] = a.offLA[b];
    ch.n[ch.nm] = a.dG[b];
    ch.offI[ch.nm] = a.offIG[b];
    ch.off[ch.nm++] = a.offLG[b];
  }
  FN_T(ST_KFAC, launch_spd_cholesky(ch, a.S, s));
  SpdBatch sa, sg;
  memset(&sa, 0, sizeof(sa));
  memset(&sg, 0, sizeof(sg));
  for (int b = 0; b < a.nb; ++b) {
    sa.n[b] = a.dA[b];
    sa.m[b] = a.dG[b];
    sa.off[b] = a.offLA[b];
    sa.offI[b] = a.offIA[b];
    sa.offB[b] = a.offY[b];
    sa.offZ[b] = a.offYt[b];  // free until the transpose
    sg.n[b] = a.dG[b];
    sg.m[b] = a.dA[b];
    sg.off[b] = a.offLG[b];
    sg.offI[b] = a.offIG[b];
    sg.offB[b] = a.offYt[b];
    sg.offZ[b] = a.offY[b];  // free after the transpose
  }
  sa.nm = sg.nm = a.nb;
  // Y = A_d^-1 M; Yt = Y^T; Yt = G_d^-1 Yt = (Y G_d^-1)^T
  FN_T(ST_KFAC, launch_spd_solve(sa, a.S, s));
  FN_T(ST_KFAC, launch_kfac_transpose(a, s));
  FN_T(ST_KFAC, launch_spd_solve(sg, a.S, s));
  FN_T(ST_KFAC, launch_kfac_write(a, s));
  return FN_OK;
}

fn_status ferminet_kfac_layout(const fn_config* cfg, fn_kfac_block* out, int32_t cap, int32_t* n_out,
                               int64_t* total) {
  Plan p;
  fn_status st = make_plan(cfg, p);
  if (st != FN_OK) return st;
  if (!n_out || !total || (cap > 0 && !out)) return FN_ERR_NULL;
  int64_t tot = 0;
  const std::vector<KfacBlk> v = kfac_blocks(p, &tot);
  *n_out = (int32_t)v.size();
  *total = tot;
  if (cap < (int32_t)v.size()) return FN_ERR_ARG;
  for (size_t i = 0; i < v.size(); ++i) {
    fn_kfac_block b;
    memset(&b, 0, sizeof(b));
    snprintf(b.name, sizeof(b.name), "%s", v[i].name);
    b.offset_A = v[i].offA;
    b.offset_G = v[i].offG;
    b.dim_A = v[i].dA;
    b.dim_G = v[i].dG;
    b.positions = v[i].npos;
    out[i] = b;
  }
  return FN_OK;
}

fn_status vmc_energy_gradient(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                              const float* nuc_pos, const float* nuc_charge, const float* params,
                              const float* e_loc, double* e_stats, float* grad, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (!e_loc || !e_stats || !grad) return FN_ERR_NULL;
  if (W == 0) return FN_ERR_ARG;  // the batch mean of an empty batch is undefined
  if (max_chunk(p, FN_ENTRY_GRAD_LOGPSI, workspace_bytes, W) < 1) return FN_ERR_WORKSPACE;
  const hipStream_t s = stream;
  FN_T(ST_ADJ_REDUCE, launch_energy_stats(e_loc, W, e_stats, nullptr, s));
  return run_adjoint(p, W, pos, nuc_pos, nuc_charge, params, nullptr, e_loc, e_stats, grad, workspace,
                     workspace_bytes, stream);
}

fn_status vmc_local_energy_gradient(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                                    const float* nuc_pos, const float* nuc_charge, const float* params, float* sign,
                                    float* logpsi, float* e_loc, float* e_kin, float* e_pot, double* e_stats,
                                    float* grad, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (!sign || !logpsi || !e_loc || !e_stats || !grad) return FN_ERR_NULL;
  if (W == 0) return FN_ERR_ARG;  // the batch mean of an empty batch is undefined
  if (p.f64) return FN_ERR_UNSUPPORTED;
  const hipStream_t s = stream;
  if (workspace_bytes < chunk_bytes(p, FN_ENTRY_LOCAL_ENERGY_GRADIENT, W)) {
    // the batch does not fit one pass: the local energy, then the gradient
    // with its own value-only pass, each in chunks
    if (max_chunk(p, FN_ENTRY_LOCAL_ENERGY, workspace_bytes, W) < 1 ||
        max_chunk(p, FN_ENTRY_GRAD_LOGPSI, workspace_bytes, W) < 1)
      return FN_ERR_WORKSPACE;
    st = ferminet_local_energy(cfg, W, pos, spins, nuc_pos, nuc_charge, params, sign, logpsi, e_loc, e_kin, e_pot,
                               workspace, workspace_bytes, stream);
    if (st != FN_OK) return st;
    return vmc_energy_gradient(cfg, W, pos, spins, nuc_pos, nuc_charge, params, e_loc, e_stats, grad, workspace,
                               workspace_bytes, stream);
  }
  Carver cv{(char*)workspace, 0};
  OnePass o;
  carve_one_pass(p, W, cv, o, false);
  float* outs[5] = {sign, logpsi, e_loc, e_kin, e_pot};
  st = one_pass_forward(p, W, pos, nuc_pos, nuc_charge, params, o, outs, s);
  if (st != FN_OK) return st;
  const AdjBufs& ab = o.ab;
  // batch statistics, cotangents (E_L - mean) / W, and the reverse pass
  FN_T(ST_ADJ_REDUCE, launch_energy_stats(e_loc, W, e_stats, ab.cot, s));
  FN_T(ST_ADJ_REDUCE, launch_fill_f32(grad, p.P, 0.0f, s));
  return backward(p, W, pos, nuc_pos, params, ab.cot, ab, grad, s);
}

fn_status vmc_train_step(const fn_config* cfg, int32_t W, float* pos, const int32_t* spins, const float* nuc_pos,
                         const float* nuc_charge, float* params, float* factors, const fn_train_options* options,
                         const float* noise, const float* uniforms, float* e_loc, double* stats, void* workspace,
                         size_t workspace_bytes, hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (!options || !factors || !e_loc || !stats) return FN_ERR_NULL;
  if (W < 1) return FN_ERR_ARG;  // the batch statistics of an empty batch are undefined
  if (p.f64) return FN_ERR_UNSUPPORTED;
  const fn_train_options o = *options;
  if (o.mcmc_steps < 0 || !std::isfinite(o.mcmc_width) || !(o.learning_rate > 0.0f) ||
      !std::isfinite(o.learning_rate) || !(o.damping > 0.0f) || !std::isfinite(o.damping) ||
      !std::isfinite(o.norm_constraint) || !(o.factor_decay >= 0.0f && o.factor_decay <= 1.0f) ||
      !std::isfinite(o.clip_scale))
    return FN_ERR_ARG;
  if ((noise == nullptr) != (uniforms == nullptr)) return FN_ERR_ARG;
  Carver cv{(char*)workspace, 0};
  TrainBufs t;
  carve_train(p, W, cv, t);
  if (workspace_bytes < cv.used) return FN_ERR_WORKSPACE;
  void* rest = (char*)workspace + cv.used;
  const size_t rb = workspace_bytes - cv.used;
  // every pass must fit (in chunks) before anything is enqueued
  if (rb < chunk_bytes(p, FN_ENTRY_KFAC_PRECONDITION, 1)) return FN_ERR_WORKSPACE;
  for (int e = FN_ENTRY_LOGPSI; e <= FN_ENTRY_KFAC; ++e)
    if (max_chunk(p, e, rb, W) < 1) return FN_ERR_WORKSPACE;
  int64_t total = 0;
  kfac_blocks(p, &total);
  const hipStream_t s = stream;
  // log|psi| of the walkers under the current parameters, then the moves
  st = ferminet_logpsi(cfg, W, pos, spins, nuc_pos, nuc_charge, params, t.sign, t.logpsi, rest, rb, s);
  if (st != FN_OK) return st;
  st = vmc_mcmc_step(cfg, W, pos, spins, nuc_pos, nuc_charge, params, t.logpsi, t.sign, o.mcmc_steps, o.mcmc_width,
                     o.seed, o.counter, noise, uniforms, t.n_acc, rest, rb, s);
  if (st != FN_OK) return st;
  if (rb >= one_pass_bytes(p, W, true)) {
    // one pass: the local energy's jet pass keeps its values for the two
    // reverse passes (energy gradient and KFAC statistics)
    Carver cp{(char*)rest, 0};
    OnePass op;
    carve_one_pass(p, W, cp, op, true);
    float* outs[5] = {t.sign, t.logpsi, e_loc, nullptr, nullptr};
    st = one_pass_forward(p, W, pos, nuc_pos, nuc_charge, params, op, outs, s);
    if (st != FN_OK) return st;
    FN_T(ST_TRAIN, launch_train_energy_stats(e_loc, t.n_acc, W, o.mcmc_steps, (double)o.clip_scale, t.e_clip,
                                             t.cot, t.wts, stats, s));
    FN_T(ST_ADJ_REDUCE, launch_fill_f32(t.grad, p.P, 0.0f, s));
    st = backward(p, W, pos, nuc_pos, params, t.cot, op.ab, t.grad, s);
    if (st != FN_OK) return st;
    FN_T(ST_ADJ_REDUCE, launch_fill_f32(t.fb, total, 0.0f, s));
    FN_T(ST_ADJ_REDUCE, launch_kfac_sqrt_weights(t.wts, W, op.ab.sc, s));
    st = backward(p, W, pos, nuc_pos, params, op.ab.sc, op.ab, nullptr, s, t.fb);
    if (st != FN_OK) return st;
    for (const KfacBlk& k : kfac_blocks(p, nullptr))
      if (k.kind != 1) {
        FN_T(ST_ADJ_REDUCE, launch_sym_mirror(t.fb + k.offA, k.dA, s));
        FN_T(ST_ADJ_REDUCE, launch_sym_mirror(t.fb + k.offG, k.dG, s));
      }
  } else {
    st = ferminet_local_energy(cfg, W, pos, spins, nuc_pos, nuc_charge, params, t.sign, t.logpsi, e_loc, nullptr,
                               nullptr, rest, rb, s);
    if (st != FN_OK) return st;
    // energy statistics over the walkers with a finite local energy, the
    // cotangents 2 (E~_w - mean E~) / W_f and the KFAC batch weights 1 / W_f
    // (both 0 for the others)
    FN_T(ST_TRAIN, launch_train_energy_stats(e_loc, t.n_acc, W, o.mcmc_steps, (double)o.clip_scale, t.e_clip,
                                             t.cot, t.wts, stats, s));
    // energy gradient 2 sum_w (E~_w - mean E~) / W_f d log|psi_w| / d theta
    st = ferminet_grad_logpsi(cfg, W, pos, spins, nuc_pos, nuc_charge, params, t.cot, t.grad, rest, rb, s);
    if (st != FN_OK) return st;
    // the batch factors
    st = ferminet_kfac_factors(cfg, W, pos, spins, nuc_pos, nuc_charge, params, t.wts, t.fb, rest, rb, s);
    if (st != FN_OK) return st;
  }
  // running averages of the batch factors
  FN_T(ST_TRAIN, launch_lincomb(factors, t.fb, 1.0f - o.factor_decay, o.factor_decay, total, s));
  st = ferminet_kfac_precondition(cfg, factors, t.grad, o.damping, t.dir, rest, rb, s);
  if (st != FN_OK) return st;
  FN_T(ST_TRAIN, launch_step_length(t.dir, t.grad, p.P, (double)o.learning_rate, (double)o.norm_constraint, t.part,
                                    stats, s));
  FN_T(ST_TRAIN, launch_apply_step(params, t.dir, p.P, stats, s));
  return FN_OK;
}

}  // extern "C"

extern "C" {

fn_status ferminet_set_option(int32_t option, int32_t value) {
  if (option != FN_OPT_FUSED_MEANFIELD || (value != 0 && value != 1)) return FN_ERR_ARG;
  fn::g_fused_meanfield.store(value != 0);
  return FN_OK;
}

fn_status ferminet_stage_timing(int32_t enable) {
  std::lock_guard<std::mutex> g(fn::g_time_mu);
  for (auto& r : fn::g_recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  fn::g_recs.clear();
  fn::g_timing = enable != 0;
  return FN_OK;
}

int32_t ferminet_stage_times(double* total_ms, int32_t* count, int32_t cap) {
  std::lock_guard<std::mutex> g(fn::g_time_mu);
  if (!total_ms || !count || cap < fn::ST_COUNT) return -1;
  for (int i = 0; i < fn::ST_COUNT; ++i) {
    total_ms[i] = 0.0;
    count[i] = 0;
  }
  for (auto& r : fn::g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      total_ms[r.stage] += ms;
      count[r.stage] += 1;
    }
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  fn::g_recs.clear();
  return fn::ST_COUNT;
}

const char* ferminet_stage_name(int32_t stage) {
  if (stage < 0 || stage >= fn::ST_COUNT) return "";
  return fn::kStageNames[stage];
}

}  // extern "C"
