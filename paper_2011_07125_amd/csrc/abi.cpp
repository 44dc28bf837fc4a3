// Host side of libferminet: argument validation, the workspace plan, walker
// chunking and the launch sequence of every entry point of ferminet.h.
// Everything here is bookkeeping; all arithmetic of the method runs in the
// HIP kernels.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/ferminet.h"
#include "common.h"
#include "kernels.h"

namespace fn {

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
  int n, nu, nd, N, L, d1, d2, K, n3;
  bool bf16, fp64;
  size_t act;  // bytes per activation element
  int din[8], ein[8], dinp[8], gwp[8];
  int64_t offV[8], offb[8], offW2[8], offc2[8], offw[2], offg[2], offpi[2], offsg[2], P;
  // packed weights (elements, activation type)
  int64_t pk_main[8], pk_mf[8], pk_orb[2], pk_total;
  int ld_main[8], ld_mf[8];
  int na(int a) const { return a == 0 ? nu : nd; }
};

static fn_status make_plan(const fn_config* c, Plan& p) {
  if (!c) return FN_ERR_NULL;
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
  if (c->precision != FN_PREC_FP32 && c->precision != FN_PREC_BF16 && c->precision != FN_PREC_FP32_FP64DET)
    return FN_ERR_CONFIG;
  {
    // the two-electron stream keeps one electron's 8-row pair jets in LDS
    const int d2p = p.d2 <= 4 ? 4 : p.d2 <= 8 ? 8 : p.d2 <= 16 ? 16 : p.d2 <= 32 ? 32 : 64;
    if ((p.n * 8 * d2p + d2p * d2p + d2p) * 4 > 65536) return FN_ERR_CONFIG;
  }
  p.bf16 = c->precision == FN_PREC_BF16;
  p.fp64 = c->precision != FN_PREC_FP32;
  p.act = 4;  // activations are float32 in HBM in every form
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
    off += (int64_t)p.K * p.na(a) * p.N;
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

// the packing plan: [dst_off, N, ldb, k0, len0, src0, k1, len1, src1, src_ld]
static int pack_plan(const Plan& p, std::vector<int64_t>& it) {
  it.clear();
  auto add = [&](int64_t dst, int64_t N, int64_t ldb, int64_t k0, int64_t l0, int64_t s0, int64_t k1, int64_t l1,
                 int64_t s1, int64_t sld) {
    int64_t v[10] = {dst, N, ldb, k0, l0, s0, k1, l1, s1, sld};
    it.insert(it.end(), v, v + 10);
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
  return (int)(it.size() / 10);
}

// ----------------------------------------------------------- workspace
enum Mode { VALUE = 0, JET = 1 };
enum Stage {
  ST_PACK, ST_FEATURES, ST_TWO_E, ST_MEANFIELD, ST_GEMM_MF, ST_GEMM_LAYER, ST_GEMM_ORB, ST_DET, ST_COMBINE,
  ST_PROPOSE, ST_ACCEPT, ST_ADJ_FWD, ST_ADJ_DET, ST_ADJ_ORB, ST_ADJ_LAYERS, ST_ADJ_TWO_E, ST_ADJ_REDUCE,
  ST_GEMM_LAYER_VALUE, ST_COUNT
};

struct Bufs {
  void* pk;
  void* H0;
  void* G[8];
  void* Ha;
  void* Hb;
  void* Hbar;
  float* Pm;
  float* phi[2];
  void* D[2];
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
  b.dstride = m == JET ? p.n3 + 4 : 2;
  const int64_t rows = Wc * p.n * b.Tp;
  b.H0 = cv.take((size_t)rows * p.dinp[0] * p.act);
  for (int l = 0; l < p.L; ++l) b.G[l] = cv.take((size_t)rows * p.gwp[l] * p.act);
  b.Ha = cv.take((size_t)rows * p.d1 * p.act);
  b.Hb = cv.take((size_t)rows * p.d1 * p.act);
  int dmax = 0;
  for (int l = 0; l < p.L; ++l) dmax = std::max(dmax, p.dinp[l]);
  b.Hbar = cv.take((size_t)Wc * b.Tp * 2 * dmax * p.act);
  b.Pm = (float*)cv.take((size_t)Wc * b.Tp * p.d1 * 4);
  const size_t rb = p.fp64 ? 8 : 4;
  for (int a = 0; a < 2; ++a) {
    b.phi[a] = (float*)cv.take((size_t)Wc * p.K * b.T * p.na(a) * p.na(a) * 4);
    b.D[a] = cv.take((size_t)Wc * p.K * b.dstride * rb);
  }
  if (mcmc) {
    b.prop = (float*)cv.take((size_t)Wc * p.n3 * 4);
    b.lp_new = (float*)cv.take((size_t)Wc * 4);
    b.sg_new = (float*)cv.take((size_t)Wc * 4);
  } else {
    b.prop = b.lp_new = b.sg_new = nullptr;
  }
}

static size_t chunk_bytes(const Plan& p, int entry, int64_t Wc) {
  Carver cv{nullptr, 0};
  Bufs b;
  cv.take((size_t)p.pk_total * p.act);
  carve_forward(p, entry == FN_ENTRY_LOCAL_ENERGY ? JET : VALUE, Wc, cv, b, entry == FN_ENTRY_MCMC);
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
    "adj_det",      "adj_orbital", "adj_layers", "adj_two_electron", "adj_reduce",     "gemm_layer_value"};
static std::mutex g_time_mu;
static bool g_timing = false;
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
  FN_T(ST_PACK, launch_pack_weights(p.bf16, params, dst, p.pk_total, it.data(), n, s));
  return FN_OK;
}

// packed weight block at element offset off: float32, or the bfloat16 hi
// plane (lo = false) / lo plane (lo = true) in the split form
static const void* wt(const Bufs& b, const Plan& p, int64_t off, bool lo) {
  if (!p.bf16) return lo ? nullptr : (const char*)b.pk + off * 4;
  return (const char*)b.pk + (off + (lo ? p.pk_total : 0)) * 2;
}

// forward pass over one chunk of Wc walkers.  jet: local energy; value:
// sign and log|psi| only.
static fn_status forward(const Plan& p, Mode m, int64_t Wc, const float* pos, const float* nuc, const float* Z,
                         const float* params, const Bufs& b, float* sign, float* logpsi, float* e_loc,
                         float* e_kin, float* e_pot, hipStream_t s) {
  const int T = b.T, Tp = b.Tp;
  FN_T(ST_FEATURES, launch_features(false, pos, nuc, (int)Wc, p.n, p.N, T, Tp, b.H0, p.dinp[0], s));
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
  }
  FN_T(ST_TWO_E, launch_two_electron(false, te, s));
  const void* Hin = b.H0;
  void* Hout = b.Ha;
  for (int l = 0; l < p.L; ++l) {
    FN_T(ST_MEANFIELD, launch_meanfield(false, Hin, p.dinp[l], (int)Wc, p.n, p.nu, Tp, p.dinp[l], b.Hbar, s));
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
    FN_T(ST_GEMM_MF, launch_jet_gemm(p.bf16 ? MODE_BF16X3 : MODE_F32, EPI_PLAIN, g, s));
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
    FN_T(m == JET ? ST_GEMM_LAYER : ST_GEMM_LAYER_VALUE, launch_jet_gemm(p.bf16 ? MODE_BF16X3 : MODE_F32, EPI_TANHJET, h, s));
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
    o.bt = wt(b, p, p.pk_orb[a], false);
    o.bt_lo = wt(b, p, p.pk_orb[a], true);
    o.ldb = p.d1;
    o.n_groups = (int)(Wc * na);
    o.rows_per = Tp;
    o.T = T;
    o.n_sub = na;
    o.n_all = p.n;
    o.e_off = a == 0 ? 0 : p.nu;
    o.N = p.K * na;
    o.phi = b.phi[a];
    o.pos = pos;
    o.nuc = nuc;
    o.n_nuc = p.N;
    o.n_elec = p.n;
    o.g_orb = params + p.offg[a];
    o.pi = params + p.offpi[a];
    o.sigma = params + p.offsg[a];
    FN_T(ST_GEMM_ORB, launch_jet_gemm(p.bf16 ? MODE_BF16X3 : MODE_F32, EPI_ORBITAL, o, s));
    FN_T(ST_DET, launch_det(p.fp64, b.phi[a], (int)Wc, p.K, na, T, p.n3, b.D[a], b.dstride, nullptr, s));
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
  FN_T(ST_COMBINE, launch_combine(p.fp64, cb, s));
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
    add(nm, p.offsg[a], (int64_t)p.K * p.na(a), p.N);
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
  if (chunk_walkers < 1 || entry < 0 || entry > 3) return FN_ERR_ARG;
  *bytes = chunk_bytes(p, entry, chunk_walkers);
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
  b.pk = cv.take((size_t)p.pk_total * p.act);
  carve_forward(p, jet ? JET : VALUE, chunk, cv, b, false);
  st = pack(p, params, b.pk, s);
  if (st != FN_OK) return st;
  for (int64_t w0 = 0; w0 < W; w0 += chunk) {
    const int64_t wc = std::min<int64_t>(chunk, W - w0);
    st = forward(p, jet ? JET : VALUE, wc, pos + w0 * p.n3, nuc_pos, nuc_charge, params, b, sign + w0, logpsi + w0,
                 jet ? e_loc + w0 : nullptr, e_kin ? e_kin + w0 : nullptr, e_pot ? e_pot + w0 : nullptr, s);
    if (st != FN_OK) return st;
  }
  return FN_OK;
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
  b.pk = cv.take((size_t)p.pk_total * p.act);
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
  if (!cotangent || !grad) return FN_ERR_NULL;
  return FN_ERR_UNSUPPORTED;
}

fn_status vmc_energy_gradient(const fn_config* cfg, int32_t W, const float* pos, const int32_t* spins,
                              const float* nuc_pos, const float* nuc_charge, const float* params,
                              const float* e_loc, double* e_stats, float* grad, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
  Plan p;
  fn_status st = check_common(cfg, W, pos, spins, nuc_pos, nuc_charge, params, workspace, p);
  if (st != FN_OK) return st;
  if (!e_loc || !e_stats || !grad) return FN_ERR_NULL;
  return FN_ERR_UNSUPPORTED;
}

}  // extern "C"

extern "C" {

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
