// FP64 CPU oracle for the FermiNet variational Monte Carlo hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
// load this file.  Only the tests, the smoke check and the bench's CPU
// baseline use it.  It shares no code, header, table or helper with the
// HIP library; the two agree only on the documented interfaces (the
// flat parameter layout, the Philox counter scheme and the noise
// transform), each written out independently.
//
// What it computes, in double precision, with the plain definitions:
//   * psi = sum_k det[phi^{k,up}] det[phi^{k,down}]                (Eq. 4,
//     with the determinant weights omega_k removed as Section 3 argues)
//   * phi^{k,a}_i(r_j) = (w^{k,a}_i . h^L_j + g^{k,a}_i) *
//        sum_m pi^{k,a}_{im} exp(-|sigma^{k,a}_{im}| |r_j - R_m|)   (Eq. 5,
//     isotropic envelope of Section 3), or with a 3x3 matrix Sigma_{im}
//     and exp(-|Sigma_{im} (r_j - R_m)|) (Eq. 5 as written: the full
//     covariance envelope that Section 3 replaces)
//   * h^L from the permutation-equivariant one/two-electron network of
//     the original FermiNet, which the paper does not restate: tanh
//     layers with a residual connection when the widths match, spin-wise
//     mean fields that include the electron itself, two-electron features
//     (r_i - r_j, |r_i - r_j|) that are zero at i == j
//   * E_L = psi^{-1} H psi with H from Eq. (2), evaluated as
//       -1/2 sum_c [d^2_c log|psi| + (d_c log|psi|)^2] + V
//     where each second derivative along one of the 3n coordinates comes
//     from one forward pass in a second-order jet number (value, first and
//     second derivative along that single coordinate).  No multi-tangent
//     jet algebra, no blocking, no split-form shortcuts.
//   * d log|psi| / d theta_p, one dual-number pass per selected parameter.
//   * for the Kronecker-factored curvature statistics (KFAC, Martens and
//     Grosse 2015, the optimiser the paper uses): the inputs of every dense
//     layer at every position (electron, electron pair), and the
//     derivative of log|psi| with respect to each pre-activation at each
//     position, one dual-number pass per (position, unit) with a unit
//     derivative added to that pre-activation.
//   * Metropolis sampling of psi^2 (Eq. 3), replayed from supplied noise
//     or from the Philox4x32-10 generator (Salmon et al., SC'11).
//
// Parity of the full network is pinned only through invariants, closed
// forms, brute force and finite differences (the paper prints no worked
// example).  See tests/test_oracle_pins.py.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#include <omp.h>

namespace {

// ---------------------------------------------------------------- numbers
// Dual: value and derivative along one parameter direction.
struct Dual {
  double v, d;
};
// Jet2: value, first and second derivative along one coordinate.
struct Jet2 {
  double v, d, dd;
};

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double val(const Jet2& x) { return x.v; }

// a derivative of 1 in the direction a dual-number pass probes
template <class S> inline S probe_unit();
template <> inline double probe_unit<double>() { return 0.0; }
template <> inline Dual probe_unit<Dual>() { return {0.0, 1.0}; }
template <> inline Jet2 probe_unit<Jet2>() { return {0.0, 0.0, 0.0}; }

template <class S> inline S cst(double c);
template <> inline double cst<double>(double c) { return c; }
template <> inline Dual cst<Dual>(double c) { return {c, 0.0}; }
template <> inline Jet2 cst<Jet2>(double c) { return {c, 0.0, 0.0}; }

// chain rule for a scalar function with value f, f' = f1, f'' = f2 at x.v
inline double chain(double, double f, double, double) { return f; }
inline Dual chain(const Dual& x, double f, double f1, double) { return {f, f1 * x.d}; }
inline Jet2 chain(const Jet2& x, double f, double f1, double f2) {
  return {f, f1 * x.d, f2 * x.d * x.d + f1 * x.dd};
}

inline Dual operator+(const Dual& a, const Dual& b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(const Dual& a, const Dual& b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator*(const Dual& a, const Dual& b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator+(const Dual& a, double b) { return {a.v + b, a.d}; }
inline Dual operator-(const Dual& a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, const Dual& b) { return {a - b.v, -b.d}; }
inline Dual operator*(const Dual& a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator*(double b, const Dual& a) { return {a.v * b, a.d * b}; }
inline Dual operator-(const Dual& a) { return {-a.v, -a.d}; }

inline Jet2 operator+(const Jet2& a, const Jet2& b) { return {a.v + b.v, a.d + b.d, a.dd + b.dd}; }
inline Jet2 operator-(const Jet2& a, const Jet2& b) { return {a.v - b.v, a.d - b.d, a.dd - b.dd}; }
inline Jet2 operator*(const Jet2& a, const Jet2& b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d, a.dd * b.v + 2.0 * a.d * b.d + a.v * b.dd};
}
inline Jet2 operator+(const Jet2& a, double b) { return {a.v + b, a.d, a.dd}; }
inline Jet2 operator-(const Jet2& a, double b) { return {a.v - b, a.d, a.dd}; }
inline Jet2 operator-(double a, const Jet2& b) { return {a - b.v, -b.d, -b.dd}; }
inline Jet2 operator*(const Jet2& a, double b) { return {a.v * b, a.d * b, a.dd * b}; }
inline Jet2 operator*(double b, const Jet2& a) { return {a.v * b, a.d * b, a.dd * b}; }
inline Jet2 operator-(const Jet2& a) { return {-a.v, -a.d, -a.dd}; }

template <class S> inline S tanh_(const S& x) {
  double t = std::tanh(val(x));
  return chain(x, t, 1.0 - t * t, -2.0 * t * (1.0 - t * t));
}
template <class S> inline S exp_(const S& x) {
  double e = std::exp(val(x));
  return chain(x, e, e, e);
}
template <class S> inline S sqrt_(const S& x) {
  double s = std::sqrt(val(x));
  return chain(x, s, 0.5 / s, -0.25 / (s * s * s));
}
template <class S> inline S log_abs(const S& x) {
  double v = val(x);
  return chain(x, std::log(std::fabs(v)), 1.0 / v, -1.0 / (v * v));
}
template <class S> inline S inv_(const S& x) {
  double v = val(x);
  return chain(x, 1.0 / v, -1.0 / (v * v), 2.0 / (v * v * v));
}
template <class S> inline S abs_(const S& x) { return val(x) < 0.0 ? -x : x; }

// ------------------------------------------------------------- the shapes
// env: 0 isotropic envelope (one sigma per orbital and nucleus), 1 full
// covariance (a 3x3 matrix Sigma per orbital and nucleus, row-major)
struct Cfg {
  int n, n_up, n_dn, N, L, d1, d2, K, env;
};

Cfg read_cfg(const int32_t* c) { return {c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], c[8]}; }

// Offsets of the parameter blocks in the flat vector.  The layout is an
// interface fixed by the library's header; it is written out here anew.
struct Layout {
  std::vector<int64_t> V, b, W2, c2;  // per layer
  int64_t w_orb[2], g_orb[2], pi[2], sg[2];
  int64_t total;
};

int din_of(const Cfg& c, int l) { return l == 0 ? 4 * c.N : c.d1; }
int ein_of(const Cfg& c, int l) { return l == 0 ? 4 : c.d2; }
int nspin(const Cfg& c, int a) { return a == 0 ? c.n_up : c.n_dn; }

Layout make_layout(const Cfg& c) {
  Layout Y;
  int64_t off = 0;
  for (int l = 0; l < c.L; ++l) {
    int din = din_of(c, l), ein = ein_of(c, l);
    Y.V.push_back(off);
    off += (int64_t)(3 * din + 2 * ein) * c.d1;
    Y.b.push_back(off);
    off += c.d1;
  }
  for (int l = 0; l + 1 < c.L; ++l) {
    int ein = ein_of(c, l);
    Y.W2.push_back(off);
    off += (int64_t)ein * c.d2;
    Y.c2.push_back(off);
    off += c.d2;
  }
  for (int a = 0; a < 2; ++a) {
    int no = c.K * nspin(c, a);
    Y.w_orb[a] = off;
    off += (int64_t)c.d1 * no;
    Y.g_orb[a] = off;
    off += no;
  }
  for (int a = 0; a < 2; ++a) {
    Y.pi[a] = off;
    off += (int64_t)c.K * nspin(c, a) * c.N;
  }
  for (int a = 0; a < 2; ++a) {
    Y.sg[a] = off;
    off += (int64_t)c.K * nspin(c, a) * c.N * (c.env ? 9 : 1);
  }
  Y.total = off;
  return Y;
}

// ------------------------------------------------------------ determinant
// sign and log|det A| by LU with partial pivoting on the value part.
// A is n x n row-major and is overwritten.  n == 0 gives (1, 0).
template <class S>
void slogdet(int n, S* a, double* sign, S* logabs) {
  double sg = 1.0;
  S la = cst<S>(0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = std::fabs(val(a[col * n + col]));
    for (int r = col + 1; r < n; ++r) {
      double m = std::fabs(val(a[r * n + col]));
      if (m > best) {
        best = m;
        piv = r;
      }
    }
    if (best == 0.0) {
      *sign = 0.0;
      *logabs = cst<S>(-std::numeric_limits<double>::infinity());
      return;
    }
    if (piv != col) {
      for (int k = 0; k < n; ++k) std::swap(a[col * n + k], a[piv * n + k]);
      sg = -sg;
    }
    S p = a[col * n + col];
    S ip = inv_(p);
    for (int r = col + 1; r < n; ++r) {
      S f = a[r * n + col] * ip;
      for (int k = col + 1; k < n; ++k) a[r * n + k] = a[r * n + k] - f * a[col * n + k];
    }
    if (val(p) < 0.0) sg = -sg;
    la = la + log_abs(p);
  }
  *sign = sg;
  *logabs = la;
}

// ------------------------------------------------------------ the network
// One evaluation of sign(psi) and log|psi| for one walker.
//   S: type of positions and activations; P: type of the parameters.
// pos: [n][3]; nuc: [N][3] (plain doubles: nuclei are fixed, Section 1's
// Born-Oppenheimer setting); prm: the flat parameter vector.
// Optional instrumentation of eval_walker: records the inputs of the dense
// layers (values) and adds probe_unit to one pre-activation.
//   probe kind 0: one-electron layer `layer`, electron `pos`, unit `unit`
//   probe kind 1: two-electron layer `layer`, pair pos = i n + j, unit
//   probe kind 2: orbital pre-envelope value u of electron `pos` (spin
//                 implied), column `unit` = k n_a + i of that spin
struct Taps {
  int kind = -1, layer = 0, pos = 0, unit = 0;
  double* rec1 = nullptr;  // [L][n][fw_max]: f_i of one-electron layer l
  double* rec2 = nullptr;  // [L-1][n n][ein_max]: h_ij entering two-electron layer l
  double* reco = nullptr;  // [n][d1]: h^L_j entering the orbitals
  int fw_max = 0, ein_max = 0;
};

template <class S, class P>
void eval_walker(const Cfg& c, const Layout& Y, const S* pos, const double* nuc, const P* prm,
                 double* sign_out, S* logabs_out, double* sk_out = nullptr, double* lk_out = nullptr,
                 double* orb_out = nullptr, const Taps* tp = nullptr) {
  const int n = c.n, N = c.N;
  // spin of electron j: up for j < n_up (the caller orders spins up first)
  auto spin_of = [&](int j) { return j < c.n_up ? 0 : 1; };
  const int nsp[2] = {c.n_up, c.n_dn};

  // input features: h_i = concat_I (r_i - R_I, |r_i - R_I|);
  //                 h_ij = (r_i - r_j, |r_i - r_j|), identically 0 at i == j.
  int din = 4 * N, ein = 4;
  std::vector<S> h1((size_t)n * din), h2((size_t)n * n * ein);
  for (int i = 0; i < n; ++i)
    for (int I = 0; I < N; ++I) {
      S d[3];
      for (int x = 0; x < 3; ++x) d[x] = pos[i * 3 + x] - nuc[I * 3 + x];
      S r = sqrt_(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int x = 0; x < 3; ++x) h1[(size_t)i * din + 4 * I + x] = d[x];
      h1[(size_t)i * din + 4 * I + 3] = r;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      S* o = &h2[((size_t)i * n + j) * ein];
      if (i == j) {
        for (int x = 0; x < 4; ++x) o[x] = cst<S>(0.0);
        continue;
      }
      S d[3];
      for (int x = 0; x < 3; ++x) d[x] = pos[i * 3 + x] - pos[j * 3 + x];
      for (int x = 0; x < 3; ++x) o[x] = d[x];
      o[3] = sqrt_(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }

  // L one-electron layers, L-1 two-electron layers
  for (int l = 0; l < c.L; ++l) {
    din = din_of(c, l);
    ein = ein_of(c, l);
    const int fw = 3 * din + 2 * ein;
    // mean fields: hbar^a = mean_{j in a} h_j ; g^a_i = mean_{j in a} h_ij
    std::vector<S> hbar((size_t)2 * din, cst<S>(0.0));
    for (int j = 0; j < n; ++j) {
      int a = spin_of(j);
      for (int f = 0; f < din; ++f) hbar[(size_t)a * din + f] = hbar[(size_t)a * din + f] + h1[(size_t)j * din + f];
    }
    for (int a = 0; a < 2; ++a)
      if (nsp[a] > 0)
        for (int f = 0; f < din; ++f) hbar[(size_t)a * din + f] = hbar[(size_t)a * din + f] * (1.0 / nsp[a]);
    std::vector<S> nh1((size_t)n * c.d1);
    std::vector<S> fvec(fw);
    const P* V = prm + Y.V[l];
    const P* b = prm + Y.b[l];
    for (int i = 0; i < n; ++i) {
      // f_i = [h_i, hbar^up, hbar^down, g^up_i, g^down_i]
      for (int f = 0; f < din; ++f) fvec[f] = h1[(size_t)i * din + f];
      for (int f = 0; f < 2 * din; ++f) fvec[din + f] = hbar[f];
      for (int a = 0; a < 2; ++a) {
        for (int f = 0; f < ein; ++f) {
          S s = cst<S>(0.0);
          for (int j = 0; j < n; ++j)
            if (spin_of(j) == a) s = s + h2[((size_t)i * n + j) * ein + f];
          fvec[3 * din + a * ein + f] = nsp[a] > 0 ? s * (1.0 / nsp[a]) : cst<S>(0.0);
        }
      }
      if (tp && tp->rec1)
        for (int k = 0; k < fw; ++k) tp->rec1[((size_t)l * n + i) * tp->fw_max + k] = val(fvec[k]);
      for (int o = 0; o < c.d1; ++o) {
        // pre = b_o + sum_k f_k V[k][o]
        S acc = cst<S>(0.0);
        for (int k = 0; k < fw; ++k) acc = acc + fvec[k] * V[(size_t)k * c.d1 + o];
        S pre = acc + b[o];
        if (tp && tp->kind == 0 && tp->layer == l && tp->pos == i && tp->unit == o) pre = pre + probe_unit<S>();
        S y = tanh_(pre);
        if (din == c.d1) y = y + h1[(size_t)i * din + o];
        nh1[(size_t)i * c.d1 + o] = y;
      }
    }
    if (l + 1 < c.L) {
      const P* W2 = prm + Y.W2[l];
      const P* c2 = prm + Y.c2[l];
      std::vector<S> nh2((size_t)n * n * c.d2);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const S* x = &h2[((size_t)i * n + j) * ein];
          if (tp && tp->rec2)
            for (int k = 0; k < ein; ++k) tp->rec2[((size_t)l * n * n + i * n + j) * tp->ein_max + k] = val(x[k]);
          for (int o = 0; o < c.d2; ++o) {
            S acc = cst<S>(0.0);
            for (int k = 0; k < ein; ++k) acc = acc + x[k] * W2[(size_t)k * c.d2 + o];
            S z = acc + c2[o];
            if (tp && tp->kind == 1 && tp->layer == l && tp->pos == i * n + j && tp->unit == o) z = z + probe_unit<S>();
            S y = tanh_(z);
            if (ein == c.d2) y = y + x[o];
            nh2[((size_t)i * n + j) * c.d2 + o] = y;
          }
        }
      h2.swap(nh2);
    }
    h1.swap(nh1);
  }

  // orbitals and determinants: A^{k,a}_{ij} = phi^{k,a}_i(r^a_j)
  const int d1 = c.d1;
  if (tp && tp->reco)
    for (size_t q = 0; q < (size_t)n * d1; ++q) tp->reco[q] = val(h1[q]);
  std::vector<double> sgn_k(c.K, 1.0);
  std::vector<S> log_k(c.K, cst<S>(0.0));
  int j0 = 0;
  for (int a = 0; a < 2; ++a) {
    const int na = nsp[a];
    const int no = c.K * na;
    const P* wo = prm + Y.w_orb[a];
    const P* go = prm + Y.g_orb[a];
    const P* pi = prm + Y.pi[a];
    const P* sg = prm + Y.sg[a];
    std::vector<S> A((size_t)na * na);
    for (int k = 0; k < c.K; ++k) {
      for (int i = 0; i < na; ++i) {
        const int col = k * na + i;
        for (int j = 0; j < na; ++j) {
          const int e = j0 + j;
          S u = cst<S>(0.0);
          for (int f = 0; f < d1; ++f) u = u + h1[(size_t)e * d1 + f] * wo[(size_t)f * no + col];
          u = u + go[col];
          if (tp && tp->kind == 2 && tp->pos == e && tp->unit == col) u = u + probe_unit<S>();
          S env = cst<S>(0.0);
          for (int m = 0; m < N; ++m) {
            S d[3];
            for (int x = 0; x < 3; ++x) d[x] = pos[e * 3 + x] - nuc[m * 3 + x];
            S arg;
            if (c.env == 0) {
              // |sigma (r - R)| = |sigma| |r - R|
              S r = sqrt_(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
              P s_abs = abs_(sg[(size_t)col * N + m]);
              arg = r * s_abs;
            } else {
              // |Sigma (r - R)|, the Euclidean norm of the 3-vector
              const P* Sg = sg + ((size_t)col * N + m) * 9;
              S u[3];
              for (int x = 0; x < 3; ++x) u[x] = Sg[3 * x] * d[0] + Sg[3 * x + 1] * d[1] + Sg[3 * x + 2] * d[2];
              arg = sqrt_(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            }
            env = env + exp_(-arg) * pi[(size_t)col * N + m];
          }
          A[(size_t)i * na + j] = u * env;
        }
      }
      if (orb_out) {
        // orbital matrices of the value pass, [K][n_up^2] then [K][n_down^2]
        double* o = orb_out + (a == 0 ? 0 : (size_t)c.K * c.n_up * c.n_up) + (size_t)k * na * na;
        for (int e = 0; e < na * na; ++e) o[e] = val(A[e]);
      }
      double s;
      S la;
      slogdet(na, A.data(), &s, &la);
      sgn_k[k] *= s;
      log_k[k] = log_k[k] + la;
    }
    j0 += na;
  }

  if (sk_out)
    for (int k = 0; k < c.K; ++k) {
      sk_out[k] = sgn_k[k];
      lk_out[k] = val(log_k[k]);
    }
  // psi = sum_k s_k exp(l_k), taken as a signed log-sum-exp
  double m = -std::numeric_limits<double>::infinity();
  for (int k = 0; k < c.K; ++k)
    if (sgn_k[k] != 0.0) m = std::max(m, val(log_k[k]));
  if (m == -std::numeric_limits<double>::infinity()) {
    *sign_out = 0.0;
    *logabs_out = cst<S>(-std::numeric_limits<double>::infinity());
    return;
  }
  S sum = cst<S>(0.0);
  for (int k = 0; k < c.K; ++k)
    if (sgn_k[k] != 0.0) sum = sum + exp_(log_k[k] - m) * sgn_k[k];
  double sv = val(sum);
  *sign_out = sv > 0.0 ? 1.0 : (sv < 0.0 ? -1.0 : 0.0);
  *logabs_out = log_abs(sum) + m;
}

// V of Eq. (2): electron-electron, electron-nucleus, nucleus-nucleus
void potential(const Cfg& c, const double* pos, const double* nuc, const double* Z, double* v_out) {
  double ee = 0.0, en = 0.0, nn = 0.0;
  for (int i = 0; i < c.n; ++i)
    for (int j = i + 1; j < c.n; ++j) {
      double dx = pos[i * 3] - pos[j * 3], dy = pos[i * 3 + 1] - pos[j * 3 + 1], dz = pos[i * 3 + 2] - pos[j * 3 + 2];
      ee += 1.0 / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  for (int i = 0; i < c.n; ++i)
    for (int I = 0; I < c.N; ++I) {
      double dx = pos[i * 3] - nuc[I * 3], dy = pos[i * 3 + 1] - nuc[I * 3 + 1], dz = pos[i * 3 + 2] - nuc[I * 3 + 2];
      en -= Z[I] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  for (int I = 0; I < c.N; ++I)
    for (int J = I + 1; J < c.N; ++J) {
      double dx = nuc[I * 3] - nuc[J * 3], dy = nuc[I * 3 + 1] - nuc[J * 3 + 1], dz = nuc[I * 3 + 2] - nuc[J * 3 + 2];
      nn += Z[I] * Z[J] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  v_out[0] = ee;
  v_out[1] = en;
  v_out[2] = nn;
}

bool cfg_ok(const Cfg& c) {
  return c.n >= 1 && c.n_up >= 0 && c.n_dn >= 0 && c.n_up + c.n_dn == c.n && c.N >= 1 && c.L >= 1 && c.d1 >= 1 &&
         c.d2 >= 1 && c.K >= 1 && (c.env == 0 || c.env == 1);
}

// ------------------------------------------------------------- Philox
// Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11):
// ten rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule.
void philox(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
    if (r < 9) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// uniform in (0, 1) from the top 23 bits: ((x >> 9) + 1/2) * 2^-23
double unit_uniform(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

// Counter scheme (the library's header states the same scheme):
//   key = (seed low 32 bits, seed high 32 bits)
//   proposal normals of walker w at step s, block b (coordinates 4b..4b+3):
//     counter = (w, b, s_lo, s_hi)        -> Box-Muller on (u0,u1), (u2,u3)
//   acceptance uniform: counter = (w, 0x80000000, s_lo, s_hi) -> u from word 0
//   where s = counter_base + step.
void draw_noise(uint64_t seed, uint64_t step, int w, int ncoord, double* z, double* u) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const double two_pi = 6.283185307179586476925286766559;
  for (int b = 0; 4 * b < ncoord; ++b) {
    uint32_t ctr[4] = {(uint32_t)w, (uint32_t)b, (uint32_t)step, (uint32_t)(step >> 32)};
    uint32_t o[4];
    philox(ctr, key, o);
    for (int p = 0; p < 2; ++p) {
      double u1 = unit_uniform(o[2 * p]), u2 = unit_uniform(o[2 * p + 1]);
      double rad = std::sqrt(-2.0 * std::log(u1));
      double z0 = rad * std::cos(two_pi * u2), z1 = rad * std::sin(two_pi * u2);
      int q = 4 * b + 2 * p;
      if (q < ncoord) z[q] = z0;
      if (q + 1 < ncoord) z[q + 1] = z1;
    }
  }
  uint32_t ctr[4] = {(uint32_t)w, 0x80000000u, (uint32_t)step, (uint32_t)(step >> 32)};
  uint32_t o[4];
  philox(ctr, key, o);
  *u = unit_uniform(o[0]);
}

}  // namespace

extern "C" {

int64_t orc_param_count(const int32_t* cfg) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  return make_layout(c).total;
}

// offsets of the blocks in layout order (V,b per layer; W2,c2 per
// two-electron layer; w,g per spin; pi per spin; sigma per spin)
int orc_param_offsets(const int32_t* cfg, int64_t* out, int cap) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  std::vector<int64_t> v;
  for (int l = 0; l < c.L; ++l) {
    v.push_back(Y.V[l]);
    v.push_back(Y.b[l]);
  }
  for (int l = 0; l + 1 < c.L; ++l) {
    v.push_back(Y.W2[l]);
    v.push_back(Y.c2[l]);
  }
  for (int a = 0; a < 2; ++a) {
    v.push_back(Y.w_orb[a]);
    v.push_back(Y.g_orb[a]);
  }
  for (int a = 0; a < 2; ++a) v.push_back(Y.pi[a]);
  for (int a = 0; a < 2; ++a) v.push_back(Y.sg[a]);
  v.push_back(Y.total);
  if ((int)v.size() > cap) return -(int)v.size();
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i];
  return (int)v.size();
}

int orc_slogdet(int n, const double* a, double* sign, double* logabs) {
  std::vector<double> m(a, a + (size_t)n * n);
  slogdet(n, m.data(), sign, logabs);
  return 0;
}

// sign, log|psi| and (if want_energy) E_L, its kinetic and potential parts
// and d log|psi| / d r (grad_pos, nullable) for W walkers.
int orc_eval(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* Z, const double* prm,
             int want_energy, int n_threads, double* sign, double* logpsi, double* e_loc, double* e_kin,
             double* e_pot, double* grad_pos) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  const int nc = 3 * c.n;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int w = 0; w < W; ++w) {
    const double* p = pos + (size_t)w * nc;
    double s;
    double la;
    eval_walker<double, double>(c, Y, p, nuc, prm, &s, &la);
    sign[w] = s;
    logpsi[w] = la;
    if (!want_energy) continue;
    double lap = 0.0, g2 = 0.0;
    std::vector<Jet2> x(nc);
    for (int q = 0; q < nc; ++q) {
      for (int r = 0; r < nc; ++r) x[r] = {p[r], r == q ? 1.0 : 0.0, 0.0};
      double sj;
      Jet2 lj;
      eval_walker<Jet2, double>(c, Y, x.data(), nuc, prm, &sj, &lj);
      lap += lj.dd;
      g2 += lj.d * lj.d;
      if (grad_pos) grad_pos[(size_t)w * nc + q] = lj.d;
    }
    double v[3];
    potential(c, p, nuc, Z, v);
    // E_L = (H psi) / psi is undefined where psi = 0 exactly (the jets of a
    // vanishing determinant carry no information): NaN
    double kin = s == 0.0 ? std::numeric_limits<double>::quiet_NaN() : -0.5 * (lap + g2);
    double pot = v[0] + v[1] + v[2];
    if (e_kin) e_kin[w] = kin;
    if (e_pot) e_pot[w] = pot;
    e_loc[w] = kin + pot;
  }
  return 0;
}

// potential terms (ee, en, nn) per walker: out [W][3]
int orc_potential(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* Z, double* out) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  for (int w = 0; w < W; ++w) potential(c, pos + (size_t)w * 3 * c.n, nuc, Z, out + 3 * w);
  return 0;
}

// d log|psi_w| / d theta_p for the n_sel parameters listed in sel:
// out [W][n_sel].  One dual-number pass per (walker, parameter).
int orc_param_grad(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* prm, int n_sel,
                   const int64_t* sel, int n_threads, double* out) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  const int nc = 3 * c.n;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
  for (int w = 0; w < W; ++w)
    for (int s = 0; s < n_sel; ++s) {
      std::vector<Dual> th(Y.total);
      for (int64_t q = 0; q < Y.total; ++q) th[q] = {prm[q], 0.0};
      th[sel[s]].d = 1.0;
      std::vector<Dual> x(nc);
      for (int r = 0; r < nc; ++r) x[r] = {pos[(size_t)w * nc + r], 0.0};
      double sg;
      Dual la;
      eval_walker<Dual, Dual>(c, Y, x.data(), nuc, th.data(), &sg, &la);
      out[(size_t)w * n_sel + s] = la.d;
    }
  return 0;
}

// Inputs of the dense layers, per walker (values):
//   f1 [W][L][n][fw_max]   f_i = [h_i, hbar^up, hbar^down, g^up_i, g^down_i]
//                          of one-electron layer l (zero-padded to fw_max)
//   f2 [W][L-1][n n][ein_max]  h_ij entering two-electron layer l
//   fo [W][n][d1]          h^L_j entering the orbitals
// fw_max = 3 max(din) + 2 max(ein), ein_max = max(4, d2).
int orc_layer_inputs(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* prm,
                     int n_threads, double* f1, double* f2, double* fo) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  const int n = c.n, nc = 3 * n;
  const int ein_max = std::max(4, c.d2), fw_max = 3 * std::max(4 * c.N, c.d1) + 2 * ein_max;
  const size_t s1 = (size_t)c.L * n * fw_max, s2 = (size_t)std::max(c.L - 1, 0) * n * n * ein_max;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int w = 0; w < W; ++w) {
    Taps tp;
    tp.rec1 = f1 + (size_t)w * s1;
    tp.rec2 = f2 + (size_t)w * s2;
    tp.reco = fo + (size_t)w * n * c.d1;
    tp.fw_max = fw_max;
    tp.ein_max = ein_max;
    std::fill(tp.rec1, tp.rec1 + s1, 0.0);
    std::fill(tp.rec2, tp.rec2 + s2, 0.0);
    double sg;
    double la;
    eval_walker<double, double>(c, Y, pos + (size_t)w * nc, nuc, prm, &sg, &la, nullptr, nullptr, nullptr, &tp);
  }
  return 0;
}

// d log|psi_w| / d z at every position and unit of one dense layer, one
// dual-number pass each: out [W][positions][units] with
//   kind 0: one-electron layer `layer`: n electrons x d1 units
//   kind 1: two-electron layer `layer`: n^2 pairs (i n + j) x d2 units
//   kind 2: orbitals of spin `layer`: its n_a electrons x K n_a columns
int orc_preact_cotangents(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* prm,
                          int kind, int layer, int n_threads, double* out) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  const int n = c.n, nc = 3 * n;
  int P, U, e0 = 0;
  if (kind == 0) {
    if (layer < 0 || layer >= c.L) return -1;
    P = n;
    U = c.d1;
  } else if (kind == 1) {
    if (layer < 0 || layer + 1 >= c.L) return -1;
    P = n * n;
    U = c.d2;
  } else if (kind == 2) {
    if (layer < 0 || layer > 1) return -1;
    P = nspin(c, layer);
    U = c.K * P;
    e0 = layer == 0 ? 0 : c.n_up;
  } else {
    return -1;
  }
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) collapse(3)
  for (int w = 0; w < W; ++w)
    for (int p = 0; p < P; ++p)
      for (int u = 0; u < U; ++u) {
        Taps tp;
        tp.kind = kind;
        tp.layer = layer;
        tp.pos = kind == 2 ? e0 + p : p;
        tp.unit = u;
        std::vector<Dual> x(nc);
        for (int r = 0; r < nc; ++r) x[r] = {pos[(size_t)w * nc + r], 0.0};
        double sg;
        Dual la;
        eval_walker<Dual, double>(c, Y, x.data(), nuc, prm, &sg, &la, nullptr, nullptr, nullptr, &tp);
        out[((size_t)w * P + p) * U + u] = la.d;
      }
  return 0;
}

// sign and log|det^up_k det^down_k| of every determinant term of Eq. (4):
// sk, lk [W][K]
int orc_det_terms(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* prm, int n_threads,
                  double* sk, double* lk) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int w = 0; w < W; ++w) {
    double s, la;
    eval_walker<double, double>(c, Y, pos + (size_t)w * 3 * c.n, nuc, prm, &s, &la, sk + (size_t)w * c.K,
                                lk + (size_t)w * c.K);
  }
  return 0;
}

// the orbital matrices A^{k,a}_{ij} = phi^{k,a}_i(r^a_j) of Eq. (4)-(5):
// out [W][K n_up^2 + K n_down^2], spin up first, row-major per matrix
int orc_orbitals(const int32_t* cfg, int W, const double* pos, const double* nuc, const double* prm, int n_threads,
                 double* out) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  const size_t per = (size_t)c.K * (c.n_up * c.n_up + c.n_dn * c.n_dn);
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int w = 0; w < W; ++w) {
    double s, la;
    eval_walker<double, double>(c, Y, pos + (size_t)w * 3 * c.n, nuc, prm, &s, &la, nullptr, nullptr,
                                out + (size_t)w * per);
  }
  return 0;
}

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

// the proposal noise [n_steps][W][3n] and acceptance uniforms [n_steps][W]
// that a Metropolis call with (seed, counter) draws
int orc_mcmc_noise(int W, int n, int n_steps, uint64_t seed, uint64_t counter, double* noise, double* uniforms) {
  const int nc = 3 * n;
  for (int s = 0; s < n_steps; ++s)
    for (int w = 0; w < W; ++w)
      draw_noise(seed, counter + (uint64_t)s, w, nc, noise + ((size_t)s * W + w) * nc, uniforms + (size_t)s * W + w);
  return 0;
}

// Metropolis random walk on psi^2 (Eq. 3's sampling): for each step,
// x' = x + width * z; accept when log u < 2 (log|psi(x')| - log|psi(x)|).
// noise/uniforms: supplied draws ([n_steps][W][3n], [n_steps][W]) or NULL to
// draw them from Philox with (seed, counter).  pos, logpsi, sign are
// updated in place; n_accepted[w] counts accepted moves.
int orc_mcmc(const int32_t* cfg, int W, double* pos, const double* nuc, const double* prm, int n_steps, double width,
             const double* noise, const double* uniforms, uint64_t seed, uint64_t counter, int n_threads,
             double* logpsi, double* sign, int32_t* n_accepted) {
  Cfg c = read_cfg(cfg);
  if (!cfg_ok(c)) return -1;
  Layout Y = make_layout(c);
  const int nc = 3 * c.n;
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int w = 0; w < W; ++w) {
    double* x = pos + (size_t)w * nc;
    std::vector<double> xp(nc), z(nc);
    int acc = 0;
    for (int s = 0; s < n_steps; ++s) {
      double u;
      if (noise) {
        for (int q = 0; q < nc; ++q) z[q] = noise[((size_t)s * W + w) * nc + q];
        u = uniforms[(size_t)s * W + w];
      } else {
        draw_noise(seed, counter + (uint64_t)s, w, nc, z.data(), &u);
      }
      for (int q = 0; q < nc; ++q) xp[q] = x[q] + width * z[q];
      double sp, lp;
      eval_walker<double, double>(c, Y, xp.data(), nuc, prm, &sp, &lp);
      bool ok = sp != 0.0 && std::log(u) < 2.0 * (lp - logpsi[w]);
      if (ok) {
        for (int q = 0; q < nc; ++q) x[q] = xp[q];
        logpsi[w] = lp;
        sign[w] = sp;
        ++acc;
      }
    }
    n_accepted[w] = acc;
  }
  return 0;
}

}  // extern "C"
