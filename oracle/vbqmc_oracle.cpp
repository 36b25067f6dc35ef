// Test infrastructure, not part of the product: a plain, slow FP64 CPU oracle
// for the Jastrow-Valence-Bond (JVB) wave function and its VMC/DMC walks.
//
// Only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
// It shares no code with the GPU library: it does its own HLSP expansion of
// the VB structures, evaluates every determinant of every structure from
// scratch with a partial-pivot LU, and never uses inverse updates.
//
// Paper passages followed (Radenkovic, Domin, Toulouse, Braida, "The
// Valence-Bond Quantum Monte Carlo Method", 2022):
//   Sec. 2.1, Eq. (PsiJVBSCF): Psi_0 = J * sum_I c_I Phi_I.
//   Sec. 2.1, Eq. (PhiI): HLSP structures from inactive, singlet-paired and
//     unpaired active orbitals; expansion into 2^{N_pairs} determinants.
//   Sec. 2.1: orbitals phi_p = sum_mu lambda_{p,mu} chi_mu; Gaussian / Slater
//     basis functions.
//   Sec. 2.1: Jastrow J = exp(f_en + f_ee + f_een), scaled variables
//     R(r) = r / (1 + kappa r) and Rbar(r) = 1 / (1 + kappa r), Pade plus
//     R^p polynomial pair terms and the electron-electron-nucleus expansion
//     in Rbar (optional: a system without its coefficients has no f_een).
//   Sec. 2.3.1, Eq. (Elav): local energy E_L = H Psi / Psi, spins fixed,
//     Metropolis-Hastings sampling of Psi^2.
//   Sec. 2.3.2, Eq. (E0DMCweights): fixed-node DMC with weighted walkers and a
//     birth/death process.
//   Sec. 2.2, Eq. (PsiJVBp) and Eq. (H0j): parameter derivatives of ln Psi and
//     of E_L (forward-mode dual numbers here).
// Readings where the paper is silent are listed in the design notes: spin
// assignment, determinant sign convention, self-pair factor, Hamiltonian,
// Metropolis proposal law, random-number layout, DMC move and branching rules.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -shared -fPIC

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Dual numbers (value + one tangent) for forward-mode parameter derivatives.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}  // NOLINT: implicit from a constant
  Dual(double x, double y) : v(x), d(y) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return {e, a.d * e}; }
inline Dual log_abs(Dual a) { return {std::log(std::fabs(a.v)), a.d / a.v}; }
inline double val(Dual a) { return a.v; }
inline double tangent(Dual a) { return a.d; }

inline double exp(double a) { return std::exp(a); }
inline double log_abs(double a) { return std::log(std::fabs(a)); }
inline double val(double a) { return a; }
inline double tangent(double) { return 0.0; }

template <class T> inline T powi(T x, int p) {
  T r = T(1.0);
  for (int k = 0; k < p; ++k) r = r * x;
  return r;
}

// ---------------------------------------------------------------------------
// The system (what the caller describes) and its expanded determinant list.
// ---------------------------------------------------------------------------
struct Det {
  int structure;            // I
  std::vector<int> up, dn;  // orbital index per slot, in slot order
};

struct System {
  int nnuc = 0;
  std::vector<double> Z, pos;  // pos[3*a + x]
  int nup = 0, ndn = 0, N = 0;
  // shells
  int nshell = 0;
  std::vector<int> sh_center, sh_kind, sh_l, sh_nprim, sh_off, sh_fn;
  std::vector<double> pexp, pcoef;
  int M = 0, norb = 0;
  std::vector<double> lam;  // norb x M
  int nstruct = 0;
  std::vector<double> c;
  std::vector<Det> dets;
  // Jastrow
  double kappa = 0;
  double ee_a_anti = 0, ee_a_par = 0;
  std::vector<double> jas;  // [b_anti, b_par, b3..b6 | per nucleus a1..a6 | per nucleus f_een c_t]
  int njas = 0;
  bool een = false;         // f_een present (its coefficients close jas)
  // semilocal pseudopotentials: per centre the nucleus, r_cut and the radial
  // parts (local, then channel l = 0, 1, ..) as [c, n, alpha] triples
  struct EcpCentre {
    int center = 0;
    double rcut = 0;
    std::vector<std::vector<double>> parts;
  };
  std::vector<EcpCentre> ecp;
  int nparam() const { return nstruct + norb * M + njas; }
};

int nfunc_of_l(int l) { return l == 0 ? 1 : (l == 1 ? 3 : 5); }

// Eq. (PhiI) expansion.  Each singlet pair of distinct orbitals (i, j) is
// a+_{i up} a+_{j dn} - a+_{i dn} a+_{j up} = a+_{i up} a+_{j dn} + a+_{j up} a+_{i dn},
// so every choice of orientation enters with +1 when each pair slot is written
// as (up orbital, down orbital).  Reordering the operator string into all up
// operators followed by all down operators costs a sign that depends only on
// the electron counts, which are the same for every structure; it is dropped.
// A self-pair (i, i) gives one determinant; its factor 2 is a normalisation
// constant and is dropped (structures are unnormalised).
void expand_term(int I, const int* inact, int ninact, const int* pairs, int npair,
                 const int* unp, int nunp, std::vector<Det>& out) {
  std::vector<int> distinct;
  for (int k = 0; k < npair; ++k)
    if (pairs[2 * k] != pairs[2 * k + 1]) distinct.push_back(k);
  int nchoice = 1 << distinct.size();
  for (int mask = 0; mask < nchoice; ++mask) {
    Det d;
    d.structure = I;
    for (int k = 0; k < ninact; ++k) {
      d.up.push_back(inact[k]);
      d.dn.push_back(inact[k]);
    }
    for (int k = 0; k < npair; ++k) {
      int i = pairs[2 * k], j = pairs[2 * k + 1];
      bool flip = false;
      for (size_t q = 0; q < distinct.size(); ++q)
        if (distinct[q] == k && ((mask >> q) & 1)) flip = true;
      d.up.push_back(flip ? j : i);
      d.dn.push_back(flip ? i : j);
    }
    for (int k = 0; k < nunp; ++k) d.up.push_back(unp[k]);
    out.push_back(d);
  }
}

// ---------------------------------------------------------------------------
// Parameters that derivatives are taken with respect to, in scalar type T.
// ---------------------------------------------------------------------------
template <class T> struct Params {
  std::vector<T> c, lam, jas;
};

template <class T> Params<T> make_params(const System& s, int seed_index) {
  Params<T> p;
  p.c.assign(s.c.begin(), s.c.end());
  p.lam.assign(s.lam.begin(), s.lam.end());
  p.jas.assign(s.jas.begin(), s.jas.end());
  return p;
}

template <> Params<Dual> make_params<Dual>(const System& s, int seed_index) {
  Params<Dual> p;
  for (double x : s.c) p.c.push_back(Dual(x));
  for (double x : s.lam) p.lam.push_back(Dual(x));
  for (double x : s.jas) p.jas.push_back(Dual(x));
  int k = seed_index;
  if (k >= 0 && k < s.nstruct) p.c[k].d = 1.0;
  k -= s.nstruct;
  if (k >= 0 && k < s.norb * s.M) p.lam[k].d = 1.0;
  k -= s.norb * s.M;
  if (k >= 0 && k < s.njas) p.jas[k].d = 1.0;
  return p;
}

// ---------------------------------------------------------------------------
// Basis functions (Sec. 2.1): chi = P_lm(d) g(|d|), d = r - A.
// Channels: 0 value, 1..3 gradient, 4 Laplacian; out[c * M + mu].
// Plain product rule: d2 chi / dx_a^2 = P_aa g + 2 P_a g_a + P g_aa.
// ---------------------------------------------------------------------------
void angular(int l, int m, const double d[3], double& P, double dP[3], double d2P[3]) {
  double x = d[0], y = d[1], z = d[2];
  for (int a = 0; a < 3; ++a) { dP[a] = 0; d2P[a] = 0; }
  if (l == 0) { P = 1; return; }
  if (l == 1) { P = d[m]; dP[m] = 1; return; }
  switch (m) {
    case 0: P = x * y; dP[0] = y; dP[1] = x; break;
    case 1: P = y * z; dP[1] = z; dP[2] = y; break;
    case 2: P = z * x; dP[2] = x; dP[0] = z; break;
    case 3: P = x * x - y * y; dP[0] = 2 * x; dP[1] = -2 * y; d2P[0] = 2; d2P[1] = -2; break;
    default:
      P = 3 * z * z - (x * x + y * y + z * z);
      dP[0] = -2 * x; dP[1] = -2 * y; dP[2] = 4 * z;
      d2P[0] = -2; d2P[1] = -2; d2P[2] = 4;
  }
}

void eval_ao(const System& s, const double r[3], double* out) {
  for (int sh = 0; sh < s.nshell; ++sh) {
    const double* A = &s.pos[3 * s.sh_center[sh]];
    double d[3] = {r[0] - A[0], r[1] - A[1], r[2] - A[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double rr = std::sqrt(r2);
    // radial value g, first derivatives g_a, second derivatives g_aa
    double g = 0, ga[3] = {0, 0, 0}, gaa[3] = {0, 0, 0};
    for (int k = 0; k < s.sh_nprim[sh]; ++k) {
      double a = s.pexp[s.sh_off[sh] + k], cf = s.pcoef[s.sh_off[sh] + k];
      if (s.sh_kind[sh] == 0) {  // Gaussian: exp(-a r^2)
        double e = cf * std::exp(-a * r2);
        g += e;
        for (int x = 0; x < 3; ++x) {
          ga[x] += -2 * a * d[x] * e;
          gaa[x] += (-2 * a + 4 * a * a * d[x] * d[x]) * e;
        }
      } else {  // Slater: exp(-a r)
        double e = cf * std::exp(-a * rr);
        g += e;
        for (int x = 0; x < 3; ++x) {
          ga[x] += -a * d[x] / rr * e;
          gaa[x] += (a * a * d[x] * d[x] / r2 - a * (1.0 / rr - d[x] * d[x] / (r2 * rr))) * e;
        }
      }
    }
    int nf = nfunc_of_l(s.sh_l[sh]);
    for (int m = 0; m < nf; ++m) {
      int mu = s.sh_fn[sh] + m;
      double P, dP[3], d2P[3];
      angular(s.sh_l[sh], m, d, P, dP, d2P);
      out[0 * s.M + mu] = P * g;
      double lap = 0;
      for (int x = 0; x < 3; ++x) {
        out[(1 + x) * s.M + mu] = dP[x] * g + P * ga[x];
        lap += d2P[x] * g + 2 * dP[x] * ga[x] + P * gaa[x];
      }
      out[4 * s.M + mu] = lap;
    }
  }
}

// ---------------------------------------------------------------------------
// Determinant by partial-pivot LU, with the inverse by forward/back solves.
// A is n x n row-major, A[i*n + j]: row i = electron, column j = slot.
// ---------------------------------------------------------------------------
template <class T>
bool lu_det_inverse(int n, std::vector<T> A, T& logabs, int& sign, std::vector<T>& inv) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  sign = 1;
  logabs = T(0.0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(val(A[i * n + k])) > std::fabs(val(A[p * n + k]))) p = i;
    if (val(A[p * n + k]) == 0.0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[p * n + j], A[k * n + j]);
      std::swap(perm[p], perm[k]);
      sign = -sign;
    }
    T piv = A[k * n + k];
    if (val(piv) < 0) sign = -sign;
    logabs = logabs + log_abs(piv);
    for (int i = k + 1; i < n; ++i) {
      T l = A[i * n + k] / piv;
      A[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[i * n + j] = A[i * n + j] - l * A[k * n + j];
    }
  }
  // inverse: solve (P A) X = P, i.e. column e of A^{-1} solves L U x = P e.
  inv.assign(n * n, T(0.0));
  std::vector<T> x(n);
  for (int col = 0; col < n; ++col) {
    for (int i = 0; i < n; ++i) x[i] = T(perm[i] == col ? 1.0 : 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) x[i] = x[i] - A[i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) x[i] = x[i] - A[i * n + j] * x[j];
      x[i] = x[i] / A[i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[i * n + col] = x[i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Pair functions of the Jastrow factor (Sec. 2.1):
// u(r) = a R / (1 + b R) + sum_{p=2..5} q_p R^p, R = r / (1 + kappa r).
// Returns u, du/dr, d2u/dr2.
// ---------------------------------------------------------------------------
template <class T>
void pair_u(double r, double kappa, T a, T b, const T* q, T& u, T& u1, T& u2) {
  double den = 1.0 + kappa * r;
  double R = r / den, R1 = 1.0 / (den * den), R2 = -2.0 * kappa / (den * den * den);
  T bb = T(1.0) + b * R;
  T uR = a / (bb * bb);
  T uRR = T(-2.0) * a * b / (bb * bb * bb);
  u = a * R / bb;
  for (int p = 2; p <= 5; ++p) {
    u = u + q[p - 2] * std::pow(R, p);
    uR = uR + q[p - 2] * (p * std::pow(R, p - 1));
    uRR = uRR + q[p - 2] * (p * (p - 1) * std::pow(R, p - 2));
  }
  u1 = uR * R1;
  u2 = uRR * (R1 * R1) + uR * R2;
}

// ---------------------------------------------------------------------------
// Electron-electron-nucleus terms f_een (Sec. 2.1).  For p = 2..5,
// k = 0..p-1 and l = 0..l_max, l_max = p - k for k > 0 and p - k - 2 for
// k = 0, the terms with m = (p - k - l) / 2 a whole number, in that loop
// order; term t of nucleus alpha contributes, for every electron pair i < j,
//   c_{t,alpha} Rbar(r_ij)^k [Rbar(r_ia)^l + Rbar(r_ja)^l] [Rbar(r_ia) Rbar(r_ja)]^m.
// ---------------------------------------------------------------------------
struct EenTerm {
  int k, l, m;
};

std::vector<EenTerm> een_terms() {
  std::vector<EenTerm> t;
  for (int p = 2; p <= 5; ++p)
    for (int k = 0; k < p; ++k) {
      int lmax = k > 0 ? p - k : p - k - 2;
      for (int l = 0; l <= lmax; ++l)
        if ((p - k - l) % 2 == 0) t.push_back({k, l, (p - k - l) / 2});
    }
  return t;
}

// Second-order jets along one coordinate direction: value, first and second
// derivative in the displacement t of one electron (the Laplacian of f_een is
// the sum of the second derivatives over the three axes).
struct Jet {
  double v, d, dd;
};
inline Jet jmul(Jet a, Jet b) { return {a.v * b.v, a.d * b.v + a.v * b.d, a.dd * b.v + 2 * a.d * b.d + a.v * b.dd}; }
inline Jet jadd(Jet a, Jet b) { return {a.v + b.v, a.d + b.d, a.dd + b.dd}; }
inline Jet jpow(Jet a, int n) {
  Jet r{1.0, 0.0, 0.0};
  for (int q = 0; q < n; ++q) r = jmul(r, a);
  return r;
}
inline Jet jsqrt(Jet a) {
  double s = std::sqrt(a.v);
  return {s, a.d / (2 * s), a.dd / (2 * s) - a.d * a.d / (4 * s * a.v)};
}
inline Jet jinv(Jet a) {  // 1 / a
  double i = 1.0 / a.v;
  return {i, -a.d * i * i, -a.dd * i * i + 2 * a.d * a.d * i * i * i};
}

// Rbar(|x - y|) as a jet: x moves along axis `ax` with x(t) = x + t e_ax
// (mv = true), or stays (mv = false); y is fixed.
Jet rbar_jet(const double* x, const double* y, int ax, bool mv, double kappa) {
  Jet q{0.0, 0.0, 0.0};
  for (int c = 0; c < 3; ++c) {
    double dv = x[c] - y[c];
    Jet e{dv, (mv && c == ax) ? 1.0 : 0.0, 0.0};
    q = jadd(q, jmul(e, e));
  }
  Jet r = jsqrt(q);
  return jinv({1.0 + kappa * r.v, kappa * r.d, kappa * r.dd});
}

// sum over the terms of nucleus alpha for one pair: a = Rbar(r_ij),
// b = Rbar(r_ia), c = Rbar(r_ja); coefficients cf[t]
template <class T>
void een_pair(const std::vector<EenTerm>& terms, Jet a, Jet b, Jet c, const T* cf, T& v, T& d, T& dd) {
  Jet bc = jmul(b, c);
  for (size_t t = 0; t < terms.size(); ++t) {
    const EenTerm& e = terms[t];
    Jet f = jmul(jmul(jpow(a, e.k), jadd(jpow(b, e.l), jpow(c, e.l))), jpow(bc, e.m));
    v = v + cf[t] * f.v;
    d = d + cf[t] * f.d;
    dd = dd + cf[t] * f.dd;
  }
}

// f_een of the configuration (U), and per electron its gradient and
// Laplacian (added into gU, lU) when want_derivs.
template <class T>
void een_all(const System& s, const T* cf, const double* R, bool want_derivs, T& U, std::vector<T>& gU,
             std::vector<T>& lU) {
  const std::vector<EenTerm> terms = een_terms();
  const int nt = (int)terms.size(), N = s.N;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j)
      for (int a = 0; a < s.nnuc; ++a) {
        const double* A = &s.pos[3 * a];
        Jet ra = rbar_jet(&R[3 * i], &R[3 * j], 0, false, s.kappa);
        Jet rb = rbar_jet(&R[3 * i], A, 0, false, s.kappa);
        Jet rc = rbar_jet(&R[3 * j], A, 0, false, s.kappa);
        T v = T(0.0), d = T(0.0), dd = T(0.0);
        een_pair(terms, ra, rb, rc, cf + nt * a, v, d, dd);
        U = U + v;
      }
  if (!want_derivs) return;
  // derivatives in electron i: every pair (i, j), j != i, each nucleus
  for (int i = 0; i < N; ++i)
    for (int ax = 0; ax < 3; ++ax) {
      T d = T(0.0), dd = T(0.0);
      for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        for (int a = 0; a < s.nnuc; ++a) {
          const double* A = &s.pos[3 * a];
          Jet ra = rbar_jet(&R[3 * i], &R[3 * j], ax, true, s.kappa);
          Jet rb = rbar_jet(&R[3 * i], A, ax, true, s.kappa);
          Jet rc = rbar_jet(&R[3 * j], A, ax, false, s.kappa);
          T v = T(0.0);
          een_pair(terms, ra, rb, rc, cf + nt * a, v, d, dd);
        }
      }
      gU[3 * i + ax] = gU[3 * i + ax] + d;
      lU[i] = lU[i] + dd;
    }
}

// ---------------------------------------------------------------------------
// Full evaluation of one configuration.
// level 0: ln|Psi| and sign; 1: + gradient; 2: + local energy.
// ---------------------------------------------------------------------------
template <class T> struct EvalOut {
  T logabs;
  int sign = 0;
  std::vector<T> grad;    // N x 3
  T eloc;
  std::vector<T> ratio;   // nstruct: Phi_I / sum_J c_J Phi_J
  T kin, pot;
  bool ok = true;
  // conditioning (reported, not part of Psi): ln|Delta^sigma_k| of every
  // determinant product k per spin, and the cancellation of the determinant
  // sum kappa_D = sum_k |c d Delta_up Delta_dn| / |D|
  std::vector<double> lspin[2];
  double kappaD = 0.0;
};

template <class T>
EvalOut<T> evaluate(const System& s, const Params<T>& P, const double* R, int level) {
  EvalOut<T> o;
  const int N = s.N, M = s.M, no = s.norb;
  // orbitals phi_p^c(r_i) = sum_mu lambda_{p mu} chi_mu^c(r_i)
  std::vector<double> ao(5 * M);
  std::vector<T> phi((size_t)N * 5 * no, T(0.0));  // [i][c][p]
  int nch = level >= 2 ? 5 : (level == 1 ? 4 : 1);
  for (int i = 0; i < N; ++i) {
    eval_ao(s, &R[3 * i], ao.data());
    for (int c = 0; c < nch; ++c)
      for (int p = 0; p < no; ++p) {
        T acc = T(0.0);
        for (int mu = 0; mu < M; ++mu) acc = acc + P.lam[p * M + mu] * ao[c * M + mu];
        phi[((size_t)i * 5 + c) * no + p] = acc;
      }
  }
  // every determinant of every structure, spin by spin
  const int nd = (int)s.dets.size();
  std::vector<T> L(nd);
  std::vector<int> sg(nd), alive(nd);
  // op[k][i][c-1]: O_i Delta^sigma(i)_k / Delta^sigma(i)_k for c = 1..4
  std::vector<T> op((size_t)nd * N * 4, T(0.0));
  o.lspin[0].assign(nd, -INFINITY);
  o.lspin[1].assign(nd, -INFINITY);
  for (int k = 0; k < nd; ++k) {
    const Det& d = s.dets[k];
    T lsum = T(0.0);
    int ssum = 1;
    bool ok = true;
    for (int spin = 0; spin < 2 && ok; ++spin) {
      const std::vector<int>& occ = spin == 0 ? d.up : d.dn;
      int n = (int)occ.size(), e0 = spin == 0 ? 0 : s.nup;
      if (n == 0) continue;
      std::vector<T> A(n * n), inv;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[i * n + j] = phi[((size_t)(e0 + i) * 5 + 0) * no + occ[j]];
      T la;
      int sgn;
      if (!lu_det_inverse(n, A, la, sgn, inv)) { ok = false; break; }
      o.lspin[spin][k] = val(la);
      lsum = lsum + la;
      ssum *= sgn;
      // row-i cofactor expansion: O_i Delta / Delta = sum_j O phi_{o_j}(r_i) (A^-1)_{j i}
      for (int i = 0; i < n && level >= 1; ++i)
        for (int c = 1; c < nch; ++c) {
          T acc = T(0.0);
          for (int j = 0; j < n; ++j) acc = acc + phi[((size_t)(e0 + i) * 5 + c) * no + occ[j]] * inv[j * n + i];
          op[((size_t)k * N + e0 + i) * 4 + (c - 1)] = acc;
        }
    }
    alive[k] = ok;
    L[k] = lsum;
    sg[k] = ssum;
  }
  // D = sum_I c_I sum_{k in I} Delta_up_k Delta_dn_k, scaled by exp(-Lmax)
  double Lmax = -INFINITY;
  for (int k = 0; k < nd; ++k)
    if (alive[k]) Lmax = std::max(Lmax, val(L[k]));
  if (!(Lmax > -INFINITY)) { o.ok = false; return o; }
  std::vector<T> term(nd, T(0.0));
  T Dt = T(0.0);
  for (int k = 0; k < nd; ++k)
    if (alive[k]) {
      term[k] = P.c[s.dets[k].structure] * (double)sg[k] * exp(L[k] - Lmax);
      Dt = Dt + term[k];
    }
  if (val(Dt) == 0.0) { o.ok = false; return o; }
  {
    double sa = 0.0;
    for (int k = 0; k < nd; ++k)
      if (alive[k]) sa += std::fabs(val(term[k]));
    o.kappaD = sa / std::fabs(val(Dt));
  }
  o.ratio.assign(s.nstruct, T(0.0));
  for (int k = 0; k < nd; ++k)
    if (alive[k]) o.ratio[s.dets[k].structure] = o.ratio[s.dets[k].structure] + (double)sg[k] * exp(L[k] - Lmax) / Dt;
  // Jastrow U, grad_i U, lap_i U
  T U = T(0.0);
  std::vector<T> gU(3 * N, T(0.0)), lU(N, T(0.0));
  const T* jee = &P.jas[0];
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a < s.nnuc; ++a) {
      const T* ja = &P.jas[6 + 6 * a];
      double dv[3] = {R[3 * i] - s.pos[3 * a], R[3 * i + 1] - s.pos[3 * a + 1], R[3 * i + 2] - s.pos[3 * a + 2]};
      double r = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      T u, u1, u2;
      pair_u(r, s.kappa, ja[0], ja[1], ja + 2, u, u1, u2);
      U = U + u;
      for (int x = 0; x < 3; ++x) gU[3 * i + x] = gU[3 * i + x] + u1 * (dv[x] / r);
      lU[i] = lU[i] + u2 + u1 * (2.0 / r);
    }
    for (int j = i + 1; j < N; ++j) {
      bool anti = (i < s.nup) != (j < s.nup);
      T a = T(anti ? s.ee_a_anti : s.ee_a_par);
      T b = anti ? jee[0] : jee[1];
      double dv[3] = {R[3 * i] - R[3 * j], R[3 * i + 1] - R[3 * j + 1], R[3 * i + 2] - R[3 * j + 2]};
      double r = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      T u, u1, u2;
      pair_u(r, s.kappa, a, b, jee + 2, u, u1, u2);
      U = U + u;
      for (int x = 0; x < 3; ++x) {
        gU[3 * i + x] = gU[3 * i + x] + u1 * (dv[x] / r);
        gU[3 * j + x] = gU[3 * j + x] - u1 * (dv[x] / r);
      }
      lU[i] = lU[i] + u2 + u1 * (2.0 / r);
      lU[j] = lU[j] + u2 + u1 * (2.0 / r);
    }
  }
  if (s.een) een_all(s, &P.jas[6 + 6 * s.nnuc], R, level >= 1, U, gU, lU);
  o.logabs = U + Lmax + log_abs(Dt);
  o.sign = val(Dt) > 0 ? 1 : -1;
  if (level == 0) return o;
  // grad_i D / D and lap_i D / D
  o.grad.assign(3 * N, T(0.0));
  std::vector<T> gD(3 * N, T(0.0)), lD(N, T(0.0));
  for (int k = 0; k < nd; ++k) {
    if (!alive[k]) continue;
    T wk = term[k] / Dt;
    for (int i = 0; i < N; ++i) {
      for (int x = 0; x < 3; ++x) gD[3 * i + x] = gD[3 * i + x] + wk * op[((size_t)k * N + i) * 4 + x];
      if (level >= 2) lD[i] = lD[i] + wk * op[((size_t)k * N + i) * 4 + 3];
    }
  }
  for (int q = 0; q < 3 * N; ++q) o.grad[q] = gU[q] + gD[q];
  if (level < 2) return o;
  // E_L = -1/2 sum_i [lap U + |grad U|^2 + 2 grad U . grad D / D + lap D / D] + V
  T kin = T(0.0);
  for (int i = 0; i < N; ++i) {
    T t = lU[i] + lD[i];
    for (int x = 0; x < 3; ++x)
      t = t + gU[3 * i + x] * gU[3 * i + x] + 2.0 * gU[3 * i + x] * gD[3 * i + x];
    kin = kin - 0.5 * t;
  }
  double V = 0;
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a < s.nnuc; ++a) {
      double dx = R[3 * i] - s.pos[3 * a], dy = R[3 * i + 1] - s.pos[3 * a + 1], dz = R[3 * i + 2] - s.pos[3 * a + 2];
      V -= s.Z[a] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    for (int j = i + 1; j < N; ++j) {
      double dx = R[3 * i] - R[3 * j], dy = R[3 * i + 1] - R[3 * j + 1], dz = R[3 * i + 2] - R[3 * j + 2];
      V += 1.0 / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  for (int a = 0; a < s.nnuc; ++a)
    for (int b = a + 1; b < s.nnuc; ++b) {
      double dx = s.pos[3 * a] - s.pos[3 * b], dy = s.pos[3 * a + 1] - s.pos[3 * b + 1], dz = s.pos[3 * a + 2] - s.pos[3 * b + 2];
      V += s.Z[a] * s.Z[b] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  o.kin = kin;
  o.pot = T(V);
  o.eloc = kin + V;
  return o;
}

// ---------------------------------------------------------------------------
// Pseudopotential energy (semilocal form, Sec. 2.1 basis choice): per centre
// and electron the local radial part, and for r < r_cut each channel l as
// (2l + 1) times the mean over the 12 icosahedron directions of P_l(cos)
// times Psi(moved) / Psi, every moved configuration evaluated afresh.
// ---------------------------------------------------------------------------
double ecp_radial(const std::vector<double>& t, double r) {
  double v = 0;
  for (size_t k = 0; k + 2 < t.size(); k += 3) {
    v += t[k] * std::pow(r, t[k + 1] - 2.0) * std::exp(-t[k + 2] * r * r);
  }
  return v;
}

double ecp_energy(const System& s, const Params<double>& P, const double* R, const EvalOut<double>& base) {
  const double g = (1.0 + std::sqrt(5.0)) / 2.0, nrm = std::sqrt(1.0 + g * g);
  double u[12][3];
  int q = 0;
  for (double s1 : {-1.0, 1.0})
    for (double s2 : {-1.0, 1.0}) {
      const double v[3][3] = {{0.0, s1, s2 * g}, {s1, s2 * g, 0.0}, {s2 * g, 0.0, s1}};
      for (int k = 0; k < 3; ++k, ++q)
        for (int x = 0; x < 3; ++x) u[q][x] = v[k][x] / nrm;
    }
  double e = 0;
  std::vector<double> Rq(R, R + 3 * s.N);
  for (const System::EcpCentre& c : s.ecp) {
    const double* a = &s.pos[3 * c.center];
    for (int i = 0; i < s.N; ++i) {
      double d[3] = {R[3 * i] - a[0], R[3 * i + 1] - a[1], R[3 * i + 2] - a[2]};
      const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      e += ecp_radial(c.parts[0], r);
      if (!(r < c.rcut) || c.parts.size() < 2) continue;
      for (int k = 0; k < 12; ++k) {
        const double x = (u[k][0] * d[0] + u[k][1] * d[1] + u[k][2] * d[2]) / r;
        const double Pl[4] = {1.0, x, 0.5 * (3 * x * x - 1), 0.5 * (5 * x * x * x - 3 * x)};
        double w = 0;
        for (size_t l = 0; l + 1 < c.parts.size(); ++l) w += (2.0 * l + 1.0) / 12.0 * ecp_radial(c.parts[l + 1], r) * Pl[l];
        for (int x3 = 0; x3 < 3; ++x3) Rq[3 * i + x3] = a[x3] + r * u[k][x3];
        EvalOut<double> o = evaluate(s, P, Rq.data(), 0);
        for (int x3 = 0; x3 < 3; ++x3) Rq[3 * i + x3] = R[3 * i + x3];
        if (o.ok) e += w * o.sign * base.sign * std::exp(o.logabs - base.logabs);
      }
    }
  }
  return e;
}

// evaluate() with the pseudopotential energy in E_L (level 2)
EvalOut<double> evaluate_h(const System& s, const Params<double>& P, const double* R, int level) {
  EvalOut<double> o = evaluate(s, P, R, level);
  if (level >= 2 && o.ok && !s.ecp.empty()) {
    const double e = ecp_energy(s, P, R, o);
    o.eloc += e;
    o.pot += e;
  }
  return o;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its
// published definition: ten rounds of two 32x32->64 multiplies with the
// round constants M0 = 0xD2511F53, M1 = 0xCD9E8D57 and a Weyl key schedule
// W0 = 0x9E3779B9, W1 = 0xBB67AE85.
// ---------------------------------------------------------------------------
void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t x[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
  }
  for (int i = 0; i < 4; ++i) out[i] = x[i];
}

// Random-number layout: key = (seed low word, seed high word);
// counter = (walker slot, step, 4 * electron + purpose, draw).
// Purposes: 0 proposal, 1 acceptance, 2 branching; electron = N for
// per-walker draws.  Each call yields two uniforms in [0, 1) with 53 bits.
void uniforms(uint64_t seed, uint32_t walker, uint32_t step, uint32_t slot, uint32_t draw, double u[2]) {
  uint32_t ctr[4] = {walker, step, slot, draw};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t o[4];
  philox(ctr, key, o);
  uint64_t a = ((uint64_t)o[1] << 32) | o[0];
  uint64_t b = ((uint64_t)o[3] << 32) | o[2];
  u[0] = (double)(a >> 11) * (1.0 / 9007199254740992.0);
  u[1] = (double)(b >> 11) * (1.0 / 9007199254740992.0);
}

// three proposal uniforms for one electron
void proposal_uniforms(uint64_t seed, uint32_t w, uint32_t step, int e, double u[3]) {
  double a[2], b[2];
  uniforms(seed, w, step, 4u * e + 0u, 0, a);
  uniforms(seed, w, step, 4u * e + 0u, 1, b);
  u[0] = a[0]; u[1] = a[1]; u[2] = b[0];
}

// three standard normals for one electron (Box-Muller on 1 - u, never log 0)
void proposal_normals(uint64_t seed, uint32_t w, uint32_t step, int e, double z[3]) {
  double a[2], b[2];
  uniforms(seed, w, step, 4u * e + 0u, 0, a);
  uniforms(seed, w, step, 4u * e + 0u, 1, b);
  const double two_pi = 6.283185307179586476925286766559;
  double r0 = std::sqrt(-2.0 * std::log(1.0 - a[0]));
  double r1 = std::sqrt(-2.0 * std::log(1.0 - b[0]));
  z[0] = r0 * std::cos(two_pi * a[1]);
  z[1] = r0 * std::sin(two_pi * a[1]);
  z[2] = r1 * std::cos(two_pi * b[1]);
}

double accept_uniform(uint64_t seed, uint32_t w, uint32_t step, int e) {
  double a[2];
  uniforms(seed, w, step, 4u * e + 1u, 0, a);
  return a[0];
}

double branch_uniform(uint64_t seed, uint32_t w, uint32_t step, int N) {
  double a[2];
  uniforms(seed, w, step, 4u * N + 2u, 0, a);
  return a[0];
}

int max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // namespace

// ===========================================================================
// C interface used by the Python wrapper (test infrastructure).
// ===========================================================================
extern "C" {

// Term description for the HLSP structures:
// term_struct[t] = structure index of term t; term_counts[3t..3t+2] =
// (n_inactive, n_pairs, n_unpaired); term_orbs = concatenation per term of
// inactive[], pairs[2*n_pairs], unpaired[].
void* orc_create(int nnuc, const double* Z, const double* pos, int nup, int ndn,
                 int nshell, const int* sh_center, const int* sh_kind, const int* sh_l,
                 const int* sh_nprim, const double* pexp, const double* pcoef,
                 int norb, const double* lam,
                 int nstruct, const double* c, int nterm, const int* term_struct,
                 const int* term_counts, const int* term_orbs,
                 double kappa, const double* ee /* a_anti, a_par, b_anti, b_par, b3..b6 */,
                 const double* en /* per nucleus a1..a6 */,
                 const double* een /* per nucleus the f_een coefficients in term order, or NULL */) {
  System* s = new System();
  s->nnuc = nnuc;
  s->Z.assign(Z, Z + nnuc);
  s->pos.assign(pos, pos + 3 * nnuc);
  s->nup = nup; s->ndn = ndn; s->N = nup + ndn;
  s->nshell = nshell;
  int off = 0, fn = 0;
  for (int k = 0; k < nshell; ++k) {
    s->sh_center.push_back(sh_center[k]);
    s->sh_kind.push_back(sh_kind[k]);
    s->sh_l.push_back(sh_l[k]);
    s->sh_nprim.push_back(sh_nprim[k]);
    s->sh_off.push_back(off);
    s->sh_fn.push_back(fn);
    for (int q = 0; q < sh_nprim[k]; ++q) {
      s->pexp.push_back(pexp[off + q]);
      s->pcoef.push_back(pcoef[off + q]);
    }
    off += sh_nprim[k];
    fn += nfunc_of_l(sh_l[k]);
  }
  s->M = fn;
  s->norb = norb;
  s->lam.assign(lam, lam + (size_t)norb * fn);
  s->nstruct = nstruct;
  s->c.assign(c, c + nstruct);
  int q = 0;
  for (int t = 0; t < nterm; ++t) {
    int ni = term_counts[3 * t], np = term_counts[3 * t + 1], nu = term_counts[3 * t + 2];
    expand_term(term_struct[t], term_orbs + q, ni, term_orbs + q + ni, np, term_orbs + q + ni + 2 * np, nu, s->dets);
    q += ni + 2 * np + nu;
  }
  s->kappa = kappa;
  s->ee_a_anti = ee[0];
  s->ee_a_par = ee[1];
  for (int k = 2; k < 8; ++k) s->jas.push_back(ee[k]);
  for (int a = 0; a < nnuc; ++a)
    for (int k = 0; k < 6; ++k) s->jas.push_back(en[6 * a + k]);
  if (een) {
    const int nt = (int)een_terms().size();
    s->een = true;
    for (int a = 0; a < nnuc; ++a)
      for (int t = 0; t < nt; ++t) s->jas.push_back(een[nt * a + t]);
  }
  s->njas = (int)s->jas.size();
  return s;
}

void orc_destroy(void* h) { delete (System*)h; }

int orc_set_ecp(void* h, int ncen, const int* center, const int* nch, const double* rcut, const int* nterms,
                const double* terms) {
  System& s = *(System*)h;
  s.ecp.clear();
  int k = 0, t = 0;
  for (int c = 0; c < ncen; ++c) {
    System::EcpCentre e;
    e.center = center[c];
    e.rcut = rcut[c];
    for (int q = 0; q <= nch[c]; ++q) {
      std::vector<double> part(terms + 3 * t, terms + 3 * (t + nterms[k]));
      t += nterms[k++];
      e.parts.push_back(part);
    }
    s.ecp.push_back(e);
  }
  return 0;
}

int orc_num_dets(void* h) { return (int)((System*)h)->dets.size(); }
int orc_num_params(void* h) { return ((System*)h)->nparam(); }
int orc_max_threads() { return max_threads(); }

// the f_een term list: (k, l, m) per term, returns the count
int orc_een_terms(int* klm) {
  std::vector<EenTerm> t = een_terms();
  for (size_t q = 0; q < t.size(); ++q) {
    klm[3 * q] = t[q].k;
    klm[3 * q + 1] = t[q].l;
    klm[3 * q + 2] = t[q].m;
  }
  return (int)t.size();
}

// determinant list: structure[k], up[k*nup..], dn[k*ndn..]
void orc_dets(void* h, int* structure, int* up, int* dn) {
  System* s = (System*)h;
  for (size_t k = 0; k < s->dets.size(); ++k) {
    structure[k] = s->dets[k].structure;
    for (int j = 0; j < s->nup; ++j) up[k * s->nup + j] = s->dets[k].up[j];
    for (int j = 0; j < s->ndn; ++j) dn[k * s->ndn + j] = s->dets[k].dn[j];
  }
}

void orc_ao(void* h, const double* r, double* out) { eval_ao(*(System*)h, r, out); }

int orc_lu(int n, const double* A, double* logabs, int* sign, double* inv) {
  std::vector<double> a(A, A + n * n), iv;
  double la;
  int sg;
  if (!lu_det_inverse(n, a, la, sg, iv)) return -1;
  *logabs = la;
  *sign = sg;
  std::copy(iv.begin(), iv.end(), inv);
  return 0;
}

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

void orc_uniforms(uint64_t seed, uint32_t walker, uint32_t step, uint32_t slot, uint32_t draw, double* u) {
  uniforms(seed, walker, step, slot, draw, u);
}

// Batched evaluation; grad / eloc / ratio / kin may be NULL.  Returns the
// number of configurations where Psi vanished (their outputs are NaN).
int orc_evaluate(void* h, int W, const double* R, int level, double* logabs, int* sign,
                 double* grad, double* eloc, double* ratio, double* kin) {
  const System& s = *(System*)h;
  Params<double> P = make_params<double>(s, -1);
  int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
  for (int w = 0; w < W; ++w) {
    EvalOut<double> o = evaluate_h(s, P, R + (size_t)w * s.N * 3, level);
    if (!o.ok) {
      ++bad;
      logabs[w] = -INFINITY;
      sign[w] = 0;
      continue;
    }
    logabs[w] = o.logabs;
    sign[w] = o.sign;
    if (grad && level >= 1)
      for (int q = 0; q < 3 * s.N; ++q) grad[(size_t)w * 3 * s.N + q] = o.grad[q];
    if (eloc && level >= 2) eloc[w] = o.eloc;
    if (kin && level >= 2) kin[w] = o.kin;
    if (ratio)
      for (int I = 0; I < s.nstruct; ++I) ratio[(size_t)w * s.nstruct + I] = o.ratio[I];
  }
  return bad;
}

// Conditioning of the determinant part at W configurations (reported beside
// the parity checks): kappa_D [W] and ln|Delta^sigma_k| per spin, [W][n_dets]
// each (-inf where a spin determinant is singular).
int orc_conditioning(void* h, int W, const double* R, double* kappaD, double* lup, double* ldn) {
  const System& s = *(System*)h;
  Params<double> P = make_params<double>(s, -1);
  const int nd = (int)s.dets.size();
  int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
  for (int w = 0; w < W; ++w) {
    EvalOut<double> o = evaluate(s, P, R + (size_t)w * s.N * 3, 0);
    if (!o.ok) ++bad;
    kappaD[w] = o.ok ? o.kappaD : INFINITY;
    for (int k = 0; k < nd; ++k) {
      lup[(size_t)w * nd + k] = o.lspin[0].empty() ? -INFINITY : o.lspin[0][k];
      ldn[(size_t)w * nd + k] = o.lspin[1].empty() ? -INFINITY : o.lspin[1][k];
    }
  }
  return bad;
}

// Parameter derivatives by forward-mode dual numbers, one pass per parameter.
// Parameter order: [c (nstruct) | lambda (norb*M row-major) |
// b_anti, b_par, b3..b6 | per nucleus a1..a6].
void orc_param_deriv(void* h, int W, const double* R, int nidx, const int* idx,
                     double* dlogpsi, double* deloc) {
  const System& s = *(System*)h;
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int w = 0; w < W; ++w)
    for (int q = 0; q < nidx; ++q) {
      Params<Dual> P = make_params<Dual>(s, idx[q]);
      EvalOut<Dual> o = evaluate(s, P, R + (size_t)w * s.N * 3, 2);
      dlogpsi[(size_t)w * nidx + q] = o.ok ? tangent(o.logabs) : NAN;
      deloc[(size_t)w * nidx + q] = o.ok ? tangent(o.eloc) : NAN;
    }
}

// Metropolis VMC (Sec. 2.3.1).  mode 0: one all-electron move per step;
// mode 1: N sequential single-electron moves per step.  Proposal
// r' = r + step_size * (2u - 1) per component; accept iff u < |Psi'/Psi|^2.
// After each step E_L is evaluated and accumulated.
int orc_vmc(void* h, int W, double* R, int nsteps, uint64_t seed, uint32_t step0,
            double step_size, int mode, double* e_sum, double* e2_sum, double* n_acc,
            double* e_last, double* sij_sum) {
  const System& s = *(System*)h;
  Params<double> P = make_params<double>(s, -1);
  const int N = s.N, nv = s.nstruct;
  int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
  for (int w = 0; w < W; ++w) {
    double* Rw = R + (size_t)w * N * 3;
    EvalOut<double> cur = evaluate(s, P, Rw, 0);
    if (!cur.ok) { ++bad; continue; }
    std::vector<double> Rn(Rw, Rw + 3 * N);
    for (int st = 0; st < nsteps; ++st) {
      uint32_t step = step0 + (uint32_t)st;
      if (mode == 0) {
        for (int e = 0; e < N; ++e) {
          double u[3];
          proposal_uniforms(seed, (uint32_t)w, step, e, u);
          for (int x = 0; x < 3; ++x) Rn[3 * e + x] = Rw[3 * e + x] + step_size * (2.0 * u[x] - 1.0);
        }
        EvalOut<double> nw = evaluate(s, P, Rn.data(), 0);
        double ua = accept_uniform(seed, (uint32_t)w, step, N);
        if (nw.ok && ua < std::exp(2.0 * (nw.logabs - cur.logabs))) {
          std::copy(Rn.begin(), Rn.end(), Rw);
          cur = nw;
          n_acc[w] += 1;
        } else {
          std::copy(Rw, Rw + 3 * N, Rn.begin());
        }
      } else {
        for (int e = 0; e < N; ++e) {
          double u[3];
          proposal_uniforms(seed, (uint32_t)w, step, e, u);
          for (int x = 0; x < 3; ++x) Rn[3 * e + x] = Rw[3 * e + x] + step_size * (2.0 * u[x] - 1.0);
          EvalOut<double> nw = evaluate(s, P, Rn.data(), 0);
          double ua = accept_uniform(seed, (uint32_t)w, step, e);
          if (nw.ok && ua < std::exp(2.0 * (nw.logabs - cur.logabs))) {
            for (int x = 0; x < 3; ++x) Rw[3 * e + x] = Rn[3 * e + x];
            cur = nw;
            n_acc[w] += 1;
          } else {
            for (int x = 0; x < 3; ++x) Rn[3 * e + x] = Rw[3 * e + x];
          }
        }
      }
      EvalOut<double> full = evaluate_h(s, P, Rw, 2);
      if (!full.ok) { ++bad; break; }
      e_sum[w] += full.eloc;
      e2_sum[w] += full.eloc * full.eloc;
      e_last[w] = full.eloc;
      if (sij_sum)
        for (int I = 0; I < nv; ++I)
          for (int J = 0; J < nv; ++J) sij_sum[((size_t)w * nv + I) * nv + J] += full.ratio[I] * full.ratio[J];
    }
  }
  return bad;
}

// Fixed-node DMC (Sec. 2.3.2) with per-electron drift-diffusion moves,
// Metropolis acceptance with the drift-diffusion Green's-function ratio,
// node-crossing rejection, weights exp(-tau (E_L + E_L')/2 - E_T)) with E_L
// clipped to E_T +- sqrt(N / tau) (the size-consistent form of cut-off of Zen
// et al., Phys. Rev. B 93, 241118 (2016), with their prefactor 0.2 widened to
// 1 for trial functions without cusps), birth/death by floor(w + u) copies
// (at most 3, children of weight 1, kept in parent order) and trial-energy
// feedback E_T = E_est - (0.1 / tau) ln(W / W_target), E_est being the running
// weighted mean of the clipped E_L over the steps of this call (so that a few
// walkers with extreme E_L cannot drag E_T away).  Population control: when
// the expected next population sum_w w falls outside [0.95, 1.05] W_target,
// every weight of the step is scaled by the one factor f that brings the sum
// to the nearer bound (the same as using E_T + ln(f) / tau in that step's
// weights), so the birth/death population stays within +-10 % of W_target up
// to the rounding noise of floor(w + u).
// R: [capacity][N][3]; eloc_io: [capacity] local energies of the walkers;
// per-step outputs (length nsteps): pop (walkers before branching),
// wsum = sum w, wesum = sum w E_L, wcsum = sum w E_L clipped (the estimator
// of the E_T feedback), etrial (E_T used in the step), acc / prop
// (accepted / proposed single-electron moves).
int orc_dmc(void* h, int* W_io, int capacity, double* R, double* eloc_io, int nsteps,
            uint64_t seed, uint32_t step0, double tau, double* etrial_io, int W_target,
            double* pop, double* wsum, double* wesum, double* wcsum, double* etrial, double* acc, double* prop,
            double* d2acc, double* d2prop) {
  const System& s = *(System*)h;
  Params<double> P = make_params<double>(s, -1);
  const int N = s.N;
  int W = *W_io;
  double ET = *etrial_io;
  double run_num = 0, run_den = 0;
  std::vector<double> Rnew((size_t)capacity * N * 3), Enew(capacity), wts(capacity), ubr(capacity);
  std::vector<int> ncopy(capacity);
  std::vector<double> nacc(capacity), nprop(capacity), sacc(capacity), sprop(capacity);
  const double cap = std::sqrt((double)N / tau);
  std::vector<double> Eclip(capacity);
  for (int st = 0; st < nsteps; ++st) {
    uint32_t step = step0 + (uint32_t)st;
    int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
    for (int w = 0; w < W; ++w) {
      double* Rw = R + (size_t)w * N * 3;
      nacc[w] = 0;
      nprop[w] = 0;
      sacc[w] = 0;
      sprop[w] = 0;
      EvalOut<double> cur = evaluate(s, P, Rw, 1);
      if (!cur.ok) { ++bad; continue; }
      std::vector<double> Rn(Rw, Rw + 3 * N);
      for (int e = 0; e < N; ++e) {
        double z[3], v[3], rp[3];
        proposal_normals(seed, (uint32_t)w, step, e, z);
        for (int x = 0; x < 3; ++x) {
          v[x] = cur.grad[3 * e + x];
          rp[x] = Rw[3 * e + x] + tau * v[x] + std::sqrt(tau) * z[x];
          Rn[3 * e + x] = rp[x];
        }
        nprop[w] += 1;
        // squared length of the proposed move (the effective time step is
        // tau times the accepted over the proposed sums)
        double d2 = 0;
        for (int x = 0; x < 3; ++x) d2 += (rp[x] - Rw[3 * e + x]) * (rp[x] - Rw[3 * e + x]);
        sprop[w] += d2;
        EvalOut<double> nw = evaluate(s, P, Rn.data(), 1);
        bool accept = false;
        if (nw.ok && nw.sign == cur.sign) {
          double fwd = 0, bwd = 0;
          for (int x = 0; x < 3; ++x) {
            double a = rp[x] - Rw[3 * e + x] - tau * v[x];
            double b = Rw[3 * e + x] - rp[x] - tau * nw.grad[3 * e + x];
            fwd += a * a;
            bwd += b * b;
          }
          double p = std::exp(2.0 * (nw.logabs - cur.logabs) + (fwd - bwd) / (2.0 * tau));
          accept = accept_uniform(seed, (uint32_t)w, step, e) < p;
        }
        if (accept) {
          for (int x = 0; x < 3; ++x) Rw[3 * e + x] = rp[x];
          cur = nw;
          nacc[w] += 1;
          sacc[w] += d2;
        } else {
          for (int x = 0; x < 3; ++x) Rn[3 * e + x] = Rw[3 * e + x];
        }
      }
      EvalOut<double> full = evaluate_h(s, P, Rw, 2);
      if (!full.ok) { ++bad; continue; }
      double eo = std::min(std::max(eloc_io[w], ET - cap), ET + cap);
      double en = std::min(std::max(full.eloc, ET - cap), ET + cap);
      wts[w] = std::exp(-tau * (0.5 * (eo + en) - ET));
      Enew[w] = full.eloc;
      Eclip[w] = en;
      ubr[w] = branch_uniform(seed, (uint32_t)w, step, N);
    }
    if (bad) return -1;
    // population control: one factor on every weight of the step
    double sw_raw = 0;
    for (int w = 0; w < W; ++w) sw_raw += wts[w];
    double f = 1.0;
    if (sw_raw > 1.05 * W_target) f = 1.05 * W_target / sw_raw;
    else if (sw_raw < 0.95 * W_target) f = 0.95 * W_target / sw_raw;
    double sw = 0, swe = 0, swc = 0, na = 0, np = 0, s2a = 0, s2p = 0;
    for (int w = 0; w < W; ++w) {
      wts[w] = f * wts[w];
      ncopy[w] = std::min(3, (int)std::floor(wts[w] + ubr[w]));
      sw += wts[w];
      swe += wts[w] * Enew[w];
      swc += wts[w] * Eclip[w];
      na += nacc[w];
      np += nprop[w];
      s2a += sacc[w];
      s2p += sprop[w];
    }
    pop[st] = W;
    wsum[st] = sw;
    wesum[st] = swe;
    wcsum[st] = swc;
    etrial[st] = ET + std::log(f) / tau;
    acc[st] = na;
    prop[st] = np;
    d2acc[st] = s2a;
    d2prop[st] = s2p;
    // stable compaction of the copies
    int Wn = 0;
    for (int w = 0; w < W; ++w) Wn += ncopy[w];
    if (Wn == 0 || Wn > capacity) return -2;
    int o = 0;
    for (int w = 0; w < W; ++w)
      for (int k = 0; k < ncopy[w]; ++k, ++o) {
        std::copy(R + (size_t)w * N * 3, R + (size_t)(w + 1) * N * 3, Rnew.begin() + (size_t)o * N * 3);
        eloc_io[o] = Enew[w];
      }
    std::copy(Rnew.begin(), Rnew.begin() + (size_t)Wn * N * 3, R);
    W = Wn;
    run_num += swc;
    run_den += sw;
    ET = run_num / run_den - (0.1 / tau) * std::log((double)W / (double)W_target);
  }
  *W_io = W;
  *etrial_io = ET;
  return 0;
}

}  // extern "C"
