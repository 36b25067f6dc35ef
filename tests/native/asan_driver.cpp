// Host-side checks under AddressSanitizer and UndefinedBehaviorSanitizer
// (built and run by tests/test_sanitizers.py; CPU only, no GPU call):
// the oracle (evaluation, parameter derivatives, VMC, DMC on a two-centre,
// two-electron system) and the host-only entry points of the C ABI (the
// linear-method estimators and step, the structure weights, argument
// errors).  Exit status 0 and no sanitizer report is the pass.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/vbqmc.h"

extern "C" {
void* orc_create(int nnuc, const double* Z, const double* pos, int nup, int ndn, int nshell, const int* sh_center,
                 const int* sh_kind, const int* sh_l, const int* sh_nprim, const double* pexp, const double* pcoef,
                 int norb, const double* lam, int nstruct, const double* c, int nterm, const int* term_struct,
                 const int* term_counts, const int* term_orbs, double kappa, const double* ee, const double* en,
                 const double* een);
void orc_destroy(void* h);
int orc_num_params(void* h);
int orc_evaluate(void* h, int W, const double* R, int level, double* logabs, int* sign, double* grad, double* eloc,
                 double* ratio, double* kin);
void orc_param_deriv(void* h, int W, const double* R, int nidx, const int* idx, double* dlogpsi, double* deloc);
int orc_vmc(void* h, int W, double* R, int nsteps, uint64_t seed, uint32_t step0, double step_size, int mode,
            double* e_sum, double* e2_sum, double* n_acc, double* e_last, double* sij_sum);
int orc_dmc(void* h, int* W_io, int capacity, double* R, double* eloc_io, int nsteps, uint64_t seed, uint32_t step0,
            double tau, double* etrial_io, int W_target, double* pop, double* wsum, double* wesum, double* wcsum,
            double* etrial, double* acc, double* prop, double* d2acc, double* d2prop);
}

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

static double urand(unsigned& s) {
  s = s * 1664525u + 1013904223u;
  return (s >> 8) * (1.0 / 16777216.0);
}

static void oracle_checks() {
  // two nuclei, one s Gaussian each, a covalent and an ionic structure, Pade
  // Jastrow with polynomial terms and f_een
  const double Z[2] = {1.0, 1.0}, pos[6] = {0, 0, -0.7, 0, 0, 0.7};
  const int shc[2] = {0, 1}, shk[2] = {0, 0}, shl[2] = {0, 0}, shn[2] = {2, 2};
  const double pe[4] = {1.2, 0.3, 1.2, 0.3}, pc[4] = {0.6, 0.5, 0.6, 0.5};
  const double lam[4] = {1.0, 0.0, 0.0, 1.0}, c[2] = {0.9, 0.3};
  const int ts[3] = {0, 1, 1}, tc[9] = {0, 1, 0, 0, 1, 0, 0, 1, 0}, to[6] = {0, 1, 0, 0, 1, 1};
  const double ee[8] = {0.5, 0.25, 1.0, 1.0, 0.01, 0.0, 0.0, 0.0};
  const double en[12] = {-0.1, 1.5, 0.02, 0, 0, 0, -0.1, 1.5, 0.02, 0, 0, 0};
  std::vector<double> een(2 * 23);
  unsigned s = 7;
  for (double& v : een) v = 0.05 * (urand(s) - 0.5);
  void* h = orc_create(2, Z, pos, 1, 1, 2, shc, shk, shl, shn, pe, pc, 2, lam, 2, c, 3, ts, tc, to, 0.8, ee, en,
                       een.data());
  CHECK(h != nullptr);
  const int W = 8, N = 2, P = orc_num_params(h);
  std::vector<double> R(W * N * 3);
  for (double& v : R) v = 2.0 * urand(s) - 1.0;
  std::vector<double> la(W), g(W * N * 3), el(W), ratio(W * 2), kin(W);
  std::vector<int> sg(W);
  CHECK(orc_evaluate(h, W, R.data(), 2, la.data(), sg.data(), g.data(), el.data(), ratio.data(), kin.data()) == 0);
  for (int w = 0; w < W; ++w) CHECK(std::isfinite(el[w]) && sg[w] != 0);
  std::vector<int> idx(P);
  for (int k = 0; k < P; ++k) idx[k] = k;
  std::vector<double> dl(W * P), de(W * P);
  orc_param_deriv(h, W, R.data(), P, idx.data(), dl.data(), de.data());
  for (double v : dl) CHECK(std::isfinite(v));
  std::vector<double> es(W, 0), e2(W, 0), na(W, 0), last(W, 0), sij(W * 4, 0);
  CHECK(orc_vmc(h, W, R.data(), 5, 11, 0, 0.5, 1, es.data(), e2.data(), na.data(), last.data(), sij.data()) == 0);
  int Wio = W, cap = 4 * W;
  std::vector<double> Rd(cap * N * 3, 0.0), Ed(cap, 0.0);
  for (int k = 0; k < W * N * 3; ++k) Rd[k] = R[k];
  for (int w = 0; w < W; ++w) Ed[w] = last[w];
  double et = -1.0;
  const int steps = 4;
  std::vector<double> hist(9 * steps);
  double* H = hist.data();
  CHECK(orc_dmc(h, &Wio, cap, Rd.data(), Ed.data(), steps, 5, 0, 0.01, &et, W, H, H + steps, H + 2 * steps,
                H + 3 * steps, H + 4 * steps, H + 5 * steps, H + 6 * steps, H + 7 * steps, H + 8 * steps) == 0);
  CHECK(Wio > 0 && Wio <= cap);
  orc_destroy(h);
}

static void abi_checks() {
  // linear-method sums of random samples -> estimators -> step
  const int P = 5, M = 40;
  int64_t n = 0;
  CHECK(vbqmc_lm_acc_doubles(P, &n) == 0 && n == 3 * (P + 1) * (P + 1));
  CHECK(vbqmc_lm_acc_doubles(0, &n) == VBQMC_EINVAL);
  std::vector<double> acc(n, 0.0);
  unsigned s = 3;
  for (int k = 0; k < M; ++k) {
    double X[P + 1], Y[P + 1];
    const double E = -1.0 + 0.2 * (urand(s) - 0.5), w = 0.5 + urand(s);
    X[0] = 1.0;
    Y[0] = E * E;
    for (int j = 1; j <= P; ++j) {
      X[j] = urand(s) - 0.5;
      Y[j] = urand(s) - 0.5;
    }
    for (int i = 0; i <= P; ++i)
      for (int j = 0; j <= P; ++j) {
        acc[i * (P + 1) + j] += w * X[i] * X[j];
        acc[(P + 1) * (P + 1) + i * (P + 1) + j] += w * E * X[i] * X[j];
        acc[2 * (P + 1) * (P + 1) + i * (P + 1) + j] += w * X[i] * Y[j];
      }
  }
  double e0 = 0, var = 0;
  std::vector<double> gl(P), gr(P), hb(P * P), sb(P * P), dp(P);
  CHECK(vbqmc_lm_estimators(P, acc.data(), &e0, gl.data(), gr.data(), hb.data(), sb.data(), &var) == 0);
  double e_lin = 0;
  const int rc = vbqmc_lm_solve(P, e0, gl.data(), gr.data(), hb.data(), sb.data(), 0.1, dp.data(), &e_lin);
  CHECK(rc == 0 || rc == VBQMC_ESINGULAR || rc == VBQMC_ENONFINITE);
  CHECK(vbqmc_lm_solve(0, e0, gl.data(), gr.data(), hb.data(), sb.data(), 0.0, dp.data(), &e_lin) == VBQMC_EINVAL);
  // structure weights of a random positive definite overlap
  const int nv = 4;
  double S[nv * nv], c[nv], w[nv];
  double A[nv * nv];
  for (double& v : A) v = urand(s) - 0.5;
  for (int i = 0; i < nv; ++i) {
    c[i] = urand(s) - 0.5;
    for (int j = 0; j < nv; ++j) {
      double a = i == j ? 1.0 : 0.0;
      for (int k = 0; k < nv; ++k) a += A[i * nv + k] * A[j * nv + k] * 0.1;
      S[i * nv + j] = a;
    }
  }
  CHECK(vbqmc_weights_chirgwin_coulson(nv, S, c, w) == 0);
  CHECK(vbqmc_weights_lowdin(nv, S, c, w) == 0);
  double sum = 0;
  for (double v : w) sum += v;
  CHECK(std::fabs(sum - 1.0) < 1e-12);
  CHECK(vbqmc_weights_lowdin(0, S, c, w) == VBQMC_EINVAL);
  // argument errors of the context calls (no context)
  CHECK(vbqmc_create(nullptr, nullptr, nullptr, nullptr) == VBQMC_EINVAL);
  CHECK(vbqmc_get_info(nullptr, nullptr) == VBQMC_EINVAL);
}

int main() {
  oracle_checks();
  abi_checks();
  if (fails) std::fprintf(stderr, "%d checks failed\n", fails);
  else std::printf("sanitized host checks passed\n");
  return fails ? 1 : 0;
}
