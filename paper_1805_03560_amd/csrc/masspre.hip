// Mass preconditioning combined with the kappa^(2k) filter (Sec. 1, 5).
//
// With heavier hopping parameters kappa_1 < ... < kappa_n < kappa_{n+1} = kappa, every factor
// carries the filter, M~(kappa) = M_oo(kappa) exp(sum_{j<=k} K(kappa)^j / j), and one gauge term
// remains, that of the target kappa (beta + 96 kappa^4 for k = 2):
//   det M_oo(kappa) = det M~(kappa_1) prod_i det M~(kappa_{i+1}) / det M~(kappa_i) exp(-sum Tr K(kappa)^j / j).
// The heaviest field has |M~(kappa_1)^{-1} phi|^2 (the filter's action at kappa_1); each ratio has
// S = |M~(kappa_{i+1})^{-1} M~(kappa_i) phi|^2.  All factors are functions of D = H_oe H_eo, so with
// x = K(kappa_{i+1}) and rho = kappa_i^2 / kappa_{i+1}^2 the ratio is g(x) / (1 - x),
// g(x) = (1 - rho x) exp(sum_{j<=k} (rho^j - 1) x^j / j): a series sum b_n x^n + alpha M_oo^{-1}
// (alpha = g(1), b_n = sum_{m<=n} g_m - alpha) whose action and force are the filter's series
// routines.  Its low orders cancel up to x^(k+1), which is what keeps the ratio forces small.
// Heat bath of a ratio: phi = M~(kappa_i)^{-1} M~(kappa_{i+1}) eta, one solve at kappa_i.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace whmc {
namespace {

whmc_status check_masspre(const whmc_masspre* mp, double kappa) {
  WHMC_CHECK(mp, WHMC_EARG, "null mass-preconditioning parameters");
  WHMC_CHECK(mp->n >= 0 && mp->n <= WHMC_MAX_MASSPRE, WHMC_EARG, "masspre: n must be in 0..WHMC_MAX_MASSPRE");
  WHMC_TRY(check_filter(&mp->filter));
  double prev = 0.0;
  for (int i = 0; i < mp->n; ++i) {
    WHMC_CHECK(mp->kappas[i] > prev, WHMC_EARG, "masspre: kappas must be positive and increasing");
    prev = mp->kappas[i];
  }
  WHMC_CHECK(kappa > prev, WHMC_EARG, "masspre: kappa must exceed every heavier kappa_i");
  return WHMC_OK;
}

// kappa_1 .. kappa_{n+1} = kappa
std::vector<double> chain(const whmc_masspre& mp, double kappa) {
  std::vector<double> k(mp.kappas, mp.kappas + mp.n);
  k.push_back(kappa);
  return k;
}

// b_0 .. b_n and alpha of M~(kappa_hi)^{-1} M~(kappa_lo), rho = kappa_lo^2 / kappa_hi^2, in long double
void ratio_coefficients(double rho, int k, int n, std::vector<double>& b, double& alpha) {
  std::vector<long double> a(n + 1, 0.0L), E(n + 1, 0.0L);
  long double r = rho, rj = 1.0L, h = 0.0L;
  for (int j = 1; j <= k; ++j) {
    rj *= r;
    h += (rj - 1.0L) / j;
    if (j <= n) a[j] = (rj - 1.0L) / j;
  }
  E[0] = 1.0L;   // exp(a(x)): m E_m = sum_i i a_i E_{m-i}
  for (int m = 1; m <= n; ++m) {
    long double s = 0.0L;
    for (int i = 1; i <= std::min(m, k); ++i) s += (long double)i * a[i] * E[m - i];
    E[m] = s / m;
  }
  const long double al = (1.0L - r) * expl(h);
  b.assign(n + 1, 0.0);
  long double s = 0.0L;
  for (int m = 0; m <= n; ++m) {
    s += E[m] - (m >= 1 ? r * E[m - 1] : 0.0L);   // g_m of (1 - rho x) exp(a(x))
    b[m] = (double)(s - al);
  }
  alpha = (double)al;
}

double* field(whmc_ctx* c, double* base, int f) { return base + (size_t)f * 24 * c->Vh; }
const double* field(whmc_ctx* c, const double* base, int f) { return base + (size_t)f * 24 * c->Vh; }

whmc_status heatbath_all(whmc_ctx* c, double* phi, const double* eta, const whmc_masspre& mp, double kappa,
                         const whmc_cg_params* sp, SolveLog* log) {
  const std::vector<double> k = chain(mp, kappa);
  const whmc_filter& f = mp.filter;
  WHMC_TRY(heatbath(c, phi, eta, &f, k[0]));
  Fields F{c, (size_t)c->Vh * 192};
  double* t;
  WHMC_TRY(F.get("mp_t", 0, &t));
  std::vector<double> b, cc;
  double alpha;
  coefficients(f.k, f.k == 0 ? 0 : f.n_max, b, cc, alpha);
  for (int i = 0; i < mp.n; ++i) {
    WHMC_TRY(heatbath(c, t, field(c, eta, i + 1), &f, k[i + 1]));                   // M~(kappa_{i+1}) eta
    WHMC_TRY(series_inverse(c, field(c, phi, i + 1), t, b, alpha, k[i], sp, log));  // M~(kappa_i)^{-1}
  }
  return WHMC_OK;
}

whmc_status action_all(whmc_ctx* c, double* S, const double* phi, const whmc_masspre& mp, double kappa,
                       const whmc_cg_params* sp, SolveLog* log) {
  const std::vector<double> k = chain(mp, kappa);
  WHMC_TRY(pf_action(c, phi, &mp.filter, k[0], sp, &S[0], log));
  Fields F{c, (size_t)c->Vh * 192};
  double* z;
  WHMC_TRY(F.get("mp_z", 0, &z));
  double* sdev = c->red.result + 10;
  for (int i = 0; i < mp.n; ++i) {
    std::vector<double> b;
    double alpha;
    ratio_coefficients((k[i] / k[i + 1]) * (k[i] / k[i + 1]), mp.filter.k, mp.filter.n_max, b, alpha);
    WHMC_TRY(series_inverse(c, z, field(c, phi, i + 1), b, alpha, k[i + 1], sp, log));
    WHMC_TRY(norm2_f64(c, z, 1, sdev));
    WHMC_TRY(read_scalar(c, sdev, &S[i + 1]));
  }
  return WHMC_OK;
}

whmc_status force_term(whmc_ctx* c, double* F, const double* phi, const whmc_masspre& mp, double kappa, int t,
                       const whmc_cg_params* sp, double scale, int accumulate, SolveLog* log) {
  const std::vector<double> k = chain(mp, kappa);
  if (t == 1) return pf_force(c, F, phi, &mp.filter, k[0], sp, scale, accumulate, log);
  const int i = t - 2;
  std::vector<double> b;
  double alpha;
  ratio_coefficients((k[i] / k[i + 1]) * (k[i] / k[i + 1]), mp.filter.k, mp.filter.n_t, b, alpha);
  return series_force(c, F, field(c, phi, i + 1), b, alpha, k[i + 1], sp, scale, accumulate, log);
}

whmc_status check_hmc(const whmc_masspre_hmc_params* p) {
  WHMC_CHECK(p, WHMC_EARG, "null mass-preconditioning hmc params");
  WHMC_TRY(check_masspre(&p->mp, p->kappa));
  WHMC_CHECK(p->m >= 1 && p->tau > 0, WHMC_EARG, "masspre hmc: m >= 1 and tau > 0 required");
  for (int l = 0; l <= p->mp.n; ++l) WHMC_CHECK(p->msub[l] >= 1, WHMC_EARG, "masspre hmc: msub[0..n] must be >= 1");
  WHMC_CHECK(p->integrator == WHMC_LEAPFROG || p->integrator == WHMC_OMELYAN, WHMC_EARG,
             "masspre hmc: unknown integrator");
  return WHMC_OK;
}

TermAction masspre_terms(whmc_ctx* c, const whmc_masspre_hmc_params* p) {
  TermAction A;
  A.nfields = p->mp.n + 1;
  A.nterms = p->mp.n + 1;
  A.beta_eff = p->beta + delta_beta(p->kappa, p->mp.filter.k);   // the gauge term of the target kappa
  A.heatbath = [=](double* phi, const double* eta, long long*, SolveLog* log) {
    return heatbath_all(c, phi, eta, p->mp, p->kappa, &p->action_solver, log);
  };
  A.action = [=](double* S, const double* phi, SolveLog* log) {
    return action_all(c, S, phi, p->mp, p->kappa, &p->action_solver, log);
  };
  A.force = [=](double* F, const double* phi, int t, double s, int acc, SolveLog* log) {
    return force_term(c, F, phi, p->mp, p->kappa, t, &p->md_solver, s, acc, log);
  };
  return A;
}

TermMD masspre_md(const whmc_masspre_hmc_params* p) { return TermMD{p->integrator, p->lambda, p->tau, p->m, p->msub}; }

}  // namespace
}  // namespace whmc

using namespace whmc;

extern "C" {

whmc_status whmc_masspre_coefficients(double rho, int k, int n, double* b, double* alpha) {
  WHMC_CHECK(rho > 0.0 && rho < 1.0, WHMC_EARG, "whmc_masspre_coefficients: rho must be in (0, 1)");
  WHMC_CHECK(k >= 0 && k <= 2, WHMC_EUNSUP, "whmc_masspre_coefficients: filter order k must be 0, 1 or 2");
  WHMC_CHECK(n >= 0 && n <= WHMC_ROOTED_MAX_N, WHMC_EARG, "whmc_masspre_coefficients: n must be in 0..1000");
  std::vector<double> bb;
  double a;
  ratio_coefficients(rho, k, n, bb, a);
  if (b) std::copy(bb.begin(), bb.end(), b);
  if (alpha) *alpha = a;
  return WHMC_OK;
}

whmc_status whmc_masspre_heatbath(whmc_ctx* c, double* phi, const double* eta, const whmc_masspre* mp, double kappa,
                                  const whmc_cg_params* solver) {
  WHMC_CHECK(c && phi && eta && phi != eta, WHMC_EARG, "whmc_masspre_heatbath: bad argument");
  WHMC_TRY(check_masspre(mp, kappa));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  return heatbath_all(c, phi, eta, *mp, kappa, &sp, nullptr);
}

whmc_status whmc_masspre_action(whmc_ctx* c, double* S, const double* phi, const whmc_masspre* mp, double kappa,
                                const whmc_cg_params* solver) {
  WHMC_CHECK(c && S && phi, WHMC_EARG, "whmc_masspre_action: null argument");
  WHMC_TRY(check_masspre(mp, kappa));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  return action_all(c, S, phi, *mp, kappa, &sp, nullptr);
}

whmc_status whmc_masspre_force(whmc_ctx* c, double* F, const double* phi, const whmc_masspre* mp, int term,
                               double kappa, const whmc_cg_params* solver, int flags) {
  WHMC_CHECK(c && F && phi, WHMC_EARG, "whmc_masspre_force: null argument");
  WHMC_TRY(check_masspre(mp, kappa));
  WHMC_CHECK(term >= 0 && term <= mp->n + 1, WHMC_EARG, "whmc_masspre_force: term must be in 0..n+1");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  int acc = (flags & WHMC_FORCE_ACCUMULATE) ? 1 : 0;
  const int lo = term == 0 ? 1 : term, hi = term == 0 ? mp->n + 1 : term;
  for (int t = lo; t <= hi; ++t) {
    WHMC_TRY(force_term(c, F, phi, *mp, kappa, t, &sp, 1.0, acc, nullptr));
    acc = 1;
  }
  return WHMC_OK;
}

whmc_status whmc_masspre_hamiltonian(whmc_ctx* c, const whmc_masspre_hmc_params* p, const double* pi,
                                     const double* phi, double* H) {
  WHMC_CHECK(c && pi && phi && H, WHMC_EARG, "whmc_masspre_hamiltonian: null argument");
  WHMC_TRY(check_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  return term_hamiltonian(c, masspre_terms(c, p), pi, phi, H, nullptr);
}

whmc_status whmc_masspre_md_integrate(whmc_ctx* c, const whmc_masspre_hmc_params* p, double* pi, const double* phi) {
  WHMC_CHECK(c && pi && phi, WHMC_EARG, "whmc_masspre_md_integrate: null argument");
  WHMC_TRY(check_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  WHMC_TRY(term_md(c, masspre_terms(c, p), masspre_md(p), pi, phi, nullptr));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  return WHMC_OK;
}

whmc_status whmc_masspre_trajectory(whmc_ctx* c, const whmc_masspre_hmc_params* p, const double* pi0,
                                    const double* eta, double u, whmc_traj_result* res) {
  WHMC_CHECK(c && pi0 && eta && res, WHMC_EARG, "whmc_masspre_trajectory: null argument");
  WHMC_TRY(check_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  return term_trajectory(c, masspre_terms(c, p), masspre_md(p), pi0, eta, u, res);
}

}  // extern "C"
