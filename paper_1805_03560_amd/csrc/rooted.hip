// Rooted polynomials as UV filters (Sec. 2.1), built on the series action and force of the
// kappa^(2k) filter.
//
// With x = K = kappa^2 H_oe H_eo and M_1 = M~ = (1 - x) exp(sum_{i<=k} x^i/i):
//   p_j = W_j^{-1} = Taylor polynomial of degree n_j of M_j^{-1/N} = exp(-(1/N) log M_j),
//   log M_{j+1} = log M_j + N log p_j,
//   M_{jmax+1}^{-1} = g(x) / (1 - x),  g = exp(-sum_{i<=k} x^i/i - N sum_j log p_j),
//   alpha = g(1) = exp(-sum_{i<=k} 1/i) prod_j p_j(1)^{-N},  b_n = sum_{m<=n} g_m - alpha,
// which is eq. (restM): the partial sums of g / (1 - x) minus their limit alpha.  The series are
// formed on the host in long double from the recurrences of exp and log of power series.
//
// Action (eq. initPseudo per term): sum_j sum_i |p_j(K) phi_{j,i}|^2 + |(sum b_n K^n + alpha
// M_oo^{-1}) phi_r|^2.  Heat bath: phi_{j,i} = p_j(K)^{-1} eta by CG on p_j^dag p_j (the
// straightforward route the paper took), phi_r = prod_j p_j(K)^N M~ eta.  The force of every
// term is the Horner construction of the filter with the term's coefficients (alpha = 0 for the
// polynomial terms: no solve).  The integrator nests the gauge action, the jmax polynomial terms
// and the remainder on jmax + 2 Sexton-Weingarten levels.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace whmc {
namespace {

using Series = std::vector<long double>;

// Taylor coefficients 0..n of exp(a(x)), a[0] = 0: E' = a' E gives m E_m = sum_{i=1..m} i a_i E_{m-i}
Series series_exp(const Series& a, int n) {
  Series E(n + 1, 0.0L);
  E[0] = 1.0L;
  for (int m = 1; m <= n; ++m) {
    long double s = 0.0L;
    for (int i = 1; i <= m && i < (int)a.size(); ++i) s += (long double)i * a[i] * E[m - i];
    E[m] = s / m;
  }
  return E;
}

// Taylor coefficients 0..n of log p(x), p[0] = 1: p L' = p' gives
// m L_m = m p_m - sum_{i=1..m-1} i L_i p_{m-i}
Series series_log(const Series& p, int n) {
  auto pc = [&](int i) { return i < (int)p.size() ? p[i] : 0.0L; };
  Series L(n + 1, 0.0L);
  for (int m = 1; m <= n; ++m) {
    long double s = m * pc(m);
    for (int i = 1; i < m; ++i) s -= (long double)i * L[i] * pc(m - i);
    L[m] = s / m;
  }
  return L;
}

struct RootedCoef {
  std::vector<std::vector<double>> p;   // p_1 .. p_jmax
  std::vector<double> b;                // b_0 .. b_nb
  double alpha = 1.0;
};

void rooted_coefficients(const whmc_rooted& r, int nb, RootedCoef& out) {
  int n = nb;
  for (int j = 0; j < r.jmax; ++j) n = std::max(n, r.n[j]);
  Series logM(n + 1, 0.0L), lg(n + 1, 0.0L);
  long double hk = 0.0L;
  for (int i = 1; i <= n; ++i) logM[i] = -1.0L / i;            // log(1 - x)
  for (int i = 1; i <= r.k; ++i) {
    hk += 1.0L / i;
    if (i <= n) {
      logM[i] += 1.0L / i;                                      // + sum_{i<=k} x^i / i
      lg[i] -= 1.0L / i;
    }
  }
  long double alpha = expl(-hk);
  out.p.clear();
  for (int j = 0; j < r.jmax; ++j) {
    const int nj = r.n[j];
    Series a(nj + 1, 0.0L);
    for (int i = 1; i <= nj; ++i) a[i] = -logM[i] / r.N;
    const Series pj = series_exp(a, nj);
    const Series L = series_log(pj, n);
    long double p1 = 0.0L;
    for (int i = nj; i >= 0; --i) p1 += pj[i];
    alpha /= powl(p1, (long double)r.N);
    for (int i = 1; i <= n; ++i) {
      logM[i] += r.N * L[i];
      lg[i] -= r.N * L[i];
    }
    out.p.emplace_back(pj.begin(), pj.end());
  }
  const Series g = series_exp(lg, nb);
  out.b.assign(nb + 1, 0.0);
  long double s = 0.0L;
  for (int m = 0; m <= nb; ++m) {
    s += g[m];
    out.b[m] = (double)(s - alpha);
  }
  out.alpha = (double)alpha;
}

whmc_status check_rooted(const whmc_rooted* r) {
  WHMC_CHECK(r, WHMC_EARG, "null rooted parameters");
  WHMC_CHECK(r->N >= 1 && r->N <= 64, WHMC_EARG, "rooted: N must be in 1..64");
  WHMC_CHECK(r->jmax >= 0 && r->jmax <= WHMC_MAX_POLY, WHMC_EARG, "rooted: jmax must be in 0..WHMC_MAX_POLY");
  for (int j = 0; j < r->jmax; ++j)
    WHMC_CHECK(r->n[j] >= 1 && r->n[j] <= WHMC_ROOTED_MAX_N, WHMC_EARG, "rooted: degrees n_j must be in 1..1000");
  WHMC_CHECK(r->k >= 0 && r->k <= 2, WHMC_EUNSUP, "rooted: filter order k must be 0, 1 or 2");
  WHMC_CHECK(r->n_t >= 0 && r->n_t <= WHMC_ROOTED_MAX_N && r->n_max >= 0 && r->n_max <= WHMC_ROOTED_MAX_N, WHMC_EARG,
             "rooted: n_t and n_max must be in 0..1000");
  return WHMC_OK;
}

whmc_status check_rooted_hmc(const whmc_rooted_hmc_params* p) {
  WHMC_CHECK(p, WHMC_EARG, "null rooted hmc params");
  WHMC_TRY(check_rooted(&p->rooted));
  WHMC_CHECK(p->m >= 1 && p->tau > 0, WHMC_EARG, "rooted hmc: m >= 1 and tau > 0 required");
  for (int l = 0; l <= p->rooted.jmax; ++l)
    WHMC_CHECK(p->msub[l] >= 1, WHMC_EARG, "rooted hmc: msub[0..jmax] must be >= 1");
  WHMC_CHECK(p->integrator == WHMC_LEAPFROG || p->integrator == WHMC_OMELYAN, WHMC_EARG,
             "rooted hmc: unknown integrator");
  return WHMC_OK;
}

int n_fields(const whmc_rooted& r) { return r.jmax * r.N + 1; }

double* field(whmc_ctx* c, double* base, int f) { return base + (size_t)f * 24 * c->Vh; }
const double* field(whmc_ctx* c, const double* base, int f) { return base + (size_t)f * 24 * c->Vh; }

// x = p(K)^{-1} eta by CG on p^dag p x = p^dag eta, to |r| <= tol |p^dag eta|
whmc_status poly_inverse(whmc_ctx* c, double* x, const double* eta, const std::vector<double>& p, double kappa,
                         double tol, int maxiter, long long* iters) {
  Fields F{c, (size_t)c->Vh * 192};
  double *r, *d, *Ad, *t, *te, *to;
  WHMC_TRY(F.get("pi_r", 0, &r));
  WHMC_TRY(F.get("pi_d", 0, &d));
  WHMC_TRY(F.get("pi_Ad", 0, &Ad));
  WHMC_TRY(F.get("pi_t", 0, &t));
  WHMC_TRY(F.get("pi_te", 0, &te));
  WHMC_TRY(F.get("pi_to", 0, &to));
  double* sdev = c->red.result + 8;
  WHMC_TRY(poly_K(c, r, eta, p, kappa, te, to, 1));
  WHMC_TRY(zero_bytes(c, x, (size_t)c->Vh * 192));
  WHMC_TRY(copy_f64(c, d, r, 1));
  double rr, pAp;
  WHMC_TRY(norm2_f64(c, r, 1, sdev));
  WHMC_TRY(read_scalar(c, sdev, &rr));
  if (rr == 0.0) return WHMC_OK;
  const double stop = tol * tol * rr;
  for (int it = 0; it < maxiter; ++it) {
    WHMC_TRY(poly_K(c, t, d, p, kappa, te, to, 0));
    WHMC_TRY(poly_K(c, Ad, t, p, kappa, te, to, 1));
    WHMC_TRY(dot_re_f64(c, d, Ad, 1, sdev));
    WHMC_TRY(read_scalar(c, sdev, &pAp));
    WHMC_CHECK(pAp > 0.0, WHMC_ENOCONV, "rooted heat bath: CG on p^dag p broke down (p(K) singular?)");
    const double a = rr / pAp;
    WHMC_TRY(axpby_f64(c, x, a, d, 1.0, 1));
    WHMC_TRY(axpby_f64(c, r, -a, Ad, 1.0, 1));
    double rn;
    WHMC_TRY(norm2_f64(c, r, 1, sdev));
    WHMC_TRY(read_scalar(c, sdev, &rn));
    if (iters) ++*iters;
    if (rn <= stop) return WHMC_OK;
    WHMC_TRY(axpby_f64(c, d, 1.0, r, rn / rr, 1));
    rr = rn;
  }
  WHMC_CHECK(false, WHMC_ENOCONV, "rooted heat bath: CG on p^dag p hit maxiter");
}

whmc_status heatbath_all(whmc_ctx* c, double* phi, const double* eta, const whmc_rooted& r, const RootedCoef& C,
                         double kappa, const whmc_cg_params* sp, long long* iters) {
  for (int j = 0; j < r.jmax; ++j)
    for (int i = 0; i < r.N; ++i)
      WHMC_TRY(poly_inverse(c, field(c, phi, j * r.N + i), field(c, eta, j * r.N + i), C.p[j], kappa, sp->tol,
                            sp->maxiter, iters));
  // phi_r = prod_j p_j(K)^N M~ eta_r
  Fields F{c, (size_t)c->Vh * 192};
  double *t, *te, *to;
  WHMC_TRY(F.get("rh_t", 0, &t));
  WHMC_TRY(F.get("rh_te", 0, &te));
  WHMC_TRY(F.get("rh_to", 0, &to));
  double* v = field(c, phi, r.jmax * r.N);
  const whmc_filter f{r.k, r.n_t, r.n_max};
  WHMC_TRY(heatbath(c, v, field(c, eta, r.jmax * r.N), &f, kappa));
  for (int j = 0; j < r.jmax; ++j)
    for (int i = 0; i < r.N; ++i) {
      WHMC_TRY(poly_K(c, t, v, C.p[j], kappa, te, to, 0));
      WHMC_TRY(copy_f64(c, v, t, 1));
    }
  return WHMC_OK;
}

// S[0..jmax-1] the polynomial terms, S[jmax] the remainder at n_max (C.b must reach n_max)
whmc_status action_all(whmc_ctx* c, double* S, const double* phi, const whmc_rooted& r, const RootedCoef& C,
                       double kappa, const whmc_cg_params* sp, SolveLog* log) {
  Fields F{c, (size_t)c->Vh * 192};
  double *z, *te, *to;
  WHMC_TRY(F.get("ra_z", 0, &z));
  WHMC_TRY(F.get("ra_te", 0, &te));
  WHMC_TRY(F.get("ra_to", 0, &to));
  double* sdev = c->red.result + 9;
  for (int j = 0; j < r.jmax; ++j) {
    S[j] = 0.0;
    for (int i = 0; i < r.N; ++i) {
      double s;
      WHMC_TRY(poly_K(c, z, field(c, phi, j * r.N + i), C.p[j], kappa, te, to, 0));
      WHMC_TRY(norm2_f64(c, z, 1, sdev));
      WHMC_TRY(read_scalar(c, sdev, &s));
      S[j] += s;
    }
  }
  const std::vector<double> b(C.b.begin(), C.b.begin() + r.n_max + 1);
  WHMC_TRY(series_inverse(c, z, field(c, phi, r.jmax * r.N), b, C.alpha, kappa, sp, log));
  WHMC_TRY(norm2_f64(c, z, 1, sdev));
  return read_scalar(c, sdev, &S[r.jmax]);
}

// pi/F += scale * force of term `term` (1..jmax polynomial, jmax+1 remainder at n_t)
whmc_status force_term(whmc_ctx* c, double* F, const double* phi, const whmc_rooted& r, const RootedCoef& C,
                       int term, double kappa, const whmc_cg_params* sp, double scale, int accumulate, SolveLog* log) {
  if (term <= r.jmax) {
    for (int i = 0; i < r.N; ++i)
      WHMC_TRY(series_force(c, F, field(c, phi, (term - 1) * r.N + i), C.p[term - 1], 0.0, kappa, sp, scale,
                            accumulate || i > 0, log));
    return WHMC_OK;
  }
  const std::vector<double> b(C.b.begin(), C.b.begin() + r.n_t + 1);
  return series_force(c, F, field(c, phi, r.jmax * r.N), b, C.alpha, kappa, sp, scale, accumulate, log);
}

// the terms of the rooted action for the shared multi-level trajectory (C must outlive the result)
TermAction rooted_terms(whmc_ctx* c, const whmc_rooted_hmc_params* p, const RootedCoef& C) {
  TermAction A;
  A.nfields = n_fields(p->rooted);
  A.nterms = p->rooted.jmax + 1;
  A.beta_eff = p->beta + delta_beta(p->kappa, p->rooted.k);
  A.heatbath = [=, &C](double* phi, const double* eta, long long* it, SolveLog*) {
    return heatbath_all(c, phi, eta, p->rooted, C, p->kappa, &p->heatbath_solver, it);
  };
  A.action = [=, &C](double* S, const double* phi, SolveLog* log) {
    return action_all(c, S, phi, p->rooted, C, p->kappa, &p->action_solver, log);
  };
  A.force = [=, &C](double* F, const double* phi, int t, double s, int acc, SolveLog* log) {
    return force_term(c, F, phi, p->rooted, C, t, p->kappa, &p->md_solver, s, acc, log);
  };
  return A;
}

TermMD rooted_md(const whmc_rooted_hmc_params* p) { return TermMD{p->integrator, p->lambda, p->tau, p->m, p->msub}; }

}  // namespace
}  // namespace whmc

using namespace whmc;

extern "C" {

whmc_status whmc_rooted_coefficients(const whmc_rooted* r, double* p, double* b, int nb, double* alpha) {
  WHMC_TRY(check_rooted(r));
  WHMC_CHECK(nb >= 0 && nb <= WHMC_ROOTED_MAX_N, WHMC_EARG, "whmc_rooted_coefficients: nb must be in 0..1000");
  RootedCoef C;
  rooted_coefficients(*r, nb, C);
  if (p)
    for (const auto& pj : C.p) p = std::copy(pj.begin(), pj.end(), p);
  if (b) std::copy(C.b.begin(), C.b.end(), b);
  if (alpha) *alpha = C.alpha;
  return WHMC_OK;
}

whmc_status whmc_rooted_heatbath(whmc_ctx* c, double* phi, const double* eta, const whmc_rooted* r, double kappa,
                                 const whmc_cg_params* solver, long long* iters) {
  WHMC_CHECK(c && phi && eta && phi != eta, WHMC_EARG, "whmc_rooted_heatbath: bad argument");
  WHMC_TRY(check_rooted(r));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  RootedCoef C;
  rooted_coefficients(*r, 0, C);
  long long it = 0;
  const whmc_status rc = heatbath_all(c, phi, eta, *r, C, kappa, &sp, &it);
  if (iters) *iters = it;
  return rc;
}

whmc_status whmc_rooted_action(whmc_ctx* c, double* S, const double* phi, const whmc_rooted* r, double kappa,
                               const whmc_cg_params* solver) {
  WHMC_CHECK(c && S && phi, WHMC_EARG, "whmc_rooted_action: null argument");
  WHMC_TRY(check_rooted(r));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  RootedCoef C;
  rooted_coefficients(*r, r->n_max, C);
  return action_all(c, S, phi, *r, C, kappa, &sp, nullptr);
}

whmc_status whmc_rooted_force(whmc_ctx* c, double* F, const double* phi, const whmc_rooted* r, int term, double kappa,
                              const whmc_cg_params* solver, int flags) {
  WHMC_CHECK(c && F && phi, WHMC_EARG, "whmc_rooted_force: null argument");
  WHMC_TRY(check_rooted(r));
  WHMC_CHECK(term >= 0 && term <= r->jmax + 1, WHMC_EARG, "whmc_rooted_force: term must be in 0..jmax+1");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  RootedCoef C;
  rooted_coefficients(*r, r->n_t, C);
  int acc = (flags & WHMC_FORCE_ACCUMULATE) ? 1 : 0;
  const int lo = term == 0 ? 1 : term, hi = term == 0 ? r->jmax + 1 : term;
  for (int t = lo; t <= hi; ++t) {
    WHMC_TRY(force_term(c, F, phi, *r, C, t, kappa, &sp, 1.0, acc, nullptr));
    acc = 1;
  }
  return WHMC_OK;
}

whmc_status whmc_rooted_hamiltonian(whmc_ctx* c, const whmc_rooted_hmc_params* p, const double* pi,
                                    const double* phi, double* H) {
  WHMC_CHECK(c && pi && phi && H, WHMC_EARG, "whmc_rooted_hamiltonian: null argument");
  WHMC_TRY(check_rooted_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  RootedCoef C;
  rooted_coefficients(p->rooted, p->rooted.n_max, C);
  return term_hamiltonian(c, rooted_terms(c, p, C), pi, phi, H, nullptr);
}

whmc_status whmc_rooted_md_integrate(whmc_ctx* c, const whmc_rooted_hmc_params* p, double* pi, const double* phi) {
  WHMC_CHECK(c && pi && phi, WHMC_EARG, "whmc_rooted_md_integrate: null argument");
  WHMC_TRY(check_rooted_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  RootedCoef C;
  rooted_coefficients(p->rooted, p->rooted.n_t, C);
  WHMC_TRY(term_md(c, rooted_terms(c, p, C), rooted_md(p), pi, phi, nullptr));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  return WHMC_OK;
}

whmc_status whmc_rooted_trajectory(whmc_ctx* c, const whmc_rooted_hmc_params* p, const double* pi0,
                                   const double* eta, double u, whmc_traj_result* res) {
  WHMC_CHECK(c && pi0 && eta && res, WHMC_EARG, "whmc_rooted_trajectory: null argument");
  WHMC_TRY(check_rooted_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  RootedCoef C;
  rooted_coefficients(p->rooted, std::max(p->rooted.n_t, p->rooted.n_max), C);
  return term_trajectory(c, rooted_terms(c, p, C), rooted_md(p), pi0, eta, u, res);
}

}  // extern "C"
