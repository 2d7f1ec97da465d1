// Host orchestration of the filtered pseudo-fermion action and force (Sec. 2, 2.2) and of the HMC
// trajectory (Sec. 1, 4.1), built from the stencil, solver and gauge launchers.
//
// Filter (K = kappa^2 H_oe H_eo on odd sites, M_oo = 1 - K):
//   M~ = M_oo exp(sum_{j<=k} K^j/j),  M~^{-1} = sum_n b_n K^n + alpha M_oo^{-1}
//   a_n = coefficients of exp(-sum_{j<=k} x^j/j) / (1 - x), alpha = exp(-sum_{j<=k} 1/j),
//   b_n = a_n - alpha = -(tail sum of the coefficients of exp(-sum x^j/j) beyond n).
// The heat bath uses c_n, the coefficients of exp(+sum_{j<=k} x^j/j): phi = M_oo sum c_n K^n eta.
//
// Force of S~ = |M~^{-1} phi|^2 truncated at n_t (Horner scheme of Sec. 2, with the adjoints
// that the variation produces):
//   Y_{n_t} = b_{n_t} phi, Y_{i-1} = b_{i-1} phi + K Y_i;   Y~ = alpha M_oo^{-1} phi;
//   X_1 = Y_0 + Y~, X_i = K^dag X_{i-1};   X~ = M_oo^{-dag} X_1;
//   F = -kappa^2 sum_pairs P_TA(G(X_full, Y_full)),  pairs (X~, Y~), (X_i, Y_i), i = 1..n_t,
//   with full-lattice pairs X_full = ((H^dag)_eo X, X), Y_full = (H_eo Y, Y).
// The two inverses come from two independent solves of A = M_oo^dag M_oo:
//   s2 = A^{-1} Y_0,  s3 = A^{-1} gamma_5 phi  =>  Y~ = alpha M_oo^dag gamma_5 s3,
//   X~ = M_oo s2 + alpha gamma_5 s3   (M_oo^dag = gamma_5 M_oo gamma_5).
// The even-site halves of the pairs are the intermediates H_eo Y_i and (H^dag)_eo X_i of the
// Horner and X recursions and are kept rather than recomputed.
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"

namespace whmc {

// ------------------------------------------------------------------ coefficients (host)
static void exp_series(int sign, int k, int n, std::vector<long double>& g) {
  g.assign(n + 1, 0.0L);
  g[0] = 1.0L;
  for (int m = 1; m <= n; ++m) {
    long double s = 0.0L;
    for (int j = 1; j <= std::min(m, k); ++j) s += g[m - j];
    g[m] = sign * s / m;
  }
}

void coefficients(int k, int n, std::vector<double>& b, std::vector<double>& c, double& alpha) {
  long double h = 0.0L;
  for (int j = 1; j <= k; ++j) h += 1.0L / j;
  alpha = (double)expl(-h);
  std::vector<long double> e, cp;
  const int tail = n + 400;
  exp_series(-1, k, tail, e);
  exp_series(+1, k, n, cp);
  b.assign(n + 1, 0.0);
  c.assign(n + 1, 0.0);
  for (int m = 0; m <= n; ++m) {
    long double t = 0.0L;
    for (int i = tail; i > m; --i) t += e[i];   // smallest terms first
    b[m] = (double)(-t);
    c[m] = (double)cp[m];
  }
}

double delta_beta(double kappa, int k) { return k >= 2 ? 96.0 * kappa * kappa * kappa * kappa : 0.0; }

whmc_cg_params default_solver() {
  whmc_cg_params p{};
  p.tol = 1e-12;
  p.maxiter = 10000;
  p.prec = WHMC_F64;
  p.links = WHMC_L18;
  p.delta = 0.1;
  p.check_every = 8;
  p.rhs_block = 0;
  p.rhs_lanes = 0;
  return p;
}

whmc_status check_filter(const whmc_filter* f) {
  WHMC_CHECK(f, WHMC_EARG, "null filter");
  WHMC_CHECK(f->k >= 0 && f->n_t >= 0 && f->n_max >= 0, WHMC_EARG, "filter: k, n_t, n_max must be >= 0");
  WHMC_CHECK(f->k <= 2, WHMC_EUNSUP, "filter: only k <= 2 has a closed-form gauge term (Sec. 2)");
  WHMC_CHECK(f->n_t <= 200 && f->n_max <= 200, WHMC_EARG, "filter: truncation orders above 200");
  return WHMC_OK;
}

// out = sum_{n<=N} coef[n] K^n v (K^dag for dagger), Horner; tmp_e, tmp_o scratch
whmc_status poly_K(whmc_ctx* c, double* out, const double* v, const std::vector<double>& coef, double kappa,
                   double* tmp_e, double* tmp_o, int dagger) {
  const int N = (int)coef.size() - 1;
  WHMC_TRY(zero_bytes(c, out, (size_t)c->Vh * 192));
  WHMC_TRY(axpby_f64(c, out, coef[N], v, 0.0, 1));
  for (int n = N - 1; n >= 0; --n) {
    WHMC_TRY(copy_f64(c, tmp_o, out, 1));
    WHMC_TRY(apply_K_f64(c, out, tmp_o, kappa, dagger, tmp_e, v, coef[n]));
  }
  return WHMC_OK;
}

// s = A^{-1} rhs with A = M_oo^dag M_oo; accumulates statistics
whmc_status solve(whmc_ctx* c, double* x, const double* rhs, double kappa, const whmc_cg_params* p, SolveLog* log) {
  whmc_cg_stats st{};
  whmc_status rc = cg_solve(c, x, rhs, &kappa, 1, p, &st);
  if (log) {
    log->iters += st.iters;
    log->n += 1;
  }
  return rc;
}

static whmc_status solve2(whmc_ctx* c, double* x, const double* rhs, double kappa, const whmc_cg_params* p,
                          SolveLog* log) {
  // two independent right-hand sides stored consecutively
  const double kap[2] = {kappa, kappa};
  std::vector<whmc_cg_stats> st(2);
  whmc_status rc = cg_solve(c, x, rhs, kap, 2, p, st.data());
  if (log) {
    log->iters += st[0].iters + st[1].iters;
    log->n += 2;
  }
  return rc;
}

// out = (sum_n b_n K^n + alpha M_oo^{-1}) phi; trailing zero coefficients are skipped and
// alpha = 0 needs no solve
whmc_status series_inverse(whmc_ctx* c, double* out, const double* phi, std::vector<double> b, double alpha,
                           double kappa, const whmc_cg_params* sp, SolveLog* log) {
  Fields F{c, (size_t)c->Vh * 192};
  double *te, *to, *g5phi, *s3, *tmp;
  WHMC_TRY(F.get("fi_te", 0, &te));
  WHMC_TRY(F.get("fi_to", 0, &to));
  WHMC_TRY(F.get("fi_g5phi", 0, &g5phi));
  WHMC_TRY(F.get("fi_s3", 0, &s3));
  WHMC_TRY(F.get("fi_tmp", 0, &tmp));
  while (b.size() > 1 && b.back() == 0.0) b.pop_back();
  const bool poly = b.size() > 1 || b[0] != 0.0;
  if (alpha != 0.0) {
    WHMC_TRY(gamma5_f64(c, g5phi, phi, 1));
    WHMC_TRY(solve(c, s3, g5phi, kappa, sp, log));
    // M_oo^{-1} phi = M_oo^dag gamma_5 s3
    WHMC_TRY(gamma5_f64(c, tmp, s3, 1));
    WHMC_TRY(apply_Moo_f64(c, poly ? to : out, tmp, kappa, 1, te));
  }
  if (!poly) {
    if (alpha == 0.0) return zero_bytes(c, out, (size_t)c->Vh * 192);
    return alpha == 1.0 ? WHMC_OK : axpby_f64(c, out, 0.0, tmp, alpha, 1);
  }
  WHMC_TRY(poly_K(c, out, phi, b, kappa, te, tmp, 0));
  return alpha == 0.0 ? WHMC_OK : axpby_f64(c, out, alpha, to, 1.0, 1);
}

// M~^{-1} phi truncated at n_max, into out
static whmc_status filtered_inverse(whmc_ctx* c, double* out, const double* phi, const whmc_filter* f, double kappa,
                                    const whmc_cg_params* sp, SolveLog* log) {
  std::vector<double> b, cc;
  double alpha;
  coefficients(f->k, f->k == 0 ? 0 : f->n_max, b, cc, alpha);
  return series_inverse(c, out, phi, b, alpha, kappa, sp, log);
}

whmc_status pf_action(whmc_ctx* c, const double* phi, const whmc_filter* f, double kappa, const whmc_cg_params* sp,
                      double* S, SolveLog* log) {
  double* z;
  Fields F{c, (size_t)c->Vh * 192};
  WHMC_TRY(F.get("act_z", 0, &z));
  WHMC_TRY(filtered_inverse(c, z, phi, f, kappa, sp, log));
  WHMC_TRY(norm2_f64(c, z, 1, c->red.result + 7));
  return read_scalar(c, c->red.result + 7, S);
}

// Force of S = |(sum_{n<=nt} b_n K^n + alpha M_oo^{-1}) phi|^2, scaled by `scale` and added to out
// (accumulate) or stored.  alpha = 0 (a polynomial action) needs no solve and has no (X~, Y~)
// pair; b_0 alone (nt = 0) carries no K and no force of its own.
whmc_status series_force(whmc_ctx* c, double* out, const double* phi, const std::vector<double>& b, double alpha,
                         double kappa, const whmc_cg_params* sp, double scale, int accumulate, SolveLog* log) {
  Fields F{c, (size_t)c->Vh * 192};
  const int nt = (int)b.size() - 1;
  double *te, *to, *rhs2, *sol2, *Yt, *Yte, *Xt, *Xte, *tmp;
  WHMC_TRY(F.get("ff_te", 0, &te));
  WHMC_TRY(F.get("ff_to", 0, &to));
  WHMC_TRY(F.get("ff_tmp", 0, &tmp));
  {
    void* v;
    WHMC_TRY(workspace(c, "ff_rhs2", 2 * F.hb, &v));
    rhs2 = (double*)v;
    WHMC_TRY(workspace(c, "ff_sol2", 2 * F.hb, &v));
    sol2 = (double*)v;
  }
  WHMC_TRY(F.get("ff_Yt", 0, &Yt));
  WHMC_TRY(F.get("ff_Yte", 0, &Yte));
  WHMC_TRY(F.get("ff_Xt", 0, &Xt));
  WHMC_TRY(F.get("ff_Xte", 0, &Xte));
  std::vector<double*> Y(nt + 1), Ye(nt + 1), X(nt + 1), Xe(nt + 1);
  for (int i = 0; i <= nt; ++i) {
    WHMC_TRY(F.get("ff_Y", i, &Y[i]));
    WHMC_TRY(F.get("ff_Ye", i, &Ye[i]));
    WHMC_TRY(F.get("ff_X", i, &X[i]));
    WHMC_TRY(F.get("ff_Xe", i, &Xe[i]));
  }
  const bool poly = nt >= 1 || b[0] != 0.0;
  const bool inv = alpha != 0.0;
  double* Y0 = rhs2;                       // first rhs of the batched solve
  double* g5phi = rhs2 + (size_t)c->Vh * 24;
  if (poly) {
    // Horner: Y_nt = b_nt phi; Y_{i-1} = b_{i-1} phi + K Y_i  (Ye[i] = H_eo Y_i)
    double* top = nt >= 1 ? Y[nt] : Y0;
    WHMC_TRY(zero_bytes(c, top, F.hb));
    WHMC_TRY(axpby_f64(c, top, b[nt], phi, 0.0, 1));
    for (int i = nt; i >= 1; --i)
      WHMC_TRY(apply_K_f64(c, i == 1 ? Y0 : Y[i - 1], Y[i], kappa, 0, Ye[i], phi, b[i - 1]));
  }
  std::vector<const double*> pXe, pXo, pYe, pYo;
  if (inv) {
    WHMC_TRY(gamma5_f64(c, g5phi, phi, 1));
    double* s2 = sol2;
    double* s3 = sol2 + (size_t)c->Vh * 24;
    if (poly) {
      WHMC_TRY(solve2(c, sol2, rhs2, kappa, sp, log));
    } else {
      WHMC_TRY(solve(c, s3, g5phi, kappa, sp, log));
    }
    // Y~ = alpha M_oo^dag g5 s3 ;  X~ = M_oo s2 + alpha g5 s3
    WHMC_TRY(gamma5_f64(c, tmp, s3, 1));
    WHMC_TRY(apply_Moo_f64(c, Yt, tmp, kappa, 1, te));
    if (alpha != 1.0) WHMC_TRY(axpby_f64(c, Yt, 0.0, tmp, alpha, 1));     // Yt = alpha * Yt
    if (poly) {
      WHMC_TRY(apply_Moo_f64(c, Xt, s2, kappa, 0, te));
      WHMC_TRY(axpby_f64(c, Xt, alpha, tmp, 1.0, 1));
    } else {
      WHMC_TRY(copy_f64(c, Xt, tmp, 1));
      if (alpha != 1.0) WHMC_TRY(axpby_f64(c, Xt, 0.0, tmp, alpha, 1));
    }
    // even halves of the (X~, Y~) pair
    WHMC_TRY(hop(c, WHMC_F64, WHMC_L18, 0, 0, Yte, Yt, nullptr, 0.0, 1.0, nullptr));
    WHMC_TRY(hop(c, WHMC_F64, WHMC_L18, 0, 1, Xte, Xt, nullptr, 0.0, 1.0, nullptr));
    pXe.push_back(Xte);
    pXo.push_back(Xt);
    pYe.push_back(Yte);
    pYo.push_back(Yt);
  }
  if (nt >= 1) {
    // X_1 = Y_0 + Y~;  X_{i+1} = K^dag X_i with Xe[i] = (H^dag)_eo X_i
    WHMC_TRY(copy_f64(c, X[1], Y0, 1));
    if (inv) WHMC_TRY(axpby_f64(c, X[1], 1.0, Yt, 1.0, 1));
    for (int i = 1; i < nt; ++i) WHMC_TRY(apply_K_f64(c, X[i + 1], X[i], kappa, 1, Xe[i], nullptr, 0.0));
    WHMC_TRY(hop(c, WHMC_F64, WHMC_L18, 0, 1, Xe[nt], X[nt], nullptr, 0.0, 1.0, nullptr));
    for (int i = 1; i <= nt; ++i) {
      pXe.push_back(Xe[i]);
      pXo.push_back(X[i]);
      pYe.push_back(Ye[i]);
      pYo.push_back(Y[i]);
    }
  }
  if (pXe.empty()) {
    if (!accumulate) WHMC_TRY(zero_bytes(c, out, (size_t)c->Vh * 64 * sizeof(double)));
    return WHMC_OK;
  }
  return pf_force_pairs(c, out, pXe.data(), pXo.data(), pYe.data(), pYo.data(), (int)pXe.size(),
                        scale * kappa * kappa, accumulate);
}

// pseudo-fermion force of the kappa^(2k) filtered action; out = (acc ? out : 0) + scale F
whmc_status pf_force(whmc_ctx* c, double* out, const double* phi, const whmc_filter* f, double kappa,
                     const whmc_cg_params* sp, double scale, int accumulate, SolveLog* log) {
  const int nt = f->k == 0 ? 0 : f->n_t;   // k = 0: plain action, no polynomial part
  std::vector<double> b, cc;
  double alpha;
  coefficients(f->k, nt, b, cc, alpha);
  return series_force(c, out, phi, b, alpha, kappa, sp, scale, accumulate, log);
}

whmc_status heatbath(whmc_ctx* c, double* phi, const double* eta, const whmc_filter* f, double kappa) {
  Fields F{c, (size_t)c->Vh * 192};
  double *te, *to, *tmp;
  WHMC_TRY(F.get("hb_te", 0, &te));
  WHMC_TRY(F.get("hb_to", 0, &to));
  WHMC_TRY(F.get("hb_tmp", 0, &tmp));
  std::vector<double> b, cc;
  double alpha;
  coefficients(f->k, f->k == 0 ? 0 : f->n_max, b, cc, alpha);
  WHMC_TRY(poly_K(c, tmp, eta, cc, kappa, te, to, 0));
  return apply_Moo_f64(c, phi, tmp, kappa, 0, te);
}

// ------------------------------------------------------------------ HMC
namespace {
// Sexton-Weingarten nesting (Sec. 1): level 0 has the T steps between its P steps, one (half)
// step of level l >= 1 holds lv[l].nsub steps of level l - 1.  P steps are queued per level and
// applied before the next T step, so consecutive P steps on the same field cost one force.
struct MDRun {
  whmc_ctx* c;
  double* pi;
  const std::vector<MDLevel>& lv;
  int integrator;
  double lambda;
  std::vector<double> pending;

  whmc_status flush() {
    static const char* names[] = {"whmc md P step, level 0", "whmc md P step, level 1", "whmc md P step, level 2",
                                  "whmc md P step, level 3", "whmc md P step, level 4", "whmc md P step, level 5+"};
    for (size_t l = 0; l < lv.size(); ++l)
      if (pending[l] != 0.0) {
        TraceRange tr(names[l < 5 ? l : 5]);
        WHMC_TRY(lv[l].force(-pending[l]));
        pending[l] = 0.0;
      }
    return WHMC_OK;
  }
  whmc_status T(double eps) {
    WHMC_TRY(flush());
    TraceRange tr("whmc md T step");
    return link_update(c, pi, eps);
  }
  whmc_status sub(int level, double span) {
    if (level == 0) return T(span);
    const int n = lv[level].nsub;
    for (int k = 0; k < n; ++k) WHMC_TRY(run(level - 1, span / n));
    return WHMC_OK;
  }
  whmc_status run(int level, double eps) {
    if (integrator == WHMC_OMELYAN) {
      pending[level] += lambda * eps;
      WHMC_TRY(sub(level, eps / 2));
      pending[level] += (1 - 2 * lambda) * eps;
      WHMC_TRY(sub(level, eps / 2));
      pending[level] += lambda * eps;
    } else {
      pending[level] += eps / 2;
      WHMC_TRY(sub(level, eps));
      pending[level] += eps / 2;
    }
    return WHMC_OK;
  }
};
}  // namespace

whmc_status md_levels(whmc_ctx* c, double* pi, const std::vector<MDLevel>& lv, int integrator, double lambda,
                      double tau, int m) {
  MDRun r{c, pi, lv, integrator, lambda, std::vector<double>(lv.size(), 0.0)};
  const int top = (int)lv.size() - 1;
  for (int k = 0; k < m; ++k) WHMC_TRY(r.run(top, tau / m));
  return r.flush();
}

whmc_status term_hamiltonian(whmc_ctx* c, const TermAction& A, const double* pi, const double* phi, double* H,
                             SolveLog* log) {
  double pp, plaq;
  std::vector<double> S(A.nterms);
  WHMC_TRY(algebra_norm2(c, pi, &pp));
  WHMC_TRY(plaquette_sum(c, &plaq));
  WHMC_TRY(A.action(S.data(), phi, log));
  *H = 0.5 * pp - A.beta_eff / 3.0 * plaq;
  for (double v : S) *H += v;
  return WHMC_OK;
}

whmc_status term_md(whmc_ctx* c, const TermAction& A, const TermMD& md, double* pi, const double* phi,
                    SolveLog* log) {
  std::vector<MDLevel> lv(A.nterms + 1);
  const double beff = A.beta_eff;
  lv[0].force = [=](double s) { return gauge_force(c, pi, beff, s, 1); };
  for (int t = 1; t <= A.nterms; ++t) {
    lv[t].force = [=, &A](double s) { return A.force(pi, phi, t, s, 1, log); };
    lv[t].nsub = md.msub[t - 1];
  }
  return md_levels(c, pi, lv, md.integrator, md.lambda, md.tau, md.m);
}

// heat bath, H0, molecular dynamics, H1, Metropolis; the gauge field is restored on rejection
whmc_status term_trajectory(whmc_ctx* c, const TermAction& A, const TermMD& md, const double* pi0, const double* eta,
                            double u, whmc_traj_result* res) {
  TraceRange tr("whmc trajectory (multi-term)");
  const auto t0 = std::chrono::steady_clock::now();
  void *pi, *phi, *Usave;
  const size_t ab = (size_t)64 * c->Vh * sizeof(double);
  const size_t ub = (size_t)8 * 9 * c->Vh * sizeof(double2);
  WHMC_TRY(workspace(c, "term_pi", ab, &pi));
  WHMC_TRY(workspace(c, "term_phi", (size_t)A.nfields * c->Vh * 192, &phi));
  WHMC_TRY(workspace(c, "hmc_Usave", ub, &Usave));
  WHMC_HIP(hipMemcpyAsync(pi, pi0, ab, hipMemcpyDeviceToDevice, c->stream));
  WHMC_HIP(hipMemcpyAsync(Usave, c->U18, ub, hipMemcpyDeviceToDevice, c->stream));
  long long hb_iters = 0;
  SolveLog log, mdlog;
  WHMC_TRY(A.heatbath((double*)phi, eta, &hb_iters, &log));
  double H0, H1;
  WHMC_TRY(term_hamiltonian(c, A, (double*)pi, (double*)phi, &H0, &log));
  WHMC_TRY(term_md(c, A, md, (double*)pi, (const double*)phi, &mdlog));
  WHMC_TRY(term_hamiltonian(c, A, (double*)pi, (double*)phi, &H1, &log));
  const double dH = H1 - H0;
  const bool finite = std::isfinite(dH);
  const bool acc = finite && u < std::exp(-dH);
  if (!acc) {
    WHMC_HIP(hipMemcpyAsync(c->U18, Usave, ub, hipMemcpyDeviceToDevice, c->stream));
    WHMC_TRY(gauge_changed(c));
  }
  double plaq;
  WHMC_TRY(plaquette_sum(c, &plaq));
  res->dH = dH;
  res->H0 = H0;
  res->H1 = H1;
  res->accepted = acc ? 1 : 0;
  res->plaquette = plaq / (18.0 * (double)c->V);
  res->cg_iters = log.iters + mdlog.iters;
  res->n_solves = log.n + mdlog.n;
  res->poly_iters = hb_iters;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  WHMC_CHECK(finite, WHMC_ENONFINITE, "trajectory: dH is not finite; the gauge field was restored");
  return WHMC_OK;
}

// gauge action on level 0, the filtered pseudo-fermion action on level 1
static whmc_status filter_md(whmc_ctx* c, const whmc_hmc_params* p, double* pi, const double* phi, SolveLog* log) {
  const double beff = p->beta + delta_beta(p->kappa, p->filter.k);
  std::vector<MDLevel> lv(2);
  lv[0].force = [=](double s) { return gauge_force(c, pi, beff, s, 1); };
  lv[1].force = [=](double s) { return pf_force(c, pi, phi, &p->filter, p->kappa, &p->md_solver, s, 1, log); };
  lv[1].nsub = p->m0;
  return md_levels(c, pi, lv, p->integrator, p->lambda, p->tau, p->m);
}

static whmc_status check_hmc(const whmc_hmc_params* p) {
  WHMC_CHECK(p, WHMC_EARG, "null hmc params");
  WHMC_TRY(check_filter(&p->filter));
  WHMC_CHECK(p->m >= 1 && p->m0 >= 1 && p->tau > 0, WHMC_EARG, "hmc: m, m0 >= 1 and tau > 0 required");
  WHMC_CHECK(p->integrator == WHMC_LEAPFROG || p->integrator == WHMC_OMELYAN, WHMC_EARG, "hmc: unknown integrator");
  return WHMC_OK;
}

static whmc_status hamiltonian(whmc_ctx* c, const whmc_hmc_params* p, const double* pi, const double* phi, double* H,
                               SolveLog* log) {
  double pp, plaq, spf;
  WHMC_TRY(algebra_norm2(c, pi, &pp));
  WHMC_TRY(plaquette_sum(c, &plaq));
  WHMC_TRY(pf_action(c, phi, &p->filter, p->kappa, &p->action_solver, &spf, log));
  const double beff = p->beta + delta_beta(p->kappa, p->filter.k);
  *H = 0.5 * pp - beff / 3.0 * plaq + spf;
  return WHMC_OK;
}

}  // namespace whmc

using namespace whmc;

extern "C" {

whmc_status whmc_filter_coefficients(int k, int n, double* b, double* c, double* alpha) {
  WHMC_CHECK(k >= 0 && k <= 64 && n >= 0 && n <= 1000, WHMC_EARG, "whmc_filter_coefficients: bad k or n");
  std::vector<double> bb, cc;
  double a;
  coefficients(k, n, bb, cc, a);
  for (int i = 0; i <= n; ++i) {
    if (b) b[i] = bb[i];
    if (c) c[i] = cc[i];
  }
  if (alpha) *alpha = a;
  return WHMC_OK;
}

whmc_status whmc_heatbath_phi(whmc_ctx* c, double* phi, const double* eta, const whmc_filter* f, double kappa) {
  WHMC_CHECK(c && phi && eta && phi != eta, WHMC_EARG, "whmc_heatbath_phi: bad argument");
  WHMC_TRY(check_filter(f));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  return heatbath(c, phi, eta, f, kappa);
}

whmc_status whmc_action(whmc_ctx* c, double* S_G, double* S_PF, const double* phi, const whmc_filter* f,
                        double kappa, double beta, const whmc_cg_params* solver) {
  WHMC_CHECK(c, WHMC_EARG, "null context");
  WHMC_TRY(check_filter(f));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  if (S_G) {
    double plaq;
    WHMC_TRY(plaquette_sum(c, &plaq));
    *S_G = -(beta + delta_beta(kappa, f->k)) / 3.0 * plaq;
  }
  if (S_PF) {
    WHMC_CHECK(phi, WHMC_EARG, "whmc_action: phi is null");
    WHMC_TRY(pf_action(c, phi, f, kappa, &sp, S_PF, nullptr));
  }
  return WHMC_OK;
}

whmc_status whmc_force(whmc_ctx* c, double* F, const double* phi, const whmc_filter* f, double kappa, double beta,
                       const whmc_cg_params* solver, int flags) {
  WHMC_CHECK(c && F, WHMC_EARG, "whmc_force: null argument");
  WHMC_TRY(check_filter(f));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  int acc = (flags & WHMC_FORCE_ACCUMULATE) ? 1 : 0;
  if (!(flags & (WHMC_FORCE_PF | WHMC_FORCE_GAUGE)) && !acc) return zero_bytes(c, F, (size_t)64 * c->Vh * 8);
  if (flags & WHMC_FORCE_GAUGE) {
    WHMC_TRY(gauge_force(c, F, beta + delta_beta(kappa, f->k), 1.0, acc));
    acc = 1;
  }
  if (flags & WHMC_FORCE_PF) {
    WHMC_CHECK(phi, WHMC_EARG, "whmc_force: phi is null");
    WHMC_TRY(pf_force(c, F, phi, f, kappa, &sp, 1.0, acc, nullptr));
  }
  return WHMC_OK;
}

whmc_status whmc_hamiltonian(whmc_ctx* c, const whmc_hmc_params* p, const double* pi, const double* phi, double* H) {
  WHMC_CHECK(c && pi && phi && H, WHMC_EARG, "whmc_hamiltonian: null argument");
  WHMC_TRY(check_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  return hamiltonian(c, p, pi, phi, H, nullptr);
}

whmc_status whmc_md_integrate(whmc_ctx* c, const whmc_hmc_params* p, double* pi, const double* phi) {
  WHMC_CHECK(c && pi && phi, WHMC_EARG, "whmc_md_integrate: null argument");
  WHMC_TRY(check_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  WHMC_TRY(filter_md(c, p, pi, phi, nullptr));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  return WHMC_OK;
}

whmc_status whmc_hmc_trajectory(whmc_ctx* c, const whmc_hmc_params* p, const double* pi0, const double* eta,
                                double u, whmc_traj_result* res) {
  WHMC_CHECK(c && pi0 && eta && res, WHMC_EARG, "whmc_hmc_trajectory: null argument");
  WHMC_TRY(check_hmc(p));
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  TraceRange tr("whmc trajectory");
  const auto t0 = std::chrono::steady_clock::now();
  void *pi, *phi, *Usave;
  const size_t ab = (size_t)64 * c->Vh * sizeof(double);
  const size_t ub = (size_t)8 * 9 * c->Vh * sizeof(double2);
  WHMC_TRY(workspace(c, "hmc_pi", ab, &pi));
  WHMC_TRY(workspace(c, "hmc_phi", (size_t)c->Vh * 192, &phi));
  WHMC_TRY(workspace(c, "hmc_Usave", ub, &Usave));
  WHMC_HIP(hipMemcpyAsync(pi, pi0, ab, hipMemcpyDeviceToDevice, c->stream));
  WHMC_HIP(hipMemcpyAsync(Usave, c->U18, ub, hipMemcpyDeviceToDevice, c->stream));
  WHMC_TRY(heatbath(c, (double*)phi, eta, &p->filter, p->kappa));
  SolveLog log;
  double H0, H1;
  WHMC_TRY(hamiltonian(c, p, (double*)pi, (double*)phi, &H0, &log));
  SolveLog mdlog;
  WHMC_TRY(filter_md(c, p, (double*)pi, (const double*)phi, &mdlog));
  WHMC_TRY(hamiltonian(c, p, (double*)pi, (double*)phi, &H1, &log));
  const double dH = H1 - H0;
  const bool finite = std::isfinite(dH);
  const bool acc = finite && u < std::exp(-dH);
  if (!acc) {
    WHMC_HIP(hipMemcpyAsync(c->U18, Usave, ub, hipMemcpyDeviceToDevice, c->stream));
    WHMC_TRY(gauge_changed(c));
  }
  double plaq;
  WHMC_TRY(plaquette_sum(c, &plaq));
  res->dH = dH;
  res->H0 = H0;
  res->H1 = H1;
  res->accepted = acc ? 1 : 0;
  res->plaquette = plaq / (18.0 * (double)c->V);
  res->cg_iters = log.iters + mdlog.iters;
  res->n_solves = log.n + mdlog.n;
  res->poly_iters = 0;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  WHMC_CHECK(finite, WHMC_ENONFINITE, "trajectory: dH is not finite; the gauge field was restored");
  return WHMC_OK;
}

}  // extern "C"
