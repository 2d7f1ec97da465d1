// The fermion matrix on the whole lattice, M = 1 - kappa H (Sec. 1), without the even/odd reduction
// of Sec. 2.2: M and M^dag, M^dag M, FP64 CG on M^dag M, and the unfiltered pseudo-fermion action and
// force S = |M^{-1} phi|^2 with X = (M M^dag)^{-1} phi, Y = M^dag X (Sec. 2).
//
// A full spinor is the even half followed by the odd half (whmc layout).  Both parities of M are
// one launch of 2 nb workgroups (site_block_pair): the XCD that computes the even sites of a region
// also computes its odd sites, so each input spinor is read near its neighbours.
//
// CG iteration (scalars on the device, as in the even/odd solver):
//   1  t = M p,  (p, M^dag M p) = |t|^2                 -> alpha
//   2  A p = M^dag t;  r -= alpha A p;  x += alpha p;  |r|^2  -> beta, stop test
//   3  p = r + beta p
#include <chrono>
#include <cmath>

#include "internal.h"
#include "stencil.h"

namespace whmc {

WHMC_DEV bool full_halted(const CGScalars* sc) { return sc->done | sc->pause; }

// out_p = in_p - kappa (H^(dag) in)_p for both parities p; NORM: |out|^2 to the partial sums;
// HALT: return at once when the solve has stopped
template <int DAG, bool NORM, bool HALT, class Lnk>
__global__ __launch_bounds__(kBlock) void k_fullM(Geom g, Lnk L, SpinorF64 in_e, SpinorF64 in_o, SpinorF64 out_e,
                                                  SpinorF64 out_o, double kappa, const CGScalars* sc, Reduce red) {
  if (HALT && full_halted(sc)) return;
  int par;
  const int i = site_block_pair(g, blockIdx.x, gridDim.x >> 1, par) * kBlock + threadIdx.x;
  double nrm = 0.0;
  if (i < g.Vh) {
    Spinor<double> acc, xv;
    hop_site<DAG>(g, par, i, L, par ? in_e : in_o, acc);
    (par ? in_o : in_e).load(i, xv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.c[s][c] = xv.c[s][c] - kappa * acc.c[s][c];
    (par ? out_o : out_e).store(i, acc);
    if (NORM) nrm = norm2(acc);
  }
  if (NORM) block_partial<kBlock>(nrm, red.partials, blockIdx.x);
}

// A p = t - kappa H^dag t at the site, then r -= alpha A p, x += alpha p, |r|^2 to the partials
template <class Lnk>
__global__ __launch_bounds__(kBlock) void k_fullM_update(Geom g, Lnk L, SpinorF64 t_e, SpinorF64 t_o, SpinorF64 p_e,
                                                         SpinorF64 p_o, SpinorF64 r_e, SpinorF64 r_o, SpinorF64 x_e,
                                                         SpinorF64 x_o, double kappa, const CGScalars* sc,
                                                         Reduce red) {
  if (full_halted(sc)) return;
  int par;
  const int i = site_block_pair(g, blockIdx.x, gridDim.x >> 1, par) * kBlock + threadIdx.x;
  const double alpha = sc->alpha;
  double nrm = 0.0;
  if (i < g.Vh) {
    Spinor<double> acc, tv, pv, rv, xv;
    hop_site<1>(g, par, i, L, par ? t_e : t_o, acc);
    (par ? t_o : t_e).load(i, tv);
    (par ? p_o : p_e).load(i, pv);
    (par ? r_o : r_e).load(i, rv);
    (par ? x_o : x_e).load(i, xv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cplx<double> ap = tv.c[s][c] - kappa * acc.c[s][c];
        rv.c[s][c] = rv.c[s][c] - alpha * ap;
        xv.c[s][c] = xv.c[s][c] + alpha * pv.c[s][c];
      }
    (par ? r_o : r_e).store(i, rv);
    (par ? x_o : x_e).store(i, xv);
    nrm = norm2(rv);
  }
  block_partial<kBlock>(nrm, red.partials, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_full_alpha(CGScalars* sc, const double* partials, int nb) {
  if (full_halted(sc)) return;
  const double pAp = sum_partials<256>(partials, nb);
  if (threadIdx.x != 0) return;
  sc->pAp = pAp;
  if (pAp > 0.0 && pAp < INFINITY) {
    sc->alpha = sc->rr / pAp;
  } else {
    sc->alpha = 0.0;
    sc->done = 1;   // breakdown: p = 0 or not finite
  }
}

__global__ __launch_bounds__(256) void k_full_beta(CGScalars* sc, const double* partials, int nb) {
  if (full_halted(sc)) return;
  const double rr_new = sum_partials<256>(partials, nb);
  if (threadIdx.x != 0) return;
  sc->beta = rr_new / sc->rr;
  sc->rr_old = sc->rr;
  sc->rr = rr_new;
  sc->iter += 1;
  if (!(rr_new < INFINITY) || rr_new <= sc->stop_rr) sc->done = 1;
}

// p = r + beta p over the flat full field (n complex entries)
__global__ void k_full_p(long long n, double2* p, const double2* r, const CGScalars* sc) {
  if (full_halted(sc)) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = sc->beta;
  const double2 rv = r[i], pv = p[i];
  p[i] = make_double2(rv.x + beta * pv.x, rv.y + beta * pv.y);
}

// |r|^2 of this pass from the device, absolute stop threshold
__global__ void k_full_init(CGScalars* sc, const double* rr, double stop_rr) {
  if (threadIdx.x != 0) return;
  sc->rr = *rr;
  sc->stop_rr = stop_rr;
  sc->done = (*rr <= stop_rr);
  sc->pause = 0;
  sc->iter = 0;
  sc->alpha = sc->beta = sc->pAp = sc->rr_old = 0.0;
}

static SpinorF64 half64(const double* base, int Vh, int par) {
  return SpinorF64{(double2*)(base + (size_t)par * 24 * Vh), Vh};
}

template <class Lnk>
static void launch_fullM(whmc_ctx* c, const Lnk& L, int dagger, double* out, const double* in, double kappa) {
  const int Vh = c->Vh;
  const dim3 grid(2 * c->stencil_blocks()), block(kBlock);
  if (dagger)
    hipLaunchKernelGGL((k_fullM<1, false, false, Lnk>), grid, block, 0, c->stream, c->g, L, half64(in, Vh, 0),
                       half64(in, Vh, 1), half64(out, Vh, 0), half64(out, Vh, 1), kappa, nullptr, c->red);
  else
    hipLaunchKernelGGL((k_fullM<0, false, false, Lnk>), grid, block, 0, c->stream, c->g, L, half64(in, Vh, 0),
                       half64(in, Vh, 1), half64(out, Vh, 0), half64(out, Vh, 1), kappa, nullptr, c->red);
}

whmc_status apply_M_full(whmc_ctx* c, double* out, const double* in, double kappa, int dagger) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  if (c->stream_links(WHMC_F64, WHMC_L18)) launch_fullM(c, LinkF64_18T<true>{c->U18, c->Vh}, dagger, out, in, kappa);
  else launch_fullM(c, LinkF64_18T<false>{c->U18, c->Vh}, dagger, out, in, kappa);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

whmc_status apply_MdagM_full(whmc_ctx* c, double* out, const double* in, double kappa, double* tmp_full) {
  WHMC_TRY(apply_M_full(c, tmp_full, in, kappa, 0));
  return apply_M_full(c, out, tmp_full, kappa, 1);
}

namespace {
struct FullTimer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double s() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};
}  // namespace

// |b - M^dag M x| / |b| in FP64 with 18-real links; r receives b - M^dag M x
static whmc_status full_residual(whmc_ctx* c, double* r, const double* x, const double* b, double kappa, double* tmp,
                                 double bb, double* rel) {
  WHMC_TRY(apply_MdagM_full(c, r, x, kappa, tmp));
  WHMC_TRY(axpby_f64(c, r, 1.0, b, -1.0, 2));
  double rr;
  WHMC_TRY(norm2_f64(c, r, 2, c->red.result + 2));
  WHMC_TRY(read_scalar(c, c->red.result + 2, &rr));
  *rel = std::sqrt(rr / bb);
  return WHMC_OK;
}

template <class Lnk>
static whmc_status cg_full_impl(whmc_ctx* c, const Lnk& L, double* x, const double* b, double kappa,
                                const whmc_cg_params* prm, whmc_cg_stats* st) {
  FullTimer tm;
  const int Vh = c->Vh;
  const size_t fb = (size_t)Vh * 384;
  void *r, *p, *t, *tmp;
  WHMC_TRY(workspace(c, "fcg_r", fb, &r));
  WHMC_TRY(workspace(c, "fcg_p", fb, &p));
  WHMC_TRY(workspace(c, "fcg_t", fb, &t));
  WHMC_TRY(workspace(c, "fcg_tmp", fb, &tmp));
  double* R = (double*)r;
  double* P = (double*)p;
  double* T = (double*)t;
  WHMC_TRY(norm2_f64(c, b, 2, c->red.result + 3));
  double bb;
  WHMC_TRY(read_scalar(c, c->red.result + 3, &bb));
  *st = whmc_cg_stats{};
  WHMC_CHECK(std::isfinite(bb), WHMC_ENONFINITE, "whmc_cg_solve_full: the right-hand side is not finite");
  WHMC_TRY(zero_bytes(c, x, fb));
  if (bb == 0.0) {
    st->converged = 1;
    st->seconds = tm.s();
    return WHMC_OK;
  }
  const dim3 grid(2 * c->stencil_blocks()), block(kBlock);
  const long long n = 24LL * Vh;   // complex entries of a full field
  const int check = prm->check_every > 0 ? prm->check_every : 8;
  int total = 0;
  double rel = 0.0;
  for (int pass = 0; pass < 4; ++pass) {
    if (pass == 0) WHMC_TRY(copy_f64(c, R, b, 2));
    else WHMC_TRY(full_residual(c, R, x, b, kappa, (double*)tmp, bb, &rel));
    WHMC_TRY(copy_f64(c, P, R, 2));
    WHMC_TRY(norm2_f64(c, R, 2, c->red.result + 4));
    hipLaunchKernelGGL(k_full_init, dim3(1), dim3(64), 0, c->stream, c->scal, c->red.result + 4,
                       prm->tol * prm->tol * bb);
    WHMC_HIP(hipGetLastError());
    CGScalars hs{};
    int pass_iters = 0;
    while (true) {
      const int k = std::min(check, prm->maxiter - total - pass_iters);
      if (k <= 0) break;
      for (int it = 0; it < k; ++it) {
        TraceRange tr("whmc full-lattice cg iteration");
        hipLaunchKernelGGL((k_fullM<0, true, true, Lnk>), grid, block, 0, c->stream, c->g, L, half64(P, Vh, 0),
                           half64(P, Vh, 1), half64(T, Vh, 0), half64(T, Vh, 1), kappa, c->scal, c->red);
        hipLaunchKernelGGL(k_full_alpha, dim3(1), dim3(256), 0, c->stream, c->scal, c->red.partials, (int)grid.x);
        hipLaunchKernelGGL((k_fullM_update<Lnk>), grid, block, 0, c->stream, c->g, L, half64(T, Vh, 0),
                           half64(T, Vh, 1), half64(P, Vh, 0), half64(P, Vh, 1), half64(R, Vh, 0), half64(R, Vh, 1),
                           half64(x, Vh, 0), half64(x, Vh, 1), kappa, c->scal, c->red);
        hipLaunchKernelGGL(k_full_beta, dim3(1), dim3(256), 0, c->stream, c->scal, c->red.partials, (int)grid.x);
        hipLaunchKernelGGL(k_full_p, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, (double2*)P,
                           (const double2*)R, c->scal);
      }
      WHMC_HIP(hipGetLastError());
      WHMC_HIP(hipMemcpyAsync(c->scal_host, c->scal, sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
      WHMC_HIP(hipStreamSynchronize(c->stream));
      hs = c->scal_host[0];
      pass_iters = hs.iter;
      if (hs.done) break;
    }
    total += pass_iters;
    WHMC_TRY(full_residual(c, R, x, b, kappa, (double*)tmp, bb, &rel));
    st->true_residual = rel;
    WHMC_CHECK(std::isfinite(rel), WHMC_ENONFINITE, "whmc_cg_solve_full: the residual is not finite");
    if (rel <= prm->tol) {
      st->converged = 1;
      break;
    }
    if (total >= prm->maxiter) break;
  }
  st->iters = total;
  st->seconds = tm.s();
  if (!st->converged) {
    set_error("whmc_cg_solve_full: no convergence: true residual " + std::to_string(rel) + " after " +
              std::to_string(total) + " iterations");
    return WHMC_ENOCONV;
  }
  return WHMC_OK;
}

whmc_status cg_full(whmc_ctx* c, double* x, const double* b, double kappa, const whmc_cg_params* prm,
                    whmc_cg_stats* st) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  WHMC_CHECK(prm->prec == WHMC_F64, WHMC_EUNSUP, "whmc_cg_solve_full: FP64 only");
  WHMC_CHECK(prm->links == WHMC_L18 || prm->links == WHMC_L12, WHMC_EARG, "whmc_cg_solve_full: links must be 12 or 18");
  whmc_cg_stats local{};
  whmc_cg_stats* s = st ? st : &local;
  const int Vh = c->Vh;
  if (prm->links == WHMC_L12) {
    WHMC_TRY(ensure_links(c, WHMC_F64, WHMC_L12));
    if (c->stream_links(WHMC_F64, WHMC_L12)) return cg_full_impl(c, LinkF64_12T<true>{c->U12, Vh}, x, b, kappa, prm, s);
    return cg_full_impl(c, LinkF64_12T<false>{c->U12, Vh}, x, b, kappa, prm, s);
  }
  if (c->stream_links(WHMC_F64, WHMC_L18)) return cg_full_impl(c, LinkF64_18T<true>{c->U18, Vh}, x, b, kappa, prm, s);
  return cg_full_impl(c, LinkF64_18T<false>{c->U18, Vh}, x, b, kappa, prm, s);
}

// X = gamma_5 (M^dag M)^{-1} gamma_5 phi = (M M^dag)^{-1} phi and Y = M^dag X
static whmc_status full_pair(whmc_ctx* c, const double* phi, double kappa, const whmc_cg_params* sp, double** X,
                             double** Y) {
  const size_t fb = (size_t)c->Vh * 384;
  void *g5, *s, *x, *y;
  WHMC_TRY(workspace(c, "fpf_g5phi", fb, &g5));
  WHMC_TRY(workspace(c, "fpf_s", fb, &s));
  WHMC_TRY(workspace(c, "fpf_X", fb, &x));
  WHMC_TRY(workspace(c, "fpf_Y", fb, &y));
  WHMC_TRY(gamma5_f64(c, (double*)g5, phi, 2));
  whmc_cg_stats st{};
  WHMC_TRY(cg_full(c, (double*)s, (const double*)g5, kappa, sp, &st));
  WHMC_TRY(gamma5_f64(c, (double*)x, (const double*)s, 2));
  WHMC_TRY(apply_M_full(c, (double*)y, (const double*)x, kappa, 1));
  *X = (double*)x;
  *Y = (double*)y;
  return WHMC_OK;
}

}  // namespace whmc

using namespace whmc;

extern "C" {

whmc_status whmc_apply_M(whmc_ctx* c, double* out, const double* in, double kappa, int dagger) {
  WHMC_CHECK(c && out && in, WHMC_EARG, "whmc_apply_M: null argument");
  WHMC_CHECK(out != in, WHMC_EARG, "whmc_apply_M: in and out must differ");
  return apply_M_full(c, out, in, kappa, dagger ? 1 : 0);
}

whmc_status whmc_cg_solve_full(whmc_ctx* c, double* x, const double* b, double kappa, const whmc_cg_params* params,
                               whmc_cg_stats* stats) {
  WHMC_CHECK(c && x && b && params, WHMC_EARG, "whmc_cg_solve_full: null argument");
  WHMC_CHECK(x != b, WHMC_EARG, "whmc_cg_solve_full: x and b must differ");
  WHMC_CHECK(params->tol > 0 && params->maxiter > 0, WHMC_EARG, "whmc_cg_solve_full: tol and maxiter must be positive");
  return cg_full(c, x, b, kappa, params, stats);
}

whmc_status whmc_action_full(whmc_ctx* c, double* S_PF, const double* phi, double kappa,
                             const whmc_cg_params* solver) {
  WHMC_CHECK(c && S_PF && phi, WHMC_EARG, "whmc_action_full: null argument");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  double *X, *Y;
  WHMC_TRY(full_pair(c, phi, kappa, &sp, &X, &Y));
  WHMC_TRY(norm2_f64(c, Y, 2, c->red.result + 7));
  return read_scalar(c, c->red.result + 7, S_PF);
}

whmc_status whmc_force_full(whmc_ctx* c, double* F, const double* phi, double kappa, double beta,
                            const whmc_cg_params* solver, int flags) {
  WHMC_CHECK(c && F, WHMC_EARG, "whmc_force_full: null argument");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const whmc_cg_params sp = solver ? *solver : default_solver();
  int acc = (flags & WHMC_FORCE_ACCUMULATE) ? 1 : 0;
  if (!(flags & (WHMC_FORCE_PF | WHMC_FORCE_GAUGE)) && !acc) return zero_bytes(c, F, (size_t)64 * c->Vh * 8);
  if (flags & WHMC_FORCE_GAUGE) {
    WHMC_TRY(gauge_force(c, F, beta, 1.0, acc));
    acc = 1;
  }
  if (flags & WHMC_FORCE_PF) {
    WHMC_CHECK(phi, WHMC_EARG, "whmc_force_full: phi is null");
    double *X, *Y;
    WHMC_TRY(full_pair(c, phi, kappa, &sp, &X, &Y));
    const size_t h = (size_t)24 * c->Vh;
    const double* Xe = X;
    const double* Xo = X + h;
    const double* Ye = Y;
    const double* Yo = Y + h;
    WHMC_TRY(pf_force_pairs(c, F, &Xe, &Xo, &Ye, &Yo, 1, kappa, acc));
  }
  return WHMC_OK;
}

}  // extern "C"
