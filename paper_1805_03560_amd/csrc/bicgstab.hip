// BiCGstab on the even/odd operator M_oo = 1 - kappa^2 H_oe H_eo (Sec. 2.2), and on its adjoint
// M_oo^dag = 1 - kappa^2 (H^dag)_oe (H^dag)_eo, in FP64: the Krylov solver the paper uses for the
// pseudo-fermion systems (Sec. 4), as an alternative to CG on M_oo^dag M_oo.
//
// Iteration (H. A. van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992) 631), with rhat = r_0 and
// complex inner products (a, b) = sum conj(a_i) b_i:
//   v = A p,  alpha = rho / (rhat, v),  s = r - alpha v,  t = A s,  omega = (t, s) / (t, t),
//   x += alpha p + omega s,  r = s - omega t,  rho' = (rhat, r),  beta = (rho' / rho)(alpha / omega),
//   p = r + beta (p - omega v).
// One iteration is two applications of A (four hops).  The scalars stay on the device; every
// kernel exits at once when the solve is done, and the host looks every check_every iterations.
// A breakdown ((rhat, v) = 0, (t, t) = 0, omega = 0 or rho' = 0) ends the pass, which then
// restarts from the true residual.  Reductions are deterministic two-pass sums.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"
#include "stencil.h"

namespace whmc {

struct BSScalars {
  double rho[2];      // (rhat, r)
  double alpha[2];
  double omega[2];
  double beta[2];
  double rr;          // |r|^2
  double stop_rr;     // stop when |r|^2 <= stop_rr
  int done;           // 1 converged, 2 breakdown
  int iter;
};
static_assert(sizeof(BSScalars) <= kMaxRhs * sizeof(CGScalars), "scalar slot too small");

WHMC_DEV bool bs_halted(const BSScalars* sc) { return sc->done != 0; }

// conj(a) b accumulated into (re, im)
WHMC_DEV void cdot_acc(const Spinor<double>& a, const Spinor<double>& b, double& re, double& im) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      re += a.c[s][c].re * b.c[s][c].re + a.c[s][c].im * b.c[s][c].im;
      im += a.c[s][c].re * b.c[s][c].im - a.c[s][c].im * b.c[s][c].re;
    }
}

// te = H_{eo}^{(DAG)} in
template <int DAG, class Lnk>
__global__ __launch_bounds__(kBlock) void k_bs_hop(Geom g, Lnk L, SpinorF64 in, SpinorF64 te, const BSScalars* sc) {
  if (bs_halted(sc)) return;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  Spinor<double> acc;
  hop_site<DAG>(g, 0, i, L, in, acc);
  te.store(i, acc);
}

// out = in - kappa^2 H_{oe}^{(DAG)} te, with the partial sums
//   MODE 0 (out = v = A p): (rhat, v)               -> 2 values
//   MODE 1 (out = t = A s): (t, s) and (t, t)        -> 3 values
template <int DAG, int MODE, class Lnk>
__global__ __launch_bounds__(kBlock) void k_bs_mv(Geom g, Lnk L, SpinorF64 te, SpinorF64 in, SpinorF64 out,
                                                  SpinorF64 aux, double k2, const BSScalars* sc, Reduce red,
                                                  int nb) {
  if (bs_halted(sc)) return;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  if (i < g.Vh) {
    Spinor<double> acc, x;
    hop_site<DAG>(g, 1, i, L, te, acc);
    in.load(i, x);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.c[s][c] = x.c[s][c] - k2 * acc.c[s][c];
    out.store(i, acc);
    if (MODE == 0) {
      Spinor<double> rh;
      aux.load(i, rh);
      cdot_acc(rh, acc, d0, d1);   // (rhat, v)
    } else {
      cdot_acc(acc, x, d0, d1);    // (t, s): in = s
      d2 = norm2(acc);             // (t, t)
    }
  }
  block_partial<kBlock>(d0, red.partials, blockIdx.x);
  block_partial<kBlock>(d1, red.partials + nb, blockIdx.x);
  if (MODE == 1) block_partial<kBlock>(d2, red.partials + 2 * nb, blockIdx.x);
}

// alpha = rho / (rhat, v)   (MODE 0)   or   omega = (t, s) / (t, t)   (MODE 1)
template <int MODE>
__global__ __launch_bounds__(256) void k_bs_fin(BSScalars* sc, const double* partials, int nb) {
  if (bs_halted(sc)) return;
  const double a = sum_partials<256>(partials, nb);
  const double b = sum_partials<256>(partials + nb, nb);
  const double c = MODE == 1 ? sum_partials<256>(partials + 2 * nb, nb) : 0.0;
  if (threadIdx.x != 0) return;
  if (MODE == 0) {
    const double den = a * a + b * b;
    if (!(den > 0.0) || !(den < INFINITY)) {
      sc->done = 2;
      return;
    }
    // rho / (a + i b)
    sc->alpha[0] = (sc->rho[0] * a + sc->rho[1] * b) / den;
    sc->alpha[1] = (sc->rho[1] * a - sc->rho[0] * b) / den;
  } else {
    if (!(c > 0.0) || !(c < INFINITY)) {
      sc->done = 2;
      return;
    }
    sc->omega[0] = a / c;
    sc->omega[1] = b / c;
    if (sc->omega[0] == 0.0 && sc->omega[1] == 0.0) sc->done = 2;
  }
}

// s = r - alpha v
__global__ __launch_bounds__(kBlock) void k_bs_s(int Vh, SpinorF64 r, SpinorF64 v, SpinorF64 s,
                                                 const BSScalars* sc) {
  if (bs_halted(sc)) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const double ar = sc->alpha[0], ai = sc->alpha[1];
  Spinor<double> rv, vv;
  r.load(i, rv);
  v.load(i, vv);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx<double> w = vv.c[a][c];
      rv.c[a][c].re -= ar * w.re - ai * w.im;
      rv.c[a][c].im -= ar * w.im + ai * w.re;
    }
  s.store(i, rv);
}

// x += alpha p + omega s,  r = s - omega t;  partial sums (rhat, r) and |r|^2
__global__ __launch_bounds__(kBlock) void k_bs_update(int Vh, SpinorF64 x, SpinorF64 p, SpinorF64 s, SpinorF64 t,
                                                      SpinorF64 r, SpinorF64 rhat, const BSScalars* sc, Reduce red,
                                                      int nb) {
  if (bs_halted(sc)) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  if (i < Vh) {
    const double ar = sc->alpha[0], ai = sc->alpha[1], wr = sc->omega[0], wi = sc->omega[1];
    Spinor<double> xv, pv, sv, tv, rh;
    x.load(i, xv);
    p.load(i, pv);
    s.load(i, sv);
    t.load(i, tv);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cplx<double> pp = pv.c[a][c], ss = sv.c[a][c], tt = tv.c[a][c];
        xv.c[a][c].re += ar * pp.re - ai * pp.im + wr * ss.re - wi * ss.im;
        xv.c[a][c].im += ar * pp.im + ai * pp.re + wr * ss.im + wi * ss.re;
        sv.c[a][c].re = ss.re - (wr * tt.re - wi * tt.im);   // r = s - omega t
        sv.c[a][c].im = ss.im - (wr * tt.im + wi * tt.re);
      }
    x.store(i, xv);
    r.store(i, sv);
    rhat.load(i, rh);
    cdot_acc(rh, sv, d0, d1);
    d2 = norm2(sv);
  }
  block_partial<kBlock>(d0, red.partials, blockIdx.x);
  block_partial<kBlock>(d1, red.partials + nb, blockIdx.x);
  block_partial<kBlock>(d2, red.partials + 2 * nb, blockIdx.x);
}

// rho' = (rhat, r), |r|^2, beta = (rho' / rho)(alpha / omega), convergence test
__global__ __launch_bounds__(256) void k_bs_fin_rho(BSScalars* sc, const double* partials, int nb) {
  if (bs_halted(sc)) return;
  const double a = sum_partials<256>(partials, nb);
  const double b = sum_partials<256>(partials + nb, nb);
  const double rr = sum_partials<256>(partials + 2 * nb, nb);
  if (threadIdx.x != 0) return;
  sc->iter += 1;
  sc->rr = rr;
  if (!(rr < INFINITY)) {
    sc->done = 2;
    return;
  }
  if (rr <= sc->stop_rr) {
    sc->done = 1;
    return;
  }
  const double den_rho = sc->rho[0] * sc->rho[0] + sc->rho[1] * sc->rho[1];
  const double den_om = sc->omega[0] * sc->omega[0] + sc->omega[1] * sc->omega[1];
  if (!(den_rho > 0.0) || !(den_om > 0.0) || (a == 0.0 && b == 0.0)) {
    sc->done = 2;
    return;
  }
  // q1 = rho' / rho, q2 = alpha / omega, beta = q1 q2
  const double q1r = (a * sc->rho[0] + b * sc->rho[1]) / den_rho;
  const double q1i = (b * sc->rho[0] - a * sc->rho[1]) / den_rho;
  const double q2r = (sc->alpha[0] * sc->omega[0] + sc->alpha[1] * sc->omega[1]) / den_om;
  const double q2i = (sc->alpha[1] * sc->omega[0] - sc->alpha[0] * sc->omega[1]) / den_om;
  sc->beta[0] = q1r * q2r - q1i * q2i;
  sc->beta[1] = q1r * q2i + q1i * q2r;
  sc->rho[0] = a;
  sc->rho[1] = b;
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kBlock) void k_bs_p(int Vh, SpinorF64 p, SpinorF64 r, SpinorF64 v,
                                                 const BSScalars* sc) {
  if (bs_halted(sc)) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const double br = sc->beta[0], bi = sc->beta[1], wr = sc->omega[0], wi = sc->omega[1];
  Spinor<double> pv, rv, vv;
  p.load(i, pv);
  r.load(i, rv);
  v.load(i, vv);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double qr = pv.c[a][c].re - (wr * vv.c[a][c].re - wi * vv.c[a][c].im);
      const double qi = pv.c[a][c].im - (wr * vv.c[a][c].im + wi * vv.c[a][c].re);
      pv.c[a][c].re = rv.c[a][c].re + br * qr - bi * qi;
      pv.c[a][c].im = rv.c[a][c].im + br * qi + bi * qr;
    }
  p.store(i, pv);
}

// start of a pass: rho = |r_0|^2 (rhat = r_0), stop threshold
__global__ void k_bs_init(BSScalars* sc, const double* rr0, double stop_rr) {
  if (threadIdx.x != 0) return;
  sc->rho[0] = *rr0;
  sc->rho[1] = 0.0;
  sc->alpha[0] = sc->alpha[1] = sc->omega[0] = sc->omega[1] = sc->beta[0] = sc->beta[1] = 0.0;
  sc->rr = *rr0;
  sc->stop_rr = stop_rr;
  sc->done = (*rr0 <= stop_rr) ? 1 : 0;
  sc->iter = 0;
}

template <int DAG, class Lnk>
static void enqueue_bs(whmc_ctx* c, const Lnk& L, SpinorF64 x, SpinorF64 r, SpinorF64 rhat, SpinorF64 p,
                       SpinorF64 v, SpinorF64 s, SpinorF64 t, SpinorF64 te, double k2, BSScalars* sc, int n) {
  const int ns = c->site_blocks(), nv = c->num_blocks();
  const dim3 gs(ns), gv(nv), blk(kBlock);
  const Reduce red = c->red;
  for (int it = 0; it < n; ++it) {
    TraceRange tr("whmc bicgstab iteration");
    hipLaunchKernelGGL((k_bs_hop<DAG, Lnk>), gs, blk, c->stencil_lds, c->stream, c->g, L, p, te, sc);
    hipLaunchKernelGGL((k_bs_mv<DAG, 0, Lnk>), gs, blk, c->stencil_lds, c->stream, c->g, L, te, p, v, rhat, k2, sc,
                       red, ns);
    hipLaunchKernelGGL(k_bs_fin<0>, dim3(1), dim3(256), 0, c->stream, sc, red.partials, ns);
    hipLaunchKernelGGL(k_bs_s, gv, blk, 0, c->stream, c->Vh, r, v, s, sc);
    hipLaunchKernelGGL((k_bs_hop<DAG, Lnk>), gs, blk, c->stencil_lds, c->stream, c->g, L, s, te, sc);
    hipLaunchKernelGGL((k_bs_mv<DAG, 1, Lnk>), gs, blk, c->stencil_lds, c->stream, c->g, L, te, s, t, s, k2, sc,
                       red, ns);
    hipLaunchKernelGGL(k_bs_fin<1>, dim3(1), dim3(256), 0, c->stream, sc, red.partials, ns);
    hipLaunchKernelGGL(k_bs_update, gv, blk, 0, c->stream, c->Vh, x, p, s, t, r, rhat, sc, red, nv);
    hipLaunchKernelGGL(k_bs_fin_rho, dim3(1), dim3(256), 0, c->stream, sc, red.partials, nv);
    hipLaunchKernelGGL(k_bs_p, gv, blk, 0, c->stream, c->Vh, p, r, v, sc);
  }
}

template <class Lnk>
static whmc_status bicgstab_f64(whmc_ctx* c, double* x, const double* b, double kappa, int dagger,
                                const whmc_cg_params* prm, whmc_cg_stats* st, Lnk L) {
  const auto t0 = std::chrono::steady_clock::now();
  const int Vh = c->Vh;
  const size_t hb = (size_t)Vh * 192;
  void *r, *rhat, *p, *v, *s, *t, *te;
  WHMC_TRY(workspace(c, "bs_r", hb, &r));
  WHMC_TRY(workspace(c, "bs_rhat", hb, &rhat));
  WHMC_TRY(workspace(c, "bs_p", hb, &p));
  WHMC_TRY(workspace(c, "bs_v", hb, &v));
  WHMC_TRY(workspace(c, "bs_s", hb, &s));
  WHMC_TRY(workspace(c, "bs_t", hb, &t));
  WHMC_TRY(workspace(c, "bs_te", hb, &te));
  auto S = [&](void* q) { return SpinorF64{(double2*)q, Vh}; };
  BSScalars* sc = reinterpret_cast<BSScalars*>(c->scal);
  const BSScalars* hs = reinterpret_cast<const BSScalars*>(c->scal_host);
  WHMC_TRY(norm2_f64(c, b, 1, c->red.result + 3));
  double bb;
  WHMC_TRY(read_scalar(c, c->red.result + 3, &bb));
  WHMC_CHECK(std::isfinite(bb), WHMC_ENONFINITE, "whmc_bicgstab_solve: the right-hand side is not finite");
  WHMC_TRY(zero_bytes(c, x, hb));
  st->iters = 0;
  st->reliable_updates = 0;
  st->converged = 0;
  st->true_residual = 0.0;
  if (bb == 0.0) {
    st->converged = 1;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return WHMC_OK;
  }
  const int check = prm->check_every > 0 ? prm->check_every : 8;
  const double k2 = kappa * kappa;
  int total = 0;
  for (int pass = 0; pass < 4; ++pass) {
    // r = b - A x (x = 0 on the first pass); rhat = p = r
    if (pass == 0) {
      WHMC_TRY(copy_f64(c, (double*)r, b, 1));
    } else {
      WHMC_TRY(apply_Moo_f64(c, (double*)r, x, kappa, dagger, (double*)te));
      WHMC_TRY(axpby_f64(c, (double*)r, 1.0, b, -1.0, 1));
    }
    WHMC_TRY(copy_f64(c, (double*)rhat, (double*)r, 1));
    WHMC_TRY(copy_f64(c, (double*)p, (double*)r, 1));
    WHMC_TRY(norm2_f64(c, (double*)r, 1, c->red.result + 4));
    hipLaunchKernelGGL(k_bs_init, dim3(1), dim3(64), 0, c->stream, sc, c->red.result + 4,
                       prm->tol * prm->tol * bb);
    WHMC_HIP(hipGetLastError());
    int pass_iters = 0;
    while (true) {
      const int n = std::min(check, prm->maxiter - total - pass_iters);
      if (n <= 0) break;
      if (dagger)
        enqueue_bs<1>(c, L, S(x), S(r), S(rhat), S(p), S(v), S(s), S(t), S(te), k2, sc, n);
      else
        enqueue_bs<0>(c, L, S(x), S(r), S(rhat), S(p), S(v), S(s), S(t), S(te), k2, sc, n);
      WHMC_HIP(hipGetLastError());
      WHMC_HIP(hipMemcpyAsync(c->scal_host, c->scal, sizeof(BSScalars), hipMemcpyDeviceToHost, c->stream));
      WHMC_HIP(hipStreamSynchronize(c->stream));
      pass_iters = hs->iter;
      if (hs->done) break;
    }
    total += pass_iters;
    // true residual |b - A x| / |b|
    WHMC_TRY(apply_Moo_f64(c, (double*)r, x, kappa, dagger, (double*)te));
    WHMC_TRY(axpby_f64(c, (double*)r, 1.0, b, -1.0, 1));
    double rr;
    WHMC_TRY(norm2_f64(c, (double*)r, 1, c->red.result + 2));
    WHMC_TRY(read_scalar(c, c->red.result + 2, &rr));
    st->true_residual = std::sqrt(rr / bb);
    WHMC_CHECK(std::isfinite(st->true_residual), WHMC_ENONFINITE, "whmc_bicgstab_solve: the residual is not finite");
    if (st->true_residual <= prm->tol) {
      st->converged = 1;
      break;
    }
    if (total >= prm->maxiter) break;
  }
  st->iters = total;
  st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return WHMC_OK;
}

}  // namespace whmc

using namespace whmc;

extern "C" whmc_status whmc_bicgstab_solve(whmc_ctx* c, double* x, const double* b, double kappa, int dagger,
                                           const whmc_cg_params* params, whmc_cg_stats* stats) {
  WHMC_CHECK(c && x && b && params, WHMC_EARG, "whmc_bicgstab_solve: null argument");
  WHMC_CHECK(x != b, WHMC_EARG, "whmc_bicgstab_solve: x and b must differ");
  WHMC_CHECK(params->tol > 0 && params->maxiter > 0, WHMC_EARG, "whmc_bicgstab_solve: tol and maxiter must be positive");
  WHMC_CHECK(params->prec == WHMC_F64, WHMC_EUNSUP, "whmc_bicgstab_solve: FP64 only");
  WHMC_CHECK(params->links == WHMC_L18 || params->links == WHMC_L12, WHMC_EARG, "whmc_bicgstab_solve: bad links");
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded (call whmc_load_gauge first)");
  WHMC_TRY(ensure_links(c, WHMC_F64, params->links));
  whmc_cg_stats local{};
  whmc_cg_stats* st = stats ? stats : &local;
  const int Vh = c->Vh;
  const bool nt = c->stream_links(WHMC_F64, params->links);
  whmc_status rc;
  if (params->links == WHMC_L18)
    rc = nt ? bicgstab_f64(c, x, b, kappa, dagger ? 1 : 0, params, st, LinkF64_18T<true>{c->U18, Vh})
            : bicgstab_f64(c, x, b, kappa, dagger ? 1 : 0, params, st, LinkF64_18T<false>{c->U18, Vh});
  else
    rc = nt ? bicgstab_f64(c, x, b, kappa, dagger ? 1 : 0, params, st, LinkF64_12T<true>{c->U12, Vh})
            : bicgstab_f64(c, x, b, kappa, dagger ? 1 : 0, params, st, LinkF64_12T<false>{c->U12, Vh});
  if (rc != WHMC_OK) return rc;
  if (!st->converged) {
    set_error("whmc_bicgstab_solve: not converged");
    return WHMC_ENOCONV;
  }
  return WHMC_OK;
}
