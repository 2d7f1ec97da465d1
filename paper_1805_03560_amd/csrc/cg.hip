// Conjugate gradient on A = M_oo^dag M_oo (Sec. 1 names CG for the pseudo-fermion systems; Sec.
// 2.2 the even/odd matrix), FP64 and mixed precision.
//
// One iteration is five stencil / vector kernels, plus two single-block kernels that finish the
// two reductions (see block_partial); the scalars (alpha, beta, |r|^2) never leave the device:
//   1  t = H_eo p
//   2  u = p - kappa^2 H_oe t,                (p, A p) = |u|^2      -> alpha = |r|^2 / |u|^2
//   3  v = (H^dag)_eo u
//   4  A p = u - kappa^2 (H^dag)_oe v;  r -= alpha A p;  x += alpha p;  |r|^2 -> beta, stop tests
//   5  p = r + beta p
// Every kernel first reads the solve's `done` / `pause` flags and returns if set, so the host can
// enqueue several iterations between convergence checks without overshooting.
//
// Mixed precision (reliable updates, Clark et al., arXiv:0911.3191, after Sleijpen & van der
// Vorst): the five kernels run on FP32 or FP16 (per-site scaled) spinors with 12-real links of
// the same precision, x and r in FP32; dot products accumulate in FP64.  When the iterated |r|
// falls below delta times its maximum since the last update (or below the target) kernel 4
// raises `pause`; the host then adds x into the FP64 solution, recomputes r = b - A x with the
// FP64 operator, restores p's orthogonality to r and resumes.
#include <chrono>
#include <cmath>
#include <type_traits>

#include "internal.h"
#include "stencil.h"

namespace whmc {

WHMC_DEV bool halted(const CGScalars* sc) { return sc->done | sc->pause; }

template <class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_cg1(Geom g, Lnk L, S p, S t, const CGScalars* sc) {
  if (halted(sc)) return;
  using R = typename S::Real;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  Spinor<R> acc;
  hop_site<0>(g, 0, i, L, p, acc);
  t.store(i, acc);
}

template <class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_cg2(Geom g, Lnk L, S t, S p, S u, double k2, CGScalars* sc, Reduce red) {
  if (halted(sc)) return;
  using R = typename S::Real;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double nrm = 0.0;
  if (i < g.Vh) {
    Spinor<R> acc, pv;
    hop_site<0>(g, 1, i, L, t, acc);
    p.load(i, pv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.c[s][c] = pv.c[s][c] - R(k2) * acc.c[s][c];
    u.store(i, acc);
    nrm = norm2(acc);
  }
  block_partial<kBlock>(nrm, red.partials, blockIdx.x);
}

// pass 2 of kernel 2: (p, A p) -> alpha
__global__ __launch_bounds__(256) void k_cg2_fin(CGScalars* sc, const double* partials, int nb) {
  if (halted(sc)) return;
  const double pAp = sum_partials<256>(partials, nb);
  if (threadIdx.x != 0) return;
  sc->pAp = pAp;
  if (pAp > 0.0 && pAp < INFINITY) {
    sc->alpha = sc->rr / pAp;
  } else {
    sc->alpha = 0.0;
    sc->done = 1;   // breakdown: p = 0 or non-finite
  }
}

template <class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_cg3(Geom g, Lnk L, S u, S v, const CGScalars* sc) {
  if (halted(sc)) return;
  using R = typename S::Real;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  Spinor<R> acc;
  hop_site<1>(g, 0, i, L, u, acc);
  v.store(i, acc);
}

template <class Lnk, class S, class SR, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_cg4(Geom g, Lnk L, S v, S u, S p, SR r, SR x, double k2, CGScalars* sc,
                                                Reduce red) {
  if (halted(sc)) return;
  using R = typename S::Real;
  using RR = typename SR::Real;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const double alpha = sc->alpha;
  double nrm = 0.0;
  if (i < g.Vh) {
    Spinor<R> acc, uv, pv;
    Spinor<RR> rv, xv;
    hop_site<1>(g, 1, i, L, v, acc);
    u.load(i, uv);
    p.load(i, pv);
    r.load(i, rv);
    x.load(i, xv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cplx<R> ap = uv.c[s][c] - R(k2) * acc.c[s][c];
        rv.c[s][c].re -= RR(alpha) * RR(ap.re);
        rv.c[s][c].im -= RR(alpha) * RR(ap.im);
        xv.c[s][c].re += RR(alpha) * RR(pv.c[s][c].re);
        xv.c[s][c].im += RR(alpha) * RR(pv.c[s][c].im);
      }
    r.store(i, rv);
    x.store(i, xv);
    nrm = norm2(rv);
  }
  block_partial<kBlock>(nrm, red.partials, blockIdx.x);
}

// pass 2 of kernel 4: new |r|^2 -> beta, stop / reliable-update tests
template <bool MIXED>
__global__ __launch_bounds__(256) void k_cg4_fin(CGScalars* sc, const double* partials, int nb) {
  if (halted(sc)) return;
  const double rr_new = sum_partials<256>(partials, nb);
  if (threadIdx.x != 0) return;
  const double rr_old = sc->rr;
  sc->beta = rr_new / rr_old;
  sc->rr_old = rr_old;
  sc->rr = rr_new;
  sc->iter += 1;
  if (!(rr_new < INFINITY)) {
    sc->done = 1;
    return;
  }
  if (MIXED) {
    sc->rmax2 = fmax(sc->rmax2, rr_new);
    if (rr_new <= sc->stop_rr || rr_new < sc->delta2 * sc->rmax2) sc->pause = 1;
  } else {
    if (rr_new <= sc->stop_rr) sc->done = 1;
  }
}

template <class S, class SR>
__global__ __launch_bounds__(kBlock) void k_cg5(int Vh, S p, SR r, const CGScalars* sc) {
  if (halted(sc)) return;
  using R = typename S::Real;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const R beta = R(sc->beta);
  Spinor<R> pv;
  Spinor<typename SR::Real> rv;
  p.load(i, pv);
  r.load(i, rv);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv.c[s][c].re = R(rv.c[s][c].re) + beta * pv.c[s][c].re;
      pv.c[s][c].im = R(rv.c[s][c].im) + beta * pv.c[s][c].im;
    }
  p.store(i, pv);
}

// scalar setup from the device-side |r|^2 (red.result[slot])
__global__ void k_cg_init(CGScalars* sc, const double* rr, double tol2, double delta2) {
  if (threadIdx.x != 0) return;
  sc->rr = *rr;
  sc->stop_rr = tol2 * (*rr);
  sc->rmax2 = *rr;
  sc->delta2 = delta2;
  sc->done = (*rr == 0.0);
  sc->pause = 0;
  sc->iter = 0;
  sc->alpha = sc->beta = sc->pAp = 0.0;
}

// after a reliable update: new |r|^2, resume
__global__ void k_cg_resume(CGScalars* sc, const double* rr) {
  if (threadIdx.x != 0) return;
  sc->rr = *rr;
  sc->rmax2 = *rr;
  sc->pause = 0;
}

// reliable update of the search direction (mixed): with r the fresh residual,
//   p <- r + beta (p - gamma r),  gamma = (r, p) / |r|^2,  beta = |r|^2 / |r_old|^2
template <class S, class SR>
__global__ __launch_bounds__(kBlock) void k_rel_p(int Vh, S p, SR r, const double* rp_rr, const CGScalars* sc) {
  using R = typename S::Real;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const double rr = sc->rr;
  const R gamma = R(rp_rr[0] / rr);
  const R beta = R(rr / sc->rr_old);
  Spinor<R> pv;
  Spinor<typename SR::Real> rv;
  p.load(i, pv);
  r.load(i, rv);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv.c[s][c].re = R(rv.c[s][c].re) + beta * (pv.c[s][c].re - gamma * R(rv.c[s][c].re));
      pv.c[s][c].im = R(rv.c[s][c].im) + beta * (pv.c[s][c].im - gamma * R(rv.c[s][c].im));
    }
  p.store(i, pv);
}

// FP64 x += low-precision x_s, then x_s = 0
template <class SR>
__global__ void k_accum_x(int Vh, double2* x, SR xs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  Spinor<typename SR::Real> v;
  xs.load(i, v);
  SpinorF64 X{x, Vh};
  Spinor<double> a;
  X.load(i, a);
  for (int s = 0; s < 4; ++s)
    for (int c = 0; c < 3; ++c) {
      a.c[s][c].re += (double)v.c[s][c].re;
      a.c[s][c].im += (double)v.c[s][c].im;
      v.c[s][c] = {0, 0};
    }
  X.store(i, a);
  xs.store(i, v);
}

// (r, p) real part with mixed storage, FP64 accumulation
template <class S, class SR>
__global__ __launch_bounds__(kBlock) void k_dot_rp(int Vh, S p, SR r, Reduce red, double* out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double s = 0.0;
  if (i < Vh) {
    Spinor<typename S::Real> pv;
    Spinor<typename SR::Real> rv;
    p.load(i, pv);
    r.load(i, rv);
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c)
        s += (double)pv.c[a][c].re * (double)rv.c[a][c].re + (double)pv.c[a][c].im * (double)rv.c[a][c].im;
  }
  block_partial<kBlock>(s, red.partials, blockIdx.x);
}

// ------------------------------------------------------------------ host drivers
struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double s() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

static whmc_status read_scalars(whmc_ctx* c, CGScalars* host, int n = 1) {
  WHMC_HIP(hipMemcpyAsync(c->scal_host, c->scal, n * sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) host[k] = c->scal_host[k];
  return WHMC_OK;
}

// true relative residual |b - A x| / |b| in FP64; r_out receives b - A x
static whmc_status true_residual(whmc_ctx* c, double* r_out, const double* x, const double* b, double kappa,
                                 double* te, double* to, double bb, double* rel) {
  WHMC_TRY(apply_MdagM_f64(c, r_out, x, kappa, te, to));
  WHMC_TRY(axpby_f64(c, r_out, 1.0, b, -1.0, 1));   // r = b - A x
  double rr;
  WHMC_TRY(norm2_f64(c, r_out, 1, c->red.result + 2));
  WHMC_TRY(read_scalar(c, c->red.result + 2, &rr));
  *rel = std::sqrt(rr / bb);
  return WHMC_OK;
}

static SpinorF64 s64(void* p, int Vh) { return SpinorF64{(double2*)p, Vh}; }
static SpinorF32 s32(void* p, int Vh) { return SpinorF32{(float4*)p, Vh}; }
static SpinorF16 s16(void* p, int Vh) { return SpinorF16{(uint4*)p, (float*)((uint4*)p + (size_t)3 * Vh), Vh}; }

template <class Lnk, class S, class SR, bool MIXED>
static whmc_status enqueue_iters(whmc_ctx* c, const Lnk& L, S p, S t, S u, S v, SR r, SR x, double kappa, int n) {
  const dim3 grid(c->site_blocks()), block(kBlock);
  // occupancy cap of the FP64 stencil kernels with 18- or 12-real links (the low-precision and 8-real
  // ones need every wave)
  const unsigned lds = std::is_same<S, SpinorF64>::value && !is_8real<Lnk>::value ? c->stencil_lds : 0u;
  const double k2 = kappa * kappa;
  for (int it = 0; it < n; ++it) {
    TraceRange tr(MIXED ? "whmc cg iteration (mixed)" : "whmc cg iteration");
    hipLaunchKernelGGL((k_cg1<Lnk, S>), grid, block, lds, c->stream, c->g, L, p, t, c->scal);
    hipLaunchKernelGGL((k_cg2<Lnk, S>), grid, block, lds, c->stream, c->g, L, t, p, u, k2, c->scal, c->red);
    hipLaunchKernelGGL(k_cg2_fin, dim3(1), dim3(256), 0, c->stream, c->scal, c->red.partials, (int)grid.x);
    hipLaunchKernelGGL((k_cg3<Lnk, S>), grid, block, lds, c->stream, c->g, L, u, v, c->scal);
    hipLaunchKernelGGL((k_cg4<Lnk, S, SR, MIXED>), grid, block, lds, c->stream, c->g, L, v, u, p, r, x, k2, c->scal,
                       c->red);
    hipLaunchKernelGGL(k_cg4_fin<MIXED>, dim3(1), dim3(256), 0, c->stream, c->scal, c->red.partials, (int)grid.x);
    hipLaunchKernelGGL((k_cg5<S, SR>), grid, block, 0, c->stream, c->Vh, p, r, c->scal);
  }
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

// plain FP64 CG for one right-hand side
template <class Lnk>
static whmc_status cg_f64(whmc_ctx* c, double* x, const double* b, double kappa, const whmc_cg_params* prm,
                          whmc_cg_stats* st, Lnk L) {
  Timer tm;
  const size_t hb = (size_t)c->Vh * 192;
  void *r, *p, *t, *u, *v, *te, *to;
  WHMC_TRY(workspace(c, "cg_r", hb, &r));
  WHMC_TRY(workspace(c, "cg_p", hb, &p));
  WHMC_TRY(workspace(c, "cg_t", hb, &t));
  WHMC_TRY(workspace(c, "cg_u", hb, &u));
  WHMC_TRY(workspace(c, "cg_v", hb, &v));
  WHMC_TRY(workspace(c, "cg_te", hb, &te));
  WHMC_TRY(workspace(c, "cg_to", hb, &to));
  const int Vh = c->Vh;
  WHMC_TRY(norm2_f64(c, b, 1, c->red.result + 3));
  double bb;
  WHMC_TRY(read_scalar(c, c->red.result + 3, &bb));
  WHMC_CHECK(std::isfinite(bb), WHMC_ENONFINITE, "cg_solve: the right-hand side is not finite");
  WHMC_TRY(zero_bytes(c, x, hb));
  st->iters = 0;
  st->reliable_updates = 0;
  st->converged = 0;
  st->true_residual = 0.0;
  if (bb == 0.0) {
    st->converged = 1;
    st->seconds = tm.s();
    return WHMC_OK;
  }
  const int check = prm->check_every > 0 ? prm->check_every : 8;
  int total = 0;
  for (int restart = 0; restart < 4; ++restart) {
    // r = b - A x (x = 0 on the first pass), p = r
    if (restart == 0) {
      WHMC_TRY(copy_f64(c, (double*)r, b, 1));
    } else {
      double rel;
      WHMC_TRY(true_residual(c, (double*)r, x, b, kappa, (double*)te, (double*)to, bb, &rel));
    }
    WHMC_TRY(copy_f64(c, (double*)p, (double*)r, 1));
    WHMC_TRY(norm2_f64(c, (double*)r, 1, c->red.result + 4));
    // relative to |r| of this pass: stop when |r| <= tol |b|
    double rr0;
    WHMC_TRY(read_scalar(c, c->red.result + 4, &rr0));
    const double tol2 = prm->tol * prm->tol * bb / (rr0 > 0 ? rr0 : 1.0);
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, c->stream, c->scal, c->red.result + 4, tol2, 0.0);
    WHMC_HIP(hipGetLastError());
    CGScalars hs{};
    int pass_iters = 0;
    while (true) {
      const int n = std::min(check, prm->maxiter - total - pass_iters);
      if (n <= 0) break;
      WHMC_TRY((enqueue_iters<Lnk, SpinorF64, SpinorF64, false>(c, L, s64(p, Vh), s64(t, Vh), s64(u, Vh),
                                                                        s64(v, Vh), s64(r, Vh), s64(x, Vh), kappa, n)));
      WHMC_TRY(read_scalars(c, &hs));
      pass_iters = hs.iter;
      if (hs.done) break;
    }
    total += pass_iters;
    double rel;
    WHMC_TRY(true_residual(c, (double*)r, x, b, kappa, (double*)te, (double*)to, bb, &rel));
    st->true_residual = rel;
    WHMC_CHECK(std::isfinite(rel), WHMC_ENONFINITE, "cg_solve: the residual is not finite");
    if (rel <= prm->tol) {
      st->converged = 1;
      break;
    }
    if (total >= prm->maxiter) break;
  }
  st->iters = total;
  st->seconds = tm.s();
  return WHMC_OK;
}

// mixed-precision CG with reliable updates, one right-hand side
template <class Lnk, class S, class SR>
static whmc_status cg_mixed(whmc_ctx* c, double* x, const double* b, double kappa, const whmc_cg_params* prm,
                            whmc_cg_stats* st, Lnk L, int sprec, S (*mk)(void*, int), SR (*mkr)(void*, int),
                            int rprec) {
  Timer tm;
  const int Vh = c->Vh;
  const size_t hb = (size_t)Vh * 192;
  const size_t sb = sprec == WHMC_F32 ? (size_t)Vh * 96 : (size_t)Vh * 52;
  const size_t rb = rprec == WHMC_F32 ? (size_t)Vh * 96 : hb;
  void *r64, *te, *to, *p, *t, *u, *v, *rs, *xs;
  WHMC_TRY(workspace(c, "cg_r", hb, &r64));
  WHMC_TRY(workspace(c, "cg_te", hb, &te));
  WHMC_TRY(workspace(c, "cg_to", hb, &to));
  WHMC_TRY(workspace(c, "mx_p", sb, &p));
  WHMC_TRY(workspace(c, "mx_t", sb, &t));
  WHMC_TRY(workspace(c, "mx_u", sb, &u));
  WHMC_TRY(workspace(c, "mx_v", sb, &v));
  WHMC_TRY(workspace(c, "mx_r", rb, &rs));
  WHMC_TRY(workspace(c, "mx_x", rb, &xs));
  WHMC_TRY(norm2_f64(c, b, 1, c->red.result + 3));
  double bb;
  WHMC_TRY(read_scalar(c, c->red.result + 3, &bb));
  WHMC_CHECK(std::isfinite(bb), WHMC_ENONFINITE, "cg_solve: the right-hand side is not finite");
  WHMC_TRY(zero_bytes(c, x, hb));
  st->iters = 0;
  st->reliable_updates = 0;
  st->converged = 0;
  st->true_residual = 0.0;
  if (bb == 0.0) {
    st->converged = 1;
    st->seconds = tm.s();
    return WHMC_OK;
  }
  WHMC_TRY(zero_bytes(c, xs, rb));
  WHMC_TRY(convert_spinor(c, rs, rprec, b, WHMC_F64, 1));
  WHMC_TRY(convert_spinor(c, p, sprec, b, WHMC_F64, 1));
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, c->stream, c->scal, c->red.result + 3,
                     prm->tol * prm->tol, prm->delta * prm->delta);
  WHMC_HIP(hipGetLastError());
  const int check = prm->check_every > 0 ? prm->check_every : 8;
  const dim3 grid(c->site_blocks()), block(kBlock);
  CGScalars hs{};
  int iters = 0;
  double rel = 1.0;
  while (iters < prm->maxiter) {
    const int n = std::min(check, prm->maxiter - iters);
    WHMC_TRY((enqueue_iters<Lnk, S, SR, true>(c, L, mk(p, Vh), mk(t, Vh), mk(u, Vh), mk(v, Vh), mkr(rs, Vh),
                                              mkr(xs, Vh), kappa, n)));
    WHMC_TRY(read_scalars(c, &hs));
    iters = hs.iter;
    if (hs.done && !hs.pause) break;   // breakdown
    if (!hs.pause) continue;
    // reliable update: x += x_s (x_s = 0), r = b - A x in FP64
    hipLaunchKernelGGL((k_accum_x<SR>), dim3((Vh + 255) / 256), dim3(256), 0, c->stream, Vh, (double2*)x, mkr(xs, Vh));
    WHMC_HIP(hipGetLastError());
    WHMC_TRY(true_residual(c, (double*)r64, x, b, kappa, (double*)te, (double*)to, bb, &rel));
    st->reliable_updates += 1;
    WHMC_CHECK(std::isfinite(rel), WHMC_ENONFINITE, "cg_solve: the residual is not finite");
    if (rel <= prm->tol) {
      st->converged = 1;
      break;
    }
    WHMC_TRY(convert_spinor(c, rs, rprec, r64, WHMC_F64, 1));
    WHMC_TRY(norm2_f64(c, (double*)r64, 1, c->red.result + 5));
    hipLaunchKernelGGL(k_cg_resume, dim3(1), dim3(64), 0, c->stream, c->scal, c->red.result + 5);
    hipLaunchKernelGGL((k_dot_rp<S, SR>), grid, block, 0, c->stream, Vh, mk(p, Vh), mkr(rs, Vh), c->red,
                       c->red.result + 6);
    WHMC_TRY(finish_sum(c, (int)grid.x, c->red.result + 6));
    hipLaunchKernelGGL((k_rel_p<S, SR>), grid, block, 0, c->stream, Vh, mk(p, Vh), mkr(rs, Vh), c->red.result + 6,
                       c->scal);
    WHMC_HIP(hipGetLastError());
  }
  if (!st->converged) {
    hipLaunchKernelGGL((k_accum_x<SR>), dim3((Vh + 255) / 256), dim3(256), 0, c->stream, Vh, (double2*)x, mkr(xs, Vh));
    WHMC_HIP(hipGetLastError());
    WHMC_TRY(true_residual(c, (double*)r64, x, b, kappa, (double*)te, (double*)to, bb, &rel));
    st->converged = rel <= prm->tol;
    st->true_residual = rel;
    WHMC_CHECK(std::isfinite(rel), WHMC_ENONFINITE, "cg_solve: the residual is not finite");
  }
  st->true_residual = rel;
  st->iters = iters;
  st->seconds = tm.s();
  return WHMC_OK;
}

whmc_status cg_solve_multi(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                           const whmc_cg_params* p, whmc_cg_stats* st);

whmc_status cg_solve(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                     const whmc_cg_params* p, whmc_cg_stats* st) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  TraceRange tr(nrhs > 1 ? "whmc cg solve (multi-rhs)" : "whmc cg solve");
  if (nrhs > 1) return cg_solve_multi(c, x, b, kappas, nrhs, p, st);
  whmc_cg_stats local{};
  whmc_cg_stats* s = st ? st : &local;
  whmc_status rc;
  const int Vh = c->Vh;
  if (p->prec == WHMC_F64 && p->links == WHMC_L12) {
    // FP64 arithmetic with 12-real links: the third row is rebuilt in FP64, exact to rounding
    WHMC_TRY(ensure_links(c, WHMC_F64, WHMC_L12));
    if (c->stream_links(WHMC_F64, WHMC_L12)) rc = cg_f64(c, x, b, kappas[0], p, s, LinkF64_12T<true>{c->U12, Vh});
    else rc = cg_f64(c, x, b, kappas[0], p, s, LinkF64_12T<false>{c->U12, Vh});
  } else if (p->prec == WHMC_F64 && p->links == WHMC_L8) {
    WHMC_TRY(ensure_links(c, WHMC_F64, WHMC_L8));
    if (c->stream_links(WHMC_F64, WHMC_L8)) rc = cg_f64(c, x, b, kappas[0], p, s, LinkF64_8T<true>{c->U8, Vh});
    else rc = cg_f64(c, x, b, kappas[0], p, s, LinkF64_8T<false>{c->U8, Vh});
  } else if (p->prec == WHMC_F64) {
    if (c->stream_links(WHMC_F64, WHMC_L18)) rc = cg_f64(c, x, b, kappas[0], p, s, LinkF64_18T<true>{c->U18, Vh});
    else rc = cg_f64(c, x, b, kappas[0], p, s, LinkF64_18T<false>{c->U18, Vh});
  } else if (p->prec == WHMC_F32) {
    WHMC_TRY(ensure_links(c, WHMC_F32, p->links));
    const bool nt = c->stream_links(WHMC_F32, p->links);
    if (p->links == WHMC_L18) {
      if (nt) rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF32_18T<true>{c->U32_18, Vh}, WHMC_F32, s32, s32, WHMC_F32);
      else rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF32_18T<false>{c->U32_18, Vh}, WHMC_F32, s32, s32, WHMC_F32);
    } else if (p->links == WHMC_L8) {
      if (nt) rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF32_8T<true>{c->U32_8, Vh}, WHMC_F32, s32, s32, WHMC_F32);
      else rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF32_8T<false>{c->U32_8, Vh}, WHMC_F32, s32, s32, WHMC_F32);
    } else {
      if (nt) rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF32_12T<true>{c->U32_12, Vh}, WHMC_F32, s32, s32, WHMC_F32);
      else rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF32_12T<false>{c->U32_12, Vh}, WHMC_F32, s32, s32, WHMC_F32);
    }
  } else {
    WHMC_CHECK(p->links == WHMC_L12 || p->links == WHMC_L8, WHMC_EUNSUP, "FP16 bulk requires 12- or 8-real links");
    WHMC_TRY(ensure_links(c, WHMC_F16, p->links));
    const bool nt = c->stream_links(WHMC_F16, p->links);
    if (p->links == WHMC_L8) {
      if (nt) rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF16_8T<true>{c->U16_8, Vh}, WHMC_F16, s16, s32, WHMC_F32);
      else rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF16_8T<false>{c->U16_8, Vh}, WHMC_F16, s16, s32, WHMC_F32);
    } else if (nt) {
      rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF16_12T<true>{c->U16_12, Vh}, WHMC_F16, s16, s32, WHMC_F32);
    } else {
      rc = cg_mixed(c, x, b, kappas[0], p, s, LinkF16_12T<false>{c->U16_12, Vh}, WHMC_F16, s16, s32, WHMC_F32);
    }
  }
  if (rc != WHMC_OK) return rc;
  if (!s->converged) {
    set_error("cg_solve: no convergence: true residual " + std::to_string(s->true_residual) + " after " +
              std::to_string(s->iters) + " iterations");
    return WHMC_ENOCONV;
  }
  return WHMC_OK;
}

}  // namespace whmc

extern "C" whmc_status whmc_cg_solve(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                                     const whmc_cg_params* params, whmc_cg_stats* stats) {
  WHMC_CHECK(c && x && b && kappas && params, WHMC_EARG, "whmc_cg_solve: null argument");
  WHMC_CHECK(nrhs >= 1 && nrhs <= whmc::kMaxRhs, WHMC_EARG, "whmc_cg_solve: nrhs must be in [1, 16]");
  WHMC_CHECK(x != b, WHMC_EARG, "whmc_cg_solve: x and b must differ");
  WHMC_CHECK(params->tol > 0 && params->maxiter > 0, WHMC_EARG, "whmc_cg_solve: tol and maxiter must be positive");
  WHMC_CHECK(params->prec >= 0 && params->prec <= 2, WHMC_EARG, "whmc_cg_solve: bad precision");
  WHMC_CHECK(params->prec == WHMC_F64 || (params->delta > 0 && params->delta < 1), WHMC_EARG,
             "whmc_cg_solve: mixed precision needs 0 < delta < 1");
  return whmc::cg_solve(c, x, b, kappas, nrhs, params, stats);
}
