// Multi right-hand-side hopping matrix and masked CG.
//
// One launch applies H to N_rhs spinor fields: each thread owns one site and a register block of
// NB right-hand sides, loads every link once and applies it to all NB projected neighbours, so the
// link bytes (the bulk of the stencil's traffic) are amortised over NB fields; grid.y runs over
// the blocks of right-hand sides.  Algorithmic bytes per site and rhs:
// (8 link loads + NB (in + out) spinors) / NB.
//
// The CG runs every rhs with its own kappa (mass-preconditioning shifts) and its own device-side
// scalars.  A converged (or paused, in mixed precision) rhs is masked: the kernels skip its loads,
// arithmetic and stores while the others keep iterating, and a block whose rhs are all masked
// exits at once.  The register block NB is chosen by the autotuner (timed on first use per
// precision, link format and N_rhs) unless the caller fixes it.
#include <chrono>
#include <cmath>
#include <string>

#include "internal.h"
#include "stencil.h"

namespace whmc {

// ------------------------------------------------------------------ field offsets
WHMC_DEV SpinorF64 field(SpinorF64 s, int r) { return SpinorF64{s.p + (size_t)r * 12 * s.stride, s.stride}; }
WHMC_DEV SpinorF32 field(SpinorF32 s, int r) { return SpinorF32{s.p + (size_t)r * 6 * s.stride, s.stride}; }
WHMC_DEV SpinorF16 field(SpinorF16 s, int r) {
  char* base = (char*)s.p + (size_t)r * 52 * s.stride;
  return SpinorF16{(uint4*)base, (float*)(base + (size_t)48 * s.stride), s.stride};
}

struct K2 {
  double v[kMaxRhs];
};

// ------------------------------------------------------------------ per-rhs partial sums
// pass 1: rhs r of this block's slice writes its block partial to partials[r * nb + block];
// pass 2 (k_m*_fin, one block per rhs) adds the nb partials of rhs r in a fixed order.
template <int BLOCK, int NB>
WHMC_DEV void block_partials_multi(const double* v, double* partials, int r0, int nrhs) {
  const int nb = gridDim.x;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    __shared__ double lds[BLOCK / 64];
    __syncthreads();
    const double s = block_sum<BLOCK>(v[k], lds);
    if (threadIdx.x == 0 && r0 + k < nrhs) partials[(size_t)(r0 + k) * nb + blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ multi-RHS stencil
template <int MU, int DAG, int NB, class Lnk, class S, typename R>
WHMC_DEV void hop_dir_multi(const Geom& g, const Coords& c, int par, int i, const Lnk& L, const S* in,
                            const bool* act, Spinor<R>* acc) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  bool wrap;
  SU3<R> U;
  {
    const int j = neighbour<MU, +1>(g, c, wrap);
    L.load(par, MU, i, U);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!act[k]) continue;
      Spinor<R> s;
      HalfSpinor<R> h, u;
      in[k].load(j, s);
      project<MU, SF>(s, h);
      if (MU == 0 && wrap) negate(h);
      mul(U, h.c[0], u.c[0]);
      mul(U, h.c[1], u.c[1]);
      accumulate<MU, SF>(acc[k], u);
    }
  }
  {
    const int j = neighbour<MU, -1>(g, c, wrap);
    L.load(1 - par, MU, j, U);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!act[k]) continue;
      Spinor<R> s;
      HalfSpinor<R> h, u;
      in[k].load(j, s);
      project<MU, SB>(s, h);
      if (MU == 0 && wrap) negate(h);
      mul_dag(U, h.c[0], u.c[0]);
      mul_dag(U, h.c[1], u.c[1]);
      accumulate<MU, SB>(acc[k], u);
    }
  }
}

template <int DAG, int NB, class Lnk, class S, typename R>
WHMC_DEV void hop_site_multi(const Geom& g, int par, int i, const Lnk& L, const S* in, const bool* act,
                             Spinor<R>* acc) {
  const Coords c = coords_of(g, i, par);
#pragma unroll
  for (int k = 0; k < NB; ++k) zero(acc[k]);
  hop_dir_multi<0, DAG, NB>(g, c, par, i, L, in, act, acc);
  hop_dir_multi<1, DAG, NB>(g, c, par, i, L, in, act, acc);
  hop_dir_multi<2, DAG, NB>(g, c, par, i, L, in, act, acc);
  hop_dir_multi<3, DAG, NB>(g, c, par, i, L, in, act, acc);
}

// plain multi-RHS hop: out_r = H_{par,1-par}^{(dag)} in_r
template <int DAG, int NB, class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_mhop(Geom g, int par, int nrhs, Lnk L, S in0, S out0) {
  using R = typename S::Real;
  const int r0 = blockIdx.y * NB;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  bool act[NB];
  S in[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    act[k] = r0 + k < nrhs;
    in[k] = field(in0, act[k] ? r0 + k : 0);
  }
  Spinor<R> acc[NB];
  hop_site_multi<DAG, NB>(g, par, i, L, in, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (act[k]) field(out0, r0 + k).store(i, acc[k]);
}

WHMC_DEV bool rhs_live(const CGScalars* sc, int r, int nrhs) { return r < nrhs && !(sc[r].done | sc[r].pause); }

template <int NB, class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_mcg1(Geom g, int nrhs, Lnk L, S p0, S t0, const CGScalars* sc) {
  using R = typename S::Real;
  const int r0 = blockIdx.y * NB;
  bool act[NB], any = false;
#pragma unroll
  for (int k = 0; k < NB; ++k) { act[k] = rhs_live(sc, r0 + k, nrhs); any |= act[k]; }
  if (!any) return;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  S in[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) in[k] = field(p0, act[k] ? r0 + k : 0);
  Spinor<R> acc[NB];
  hop_site_multi<0, NB>(g, 0, i, L, in, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (act[k]) field(t0, r0 + k).store(i, acc[k]);
}

template <int NB, class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_mcg2(Geom g, int nrhs, Lnk L, S t0, S p0, S u0, K2 k2, CGScalars* sc,
                                                 Reduce red) {
  using R = typename S::Real;
  const int r0 = blockIdx.y * NB;
  bool act[NB], any = false;
#pragma unroll
  for (int k = 0; k < NB; ++k) { act[k] = rhs_live(sc, r0 + k, nrhs); any |= act[k]; }
  if (!any) return;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double nrm[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) nrm[k] = 0.0;
  if (i < g.Vh) {
    S in[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) in[k] = field(t0, act[k] ? r0 + k : 0);
    Spinor<R> acc[NB];
    hop_site_multi<0, NB>(g, 1, i, L, in, act, acc);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!act[k]) continue;
      Spinor<R> pv;
      field(p0, r0 + k).load(i, pv);
      const R kk = R(k2.v[r0 + k]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[k].c[s][c] = pv.c[s][c] - kk * acc[k].c[s][c];
      field(u0, r0 + k).store(i, acc[k]);
      nrm[k] = norm2(acc[k]);
    }
  }
  block_partials_multi<kBlock, NB>(nrm, red.partials, r0, nrhs);
}

__global__ __launch_bounds__(256) void k_mcg2_fin(CGScalars* sc, int nrhs, const double* partials, int nb) {
  const int r = blockIdx.x;
  if (!rhs_live(sc, r, nrhs)) return;
  const double pAp = sum_partials<256>(partials + (size_t)r * nb, nb);
  if (threadIdx.x != 0) return;
  sc[r].pAp = pAp;
  if (pAp > 0.0 && pAp < INFINITY) {
    sc[r].alpha = sc[r].rr / pAp;
  } else {
    sc[r].alpha = 0.0;
    sc[r].done = 1;
  }
}

template <int NB, class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_mcg3(Geom g, int nrhs, Lnk L, S u0, S v0, const CGScalars* sc) {
  using R = typename S::Real;
  const int r0 = blockIdx.y * NB;
  bool act[NB], any = false;
#pragma unroll
  for (int k = 0; k < NB; ++k) { act[k] = rhs_live(sc, r0 + k, nrhs); any |= act[k]; }
  if (!any) return;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  S in[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) in[k] = field(u0, act[k] ? r0 + k : 0);
  Spinor<R> acc[NB];
  hop_site_multi<1, NB>(g, 0, i, L, in, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (act[k]) field(v0, r0 + k).store(i, acc[k]);
}

template <int NB, class Lnk, class S, class SR, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_mcg4(Geom g, int nrhs, Lnk L, S v0, S u0, S p0, SR rr0, SR x0, K2 k2,
                                                 CGScalars* sc, Reduce red) {
  using R = typename S::Real;
  using RR = typename SR::Real;
  const int r0 = blockIdx.y * NB;
  bool act[NB], any = false;
#pragma unroll
  for (int k = 0; k < NB; ++k) { act[k] = rhs_live(sc, r0 + k, nrhs); any |= act[k]; }
  if (!any) return;
  const int i = site_block(g, blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double nrm[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) nrm[k] = 0.0;
  if (i < g.Vh) {
    S in[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) in[k] = field(v0, act[k] ? r0 + k : 0);
    Spinor<R> acc[NB];
    hop_site_multi<1, NB>(g, 1, i, L, in, act, acc);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!act[k]) continue;
      const int r = r0 + k;
      const RR alpha = RR(sc[r].alpha);
      const R kk = R(k2.v[r]);
      Spinor<R> uv, pv;
      Spinor<RR> rv, xv;
      field(u0, r).load(i, uv);
      field(p0, r).load(i, pv);
      field(rr0, r).load(i, rv);
      field(x0, r).load(i, xv);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cplx<R> ap = uv.c[s][c] - kk * acc[k].c[s][c];
          rv.c[s][c].re -= alpha * RR(ap.re);
          rv.c[s][c].im -= alpha * RR(ap.im);
          xv.c[s][c].re += alpha * RR(pv.c[s][c].re);
          xv.c[s][c].im += alpha * RR(pv.c[s][c].im);
        }
      field(rr0, r).store(i, rv);
      field(x0, r).store(i, xv);
      nrm[k] = norm2(rv);
    }
  }
  block_partials_multi<kBlock, NB>(nrm, red.partials, r0, nrhs);
}

template <bool MIXED>
__global__ __launch_bounds__(256) void k_mcg4_fin(CGScalars* sc, int nrhs, const double* partials, int nb) {
  const int r = blockIdx.x;
  if (!rhs_live(sc, r, nrhs)) return;
  const double rr_new = sum_partials<256>(partials + (size_t)r * nb, nb);
  if (threadIdx.x != 0) return;
  CGScalars& q = sc[r];
  const double rr_old = q.rr;
  q.beta = rr_new / rr_old;
  q.rr_old = rr_old;
  q.rr = rr_new;
  q.iter += 1;
  if (!(rr_new < INFINITY)) {
    q.done = 1;
    return;
  }
  if (MIXED) {
    q.rmax2 = fmax(q.rmax2, rr_new);
    if (rr_new <= q.stop_rr || rr_new < q.delta2 * q.rmax2) q.pause = 1;
  } else {
    if (rr_new <= q.stop_rr) q.done = 1;
  }
}

template <class S, class SR>
__global__ __launch_bounds__(kBlock) void k_mcg5(int Vh, int nrhs, S p0, SR r0_, const CGScalars* sc) {
  using R = typename S::Real;
  const int r = blockIdx.y;
  if (!rhs_live(sc, r, nrhs)) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const R beta = R(sc[r].beta);
  Spinor<R> pv;
  Spinor<typename SR::Real> rv;
  S p = field(p0, r);
  field(r0_, r).load(i, rv);
  p.load(i, pv);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pv.c[s][c].re = R(rv.c[s][c].re) + beta * pv.c[s][c].re;
      pv.c[s][c].im = R(rv.c[s][c].im) + beta * pv.c[s][c].im;
    }
  p.store(i, pv);
}

// ------------------------------------------------------------------ host side
static SpinorF64 h64(void* p, int Vh) { return SpinorF64{(double2*)p, Vh}; }
static SpinorF32 h32(void* p, int Vh) { return SpinorF32{(float4*)p, Vh}; }
static SpinorF16 h16(void* p, int Vh) { return SpinorF16{(uint4*)p, (float*)((uint4*)p + (size_t)3 * Vh), Vh}; }
static size_t field_bytes(int prec, int Vh) { return (size_t)Vh * (prec == WHMC_F64 ? 192 : prec == WHMC_F32 ? 96 : 52); }

template <int NB, class Lnk, class S>
static void launch_mhop(whmc_ctx* c, int par, int dag, int nrhs, const Lnk& L, S in, S out) {
  dim3 grid(c->num_blocks(), (nrhs + NB - 1) / NB), block(kBlock);
  if (dag) hipLaunchKernelGGL((k_mhop<1, NB, Lnk, S>), grid, block, 0, c->stream, c->g, par, nrhs, L, in, out);
  else hipLaunchKernelGGL((k_mhop<0, NB, Lnk, S>), grid, block, 0, c->stream, c->g, par, nrhs, L, in, out);
}

template <class Lnk, class S>
static whmc_status mhop_nb(whmc_ctx* c, int nb, int par, int dag, int nrhs, const Lnk& L, S in, S out) {
  switch (nb) {
    case 1: launch_mhop<1>(c, par, dag, nrhs, L, in, out); break;
    case 2: launch_mhop<2>(c, par, dag, nrhs, L, in, out); break;
    case 3: launch_mhop<3>(c, par, dag, nrhs, L, in, out); break;
    case 4: launch_mhop<4>(c, par, dag, nrhs, L, in, out); break;
    default: set_error("rhs_block must be 1..4"); return WHMC_EARG;
  }
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

// dispatch on precision / link format / cache policy; f(L, S-maker) is called with the typed link
// accessor and a function turning a device pointer into the spinor accessor of that precision.
template <class F>
static whmc_status with_format(whmc_ctx* c, int prec, int links, F&& f) {
  WHMC_TRY(ensure_links(c, prec, links));
  const int Vh = c->Vh;
  const bool nt = c->stream_links(prec, links);
  if (prec == WHMC_F64 && links == WHMC_L18) {
    if (nt) return f(LinkF64_18T<true>{c->U18, Vh}, h64);
    return f(LinkF64_18T<false>{c->U18, Vh}, h64);
  }
  if (prec == WHMC_F64 && links == WHMC_L12) {
    if (nt) return f(LinkF64_12T<true>{c->U12, Vh}, h64);
    return f(LinkF64_12T<false>{c->U12, Vh}, h64);
  }
  if (prec == WHMC_F32 && links == WHMC_L12) {
    if (nt) return f(LinkF32_12T<true>{c->U32_12, Vh}, h32);
    return f(LinkF32_12T<false>{c->U32_12, Vh}, h32);
  }
  if (prec == WHMC_F16 && links == WHMC_L12) {
    if (nt) return f(LinkF16_12T<true>{c->U16_12, Vh}, h16);
    return f(LinkF16_12T<false>{c->U16_12, Vh}, h16);
  }
  set_error("multi-RHS kernels support FP64 with 18- or 12-real links and FP32 / FP16 with 12-real links");
  return WHMC_EUNSUP;
}

whmc_status mhop(whmc_ctx* c, int prec, int links, int par, int dag, int nrhs, int nb, void* out, const void* in) {
  return with_format(c, prec, links, [&](auto L, auto mk) {
    return mhop_nb(c, nb, par, dag, nrhs, L, mk((void*)in, c->Vh), mk(out, c->Vh));
  });
}

// ---- autotuner: time the multi-RHS hop for every register block and keep the fastest
whmc_status autotune_rhs_block(whmc_ctx* c, int prec, int links, int nrhs, int* best_nb, double* best_us) {
  const std::string key = std::to_string(prec) + "/" + std::to_string(links) + "/" + std::to_string(nrhs);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    *best_nb = it->second.first;
    if (best_us) *best_us = it->second.second;
    return WHMC_OK;
  }
  const size_t fb = field_bytes(prec, c->Vh);
  void *in, *out;
  WHMC_TRY(workspace(c, "tune_in", fb * nrhs, &in));
  WHMC_TRY(workspace(c, "tune_out", fb * nrhs, &out));
  WHMC_TRY(zero_bytes(c, in, fb * nrhs));
  hipEvent_t e0, e1;
  WHMC_HIP(hipEventCreate(&e0));
  WHMC_HIP(hipEventCreate(&e1));
  int bnb = 1;
  double bt = 1e30;
  const int maxnb = nrhs < 4 ? nrhs : 4;
  for (int nb = 1; nb <= maxnb; ++nb) {
    WHMC_TRY(mhop(c, prec, links, 0, 0, nrhs, nb, out, in));   // warm-up
    WHMC_HIP(hipEventRecord(e0, c->stream));
    for (int rep = 0; rep < 3; ++rep) WHMC_TRY(mhop(c, prec, links, 0, 0, nrhs, nb, out, in));
    WHMC_HIP(hipEventRecord(e1, c->stream));
    WHMC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    WHMC_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double us = ms * 1e3 / 3.0;
    if (us < bt) {
      bt = us;
      bnb = nb;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned[key] = {bnb, bt};
  *best_nb = bnb;
  if (best_us) *best_us = bt;
  return WHMC_OK;
}

// ---- masked multi-RHS CG
struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double s() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

__global__ void k_minit(CGScalars* sc, const double* rr, int n, double tol2, double delta2) {
  const int r = threadIdx.x;
  if (r >= n) return;
  sc[r].rr = rr[r];
  sc[r].stop_rr = tol2 * rr[r];
  sc[r].rmax2 = rr[r];
  sc[r].delta2 = delta2;
  sc[r].done = (rr[r] == 0.0);
  sc[r].pause = 0;
  sc[r].iter = 0;
  sc[r].alpha = sc[r].beta = sc[r].pAp = sc[r].rr_old = 0.0;
  sc[r].active = 1;
}

__global__ void k_mresume(CGScalars* sc, int r, const double* rr, int converged) {
  if (threadIdx.x != 0) return;
  if (converged) {
    sc[r].done = 1;
  } else {
    sc[r].rr = *rr;
    sc[r].rmax2 = *rr;
  }
  sc[r].pause = 0;
}

// FP64 restart of rhs r from its true residual: |r|^2 from the device, threshold tol^2 |b|^2
__global__ void k_mrestart(CGScalars* sc, int r, const double* rr, double stop_rr) {
  if (threadIdx.x != 0) return;
  sc[r].rr = *rr;
  sc[r].stop_rr = stop_rr;
  sc[r].rmax2 = *rr;
  sc[r].done = (*rr <= stop_rr);
  sc[r].pause = 0;
}

template <class SR>
__global__ void k_maccum_x(int Vh, double2* x, SR xs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vh) return;
  Spinor<typename SR::Real> v;
  xs.load(i, v);
  SpinorF64 X{x, Vh};
  Spinor<double> a;
  X.load(i, a);
  for (int s = 0; s < 4; ++s)
    for (int cc = 0; cc < 3; ++cc) {
      a.c[s][cc].re += (double)v.c[s][cc].re;
      a.c[s][cc].im += (double)v.c[s][cc].im;
      v.c[s][cc] = {0, 0};
    }
  X.store(i, a);
  xs.store(i, v);
}

template <class S, class SR>
__global__ __launch_bounds__(kBlock) void k_mdot_rp(int Vh, S p, SR r, Reduce red, double* out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double s = 0.0;
  if (i < Vh) {
    Spinor<typename S::Real> pv;
    Spinor<typename SR::Real> rv;
    p.load(i, pv);
    r.load(i, rv);
    for (int a = 0; a < 4; ++a)
      for (int cc = 0; cc < 3; ++cc)
        s += (double)pv.c[a][cc].re * (double)rv.c[a][cc].re + (double)pv.c[a][cc].im * (double)rv.c[a][cc].im;
  }
  block_partial<kBlock>(s, red.partials, blockIdx.x);
}

template <class S, class SR>
__global__ __launch_bounds__(kBlock) void k_mrel_p(int Vh, S p, SR r, const double* rp, const CGScalars* sc) {
  using R = typename S::Real;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= Vh) return;
  const double rr = sc->rr;
  const R gamma = R(rp[0] / rr);
  const R beta = R(rr / sc->rr_old);
  Spinor<R> pv;
  Spinor<typename SR::Real> rv;
  p.load(i, pv);
  r.load(i, rv);
  for (int s = 0; s < 4; ++s)
    for (int cc = 0; cc < 3; ++cc) {
      pv.c[s][cc].re = R(rv.c[s][cc].re) + beta * (pv.c[s][cc].re - gamma * R(rv.c[s][cc].re));
      pv.c[s][cc].im = R(rv.c[s][cc].im) + beta * (pv.c[s][cc].im - gamma * R(rv.c[s][cc].im));
    }
  p.store(i, pv);
}

template <int NB, bool MIXED, class Lnk, class S, class SR>
static void enqueue_multi(whmc_ctx* c, int nrhs, const Lnk& L, S p, S t, S u, S v, SR r, SR x, const K2& k2, int n) {
  const dim3 grid(c->num_blocks(), (nrhs + NB - 1) / NB), block(kBlock), grid5(c->num_blocks(), nrhs);
  for (int it = 0; it < n; ++it) {
    hipLaunchKernelGGL((k_mcg1<NB, Lnk, S>), grid, block, 0, c->stream, c->g, nrhs, L, p, t, c->scal);
    hipLaunchKernelGGL((k_mcg2<NB, Lnk, S>), grid, block, 0, c->stream, c->g, nrhs, L, t, p, u, k2, c->scal, c->red);
    hipLaunchKernelGGL(k_mcg2_fin, dim3(nrhs), dim3(256), 0, c->stream, c->scal, nrhs, c->red.partials, (int)grid.x);
    hipLaunchKernelGGL((k_mcg3<NB, Lnk, S>), grid, block, 0, c->stream, c->g, nrhs, L, u, v, c->scal);
    hipLaunchKernelGGL((k_mcg4<NB, Lnk, S, SR, MIXED>), grid, block, 0, c->stream, c->g, nrhs, L, v, u, p, r, x, k2,
                       c->scal, c->red);
    hipLaunchKernelGGL(k_mcg4_fin<MIXED>, dim3(nrhs), dim3(256), 0, c->stream, c->scal, nrhs, c->red.partials,
                       (int)grid.x);
    hipLaunchKernelGGL((k_mcg5<S, SR>), grid5, block, 0, c->stream, c->Vh, nrhs, p, r, c->scal);
  }
}

template <bool MIXED, class Lnk, class S, class SR>
static whmc_status enqueue_multi_nb(whmc_ctx* c, int nb, int nrhs, const Lnk& L, S p, S t, S u, S v, SR r, SR x,
                                    const K2& k2, int n) {
  switch (nb) {
    case 1: enqueue_multi<1, MIXED>(c, nrhs, L, p, t, u, v, r, x, k2, n); break;
    case 2: enqueue_multi<2, MIXED>(c, nrhs, L, p, t, u, v, r, x, k2, n); break;
    case 3: enqueue_multi<3, MIXED>(c, nrhs, L, p, t, u, v, r, x, k2, n); break;
    default: enqueue_multi<4, MIXED>(c, nrhs, L, p, t, u, v, r, x, k2, n); break;
  }
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

static whmc_status true_residual_r(whmc_ctx* c, double* r_out, const double* x, const double* b, double kappa,
                                   double* te, double* to, double bb, double* rel) {
  WHMC_TRY(apply_MdagM_f64(c, r_out, x, kappa, te, to));
  WHMC_TRY(axpby_f64(c, r_out, 1.0, b, -1.0, 1));
  double rr;
  WHMC_TRY(norm2_f64(c, r_out, 1, c->red.result + 2));
  WHMC_TRY(read_scalar(c, c->red.result + 2, &rr));
  *rel = std::sqrt(rr / bb);
  return WHMC_OK;
}

whmc_status cg_solve_multi(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                           const whmc_cg_params* prm, whmc_cg_stats* st) {
  Timer tm;
  const bool mixed = prm->prec != WHMC_F64;
  const int prec = prm->prec;
  const int links = prm->links;
  if (mixed && links != WHMC_L12) {
    // no multi-RHS kernels for this format: solve the right-hand sides one after the other
    whmc_cg_params one = *prm;
    whmc_status worst = WHMC_OK;
    for (int r = 0; r < nrhs; ++r) {
      whmc_status rc = cg_solve(c, x + (size_t)r * 24 * c->Vh, b + (size_t)r * 24 * c->Vh, kappas + r, 1, &one,
                                st ? st + r : nullptr);
      if (rc == WHMC_ENOCONV) worst = rc;
      else if (rc != WHMC_OK) return rc;
    }
    return worst;
  }
  const int Vh = c->Vh;
  const size_t hb = (size_t)Vh * 192;
  const size_t sb = field_bytes(prec, Vh);
  const int rprec = mixed ? WHMC_F32 : WHMC_F64;
  const size_t rb = field_bytes(rprec, Vh);
  int nb = prm->rhs_block;
  if (nb <= 0) WHMC_TRY(autotune_rhs_block(c, prec, links, nrhs, &nb, nullptr));
  WHMC_CHECK(nb >= 1 && nb <= 4, WHMC_EARG, "rhs_block must be 0 (autotune) or 1..4");
  void *p, *t, *u, *v, *rs, *xs, *r64, *te, *to;
  WHMC_TRY(workspace(c, "m_p", sb * nrhs, &p));
  WHMC_TRY(workspace(c, "m_t", sb * nrhs, &t));
  WHMC_TRY(workspace(c, "m_u", sb * nrhs, &u));
  WHMC_TRY(workspace(c, "m_v", sb * nrhs, &v));
  WHMC_TRY(workspace(c, "m_r", rb * nrhs, &rs));
  WHMC_TRY(workspace(c, "m_x", rb * nrhs, &xs));
  WHMC_TRY(workspace(c, "cg_r", hb, &r64));
  WHMC_TRY(workspace(c, "cg_te", hb, &te));
  WHMC_TRY(workspace(c, "cg_to", hb, &to));
  std::vector<double> bb(nrhs);
  for (int r = 0; r < nrhs; ++r) WHMC_TRY(norm2_f64(c, b + (size_t)r * 24 * Vh, 1, c->red.result + 16 + r));
  WHMC_HIP(hipMemcpyAsync(c->host_pinned + 16, c->red.result + 16, nrhs * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  for (int r = 0; r < nrhs; ++r) bb[r] = c->host_pinned[16 + r];
  WHMC_TRY(zero_bytes(c, x, hb * nrhs));
  // sloppy (or FP64) copies: r = b, p = b, x_s = 0
  if (mixed) {
    WHMC_TRY(convert_spinor(c, rs, rprec, b, WHMC_F64, nrhs));
    WHMC_TRY(convert_spinor(c, p, prec, b, WHMC_F64, nrhs));
  } else {
    WHMC_HIP(hipMemcpyAsync(rs, b, hb * nrhs, hipMemcpyDeviceToDevice, c->stream));
    WHMC_HIP(hipMemcpyAsync(p, b, hb * nrhs, hipMemcpyDeviceToDevice, c->stream));
  }
  WHMC_TRY(zero_bytes(c, xs, rb * nrhs));
  hipLaunchKernelGGL(k_minit, dim3(1), dim3(64), 0, c->stream, c->scal, c->red.result + 16, nrhs,
                     prm->tol * prm->tol, prm->delta * prm->delta);
  WHMC_HIP(hipGetLastError());
  K2 k2{};
  for (int r = 0; r < nrhs; ++r) k2.v[r] = kappas[r] * kappas[r];
  std::vector<int> rel_updates(nrhs, 0), conv(nrhs, 0);
  const int check = prm->check_every > 0 ? prm->check_every : 8;
  CGScalars* hs = c->scal_host;
  std::vector<double> rel_final(nrhs, 0.0);
  bool all = false;
  for (int pass = 0; pass < 4 && !all; ++pass) {
    int max_iter_seen = 0;
    while (true) {
      WHMC_TRY(with_format(c, prec, links, [&](auto L, auto mk) {
        if (mixed)
          return enqueue_multi_nb<true>(c, nb, nrhs, L, mk(p, Vh), mk(t, Vh), mk(u, Vh), mk(v, Vh), h32(rs, Vh),
                                        h32(xs, Vh), k2, check);
        return enqueue_multi_nb<false>(c, nb, nrhs, L, mk(p, Vh), mk(t, Vh), mk(u, Vh), mk(v, Vh), h64(rs, Vh),
                                       h64(xs, Vh), k2, check);
      }));
      WHMC_HIP(hipMemcpyAsync(hs, c->scal, nrhs * sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
      WHMC_HIP(hipStreamSynchronize(c->stream));
      bool live = false;
      max_iter_seen = 0;
      for (int r = 0; r < nrhs; ++r) max_iter_seen = std::max(max_iter_seen, hs[r].iter);
      for (int r = 0; r < nrhs; ++r) {
        const CGScalars q = hs[r];
        if (mixed && q.pause && !q.done) {
          // reliable update of rhs r in FP64
          double* xr = x + (size_t)r * 24 * Vh;
          const double* br = b + (size_t)r * 24 * Vh;
          char* xsr = (char*)xs + rb * r;
          char* rsr = (char*)rs + rb * r;
          char* pr = (char*)p + sb * r;
          hipLaunchKernelGGL((k_maccum_x<SpinorF32>), dim3((Vh + 255) / 256), dim3(256), 0, c->stream, Vh,
                             (double2*)xr, h32(xsr, Vh));
          WHMC_HIP(hipGetLastError());
          double rel;
          WHMC_TRY(true_residual_r(c, (double*)r64, xr, br, kappas[r], (double*)te, (double*)to, bb[r], &rel));
          rel_updates[r] += 1;
          const int ok = rel <= prm->tol;
          if (!ok) {
            WHMC_TRY(convert_spinor(c, rsr, WHMC_F32, r64, WHMC_F64, 1));
            WHMC_TRY(norm2_f64(c, (double*)r64, 1, c->red.result + 5));
          }
          hipLaunchKernelGGL(k_mresume, dim3(1), dim3(64), 0, c->stream, c->scal, r, c->red.result + 5, ok);
          if (!ok) {
            const dim3 gr(c->num_blocks());
            WHMC_TRY(with_format(c, prec, links, [&](auto L, auto mk) {
              (void)L;
              hipLaunchKernelGGL((k_mdot_rp<decltype(mk(pr, Vh)), SpinorF32>), gr, dim3(kBlock), 0, c->stream, Vh,
                                 mk(pr, Vh), h32(rsr, Vh), c->red, c->red.result + 6);
              if (finish_sum(c, (int)gr.x, c->red.result + 6) != WHMC_OK) return WHMC_EHIP;
              hipLaunchKernelGGL((k_mrel_p<decltype(mk(pr, Vh)), SpinorF32>), gr, dim3(kBlock), 0, c->stream, Vh,
                                 mk(pr, Vh), h32(rsr, Vh), c->red.result + 6, c->scal + r);
              return WHMC_OK;
            }));
          }
          WHMC_HIP(hipGetLastError());
          conv[r] = ok;
          if (!ok) live = true;
        } else if (!q.done) {
          live = true;
        }
      }
      if (!live || max_iter_seen >= prm->maxiter) break;
    }
    // FP64 solutions and their true residuals
    WHMC_HIP(hipMemcpyAsync(hs, c->scal, nrhs * sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
    WHMC_HIP(hipStreamSynchronize(c->stream));
    all = true;
    for (int r = 0; r < nrhs; ++r) {
      double* xr = x + (size_t)r * 24 * Vh;
      const double* br = b + (size_t)r * 24 * Vh;
      if (mixed) {
        if (!conv[r]) {
          hipLaunchKernelGGL((k_maccum_x<SpinorF32>), dim3((Vh + 255) / 256), dim3(256), 0, c->stream, Vh,
                             (double2*)xr, h32((char*)xs + rb * r, Vh));
          WHMC_HIP(hipGetLastError());
        }
      } else {
        WHMC_HIP(hipMemcpyAsync(xr, (char*)xs + rb * r, hb, hipMemcpyDeviceToDevice, c->stream));
      }
      double rel = 0.0;
      if (bb[r] != 0.0)
        WHMC_TRY(true_residual_r(c, (double*)r64, xr, br, kappas[r], (double*)te, (double*)to, bb[r], &rel));
      rel_final[r] = rel;
      const bool ok = rel <= prm->tol;
      if (!ok && !mixed) {
        // restart this rhs from its true residual (r64 = b - A x): r = p = r64, x continues
        WHMC_HIP(hipMemcpyAsync((char*)rs + rb * r, r64, hb, hipMemcpyDeviceToDevice, c->stream));
        WHMC_HIP(hipMemcpyAsync((char*)p + sb * r, r64, hb, hipMemcpyDeviceToDevice, c->stream));
        WHMC_TRY(norm2_f64(c, (double*)r64, 1, c->red.result + 5));
        hipLaunchKernelGGL(k_mrestart, dim3(1), dim3(64), 0, c->stream, c->scal, r, c->red.result + 5,
                           prm->tol * prm->tol * bb[r]);
        WHMC_HIP(hipGetLastError());
      }
      all = all && ok;
    }
    if (mixed || max_iter_seen >= prm->maxiter) break;
  }
  const double secs = tm.s();
  if (st)
    for (int r = 0; r < nrhs; ++r) {
      st[r].iters = hs[r].iter;
      st[r].reliable_updates = rel_updates[r];
      st[r].converged = rel_final[r] <= prm->tol;
      st[r].true_residual = rel_final[r];
      st[r].seconds = secs;
    }
  if (!all) {
    set_error("multi-RHS CG: not every right-hand side reached the tolerance");
    return WHMC_ENOCONV;
  }
  return WHMC_OK;
}

}  // namespace whmc

using namespace whmc;

extern "C" whmc_status whmc_apply_H_multi(whmc_ctx* c, void* out, const void* in, int out_parity, int dagger,
                                          int prec, int links, int nrhs, int rhs_block) {
  WHMC_CHECK(c && out && in && out != in, WHMC_EARG, "whmc_apply_H_multi: bad pointers");
  WHMC_CHECK(out_parity == 0 || out_parity == 1, WHMC_EARG, "whmc_apply_H_multi: out_parity must be 0 or 1");
  WHMC_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, WHMC_EARG, "whmc_apply_H_multi: nrhs must be in [1, 16]");
  int nb = rhs_block;
  if (nb <= 0) WHMC_TRY(autotune_rhs_block(c, prec, links, nrhs, &nb, nullptr));
  return mhop(c, prec, links, out_parity, dagger ? 1 : 0, nrhs, nb, out, in);
}

extern "C" whmc_status whmc_autotune(whmc_ctx* c, int prec, int links, int nrhs, int* rhs_block, double* us) {
  WHMC_CHECK(c && rhs_block, WHMC_EARG, "whmc_autotune: null argument");
  WHMC_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, WHMC_EARG, "whmc_autotune: nrhs must be in [1, 16]");
  return autotune_rhs_block(c, prec, links, nrhs, rhs_block, us);
}
