// Multi right-hand-side hopping matrix and masked CG.
//
// One launch applies H to N_rhs spinor fields.  Each thread owns one (site, rhs) pair and does the
// single-rhs arithmetic, so its register use is that of the single-rhs hop.  The right-hand sides
// form G = ceil(N_rhs / R) groups of R = 1, 2, 4 or 8; a workgroup of kBlock threads covers
// kBlock / R sites (part `sub` of a kBlock-site block) for the R right-hand sides of one group.  In
// every wavefront the lanes of one site for the R right-hand sides issue the same link addresses
// in the same load instruction, which the memory pipeline serves once, and the R * G workgroups of
// a site block run back to back on the same XCD, where the links are still in its L2.
// Algorithmic bytes per site and rhs: (8 link loads + N_rhs (in + out) spinors) / N_rhs.
//
// The CG runs every rhs with its own kappa (mass-preconditioning shifts) and its own device-side
// scalars.  A converged (or paused, in mixed precision) rhs is masked: its threads skip loads,
// arithmetic and stores while the others keep iterating, and a workgroup whose right-hand sides
// are all masked exits at once.  R is chosen by the autotuner (timed on first use per precision,
// link format and N_rhs) unless the caller fixes it.
#include <chrono>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

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

// ------------------------------------------------------------------ lane layout
// The right-hand sides form groups of R * NB.  The workgroups of a site block are numbered
// u = grp * R + sub (sub fastest); wavefront w of workgroup (grp, sub) holds the sites
// sub * kBlock / R + w * S + (0 .. S-1) of the block (S = 64 / R), and lane l has site ... + l % S
// and the NB right-hand sides rb .. rb + NB - 1, rb = grp * R * NB + (l / S) * NB.
template <int NB, int R>
struct MLane {
  int i;      // cb site index (>= Vh: padding workgroup or ragged tail)
  int rb;     // first rhs of the lane's register block
  int r0;     // first rhs of the workgroup's group
  int sub;    // part of the site block
  int slot;   // partial-sum slot of this workgroup among the workgroups of its (grp, sub)
};

template <int NB, int R>
WHMC_DEV MLane<NB, R> mlane(const Geom& g, int G, int order) {
  constexpr int S = 64 / R;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  int u, sb;
  MLane<NB, R> m;
  if (order == 1) {
    // group-major: the per = (site grid) * R workgroups of rhs group 0 sweep the lattice first,
    // then those of group 1, ...; inside a group the R parts of a site block run back to back
    const int per = gridDim.x / G;
    const int grp = blockIdx.x / per;
    int sub;
    sb = site_block_grp(g, blockIdx.x - grp * per, per, R, sub, m.slot);
    u = grp * R + sub;
  } else {
    // block-major: the G * R workgroups of a site block run back to back (links shared in L2)
    sb = site_block_grp(g, blockIdx.x, gridDim.x, G * R, u, m.slot);
  }
  const int grp = u / R;
  m.sub = u - grp * R;
  m.r0 = grp * R * NB;
  m.rb = m.r0 + (l / S) * NB;
  m.i = sb * kBlock + m.sub * (kBlock / R) + w * S + (l % S);
  return m;
}

WHMC_DEV bool rhs_live(const CGScalars* sc, int r, int nrhs) { return r < nrhs && !(sc[r].done | sc[r].pause); }

// which right-hand sides a launch works on: all of them ...
struct AllRhs {
  int nrhs;
  WHMC_DEV bool operator()(int r) const { return r < nrhs; }
};
// ... those still iterating (device-side CG flags) ...
struct ByScalars {
  const CGScalars* sc;
  int nrhs;
  WHMC_DEV bool operator()(int r) const { return rhs_live(sc, r, nrhs); }
};
// ... or a set chosen by the host (bit r of mask)
struct BySet {
  unsigned mask;
  int nrhs;
  WHMC_DEV bool operator()(int r) const { return r < nrhs && ((mask >> r) & 1u); }
};

template <int N, class P>
WHMC_DEV bool any_live(const P& live, int r0) {
  bool any = false;
#pragma unroll
  for (int q = 0; q < N; ++q) any |= live(r0 + q);
  return any;
}

// ------------------------------------------------------------------ per-rhs partial sums
// pass 1: the workgroup sums each of its R * NB right-hand sides (lane shuffles inside the S-lane
// run of that rhs, then the wavefronts in a fixed order) and writes rhs r's sum to row
// r * R + sub, slot slot of partials (rows of nslots doubles: rhs r owns rows r * R .. r * R + R - 1);
// pass 2 (k_m*_fin, one block per rhs) adds the R * nslots partials of rhs r in a fixed order.
template <int NB, int R>
WHMC_DEV void mpartials(const double* v, double* partials, const MLane<NB, R>& m, int nrhs, int nslots) {
  constexpr int S = 64 / R, W = kBlock / 64;
  __shared__ double lds[W][R * NB];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = S / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (l % S == 0) lds[w][(l / S) * NB + k] = x;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < R * NB && m.r0 + t < nrhs) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) s += lds[k][t];
    partials[((size_t)(m.r0 + t) * R + m.sub) * nslots + m.slot] = s;
  }
}

// ------------------------------------------------------------------ multi-RHS stencil
// one link load (and, for 12-real links, one third-row reconstruction) serves the NB right-hand
// sides of the thread's register block
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

// out_k = H_{par,1-par}^{(DAG)} in_k for the live rhs of the lane's register block
template <int DAG, int NB, int R, class Lnk, class S, class P>
WHMC_DEV void mhop_body(const Geom& g, int par, const MLane<NB, R>& m, const Lnk& L, S in0, S out0, const P& live) {
  using Re = typename S::Real;
  bool act[NB], any = false;
  S in[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    act[k] = live(m.rb + k);
    any |= act[k];
    in[k] = field(in0, act[k] ? m.rb + k : 0);
  }
  if (!any) return;
  Spinor<Re> acc[NB];
  hop_site_multi<DAG, NB>(g, par, m.i, L, in, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (act[k]) field(out0, m.rb + k).store(m.i, acc[k]);
}

// plain multi-RHS hop: out_r = H_{par,1-par}^{(dag)} in_r
template <int DAG, int NB, int R, class Lnk, class S>
__global__ __launch_bounds__(kBlock) void k_mhop(Geom g, int par, int nrhs, int G, int order, Lnk L, S in0, S out0) {
  const MLane<NB, R> m = mlane<NB, R>(g, G, order);
  if (m.i >= g.Vh) return;
  mhop_body<DAG>(g, par, m, L, in0, out0, AllRhs{nrhs});
}

// CG kernel 1: t = H_eo p
template <int NB, int R, class Lnk, class S, class P>
__global__ __launch_bounds__(kBlock) void k_mcg1(Geom g, int G, int order, Lnk L, S p0, S t0, P live) {
  const MLane<NB, R> m = mlane<NB, R>(g, G, order);
  if (m.i >= g.Vh) return;
  mhop_body<0>(g, 0, m, L, p0, t0, live);
}

// CG kernel 3: v = H^dag_eo u
template <int NB, int R, class Lnk, class S, class P>
__global__ __launch_bounds__(kBlock) void k_mcg3(Geom g, int G, int order, Lnk L, S u0, S v0, P live) {
  const MLane<NB, R> m = mlane<NB, R>(g, G, order);
  if (m.i >= g.Vh) return;
  mhop_body<1>(g, 0, m, L, u0, v0, live);
}

// CG kernel 2: u = p - kappa^2 H_oe t, |u|^2 = (p, A p)
template <int NB, int R, class Lnk, class S, class P>
__global__ __launch_bounds__(kBlock) void k_mcg2(Geom g, int nrhs, int G, int order, Lnk L, S t0, S p0, S u0, K2 k2, P live,
                                                 Reduce red, int nslots) {
  using Re = typename S::Real;
  const MLane<NB, R> m = mlane<NB, R>(g, G, order);
  if (!any_live<R * NB>(live, m.r0)) return;   // uniform over the workgroup
  double nrm[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) nrm[k] = 0.0;
  if (m.i < g.Vh) {
    bool act[NB], any = false;
    S in[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      act[k] = live(m.rb + k);
      any |= act[k];
      in[k] = field(t0, act[k] ? m.rb + k : 0);
    }
    if (any) {
      Spinor<Re> acc[NB];
      hop_site_multi<0, NB>(g, 1, m.i, L, in, act, acc);
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (!act[k]) continue;
        const int r = m.rb + k;
        Spinor<Re> pv;
        field(p0, r).load(m.i, pv);
        const Re kk = Re(k2.v[r]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[k].c[s][c] = pv.c[s][c] - kk * acc[k].c[s][c];
        field(u0, r).store(m.i, acc[k]);
        nrm[k] = norm2(acc[k]);
      }
    }
  }
  mpartials<NB, R>(nrm, red.partials, m, nrhs, nslots);
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

// CG kernel 4: A p = u - kappa^2 H^dag_oe v;  r -= alpha A p,  x += alpha p,  |r|^2
template <int NB, int R, class Lnk, class S, class SR, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_mcg4(Geom g, int nrhs, int G, int order, Lnk L, S v0, S u0, S p0, SR rr0, SR x0,
                                                 K2 k2, CGScalars* sc, Reduce red, int nslots) {
  using Re = typename S::Real;
  using RR = typename SR::Real;
  const MLane<NB, R> m = mlane<NB, R>(g, G, order);
  const ByScalars live{sc, nrhs};
  if (!any_live<R * NB>(live, m.r0)) return;   // uniform over the workgroup
  double nrm[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) nrm[k] = 0.0;
  if (m.i < g.Vh) {
    const int i = m.i;
    bool act[NB], any = false;
    S in[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      act[k] = live(m.rb + k);
      any |= act[k];
      in[k] = field(v0, act[k] ? m.rb + k : 0);
    }
    if (any) {
      Spinor<Re> acc[NB];
      hop_site_multi<1, NB>(g, 1, i, L, in, act, acc);
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (!act[k]) continue;
        const int r = m.rb + k;
        const RR alpha = RR(sc[r].alpha);
        const Re kk = Re(k2.v[r]);
        Spinor<Re> uv, pv;
        Spinor<RR> rv, xv;
        field(u0, r).load(i, uv);
        field(p0, r).load(i, pv);
        field(rr0, r).load(i, rv);
        field(x0, r).load(i, xv);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            cplx<Re> ap = uv.c[s][c] - kk * acc[k].c[s][c];
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
  }
  mpartials<NB, R>(nrm, red.partials, m, nrhs, nslots);
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

// FP64 residual of the host-chosen right-hand sides, last hop of M^dag M fused:
// r_r = b_r - (u_r - kappa_r^2 H^dag_oe v_r), |r_r|^2 to the partial sums
template <int R, class Lnk>
__global__ __launch_bounds__(kBlock) void k_mres(Geom g, int nrhs, int G, int order, Lnk L, SpinorF64 v0, SpinorF64 u0,
                                                 SpinorF64 b0, SpinorF64 r0, K2 k2, BySet live, Reduce red,
                                                 int nslots) {
  const MLane<1, R> m = mlane<1, R>(g, G, order);
  if (!any_live<R>(live, m.r0)) return;   // uniform over the workgroup
  double nrm = 0.0;
  if (m.i < g.Vh && live(m.rb)) {
    const int r = m.rb, i = m.i;
    Spinor<double> acc, uv, bv;
    hop_site<1>(g, 1, i, L, field(v0, r), acc);
    field(u0, r).load(i, uv);
    field(b0, r).load(i, bv);
    const double kk = k2.v[r];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.c[s][c] = bv.c[s][c] - (uv.c[s][c] - kk * acc.c[s][c]);
    field(r0, r).store(i, acc);
    nrm = norm2(acc);
  }
  mpartials<1, R>(&nrm, red.partials, m, nrhs, nslots);
}

// pass 2 of k_mres: out[r] = |r_r|^2 for the chosen right-hand sides
__global__ __launch_bounds__(256) void k_mres_fin(BySet live, const double* partials, int nb, double* out) {
  const int r = blockIdx.x;
  if (!live(r)) return;
  const double rr = sum_partials<256>(partials + (size_t)r * nb, nb);
  if (threadIdx.x == 0) out[r] = rr;
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

// Blocking of the multi-RHS kernels: NB right-hand sides per thread (register block), R lanes
// per site sharing each link load, and the order of the workgroups: 0 = block-major (all groups of
// right-hand sides of a site block back to back, links reused from L2), 1 = group-major (each group
// of R * NB right-hand sides sweeps the lattice before the next: the neighbour spinors of the group
// stay in L2 while the links are read once per group).  FP64 keeps NB = 1 (its single-rhs hop
// already fills the register file); the low-precision formats also block in registers.
struct Blocking {
  int nb, lanes, order;
};

template <class Lnk>
static constexpr bool is_f64_links() { return std::is_same<typename Lnk::Real, double>::value; }

// call f(integral_constant<NB>, integral_constant<R>) for an allowed blocking of this link format
template <class Lnk, class F>
static whmc_status with_blocking(Blocking b, F&& f) {
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  if constexpr (is_f64_links<Lnk>()) {
    if (b.nb == 1 && b.lanes == 1) return f(I1{}, I1{});
    if (b.nb == 1 && b.lanes == 2) return f(I1{}, I2{});
    if (b.nb == 1 && b.lanes == 4) return f(I1{}, I4{});
    if (b.nb == 2 && b.lanes == 1) return f(I2{}, I1{});
    if (b.nb == 2 && b.lanes == 2) return f(I2{}, I2{});
  } else {
    if (b.nb == 1 && b.lanes == 1) return f(I1{}, I1{});
    if (b.nb == 1 && b.lanes == 2) return f(I1{}, I2{});
    if (b.nb == 2 && b.lanes == 1) return f(I2{}, I1{});
    if (b.nb == 2 && b.lanes == 2) return f(I2{}, I2{});
    if (b.nb == 4 && b.lanes == 1) return f(I4{}, I1{});
    if (b.nb == 4 && b.lanes == 2) return f(I4{}, I2{});
  }
  set_error("multi-RHS blocking: FP64 takes rhs_block 1 with rhs_lanes 1, 2 or 4, or rhs_block 2 with rhs_lanes 1 or 2; "
            "FP32 / FP16 take rhs_block 1, 2 or 4 with rhs_lanes 1 or 2");
  return WHMC_EARG;
}

// the blockings the autotuner tries for a precision, nrhs right-hand sides
static std::vector<Blocking> candidates(int prec, int nrhs) {
  std::vector<Blocking> out;
  const int nbs[3] = {1, 2, 4}, ls[3] = {1, 2, 4};
  for (int nb : nbs) {
    if (prec == WHMC_F64 && nb > 2) break;
    for (int l : ls) {
      if ((prec != WHMC_F64 || nb > 1) && l > 2) break;
      const int group = nb * l;
      if (group > 1 && group / 2 >= nrhs) continue;   // wider than needed: idle lanes or registers
      out.push_back({nb, l, 0});
      if (nrhs > group) out.push_back({nb, l, 1});      // several groups: try group-major too
    }
  }
  return out;
}

template <int NB, int R, class Lnk, class S>
static void launch_mhop(whmc_ctx* c, int par, int dag, int nrhs, int order, const Lnk& L, S in, S out) {
  const int G = (nrhs + R * NB - 1) / (R * NB);
  const dim3 grid(c->stencil_blocks() * G * R), block(kBlock);
  if (dag)
    hipLaunchKernelGGL((k_mhop<1, NB, R, Lnk, S>), grid, block, 0, c->stream, c->g, par, nrhs, G, order, L, in, out);
  else
    hipLaunchKernelGGL((k_mhop<0, NB, R, Lnk, S>), grid, block, 0, c->stream, c->g, par, nrhs, G, order, L, in, out);
}

// Links are streamed past the caches (non-temporal loads, for link arrays above the stream
// threshold) only where one launch reads each link once: with block-major order and several rhs
// groups, the groups of a site block run back to back and re-read the block's links from L2.
static bool stream_multi(const whmc_ctx* c, int prec, int links, int nrhs, const Blocking& b) {
  const int G = (nrhs + b.nb * b.lanes - 1) / (b.nb * b.lanes);
  return c->stream_links(prec, links) && (G == 1 || b.order == 1);
}

// dispatch on precision / link format / cache policy (nt: non-temporal link loads); f(L, S-maker)
// is called with the typed link accessor and a function turning a device pointer into the spinor
// accessor of that precision.
template <class F>
static whmc_status with_format(whmc_ctx* c, int prec, int links, bool nt, F&& f) {
  WHMC_TRY(ensure_links(c, prec, links));
  const int Vh = c->Vh;
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
  if (prec == WHMC_F64 && links == WHMC_L8) {
    if (nt) return f(LinkF64_8T<true>{c->U8, Vh}, h64);
    return f(LinkF64_8T<false>{c->U8, Vh}, h64);
  }
  if (prec == WHMC_F32 && links == WHMC_L8) {
    if (nt) return f(LinkF32_8T<true>{c->U32_8, Vh}, h32);
    return f(LinkF32_8T<false>{c->U32_8, Vh}, h32);
  }
  if (prec == WHMC_F16 && links == WHMC_L8) {
    if (nt) return f(LinkF16_8T<true>{c->U16_8, Vh}, h16);
    return f(LinkF16_8T<false>{c->U16_8, Vh}, h16);
  }
  set_error("multi-RHS kernels support FP64 with 18-, 12- or 8-real links and FP32 / FP16 with 12- or 8-real links");
  return WHMC_EUNSUP;
}

static whmc_status mhop(whmc_ctx* c, int prec, int links, int par, int dag, int nrhs, Blocking b, void* out,
                        const void* in) {
  WHMC_TRY(with_format(c, prec, links, stream_multi(c, prec, links, nrhs, b), [&](auto L, auto mk) {
    return with_blocking<decltype(L)>(b, [&](auto nb, auto lanes) {
      launch_mhop<decltype(nb)::value, decltype(lanes)::value>(c, par, dag, nrhs, b.order, L, mk((void*)in, c->Vh),
                                                                mk(out, c->Vh));
      return WHMC_OK;
    });
  }));
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

// ---- autotuner: time the multi-RHS hop for every candidate blocking and keep the fastest
static whmc_status autotune_blocking(whmc_ctx* c, int prec, int links, int nrhs, Blocking* best, double* best_us) {
  const std::string key = std::to_string(prec) + "/" + std::to_string(links) + "/" + std::to_string(nrhs);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    best->nb = it->second.first / 256;
    best->lanes = (it->second.first / 16) % 16;
    best->order = it->second.first % 16;
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
  Blocking bb{1, 1, 0};
  double bt = 1e30;
  for (const Blocking& b : candidates(prec, nrhs)) {
    WHMC_TRY(mhop(c, prec, links, 0, 0, nrhs, b, out, in));   // warm-up
    WHMC_HIP(hipEventRecord(e0, c->stream));
    for (int rep = 0; rep < 3; ++rep) WHMC_TRY(mhop(c, prec, links, 0, 0, nrhs, b, out, in));
    WHMC_HIP(hipEventRecord(e1, c->stream));
    WHMC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    WHMC_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double us = ms * 1e3 / 3.0;
    if (us < bt) {
      bt = us;
      bb = b;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned[key] = {bb.nb * 256 + bb.lanes * 16 + bb.order, bt};
  *best = bb;
  if (best_us) *best_us = bt;
  return WHMC_OK;
}

// the blocking a call asks for: nb = lanes = 0 = autotuned (order included), else the given values
// (0 read as 1) with the given order
static whmc_status resolve_blocking(whmc_ctx* c, int prec, int links, int nrhs, int nb, int lanes, int order,
                                    Blocking* b) {
  if (nb <= 0 && lanes <= 0) return autotune_blocking(c, prec, links, nrhs, b, nullptr);
  WHMC_CHECK(order == 0 || order == 1, WHMC_EARG, "multi-RHS order must be 0 (block-major) or 1 (group-major)");
  b->nb = nb > 0 ? nb : 1;
  b->lanes = lanes > 0 ? lanes : 1;
  b->order = order;
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

template <int NB, int R, bool MIXED, class Lnk, class S, class SR>
static void enqueue_multi(whmc_ctx* c, int nrhs, int order, const Lnk& L, S p, S t, S u, S v, SR r, SR x, const K2& k2,
                          int n) {
  const int G = (nrhs + R * NB - 1) / (R * NB), ns = c->stencil_blocks();
  const dim3 grid(ns * G * R), block(kBlock), grid5(c->num_blocks(), nrhs);
  const ByScalars live{c->scal, nrhs};
  for (int it = 0; it < n; ++it) {
    TraceRange tr("whmc multi-rhs cg iteration");
    hipLaunchKernelGGL((k_mcg1<NB, R, Lnk, S, ByScalars>), grid, block, 0, c->stream, c->g, G, order, L, p, t, live);
    hipLaunchKernelGGL((k_mcg2<NB, R, Lnk, S, ByScalars>), grid, block, 0, c->stream, c->g, nrhs, G, order, L, t, p, u,
                       k2,
                       live, c->red, ns);
    hipLaunchKernelGGL(k_mcg2_fin, dim3(nrhs), dim3(256), 0, c->stream, c->scal, nrhs, c->red.partials, ns * R);
    hipLaunchKernelGGL((k_mcg3<NB, R, Lnk, S, ByScalars>), grid, block, 0, c->stream, c->g, G, order, L, u, v, live);
    hipLaunchKernelGGL((k_mcg4<NB, R, Lnk, S, SR, MIXED>), grid, block, 0, c->stream, c->g, nrhs, G, order, L, v, u, p,
                       r, x,
                       k2, c->scal, c->red, ns);
    hipLaunchKernelGGL(k_mcg4_fin<MIXED>, dim3(nrhs), dim3(256), 0, c->stream, c->scal, nrhs, c->red.partials,
                       ns * R);
    hipLaunchKernelGGL((k_mcg5<S, SR>), grid5, block, 0, c->stream, c->Vh, nrhs, p, r, c->scal);
  }
}

// r_r = b_r - M_oo(kappa_r)^dag M_oo(kappa_r) x_r for every rhs r in mask, FP64 with 18-real links,
// through the multi-RHS kernels (one pass over the links serves all of them); |r_r|^2 lands in
// rr_dev[r].  t, u, v, r64 are FP64 scratch of nrhs half fields each.
template <int R, class Lnk>
static void enqueue_residual(whmc_ctx* c, unsigned mask, int nrhs, int order, const Lnk& L, SpinorF64 x, SpinorF64 b,
                             const K2& k2, SpinorF64 t, SpinorF64 u, SpinorF64 v, SpinorF64 r64, double* rr_dev) {
  const int G = (nrhs + R - 1) / R, ns = c->stencil_blocks();
  const dim3 grid(ns * G * R), block(kBlock);
  const BySet live{mask, nrhs};
  hipLaunchKernelGGL((k_mcg1<1, R, Lnk, SpinorF64, BySet>), grid, block, 0, c->stream, c->g, G, order, L, x, t, live);
  hipLaunchKernelGGL((k_mcg2<1, R, Lnk, SpinorF64, BySet>), grid, block, 0, c->stream, c->g, nrhs, G, order, L, t, x,
                     u, k2,
                     live, c->red, ns);
  hipLaunchKernelGGL((k_mcg3<1, R, Lnk, SpinorF64, BySet>), grid, block, 0, c->stream, c->g, G, order, L, u, v, live);
  hipLaunchKernelGGL((k_mres<R, Lnk>), grid, block, 0, c->stream, c->g, nrhs, G, order, L, v, u, b, r64, k2, live,
                     c->red,
                     ns);
  hipLaunchKernelGGL(k_mres_fin, dim3(nrhs), dim3(256), 0, c->stream, live, c->red.partials, ns * R, rr_dev);
}

static whmc_status residual_multi(whmc_ctx* c, unsigned mask, int nrhs, const double* x, const double* b,
                                  const K2& k2, void* t, void* u, void* v, void* r64, double* rr_dev) {
  Blocking bk;
  WHMC_TRY(autotune_blocking(c, WHMC_F64, WHMC_L18, nrhs, &bk, nullptr));
  const int Vh = c->Vh;
  auto run = [&](auto L) {
    return with_blocking<decltype(L)>(bk, [&](auto nb, auto lanes) {
      (void)nb;
      enqueue_residual<decltype(lanes)::value>(c, mask, nrhs, bk.order, L, h64((void*)x, Vh), h64((void*)b, Vh), k2,
                                               h64(t, Vh),
                                               h64(u, Vh), h64(v, Vh), h64(r64, Vh), rr_dev);
      return WHMC_OK;
    });
  };
  const Blocking b1{1, bk.lanes, bk.order};   // the residual kernels hold one rhs per thread
  if (stream_multi(c, WHMC_F64, WHMC_L18, nrhs, b1)) WHMC_TRY(run(LinkF64_18T<true>{c->U18, Vh}));
  else WHMC_TRY(run(LinkF64_18T<false>{c->U18, Vh}));
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

whmc_status cg_solve_multi(whmc_ctx* c, double* x, const double* b, const double* kappas, int nrhs,
                           const whmc_cg_params* prm, whmc_cg_stats* st) {
  Timer tm;
  const bool mixed = prm->prec != WHMC_F64;
  const int prec = prm->prec;
  const int links = prm->links;
  if (mixed && links == WHMC_L18) {
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
  Blocking bk;
  WHMC_TRY(resolve_blocking(c, prec, links, nrhs, prm->rhs_block, prm->rhs_lanes, prm->rhs_order, &bk));
  void *p, *t, *u, *v, *rs, *xs, *r64, *ft, *fu, *fv;
  WHMC_TRY(workspace(c, "m_p", sb * nrhs, &p));
  WHMC_TRY(workspace(c, "m_t", sb * nrhs, &t));
  WHMC_TRY(workspace(c, "m_u", sb * nrhs, &u));
  WHMC_TRY(workspace(c, "m_v", sb * nrhs, &v));
  WHMC_TRY(workspace(c, "m_r", rb * nrhs, &rs));
  WHMC_TRY(workspace(c, "m_x", rb * nrhs, &xs));
  WHMC_TRY(workspace(c, "m_r64", hb * nrhs, &r64));
  // FP64 scratch of the batched true residuals (the iteration's own fields when those are FP64)
  if (mixed) {
    WHMC_TRY(workspace(c, "m_ft", hb * nrhs, &ft));
    WHMC_TRY(workspace(c, "m_fu", hb * nrhs, &fu));
    WHMC_TRY(workspace(c, "m_fv", hb * nrhs, &fv));
  } else {
    ft = t, fu = u, fv = v;
  }
  double* rr_dev = c->red.result + 32;
  double* rr_host = c->host_pinned + 32;
  std::vector<double> bb(nrhs);
  for (int r = 0; r < nrhs; ++r) WHMC_TRY(norm2_f64(c, b + (size_t)r * 24 * Vh, 1, c->red.result + 16 + r));
  WHMC_HIP(hipMemcpyAsync(c->host_pinned + 16, c->red.result + 16, nrhs * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
  WHMC_HIP(hipStreamSynchronize(c->stream));
  for (int r = 0; r < nrhs; ++r) {
    bb[r] = c->host_pinned[16 + r];
    WHMC_CHECK(std::isfinite(bb[r]), WHMC_ENONFINITE,
               "multi-RHS CG: right-hand side " + std::to_string(r) + " is not finite");
  }
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
      WHMC_TRY(with_format(c, prec, links, stream_multi(c, prec, links, nrhs, bk), [&](auto L, auto mk) {
        return with_blocking<decltype(L)>(bk, [&](auto nbc, auto lanes) {
          constexpr int NB = decltype(nbc)::value, R = decltype(lanes)::value;
          // FP64 links run the plain FP64 CG, low-precision links the mixed one
          if constexpr (is_f64_links<decltype(L)>())
            enqueue_multi<NB, R, false>(c, nrhs, bk.order, L, mk(p, Vh), mk(t, Vh), mk(u, Vh), mk(v, Vh), h64(rs, Vh),
                                        h64(xs, Vh), k2, check);
          else
            enqueue_multi<NB, R, true>(c, nrhs, bk.order, L, mk(p, Vh), mk(t, Vh), mk(u, Vh), mk(v, Vh), h32(rs, Vh),
                                       h32(xs, Vh), k2, check);
          return WHMC_OK;
        });
      }));
      WHMC_HIP(hipGetLastError());
      WHMC_HIP(hipMemcpyAsync(hs, c->scal, nrhs * sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
      WHMC_HIP(hipStreamSynchronize(c->stream));
      bool live = false;
      max_iter_seen = 0;
      for (int r = 0; r < nrhs; ++r) max_iter_seen = std::max(max_iter_seen, hs[r].iter);
      unsigned paused = 0;
      for (int r = 0; r < nrhs; ++r) {
        if (mixed && hs[r].pause && !hs[r].done) paused |= 1u << r;
        else if (!hs[r].done) live = true;
      }
      if (paused) {
        // reliable updates of the paused right-hand sides, batched: x += x_s in FP64, then
        // r = b - A x and |r|^2 for all of them in one multi-RHS FP64 pass
        for (int r = 0; r < nrhs; ++r)
          if ((paused >> r) & 1u)
            hipLaunchKernelGGL((k_maccum_x<SpinorF32>), dim3((Vh + 255) / 256), dim3(256), 0, c->stream, Vh,
                               (double2*)(x + (size_t)r * 24 * Vh), h32((char*)xs + rb * r, Vh));
        WHMC_HIP(hipGetLastError());
        WHMC_TRY(residual_multi(c, paused, nrhs, x, b, k2, ft, fu, fv, r64, rr_dev));
        WHMC_HIP(hipMemcpyAsync(rr_host, rr_dev, nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        WHMC_HIP(hipStreamSynchronize(c->stream));
        for (int r = 0; r < nrhs; ++r) {
          if (!((paused >> r) & 1u)) continue;
          char* rsr = (char*)rs + rb * r;
          char* pr = (char*)p + sb * r;
          const double rel = std::sqrt(rr_host[r] / bb[r]);
          rel_updates[r] += 1;
          const int ok = rel <= prm->tol;
          if (!ok) WHMC_TRY(convert_spinor(c, rsr, WHMC_F32, (char*)r64 + hb * r, WHMC_F64, 1));
          hipLaunchKernelGGL(k_mresume, dim3(1), dim3(64), 0, c->stream, c->scal, r, rr_dev + r, ok);
          if (!ok) {
            const dim3 gr(c->num_blocks());
            WHMC_TRY(with_format(c, prec, links, false, [&](auto L, auto mk) {
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
        }
      }
      if (!live || max_iter_seen >= prm->maxiter) break;
    }
    // FP64 solutions and their true residuals
    WHMC_HIP(hipMemcpyAsync(hs, c->scal, nrhs * sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
    WHMC_HIP(hipStreamSynchronize(c->stream));
    all = true;
    unsigned nonzero = 0;
    for (int r = 0; r < nrhs; ++r) {
      double* xr = x + (size_t)r * 24 * Vh;
      if (mixed) {
        if (!conv[r]) {
          hipLaunchKernelGGL((k_maccum_x<SpinorF32>), dim3((Vh + 255) / 256), dim3(256), 0, c->stream, Vh,
                             (double2*)xr, h32((char*)xs + rb * r, Vh));
          WHMC_HIP(hipGetLastError());
        }
      } else {
        WHMC_HIP(hipMemcpyAsync(xr, (char*)xs + rb * r, hb, hipMemcpyDeviceToDevice, c->stream));
      }
      if (bb[r] != 0.0) nonzero |= 1u << r;
    }
    if (nonzero) {
      WHMC_TRY(residual_multi(c, nonzero, nrhs, x, b, k2, ft, fu, fv, r64, rr_dev));
      WHMC_HIP(hipMemcpyAsync(rr_host, rr_dev, nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      WHMC_HIP(hipStreamSynchronize(c->stream));
    }
    for (int r = 0; r < nrhs; ++r) {
      const double rel = ((nonzero >> r) & 1u) ? std::sqrt(rr_host[r] / bb[r]) : 0.0;
      rel_final[r] = rel;
      const bool ok = rel <= prm->tol;
      if (!ok && !mixed) {
        // restart this rhs from its true residual b - A x: r = p = that residual, x continues
        WHMC_HIP(hipMemcpyAsync((char*)rs + rb * r, (char*)r64 + hb * r, hb, hipMemcpyDeviceToDevice, c->stream));
        WHMC_HIP(hipMemcpyAsync((char*)p + sb * r, (char*)r64 + hb * r, hb, hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(k_mrestart, dim3(1), dim3(64), 0, c->stream, c->scal, r, rr_dev + r,
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
  for (int r = 0; r < nrhs; ++r)
    WHMC_CHECK(std::isfinite(rel_final[r]), WHMC_ENONFINITE,
               "multi-RHS CG: the residual of right-hand side " + std::to_string(r) + " is not finite");
  if (!all) {
    set_error("multi-RHS CG: not every right-hand side reached the tolerance");
    return WHMC_ENOCONV;
  }
  return WHMC_OK;
}

}  // namespace whmc

using namespace whmc;

extern "C" whmc_status whmc_apply_H_multi(whmc_ctx* c, void* out, const void* in, int out_parity, int dagger,
                                          int prec, int links, int nrhs, int rhs_block, int rhs_lanes, int rhs_order) {
  WHMC_CHECK(c && out && in && out != in, WHMC_EARG, "whmc_apply_H_multi: bad pointers");
  WHMC_CHECK(out_parity == 0 || out_parity == 1, WHMC_EARG, "whmc_apply_H_multi: out_parity must be 0 or 1");
  WHMC_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, WHMC_EARG, "whmc_apply_H_multi: nrhs must be in [1, 16]");
  Blocking b;
  WHMC_TRY(resolve_blocking(c, prec, links, nrhs, rhs_block, rhs_lanes, rhs_order, &b));
  return mhop(c, prec, links, out_parity, dagger ? 1 : 0, nrhs, b, out, in);
}

extern "C" whmc_status whmc_autotune(whmc_ctx* c, int prec, int links, int nrhs, int* rhs_block, int* rhs_lanes,
                                     int* rhs_order, double* us) {
  WHMC_CHECK(c && rhs_block && rhs_lanes, WHMC_EARG, "whmc_autotune: null argument");
  WHMC_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, WHMC_EARG, "whmc_autotune: nrhs must be in [1, 16]");
  Blocking b;
  WHMC_TRY(autotune_blocking(c, prec, links, nrhs, &b, us));
  *rhs_block = b.nb;
  *rhs_lanes = b.lanes;
  if (rhs_order) *rhs_order = b.order;
  return WHMC_OK;
}
