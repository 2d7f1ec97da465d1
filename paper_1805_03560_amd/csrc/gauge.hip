// Gauge-field kernels: plaquette action and force (Sec. 1), the pseudo-fermion force contraction
// (Sec. 2), momentum and link updates of the molecular dynamics (Sec. 1), algebra layouts.
//
// Forces are defined by (omega, F) = delta_omega S for delta U = omega U.  For any 3x3 G the
// antihermitian traceless projection has coordinates f_a = -2 Re Tr(T_a G) = Im Tr(lambda_a G)
// on T_a = i lambda_a / 2, which is what ta_coords() evaluates without forming the projection.
#include "internal.h"
#include "stencil.h"

namespace whmc {

// ------------------------------------------------------------------ SU(3) helpers
template <typename R> WHMC_DEV void matmul(const SU3<R>& A, const SU3<R>& B, SU3<R>& C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<R> s = cmul(A.e[i][0], B.e[0][j]);
      s = s + cmul(A.e[i][1], B.e[1][j]);
      s = s + cmul(A.e[i][2], B.e[2][j]);
      C.e[i][j] = s;
    }
}
// C = A B^dag
template <typename R> WHMC_DEV void matmul_nd(const SU3<R>& A, const SU3<R>& B, SU3<R>& C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<R> s = cmul(A.e[i][0], conj(B.e[j][0]));
      s = s + cmul(A.e[i][1], conj(B.e[j][1]));
      s = s + cmul(A.e[i][2], conj(B.e[j][2]));
      C.e[i][j] = s;
    }
}
// C = A^dag B
template <typename R> WHMC_DEV void matmul_dn(const SU3<R>& A, const SU3<R>& B, SU3<R>& C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<R> s = cjmul(A.e[0][i], B.e[0][j]);
      s = s + cjmul(A.e[1][i], B.e[1][j]);
      s = s + cjmul(A.e[2][i], B.e[2][j]);
      C.e[i][j] = s;
    }
}

WHMC_DEV void ta_coords(const SU3<double>& G, double* f) {
  const double inv_sqrt3 = 0.57735026918962576451;
  f[0] = G.e[0][1].im + G.e[1][0].im;
  f[1] = G.e[0][1].re - G.e[1][0].re;
  f[2] = G.e[0][0].im - G.e[1][1].im;
  f[3] = G.e[0][2].im + G.e[2][0].im;
  f[4] = G.e[0][2].re - G.e[2][0].re;
  f[5] = G.e[1][2].im + G.e[2][1].im;
  f[6] = G.e[1][2].re - G.e[2][1].re;
  f[7] = (G.e[0][0].im + G.e[1][1].im - 2.0 * G.e[2][2].im) * inv_sqrt3;
}

// A = sum_a c_a T_a, T_a = i lambda_a / 2
WHMC_DEV void from_coords(const double* a, SU3<double>& A) {
  const double inv_sqrt3 = 0.57735026918962576451;
  A.e[0][1] = {0.5 * a[1], 0.5 * a[0]};
  A.e[1][0] = {-0.5 * a[1], 0.5 * a[0]};
  A.e[0][2] = {0.5 * a[4], 0.5 * a[3]};
  A.e[2][0] = {-0.5 * a[4], 0.5 * a[3]};
  A.e[1][2] = {0.5 * a[6], 0.5 * a[5]};
  A.e[2][1] = {-0.5 * a[6], 0.5 * a[5]};
  A.e[0][0] = {0.0, 0.5 * (a[2] + a[7] * inv_sqrt3)};
  A.e[1][1] = {0.0, 0.5 * (-a[2] + a[7] * inv_sqrt3)};
  A.e[2][2] = {0.0, -a[7] * inv_sqrt3};
}

// exp(A) for a 3x3 matrix by scaling and squaring: Taylor series of degree 12 on A / 2^s with
// |A / 2^s|_inf <= 1/4 (truncation below 3e-18 relative), then s squarings.
WHMC_DEV void expm3(const SU3<double>& A, SU3<double>& E) {
  double nrm = 0.0;
  for (int i = 0; i < 3; ++i) {
    double r = 0.0;
    for (int j = 0; j < 3; ++j) r += sqrt(norm2(A.e[i][j]));
    nrm = fmax(nrm, r);
  }
  int s = 0;
  while (nrm > 0.25 && s < 60) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
  SU3<double> B;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B.e[i][j] = sc * A.e[i][j];
  // Horner: E = I + B (1 + B/2 (1 + B/3 (... (1 + B/12))))
  SU3<double> P, T;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P.e[i][j] = {i == j ? 1.0 : 0.0, 0.0};
  for (int k = 12; k >= 1; --k) {
    matmul(B, P, T);
    const double inv = 1.0 / k;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P.e[i][j] = {(i == j ? 1.0 : 0.0) + inv * T.e[i][j].re, inv * T.e[i][j].im};
  }
  for (int k = 0; k < s; ++k) {
    matmul(P, P, T);
    P = T;
  }
  E = P;
}

// ------------------------------------------------------------------ site helpers (full lattice)
struct Site {
  int par, cb;
};

// coordinates within one step of the lattice, -1 .. L, wrapped periodically (compares, no division)
WHMC_DEV int wrap1(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

WHMC_DEV Site site_at(const Geom& g, int t, int z, int y, int x) {
  t = wrap1(t, g.L[0]);
  z = wrap1(z, g.L[1]);
  y = wrap1(y, g.L[2]);
  x = wrap1(x, g.L[3]);
  const int lex = ((t * g.L[1] + z) * g.L[2] + y) * g.L[3] + x;
  return {(t + z + y + x) & 1, lex >> 1};
}

WHMC_DEV Site shift(const Geom& g, const Coords& c, int mu, int d, int nu = 0, int e = 0) {
  int p[4] = {c.t, c.z, c.y, c.x};
  p[mu] += d;
  p[nu] += e;
  return site_at(g, p[0], p[1], p[2], p[3]);
}

WHMC_DEV void load_link(const double2* U18, int Vh, Site s, int mu, SU3<double>& U) {
  LinkF64_18{U18, Vh}.load(s.par, mu, s.cb, U);
}
// Link-parallel grid over both parities and the 4 directions (gauge force): the 8 (parity, mu)
// workgroups of a block of sites run back to back on one XCD (site_block_grp with 8 groups), so the
// neighbour links they share are read from HBM once and then from its L2.  Measured at 32^3 x 64:
// 2.8 -> 1.3 ms against parity and mu on grid.z / grid.y.
WHMC_DEV int link_site(const Geom& g, int& par, int& mu) {
  int grp, slot;
  const int sb = site_block_grp(g, blockIdx.x, gridDim.x, 8, grp, slot);
  par = grp >> 2;
  mu = grp & 3;
  return sb * kBlock + threadIdx.x;
}

// ------------------------------------------------------------------ plaquette
__global__ __launch_bounds__(kBlock) void k_plaquette(Geom g, const double2* __restrict__ U18, Reduce red,
                                                      double* out) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;   // over both parities
  double s = 0.0;
  if (idx < 2 * g.Vh) {
    const int par = idx >= g.Vh, i = idx - par * g.Vh;
    const Coords c = coords_of(g, i, par);
    const Site x{par, i};
    for (int mu = 1; mu < 4; ++mu)
      for (int nu = 0; nu < mu; ++nu) {
        SU3<double> a, b, cc, d, t1, t2;
        load_link(U18, g.Vh, x, mu, a);
        load_link(U18, g.Vh, shift(g, c, mu, 1), nu, b);
        load_link(U18, g.Vh, shift(g, c, nu, 1), mu, cc);
        load_link(U18, g.Vh, x, nu, d);
        matmul(a, b, t1);        // U_mu(x) U_nu(x+mu)
        matmul_nd(t1, cc, t2);   // ... U_mu(x+nu)^dag
        // Re Tr(t2 d^dag)
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) s += t2.e[k][l].re * d.e[k][l].re + t2.e[k][l].im * d.e[k][l].im;
      }
  }
  block_partial<kBlock>(s, red.partials, blockIdx.x);
}

whmc_status plaquette_sum(whmc_ctx* c, double* host_out) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const int nb = (2 * c->Vh + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_plaquette, dim3(nb), dim3(kBlock), 0, c->stream, c->g, c->U18, c->red, c->red.result);
  WHMC_HIP(hipGetLastError());
  WHMC_TRY(finish_sum(c, nb, c->red.result));
  return read_scalar(c, c->red.result, host_out);
}

// ------------------------------------------------------------------ gauge force
// F_{x,mu} = (beta/6) P_TA(U_{x,mu} Sigma_{x,mu}), Sigma = sum of the six staples.
// out = (accumulate ? out : 0) + scale * F, one thread per link.
__global__ __launch_bounds__(kBlock) void k_gauge_force(Geom g, const double2* __restrict__ U18, double* F,
                                                        double coef, int accumulate) {
  int par, mu;
  const int i = link_site(g, par, mu);
  if (i >= g.Vh) return;
  const Coords c = coords_of(g, i, par);
  SU3<double> S, a, b, d, t1, t2;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) S.e[p][q] = {0.0, 0.0};
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    // up: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    load_link(U18, g.Vh, shift(g, c, mu, 1), nu, a);
    load_link(U18, g.Vh, shift(g, c, nu, 1), mu, b);
    load_link(U18, g.Vh, Site{par, i}, nu, d);
    matmul_nd(a, b, t1);
    matmul_nd(t1, d, t2);
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) S.e[p][q] = S.e[p][q] + t2.e[p][q];
    // down: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
    load_link(U18, g.Vh, shift(g, c, mu, 1, nu, -1), nu, a);
    load_link(U18, g.Vh, shift(g, c, nu, -1), mu, b);
    load_link(U18, g.Vh, shift(g, c, nu, -1), nu, d);
    {
      SU3<double> ad;   // a^dag, then t1 = a^dag b^dag
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) ad.e[p][q] = conj(a.e[q][p]);
      matmul_nd(ad, b, t1);
    }
    matmul(t1, d, t2);
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) S.e[p][q] = S.e[p][q] + t2.e[p][q];
  }
  load_link(U18, g.Vh, Site{par, i}, mu, a);
  matmul(a, S, t1);
  double f[8];
  ta_coords(t1, f);
  double* out = F + ((size_t)(par * 4 + mu) * 8) * g.Vh + i;
  for (int k = 0; k < 8; ++k) {
    const double v = coef * f[k];
    out[(size_t)k * g.Vh] = accumulate ? out[(size_t)k * g.Vh] + v : v;
  }
}

whmc_status gauge_force(whmc_ctx* c, double* F, double beta_eff, double scale, int accumulate) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const dim3 grid(8 * c->stencil_blocks());
  hipLaunchKernelGGL(k_gauge_force, grid, dim3(kBlock), 0, c->stream, c->g, c->U18, F, scale * beta_eff / 6.0,
                     accumulate);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

// ------------------------------------------------------------------ pseudo-fermion force
// For full-lattice pairs (X, Y), with s = -1 on links that wrap in time:
//   G_{x,mu} = s [ U_{x,mu} Q - R U_{x,mu}^dag ],
//   Q_{ca} = sum_s [(1 - g_mu) Y(x+mu)]_{sc} conj(X(x)_{sa})   = sum over 2 projected spins
//   R_{ca} = sum_s [(1 + g_mu) Y(x)]_{sc} conj(X(x+mu)_{sa})
// and F = -kappa_eff P_TA(sum_pairs G).  The projected forms follow from (1 -/+ g) = [h; -/+ A^dag h].
struct PairPtrs {
  const double2* Xe[24];
  const double2* Xo[24];
  const double2* Ye[24];
  const double2* Yo[24];
};

template <int MU>
WHMC_DEV void force_link(const Geom& g, int par, int i, const double2* U18, const PairPtrs& P, int npairs,
                         double kappa_eff, double* F, int accumulate) {
  const Coords c = coords_of(g, i, par);
  bool wrap;
  const int j = neighbour<MU, +1>(g, c, wrap);
  SU3<double> Qs, Rs;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) Qs.e[p][q] = Rs.e[p][q] = {0.0, 0.0};
  for (int k = 0; k < npairs; ++k) {
    const double2* Xh = par ? P.Xo[k] : P.Xe[k];
    const double2* Yh = par ? P.Yo[k] : P.Ye[k];
    const double2* Xn = par ? P.Xe[k] : P.Xo[k];
    const double2* Yn = par ? P.Ye[k] : P.Yo[k];
    Spinor<double> X, Y, Xf, Yf;
    SpinorF64{(double2*)Xh, g.Vh}.load(i, X);
    SpinorF64{(double2*)Yh, g.Vh}.load(i, Y);
    SpinorF64{(double2*)Xn, g.Vh}.load(j, Xf);
    SpinorF64{(double2*)Yn, g.Vh}.load(j, Yf);
    HalfSpinor<double> hq, gq, hr, gr;
    project<MU, -1>(Yf, hq);
    project<MU, -1>(X, gq);
    project<MU, +1>(Y, hr);
    project<MU, +1>(Xf, gr);
    for (int s = 0; s < 2; ++s)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          Qs.e[a][b] = Qs.e[a][b] + cjmul(gq.c[s][b], hq.c[s][a]);
          Rs.e[a][b] = Rs.e[a][b] + cjmul(gr.c[s][b], hr.c[s][a]);
        }
  }
  SU3<double> U, A, B;
  LinkF64_18{U18, g.Vh}.load(par, MU, i, U);
  matmul(U, Qs, A);
  matmul_nd(Rs, U, B);
  const double sgn = (MU == 0 && wrap) ? -1.0 : 1.0;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) A.e[p][q] = sgn * (A.e[p][q] - B.e[p][q]);
  double f[8];
  ta_coords(A, f);
  double* out = F + ((size_t)(par * 4 + MU) * 8) * g.Vh + i;
  for (int k = 0; k < 8; ++k) {
    const double v = -kappa_eff * f[k];
    out[(size_t)k * g.Vh] = accumulate ? out[(size_t)k * g.Vh] + v : v;
  }
}

// Site-parallel form: one thread per site of either parity (both in one grid, the XCD that handles a
// region does both of its parities) and the four links leaving the site, one after the other, so
// the site's own X, Y of every pair are re-read by the same thread from its L1 instead of by four
// workgroups.  The pairs of a launch (chunks of ctx->force_chunk) are summed per link first.
__global__ __launch_bounds__(kBlock) void k_pf_force_site(Geom g, const double2* __restrict__ U18, PairPtrs P,
                                                          int npairs, double kappa_eff, double* F, int accumulate) {
  int par;
  const int i = site_block_pair(g, blockIdx.x, gridDim.x >> 1, par) * kBlock + threadIdx.x;
  if (i >= g.Vh) return;
  force_link<0>(g, par, i, U18, P, npairs, kappa_eff, F, accumulate);
  force_link<1>(g, par, i, U18, P, npairs, kappa_eff, F, accumulate);
  force_link<2>(g, par, i, U18, P, npairs, kappa_eff, F, accumulate);
  force_link<3>(g, par, i, U18, P, npairs, kappa_eff, F, accumulate);
}

// Link-parallel form in lockstep.  One workgroup of 512 threads holds the eight (parity, mu) link
// threads of 64 sites, one wavefront each, and all of them step through the pairs together (a barrier
// per pair).  The four directions of a parity share the local X, Y of a pair through LDS, each loading
// three of the twelve components, and the other parity's wavefronts read as their own sites what these
// read as x / y neighbours, all while the data is in L2.  When the eight workgroups of a site block ran
// independently, each looping over all pairs, they drifted a pair or two apart, and L2 could not hold
// a whole pair's data in between.  One such workgroup fills a compute unit (two waves per SIMD), and
// the blocks of a slice range run side by side on one XCD (site_block_grp, two halves of a 128-site
// block per workgroup pair), so the z neighbours are fetched by concurrent workgroups too.
//
// FP64 spinor of site i in the 64-site block layout, addressed as a uniform base pointer (a pair's
// field) plus a 32-bit byte offset per lane (measured 10 % faster than 64-bit offsets): a half field
// is 192 Vh bytes, and pf_force_pairs launches this kernel only where that is below 4 GiB.  The 12
// components of a site are w = 64 (or Vh % 64 in the last partial block) entries apart.
WHMC_DEV unsigned spinor_offset(int Vh, int i, unsigned& w16) {
  const int blk = i >> 6;
  w16 = (blk < (Vh >> 6) ? 64u : (unsigned)(Vh & 63)) * 16u;
  return ((unsigned)blk * 64u * 12u + (unsigned)(i & 63)) * 16u;
}
WHMC_DEV void load_spinor_at(const double2* base, unsigned off, unsigned w16, Spinor<double>& s) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 v = *(const double2*)((const char*)base + (off + (unsigned)k * w16));
    s.c[k / 3][k % 3] = {v.x, v.y};
  }
}

// F_{x,mu} (+)= -kappa_eff P_TA(s [U Q - R U^dag])
template <int MU>
WHMC_DEV void finish_link(const Geom& g, int par, int i, bool wrap, const double2* U18, const SU3<double>& Qs,
                          const SU3<double>& Rs, double kappa_eff, double* F, int accumulate) {
  SU3<double> U, A, B;
  LinkF64_18{U18, g.Vh}.load(par, MU, i, U);
  matmul(U, Qs, A);
  matmul_nd(Rs, U, B);
  const double sgn = (MU == 0 && wrap) ? -1.0 : 1.0;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) A.e[p][q] = sgn * (A.e[p][q] - B.e[p][q]);
  double f[8];
  ta_coords(A, f);
  double* out = F + ((size_t)(par * 4 + MU) * 8) * g.Vh + i;
  for (int k = 0; k < 8; ++k) {
    const double v = -kappa_eff * f[k];
    out[(size_t)k * g.Vh] = accumulate ? out[(size_t)k * g.Vh] + v : v;
  }
}

// Q += sum_s [(1 - g_mu) Yn]_s conj([(1 - g_mu) X]_s), R += sum_s [(1 + g_mu) Y]_s conj([(1 + g_mu) Xn]_s)
// for one pair: X, Y at the link's site (from LDS), Xn, Yn at its forward neighbour (in registers)
template <int MU>
WHMC_DEV void pair_step_lds(const double2 (*L)[12][64], int lane, const Spinor<double>& sXn,
                            const Spinor<double>& sYn, SU3<double>& Qs, SU3<double>& Rs) {
  {
    HalfSpinor<double> h, q;
    {
      Spinor<double> s;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const double2 v = L[0][k][lane];
        s.c[k / 3][k % 3] = {v.x, v.y};
      }
      project<MU, -1>(s, q);
    }
    project<MU, -1>(sYn, h);
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) Qs.e[a][bb] = Qs.e[a][bb] + cjmul(q.c[c][bb], h.c[c][a]);
  }
  {
    HalfSpinor<double> h, q;
    {
      Spinor<double> s;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const double2 v = L[1][k][lane];
        s.c[k / 3][k % 3] = {v.x, v.y};
      }
      project<MU, +1>(s, h);
    }
    project<MU, +1>(sXn, q);
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) Rs.e[a][bb] = Rs.e[a][bb] + cjmul(q.c[c][bb], h.c[c][a]);
  }
}

constexpr int kForceWG = 512;

__global__ __launch_bounds__(kForceWG) void k_pf_force(Geom g, const double2* __restrict__ U18, PairPtrs P,
                                                       int npairs, double kappa_eff, double* F, int accumulate) {
  int half, slot;
  const int sb = site_block_grp(g, blockIdx.x, gridDim.x, 2, half, slot);
  const int base = sb * kBlock + half * 64;
  if (base >= g.Vh) return;   // the whole workgroup: no barrier is left waiting
  const int par = threadIdx.x >> 8, mu = (threadIdx.x >> 6) & 3;
  const int i = base + (threadIdx.x & 63);
  const bool live = i < g.Vh;   // lanes past the last site of a partial block still meet every barrier
  const int ii = live ? i : base;
  const Coords c = coords_of(g, ii, par);
  bool wrap = false;
  int j;
  switch (mu) {
    case 0: j = neighbour<0, +1>(g, c, wrap); break;
    case 1: j = neighbour<1, +1>(g, c, wrap); break;
    case 2: j = neighbour<2, +1>(g, c, wrap); break;
    default: j = neighbour<3, +1>(g, c, wrap); break;
  }
  unsigned wi, wj;
  const unsigned oi = spinor_offset(g.Vh, ii, wi), oj = spinor_offset(g.Vh, j, wj);
  SU3<double> Qs, Rs;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) Qs.e[p][q] = Rs.e[p][q] = {0.0, 0.0};
  // local X, Y of a pair: each of the four direction wavefronts of a parity loads three of the twelve
  // components of both and writes them to LDS (two buffers, alternating per pair)
  __shared__ double2 lds[2][2][2][12][64];   // [buffer][parity][X / Y][component][lane]
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int k = 0; k < npairs; ++k) {
    const double2* Xh = par ? P.Xo[k] : P.Xe[k];
    const double2* Yh = par ? P.Yo[k] : P.Ye[k];
    const double2* Xn = par ? P.Xe[k] : P.Xo[k];
    const double2* Yn = par ? P.Ye[k] : P.Yo[k];
    const int b = k & 1;
    if (live) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const unsigned kc = (unsigned)(3 * mu + q);
        lds[b][par][0][3 * mu + q][lane] = *(const double2*)((const char*)Xh + (oi + kc * wi));
        lds[b][par][1][3 * mu + q][lane] = *(const double2*)((const char*)Yh + (oi + kc * wi));
      }
    }
    Spinor<double> sXn, sYn;
    if (live) {
      load_spinor_at(Xn, oj, wj, sXn);
      load_spinor_at(Yn, oj, wj, sYn);
    }
    __syncthreads();
    if (live) {
      switch (mu) {
        case 0: pair_step_lds<0>(lds[b][par], lane, sXn, sYn, Qs, Rs); break;
        case 1: pair_step_lds<1>(lds[b][par], lane, sXn, sYn, Qs, Rs); break;
        case 2: pair_step_lds<2>(lds[b][par], lane, sXn, sYn, Qs, Rs); break;
        default: pair_step_lds<3>(lds[b][par], lane, sXn, sYn, Qs, Rs); break;
      }
    }
  }
  if (!live) return;
  switch (mu) {
    case 0: finish_link<0>(g, par, i, wrap, U18, Qs, Rs, kappa_eff, F, accumulate); break;
    case 1: finish_link<1>(g, par, i, wrap, U18, Qs, Rs, kappa_eff, F, accumulate); break;
    case 2: finish_link<2>(g, par, i, wrap, U18, Qs, Rs, kappa_eff, F, accumulate); break;
    default: finish_link<3>(g, par, i, wrap, U18, Qs, Rs, kappa_eff, F, accumulate); break;
  }
}

whmc_status pf_force_pairs(whmc_ctx* c, double* F, const double* const* X_e, const double* const* X_o,
                           const double* const* Y_e, const double* const* Y_o, int npairs, double kappa_eff,
                           int accumulate) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  const int chunk = c->force_chunk >= 1 && c->force_chunk <= 24 ? c->force_chunk : 24;
  int done = 0;
  while (done < npairs) {
    const int n = npairs - done < chunk ? npairs - done : chunk;
    PairPtrs P{};
    for (int k = 0; k < n; ++k) {
      P.Xe[k] = (const double2*)X_e[done + k];
      P.Xo[k] = (const double2*)X_o[done + k];
      P.Ye[k] = (const double2*)Y_e[done + k];
      P.Yo[k] = (const double2*)Y_o[done + k];
    }
    const int acc = (accumulate || done > 0) ? 1 : 0;
    // the lockstep kernel's 32-bit byte offsets cover half fields up to 4 GiB (Vh up to 2^32 / 192)
    const bool narrow = (unsigned long long)c->g.Vh * 192ull <= 0xFFFFFFFFull;
    if (c->force_kernel == 1 || !narrow)
      hipLaunchKernelGGL(k_pf_force_site, dim3(2 * c->stencil_blocks()), dim3(kBlock), 0, c->stream, c->g, c->U18, P,
                         n, kappa_eff, F, acc);
    else
      hipLaunchKernelGGL(k_pf_force, dim3(2 * c->stencil_blocks()), dim3(kForceWG), 0, c->stream, c->g, c->U18, P,
                         n, kappa_eff, F, acc);
    WHMC_HIP(hipGetLastError());
    done += n;
  }
  return WHMC_OK;
}

// ------------------------------------------------------------------ molecular dynamics updates
__global__ void k_mom_update(long long n, double* pi, const double* F, double eps) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pi[i] -= eps * F[i];
}

whmc_status mom_update(whmc_ctx* c, double* pi, const double* F, double eps) {
  const long long n = 64LL * c->Vh;
  hipLaunchKernelGGL(k_mom_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, pi, F, eps);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

// U_{x,mu} <- exp(eps Pi_{x,mu}) U_{x,mu}, one thread per link
__global__ __launch_bounds__(kBlock) void k_link_update(int Vh, double2* U18, const double* pi, double eps) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int pm = blockIdx.y;   // parity * 4 + mu
  if (i >= Vh) return;
  double a[8];
  for (int k = 0; k < 8; ++k) a[k] = eps * pi[((size_t)pm * 8 + k) * Vh + i];
  SU3<double> A, E, U, N;
  from_coords(a, A);
  expm3(A, E);
  double2* q = U18 + (size_t)pm * 9 * Vh;
  for (int k = 0; k < 9; ++k) {
    double2 v = q[aos(k, i, 9, Vh)];
    U.e[k / 3][k % 3] = {v.x, v.y};
  }
  matmul(E, U, N);
  for (int k = 0; k < 9; ++k) q[aos(k, i, 9, Vh)] = make_double2(N.e[k / 3][k % 3].re, N.e[k / 3][k % 3].im);
}

whmc_status link_update(whmc_ctx* c, const double* pi, double eps) {
  WHMC_CHECK(c->gauge_loaded, WHMC_ESTATE, "no gauge field loaded");
  hipLaunchKernelGGL(k_link_update, dim3(c->num_blocks(), 8), dim3(kBlock), 0, c->stream, c->Vh, c->U18, pi, eps);
  WHMC_HIP(hipGetLastError());
  return gauge_changed(c);
}

__global__ __launch_bounds__(kBlock) void k_sumsq(long long n, const double* x, Reduce red, double* out) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    s += x[i] * x[i];
  block_partial<kBlock>(s, red.partials, blockIdx.x);
}

whmc_status algebra_norm2(whmc_ctx* c, const double* pi, double* host_out) {
  const long long n = 64LL * c->Vh;
  long long nb = (n + kBlock - 1) / kBlock;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_sumsq, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, n, pi, c->red, c->red.result + 1);
  WHMC_HIP(hipGetLastError());
  WHMC_TRY(finish_sum(c, (int)nb, c->red.result + 1));
  return read_scalar(c, c->red.result + 1, host_out);
}

// canonical [V][4][8] <-> [2][4][8][Vh]
__global__ void k_pack_algebra(Geom g, double* dst, const double* src, int unpack) {
  const long long lex = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= 2LL * g.Vh) return;
  int x = (int)(lex % g.L[3]);
  long long r = lex / g.L[3];
  int y = (int)(r % g.L[2]);
  r /= g.L[2];
  int z = (int)(r % g.L[1]);
  int t = (int)(r / g.L[1]);
  const int par = (t + z + y + x) & 1, cb = (int)(lex >> 1);
  for (int mu = 0; mu < 4; ++mu)
    for (int a = 0; a < 8; ++a) {
      const size_t ci = ((size_t)lex * 4 + mu) * 8 + a;
      const size_t si = ((size_t)(par * 4 + mu) * 8 + a) * g.Vh + cb;
      if (unpack) dst[ci] = src[si];
      else dst[si] = src[ci];
    }
}

whmc_status pack_algebra(whmc_ctx* c, double* dst, const double* src, int unpack) {
  const long long V = c->V;
  hipLaunchKernelGGL(k_pack_algebra, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, c->stream, c->g, dst, src,
                     unpack);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

// Transpose of the differential of the exponential map, for S(exp(omega) U0): with
// d/dt exp(omega + t eta) = [sum_k ad_omega^k(eta) / (k+1)!] exp(omega) and ad_omega antisymmetric
// for (A,B) = -2 Re Tr(AB), the gradient in eta is  sum_k (-ad_omega)^k F / (k+1)!.
__global__ __launch_bounds__(kBlock) void k_dexp_t(int Vh, const double* omega, const double* F, double* out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int pm = blockIdx.y;
  if (i >= Vh) return;
  double a[8], f[8];
  for (int k = 0; k < 8; ++k) {
    a[k] = omega[((size_t)pm * 8 + k) * Vh + i];
    f[k] = F[((size_t)pm * 8 + k) * Vh + i];
  }
  SU3<double> W, T, R, A, B;
  from_coords(a, W);
  from_coords(f, T);
  R = T;
  for (int k = 1; k <= 30; ++k) {
    matmul(W, T, A);
    matmul(T, W, B);
    const double s = -1.0 / (k + 1);
    double mx = 0.0;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        T.e[p][q] = s * (A.e[p][q] - B.e[p][q]);
        R.e[p][q] = R.e[p][q] + T.e[p][q];
        mx = fmax(mx, fmax(fabs(T.e[p][q].re), fabs(T.e[p][q].im)));
      }
    if (mx < 1e-18) break;
  }
  double g[8];
  ta_coords(R, g);
  // ta_coords returns Im Tr(lambda_a R) = coordinates of the (already antihermitian) R
  for (int k = 0; k < 8; ++k) out[((size_t)pm * 8 + k) * Vh + i] = g[k];
}

}  // namespace whmc

extern "C" whmc_status whmc_update_links(whmc_ctx* c, const double* pi, double eps) {
  WHMC_CHECK(c && pi, WHMC_EARG, "whmc_update_links: null argument");
  return whmc::link_update(c, pi, eps);
}

extern "C" whmc_status whmc_update_momenta(whmc_ctx* c, double* pi, const double* F, double eps) {
  WHMC_CHECK(c && pi && F && pi != F, WHMC_EARG, "whmc_update_momenta: bad argument");
  return whmc::mom_update(c, pi, F, eps);
}

extern "C" whmc_status whmc_dexp_transpose(whmc_ctx* c, double* out, const double* omega, const double* F) {
  WHMC_CHECK(c && out && omega && F, WHMC_EARG, "whmc_dexp_transpose: null argument");
  WHMC_CHECK(out != omega && out != F, WHMC_EARG, "whmc_dexp_transpose: out must not alias the inputs");
  hipLaunchKernelGGL(whmc::k_dexp_t, dim3(c->num_blocks(), 8), dim3(whmc::kBlock), 0, c->stream, c->Vh, omega, F,
                     out);
  WHMC_HIP(hipGetLastError());
  return WHMC_OK;
}

extern "C" whmc_status whmc_plaquette(whmc_ctx* c, double* plaq) {
  WHMC_CHECK(c && plaq, WHMC_EARG, "whmc_plaquette: null argument");
  double s = 0.0;
  WHMC_TRY(whmc::plaquette_sum(c, &s));
  *plaq = s / (3.0 * 6.0 * (double)c->V);
  return WHMC_OK;
}
