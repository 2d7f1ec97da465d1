// The Wilson hopping stencil on one site (Sec. 1, definition of H):
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_{x,mu} psi(x+mu) + (1 + gamma_mu) U^dag_{x-mu,mu} psi(x-mu)
// and its adjoint H^dag = gamma_5 H gamma_5, which swaps the two projectors.  Each neighbour
// spinor is first projected to a two-spin half spinor, multiplied by the link, and the lower two
// spin components are rebuilt from the upper two.  Fermion hops across the time boundary carry
// a factor -1 (Sec. 4); the stored links never contain that sign.
//
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_0 = 1, A_k = -i sigma_k (k = 1,2,3),
// so (1 + s gamma_mu) psi = [h ; s A^dag h] with h = psi_up + s A psi_down.
#pragma once
#include "device.h"

namespace whmc {

// h = psi_up + SGN * A_mu psi_down
template <int MU, int SGN, typename R>
WHMC_DEV void project(const Spinor<R>& s, HalfSpinor<R>& h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<R> a0, a1;
    if (MU == 0) { a0 = s.c[2][c]; a1 = s.c[3][c]; }
    if (MU == 1) { a0 = times_mi(s.c[3][c]); a1 = times_mi(s.c[2][c]); }
    if (MU == 2) { a0 = -s.c[3][c]; a1 = s.c[2][c]; }
    if (MU == 3) { a0 = times_mi(s.c[2][c]); a1 = times_i(s.c[3][c]); }
    if (SGN > 0) { h.c[0][c] = s.c[0][c] + a0; h.c[1][c] = s.c[1][c] + a1; }
    else         { h.c[0][c] = s.c[0][c] - a0; h.c[1][c] = s.c[1][c] - a1; }
  }
}

// acc += [u ; SGN * A_mu^dag u]
template <int MU, int SGN, typename R>
WHMC_DEV void accumulate(Spinor<R>& acc, const HalfSpinor<R>& u) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc.c[0][c] = acc.c[0][c] + u.c[0][c];
    acc.c[1][c] = acc.c[1][c] + u.c[1][c];
    cplx<R> b0, b1;
    if (MU == 0) { b0 = u.c[0][c]; b1 = u.c[1][c]; }
    if (MU == 1) { b0 = times_i(u.c[1][c]); b1 = times_i(u.c[0][c]); }
    if (MU == 2) { b0 = u.c[1][c]; b1 = -u.c[0][c]; }
    if (MU == 3) { b0 = times_i(u.c[0][c]); b1 = times_mi(u.c[1][c]); }
    if (SGN > 0) { acc.c[2][c] = acc.c[2][c] + b0; acc.c[3][c] = acc.c[3][c] + b1; }
    else         { acc.c[2][c] = acc.c[2][c] - b0; acc.c[3][c] = acc.c[3][c] - b1; }
  }
}

template <typename R> WHMC_DEV void negate(HalfSpinor<R>& h) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) h.c[s][c] = -h.c[s][c];
}

// contribution of direction MU (forward and backward) to the output site
template <int MU, int DAG, class Lnk, class SIn, typename R>
WHMC_DEV void hop_dir(const Geom& g, const Coords& c, int par, int i, const Lnk& L, const SIn& in,
                      Spinor<R>& acc) {
  constexpr int SF = DAG ? +1 : -1;  // forward hop projector sign
  constexpr int SB = -SF;
  bool wrap;
  Spinor<R> s;
  HalfSpinor<R> h, u;
  SU3<R> U;
  {
    const int j = neighbour<MU, +1>(g, c, wrap);
    in.load(j, s);
    L.load(par, MU, i, U);
    project<MU, SF>(s, h);
    if (MU == 0 && wrap) negate(h);
    mul(U, h.c[0], u.c[0]);
    mul(U, h.c[1], u.c[1]);
    accumulate<MU, SF>(acc, u);
  }
  {
    const int j = neighbour<MU, -1>(g, c, wrap);
    in.load(j, s);
    L.load(1 - par, MU, j, U);
    project<MU, SB>(s, h);
    if (MU == 0 && wrap) negate(h);
    mul_dag(U, h.c[0], u.c[0]);
    mul_dag(U, h.c[1], u.c[1]);
    accumulate<MU, SB>(acc, u);
  }
}

// acc = (H psi)(x) (DAG = 0) or (H^dag psi)(x) (DAG = 1) for the site x of parity par, cb i;
// the input field lives on the opposite parity.
template <int DAG, class Lnk, class SIn, typename R>
WHMC_DEV void hop_site(const Geom& g, int par, int i, const Lnk& L, const SIn& in, Spinor<R>& acc) {
  const Coords c = coords_of(g, i, par);
  zero(acc);
  hop_dir<0, DAG>(g, c, par, i, L, in, acc);
  hop_dir<1, DAG>(g, c, par, i, L, in, acc);
  hop_dir<2, DAG>(g, c, par, i, L, in, acc);
  hop_dir<3, DAG>(g, c, par, i, L, in, acc);
}

template <typename R, typename S> WHMC_DEV void scale(Spinor<R>& a, S s) {
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int c = 0; c < 3; ++c) a.c[p][c] = R(s) * a.c[p][c];
}

template <typename R> WHMC_DEV double norm2(const Spinor<R>& a) {
  R s = R(0);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int c = 0; c < 3; ++c) s += a.c[p][c].re * a.c[p][c].re + a.c[p][c].im * a.c[p][c].im;
  return double(s);
}

}  // namespace whmc
