"""Wilson hopping matrix, fermion matrix and even/odd Schur complement (oracle, test only).

Sec. 1 defines
    M = 1 - kappa H,
    H_xy = sum_mu [ (1 - gamma_mu) U_{x,mu} delta_{x+mu,y} + (1 + gamma_mu) U^dag_{x-mu,mu} delta_{x-mu,y} ]
with no factor 1/2 (free critical kappa = 1/8).  Sec. 2.2 defines the even/odd preconditioned
matrix on the odd sites,
    M_oo = 1 - kappa^2 H_oe H_eo ,
and M^dag = gamma_5 M gamma_5 follows from the definition of H.

Fields: U has shape (L_t, L_z, L_y, L_x, 4, 3, 3); a full spinor (L_t, L_z, L_y, L_x, 4, 3);
a half spinor (V/2, 4, 3) in checkerboard order.
"""
import numpy as np

from .gamma import GAMMA5, P_MINUS, P_PLUS


def spin_mul(S, psi):
    """apply a 4x4 spin matrix to every site of a spinor field."""
    return np.einsum("st,...tc->...sc", S, psi)


def colour_mul(U, psi):
    """(U psi)_{s a} = sum_b U_{ab} psi_{s b} site by site."""
    return np.einsum("...ab,...sb->...sa", U, psi)


def colour_mul_dag(U, psi):
    """(U^dag psi)_{s a} = sum_b conj(U_{ba}) psi_{s b}."""
    return np.einsum("...ba,...sb->...sa", U.conj(), psi)


def apply_H(lat, U, psi):
    """(H psi)(x) on the full lattice, straight from the definition of H (Sec. 1)."""
    out = np.zeros_like(psi)
    for mu in range(4):
        out += spin_mul(P_MINUS[mu], colour_mul(U[..., mu, :, :], lat.fwd(psi, mu)))
        U_back = lat.bwd(U[..., mu, :, :], mu, fermion=False)        # U_{x-mu, mu}
        out += spin_mul(P_PLUS[mu], colour_mul_dag(U_back, lat.bwd(psi, mu)))
    return out


def apply_Hdag(lat, U, psi):
    """H^dag = gamma_5 H gamma_5."""
    return spin_mul(GAMMA5, apply_H(lat, U, spin_mul(GAMMA5, psi)))


def apply_M(lat, U, psi, kappa):
    """M psi = psi - kappa H psi (Sec. 1)."""
    return psi - kappa * apply_H(lat, U, psi)


def apply_Mdag(lat, U, psi, kappa):
    return psi - kappa * apply_Hdag(lat, U, psi)


# ---------------------------------------------------------------- even / odd blocks

def apply_Hblock(lat, U, half_in, out_parity, dagger=False):
    """H_{p,1-p} (or its adjoint block) mapping a half field of parity 1-p to parity p.

    H_eo = apply_Hblock(..., out_parity=0); H_oe = apply_Hblock(..., out_parity=1).
    With dagger=True it applies the (p, 1-p) block of H^dag, i.e. (H_{1-p,p})^dag.
    """
    full = lat.to_full(half_in, 1 - out_parity)
    res = apply_Hdag(lat, U, full) if dagger else apply_H(lat, U, full)
    return lat.to_half(res, out_parity)


def apply_K(lat, U, x_odd, kappa):
    """K = kappa^2 H_oe H_eo on odd-site vectors (Sec. 2.2: kappa H is replaced by K)."""
    return kappa ** 2 * apply_Hblock(lat, U, apply_Hblock(lat, U, x_odd, 0), 1)


def apply_Kdag(lat, U, x_odd, kappa):
    """K^dag = kappa^2 H_eo^dag H_oe^dag."""
    return kappa ** 2 * apply_Hblock(lat, U, apply_Hblock(lat, U, x_odd, 0, dagger=True), 1, dagger=True)


def apply_Moo(lat, U, x_odd, kappa):
    """M_oo x = x - kappa^2 H_oe H_eo x (Sec. 2.2)."""
    return x_odd - apply_K(lat, U, x_odd, kappa)


def apply_Moo_dag(lat, U, x_odd, kappa):
    return x_odd - apply_Kdag(lat, U, x_odd, kappa)


def apply_MooDagMoo(lat, U, x_odd, kappa):
    return apply_Moo_dag(lat, U, apply_Moo(lat, U, x_odd, kappa), kappa)


def gamma5_half(x):
    return np.einsum("st,...tc->...sc", GAMMA5, x)


# ---------------------------------------------------------------- dense matrices (tiny lattices)

def dense_H(lat, U):
    """Dense 12V x 12V hopping matrix built entry by entry from the definition (Sec. 1).

    Row/column index = 12*lex + 3*spin + colour.  Independent of ``apply_H``: it walks the
    sites and directions explicitly instead of shifting whole fields.  On a lattice with an
    extent 2 the forward and backward neighbours coincide and both terms add up.
    """
    n = 12 * lat.V
    Hm = np.zeros((n, n), dtype=np.complex128)
    Uf = U.reshape(lat.V, 4, 3, 3)
    for x in range(lat.V):
        for mu in range(4):
            y, s = lat.neighbour(x, mu, +1)
            Hm[12 * x:12 * x + 12, 12 * y:12 * y + 12] += s * np.kron(P_MINUS[mu], Uf[x, mu])
            y, s = lat.neighbour(x, mu, -1)
            Hm[12 * x:12 * x + 12, 12 * y:12 * y + 12] += s * np.kron(P_PLUS[mu], Uf[y, mu].conj().T)
    return Hm


def dense_blocks(lat, Hm):
    """split a dense full-lattice matrix into its (even, odd) blocks in checkerboard order."""
    idx = [(12 * lat.sites_of_parity(p)[:, None] + np.arange(12)[None, :]).reshape(-1) for p in (0, 1)]
    return {
        "ee": Hm[np.ix_(idx[0], idx[0])], "eo": Hm[np.ix_(idx[0], idx[1])],
        "oe": Hm[np.ix_(idx[1], idx[0])], "oo": Hm[np.ix_(idx[1], idx[1])],
    }


# ---------------------------------------------------------------- single sites (large lattices)

def hop_at_sites(lat, U, psi_full, lex_sites, dagger=False):
    """(H psi)(x) (or (H^dag psi)(x)) only at the listed sites, by explicit neighbour gathers.

    Used to check full-size lattices where a whole-field numpy application is too slow.
    U may be any array indexable as U[lex, mu] -> 3x3 (e.g. a (V, 4, 3, 3) view);
    psi_full indexable as psi[lex] -> 4x3.
    """
    lex_sites = np.asarray(lex_sites)
    out = np.zeros((len(lex_sites), 4, 3), dtype=np.complex128)
    pm, pp = (P_PLUS, P_MINUS) if dagger else (P_MINUS, P_PLUS)
    for mu in range(4):
        yf, sf = lat.neighbour(lex_sites, mu, +1)
        v = np.einsum("nab,nsb->nsa", U[lex_sites, mu], psi_full[yf]) * sf[:, None, None]
        out += np.einsum("st,ntc->nsc", pm[mu], v)
        yb, sb = lat.neighbour(lex_sites, mu, -1)
        v = np.einsum("nba,nsb->nsa", U[yb, mu].conj(), psi_full[yb]) * sb[:, None, None]
        out += np.einsum("st,ntc->nsc", pp[mu], v)
    return out
