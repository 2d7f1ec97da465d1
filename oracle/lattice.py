"""Lattice geometry for the oracle (test infrastructure only).

Site order, parity and boundary conditions follow the conventions in ``oracle/__init__``:
lexicographic (t, z, y, x), parity (t+z+y+x) mod 2, checkerboard index lex // 2, gauge field
periodic, fermion field anti-periodic in time (Sec. 4).
"""
import numpy as np


class Lattice:
    def __init__(self, dims):
        dims = tuple(int(d) for d in dims)
        if len(dims) != 4 or min(dims) < 1:
            raise ValueError("dims must be four positive extents (L_t, L_z, L_y, L_x)")
        self.dims = dims
        self.V = int(np.prod(dims))
        grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
        self.coords = grids                          # t, z, y, x arrays of shape dims
        self.parity = (grids[0] + grids[1] + grids[2] + grids[3]) % 2
        self.lex = np.arange(self.V).reshape(dims)

    # ---------------------------------------------------------------- even / odd
    @property
    def Vh(self):
        if self.V % 2 or self.dims[3] % 2:
            raise ValueError("even/odd ordering needs an even L_x")
        return self.V // 2

    def sites_of_parity(self, p):
        """lex indices of all sites of parity p, in increasing order (= checkerboard order)."""
        return np.flatnonzero(self.parity.reshape(-1) == p)

    def to_half(self, full, p):
        """full field (dims..., *inner) -> half-lattice field (Vh, *inner) of parity p."""
        flat = full.reshape((self.V,) + full.shape[4:])
        return flat[self.sites_of_parity(p)].copy()

    def to_full(self, half, p):
        """half-lattice field of parity p -> full field, zero on the other parity."""
        out = np.zeros((self.V,) + half.shape[1:], dtype=half.dtype)
        out[self.sites_of_parity(p)] = half
        return out.reshape(self.dims + half.shape[1:])

    # ---------------------------------------------------------------- shifts
    def fwd(self, field, mu, fermion=True):
        """field(x + mu_hat); for fermions a hop across the time boundary carries -1."""
        out = np.roll(field, -1, axis=mu)
        if fermion and mu == 0:
            out[self.dims[0] - 1] *= -1.0
        return out

    def bwd(self, field, mu, fermion=True):
        """field(x - mu_hat); for fermions a hop across the time boundary carries -1."""
        out = np.roll(field, 1, axis=mu)
        if fermion and mu == 0:
            out[0] *= -1.0
        return out

    # ---------------------------------------------------------------- per-site helpers
    def coord_of(self, lex):
        lex = np.asarray(lex)
        t, r = np.divmod(lex, self.dims[1] * self.dims[2] * self.dims[3])
        z, r = np.divmod(r, self.dims[2] * self.dims[3])
        y, x = np.divmod(r, self.dims[3])
        return t, z, y, x

    def lex_of(self, t, z, y, x):
        T, Z, Y, X = self.dims
        return ((np.asarray(t) % T * Z + np.asarray(z) % Z) * Y + np.asarray(y) % Y) * X + np.asarray(x) % X

    def neighbour(self, lex, mu, step):
        """lex index of x + step*mu_hat (periodic) and the fermion sign of that hop."""
        c = list(self.coord_of(lex))
        c[mu] = c[mu] + step
        sign = np.ones(np.shape(lex))
        if mu == 0:
            crossed = (c[0] < 0) | (c[0] >= self.dims[0])
            sign = np.where(crossed, -1.0, 1.0)
        return self.lex_of(*c), sign
