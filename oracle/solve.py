"""Conjugate gradient for the oracle (test infrastructure only).

Sec. 1 names CG (and BiCGstab) as the iterative solvers for the pseudo-fermion systems; this is
the textbook Hestenes-Stiefel CG for a hermitian positive definite operator A, started at
x0 = 0 and stopped when the *true* residual |b - A x| / |b| is at or below tol.
"""
import numpy as np


def vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def norm2(a):
    return float(np.vdot(a.reshape(-1), a.reshape(-1)).real)


def cg(apply_A, b, tol=1e-12, maxiter=10000):
    """solve A x = b; returns (x, iterations, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = norm2(r)
    bb = norm2(b)
    if bb == 0.0:
        return x, 0, 0.0
    it = 0
    while it < maxiter:
        if rr <= tol * tol * bb:
            true_r = np.sqrt(norm2(b - apply_A(x)) / bb)
            if true_r <= tol:
                return x, it, true_r
            r = b - apply_A(x)          # restart from the true residual
            rr = norm2(r)
            p = r.copy()
        Ap = apply_A(p)
        alpha = rr / vdot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = norm2(r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    true_r = np.sqrt(norm2(b - apply_A(x)) / bb)
    return x, it, true_r
