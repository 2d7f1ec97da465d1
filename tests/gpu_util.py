"""Helpers for the GPU parity tests: move oracle-layout numpy arrays through the library's
pack/unpack entry points and compare results."""
import numpy as np
import torch

from paper_1805_03560_amd import whmc


def dev():
    return torch.device("cuda", 0)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def make_ctx(dims, U):
    ctx = whmc.Context(dims)
    ctx.load_gauge(to_dev(U), unitarity_tol=1e-11)
    return ctx


def pack_half(ctx, x):
    """numpy (Vh,4,3) or (n,Vh,4,3) complex128 -> whmc layout FP64 buffer (device)."""
    return ctx.pack_spinor(to_dev(x), 0)


def unpack_half(ctx, buf, n=1):
    return ctx.unpack_spinor(buf, 0, n).cpu().numpy()


def pack_full(ctx, x):
    return ctx.pack_spinor(to_dev(x.reshape(-1, 4, 3)), -1)


def unpack_full(ctx, buf):
    return ctx.unpack_spinor(buf, -1).cpu().numpy().reshape(ctx.dims + (4, 3))


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def algebra_to_numpy(ctx, buf):
    return ctx.unpack_algebra(buf).cpu().numpy()


_ORACLE_CACHE = {}


def oracle_cached(key, compute):
    """compute(), an oracle reference, evaluated once per test session for a hashable key that names
    everything it depends on (the generator, seeds and parameters the test builds its inputs from):
    parametrizations of a test that vary only the GPU side (blocking, kernel variant, format) share
    the reference instead of recomputing it"""
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = compute()
    return _ORACLE_CACHE[key]
