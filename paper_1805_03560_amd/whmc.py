"""Thin Python binding of libwhmc (the C ABI in include/whmc.h).

Argument marshalling only: every step of the computation runs in the HIP library.  Fields are
torch tensors on the context's GPU (PyTorch supplies device memory and the stream); the library
is called on torch's current stream so that torch and library work stay ordered.

Layouts (see include/whmc.h): canonical complex128 tensors for import/export, and the library's
structure-of-arrays "whmc layout" for everything the hot path touches.  ``half_spinor()`` etc.
allocate correctly sized whmc-layout buffers.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwhmc.so")

F64, F32, F16 = 0, 1, 2
L8, L12, L18 = 8, 12, 18
LEAPFROG, OMELYAN = 0, 1
FORCE_PF, FORCE_GAUGE, FORCE_ACCUMULATE = 1, 2, 4
_STATUS = {0: "OK", 1: "EARG", 2: "EHIP", 3: "ENOCONV", 4: "EUNSUP", 5: "ENOTSU3", 6: "ESTATE", 7: "ENONFINITE"}
OPT_STREAM_THRESHOLD, OPT_HOP_SCHEDULE, OPT_HOP_CHUNK, OPT_FORCE_KERNEL, OPT_FORCE_CHUNK, OPT_HOP_WG_PER_CU = 1, 2, 3, 4, 5, 6
_HALF_BYTES = {F64: 192, F32: 96, F16: 52}
NOALLOC_SCRATCH_BYTES = 32 << 20


class WhmcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"whmc {_STATUS.get(status, status)}: {message}")
        self.status = status


class CGParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("prec", ctypes.c_int),
                ("links", ctypes.c_int), ("delta", ctypes.c_double), ("check_every", ctypes.c_int),
                ("rhs_block", ctypes.c_int), ("rhs_lanes", ctypes.c_int), ("rhs_order", ctypes.c_int)]


class CGStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Filter(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("n_t", ctypes.c_int), ("n_max", ctypes.c_int)]


class HMCParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("kappa", ctypes.c_double), ("filter", Filter),
                ("integrator", ctypes.c_int), ("lam", ctypes.c_double), ("m", ctypes.c_int), ("m0", ctypes.c_int),
                ("tau", ctypes.c_double), ("md_solver", CGParams), ("action_solver", CGParams)]


class TrajResult(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("H0", ctypes.c_double), ("H1", ctypes.c_double),
                ("accepted", ctypes.c_int), ("plaquette", ctypes.c_double), ("cg_iters", ctypes.c_longlong),
                ("n_solves", ctypes.c_int), ("seconds", ctypes.c_double), ("poly_iters", ctypes.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MAX_POLY = 4


class Rooted(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("jmax", ctypes.c_int), ("n", ctypes.c_int * MAX_POLY), ("k", ctypes.c_int),
                ("n_t", ctypes.c_int), ("n_max", ctypes.c_int)]


class RootedHMCParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("kappa", ctypes.c_double), ("rooted", Rooted),
                ("integrator", ctypes.c_int), ("lam", ctypes.c_double), ("m", ctypes.c_int),
                ("msub", ctypes.c_int * (MAX_POLY + 1)), ("tau", ctypes.c_double), ("md_solver", CGParams),
                ("action_solver", CGParams), ("heatbath_solver", CGParams)]


MAX_MASSPRE = 4


class MassPre(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("kappas", ctypes.c_double * MAX_MASSPRE), ("filter", Filter)]


class MassPreHMCParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("kappa", ctypes.c_double), ("mp", MassPre),
                ("integrator", ctypes.c_int), ("lam", ctypes.c_double), ("m", ctypes.c_int),
                ("msub", ctypes.c_int * (MAX_MASSPRE + 1)), ("tau", ctypes.c_double), ("md_solver", CGParams),
                ("action_solver", CGParams)]


def masspre(kappas, k=2, n_t=15, n_max=29):
    """mass preconditioning with heavier hopping parameters kappas (increasing), the kappa^(2k)
    filter on the heaviest factor (Sec. 1, 5)."""
    ks = [float(v) for v in kappas]
    if len(ks) > MAX_MASSPRE:
        raise ValueError(f"at most {MAX_MASSPRE} heavier kappas")
    return MassPre(len(ks), (ctypes.c_double * MAX_MASSPRE)(*(ks + [0.0] * (MAX_MASSPRE - len(ks)))),
                   Filter(k, n_t, n_max))


def rooted(N, ns, k=0, n_t=0, n_max=0):
    """rooted-polynomial action (Sec. 2.1): root order N, degrees ns = (n_1, ..., n_jmax)."""
    ns = [int(v) for v in ns]
    if len(ns) > MAX_POLY:
        raise ValueError(f"at most {MAX_POLY} polynomials")
    return Rooted(int(N), len(ns), (ctypes.c_int * MAX_POLY)(*(ns + [0] * (MAX_POLY - len(ns)))), int(k), int(n_t),
                  int(n_max))


def cg_params(tol=1e-10, maxiter=10000, prec=F64, links=L18, delta=0.1, check_every=8, rhs_block=0, rhs_lanes=0,
              rhs_order=0):
    return CGParams(tol, maxiter, prec, links, delta, check_every, rhs_block, rhs_lanes, rhs_order)


_lib = None
_P = ctypes.c_void_p
_SIGS = {
    "whmc_abi_version": ([], ctypes.c_int),
    "whmc_last_error": ([], ctypes.c_char_p),
    "whmc_create": ([ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int), ctypes.c_int, _P], ctypes.c_int),
    "whmc_destroy": ([_P], None),
    "whmc_set_stream": ([_P, _P], ctypes.c_int),
    "whmc_set_option": ([_P, ctypes.c_int, ctypes.c_longlong], ctypes.c_int),
    "whmc_get_option": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
    "whmc_autotune_hop": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "whmc_field_bytes": ([_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "whmc_load_gauge": ([_P, _P, ctypes.c_double], ctypes.c_int),
    "whmc_export_gauge": ([_P, _P], ctypes.c_int),
    "whmc_pack_spinor": ([_P, _P, _P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "whmc_unpack_spinor": ([_P, _P, _P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "whmc_convert_spinor": ([_P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "whmc_pack_algebra": ([_P, _P, _P], ctypes.c_int),
    "whmc_unpack_algebra": ([_P, _P, _P], ctypes.c_int),
    "whmc_apply_H": ([_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "whmc_apply_Moo": ([_P, _P, _P, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "whmc_apply_H_multi": ([_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "whmc_autotune": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)],
                      ctypes.c_int),
    "whmc_bicgstab_solve": ([_P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.POINTER(CGParams),
                             ctypes.POINTER(CGStats)], ctypes.c_int),
    "whmc_apply_MdagM": ([_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "whmc_apply_M": ([_P, _P, _P, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "whmc_apply_MdagM_noalloc": ([_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int],
                                 ctypes.c_int),
    "whmc_cg_solve_full": ([_P, _P, _P, ctypes.c_double, ctypes.POINTER(CGParams), ctypes.POINTER(CGStats)],
                           ctypes.c_int),
    "whmc_action_full": ([_P, ctypes.POINTER(ctypes.c_double), _P, ctypes.c_double, ctypes.POINTER(CGParams)],
                         ctypes.c_int),
    "whmc_force_full": ([_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(CGParams), ctypes.c_int],
                        ctypes.c_int),
    "whmc_cg_solve": ([_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(CGParams),
                       ctypes.POINTER(CGStats)], ctypes.c_int),
    "whmc_filter_coefficients": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "whmc_heatbath_phi": ([_P, _P, _P, ctypes.POINTER(Filter), ctypes.c_double], ctypes.c_int),
    "whmc_action": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P,
                     ctypes.POINTER(Filter), ctypes.c_double, ctypes.c_double, ctypes.POINTER(CGParams)],
                    ctypes.c_int),
    "whmc_plaquette": ([_P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "whmc_force": ([_P, _P, _P, ctypes.POINTER(Filter), ctypes.c_double, ctypes.c_double,
                    ctypes.POINTER(CGParams), ctypes.c_int], ctypes.c_int),
    "whmc_update_links": ([_P, _P, ctypes.c_double], ctypes.c_int),
    "whmc_update_momenta": ([_P, _P, _P, ctypes.c_double], ctypes.c_int),
    "whmc_dexp_transpose": ([_P, _P, _P, _P], ctypes.c_int),
    "whmc_hmc_trajectory": ([_P, ctypes.POINTER(HMCParams), _P, _P, ctypes.c_double, ctypes.POINTER(TrajResult)],
                            ctypes.c_int),
    "whmc_md_integrate": ([_P, ctypes.POINTER(HMCParams), _P, _P], ctypes.c_int),
    "whmc_hamiltonian": ([_P, ctypes.POINTER(HMCParams), _P, _P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "whmc_rooted_coefficients": ([ctypes.POINTER(Rooted), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
                                 ctypes.c_int),
    "whmc_rooted_heatbath": ([_P, _P, _P, ctypes.POINTER(Rooted), ctypes.c_double, ctypes.POINTER(CGParams),
                              ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
    "whmc_rooted_action": ([_P, ctypes.POINTER(ctypes.c_double), _P, ctypes.POINTER(Rooted), ctypes.c_double,
                            ctypes.POINTER(CGParams)], ctypes.c_int),
    "whmc_rooted_force": ([_P, _P, _P, ctypes.POINTER(Rooted), ctypes.c_int, ctypes.c_double,
                           ctypes.POINTER(CGParams), ctypes.c_int], ctypes.c_int),
    "whmc_rooted_trajectory": ([_P, ctypes.POINTER(RootedHMCParams), _P, _P, ctypes.c_double,
                                ctypes.POINTER(TrajResult)], ctypes.c_int),
    "whmc_rooted_md_integrate": ([_P, ctypes.POINTER(RootedHMCParams), _P, _P], ctypes.c_int),
    "whmc_rooted_hamiltonian": ([_P, ctypes.POINTER(RootedHMCParams), _P, _P, ctypes.POINTER(ctypes.c_double)],
                                ctypes.c_int),
    "whmc_masspre_coefficients": ([ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "whmc_masspre_heatbath": ([_P, _P, _P, ctypes.POINTER(MassPre), ctypes.c_double, ctypes.POINTER(CGParams)],
                              ctypes.c_int),
    "whmc_masspre_action": ([_P, ctypes.POINTER(ctypes.c_double), _P, ctypes.POINTER(MassPre), ctypes.c_double,
                             ctypes.POINTER(CGParams)], ctypes.c_int),
    "whmc_masspre_force": ([_P, _P, _P, ctypes.POINTER(MassPre), ctypes.c_int, ctypes.c_double,
                            ctypes.POINTER(CGParams), ctypes.c_int], ctypes.c_int),
    "whmc_masspre_trajectory": ([_P, ctypes.POINTER(MassPreHMCParams), _P, _P, ctypes.c_double,
                                 ctypes.POINTER(TrajResult)], ctypes.c_int),
    "whmc_masspre_md_integrate": ([_P, ctypes.POINTER(MassPreHMCParams), _P, _P], ctypes.c_int),
    "whmc_masspre_hamiltonian": ([_P, ctypes.POINTER(MassPreHMCParams), _P, _P, ctypes.POINTER(ctypes.c_double)],
                                 ctypes.c_int),
}


def lib():
    """load libwhmc.so; raises if the library has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_03560_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise WhmcError(status, lib().whmc_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to whmc must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def filter_coefficients(k, n):
    b = (ctypes.c_double * (n + 1))()
    c = (ctypes.c_double * (n + 1))()
    a = ctypes.c_double()
    _check(lib().whmc_filter_coefficients(k, n, b, c, ctypes.byref(a)))
    return list(b), list(c), a.value


def masspre_coefficients(rho, k, n):
    """(b[0..n], alpha) of one mass-preconditioning ratio, computed by the library."""
    b = (ctypes.c_double * (n + 1))()
    a = ctypes.c_double()
    _check(lib().whmc_masspre_coefficients(float(rho), int(k), int(n), b, ctypes.byref(a)))
    return list(b), a.value


def rooted_coefficients(r, nb):
    """([p_1, ..., p_jmax], b[0..nb], alpha) of the rooted action r, computed by the library."""
    ns = [r.n[j] for j in range(r.jmax)]
    p = (ctypes.c_double * max(1, sum(n + 1 for n in ns)))()
    b = (ctypes.c_double * (nb + 1))()
    a = ctypes.c_double()
    _check(lib().whmc_rooted_coefficients(ctypes.byref(r), p, b, int(nb), ctypes.byref(a)))
    out, o = [], 0
    for n in ns:
        out.append(list(p[o:o + n + 1]))
        o += n + 1
    return out, list(b), a.value


class Context:
    """one lattice on one GPU; wraps a whmc_ctx."""

    def __init__(self, dims, device=0, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.Vh = self.V // 2
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _P()
        arr = (ctypes.c_int * 4)(*self.dims)
        _check(lib().whmc_create(ctypes.byref(h), arr, device, _P(stream.cuda_stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().whmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ buffers
    def half_spinor(self, prec=F64, n=1):
        nbytes = _HALF_BYTES[prec] * self.Vh * n
        if prec == F64:
            return torch.zeros(n * 24 * self.Vh, dtype=torch.float64, device=self.device)
        if prec == F32:
            return torch.zeros(n * 24 * self.Vh, dtype=torch.float32, device=self.device)
        return torch.zeros(nbytes, dtype=torch.uint8, device=self.device)

    def full_spinor(self, prec=F64):
        return self.half_spinor(prec, 2)

    def algebra(self):
        return torch.zeros(self.V * 32, dtype=torch.float64, device=self.device)

    def _dev(self, t, name):
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        return t

    # ------------------------------------------------------------ gauge field
    def load_gauge(self, U, unitarity_tol=1e-12):
        U = self._dev(U, "U").contiguous()
        if U.dtype != torch.complex128 or tuple(U.shape) != self.dims + (4, 3, 3):
            raise ValueError("U must be complex128 of shape (L_t, L_z, L_y, L_x, 4, 3, 3)")
        _check(lib().whmc_load_gauge(self._h, _ptr(U), unitarity_tol))

    def export_gauge(self):
        U = torch.empty(self.dims + (4, 3, 3), dtype=torch.complex128, device=self.device)
        _check(lib().whmc_export_gauge(self._h, _ptr(U)))
        return U

    # ------------------------------------------------------------ layouts
    def pack_spinor(self, psi, parity):
        """canonical complex128 (Vh,4,3) [parity 0/1] or (V,4,3)/(dims,4,3) [parity -1], optionally
        with a leading field axis -> whmc layout float64 buffer."""
        psi = self._dev(psi, "psi").contiguous()
        n_sites = self.V if parity < 0 else self.Vh
        nf = psi.numel() // (12 * n_sites)
        out = torch.empty(nf * n_sites * 24, dtype=torch.float64, device=self.device)
        _check(lib().whmc_pack_spinor(self._h, _ptr(out), _ptr(torch.view_as_real(psi)), parity, nf))
        return out

    def unpack_spinor(self, buf, parity, nfields=1):
        n_sites = self.V if parity < 0 else self.Vh
        out = torch.empty((nfields, n_sites, 4, 3) if nfields > 1 else (n_sites, 4, 3), dtype=torch.complex128,
                          device=self.device)
        _check(lib().whmc_unpack_spinor(self._h, _ptr(torch.view_as_real(out)), _ptr(buf), parity, nfields))
        return out

    def convert_spinor(self, src, src_prec, dst_prec, nhalf=1):
        dst = self.half_spinor(dst_prec, nhalf)
        _check(lib().whmc_convert_spinor(self._h, _ptr(dst), dst_prec, _ptr(src), src_prec, nhalf))
        return dst

    def pack_algebra(self, a):
        a = self._dev(a, "a").contiguous()
        out = torch.empty(self.V * 32, dtype=torch.float64, device=self.device)
        _check(lib().whmc_pack_algebra(self._h, _ptr(out), _ptr(a)))
        return out

    def unpack_algebra(self, buf):
        out = torch.empty(self.dims + (4, 8), dtype=torch.float64, device=self.device)
        _check(lib().whmc_unpack_algebra(self._h, _ptr(out), _ptr(buf)))
        return out

    # ------------------------------------------------------------ operators
    def apply_H(self, inp, out_parity, dagger=False, prec=F64, links=L18, out=None):
        if out is None:
            out = self.half_spinor(prec, 2 if out_parity < 0 else 1)
        _check(lib().whmc_apply_H(self._h, _ptr(out), _ptr(inp), out_parity, int(dagger), prec, links))
        return out

    def apply_H_multi(self, inp, out_parity, nrhs, dagger=False, prec=F64, links=L18, rhs_block=0, rhs_lanes=0,
                      rhs_order=0, out=None):
        if out is None:
            out = self.half_spinor(prec, nrhs)
        _check(lib().whmc_apply_H_multi(self._h, _ptr(out), _ptr(inp), out_parity, int(dagger), prec, links, nrhs,
                                        rhs_block, rhs_lanes, rhs_order))
        return out

    def autotune(self, prec, links, nrhs):
        """-> (rhs_block, rhs_lanes, rhs_order, microseconds per launch) of the fastest multi-RHS blocking"""
        nb, lanes, order, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().whmc_autotune(self._h, prec, links, nrhs, ctypes.byref(nb), ctypes.byref(lanes),
                                   ctypes.byref(order), ctypes.byref(us)))
        return nb.value, lanes.value, order.value, us.value

    def apply_Moo(self, inp, kappa, dagger=False, out=None):
        out = self.half_spinor() if out is None else out
        _check(lib().whmc_apply_Moo(self._h, _ptr(out), _ptr(inp), kappa, int(dagger)))
        return out

    def apply_MdagM(self, inp, kappas, out=None, eo=True):
        """M_oo^dag M_oo on odd-site half fields (eo=True) or M^dag M on full spinors (eo=False)."""
        kappas = [float(k) for k in (kappas if hasattr(kappas, "__len__") else [kappas])]
        n = len(kappas)
        out = self.half_spinor(F64, n if eo else 2 * n) if out is None else out
        _check(lib().whmc_apply_MdagM(self._h, _ptr(out), _ptr(inp), (ctypes.c_double * n)(*kappas), n, int(bool(eo))))
        return out

    def apply_MdagM_noalloc(self, inp, kappas, out, eo=True):
        """apply_MdagM through the entry point that allocates nothing (static scratch); out must be given"""
        kappas = [float(k) for k in (kappas if hasattr(kappas, "__len__") else [kappas])]
        n = len(kappas)
        _check(lib().whmc_apply_MdagM_noalloc(self._h, _ptr(out), _ptr(inp), (ctypes.c_double * n)(*kappas), n,
                                              int(bool(eo))))
        return out

    def apply_M(self, inp, kappa, dagger=False, out=None):
        """full-lattice M = 1 - kappa H (or M^dag) on a full spinor"""
        out = self.full_spinor() if out is None else out
        _check(lib().whmc_apply_M(self._h, _ptr(out), _ptr(inp), float(kappa), int(bool(dagger))))
        return out

    def cg_solve_full(self, b, kappa, params=None, x=None, raise_on_noconv=True):
        """x = (M^dag M)^{-1} b on the full lattice, FP64 CG"""
        params = params or cg_params()
        x = self.full_spinor() if x is None else x
        st = CGStats()
        rc = lib().whmc_cg_solve_full(self._h, _ptr(x), _ptr(b), float(kappa), ctypes.byref(params), ctypes.byref(st))
        if rc != 0 and (rc != 3 or raise_on_noconv):
            _check(rc)
        return x, st.as_dict()

    def action_full(self, phi, kappa, solver=None):
        s = ctypes.c_double()
        _check(lib().whmc_action_full(self._h, ctypes.byref(s), _ptr(phi), float(kappa),
                                      ctypes.byref(solver) if solver is not None else None))
        return s.value

    def force_full(self, phi, kappa, beta=0.0, flags=FORCE_PF, solver=None, out=None):
        out = self.algebra() if out is None else out
        _check(lib().whmc_force_full(self._h, _ptr(out), _ptr(phi), float(kappa), float(beta),
                                     ctypes.byref(solver) if solver is not None else None, int(flags)))
        return out

    def autotune_hop(self):
        """-> (schedule, chunk, microseconds per hop) of the fastest single-RHS stencil schedule; the
        occupancy cap it chose is get_option(OPT_HOP_WG_PER_CU)"""
        sc, ch, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().whmc_autotune_hop(self._h, ctypes.byref(sc), ctypes.byref(ch), ctypes.byref(us)))
        return sc.value, ch.value, us.value

    def set_option(self, option, value):
        _check(lib().whmc_set_option(self._h, int(option), int(value)))

    def get_option(self, option):
        v = ctypes.c_longlong()
        _check(lib().whmc_get_option(self._h, int(option), ctypes.byref(v)))
        return v.value

    def cg_solve(self, b, kappas, params=None, x=None, raise_on_noconv=True):
        kappas = [float(k) for k in (kappas if hasattr(kappas, "__len__") else [kappas])]
        n = len(kappas)
        params = params or cg_params()
        x = self.half_spinor(F64, n) if x is None else x
        stats = (CGStats * n)()
        rc = lib().whmc_cg_solve(self._h, _ptr(x), _ptr(b), (ctypes.c_double * n)(*kappas), n, ctypes.byref(params),
                                 stats)
        if rc != 0 and (rc != 3 or raise_on_noconv):
            _check(rc)
        return x, [s.as_dict() for s in stats]

    def bicgstab_solve(self, b, kappa, dagger=False, params=None, x=None, raise_on_noconv=True):
        """x = M_oo(kappa)^{-1} b (dagger: M_oo^dag x = b) by BiCGstab, FP64"""
        params = params or cg_params()
        x = self.half_spinor(F64) if x is None else x
        st = CGStats()
        rc = lib().whmc_bicgstab_solve(self._h, _ptr(x), _ptr(b), float(kappa), int(bool(dagger)),
                                       ctypes.byref(params), ctypes.byref(st))
        if rc != 0 and (rc != 3 or raise_on_noconv):
            _check(rc)
        return x, st.as_dict()

    # ------------------------------------------------------------ actions, forces, HMC
    def heatbath_phi(self, eta, k, n_t, n_max, kappa):
        phi = self.half_spinor()
        f = Filter(k, n_t, n_max)
        _check(lib().whmc_heatbath_phi(self._h, _ptr(phi), _ptr(eta), ctypes.byref(f), kappa))
        return phi

    def action(self, phi, k, n_t, n_max, kappa, beta, solver=None):
        sg, spf = ctypes.c_double(), ctypes.c_double()
        f = Filter(k, n_t, n_max)
        _check(lib().whmc_action(self._h, ctypes.byref(sg), ctypes.byref(spf), _ptr(phi), ctypes.byref(f), kappa,
                                 beta, ctypes.byref(solver) if solver is not None else None))
        return sg.value, spf.value

    def plaquette(self):
        p = ctypes.c_double()
        _check(lib().whmc_plaquette(self._h, ctypes.byref(p)))
        return p.value

    def force(self, phi, k, n_t, n_max, kappa, beta, flags=FORCE_PF, solver=None, out=None):
        out = self.algebra() if out is None else out
        f = Filter(k, n_t, n_max)
        _check(lib().whmc_force(self._h, _ptr(out), _ptr(phi), ctypes.byref(f), kappa, beta,
                                ctypes.byref(solver) if solver is not None else None, flags))
        return out

    def update_links(self, pi, eps):
        _check(lib().whmc_update_links(self._h, _ptr(pi), float(eps)))

    def update_momenta(self, pi, F, eps):
        _check(lib().whmc_update_momenta(self._h, _ptr(pi), _ptr(F), float(eps)))
        return pi

    def dexp_transpose(self, omega, F):
        out = self.algebra()
        _check(lib().whmc_dexp_transpose(self._h, _ptr(out), _ptr(omega), _ptr(F)))
        return out

    def hmc_trajectory(self, params, pi0, eta, u):
        res = TrajResult()
        _check(lib().whmc_hmc_trajectory(self._h, ctypes.byref(params), _ptr(pi0), _ptr(eta), float(u),
                                         ctypes.byref(res)))
        return res.as_dict()

    def md_integrate(self, params, pi, phi):
        _check(lib().whmc_md_integrate(self._h, ctypes.byref(params), _ptr(pi), _ptr(phi)))
        return pi

    def hamiltonian(self, params, pi, phi):
        h = ctypes.c_double()
        _check(lib().whmc_hamiltonian(self._h, ctypes.byref(params), _ptr(pi), _ptr(phi), ctypes.byref(h)))
        return h.value

    # ------------------------------------------------------------ mass preconditioning (Sec. 1, 5)
    def masspre_heatbath(self, eta, mp, kappa, solver=None):
        phi = torch.empty_like(eta)
        _check(lib().whmc_masspre_heatbath(self._h, _ptr(phi), _ptr(eta), ctypes.byref(mp), float(kappa),
                                           ctypes.byref(solver) if solver is not None else None))
        return phi

    def masspre_action(self, phi, mp, kappa, solver=None):
        S = (ctypes.c_double * (mp.n + 1))()
        _check(lib().whmc_masspre_action(self._h, S, _ptr(phi), ctypes.byref(mp), float(kappa),
                                         ctypes.byref(solver) if solver is not None else None))
        return list(S)

    def masspre_force(self, phi, mp, kappa, term=0, solver=None, out=None, accumulate=False):
        out = self.algebra() if out is None else out
        _check(lib().whmc_masspre_force(self._h, _ptr(out), _ptr(phi), ctypes.byref(mp), int(term), float(kappa),
                                        ctypes.byref(solver) if solver is not None else None,
                                        FORCE_ACCUMULATE if accumulate else 0))
        return out

    def masspre_trajectory(self, params, pi0, eta, u):
        res = TrajResult()
        _check(lib().whmc_masspre_trajectory(self._h, ctypes.byref(params), _ptr(pi0), _ptr(eta), float(u),
                                             ctypes.byref(res)))
        return res.as_dict()

    def masspre_md_integrate(self, params, pi, phi):
        _check(lib().whmc_masspre_md_integrate(self._h, ctypes.byref(params), _ptr(pi), _ptr(phi)))
        return pi

    def masspre_hamiltonian(self, params, pi, phi):
        h = ctypes.c_double()
        _check(lib().whmc_masspre_hamiltonian(self._h, ctypes.byref(params), _ptr(pi), _ptr(phi), ctypes.byref(h)))
        return h.value

    # ------------------------------------------------------------ rooted polynomials (Sec. 2.1)
    def rooted_heatbath(self, eta, r, kappa, solver=None):
        """(phi, iterations): the jmax*N + 1 fields of the rooted action from the sources eta."""
        phi = torch.empty_like(eta)
        it = ctypes.c_longlong()
        _check(lib().whmc_rooted_heatbath(self._h, _ptr(phi), _ptr(eta), ctypes.byref(r), float(kappa),
                                          ctypes.byref(solver) if solver is not None else None, ctypes.byref(it)))
        return phi, it.value

    def rooted_action(self, phi, r, kappa, solver=None):
        """[S_1, ..., S_jmax, S_r]"""
        S = (ctypes.c_double * (r.jmax + 1))()
        _check(lib().whmc_rooted_action(self._h, S, _ptr(phi), ctypes.byref(r), float(kappa),
                                        ctypes.byref(solver) if solver is not None else None))
        return list(S)

    def rooted_force(self, phi, r, kappa, term=0, solver=None, out=None, accumulate=False):
        out = self.algebra() if out is None else out
        _check(lib().whmc_rooted_force(self._h, _ptr(out), _ptr(phi), ctypes.byref(r), int(term), float(kappa),
                                       ctypes.byref(solver) if solver is not None else None,
                                       FORCE_ACCUMULATE if accumulate else 0))
        return out

    def rooted_trajectory(self, params, pi0, eta, u):
        res = TrajResult()
        _check(lib().whmc_rooted_trajectory(self._h, ctypes.byref(params), _ptr(pi0), _ptr(eta), float(u),
                                            ctypes.byref(res)))
        return res.as_dict()

    def rooted_md_integrate(self, params, pi, phi):
        _check(lib().whmc_rooted_md_integrate(self._h, ctypes.byref(params), _ptr(pi), _ptr(phi)))
        return pi

    def rooted_hamiltonian(self, params, pi, phi):
        h = ctypes.c_double()
        _check(lib().whmc_rooted_hamiltonian(self._h, ctypes.byref(params), _ptr(pi), _ptr(phi), ctypes.byref(h)))
        return h.value


def rooted_hmc_params(beta=5.6, kappa=0.1575, rooted_action=None, integrator=LEAPFROG, lam=1.0 / 6.0, m=5,
                      msub=(6, 5, 4), tau=1.4142135623730951, md_solver=None, action_solver=None,
                      heatbath_solver=None):
    """multi-level HMC with the rooted action; msub = (m_0, m_1, ..., m_jmax) as in Sec. 4.2."""
    if rooted_action is None:
        raise ValueError("rooted_hmc_params needs rooted_action=whmc.rooted(...)")
    ms = [int(v) for v in msub]
    ms = ms + [1] * (MAX_POLY + 1 - len(ms))
    return RootedHMCParams(beta, kappa, rooted_action, integrator, lam, m, (ctypes.c_int * (MAX_POLY + 1))(*ms), tau,
                           md_solver or cg_params(tol=1e-12), action_solver or cg_params(tol=1e-12),
                           heatbath_solver or cg_params(tol=1e-12))


def masspre_hmc_params(beta=5.6, kappa=0.156, mp=None, integrator=OMELYAN, lam=1.0 / 6.0, m=6, msub=(4, 1),
                       tau=1.4142135623730951, md_solver=None, action_solver=None):
    """multi-level HMC with mass preconditioning; msub = (m_0, m_1, ..., m_n)."""
    if mp is None:
        raise ValueError("masspre_hmc_params needs mp=whmc.masspre(...)")
    ms = [int(v) for v in msub]
    ms = ms + [1] * (MAX_MASSPRE + 1 - len(ms))
    return MassPreHMCParams(beta, kappa, mp, integrator, lam, m, (ctypes.c_int * (MAX_MASSPRE + 1))(*ms), tau,
                            md_solver or cg_params(tol=1e-12), action_solver or cg_params(tol=1e-12))


def hmc_params(beta=5.6, kappa=0.156, k=0, n_t=0, n_max=0, integrator=OMELYAN, lam=1.0 / 6.0, m=10, m0=4, tau=1.0,
               md_solver=None, action_solver=None):
    return HMCParams(beta, kappa, Filter(k, n_t, n_max), integrator, lam, m, m0, tau,
                     md_solver or cg_params(tol=1e-12), action_solver or cg_params(tol=1e-12))
