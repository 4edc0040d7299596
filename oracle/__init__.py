"""FP64 CPU oracle for the Wilson-Dirac hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The GPU library never imports, links
or executes anything here, and nothing here imports the GPU package.

Modules:
  oracle.c   plain C (double complex, OpenMP over sites): representation maps,
             hopping term, Wilson-Dirac operator, even-odd blocks, CG on the
             normal equations (full and Schur), true residual.
  dense.py   dense-matrix brute force of the operator on tiny lattices
             (numpy), and the free-field momentum-space closed form.
  quant.py   the FP16 per-site-scale quantiser, step by step.
  ptc.py     the parallel-transport convolution network and FGCR.

Functions take and return complex128 numpy arrays in the canonical layout
(site s = ((t*LZ+z)*LY+y)*LX+x; spinor [V][4][d]; links [V][4][d][d]).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

REP_CODE = {"fund": 0, "adj": 1, "sym": 2, "asym": 3}


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (C99 complex, OpenMP) into liboracle.so."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_represent.argtypes = [C.c_int, C.c_int, C.c_long, dp, dp]
        L.orc_represent.restype = C.c_int
        L.orc_rep_dim.argtypes = [C.c_int, C.c_int]
        L.orc_hop.argtypes = [ip, ip, C.c_int, dp, C.c_int, C.c_int, dp, dp]
        L.orc_dslash.argtypes = [ip, ip, C.c_int, dp, C.c_double, C.c_int, dp, dp]
        L.orc_dslash_sites.argtypes = [ip, ip, C.c_int, dp, C.c_double, C.c_int, dp, C.c_long,
                                       C.POINTER(C.c_long), dp]
        L.orc_true_residual.argtypes = [ip, ip, C.c_int, dp, C.c_double, dp, dp]
        L.orc_true_residual.restype = C.c_double
        L.orc_solve.argtypes = [ip, ip, C.c_int, dp, C.c_double, C.c_int, dp, dp, C.c_double,
                                C.c_int, dp]
        L.orc_solve.restype = C.c_int
        L.orc_cgnr_raw.argtypes = [ip, ip, C.c_int, dp, C.c_double, C.c_int, dp, dp, C.c_double,
                                   C.c_int, dp]
        L.orc_cgnr_raw.restype = C.c_int
        L.orc_op_apply.argtypes = [ip, ip, C.c_int, dp, C.c_double, C.c_int, C.c_int, dp, dp]
        L.orc_gamma.argtypes = [C.c_int, dp]
        L.orc_parity.argtypes = [ip, C.c_long]
        for name in ("orc_ptc_layer", "orc_ptc_layer_adjoint", "orc_ptc_weight_grad"):
            getattr(L, name).argtypes = [ip, ip, C.c_int, dp, C.c_int, C.c_int, dp, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(seq):
    return (C.c_int * 4)(*[int(v) for v in seq])


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def gamma(mu: int) -> np.ndarray:
    out = np.zeros((4, 4), np.complex128)
    lib().orc_gamma(mu, _dp(out))
    return out


def rep_dim(N: int, rep: str) -> int:
    return lib().orc_rep_dim(N, REP_CODE[rep])


def represent(U: np.ndarray, rep: str) -> np.ndarray:
    """R(U) for links of any leading shape [..., N, N] -> [..., d, d]."""
    U = _c128(U)
    N = U.shape[-1]
    d = rep_dim(N, rep)
    lead = U.shape[:-2]
    n = int(np.prod(lead)) if lead else 1
    R = np.zeros(lead + (d, d), np.complex128)
    rc = lib().orc_represent(N, REP_CODE[rep], n, _dp(U), _dp(R))
    if rc != d:
        raise ValueError("bad representation")
    return R


def _d_of(U):
    return U.shape[-1]


def _check(lat, U, *fields):
    """The C loops read V*4*d*d link and V*4*d spinor elements: refuse arrays
    of any other size instead of reading past them."""
    V = int(np.prod(lat.dims))
    d = _d_of(U)
    if U.size != V * 4 * d * d:
        raise ValueError(f"links: {U.size} elements, expected V*4*d*d = {V * 4 * d * d}")
    for f in fields:
        if f is not None and f.size != V * 4 * d:
            raise ValueError(f"spinor field: {f.size} elements, expected V*4*d = {V * 4 * d}")


def hop(lat, U, psi, dagger=False, parity=-1):
    """H psi (D = 1 - kappa H); parity >= 0 gives the even-odd block that
    writes sites of that parity (other sites zero)."""
    U, psi = _c128(U), _c128(psi)
    _check(lat, U, psi)
    out = np.zeros_like(psi)
    lib().orc_hop(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), int(dagger), int(parity),
                  _dp(psi), _dp(out))
    return out


def dslash(lat, U, kappa, psi, dagger=False):
    """D_W psi = psi - kappa H psi (dagger: D_W^dag psi)."""
    U, psi = _c128(U), _c128(psi)
    _check(lat, U, psi)
    out = np.zeros_like(psi)
    lib().orc_dslash(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), float(kappa), int(dagger),
                     _dp(psi), _dp(out))
    return out


def dslash_sites(lat, U, kappa, psi, sites, dagger=False):
    """(D_W psi)(x) at the listed canonical site indices only."""
    U, psi = _c128(U), _c128(psi)
    _check(lat, U, psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    if len(sites) and (sites.min() < 0 or sites.max() >= int(np.prod(lat.dims))):
        raise ValueError("site index outside the lattice")
    d = _d_of(U)
    out = np.zeros((len(sites), 4, d), np.complex128)
    lib().orc_dslash_sites(_ip(lat.dims), _ip(lat.bc), d, _dp(U), float(kappa), int(dagger),
                           _dp(psi), len(sites), sites.ctypes.data_as(C.POINTER(C.c_long)),
                           _dp(out))
    return out


def schur_apply(lat, U, kappa, psi, dagger=False):
    """Dhat psi on even sites (odd sites of the result are zero)."""
    U, psi = _c128(U), _c128(psi)
    _check(lat, U, psi)
    out = np.zeros_like(psi)
    lib().orc_op_apply(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), float(kappa), 1,
                       int(dagger), _dp(psi), _dp(out))
    return out


def true_residual(lat, U, kappa, b, x) -> float:
    U, b, x = _c128(U), _c128(b), _c128(x)
    _check(lat, U, b, x)
    return lib().orc_true_residual(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), float(kappa),
                                   _dp(b), _dp(x))


def solve(lat, U, kappa, b, tol=1e-10, schur=False, maxit=100000):
    """x with ||b - D x|| / ||b|| <= tol.  Returns (x, info dict)."""
    U, b = _c128(U), _c128(b)
    _check(lat, U, b)
    x = np.zeros_like(b)
    info = np.zeros(3)
    rc = lib().orc_solve(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), float(kappa), int(schur),
                         _dp(b), _dp(x), float(tol), int(maxit), _dp(info))
    return x, dict(converged=(rc == 0), iters=int(info[0]), true_res=float(info[1]),
                   restarts=int(info[2]))


def cgnr_raw(lat, U, kappa, b, x0=None, tol=1e-10, maxit=100000, schur=False):
    """CG on the normal equations to a normal-residual target; returns
    (x, iterations, relative normal residual)."""
    U, b = _c128(U), _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    _check(lat, U, b, x)
    rel = C.c_double(0)
    it = lib().orc_cgnr_raw(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), float(kappa),
                            int(schur), _dp(b), _dp(x), float(tol), int(maxit), C.byref(rel))
    return x, it, rel.value


def ptc_layer(lat, U, W, inp):
    """PTC layer: W [cout][cin][9][4][4], inp [cin][V][4][d] -> [cout][V][4][d]."""
    U, W, inp = _c128(U), _c128(W), _c128(inp)
    cout, cin = W.shape[:2]
    out = np.zeros((cout,) + inp.shape[1:], np.complex128)
    lib().orc_ptc_layer(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), cin, cout, _dp(W), _dp(inp), _dp(out))
    return out


def ptc_layer_adjoint(lat, U, W, inp):
    """Adjoint of ptc_layer: inp [cout][V][4][d] -> [cin][V][4][d]."""
    U, W, inp = _c128(U), _c128(W), _c128(inp)
    cout, cin = W.shape[:2]
    out = np.zeros((cin,) + inp.shape[1:], np.complex128)
    lib().orc_ptc_layer_adjoint(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), cin, cout, _dp(W), _dp(inp),
                                _dp(out))
    return out


def ptc_weight_grad(lat, U, G, v, cin, cout):
    """dW [cout][cin][9][4][4] for output gradient G [cout][..] and input v [cin][..]."""
    U, G, v = _c128(U), _c128(G), _c128(v)
    dW = np.zeros((cout, cin, 9, 4, 4), np.complex128)
    lib().orc_ptc_weight_grad(_ip(lat.dims), _ip(lat.bc), _d_of(U), _dp(U), cin, cout, _dp(G), _dp(v),
                              _dp(dW))
    return dW


def parity_mask(lat) -> np.ndarray:
    """1 for odd sites, 0 for even, in canonical site order."""
    T, X, Y, Z = lat.dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return ((t + z + y + x) & 1).reshape(-1)
