"""ctypes binding of libbsm (include/bsm.h): argument marshalling only.

Every call forwards to the HIP library; there is no fallback of any kind.
Device buffers are torch tensors (any dtype; the library sees their data
pointer), streams are torch CUDA streams (default: the current stream).
If libbsm.so is missing the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsm.so")
if os.environ.get("BSM_LIB"):
    raise RuntimeError("BSM_LIB is not supported: the binding loads only the in-tree libbsm.so")

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NOMEM, ERR_NOT_CONVERGED, ERR_NONFINITE = range(7)
REP = {"fund": 0, "adj": 1, "sym": 2, "asym": 3}
F64, F32, F16S = 0, 1, 2
PREC = {"f64": F64, "f32": F32, "f16s": F16S}
SOLVER_PLAIN, SOLVER_MIXED, SOLVER_BATCHED, SOLVER_FGCR_NET, SOLVER_SHIFTED = 0, 1, 2, 3, 4
TASK = {"vector": 0, "matvec": 1, "dphi": 2}


class BsmError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class Lattice(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("bc", C.c_int32 * 4)]


class FieldDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("rep", C.c_int32), ("d_R", C.c_int32), ("prec", C.c_int32),
                ("link_prec", C.c_int32)]


class SolverParams(C.Structure):
    _fields_ = [("variant", C.c_int32), ("schur", C.c_int32), ("kappa", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("delta", C.c_double),
                ("check_every", C.c_int32), ("restart", C.c_int32), ("precond_layers", C.c_int32),
                ("n_rhs", C.c_int32), ("kappas", C.POINTER(C.c_double)), ("channels", C.c_int32),
                ("net", C.c_void_p)]


class SolverStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("reliable_updates", C.c_int32), ("restarts", C.c_int32),
                ("converged", C.c_int32), ("true_rel_res", C.c_double), ("seconds", C.c_double),
                ("fell_back", C.c_int32), ("precond_applies", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainParams(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("batch", C.c_int32), ("steps", C.c_int32), ("seed", C.c_uint64), ("step0", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
_vp = C.c_void_p
_SIGS = {
    "bsm_ctx_create": (C.c_int, [C.POINTER(Lattice), C.POINTER(_vp)]),
    "bsm_ctx_destroy": (None, [_vp]),
    "bsm_last_error": (C.c_char_p, []),
    "bsm_rep_dim": (C.c_int32, [C.c_int32, C.c_int32]),
    "bsm_reduction_slots": (C.c_int64, [C.POINTER(Lattice)]),
    "bsm_hop_norm_slots": (C.c_int64, [C.POINTER(Lattice), C.POINTER(FieldDesc)]),
    "bsm_gauge_bytes": (C.c_size_t, [_vp, C.POINTER(FieldDesc)]),
    "bsm_spinor_bytes": (C.c_size_t, [_vp, C.POINTER(FieldDesc), C.c_int32, C.c_int32]),
    "bsm_pack_spinor": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, _vp, _vp, _vp]),
    "bsm_unpack_spinor": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, _vp, _vp, _vp]),
    "bsm_gauge_represent": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp, _vp]),
    "bsm_unpack_gauge": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp, _vp]),
    "bsm_dslash_apply": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_double, C.c_int32, _vp, _vp, _vp]),
    "bsm_dslash_eo": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, C.c_int32, C.c_double, _vp,
                                C.c_double, _vp, _vp, _vp]),
    "bsm_set_hop_plan": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, C.c_int32]),
    "bsm_get_hop_plan": (C.c_int, [_vp, C.POINTER(FieldDesc), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_float)]),
    "bsm_autotune": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp]),
    "bsm_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, C.c_int32, C.c_int32, _vp]),
    "bsm_stream_read": (C.c_int, [_vp, C.c_size_t, C.c_int32, C.c_int32, _vp, _vp]),
    "bsm_vec_axpby": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, C.c_double, _vp, C.c_double, _vp,
                                C.c_int32, _vp, _vp]),
    "bsm_vec_dot": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "bsm_block_bytes": (C.c_size_t, [_vp, C.POINTER(FieldDesc)]),
    "bsm_block_gauge_bytes": (C.c_size_t, [_vp, C.POINTER(FieldDesc)]),
    "bsm_pack_block": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, _vp, _vp, _vp]),
    "bsm_unpack_block": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, _vp, _vp, _vp]),
    "bsm_gauge_to_block": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp, _vp]),
    "bsm_dslash_eo_block": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_double), _vp, C.POINTER(C.c_double), _vp, _vp, _vp]),
    "bsm_block_autotune": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp]),
    "bsm_set_block_plan": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "bsm_get_block_plan": (C.c_int, [_vp, C.POINTER(FieldDesc), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "bsm_batched_solve": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.POINTER(SolverParams), C.c_int32,
                                    C.POINTER(C.c_double), _vp, _vp, C.POINTER(SolverStats), _vp]),
    "bsm_net_bytes": (C.c_size_t, [C.c_int32]),
    "bsm_ptc_layer": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]),
    "bsm_ptc_layer_adjoint": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, C.c_int32, _vp, _vp, _vp,
                                        _vp]),
    "bsm_ptc_weight_grad": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]),
    "bsm_precond_apply": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "bsm_precond_backward": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bsm_precond_apply_collapsed_noalloc": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, _vp, _vp, _vp,
                                                      _vp]),
    "bsm_precond_apply_collapsed": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "bsm_precond_train": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_int32, _vp, _vp, _vp, _vp, C.c_int32,
                                    C.POINTER(TrainParams), C.POINTER(C.c_float), _vp]),
    "bsm_precond_pairs": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.c_double, C.c_int32, _vp, C.c_int32,
                                    C.POINTER(C.c_int32), _vp, _vp, _vp]),
    "bsm_fgcr_solve": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp, C.POINTER(SolverParams), C.c_int32, _vp,
                                 _vp, _vp, C.POINTER(SolverStats), _vp]),
    "bsm_shifted_solve": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, C.POINTER(SolverParams), C.c_int32,
                                    C.POINTER(C.c_double), _vp, _vp, C.POINTER(SolverStats), _vp]),
    "bsm_cg_solve": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp, C.POINTER(SolverParams), _vp, _vp,
                               C.POINTER(SolverStats), _vp]),
    "bsm_link_matvec": (C.c_int, [_vp, C.POINTER(FieldDesc), _vp, _vp, _vp, _vp]),
    "bsm_task_cost": (C.c_int, [C.POINTER(Lattice), C.POINTER(FieldDesc), C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
    "bsm_task_run": (C.c_int, [_vp, C.POINTER(FieldDesc), C.c_int32, _vp, C.c_double, _vp, _vp, C.c_double, _vp,
                               C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
}


def exported_symbols():
    return sorted(_SIGS)


def lib():
    """Load libbsm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status != OK:
        raise BsmError(status, where, lib().bsm_last_error().decode())
    return status


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


LINKS_FUNDAMENTAL = 16


def desc(N: int, rep: str, prec="f64", link_prec=None, fundamental_links=False) -> FieldDesc:
    """fundamental_links: the gauge field holds U and the operators form the
    representation on the fly (BSM_LINKS_FUNDAMENTAL)"""
    r = REP[rep] if isinstance(rep, str) else int(rep)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    lp = p if link_prec is None else (PREC[link_prec] if isinstance(link_prec, str) else int(link_prec))
    if link_prec is None and p == F16S:
        lp = F32
    if fundamental_links:
        lp |= LINKS_FUNDAMENTAL
    return FieldDesc(N, r, bsm_rep_dim(N, r), p, lp)


def bsm_rep_dim(N: int, rep) -> int:
    return lib().bsm_rep_dim(int(N), REP[rep] if isinstance(rep, str) else int(rep))


class Context:
    """bsm_ctx for one lattice: dims = (T, LX, LY, LZ), bc per direction."""

    def __init__(self, dims, bc=(-1, 1, 1, 1)):
        lat = Lattice((C.c_int32 * 4)(*dims), (C.c_int32 * 4)(*bc))
        h = C.c_void_p()
        _check(lib().bsm_ctx_create(C.byref(lat), C.byref(h)), "bsm_ctx_create")
        self.handle = h
        self.dims = tuple(dims)
        self.bc = tuple(bc)

    def close(self):
        if self.handle:
            lib().bsm_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # sizes
    def gauge_bytes(self, d: FieldDesc) -> int:
        n = lib().bsm_gauge_bytes(self.handle, C.byref(d))
        if n == 0:
            _check(ERR_ARG, "bsm_gauge_bytes")
        return n

    def spinor_bytes(self, d: FieldDesc, nparity=2, n_rhs=1) -> int:
        n = lib().bsm_spinor_bytes(self.handle, C.byref(d), nparity, n_rhs)
        if n == 0:
            _check(ERR_ARG, "bsm_spinor_bytes")
        return n

    # allocation helpers (torch owns the memory)
    def new_gauge(self, d: FieldDesc, device="cuda"):
        import torch
        return torch.zeros(self.gauge_bytes(d), dtype=torch.uint8, device=device)

    def new_spinor(self, d: FieldDesc, nparity=2, n_rhs=1, device="cuda"):
        import torch
        return torch.zeros(self.spinor_bytes(d, nparity, n_rhs), dtype=torch.uint8, device=device)

    # C-ABI calls
    def bsm_pack_spinor(self, d, canon, internal, n_rhs=1, stream=None):
        _check(lib().bsm_pack_spinor(self.handle, C.byref(d), n_rhs, _ptr(canon), _ptr(internal),
                                     _stream(stream)), "bsm_pack_spinor")

    def bsm_unpack_spinor(self, d, internal, canon, n_rhs=1, stream=None):
        _check(lib().bsm_unpack_spinor(self.handle, C.byref(d), n_rhs, _ptr(internal), _ptr(canon),
                                       _stream(stream)), "bsm_unpack_spinor")

    def bsm_gauge_represent(self, d, U_fund, U_rep, stream=None):
        _check(lib().bsm_gauge_represent(self.handle, C.byref(d), _ptr(U_fund), _ptr(U_rep),
                                         _stream(stream)), "bsm_gauge_represent")

    def bsm_unpack_gauge(self, d, U_rep, canon, stream=None):
        _check(lib().bsm_unpack_gauge(self.handle, C.byref(d), _ptr(U_rep), _ptr(canon), _stream(stream)),
               "bsm_unpack_gauge")

    def bsm_dslash_apply(self, d, U_rep, kappa, dagger, inp, out, stream=None):
        _check(lib().bsm_dslash_apply(self.handle, C.byref(d), _ptr(U_rep), float(kappa), int(dagger),
                                      _ptr(inp), _ptr(out), _stream(stream)), "bsm_dslash_apply")

    def bsm_dslash_eo(self, d, U_rep, out_parity, dagger, a, x, b, inp, out, stream=None):
        _check(lib().bsm_dslash_eo(self.handle, C.byref(d), _ptr(U_rep), int(out_parity), int(dagger),
                                   float(a), _ptr(x), float(b), _ptr(inp), _ptr(out), _stream(stream)),
               "bsm_dslash_eo")

    def bsm_set_hop_plan(self, d, order, tchunk=1):
        _check(lib().bsm_set_hop_plan(self.handle, C.byref(d), int(order), int(tchunk)), "bsm_set_hop_plan")

    def bsm_get_hop_plan(self, d):
        o, t, us = C.c_int32(), C.c_int32(), C.c_float()
        _check(lib().bsm_get_hop_plan(self.handle, C.byref(d), C.byref(o), C.byref(t), C.byref(us)),
               "bsm_get_hop_plan")
        return dict(order=o.value, tchunk=t.value, us=us.value)

    def bsm_autotune(self, d, U_rep, stream=None):
        _check(lib().bsm_autotune(self.handle, C.byref(d), _ptr(U_rep), _stream(stream)), "bsm_autotune")
        return self.bsm_get_hop_plan(d)

    def bsm_vec_axpby(self, d, nparity, a, x, b, y, out, prec_out=None, stream=None):
        po = d.prec if prec_out is None else (PREC[prec_out] if isinstance(prec_out, str) else prec_out)
        _check(lib().bsm_vec_axpby(self.handle, C.byref(d), int(nparity), float(a), _ptr(x), float(b),
                                   _ptr(y), int(po), _ptr(out), _stream(stream)), "bsm_vec_axpby")

    def bsm_vec_dot(self, d, nparity, x, y=None, stream=None) -> float:
        r = C.c_double(0)
        _check(lib().bsm_vec_dot(self.handle, C.byref(d), int(nparity), _ptr(x), _ptr(y), C.byref(r),
                                 _stream(stream)), "bsm_vec_dot")
        return r.value

    # block (multi-RHS) fields
    def block_bytes(self, d):
        n = lib().bsm_block_bytes(self.handle, C.byref(d))
        if n == 0:
            _check(ERR_UNSUPPORTED, "bsm_block_bytes")
        return n

    def new_block(self, d, device="cuda"):
        import torch
        return torch.zeros(self.block_bytes(d), dtype=torch.uint8, device=device)

    def new_block_gauge(self, d, device="cuda"):
        import torch
        n = lib().bsm_block_gauge_bytes(self.handle, C.byref(d))
        if n == 0:
            _check(ERR_UNSUPPORTED, "bsm_block_gauge_bytes")
        return torch.zeros(n, dtype=torch.uint8, device=device)

    def bsm_pack_block(self, d, canon, block, n_rhs, stream=None):
        _check(lib().bsm_pack_block(self.handle, C.byref(d), int(n_rhs), _ptr(canon), _ptr(block),
                                    _stream(stream)), "bsm_pack_block")

    def bsm_unpack_block(self, d, block, canon, n_rhs, stream=None):
        _check(lib().bsm_unpack_block(self.handle, C.byref(d), int(n_rhs), _ptr(block), _ptr(canon),
                                      _stream(stream)), "bsm_unpack_block")

    def bsm_gauge_to_block(self, d, U_rep, U_block, stream=None):
        _check(lib().bsm_gauge_to_block(self.handle, C.byref(d), _ptr(U_rep), _ptr(U_block), _stream(stream)),
               "bsm_gauge_to_block")

    def bsm_dslash_eo_block(self, d, U_block, out_parity, dagger, a, x, b, inp, out, stream=None):
        _check(lib().bsm_dslash_eo_block(self.handle, C.byref(d), _ptr(U_block), int(out_parity), int(dagger),
                                         _darr(a, 16), _ptr(x), _darr(b, 16), _ptr(inp), _ptr(out),
                                         _stream(stream)), "bsm_dslash_eo_block")

    def bsm_block_autotune(self, d, U_block, stream=None):
        _check(lib().bsm_block_autotune(self.handle, C.byref(d), _ptr(U_block), _stream(stream)),
               "bsm_block_autotune")
        return self.bsm_get_block_plan(d)

    def bsm_set_block_plan(self, d, sites_per_wave, waves_per_group, tiled=0, xcd_chunk=0):
        _check(lib().bsm_set_block_plan(self.handle, C.byref(d), int(sites_per_wave), int(waves_per_group),
                                        int(tiled), int(xcd_chunk)), "bsm_set_block_plan")

    def bsm_get_block_plan(self, d):
        s, w, t, c, us = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_float()
        _check(lib().bsm_get_block_plan(self.handle, C.byref(d), C.byref(s), C.byref(w), C.byref(t), C.byref(c),
                                        C.byref(us)), "bsm_get_block_plan")
        return dict(sites_per_wave=s.value, waves_per_group=w.value, tiled=t.value, xcd_chunk=c.value,
                    us=us.value)

    def bsm_batched_solve(self, d, U_rep64, params: SolverParams, kappas, b, x, stream=None, check=True):
        n = len(kappas)
        st = (SolverStats * n)()
        status = lib().bsm_batched_solve(self.handle, C.byref(d), _ptr(U_rep64), C.byref(params), n,
                                         _darr(kappas), _ptr(b), _ptr(x), st, _stream(stream))
        if check and status != OK:
            _check(status, "bsm_batched_solve")
        return status, [s.as_dict() for s in st]

    def bsm_shifted_solve(self, d, U_rep64, params: SolverParams, kappas, b, x, stream=None, check=True):
        n = len(kappas)
        st = (SolverStats * n)()
        status = lib().bsm_shifted_solve(self.handle, C.byref(d), _ptr(U_rep64), C.byref(params), n,
                                         _darr(kappas), _ptr(b), _ptr(x), st, _stream(stream))
        if check and status != OK:
            _check(status, "bsm_shifted_solve")
        return status, [s.as_dict() for s in st]

    def bsm_cg_solve(self, d, U_rep, U_rep64, params: SolverParams, b, x, stream=None, check=True):
        """stats: one dict, or a list of n_rhs dicts for the BATCHED and SHIFTED variants"""
        n = params.n_rhs if params.variant in (SOLVER_BATCHED, SOLVER_SHIFTED) else 1
        st = (SolverStats * max(1, n))()
        status = lib().bsm_cg_solve(self.handle, C.byref(d), _ptr(U_rep), _ptr(U_rep64), C.byref(params),
                                    _ptr(b), _ptr(x), st, _stream(stream))
        if check and status not in (OK,):
            _check(status, "bsm_cg_solve")
        if params.variant in (SOLVER_BATCHED, SOLVER_SHIFTED):
            return status, [s.as_dict() for s in st]
        return status, st[0].as_dict()

    # ------------------------------------------------ learned preconditioner
    def new_net(self, channels, device="cuda"):
        import torch
        return torch.zeros(lib().bsm_net_bytes(int(channels)) // 4, dtype=torch.float32, device=device)

    def bsm_ptc_layer(self, d, U_rep, cin, cout, W, inp, out, stream=None):
        _check(lib().bsm_ptc_layer(self.handle, C.byref(d), _ptr(U_rep), int(cin), int(cout), _ptr(W), _ptr(inp),
                                   _ptr(out), _stream(stream)), "bsm_ptc_layer")

    def bsm_ptc_layer_adjoint(self, d, U_rep, cin, cout, W, inp, out, stream=None):
        _check(lib().bsm_ptc_layer_adjoint(self.handle, C.byref(d), _ptr(U_rep), int(cin), int(cout), _ptr(W),
                                           _ptr(inp), _ptr(out), _stream(stream)), "bsm_ptc_layer_adjoint")

    def bsm_ptc_weight_grad(self, d, U_rep, cin, cout, G, v, dW, stream=None):
        _check(lib().bsm_ptc_weight_grad(self.handle, C.byref(d), _ptr(U_rep), int(cin), int(cout), _ptr(G),
                                         _ptr(v), _ptr(dW), _stream(stream)), "bsm_ptc_weight_grad")

    def bsm_precond_apply(self, d, U_rep, channels, net, r, z, stream=None):
        _check(lib().bsm_precond_apply(self.handle, C.byref(d), _ptr(U_rep), int(channels), _ptr(net), _ptr(r),
                                       _ptr(z), _stream(stream)), "bsm_precond_apply")

    def bsm_precond_backward(self, d, U_rep, channels, net, r, dz, dr, dweights, stream=None):
        _check(lib().bsm_precond_backward(self.handle, C.byref(d), _ptr(U_rep), int(channels), _ptr(net), _ptr(r),
                                          _ptr(dz), _ptr(dr) if dr is not None else None, _ptr(dweights),
                                          _stream(stream)), "bsm_precond_backward")

    def bsm_precond_apply_collapsed(self, d, U_rep, channels, net, r, z, stream=None):
        _check(lib().bsm_precond_apply_collapsed(self.handle, C.byref(d), _ptr(U_rep), int(channels), _ptr(net),
                                                 _ptr(r), _ptr(z), _stream(stream)), "bsm_precond_apply_collapsed")

    def bsm_precond_apply_collapsed_noalloc(self, d, U_rep, channels, net, r, z, stream=None):
        _check(lib().bsm_precond_apply_collapsed_noalloc(self.handle, C.byref(d), _ptr(U_rep), int(channels),
                                                         _ptr(net), _ptr(r), _ptr(z), _stream(stream)),
               "bsm_precond_apply_collapsed_noalloc")

    def bsm_precond_train(self, d, U_rep, channels, net, adam_state, r_pairs, e_pairs, n_pairs,
                          params: TrainParams, stream=None):
        losses = (C.c_float * max(1, params.steps))()
        _check(lib().bsm_precond_train(self.handle, C.byref(d), _ptr(U_rep), int(channels), _ptr(net),
                                       _ptr(adam_state), _ptr(r_pairs), _ptr(e_pairs), int(n_pairs),
                                       C.byref(params), losses, _stream(stream)), "bsm_precond_train")
        return list(losses)[:params.steps]

    def bsm_precond_pairs(self, d64, U_rep64, kappa, n_solves, x_star, iters, r_out, e_out, stream=None):
        it = (C.c_int32 * len(iters))(*[int(i) for i in iters])
        _check(lib().bsm_precond_pairs(self.handle, C.byref(d64), _ptr(U_rep64), float(kappa), int(n_solves),
                                       _ptr(x_star), len(iters), it, _ptr(r_out), _ptr(e_out), _stream(stream)),
               "bsm_precond_pairs")

    def bsm_fgcr_solve(self, d, U_rep, U_rep64, params: SolverParams, channels, net, b, x, stream=None,
                       check=True):
        st = SolverStats()
        status = lib().bsm_fgcr_solve(self.handle, C.byref(d), _ptr(U_rep), _ptr(U_rep64), C.byref(params),
                                      int(channels), _ptr(net), _ptr(b), _ptr(x), C.byref(st), _stream(stream))
        if check and status != OK:
            _check(status, "bsm_fgcr_solve")
        return status, st.as_dict()

    def bsm_link_matvec(self, d, U_rep, inp, out, stream=None):
        _check(lib().bsm_link_matvec(self.handle, C.byref(d), _ptr(U_rep), _ptr(inp), _ptr(out),
                                     _stream(stream)), "bsm_link_matvec")

    def bsm_task_run(self, d, task, U_rep, kappa, inp, out, min_seconds, stream=None):
        """(repetitions, seconds) of the timed doubling loop of one task"""
        it, sec = C.c_int64(), C.c_double()
        t = TASK[task] if isinstance(task, str) else int(task)
        _check(lib().bsm_task_run(self.handle, C.byref(d), t, _ptr(U_rep), float(kappa), _ptr(inp), _ptr(out),
                                  float(min_seconds), _stream(stream), C.byref(it), C.byref(sec)),
               "bsm_task_run")
        return it.value, sec.value


def _darr(vals, n=None):
    if vals is None:
        return None
    vals = list(vals)
    if n is not None:
        vals = vals + [0.0] * (n - len(vals))
    return (C.c_double * len(vals))(*[float(v) for v in vals])


def solver_params(kappa, tol=1e-10, schur=True, variant=SOLVER_PLAIN, max_iter=100000, delta=0.1,
                  check_every=0, restart=16, precond_layers=0, kappas=None, channels=0,
                  net=None) -> SolverParams:
    """kappas (BATCHED) and net (FGCR_NET, a device tensor) are kept alive on
    the returned structure; check_every 0 takes each solver's default."""
    ka = _darr(kappas)
    p = SolverParams(variant, int(schur), float(kappa), float(tol), int(max_iter), float(delta),
                     int(check_every), int(restart), int(precond_layers), len(kappas) if kappas is not None else 1,
                     C.cast(ka, C.POINTER(C.c_double)) if ka is not None else None, int(channels),
                     net.data_ptr() if net is not None else None)
    p._keep = (ka, net)
    return p


def bsm_task_cost(dims, d: FieldDesc, task, bc=(-1, 1, 1, 1)):
    """(flops, algorithmic bytes) of one repetition of a benchmark task"""
    lat = Lattice((C.c_int32 * 4)(*dims), (C.c_int32 * 4)(*bc))
    f, b = C.c_double(), C.c_double()
    t = TASK[task] if isinstance(task, str) else int(task)
    _check(lib().bsm_task_cost(C.byref(lat), C.byref(d), t, C.byref(f), C.byref(b)), "bsm_task_cost")
    return f.value, b.value


def train_params(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, batch=4, steps=100, seed=0, step0=0) -> TrainParams:
    return TrainParams(float(lr), float(beta1), float(beta2), float(eps), int(batch), int(steps), int(seed),
                       int(step0))


def bsm_stream_copy(src, dst, nbytes=None, nontemporal=0, blocks=0, stream=None):
    n = src.numel() * src.element_size() if nbytes is None else nbytes
    _check(lib().bsm_stream_copy(_ptr(src), _ptr(dst), n, int(nontemporal), int(blocks), _stream(stream)),
           "bsm_stream_copy")


def bsm_stream_read(src, out, nbytes=None, blocks=0, nontemporal=0, stream=None):
    n = src.numel() * src.element_size() if nbytes is None else nbytes
    _check(lib().bsm_stream_read(_ptr(src), n, int(nontemporal), int(blocks), _ptr(out), _stream(stream)),
           "bsm_stream_read")


# ------------------------------------------------------------- conveniences
def to_device_c128(a: np.ndarray, device="cuda"):
    """numpy complex128 -> torch complex128 on the GPU (same bytes)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)
