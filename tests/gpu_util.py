"""Helpers for the GPU parity tests: upload, represent, pack, run, unpack."""
import sys

import numpy as np

from paper_1401_3733_amd import bsm


def note(msg):
    """Print and flush what names the case before each GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


def c128(a):
    return bsm.to_device_c128(a)


def host(t):
    return t.cpu().numpy()


def dev_build_d():
    """d_R values compiled in a restricted development build, or None."""
    import os
    stamp = os.path.join(os.path.dirname(bsm.LIB_PATH), "libbsm.dev")
    if not os.path.exists(stamp):
        return None
    return {int(x) for x in open(stamp).read().split(",")}


class Setup:
    """Context + represented links on the GPU for one lattice and (N, rep)."""

    def __init__(self, lat, N, rep, Uf, prec="f64", link_prec=None, fundamental_links=False):
        import torch
        ds = dev_build_d()
        if ds is not None:
            raise RuntimeError(f"libbsm.so is a development build restricted to d_R in {sorted(ds)}: "
                               "rebuild the full library before running the GPU tests")
        self.lat = lat
        self.ctx = bsm.Context(lat.dims, lat.bc)
        self.desc = bsm.desc(N, rep, prec, link_prec, fundamental_links=fundamental_links)
        self.d = self.desc.d_R
        self.Uf_dev = c128(Uf)
        self.U = self.ctx.new_gauge(self.desc)
        self.ctx.bsm_gauge_represent(self.desc, self.Uf_dev, self.U)
        torch.cuda.synchronize()

    def pack(self, psi, n_rhs=1, desc=None):
        desc = desc or self.desc
        buf = self.ctx.new_spinor(desc, 2, n_rhs)
        self.ctx.bsm_pack_spinor(desc, c128(psi), buf, n_rhs)
        return buf

    def unpack(self, buf, n_rhs=1, desc=None):
        import torch
        desc = desc or self.desc
        shape = (self.lat.V, 4, self.d) if n_rhs == 1 else (n_rhs, self.lat.V, 4, self.d)
        out = torch.zeros(shape, dtype=torch.complex128, device="cuda")
        self.ctx.bsm_unpack_spinor(desc, buf, out, n_rhs)
        torch.cuda.synchronize()
        return host(out)

    def block(self, buf, parity, desc=None):
        """view of one parity block of a full internal field"""
        desc = desc or self.desc
        nb = self.ctx.spinor_bytes(desc, 1, 1)
        return buf[parity * nb:(parity + 1) * nb]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))
