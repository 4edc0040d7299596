"""Solvers on a lattice whose half volume is not a multiple of 64, so every
component plane ends in padding sites, with solves of different precisions
and forms sharing one context (and so one set of scratch buffers, re-carved
between them).  Every solution is checked against the oracle: reductions must
not see whatever an earlier solve left in the padding."""
import numpy as np
import pytest

import oracle
from paper_1401_3733_amd import bsm
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import c128, host, note, rel

pytestmark = pytest.mark.gpu

LAT = gen.Lattice(4, 6, 4, 6)    # 288 sites per parity: planes of 320, 32 padding sites
KAPPA = 0.13


def _gauge(ctx, d, Uf_dev):
    U = ctx.new_gauge(d)
    ctx.bsm_gauge_represent(d, Uf_dev, U)
    return U


def _unpack(ctx, d, buf, n_rhs=1):
    import torch
    dim = d.d_R
    shape = (LAT.V, 4, dim) if n_rhs == 1 else (n_rhs, LAT.V, 4, dim)
    out = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    ctx.bsm_unpack_spinor(d, buf, out, n_rhs)
    torch.cuda.synchronize()
    return host(out)


def test_solver_sequence_on_padded_lattice_shares_scratch():
    import torch
    Uf = gen.gauge_links(LAT, 3, "near_identity", 800, eps=0.3)
    UR = oracle.represent(Uf, "fund")
    ctx = bsm.Context(LAT.dims, LAT.bc)
    d64, d32 = bsm.desc(3, "fund", "f64"), bsm.desc(3, "fund", "f32")
    d16, d16l = bsm.desc(3, "fund", "f16s", "f32"), bsm.desc(3, "fund", "f16s", "f16s")
    Uf_dev = c128(Uf)
    U64, U32, U16 = _gauge(ctx, d64, Uf_dev), _gauge(ctx, d32, Uf_dev), _gauge(ctx, d16l, Uf_dev)
    b = gen.gaussian_spinor(LAT, 3, 801)
    bb = ctx.new_spinor(d64)
    ctx.bsm_pack_spinor(d64, c128(b), bb)
    xo, _ = oracle.solve(LAT, UR, KAPPA, b, tol=1e-13, schur=True)
    mixed = dict(variant=bsm.SOLVER_MIXED, delta=0.1)
    runs = [("plain schur", lambda x: ctx.bsm_cg_solve(d64, U64, U64, bsm.solver_params(KAPPA), bb, x, check=False)),
            ("mixed f16s", lambda x: ctx.bsm_cg_solve(d16, U32, U64, bsm.solver_params(KAPPA, **mixed), bb, x,
                                                     check=False)),
            ("plain full", lambda x: ctx.bsm_cg_solve(d64, U64, U64, bsm.solver_params(KAPPA, schur=False), bb, x,
                                                     check=False)),
            ("mixed f16s/f16 links", lambda x: ctx.bsm_cg_solve(d16l, U16, U64, bsm.solver_params(KAPPA, **mixed),
                                                               bb, x, check=False)),
            ("gcr", lambda x: ctx.bsm_fgcr_solve(d32, U32, U64, bsm.solver_params(KAPPA, restart=8), 1, None, bb, x,
                                                check=False)),
            ("mixed f32", lambda x: ctx.bsm_cg_solve(d32, U32, U64, bsm.solver_params(KAPPA, **mixed), bb, x,
                                                    check=False))]
    for rnd in range(2):
        for name, run in runs:
            note(f"padded lattice, round {rnd}: {name}")
            x = torch.zeros_like(bb)
            status, stats = run(x)
            xs = _unpack(ctx, d64, x)
            tr = oracle.true_residual(LAT, UR, KAPPA, b, xs)
            print(name, status, stats["iters"], tr)
            assert status == 0 and stats["converged"], (name, stats)
            assert tr <= 1e-10, name
            assert rel(xs, xo) <= 1e-9, name


def test_batched_solve_on_padded_lattice_after_other_solves():
    import torch
    Uf = gen.gauge_links(LAT, 2, "haar", 810)
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    ctx = bsm.Context(LAT.dims, LAT.bc)
    d64 = bsm.desc(2, "adj", "f64")
    d32 = bsm.desc(2, "adj", "f32")
    Uf_dev = c128(Uf)
    U64, U32 = _gauge(ctx, d64, Uf_dev), _gauge(ctx, d32, Uf_dev)
    n = 16
    kappas = list(np.linspace(0.10, 0.125, n))
    b = gen.gaussian_spinor(LAT, 3, 811, n_rhs=n)
    bb = ctx.new_spinor(d64, 2, n)
    ctx.bsm_pack_spinor(d64, c128(b), bb, n)
    nb1 = ctx.spinor_bytes(d64)
    # a mixed solve first, so the batched solver re-carves used scratch
    note("padded lattice: mixed solve before the batched one")
    x1 = torch.zeros(nb1, dtype=torch.uint8, device="cuda")
    status, _ = ctx.bsm_cg_solve(d32, U32, U64, bsm.solver_params(0.11, variant=bsm.SOLVER_MIXED), bb[:nb1], x1,
                                 check=False)
    assert status == 0
    for rnd in range(2):
        note(f"padded lattice: batched solve, round {rnd}")
        x = torch.zeros_like(bb)
        status, stats = ctx.bsm_batched_solve(d64, U64, bsm.solver_params(0.1, 1e-10, check_every=8), kappas, bb, x)
        xs = _unpack(ctx, d64, x, n)
        assert status == 0
        for r in range(n):
            assert stats[r]["converged"], (r, stats[r])
            assert oracle.true_residual(LAT, UR, kappas[r], b[r], xs[r]) <= 1e-10, r
