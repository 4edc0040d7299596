"""GPU CG solves against the FP64 oracle solution.

Gate: FP64 full-lattice true relative residual <= 1e-10 (computed by the
oracle from the GPU solution), and the solution within 1e-9 relative of the
oracle solution converged to 1e-13.  The second bound holds when
cond(D) * 1e-10 <= 1e-9, which these small lattices satisfy.
"""
import numpy as np
import pytest

import oracle
from paper_1401_3733_amd import bsm
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, note, rel

pytestmark = pytest.mark.gpu


def _solve(S, b, params, U64=None, desc=None):
    import torch
    desc = desc or S.desc
    bb = S.pack(b, desc=S.desc64) if hasattr(S, "desc64") else S.pack(b)
    x = torch.zeros_like(bb)
    st, stats = S.ctx.bsm_cg_solve(desc, S.U, U64 if U64 is not None else S.U, params, bb, x)
    xs = S.unpack(x, desc=S.desc64) if hasattr(S, "desc64") else S.unpack(x)
    return st, stats, xs


def test_cfg1_plain_cgnr_full_lattice():
    c = gen.CONFIGS[1]
    lat = gen.config_lattice(1)
    note("cg cfg1 plain full")
    Uf = gen.config_links(1, lat)
    S = Setup(lat, 2, "fund", Uf)
    b = gen.config_source(1, 2, lat)
    st, stats, x = _solve(S, b, bsm.solver_params(c["kappa"], 1e-10, schur=False))
    assert st == 0 and stats["converged"]
    tr = oracle.true_residual(lat, Uf, c["kappa"], b, x)
    assert tr <= 1e-10 and abs(tr - stats["true_rel_res"]) < 1e-12
    xo, info = oracle.solve(lat, Uf, c["kappa"], b, tol=1e-13)
    assert rel(x, xo) <= 1e-9


@pytest.mark.parametrize("N,rep,kappa", [(3, "fund", 0.13), (3, "sym", 0.125), (4, "adj", 0.12)])
def test_schur_plain(N, rep, kappa):
    note(f"cg schur plain N={N} rep={rep}")
    lat = gen.Lattice(8, 4, 6, 4)
    Uf = gen.gauge_links(lat, N, "near_identity" if rep != "adj" else "haar", 20 + N, eps=0.3)
    S = Setup(lat, N, rep, Uf)
    UR = oracle.represent(Uf, rep)
    if rep == "adj":
        UR = UR.real.astype(np.complex128)
    b = gen.gaussian_spinor(lat, S.d, 30)
    st, stats, x = _solve(S, b, bsm.solver_params(kappa, 1e-10, schur=True))
    assert st == 0
    assert oracle.true_residual(lat, UR, kappa, b, x) <= 1e-10
    xo, _ = oracle.solve(lat, UR, kappa, b, tol=1e-13, schur=True)
    assert rel(x, xo) <= 1e-9


@pytest.mark.parametrize("prec,link_prec", [("f32", "f32"), ("f16s", "f32"), ("f16s", "f16s")])
@pytest.mark.parametrize("schur", [True, False])
def test_mixed_reliable_update(prec, link_prec, schur):
    note(f"cg mixed {prec}/{link_prec} schur={schur}")
    lat = gen.Lattice(8, 4, 6, 4)
    Uf = gen.gauge_links(lat, 3, "near_identity", 40, eps=0.3)
    S64 = Setup(lat, 3, "sym", Uf)
    Slo = Setup(lat, 3, "sym", Uf, prec=prec, link_prec=link_prec)
    Slo.desc64 = S64.desc
    UR = oracle.represent(Uf, "sym")
    b = gen.gaussian_spinor(lat, 6, 41)
    prm = bsm.solver_params(0.125, 1e-10, schur=schur, variant=bsm.SOLVER_MIXED, delta=0.1)
    st, stats, x = _solve(Slo, b, prm, U64=S64.U, desc=Slo.desc)
    print(stats)
    assert st == 0 and stats["reliable_updates"] >= 1
    assert oracle.true_residual(lat, UR, 0.125, b, x) <= 1e-10
    xo, _ = oracle.solve(lat, UR, 0.125, b, tol=1e-13, schur=True)
    assert rel(x, xo) <= 1e-9


@pytest.mark.parametrize("check_every", [1, 3, 40])
def test_mixed_chunk_lengths(check_every):
    """The mixed solver enqueues check_every iterations between host reads and
    takes its reliable updates at chunk boundaries: every chunk length,
    including one longer than the solve, reaches the oracle's solution."""
    note(f"cg mixed chunk {check_every}")
    lat = gen.Lattice(8, 4, 6, 4)
    Uf = gen.gauge_links(lat, 3, "near_identity", 42, eps=0.3)
    S64 = Setup(lat, 3, "fund", Uf)
    Slo = Setup(lat, 3, "fund", Uf, prec="f16s", link_prec="f16s")
    Slo.desc64 = S64.desc
    b = gen.gaussian_spinor(lat, 3, 43)
    prm = bsm.solver_params(0.13, 1e-10, schur=True, variant=bsm.SOLVER_MIXED, check_every=check_every)
    st, stats, x = _solve(Slo, b, prm, U64=S64.U, desc=Slo.desc)
    print(stats)
    assert st == 0 and stats["reliable_updates"] >= 1
    tr = oracle.true_residual(lat, Uf, 0.13, b, x)
    assert tr <= 1e-10 and abs(tr - stats["true_rel_res"]) < 1e-12
    xo, _ = oracle.solve(lat, Uf, 0.13, b, tol=1e-13, schur=True)
    assert rel(x, xo) <= 1e-9


def test_mixed_max_iter_inside_a_chunk():
    """max_iter that ends inside a chunk of 8: the solver stops there and
    reports NOT_CONVERGED with the FP64 true residual of the iterate it
    returns (checked by the oracle)."""
    note("cg mixed max_iter 5")
    lat = gen.Lattice(4, 4, 4, 4)
    Uf = gen.gauge_links(lat, 3, "haar", 44)
    S64 = Setup(lat, 3, "fund", Uf)
    Slo = Setup(lat, 3, "fund", Uf, prec="f32", link_prec="f32")
    Slo.desc64 = S64.desc
    b = gen.gaussian_spinor(lat, 3, 45)
    import torch
    bb = Slo.pack(b, desc=S64.desc)
    x = torch.zeros_like(bb)
    prm = bsm.solver_params(0.12, 1e-10, schur=True, variant=bsm.SOLVER_MIXED, max_iter=5, check_every=8)
    status, stats = Slo.ctx.bsm_cg_solve(Slo.desc, Slo.U, S64.U, prm, bb, x, check=False)
    assert status == bsm.ERR_NOT_CONVERGED and stats["iters"] == 5
    xs = Slo.unpack(x, desc=S64.desc)
    tr = oracle.true_residual(lat, Uf, 0.12, b, xs)
    assert 1e-10 < tr < 1.0 and abs(tr - stats["true_rel_res"]) < 1e-12


def test_zero_source_and_max_iter():
    lat = gen.Lattice(4, 4, 4, 4)
    Uf = gen.gauge_links(lat, 3, "haar", 3)
    S = Setup(lat, 3, "fund", Uf)
    st, stats, x = _solve(S, np.zeros((lat.V, 4, 3), complex), bsm.solver_params(0.12, 1e-10))
    assert st == 0 and np.all(x == 0)
    b = gen.gaussian_spinor(lat, 3, 4)
    import torch
    bb = S.pack(b)
    x = torch.zeros_like(bb)
    status, stats = S.ctx.bsm_cg_solve(S.desc, S.U, S.U, bsm.solver_params(0.12, 1e-10, max_iter=2),
                                       bb, x, check=False)
    assert status == bsm.ERR_NOT_CONVERGED and stats["iters"] <= 2 + 8


def test_nonfinite_source_reported():
    lat = gen.Lattice(4, 4, 4, 4)
    S = Setup(lat, 3, "fund", gen.gauge_links(lat, 3, "haar", 5))
    b = gen.gaussian_spinor(lat, 3, 6)
    b[3, 1, 2] = np.nan
    import torch
    bb = S.pack(b)
    x = torch.zeros_like(bb)
    status, _ = S.ctx.bsm_cg_solve(S.desc, S.U, S.U, bsm.solver_params(0.12, 1e-10), bb, x, check=False)
    assert status == bsm.ERR_NONFINITE


@pytest.mark.parametrize("schur", [False, True])
def test_first_iterates_follow_the_recurrence(schur):
    """After k iterations (no convergence check can fire) the GPU iterate
    equals k steps of textbook CG on the normal equations, run in numpy
    with the oracle operators."""
    note(f"cg iterates schur={schur}")
    lat = gen.Lattice(4, 4, 4, 4)
    Uf = gen.gauge_links(lat, 2, "haar", 61)
    S = Setup(lat, 2, "fund", Uf)
    b = gen.gaussian_spinor(lat, 2, 62)
    kappa = 0.12
    par = oracle.parity_mask(lat)
    ev = (par == 0)[:, None, None]
    if schur:
        bh = (b + kappa * oracle.hop(lat, Uf, b, parity=0)) * ev
        M = lambda v: oracle.schur_apply(lat, Uf, kappa, v)
        Md = lambda v: oracle.schur_apply(lat, Uf, kappa, v, dagger=True)
    else:
        bh = b
        M = lambda v: oracle.dslash(lat, Uf, kappa, v)
        Md = lambda v: oracle.dslash(lat, Uf, kappa, v, dagger=True)
    x = np.zeros_like(b)
    r = Md(bh)
    p = r.copy()
    rr = np.vdot(r, r).real
    import torch
    bb = S.pack(b)
    for k in range(1, 4):
        Ap = Md(M(p))
        al = rr / np.vdot(p, Ap).real
        x = x + al * p
        r = r - al * Ap
        rn = np.vdot(r, r).real
        p = r + (rn / rr) * p
        rr = rn
        xg = torch.zeros_like(bb)
        status, st = S.ctx.bsm_cg_solve(S.desc, S.U, S.U, bsm.solver_params(kappa, 1e-10, schur=schur,
                                        max_iter=k, check_every=1), bb, xg, check=False)
        got = S.unpack(xg)
        if schur:
            got = got * ev
        print(k, st, rel(got, x))
        assert rel(got, x) < 1e-12, (k, rel(got, x))
