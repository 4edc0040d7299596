"""The benchmark tasks of Section III on the GPU: the link x spinor kernel
against the oracle (element by element on small lattices with a ragged tail,
sampled sites at the full 32^3 x 64 size the benchmark times), and the
doubling timed loop's contract."""
import numpy as np
import pytest

import oracle
from oracle import tasks
from paper_1401_3733_amd import bsm
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, note, rel

pytestmark = pytest.mark.gpu

LAT = gen.Lattice(8, 6, 4, 6)      # 576 sites per parity: two 256-site tiles and a 64-site tail


@pytest.mark.parametrize("N,rep,prec,lprec,tol", [
    (2, "fund", "f64", None, 1e-14), (3, "fund", "f64", None, 1e-14), (3, "fund", "f32", None, 1e-6),
    (6, "fund", "f32", None, 1e-6), (6, "fund", "f64", None, 1e-14), (5, "fund", "f64", None, 1e-14),
    (15, "fund", "f32", None, 1e-6), (15, "fund", "f64", None, 1e-14),
    (2, "adj", "f64", None, 1e-14), (3, "adj", "f32", None, 1e-6), (4, "adj", "f32", None, 1e-6),
    (4, "adj", "f64", None, 1e-14), (3, "sym", "f16s", "f32", 2e-3), (3, "sym", "f16s", "f16s", 2e-3),
    (4, "asym", "f32", None, 1e-6)])
def test_link_matvec_against_oracle(N, rep, prec, lprec, tol):
    note(f"link matvec SU({N}) {rep} {prec}/{lprec}")
    Uf = gen.gauge_links(LAT, N, "haar", 700 + N)
    S = Setup(LAT, N, rep, Uf, prec=prec, link_prec=lprec)
    psi = gen.gaussian_spinor(LAT, S.d, 701)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_link_matvec(S.desc, S.U, S.pack(psi), out)
    got = S.unpack(out)
    ref = tasks.link_matvec(oracle.represent(Uf, rep), psi)
    err = rel(got, ref)
    print(f"rel L2 error {err:.3e}")
    assert err <= tol
    # every site, not only the norm: the worst site stays within a few times the bound
    site_err = np.linalg.norm((got - ref).reshape(LAT.V, -1), axis=1) / np.linalg.norm(ref.reshape(LAT.V, -1), axis=1)
    assert site_err.max() <= 20 * tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_link_matvec_full_size_sampled(prec, tol):
    """32^3 x 64 SU(2) Haar links, the launch the benchmark times: the
    operation is site-local, so sampled output sites are checked against the
    oracle on the same sites."""
    note(f"link matvec full size SU(2) {prec}")
    lat = gen.Lattice(64, 32, 32, 32)
    Uf = gen.gauge_links(lat, 2, "haar", gen.SEED_GAUGE + 62)
    psi = gen.gaussian_spinor(lat, 2, gen.SEED_SOURCE + 62)
    S = Setup(lat, 2, "fund", Uf, prec=prec)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_link_matvec(S.desc, S.U, S.pack(psi), out)
    got = S.unpack(out)
    rng = np.random.default_rng(62)
    sample = np.concatenate([np.arange(512), np.arange(lat.V - 512, lat.V), rng.choice(lat.V, 4096, replace=False)])
    ref = tasks.link_matvec(Uf[sample], psi[sample])
    err = rel(got[sample], ref)
    print(f"sampled rel L2 error {err:.3e}")
    assert err <= tol


def _setup_small(prec="f64", N=3):
    Uf = gen.gauge_links(LAT, N, "haar", 710)
    S = Setup(LAT, N, "fund", Uf, prec=prec)
    psi = gen.gaussian_spinor(LAT, S.d, 711)
    return S, Uf, psi


def test_timed_loop_doubles_and_repeats_the_same_operation():
    note("task loop matvec / dphi")
    S, Uf, psi = _setup_small()
    inp = S.pack(psi)
    one = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_link_matvec(S.desc, S.U, inp, one)
    out = S.ctx.new_spinor(S.desc)
    it, sec = S.ctx.bsm_task_run(S.desc, "matvec", S.U, 0.0, inp, out, 0.01)
    assert sec >= 0.01 and it >= 1
    assert (it + 1) & it == 0, "1 + 2 + 4 + ... repetitions"
    assert bool((out == one).all())
    S.ctx.bsm_dslash_apply(S.desc, S.U, 0.13, 0, inp, one)
    it, sec = S.ctx.bsm_task_run(S.desc, "dphi", S.U, 0.13, inp, out, 0.01)
    assert sec >= 0.01 and (it + 1) & it == 0
    assert bool((out == one).all())
    assert rel(S.unpack(out), oracle.dslash(LAT, Uf, 0.13, psi)) <= 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", 1e-15), ("f32", 3e-7)])
def test_timed_loop_vector_task_closed_form(prec, tol):
    """out = (in + out) / 2 repeated n times from out = 0 gives in (1 - 2^-n),
    n counting the untimed validating call."""
    note(f"task loop vector {prec}")
    S, _, psi = _setup_small(prec)
    inp = S.pack(psi)
    xs = S.unpack(inp)
    out = S.ctx.new_spinor(S.desc)
    it, sec = S.ctx.bsm_task_run(S.desc, "vector", None, 0.0, inp, out, 0.005)
    assert sec >= 0.005 and (it + 1) & it == 0
    n = it + 1
    assert rel(S.unpack(out), xs * (1.0 - 2.0 ** -min(n, 1000))) <= tol


def test_task_entry_points_reject_bad_arguments():
    note("task argument checks")
    S, _, psi = _setup_small()
    inp = S.pack(psi)
    out = S.ctx.new_spinor(S.desc)
    for secs in (0.0, -1.0, 4000.0, float("nan")):
        with pytest.raises(bsm.BsmError):
            S.ctx.bsm_task_run(S.desc, "matvec", S.U, 0.0, inp, out, secs)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_task_run(S.desc, 3, S.U, 0.0, inp, out, 0.01)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_task_run(S.desc, "matvec", None, 0.0, inp, out, 0.01)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_link_matvec(S.desc, S.U, inp, inp)
    d_mixed = bsm.desc(3, "fund", "f64", "f32")
    with pytest.raises(bsm.BsmError) as e:
        S.ctx.bsm_link_matvec(d_mixed, S.U, inp, out)
    assert e.value.status == bsm.ERR_UNSUPPORTED
