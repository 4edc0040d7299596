"""Pins of the benchmark-task oracle (Section III's vector and matrix-vector
tasks, and the flop model) against closed forms, and the library's host-only
cost query against the oracle's flop count."""
import numpy as np
import pytest

import oracle
from oracle import tasks
from paper_1401_3733_amd import inputs as gen


def _cyclic_shift(d, k):
    """Permutation matrix with (P psi)_i = psi_{(i + k) mod d}."""
    P = np.zeros((d, d), np.complex128)
    for i in range(d):
        P[i, (i + k) % d] = 1.0
    return P


def test_matvec_identity_links_sum_four_directions():
    lat = gen.Lattice(2, 2, 2, 4)
    psi = gen.gaussian_spinor(lat, 3, 11)
    U = gen.unit_links(lat, 3)
    assert np.array_equal(tasks.link_matvec(U, psi), 4.0 * psi)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_matvec_row_and_direction_indexing(d):
    """U_mu = cyclic shift by mu + 1: out_i = sum_k psi_{(i+k) mod d}, k = 1..4,
    written out with explicit loops.  A transposed link shifts the other way
    and a direction mix-up changes which shifts are summed."""
    lat = gen.Lattice(2, 2, 2, 2)
    V = lat.V
    psi = gen.gaussian_spinor(lat, d, 12)
    U = np.empty((V, 4, d, d), np.complex128)
    for mu in range(4):
        U[:, mu] = _cyclic_shift(d, mu + 1)
    want = np.zeros_like(psi)
    for x in range(V):
        for s in range(4):
            for i in range(d):
                for k in range(1, 5):
                    want[x, s, i] += psi[x, s, (i + k) % d]
    assert np.allclose(tasks.link_matvec(U, psi), want, rtol=0, atol=1e-14)


def test_matvec_norm_with_phased_unitaries():
    """U_mu(x) = exp(i theta_mu(x)) W(x) with W(x) Haar unitary: the output is
    W(x) psi(x)_s times sum_mu exp(i theta_mu(x)), so its norm per site and
    spin is |sum_mu exp(i theta_mu(x))| |psi(x)_s|."""
    lat = gen.Lattice(2, 4, 2, 2)
    V, d = lat.V, 4
    rng = np.random.default_rng(13)
    W = gen.haar_sun(V, d, 14)
    theta = rng.uniform(0, 2 * np.pi, (V, 4))
    U = np.exp(1j * theta)[:, :, None, None] * W[:, None]
    psi = gen.gaussian_spinor(lat, d, 15)
    out = tasks.link_matvec(U, psi)
    fac = np.abs(np.exp(1j * theta).sum(axis=1))
    assert np.allclose(np.linalg.norm(out, axis=2), fac[:, None] * np.linalg.norm(psi, axis=2),
                       rtol=1e-13, atol=0)


def test_matvec_adjoint_links_are_real_and_local():
    """Adjoint links (real orthogonal) applied to a source at one site leave
    every other site zero and preserve the site's norm per direction; with all
    four directions equal the norm is 4x."""
    lat = gen.Lattice(2, 2, 2, 2)
    Uf = gen.gauge_links(lat, 2, "haar", 16)
    for mu in range(1, 4):
        Uf[:, mu] = Uf[:, 0]
    R = oracle.represent(Uf, "adj")
    assert np.abs(R.imag).max() == 0.0
    psi = np.zeros((lat.V, 4, 3), np.complex128)
    psi[5] = gen.gaussian_spinor(lat, 3, 17)[5]
    out = tasks.link_matvec(R, psi)
    assert np.count_nonzero(np.abs(out).sum(axis=(1, 2))) == 1
    assert np.allclose(np.linalg.norm(out[5], axis=1), 4 * np.linalg.norm(psi[5], axis=1), rtol=1e-13)


def test_axpby_closed_forms():
    lat = gen.Lattice(2, 2, 2, 2)
    x = gen.gaussian_spinor(lat, 3, 18)
    assert np.array_equal(tasks.axpby(0.5, x, 0.5, x), x)
    assert np.array_equal(tasks.axpby(1.0, x, -1.0, x), np.zeros_like(x))


def test_flop_model_pins():
    # the standard SU(3) Wilson hopping count is 1320 flops per site; the
    # diagonal term of D adds one multiply and one add per real (16 d)
    assert tasks.task_flops_per_site("dphi", 3, False) == 1320 + 48
    # d = 1 by hand: per spin 4 complex multiplies (24) and 3 complex adds (6)
    assert tasks.task_flops_per_site("matvec", 1, False) == 4 * (24 + 6)
    # real x complex multiply is 2 flops: d = 1 real links, per spin 4 * 2 + 3 * 2
    assert tasks.task_flops_per_site("matvec", 1, True) == 4 * (8 + 6)
    assert tasks.task_flops_per_site("vector", 3, False) == 72


@pytest.mark.parametrize("N,rep,prec", [(2, "fund", "f64"), (3, "fund", "f32"), (6, "fund", "f32"),
                                         (4, "adj", "f32"), (3, "sym", "f16s")])
@pytest.mark.parametrize("task", ["vector", "matvec", "dphi"])
def test_library_task_cost_matches_oracle(N, rep, prec, task):
    """bsm_task_cost is host-only: no GPU needed."""
    from paper_1401_3733_amd import bsm
    d = bsm.desc(N, rep, prec)
    dims = (8, 6, 4, 6)
    V = 8 * 6 * 4 * 6
    flops, nbytes = bsm.bsm_task_cost(dims, d, task)
    real = rep == "adj"
    assert flops == tasks.task_flops_per_site(task, d.d_R, real) * V
    rb = {"f64": 8, "f32": 4, "f16s": 2}[prec]
    site = 8 * d.d_R * rb + (4 if prec == "f16s" else 0)
    lb = {"f64": 8, "f32": 4, "f16s": 2}[{"f64": "f64", "f32": "f32", "f16s": "f32"}[prec]]
    link = d.d_R ** 2 * lb * (1 if real else 2)
    want = 3 * site if task == "vector" else 4 * link + 2 * site
    assert nbytes == want * V


def test_library_task_cost_headline_bytes():
    """SU(3) fundamental FP32 Dphi: 4 links of 72 B and 2 spinors of 96 B = 480 B per site."""
    from paper_1401_3733_amd import bsm
    f, b = bsm.bsm_task_cost((64, 32, 32, 32), bsm.desc(3, "fund", "f32"), "dphi")
    assert b == 480 * 32 ** 3 * 64


def test_library_task_cost_rejects_bad_arguments():
    from paper_1401_3733_amd import bsm
    d = bsm.desc(3, "fund", "f32")
    with pytest.raises(bsm.BsmError):
        bsm.bsm_task_cost((8, 5, 4, 6), d, "dphi")
    with pytest.raises(bsm.BsmError):
        bsm.bsm_task_cost((8, 6, 4, 6), d, 7)
    bad = bsm.FieldDesc(3, 0, 4, 1, 1)     # d_R does not match SU(3) fundamental
    with pytest.raises(bsm.BsmError):
        bsm.bsm_task_cost((8, 6, 4, 6), bad, "vector")
