"""Seeded input generators: group membership, Haar moments, reproducibility."""
import numpy as np
import pytest

from paper_1401_3733_amd import inputs as gen


@pytest.mark.parametrize("N", [2, 3, 4, 6])
def test_haar_is_special_unitary_with_haar_moments(N):
    U = gen.haar_sun(40000, N, 123)
    eye = np.eye(N)
    assert np.abs(U[:50] @ U[:50].conj().transpose(0, 2, 1) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(U[:200]) - 1).max() < 1e-12
    tr = np.trace(U, axis1=1, axis2=2)
    # E Tr U = 0 and E |Tr U|^2 = 1 for Haar measure on SU(N), N >= 2
    assert abs(tr.mean()) < 0.03
    assert abs((np.abs(tr) ** 2).mean() - 1) < 0.05


def test_near_identity_links():
    U = gen.near_identity_sun(20000, 3, 0.3, 5)
    assert np.abs(U[:50] @ U[:50].conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U[:200]) - 1).max() < 1e-12
    ml = np.trace(U, axis1=1, axis2=2).real.mean() / 3
    # E Re Tr exp(i e H)/N ~ 1 - e^2 E Tr H^2 / (2N) = 1 - 0.09 * 4 / 6
    assert abs(ml - 0.94) < 0.01


def test_seeds_reproducible_and_distinct():
    lat = gen.Lattice(2, 2, 2, 2)
    a = gen.gaussian_spinor(lat, 3, 7)
    assert np.array_equal(a, gen.gaussian_spinor(lat, 3, 7))
    assert not np.array_equal(a, gen.gaussian_spinor(lat, 3, 8))
    U1 = gen.gauge_links(lat, 3, "near_identity", 4, eps=0.3)
    assert np.array_equal(U1, gen.gauge_links(lat, 3, "near_identity", 4, eps=0.3))


def test_spinor_scale():
    lat = gen.Lattice(8, 8, 8, 8)
    a = gen.gaussian_spinor(lat, 3, 1)
    assert abs(np.mean(np.abs(a) ** 2) - 1) < 0.01
    assert abs(np.mean(a.real ** 2) - 0.5) < 0.01
