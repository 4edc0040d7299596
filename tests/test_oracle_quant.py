"""The FP16 per-site-scale quantiser against the binary16 rounding bound."""
import numpy as np

from oracle import quant
from paper_1401_3733_amd import inputs as gen


def test_round_trip_bound_and_zero_site():
    lat = gen.Lattice(4, 4, 2, 2)
    psi = gen.gaussian_spinor(lat, 3, 1)
    psi[5] = 0.0                              # a site with s = 0
    psi[6] *= 1e-30                           # tiny but nonzero: scale keeps it representable
    q, s = quant.quantise(psi)
    assert q.dtype == np.float16 and s.dtype == np.float32
    assert s[5] == 0 and np.all(q[5] == 0)
    back = quant.dequantise(q, s, 3)
    # reference values the quantiser saw: psi rounded to float32
    ref = psi.real.astype(np.float32).astype(np.float64) + 1j * psi.imag.astype(np.float32).astype(np.float64)
    err = np.abs(np.stack([(back - ref).real, (back - ref).imag], -1)).reshape(lat.V, -1).max(axis=1)
    # relative error 2^-11 (RNE in binary16) plus the float32 product rounding,
    # plus the subnormal floor s * 2^-25 for tiny components
    assert np.all(err <= s.astype(np.float64) * (2.0 ** -11 + 2.0 ** -23) + s * 2.0 ** -25)
    # the largest component of every nonzero site is stored as exactly +-1
    assert np.all(np.abs(q[s > 0]).max(axis=1) == 1.0)
