"""FP16 storage with a per-site scale, step by step.

TEST INFRASTRUCTURE ONLY.  A spinor site holds 4 d complex numbers, i.e. 8 d
reals.  Stored form:
  s   = max |v_k| over the 8 d reals of the site, as a float32 (v first
        rounded to float32);
  inv = 1 / s rounded to float32 (0 when s == 0);
  q_k = binary16(round-to-nearest-even(float32(v_k * inv)));
  decoded v_k = float32(q_k) * s.
Both the product and the conversion are single roundings, so the decision of
every stored code is taken in float32 and binary16 exactly as written here.
Round-trip error per component is at most s * 2^-11 when v_k * inv lies in
the binary16 normal range (|v_k * inv| >= 2^-14) and at most s * 2^-25
absolute below it.
"""
from __future__ import annotations

import numpy as np


def quantise(psi: np.ndarray):
    """psi complex [..., V, 4, d] -> (codes float16 [..., V, 8 d], scale float32 [..., V])."""
    lead = psi.shape[:-2]
    re = np.stack([psi.real, psi.imag], axis=-1).reshape(lead + (-1,)).astype(np.float32)
    s = np.max(np.abs(re), axis=-1).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(s > 0, np.float32(1.0) / s, np.float32(0.0)).astype(np.float32)
    prod = (re * inv[..., None]).astype(np.float32)
    q = prod.astype(np.float16)
    return q, s


def dequantise(q: np.ndarray, s: np.ndarray, d: int) -> np.ndarray:
    v = q.astype(np.float32) * s[..., None]
    v = v.astype(np.float64).reshape(q.shape[:-1] + (4, d, 2))
    return v[..., 0] + 1j * v[..., 1]
