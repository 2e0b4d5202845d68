"""Pins of the oracle's RAMBO phase-space generator (the reference for the
device generator) against what the construction fixes: momentum
conservation, mass shells, the closed-form massless volumes (n = 2: 1/(8 pi),
n = 3: s/(256 pi^3)), the two-body massive weight beta/(8 pi), isotropy, and
agreement with the independent numpy implementation that writes the batch
inputs (same uniforms, different code)."""
import math

import numpy as np
import pytest

from nlo_inputs.philox import uniforms
from nlo_inputs.rambo import rambo as rambo_inputs


def _u(n, nfin, stream):
    ev = np.arange(n, dtype=np.uint64)
    u = np.empty((n, nfin, 4))
    for k in range(nfin):
        u[:, k, 0:2] = uniforms(7439, stream, ev, 2 * k)
        u[:, k, 2:4] = uniforms(7439, stream, ev, 2 * k + 1)
    rs = 400.0 + 1600.0 * uniforms(7439, stream, ev, 64)[:, 0]
    return u, rs


@pytest.mark.parametrize("masses", [[0.0, 0.0], [0.0, 0.0, 0.0], [173.0, 173.0], [173.0, 173.0, 0.0],
                                    [173.0, 173.0, 0.0, 0.0]])
def test_rambo_invariants(orc, masses):
    n = 3000
    u, rs = _u(n, len(masses), 71)
    p, w = orc.rambo(rs, masses, u)
    tot = p.sum(axis=1)
    assert np.max(np.abs(tot[:, 0] - rs) / rs) < 1e-13
    assert np.max(np.abs(tot[:, 1:]) / rs[:, None]) < 1e-13
    m2 = p[..., 0] ** 2 - (p[..., 1:] ** 2).sum(axis=-1)
    assert np.max(np.abs(m2 - np.array(masses) ** 2) / rs[:, None] ** 2) < 1e-12
    assert np.all(p[..., 0] > 0) and np.all(w > 0)
    # the independent input generator, same uniforms
    q, v = rambo_inputs(rs, masses, u)
    assert np.max(np.abs(p - q) / rs[:, None, None]) < 1e-12
    assert np.max(np.abs(w / v - 1)) < 1e-12


def test_rambo_weights_closed_forms(orc):
    n = 500
    u, rs = _u(n, 2, 72)
    _, w2 = orc.rambo(rs, [0.0, 0.0], u)
    assert np.allclose(w2, 1.0 / (8 * math.pi), rtol=1e-14)
    u, rs = _u(n, 3, 73)
    _, w3 = orc.rambo(rs, [0.0, 0.0, 0.0], u)
    assert np.allclose(w3, rs ** 2 / (256 * math.pi ** 3), rtol=1e-13)
    u, rs = _u(n, 2, 74)
    _, wm = orc.rambo(rs, [173.0, 173.0], u)
    beta = np.sqrt(1 - 4 * 173.0 ** 2 / rs ** 2)
    assert np.allclose(wm, beta / (8 * math.pi), rtol=1e-12)


def test_rambo_isotropy(orc):
    n = 200000
    u, rs = _u(n, 2, 75)
    p, _ = orc.rambo(np.full(n, 1000.0), [0.0, 0.0], u)
    c = p[:, 0, 3] / p[:, 0, 0]
    # <cos> = 0, <cos^2> = 1/3 within 5 standard errors
    assert abs(c.mean()) < 5 * math.sqrt(1 / 3 / n)
    assert abs((c ** 2).mean() - 1 / 3) < 5 * math.sqrt((1 / 5 - 1 / 9) / n)
    phi = np.arctan2(p[:, 0, 2], p[:, 0, 1])
    assert abs(np.cos(phi).mean()) < 5 * math.sqrt(0.5 / n)
