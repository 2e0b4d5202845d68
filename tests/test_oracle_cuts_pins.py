"""Pins of the oracle's cut predicates (oracle/cuts.py) against what the jet
definition and kinematics fix:

  anti-kT: two partons closer than R in (rapidity, azimuth) form one jet with
      the summed four-momentum, farther apart two; the azimuth difference
      wraps at +-pi;
  infrared and collinear safety: splitting a parton into two exactly
      collinear ones (any momentum fraction), or adding a parton of vanishing
      energy anywhere, leaves the jets and the decision unchanged;
  longitudinal boosts leave jets' transverse momenta and the clustering
  unchanged, and shift every rapidity by the boost's;
  rapidity against atanh(p_z / E) for massless and massive momenta;
  FKS masks: S and (final-state emitter) C equal B; at tiny xi and, for a
      final-state emitter, at y -> 1 the real-emission mask tends to the Born
      mask (IR safety of the masks themselves); for the beams the y = +-1
      kinematics is the Born final state boosted along z, so transverse-only
      cuts give C = B at both ends."""
import math

import numpy as np
import pytest

from nlo_inputs.workloads import events
from oracle import cuts as oc


def _p(pt, y, phi, m=0.0):
    mt = math.sqrt(pt * pt + m * m)
    return np.array([mt * math.cosh(y), pt * math.cos(phi), pt * math.sin(phi), mt * math.sinh(y)])


def _boost_z(p, eta):
    e, px, py, pz = p
    return np.array([e * math.cosh(eta) + pz * math.sinh(eta), px, py, pz * math.cosh(eta) + e * math.sinh(eta)])


def _tie():
    return oc._Tie(1e-9)


def test_two_partons_merge_within_r():
    R = 0.4
    a = _p(50.0, 0.3, 1.0)
    near = _p(30.0, 0.3 + 0.25, 1.0 + 0.25)     # dR = 0.354 < 0.4
    far = _p(30.0, 0.3 + 0.3, 1.0 + 0.3)        # dR = 0.424 > 0.4
    j = oc.anti_kt([a, near], R, _tie())
    assert len(j) == 1 and np.allclose(j[0], a + near, rtol=1e-15)
    assert len(oc.anti_kt([a, far], R, _tie())) == 2
    # azimuth wraps: phi = pi - 0.01 and -pi + 0.01 are 0.02 apart
    w = oc.anti_kt([_p(40.0, 0.0, math.pi - 0.01), _p(40.0, 0.0, -math.pi + 0.01)], R, _tie())
    assert len(w) == 1


@pytest.mark.parametrize("z", [0.5, 0.1, 1e-6])
def test_collinear_and_soft_safety(z):
    cuts = dict(jet_r=0.7, jet_ptmin=20.0, jet_ymax=2.5, njet_min=2, top_ptmin=0.0, top_ymax=1e9, lep_ptmin=0.0,
                lep_ymax=1e9)
    rng = np.random.default_rng(3)
    for _ in range(50):
        ps = [_p(rng.uniform(5, 80), rng.uniform(-3, 3), rng.uniform(-math.pi, math.pi)) for _ in range(3)]
        base = oc.anti_kt(ps, cuts["jet_r"], _tie())
        ok0, _ = oc.event_pass(ps, "qqq", cuts)
        # collinear split of parton 0 into z and 1 - z
        split = [z * ps[0], (1 - z) * ps[0]] + ps[1:]
        js = oc.anti_kt(split, cuts["jet_r"], _tie())
        assert len(js) == len(base)
        assert sorted(round(oc.pt(j), 9) for j in js) == sorted(round(oc.pt(j), 9) for j in base)
        assert oc.event_pass(split, "qqqq", cuts)[0] == ok0
        # a parton of vanishing energy anywhere
        soft = ps + [_p(1e-10, rng.uniform(-3, 3), rng.uniform(-math.pi, math.pi))]
        jsoft = oc.anti_kt(soft, cuts["jet_r"], _tie())
        hard = [j for j in jsoft if oc.pt(j) > 1e-6]
        assert len(hard) == len(base)
        assert oc.event_pass(soft, "qqqq", cuts)[0] == ok0
        # exactly along the beam: not clustered
        assert len(oc.anti_kt(ps + [np.array([7.0, 0.0, 0.0, 7.0])], cuts["jet_r"], _tie())) == len(base)


def test_longitudinal_boost_invariance():
    rng = np.random.default_rng(4)
    for _ in range(50):
        ps = [_p(rng.uniform(5, 80), rng.uniform(-2, 2), rng.uniform(-math.pi, math.pi)) for _ in range(4)]
        eta = rng.uniform(-1.5, 1.5)
        a = sorted(oc.anti_kt(ps, 0.5, _tie()), key=oc.pt)
        b = sorted(oc.anti_kt([_boost_z(p, eta) for p in ps], 0.5, _tie()), key=oc.pt)
        assert len(a) == len(b)
        for x, y in zip(a, b):
            assert abs(oc.pt(x) - oc.pt(y)) <= 1e-12 * oc.pt(x)
            assert abs(oc.rapidity(y) - oc.rapidity(x) - eta) <= 1e-11


def test_rapidity_closed_form():
    for m in (0.0, 173.0):
        for y in (-4.0, -0.7, 0.0, 0.2, 3.5):
            p = _p(37.0, y, 0.3, m)
            assert abs(oc.rapidity(p) - math.atanh(p[3] / p[0])) <= 1e-12 * max(1.0, abs(y))
            assert abs(oc.rapidity(p) - y) <= 1e-12 * max(1.0, abs(y))


CUTS = dict(jet_r=0.5, jet_ptmin=30.0, jet_ymax=2.0, njet_min=1, top_ptmin=40.0, top_ymax=2.5, lep_ptmin=0.0,
            lep_ymax=1e9)


@pytest.mark.parametrize("real,born,i,j,rs,cuts", [
    ("ee_uug", "ee_uu", 4, 2, 1000.0, dict(CUTS, njet_min=2, jet_ptmin=300.0, jet_ymax=1.0)),
    ("gg_ttgg", "gg_ttg", 4, 5, (400.0, 2000.0), CUTS),
    ("gg_ttg", "gg_tt", 4, -1, (400.0, 2000.0), dict(CUTS, njet_min=0, jet_ymax=1e9, top_ymax=1e9)),
])
def test_fks_masks_ir_limits(orc, real, born, i, j, rs, cuts):
    n = 300
    mom, _ = events(born, n, rs, stream=97)
    rng = np.random.default_rng(5)
    xt, y, phi = rng.uniform(0.05, 0.95, n), rng.uniform(-0.9, 0.9, n), rng.uniform(0, 2 * math.pi, n)
    m, hit = oc.fks_masks(orc, real, i, j, born, mom, xt, y, phi, cuts)
    assert np.array_equal(m[2], m[0])
    if j >= 0:
        assert np.array_equal(m[3], m[0])
    else:       # transverse-only cuts: both collinear ends pass exactly when the Born does
        assert np.array_equal(m[3], 2 | 4 * m[0] | 8 * m[0])
    # the real mask tends to the Born one in the soft limit ...
    ms, hs = oc.fks_masks(orc, real, i, j, born, mom, np.full(n, 1e-10), y, phi, cuts)
    good = ~(hit | hs)
    assert np.array_equal(ms[1][good], ms[0][good])
    # ... and, for a final-state emitter, in the collinear one
    if j >= 0:
        mc, hc = oc.fks_masks(orc, real, i, j, born, mom, xt, np.full(n, 1 - 1e-12), phi, cuts)
        good = ~(hit | hc)
        assert np.array_equal(mc[1][good], mc[0][good])
    # the cuts do something on these sets
    assert 0.05 < m[0].mean() < 0.95 or j < 0
