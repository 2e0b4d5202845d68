"""Pins of the subtracted weight W itself, on the binary128 oracle.

The FKS subtraction (the paper's NLO section: real emission minus soft and
collinear counterterms, made locally integrable) makes W a difference of
terms that each grow like 1/(xi (1-y)).  What the mathematics fixes about W,
independently of the conventions chosen for maps and sector functions:

* soft limit: at fixed y, W tends to a finite limit as xi -> 0, linearly in
  xi (the counterterms remove the 1/xi pole of xi^2 |M_R|^2 and its
  collinear end);
* collinear limit: at fixed xi, xi (1-y) W -> 0 as y -> 1 (and
  xi (1-y^2) W -> 0 as y -> -1 for the beams), like sqrt(1-|y|): the
  spin-correlated collinear counterterm removes the pole pointwise, the
  remainder is the azimuthal sqrt(1-y) term;
* W is a smooth function of the radiation variables, so a relative change of
  1e-9 in xi_tilde changes W by about 1e-9 relatively; only rounding noise
  moves it by more.

A sign slip in the combination of g_R, g_S, g_C and g_SC breaks the first two
(a planted one is shown to fail), and a W that is rounding noise breaks the
third.  In double precision the oracle's own W fails the third on about a
third of these events (rounding of the near-singular real momenta); the
binary128 build is the reference."""
import numpy as np
import pytest

from nlo_inputs.workloads import events, fks_variables

SECTORS = [
    ("ee_uug", 4, 2, "ee_uu", 1000.0),
    ("ee_uug", 4, 3, "ee_uu", 1000.0),
    ("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0)),
    ("uu_ttg", 4, -1, "uu_tt", (400.0, 2000.0)),
    ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 5, 4, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 4, -1, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 5, -1, "gg_ttg", (400.0, 2000.0)),
    ("ug_ttu", 4, -1, "gg_tt", (400.0, 2000.0)),
]


def _terms(r):
    return (np.abs(r["g_R"]) + np.abs(r["g_S"]) + np.abs(r["g_C"]) + np.abs(r["g_SC"])
            + np.abs(r["g_Cm"]) + np.abs(r["g_SCm"]))


def _fks_q(orc, sector, mom, xt, y, phi):
    real, i, j, _, _ = sector
    return orc.fks(real, i, j, mom, xt, y, phi, kind="quad")


@pytest.mark.parametrize("sector", SECTORS, ids=lambda s: "%s_%d_%d" % s[:3])
def test_w_soft_convergence(orc, sector):
    """At fixed y, W(xi) - W(0) is linear in xi down to xi_tilde = 1e-9."""
    real, i, j, born, rs = sector
    nb = 2 if real == "gg_ttgg" else 4
    mom, _ = events(born, nb, rs, stream=61)
    xts = [1e-5, 1e-6, 1e-7, 1e-8, 1e-9]
    for y in ((0.3,) if j >= 0 else (0.3, -0.6)):
        W = np.array([_fks_q(orc, sector, mom, xt, y, 1.1)["W"] for xt in xts])
        assert np.all(np.isfinite(W)) and np.all(W[-1] != 0.0)
        d = np.abs(np.diff(W, axis=0))                 # |W(xi_k) - W(xi_k+1)|
        ratio = d[:-1] / d[1:]
        assert np.all((ratio > 7.0) & (ratio < 14.0)), ratio
        assert np.all(np.abs(W[-2] / W[-1] - 1) < 1e-6)


@pytest.mark.parametrize("sector", SECTORS, ids=lambda s: "%s_%d_%d" % s[:3])
def test_w_collinear_vanishing(orc, sector):
    """xi (1-|y|) W / sum|g_X| -> 0 like sqrt(1-|y|) at every collinear end."""
    real, i, j, born, rs = sector
    nb = 2 if real == "gg_ttgg" else 4
    mom, _ = events(born, nb, rs, stream=62)
    omys = np.array([1e-4, 1e-6, 1e-8, 1e-10])
    for sign in ((1.0,) if j >= 0 else (1.0, -1.0)):
        r = []
        for omy in omys:
            res = _fks_q(orc, sector, mom, 0.3, sign * (1.0 - omy), 0.7)
            r.append(res["xi"] * omy * np.abs(res["W"]) / _terms(res))
        r = np.array(r)
        assert np.all(r[-1] < 1e-4), r[-1]
        slope = np.log(r[0] / r[-1]) / np.log(omys[0] / omys[-1])
        assert np.all(slope > 0.4), slope


def test_w_pins_catch_a_sign_slip(orc):
    """A planted mistake in the oracle's combination (+g_C instead of -g_C)
    fails both limits: W grows like 1/xi at fixed y, and xi (1-y) W tends to
    a constant at fixed xi."""
    sector = SECTORS[0]
    mom, _ = events("ee_uu", 4, 1000.0, stream=61)
    W = []
    for xt in (1e-7, 1e-8, 1e-9):
        r = _fks_q(orc, sector, mom, xt, 0.3, 1.1)
        W.append(r["W"] + 2 * r["g_C"] / (r["xi"] * 0.7))
    W = np.array(W)
    assert np.all(np.abs(W[2] / W[1]) > 5.0)            # 1/xi growth, not convergence
    r = []
    for omy in (1e-6, 1e-10):
        res = _fks_q(orc, sector, mom, 0.3, 1.0 - omy, 0.7)
        Wb = res["W"] + 2 * res["g_C"] / (res["xi"] * omy)
        r.append(res["xi"] * omy * np.abs(Wb) / _terms(res))
    assert np.all(r[1] > 0.1 * r[0]) and np.all(r[1] > 1e-2)


# stress sets: xi_tilde and 1-|y| log-uniform in [1e-6, 1] (stream 42)
JITTER = [
    ("ee_uug", 4, 2, "ee_uu", 1000.0, 4096),
    ("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0), 512),
    ("uu_ttg", 4, -1, "uu_tt", (400.0, 2000.0), 512),
    ("ug_ttu", 4, -1, "gg_tt", (400.0, 2000.0), 256),
    ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0), 48),
    ("gg_ttgg", 4, -1, "gg_ttg", (400.0, 2000.0), 64),
]


@pytest.mark.slow
@pytest.mark.parametrize("sector", JITTER, ids=lambda s: "%s_%d_%d" % s[:3])
def test_w_input_jitter(orc, sector):
    """A relative change of 1e-9 in xi_tilde moves the binary128 W by at most
    1e-6 of itself on every event of the stress set."""
    real, i, j, born, rs, n = sector
    mom, _ = events(born, n, rs, stream=42)
    xt, y, phi = fks_variables(n, stream=42, initial_state=(j < 0))
    a = _fks_q(orc, sector[:5], mom, xt, y, phi)
    b = _fks_q(orc, sector[:5], mom, xt * (1 + 1e-9), y, phi)
    rel = np.abs(b["W"] - a["W"]) / np.abs(a["W"])
    print(real, i, j, "jitter max %.2e median %.2e" % (rel.max(), np.median(rel)))
    assert np.all(rel <= 1e-6)
