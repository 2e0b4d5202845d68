"""Pins of the integrated counterterms and the virtual correction of e+e- ->
q qbar (oracle/nlo.py):

  the four-dimensional parts of the counterterm integrand G agree with the
  oracle's counterterms: at eps = 0, G(xi, y) = j g_R / norm at the real
  point equals the textbook three-jet density (x1^2 + x2^2) / ((1-x1)(1-x2))
  times xi^2 (1-y) S and the Jacobian 2 (1-xi) / D^2; G(0, y) and G(xi, 1)
  equal the oracle's g_S and g_C in the same units;
  the Laurent expansion: the soft, collinear and double-limit integrals,
  evaluated numerically at eps = -0.01 ... -0.08 (where they converge) in
  extended precision, match 1/eps^2 + 3/(2 eps) + 13/2 - 5 zeta_2 per sector;
  the poles cancel against the quark form factor's;
  the physics: sigma_B + sigma_(V+I) + the integrated subtracted real
  emission (the oracle's VEGAS over both FKS sectors) = sigma_B (1 + alpha_s/pi)
  within its Monte Carlo error."""
import math

import numpy as np
import pytest

from nlo_inputs.workloads import events
from oracle import nlo

ALPHA, ALPHA_S = 1.0 / 132.507, 0.118
GEV2_PB = 0.3893793721e9


def _fractions(real):
    """energy fractions x_k = 2 E_k / sqrt(s) of the final state of e+e- -> u ubar g"""
    rs = real[0, 0] + real[1, 0]
    return 2 * real[2, 0] / rs, 2 * real[3, 0] / rs, 2 * real[4, 0] / rs


def test_four_dimensional_parts_of_g(orc):
    """The counterterm integrand at eps = 0 against the oracle's pinned
    counterterms: G(0, y) = 2 j(0,y)/j0 ... in the units of the derivation,
    f(0, y) = xi^2 (1-y) |M|^2 S -> 4 (the eikonal times S^soft = (1+y)/2) and
    f(xi, 1) = 2 [xi^2 + 2 (1-xi)] / (1-xi) (P_qq at z = 1 - xi); and the
    map's energy fractions x_3 = xi, x_1 = 2 (1-xi) / D."""
    n = 200
    mom, _ = events("ee_uu", n, 1000.0, stream=601)
    rng = np.random.default_rng(6)
    xt, y, phi = rng.uniform(0.01, 0.99, n), rng.uniform(-0.99, 0.99, n), rng.uniform(0, 2 * math.pi, n)
    r = orc.fks("ee_uug", 4, 2, mom, xt, y, phi, want_real=True)
    s = 1e6
    g2 = 4 * math.pi * ALPHA_S
    norm = r["B"] * 2 * nlo.CF * g2 / s
    x1, x2, x3 = _fractions(r["real_mom"])
    xi = r["xi"]
    D = 2 - xi * (1 - y)
    assert np.allclose(x3, xi, rtol=1e-12) and np.allclose(x1, 2 * (1 - xi) / D, rtol=1e-12)
    assert np.allclose(1 - x2, (1 - xi) * xi * (1 - y) / D, rtol=1e-9)
    assert np.allclose(r["g_S"] / norm, 4.0, rtol=1e-10)
    assert np.allclose(r["g_C"] / norm, 2 * (xi ** 2 + 2 * (1 - xi)) / (1 - xi), rtol=1e-10)
    # the phase-space factor: j / j0 = 4 (1-xi) / D^2
    j0 = s / (64 * math.pi ** 3)
    assert np.allclose(r["jac"] / (xi / xt) / j0, 4 * (1 - xi) / D ** 2, rtol=1e-12)


def _terms(eps):
    """soft, collinear and double-limit integrals of one sector at eps < 0,
    in 40-digit arithmetic"""
    import mpmath as mp
    mp.mp.dps = 40
    e = mp.mpf(eps)
    G0 = lambda y: 2 * ((1 + y) / 4) ** (-e)
    G01 = 2 * mp.mpf(2) ** e
    G1 = lambda x: ((1 - e) * x ** 2 + 2 * (1 - x)) * ((1 - x) ** 2 / 2) ** (-e)
    soft = (-1 / (2 * e)) * mp.quad(lambda y: (1 - y) ** (-1 - e) * (G0(y) - G01), [-1, 0, 1])
    coll = (-mp.mpf(2) ** (-e) / e) * mp.quad(lambda x: x ** (-1 - 2 * e) * (G1(x) - G01), [0, 0.5, 1])
    double = G01 * (-1 / (2 * e)) * (-mp.mpf(2) ** (-e) / e)
    return soft, coll, double


def test_counterterm_laurent_expansion():
    """T(eps) - a/eps^2 - b/eps -> c as eps -> 0 (quadratic extrapolation from
    eps = -1e-3, -2e-3, -4e-3), with (a, b, c) the derivation's"""
    import mpmath as mp
    a, b, c = nlo.counterterm_laurent()
    eps = [mp.mpf("-0.001"), mp.mpf("-0.002"), mp.mpf("-0.004")]
    r = [sum(_terms(e)) - a / e ** 2 - b / e for e in eps]
    # r = c + d eps + f eps^2: solve the 3 x 3 system
    M = mp.matrix([[1, e, e * e] for e in eps])
    cfit = mp.lu_solve(M, mp.matrix(r))[0]
    print("finite part: extrapolated %.10f, derived %.10f" % (float(cfit), c))
    assert abs(float(cfit) - c) < 1e-6
    # the poles themselves: eps^2 T -> a and the next order
    t = sum(_terms(eps[0]))
    assert abs(float(eps[0] ** 2 * t) - a) < 2e-3
    # the soft integral alone is -zeta_2 + O(eps)
    assert abs(float(_terms(eps[0])[0]) + nlo.ZETA2) < 1e-2


def test_poles_cancel_against_the_form_factor():
    a, b, c = nlo.counterterm_laurent()
    assert 2 * a - 2 == 0 and 2 * b - 3 == 0           # two sectors against -2/eps^2 - 3/eps
    # finite: two sectors (13 - 10 zeta_2) plus the form factor's -8 + pi^2
    assert abs(2 * c - 8 + math.pi ** 2 - (5 - 4 * nlo.ZETA2)) < 1e-14
    assert abs(nlo.vi_coefficient(ALPHA_S) - ALPHA_S * nlo.CF / (2 * math.pi) * (5 - 2 * math.pi ** 2 / 3)) < 1e-15


def test_nlo_k_factor_ee(orc):
    """sigma_B + sigma_(V+I) + sigma_R^sub = sigma_B (1 + alpha_s / pi) at 1000 GeV"""
    from oracle.vegas import integrate, subtracted_integrand
    rs = 1000.0
    s = rs * rs
    sigma_b = 3 * (2.0 / 3.0) ** 2 * 4 * math.pi * ALPHA ** 2 / (3 * s) * GEV2_PB
    f = subtracted_integrand(orc, "ee_uug", [(4, 2), (4, 3)], "ee_uu", rs, [0.0, 0.0])
    sr, er, chi2, _ = integrate(f, 11, 20000, 6, 2, seed=7439, stream=602)
    k = 1 + nlo.vi_coefficient(ALPHA_S) + sr / sigma_b
    print("sigma_B %.8f pb, sigma_R^sub %.8f +- %.8f pb (chi2/dof %.2f); K - 1 = %.6f +- %.6f, alpha_s/pi = %.6f"
          % (sigma_b, sr, er, chi2, k - 1, er / sigma_b, ALPHA_S / math.pi))
    assert abs(k - 1 - ALPHA_S / math.pi) < 4 * er / sigma_b
    assert er / sigma_b < 0.01 * ALPHA_S / math.pi
