"""Pins of the oracle's adaptive integration of the subtracted real emission
(oracle/vegas.py and the map's phase-space factor), each against something
other than the oracle itself:

  VEGAS map: for ANY grid the map's weight integrates to 1 and x to 1/2
      (the midpoint rule is exact on each bin, where x is linear in u);
  VEGAS refine: a flat histogram leaves the uniform grid unchanged;
  VEGAS result: a product of narrow Gaussians against its erf closed form,
      the adapted error well below plain Monte Carlo's on the same points;
  final-state map: at fixed gluon energy, the measure dPhi_n xi j dy dphi
      integrated over the angles equals the Dalitz density dE_i dE_j / (32
      pi^3) of the three-body phase space (i, j, recoil of mass M) over its
      E_j range -- massless (e+e- -> u ubar g) and with the t tbar recoil of
      g g -> t tbar g g;
  initial-state map: at fixed real energy, integrating xi j dxi dy dphi
      Phi_2(t tbar) over xi gives the three-body volume of t tbar g from its
      Dalitz area, Phi_3 = int dm12^2 dm23^2 / (128 pi^3 s).
"""
import math

import numpy as np
import pytest

from nlo_inputs.workloads import events
from physics import M_TOP, mdot


# ----------------------------------------------------------------- VEGAS

def test_grid_map_unbiased_on_any_grid():
    from oracle.vegas import Grid
    rng = np.random.default_rng(5)
    g = Grid(2)
    for d in range(2):
        w = rng.uniform(0.01, 1.0, g.nb)
        g.edges[d, 1:] = np.cumsum(w) / w.sum()
        g.edges[d, -1] = 1.0
    m = 8                                     # points per bin and variable, on a product lattice
    u1 = (np.arange(g.nb * m) + 0.5) / (g.nb * m)
    ua, ub = np.meshgrid(u1, u1, indexing="ij")
    u = np.stack([ua.ravel(), ub.ravel()], axis=1)
    x, wt, bins = g.map(u)
    assert abs(wt.mean() - 1) < 1e-13
    assert np.all(np.abs((wt[:, None] * x).mean(axis=0) - 0.5) < 1e-13)
    assert abs((wt * x[:, 0] * x[:, 1]).mean() - 0.25) < 1e-13
    assert np.all(np.diff(x[:: u1.size, 0]) > 0) and x.min() >= 0 and x.max() <= 1
    assert np.array_equal(bins[:, 1], np.minimum((u[:, 1] * g.nb).astype(int), g.nb - 1))


def test_refine_flat_histogram_keeps_grid():
    from oracle.vegas import Grid
    g = Grid(3)
    u = (np.arange(g.nb * 10) + 0.5) / (g.nb * 10)
    x, w, bins = g.map(np.stack([u, u, u], axis=1))
    g.refine(np.ones(u.size), bins)
    assert np.allclose(g.edges, np.linspace(0, 1, g.nb + 1)[None, :], atol=1e-14, rtol=0)


def test_vegas_gaussian_product():
    from oracle.vegas import integrate
    mu = np.array([0.3, 0.45, 0.6, 0.75])
    sig = 0.04

    def f(x):
        return np.prod(np.exp(-0.5 * ((x - mu) / sig) ** 2) / (sig * math.sqrt(2 * math.pi)), axis=1)

    exact = np.prod([0.5 * (math.erf((1 - m) / (sig * math.sqrt(2))) + math.erf(m / (sig * math.sqrt(2))))
                     for m in mu])
    res, err, chi2, its = integrate(f, 4, 20000, 10, 4, seed=7439, stream=91)
    print("vegas %.6f +- %.6f exact %.6f chi2/dof %.2f plain err %.4f" % (res, err, exact, chi2, its[0][1]))
    assert abs(res - exact) < 4 * err
    assert err < 0.02 * exact
    assert its[-1][1] < 0.05 * its[0][1]       # first iteration: uniform grid = plain Monte Carlo
    assert chi2 < 3


# ------------------------------------------------------- phase-space factor

def _dalitz_ej_range(s, ei, m2rec):
    """the largest (cos theta_ij = -1) and smallest (+1) E_j for massless i, j
    and a recoil of mass^2 m2rec, from energy conservation"""
    rs = math.sqrt(s)
    num = s - m2rec - 2 * rs * ei
    return num / (2 * rs - 4 * ei), num / (2 * rs)


@pytest.mark.parametrize("real,born,i,j,rs", [("ee_uug", "ee_uu", 4, 2, 1000.0),
                                              ("gg_ttgg", "gg_ttg", 4, 5, 1300.0)])
def test_fsr_measure_is_dalitz_density(orc, real, born, i, j, rs):
    mom, _ = events(born, 2, rs, stream=93)
    s = rs * rs
    t, wt = np.polynomial.legendre.leggauss(400)
    t, wt = 0.5 * (t + 1), 0.5 * wt
    yv, wy = -1 + 2 * t * t, 4 * t * wt             # points gathered at y -> -1
    for e in range(2):
        kb = mom[:, :, e]
        jb = j if real == "ee_uug" else j - 1     # Born position of the emitter
        kj = kb[jb]
        krec = np.array([rs - kj[0], -kj[1], -kj[2], -kj[3]])
        m2rec = krec[0] ** 2 - krec[1:] @ krec[1:]
        for xt in (0.05, 0.3, 0.7, 0.95):
            n = yv.size
            xi, jac, _ = orc.fks_map(real, i, j, np.repeat(kb[:, :, None], n, axis=2), xt, yv, 0.4)
            xmax = xi[0] / xt
            ei = 0.5 * xi[0] * rs
            # Born (j, recoil) two-body volume times the angular integral, per dE_i
            fks = (1 - m2rec / s) / (8 * math.pi) * 2 * math.pi * np.sum(wy * xi * jac / xmax) * 2 / rs
            hi, lo = _dalitz_ej_range(s, ei, m2rec)
            ref = (hi - lo) / (32 * math.pi ** 3)
            assert abs(fks / ref - 1) < 1e-11, (e, xt, fks / ref - 1)


def _tt_born(sb, cth, phi):
    e = 0.5 * math.sqrt(sb)
    p = math.sqrt(e * e - M_TOP * M_TOP)
    st = math.sqrt(1 - cth * cth)
    v = p * np.array([st * math.cos(phi), st * math.sin(phi), cth])
    return np.array([[e, 0, 0, e], [e, 0, 0, -e], [e, *v], [e, *(-v)]])


def test_isr_measure_is_three_body_volume(orc):
    sr = 900.0 ** 2
    m2 = M_TOP ** 2
    # Dalitz area of t tbar g at fixed s: int dq beta(q) (s - q), q = m_{t tbar}^2
    q, wq = np.polynomial.legendre.leggauss(200)
    tq = 0.5 * (q + 1)
    qq = 4 * m2 + (sr - 4 * m2) * tq * tq            # q - 4 m^2 ~ t^2: smooth beta
    jq = (sr - 4 * m2) * 2 * tq * 0.5 * wq
    area = np.sum(jq * np.sqrt(1 - 4 * m2 / qq) * (sr - qq))
    phi3 = area / (128 * math.pi ** 3 * sr)
    # the map at fixed real energy: Born points at s_B = s_R (1 - xi)
    xi = 1 - qq / sr
    kb = np.stack([_tt_born(sb, 0.3, 1.1) for sb in qq], axis=2)
    # xi_tilde = xi / xi_max(s_B); xi_max comes back as xi_out / xi_tilde
    xi_b, jac_b, _ = orc.fks_map("gg_ttg", 4, -1, kb, np.full(qq.size, 0.5), 0.2, 0.9)
    xmax = xi_b / 0.5
    assert np.all(xi < xmax)
    xo, jac, real = orc.fks_map("gg_ttg", 4, -1, kb, xi / xmax, 0.2, 0.9)
    assert np.allclose(xo, xi, rtol=1e-13, atol=0)
    s_real = mdot(real[0] + real[1], real[0] + real[1])
    assert np.allclose(s_real, sr, rtol=1e-13)
    tot = real[2] + real[3] + real[4]
    assert np.allclose(tot, (real[0] + real[1]), atol=1e-9)
    beta = np.sqrt(1 - 4 * m2 / qq)
    dxi = jq / sr                                     # d xi = dq / s_R
    fks = np.sum(dxi * 4 * math.pi * xi * (jac / xmax) * beta / (8 * math.pi))
    print("Phi_3(t tbar g, 900 GeV) Dalitz %.12e map %.12e" % (phi3, fks))
    assert abs(fks / phi3 - 1) < 1e-10


# ----------------------------------------------------- the integrand itself

def test_subtracted_integrand_deterministic_and_conditioned(orc):
    """The same seed gives the same integral; the double-precision integrand
    matches the binary128 one to 1e-10 of the summed |f| of the sample."""
    from oracle.vegas import integrate, subtracted_integrand, uniforms_block
    f = subtracted_integrand(orc, "ee_uug", [(4, 2), (4, 3)], "ee_uu", 1000.0, [0.0, 0.0])
    a = integrate(f, 11, 2000, 3, 1, seed=7439, stream=95)
    b = integrate(f, 11, 2000, 3, 1, seed=7439, stream=95)
    assert a[0] == b[0] and a[1] == b[1] and np.isfinite(a[0]) and a[1] > 0
    x = uniforms_block(7439, 95, 0, 256, 11)
    fq = subtracted_integrand(orc, "ee_uug", [(4, 2), (4, 3)], "ee_uu", 1000.0, [0.0, 0.0], kind="quad")(x)
    fd = f(x)
    assert np.max(np.abs(fd - fq)) < 1e-10 * np.sum(np.abs(fq))
