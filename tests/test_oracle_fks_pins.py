"""Pins of the oracle's FKS subtraction (colour-linked and spin-correlated
Borns, maps, sector functions, counterterms) against what the mathematics
fixes independently of the chosen conventions:

* colour conservation sum_l B_kl = 0 and Casimirs B_kk = C_k B,
* azimuthal completeness of the spin-correlated Born,
* the maps reproduce the Born momenta in the soft and collinear limits,
  conserve momentum and keep every particle on shell,
* the sector functions partition unity,
* the real matrix element divided by each counterterm tends to 1 in its
  limit, at the rate the expansion predicts (linear in xi for soft,
  square root of 1-y for collinear),
* the soft and collinear counterterms share their double limit,
* for e+e- -> u ubar g the soft counterterm equals its closed form,
* for u g -> t tbar u with the final quark as FKS parton, the two collinear
  ends reach different Borns (g g -> t tbar through P_gq with its spin
  correlation, u ubar -> t tbar through P_qg) and the soft quark is not
  singular.
The real matrix element in these ratios is the independently pinned |M|^2,
so a wrong eikonal factor, colour correlator, splitting kernel or
spin-correlation sign fails a limit."""
import math

import numpy as np
import pytest

from nlo_inputs.workloads import events
from physics import G2, M_TOP, mdot

CF, CA = 4.0 / 3.0, 3.0

# real process, FKS pair (i, j) (j = -1: both beams), Born process, sqrt(s)
SECTORS = [
    ("ee_uug", 4, 2, "ee_uu", 1000.0),
    ("ee_uug", 4, 3, "ee_uu", 1000.0),
    ("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0)),
    ("uu_ttg", 4, -1, "uu_tt", (400.0, 2000.0)),
    ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 5, 4, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 4, -1, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 5, -1, "gg_ttg", (400.0, 2000.0)),
]
# the FKS parton is a quark: collinear limits only, Born flavour changes at each end
QUARK_SECTORS = [("ug_ttu", 4, -1, "gg_tt", (400.0, 2000.0))]


def test_colour_linked_borns(orc):
    casimir = {"ee_uu": [CF, CF], "gg_tt": [CA, CA, CF, CF], "uu_tt": [CF] * 4, "gg_ttg": [CA, CA, CF, CF, CA]}
    for proc, rs in [("ee_uu", 1000.0), ("gg_tt", (400.0, 2000.0)), ("uu_tt", (400.0, 2000.0)),
                     ("gg_ttg", (400.0, 2000.0))]:
        mom, _ = events(proc, 16, rs, stream=21)
        B, Bkl = orc.born_correlations(proc, mom)
        assert np.allclose(B, orc.me2(proc, mom), rtol=1e-14)
        assert np.max(np.abs(Bkl.sum(axis=2)) / B[:, None]) < 1e-13
        assert np.allclose(Bkl, np.transpose(Bkl, (0, 2, 1)), rtol=1e-12, atol=0)
        diag = np.diagonal(Bkl, axis1=1, axis2=2) / B[:, None]
        assert np.allclose(diag, casimir[proc], rtol=1e-13)
    # two coloured partons: B_12 = -C_F B
    mom, _ = events("ee_uu", 4, 1000.0, stream=21)
    B, Bkl = orc.born_correlations("ee_uu", mom)
    assert np.allclose(Bkl[:, 0, 1], -CF * B, rtol=1e-14)


def test_spin_correlated_born_completeness(orc):
    """Two orthogonal transverse directions sum to the polarisation sum: for a
    gluon leg with momentum k, B(e1) + B(e2) = B for unit e1, e2 orthogonal to
    each other and to k (e.e = -1)."""
    for proc, leg in [("gg_tt", 0), ("gg_tt", 1), ("gg_ttg", 4), ("gg_ttg", 0)]:
        mom, _ = events(proc, 6, (400.0, 2000.0), stream=22)
        for e in range(mom.shape[2]):
            k = mom[leg, 1:, e]
            kh = k / np.linalg.norm(k)
            a = np.cross(kh, [0.3, -0.7, 0.2])
            a /= np.linalg.norm(a)
            b = np.cross(kh, a)
            for phi in (0.0, 0.4, 2.1):
                e1 = np.cos(phi) * a + np.sin(phi) * b
                e2 = -np.sin(phi) * a + np.cos(phi) * b
                s = sum(orc.born_spin_correlated(proc, mom[:, :, e:e + 1], leg, np.r_[0.0, ev])[0] for ev in (e1, e2))
                assert abs(s / orc.me2(proc, mom[:, :, e:e + 1])[0] - 1) < 1e-12


@pytest.mark.parametrize("real,i,j,born,rs", SECTORS + QUARK_SECTORS)
def test_maps(orc, real, i, j, born, rs):
    mom, _ = events(born, 8, rs, stream=23)
    nb = mom.shape[0]
    rng = np.random.default_rng(5)
    xt = rng.uniform(0.05, 1.0, 8)
    y = rng.uniform(-0.95, 0.95, 8)
    phi = rng.uniform(0, 2 * math.pi, 8)
    r = orc.fks(real, i, j, mom, xt, y, phi, want_real=True)
    k = r["real_mom"]
    scale = k[0, 0] + k[1, 0]
    # momentum conservation and mass shells
    assert np.max(np.abs(k[0] + k[1] - k[2:].sum(axis=0)) / scale) < 1e-13
    m2 = k[:, 0] ** 2 - (k[:, 1:] ** 2).sum(axis=1)
    masses = np.array([M_TOP if (real != "ee_uug" and q in (2, 3)) else 0.0 for q in range(k.shape[0])])
    assert np.max(np.abs(m2 - masses[:, None] ** 2)) < 1e-9 * scale.max() ** 2
    # xi is the energy fraction of parton i in the real frame; y its angle
    assert np.allclose(r["xi"], 2 * k[i, 0] / scale, rtol=1e-12)
    ref = k[j, 1:] if j >= 0 else np.array([np.zeros(8), np.zeros(8), np.ones(8)])
    cos = (k[i, 1:] * ref).sum(axis=0) / (np.linalg.norm(k[i, 1:], axis=0) * np.linalg.norm(ref, axis=0))
    assert np.allclose(cos, y, atol=1e-12)
    # soft limit: the Born momenta come back (with k_i -> 0)
    rs0 = orc.fks(real, i, j, mom, 1e-12, y, phi, want_real=True)["real_mom"]
    rest = [q for q in range(k.shape[0]) if q != i]
    bmap = [q for q in rest]
    assert np.max(np.abs(rs0[bmap] - mom)) < 1e-9 * scale.max()
    # collinear limit (final-state j): k_i + k_j = kbar_j, recoil unchanged
    if j >= 0:
        rc = orc.fks(real, i, j, mom, xt, 1.0, phi, want_real=True)["real_mom"]
        jb = bmap.index(j)
        assert np.max(np.abs(rc[i] + rc[j] - mom[jb])) < 1e-10 * scale.max()
        other = [q for q in rest if q != j]
        assert np.max(np.abs(rc[other] - mom[[bmap.index(q) for q in other]])) < 1e-10 * scale.max()


@pytest.mark.parametrize("real", ["ee_uug", "gg_ttgg"])
def test_sector_partition_of_unity(orc, real):
    born = {"ee_uug": "ee_uu", "gg_ttgg": "gg_ttg"}[real]
    rs = 1000.0 if real == "ee_uug" else (400.0, 2000.0)
    mom, _ = events(born, 32, rs, stream=24)
    i, j = (4, 2) if real == "ee_uug" else (4, 5)
    rng = np.random.default_rng(6)
    r = orc.fks(real, i, j, mom, rng.uniform(0.01, 1, 32), rng.uniform(-0.99, 0.99, 32),
                rng.uniform(0, 6.28, 32), want_real=True)
    S = orc.sector_functions(real, r["real_mom"])
    assert np.allclose(S.sum(axis=1), 1.0, rtol=1e-14)
    assert np.all(S >= 0)


@pytest.mark.parametrize("real,i,j,born,rs", SECTORS)
def test_soft_limit(orc, real, i, j, born, rs):
    mom, _ = events(born, 6, rs, stream=25)
    dev = []
    for xt in (1e-4, 1e-6):
        r = orc.fks(real, i, j, mom, xt, 0.35, 1.3)
        dev.append(np.abs(r["g_R"] / r["g_S"] - 1))
    assert np.all(dev[1] < 1e-4)
    slope = np.log(dev[0] / dev[1]) / np.log(100.0)
    assert np.all(slope > 0.8)


@pytest.mark.parametrize("real,i,j,born,rs", SECTORS + QUARK_SECTORS)
def test_collinear_limits(orc, real, i, j, born, rs):
    mom, _ = events(born, 6, rs, stream=26)
    for sign, key in ((1, "g_C"), (-1, "g_Cm")):
        if j >= 0 and sign < 0:
            continue
        dev = []
        for omy in (1e-4, 1e-6):
            r = orc.fks(real, i, j, mom, 0.25, sign * (1 - omy), 0.9)
            dev.append(np.abs(r["g_R"] / r[key] - 1))
        assert np.all(dev[1] < 1e-2)
        slope = np.log(dev[0] / dev[1]) / np.log(100.0)
        assert np.all(slope > 0.4)


@pytest.mark.parametrize("real,i,j,born,rs", SECTORS)
def test_soft_collinear_consistency(orc, real, i, j, born, rs):
    mom, _ = events(born, 4, rs, stream=27)
    for sign, kc, ksc in ((1, "g_C", "g_SC"), (-1, "g_Cm", "g_SCm")):
        if j >= 0 and sign < 0:
            continue
        a = orc.fks(real, i, j, mom, 0.3, sign * (1 - 1e-11), 0.7)
        b = orc.fks(real, i, j, mom, 1e-11, sign * 0.5, 0.7)
        assert np.allclose(a["g_S"], a[ksc], rtol=1e-5)       # y -> +-1 of the soft term
        assert np.allclose(b[kc], b[ksc], rtol=1e-9)          # xi -> 0 of the collinear term


def test_ee_uug_soft_counterterm_closed_form(orc):
    """g_S = (1-y)(4/s) g^2 [2 C_F (k1.k2)/((k1.n)(k2.n))] B with the photon
    Born B = 2 N_c Q_u^2 e^4 (t^2+u^2)/s^2 and n = (1, nhat_i)."""
    mom, _ = events("ee_uu", 64, 1000.0, stream=28)
    y, phi = 0.2, 0.8
    r = orc.fks("ee_uug", 4, 2, mom, 1e-9, y, phi, want_real=True)
    k = r["real_mom"]
    nh = k[4, 1:] / np.linalg.norm(k[4, 1:], axis=0)
    n = np.vstack([np.ones(64), nh])
    p1, p2, k1, k2 = mom
    s = 2 * mdot(p1, p2)
    t, u = -2 * mdot(p1, k1), -2 * mdot(p1, k2)
    E2 = 4 * math.pi / 132.507
    B = 2 * 3 * (2 / 3) ** 2 * E2 ** 2 * (t ** 2 + u ** 2) / s ** 2
    eik = 2 * CF * mdot(k1, k2) / (mdot(k1, n) * mdot(k2, n))
    # sector function in the soft limit (pairs (g,u) and (g,ubar))
    d2 = (2 * k1[0] / np.sqrt(s)) * (1 - (nh * k1[1:]).sum(0) / np.linalg.norm(k1[1:], axis=0))
    d3 = (2 * k2[0] / np.sqrt(s)) * (1 - (nh * k2[1:]).sum(0) / np.linalg.norm(k2[1:], axis=0))
    S = (1 / d2) / (1 / d2 + 1 / d3)
    want = (1 - y) * 4 / s * G2 * eik * B * S
    assert np.allclose(r["g_S"], want, rtol=1e-9)


def test_quark_emission_sector(orc):
    """u g -> t tbar u, FKS parton = final u: no soft counterterm; g_R
    vanishes linearly in xi (a soft quark is not singular), so W has a finite
    soft limit; the collinear counterterms are the unpolarised splitting
    functions times independently pinned Borns (checked above), and their
    azimuthal average reproduces P_gq = C_F (1 + (1-x)^2)/x on the y -> +1 side."""
    mom, _ = events("gg_tt", 6, (400.0, 2000.0), stream=28)
    r1 = orc.fks("ug_ttu", 4, -1, mom, 1e-5, 0.3, 1.0)
    r2 = orc.fks("ug_ttu", 4, -1, mom, 1e-7, 0.3, 1.0)
    for k in ("g_S", "g_SC", "g_SCm"):
        assert np.all(r1[k] == 0.0)
    assert np.allclose(r1["g_R"] / r1["xi"], r2["g_R"] / r2["xi"], rtol=1e-3)
    assert np.allclose(r1["W"], r2["W"], rtol=1e-3)
    # azimuthal average at fixed y = 1 - 1e-9 (phi and phi + pi/2 cancel the
    # cos 2 phi term of the spin correlation)
    xt = 0.4
    a = orc.fks("ug_ttu", 4, -1, mom, xt, 1 - 1e-9, 0.2)
    b = orc.fks("ug_ttu", 4, -1, mom, xt, 1 - 1e-9, 0.2 + math.pi / 2)
    x = 1 - a["xi"]
    born = orc.me2("gg_tt", mom)
    pgq = CF * (1 + (1 - x) ** 2) / x
    sb = (mom[0, 0] + mom[1, 0]) ** 2
    assert np.allclose(0.5 * (a["g_C"] + b["g_C"]), 8 * a["xi"] * G2 / sb * pgq * born, rtol=1e-12)
    # the y -> -1 side: P_qg = T_R (x^2 + (1-x)^2) times the u ubar -> t tbar Born
    c = orc.fks("ug_ttu", 4, -1, mom, xt, -(1 - 1e-9), 0.2)
    pqg = 0.5 * (x ** 2 + (1 - x) ** 2)
    assert np.allclose(c["g_Cm"], 8 * c["xi"] * G2 / sb * pqg * orc.me2("uu_tt", mom), rtol=1e-12)
