"""Pins of the FP64 oracle against results fixed by the paper and by the
mathematics, independent of the oracle itself:

* closed forms of textbook 2->2 and 2->3 processes,
* the colour-dressed brute-force evaluation (full Feynman rules, explicit
  colour sums) against the colour-ordered recursion,
* gauge invariance, Lorentz invariance, Bose symmetry, coupling scaling,
  equal |M_h|^2 for reversed helicities,
* exact colour-matrix identities,
* spinor and polarisation identities (Dirac equation, completeness).
A plausible mistake anywhere in the oracle (a dropped diagram, a wrong sign or
coupling, a transposed colour string) fails at least one of these."""
import math
from fractions import Fraction

import numpy as np
import pytest

from nlo_inputs.workloads import events, to_aos
from nlo_inputs.philox import philox4x32
from nlo_inputs.rambo import massless_volume
from physics import ALPHA, ALPHA_S, E2, G2, M_TOP, mdot, boost_matrix, rotation_matrix, transform


# ---------------------------------------------------------------------------
# input generator
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    # Random123 known-answer vectors for philox4x32-10
    cases = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, want in cases:
        got = philox4x32(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(x) for x in got] == want


def test_rambo_invariants():
    for proc, rs in [("ee_uug", 1000.0), ("gg_ttg", (400.0, 2000.0)), ("gg_ttgg", (400.0, 2000.0))]:
        mom, w = events(proc, 4096, rs, stream=9)
        ptot = mom[0] + mom[1] - mom[2:].sum(axis=0)
        scale = mom[0, 0] + mom[1, 0]
        assert np.max(np.abs(ptot) / scale) < 1e-13
        m2 = mom[:, 0] ** 2 - (mom[:, 1:] ** 2).sum(axis=1)
        for k, name in enumerate(["t", "t~"] if proc.startswith("gg") else []):
            assert np.max(np.abs(m2[2 + k] - M_TOP ** 2)) < 1e-8 * M_TOP ** 2
    # massless 3-body weight is the constant volume s/(256 pi^3)
    _, w = events("ee_uug", 64, 1000.0, stream=9)
    assert np.allclose(w, 1000.0 ** 2 / (256 * math.pi ** 3), rtol=1e-13)
    assert abs(massless_volume(2, 1.0) - 1 / (8 * math.pi)) < 1e-16
    # 2-body massive weight = beta / (8 pi)
    mom, w = events("gg_tt", 64, 500.0, stream=9)
    beta = math.sqrt(1 - 4 * M_TOP ** 2 / 500.0 ** 2)
    assert np.allclose(w, beta / (8 * math.pi), rtol=1e-12)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
def _stu(mom):
    s = 2 * mdot(mom[0], mom[1])
    t = -2 * mdot(mom[0], mom[2])
    u = -2 * mdot(mom[0], mom[3])
    return s, t, u


def test_ee_mumu_closed_form(orc):
    mom, _ = events("ee_mumu", 1 << 12, 91.188, stream=1)
    s, t, u = _stu(mom)
    cf = 2 * E2 ** 2 * (t ** 2 + u ** 2) / s ** 2
    m = orc.me2("ee_mumu", mom)
    assert np.max(np.abs(m / cf - 1)) < 1e-13
    # raw helicity sum = 4 x the spin average; exactly 4 of 16 helicities nonzero
    hel = orc.me2_hel("ee_mumu", mom[:, :, :64])
    assert np.allclose(hel.sum(axis=0), m[:64], rtol=1e-14)
    nz = np.any(hel != 0.0, axis=1)
    assert nz.sum() == 4
    # massless fermion lines: opposite helicities on each line (all-incoming)
    for h in np.nonzero(nz)[0]:
        lam = [(h >> (3 - k)) & 1 for k in range(4)]
        assert lam[0] != lam[1] and lam[2] != lam[3]


def test_ee_uu_closed_form(orc):
    mom, _ = events("ee_uu", 1 << 12, 1000.0, stream=1)
    s, t, u = _stu(mom)
    cf = 2 * 3 * (2 / 3) ** 2 * E2 ** 2 * (t ** 2 + u ** 2) / s ** 2
    assert np.max(np.abs(orc.me2("ee_uu", mom) / cf - 1)) < 1e-13


def test_ee_uug_closed_form(orc):
    """e+e- -> q qbar g through a photon: per-point form and the exact average
    over the six beam orientations +-x, +-y, +-z (x1^2+x2^2)/((1-x1)(1-x2))."""
    mom, _ = events("ee_uug", 1 << 12, 1000.0, stream=2)
    p1, p2, k1, k2, k3 = mom
    s = 2 * mdot(p1, p2)
    NC, CF, Qu = 3.0, 4.0 / 3.0, 2.0 / 3.0
    num = mdot(p1, k1) ** 2 + mdot(p1, k2) ** 2 + mdot(p2, k1) ** 2 + mdot(p2, k2) ** 2
    cf = 4 * NC * CF * Qu ** 2 * E2 ** 2 * G2 * num / (s * mdot(k1, k3) * mdot(k2, k3))
    m = orc.me2("ee_uug", mom)
    # FP64 conditioning: the propagator denominators k.k3 = E E3 (1 - cos) lose
    # digits for nearly collinear pairs
    kappa = np.maximum(k1[0] * k3[0] / mdot(k1, k3), k2[0] * k3[0] / mdot(k2, k3))
    assert np.all(np.abs(m / cf - 1) < 3e-13 + 2e-15 * kappa)
    # orientation average: rotate the final state so that the beam points
    # along each of the six axes
    sub = mom[:, :, :256]
    acc = np.zeros(sub.shape[2])
    rots = [rotation_matrix([0, 1, 0], 0.0), rotation_matrix([0, 1, 0], math.pi),
            rotation_matrix([0, 1, 0], math.pi / 2), rotation_matrix([0, 1, 0], -math.pi / 2),
            rotation_matrix([1, 0, 0], math.pi / 2), rotation_matrix([1, 0, 0], -math.pi / 2)]
    for R in rots:
        r = sub.copy()
        r[2:] = transform(sub[2:], R)
        acc += orc.me2("ee_uug", r)
    acc /= 6
    rs = math.sqrt(1000.0 ** 2)
    x1 = 2 * sub[2, 0] / rs
    x2 = 2 * sub[3, 0] / rs
    F = (x1 ** 2 + x2 ** 2) / ((1 - x1) * (1 - x2))
    want = (8.0 / 3.0) * NC * CF * Qu ** 2 * E2 ** 2 * G2 * F / 1000.0 ** 2
    assert np.max(np.abs(acc / want - 1)) < 1e-12


def _tau_rho(mom):
    s = 2 * mdot(mom[0], mom[1])
    t1 = 2 * mdot(mom[0], mom[2]) / s
    t2 = 2 * mdot(mom[1], mom[2]) / s
    return t1, t2, 4 * M_TOP ** 2 / s


def test_gg_tt_closed_form(orc):
    mom, _ = events("gg_tt", 1 << 12, (400.0, 2000.0), stream=31)
    t1, t2, rho = _tau_rho(mom)
    cf = G2 ** 2 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))
    assert np.max(np.abs(orc.me2("gg_tt", mom) / cf - 1)) < 1e-12


def test_uu_tt_closed_form(orc):
    mom, _ = events("uu_tt", 1 << 12, (400.0, 2000.0), stream=31)
    t1, t2, rho = _tau_rho(mom)
    cf = G2 ** 2 * (4 / 9) * (t1 ** 2 + t2 ** 2 + rho / 2)
    assert np.max(np.abs(orc.me2("uu_tt", mom) / cf - 1)) < 1e-12


# ---------------------------------------------------------------------------
# brute-force colour-dressed Feynman rules vs colour-ordered recursion
# ---------------------------------------------------------------------------
def test_brute_force_gg_tt_and_gg_ttg(orc):
    for proc, n in [("gg_tt", 8), ("gg_ttg", 3)]:
        mom, _ = events(proc, n, (400.0, 2000.0), stream=77)
        a = orc.me2(proc, mom)
        b = orc.me2_brute(proc, mom)
        assert np.max(np.abs(a / b - 1)) < 1e-12


@pytest.mark.slow
def test_brute_force_gg_ttgg_helicities(orc):
    mom, _ = events("gg_ttgg", 1, (400.0, 2000.0), stream=77)
    hel = orc.me2_hel("gg_ttgg", mom)
    for h in (0, 21, 46):
        b = orc.me2_brute("gg_ttgg", mom, hel=h)
        assert abs(b[0] / hel[h, 0] - 1) < 1e-12


# ---------------------------------------------------------------------------
# colour matrices
# ---------------------------------------------------------------------------
def _rational(x, den=1458):
    return Fraction(round(x * den), den)


def test_colour_matrices(orc):
    C = orc.colour_matrix("gg_tt")
    assert np.allclose(C, [[16 / 3, -2 / 3], [-2 / 3, 16 / 3]], atol=1e-14)
    for proc, n in [("gg_tt", 2), ("gg_ttg", 3), ("gg_ttgg", 4)]:
        C = orc.colour_matrix(proc).real
        assert np.allclose(C, C.T, atol=1e-13)
        assert np.min(np.linalg.eigvalsh(C)) > -1e-12
        # diagonal of a string of n generators: N_c C_F^n
        assert np.allclose(np.diag(C), 3 * (4 / 3) ** n, rtol=1e-13)
        # exact rationals with denominator dividing 2 * 3^6
        for x in C.ravel():
            assert abs(float(_rational(x)) - x) < 1e-12
        # sum over all strings: sum_{sigma,sigma'} C = |sum_sigma T^sigma|^2 is
        # independent of ordering; row sums equal by symmetry of permutations
        rs = C.sum(axis=1)
        assert np.allclose(rs, rs[0], rtol=1e-12)
    # two quark lines exchanging one gluon: sum |T^a_ij T^a_kl|^2 = 2
    assert abs(orc.colour_matrix("uu_tt")[0, 0].real - 2.0) < 1e-14


# ---------------------------------------------------------------------------
# gauge invariance, Lorentz invariance, Bose symmetry, coupling scaling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("proc", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_gauge_invariance_colour_ordered(orc, proc):
    """Each colour-ordered amplitude vanishes when one gluon polarisation is
    replaced by its momentum (Ward identity), for every helicity."""
    mom, _ = events(proc, 3, (400.0, 2000.0), stream=12)
    P = to_aos(mom)
    npart = mom.shape[0]
    gluons = [k for k, c in enumerate(orc.PROCS and ["g"] * npart) if k in (0, 1, 4, 5) and k < npart]
    for e in range(P.shape[0]):
        for h in (0, 5, (1 << npart) - 1):
            ref = np.max(np.abs(orc.flows(proc, P[e], h)))
            for leg in gluons:
                kvec = P[e, leg] / P[e, leg, 0]
                A = orc.flows(proc, P[e], h, override_leg=leg, override_vec=kvec.astype(complex))
                assert np.max(np.abs(A)) < 1e-12 * ref


@pytest.mark.parametrize("proc,leg", [("uu_ttg", 4), ("ug_ttu", 1), ("ee_uug", 4)])
def test_gauge_invariance_diagrams(orc, proc, leg):
    """Diagram amplitudes contracted with the colour matrix: |M|^2 with the
    gluon polarisation replaced by its momentum vanishes."""
    mom, _ = events(proc, 4, (400.0, 2000.0) if proc != "ee_uug" else 1000.0, stream=13)
    P = to_aos(mom)
    K = orc.colour_matrix(proc)
    for e in range(P.shape[0]):
        for h in (0, 9, 22, 31):
            A0 = orc.flows(proc, P[e], h)
            ref = abs(np.conj(A0) @ K @ A0) + np.max(np.abs(A0)) ** 2
            kvec = P[e, leg] / P[e, leg, 0]
            A = orc.flows(proc, P[e], h, override_leg=leg, override_vec=kvec.astype(complex))
            assert abs(np.conj(A) @ K @ A) <= 1e-12 * ref


@pytest.mark.parametrize("proc", ["ee_mumu", "ee_uug", "gg_tt", "uu_tt", "gg_ttg", "uu_ttg", "ug_ttu", "gg_ttgg"])
def test_lorentz_invariance(orc, proc):
    rs = 1000.0 if proc.startswith("ee") else (400.0, 2000.0)
    mom, _ = events(proc, 64, rs, stream=14)
    L = boost_matrix(np.array([0.3, -0.5, 0.6])) @ rotation_matrix([1, 2, 3], 0.7)
    a = orc.me2(proc, mom)
    b = orc.me2(proc, transform(mom, L))
    assert np.max(np.abs(a / b - 1)) < 1e-11


@pytest.mark.parametrize("proc", ["ee_mumu", "ee_uu", "ee_uug", "gg_tt", "uu_tt", "gg_ttg", "uu_ttg", "ug_ttu",
                                  "gg_ttgg"])
def test_helicity_reversal_symmetry(orc, proc):
    """Real vector couplings and no widths: reversing every helicity turns a
    tree amplitude at real momenta into a phase times its complex conjugate,
    so each colour-summed |M_h|^2 equals |M_-h|^2 (the GPU kernels sum one of
    each pair and double it; the oracle sums all helicities)."""
    rs = 1000.0 if proc.startswith("ee") else (400.0, 2000.0)
    mom, _ = events(proc, 48, rs, stream=16)
    ph = orc.me2_hel(proc, mom)
    nh = ph.shape[0]
    assert np.max(ph) > 0
    flip = ph[nh - 1 - np.arange(nh)]
    assert np.max(np.abs(ph - flip) / ph.max(axis=0)) < 1e-12
    # not a tautology: single helicities differ from each other
    assert np.max(np.abs(ph - np.roll(ph, 1, axis=0)) / ph.max(axis=0)) > 1e-3


@pytest.mark.parametrize("proc,swap", [("gg_tt", (0, 1)), ("gg_ttg", (0, 1)), ("gg_ttgg", (0, 1)), ("gg_ttgg", (4, 5))])
def test_bose_symmetry(orc, proc, swap):
    mom, _ = events(proc, 64, (400.0, 2000.0), stream=15)
    sw = mom.copy()
    i, j = swap
    sw[[i, j]] = sw[[j, i]]
    assert np.max(np.abs(orc.me2(proc, mom) / orc.me2(proc, sw) - 1)) < 1e-12


def test_coupling_scaling(orc):
    for proc in ["ee_uug", "gg_ttg", "uu_ttg"]:
        info = orc.proc_info(proc)
        mom, _ = events(proc, 16, (400.0, 2000.0) if proc != "ee_uug" else 1000.0, stream=16)
        a = orc.me2(proc, mom)
        orc.set_params(alpha=2 * ALPHA, alpha_s=2 * ALPHA_S)
        try:
            b = orc.me2(proc, mom)
        finally:
            orc.set_params()
        assert np.allclose(b / a, 2.0 ** (info["a_pow"] + info["as_pow"]), rtol=1e-13)


# ---------------------------------------------------------------------------
# wavefunctions
# ---------------------------------------------------------------------------
def _gammas():
    s = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1, -1])]
    G = [np.block([[np.zeros((2, 2)), s[0]], [s[0], np.zeros((2, 2))]])]
    for k in (1, 2, 3):
        G.append(np.block([[np.zeros((2, 2)), s[k]], [-s[k], np.zeros((2, 2))]]))
    return [g.astype(complex) for g in G]


def _slash(G, p):
    return G[0] * p[0] - G[1] * p[1] - G[2] * p[2] - G[3] * p[3]


def test_spinor_and_polarisation_identities(orc):
    G = _gammas()
    mom, _ = events("gg_tt", 8, (400.0, 2000.0), stream=17)
    P = to_aos(mom)
    for e in range(P.shape[0]):
        p = P[e, 2]
        m = M_TOP
        # leg 2 is an outgoing top: row spinor ubar; u = gamma0 ubar^dagger
        us = [G[0] @ np.conj(orc.wavefunction("gg_tt", P[e], 2, lam)) for lam in (-1, 1)]
        for u in us:
            assert np.max(np.abs((_slash(G, p) - m * np.eye(4)) @ u)) < 1e-10 * p[0]
        S = sum(np.outer(u, np.conj(u) @ G[0]) for u in us)
        assert np.max(np.abs(S - (_slash(G, p) + m * np.eye(4)))) < 1e-10 * p[0]
        # leg 3 is an outgoing antitop: column spinor v
        pv = P[e, 3]
        vs = [orc.wavefunction("gg_tt", P[e], 3, lam) for lam in (-1, 1)]
        for v in vs:
            assert np.max(np.abs((_slash(G, pv) + m * np.eye(4)) @ v)) < 1e-10 * pv[0]
        S = sum(np.outer(v, np.conj(v) @ G[0]) for v in vs)
        assert np.max(np.abs(S - (_slash(G, pv) - m * np.eye(4)))) < 1e-10 * pv[0]
        # incoming gluon polarisations: transverse, normalised, complete
        k = P[e, 0]
        eps = [orc.wavefunction("gg_tt", P[e], 0, lam) for lam in (-1, 1)]
        for ep in eps:
            assert abs(mdot(ep, k)) < 1e-12 * k[0]
            assert abs(mdot(ep, np.conj(ep)) + 1) < 1e-14
        assert abs(mdot(eps[0], np.conj(eps[1]))) < 1e-14
    # massless spinors carry exact structural zeros
    mom, _ = events("uu_tt", 4, 1000.0, stream=17)
    P = to_aos(mom)
    u_plus = orc.wavefunction("uu_tt", P[0], 0, +1)
    u_minus = orc.wavefunction("uu_tt", P[0], 0, -1)
    assert np.all(u_plus[:2] == 0) and np.all(u_minus[2:] == 0)
