"""Partonic cross sections from the oracle against textbook closed forms:
the |M|^2 of these processes are pinned pointwise elsewhere, so these pins
check the phase-space normalisation (RAMBO weights, flux 1/(2s), pb
conversion) that the device cross section relies on.

  e+e- -> mu+mu- (photon):  sigma = 4 pi alpha^2 / (3 s)
  u ubar -> t tbar:         sigma = (8 pi alpha_s^2 / (27 s)) beta (1 + rho/2)
  g g -> t tbar:            sigma = (pi alpha_s^2 / (3 s)) [(1 + rho + rho^2/16) ln((1+beta)/(1-beta))
                                                           - beta (7/4 + 31 rho/16)]
with rho = 4 m^2/s and beta = sqrt(1 - rho) (Combridge 1979)."""
import math

import pytest

from oracle.xs import GEV2_PB, sigma_mc, sigma_quadrature

ALPHA, ALPHA_S, MT = 1.0 / 132.507, 0.118, 173.0


def closed_form(proc, rs):
    s = rs * rs
    if proc == "ee_mumu":
        return 4 * math.pi * ALPHA ** 2 / (3 * s) * GEV2_PB
    rho = 4 * MT * MT / s
    beta = math.sqrt(1 - rho)
    if proc == "uu_tt":
        return 8 * math.pi * ALPHA_S ** 2 / (27 * s) * beta * (1 + rho / 2) * GEV2_PB
    return (math.pi * ALPHA_S ** 2 / (3 * s) * ((1 + rho + rho * rho / 16) * math.log((1 + beta) / (1 - beta))
                                               - beta * (7 / 4 + 31 * rho / 16))) * GEV2_PB


@pytest.mark.parametrize("proc,rs,m", [("ee_mumu", 91.188, 0.0), ("ee_mumu", 500.0, 0.0), ("uu_tt", 400.0, MT),
                                       ("uu_tt", 1500.0, MT), ("gg_tt", 400.0, MT), ("gg_tt", 1500.0, MT)])
def test_quadrature_matches_closed_form(orc, proc, rs, m):
    assert abs(sigma_quadrature(orc, proc, rs, m, m) / closed_form(proc, rs) - 1) < 1e-12


@pytest.mark.parametrize("proc,rs,masses", [("ee_mumu", 500.0, [0.0, 0.0]), ("gg_tt", 800.0, [MT, MT])])
def test_monte_carlo_matches_closed_form(orc, proc, rs, masses):
    mean, err, _ = sigma_mc(orc, proc, rs, masses, 100000, stream=81)
    ref = closed_form(proc, rs)
    assert abs(mean - ref) < 5 * err
    assert err < 0.05 * ref
