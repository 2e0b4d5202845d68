"""Device VEGAS integration of the subtracted real emission
(nlo_integrate_subtracted, through the C ABI) against the oracle's integrator
(oracle/vegas.py) on the same seeded points.

Both sides draw the same Philox uniforms, so the VEGAS bins of every point are
identical and only rounding separates the two: the points' coordinates differ
through the grid edges (refined from histograms summed in another order), and
every integrand value through the device's FP64 arithmetic.  The reference is
the oracle in binary128 wherever it finishes in seconds (every process but
g g -> t tbar g g): VEGAS concentrates points at tiny xi (1-y), where the
terms of the subtracted weight cancel by up to 1e8 and the oracle's own double
build is off by up to 5e-10 of the conditioning scale (its real momenta carry
the rounding of their construction; the device forms the FKS-pair invariant
from the map variables instead).

Bars: every iteration's mean within 2e-12 of the mean conditioning scale of
the integrand (the oracle's sum over the counterterms of |j_X g_X| /
(2 s_B kappa)), the device's per-point FP64 bound with a factor 2 for the
coordinates, plus 1e-12 of the estimate; its standard error likewise.  For
g g -> t tbar g g, against the double oracle: every iteration within 1e-6 of
its standard error.  MIXED within 2 % of the standard error of FP64.  Sizes
span several blocks and a ragged tail.  Two device runs with the same seed are
bitwise equal (every reduction has a fixed order).  At the benchmark's size
(2^20 points per iteration, 10 iterations, g g -> t tbar g at sqrt(s_B) = 600
GeV) the result is reproducible, its iterations are consistent (chi^2/dof <
3) and it agrees with a small run within their combined errors."""
import math

import numpy as np
import pytest

from physics import M_TOP

pytestmark = pytest.mark.gpu

SEED = 7439
#        real       Born      sectors                               sqrt(s_B)  masses          n   niter nadapt oracle
CASES = [("ee_uug", "ee_uu", [(4, 2), (4, 3)], 1000.0, [0.0, 0.0], 4096, 4, 2, "quad"),
         ("gg_ttg", "gg_tt", [(4, -1)], 600.0, [M_TOP, M_TOP], 2000, 3, 1, "quad"),
         ("uu_ttg", "uu_tt", [(4, -1)], 600.0, [M_TOP, M_TOP], 2000, 3, 1, "quad"),
         ("ug_ttu", "gg_tt", [(4, -1)], 600.0, [M_TOP, M_TOP], 2000, 3, 1, "quad"),
         ("gg_ttgg", "gg_ttg", [(4, 5), (5, 4), (4, -1), (5, -1)], 800.0, [M_TOP, M_TOP, 0.0], 1000, 3, 1,
          "double")]
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _oracle(orc, case, stream):
    from oracle.vegas import integrate, subtracted_integrand
    real, born, secs, rs, masses, n, niter, nadapt, kind = case
    f = subtracted_integrand(orc, real, secs, born, rs, masses, kind=kind, with_scale=True)
    return integrate(f, 4 * len(masses) + 3, n, niter, nadapt, SEED, stream)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_integrate_matches_oracle(gpu, orc, case):
    real, born, secs, rs, masses, n, niter, nadapt, kind = case
    stream = 300 + IDS.index(real)
    print("integrate %s sqrt(s_B)=%g n=%d niter=%d oracle %s" % (real, rs, n, niter, kind), flush=True)
    ref = _oracle(orc, case, stream)
    got = gpu.integrate_subtracted(real, rs, n, niter, nadapt, stream, "fp64", seed=SEED)
    again = gpu.integrate_subtracted(real, rs, n, niter, nadapt, stream, "fp64", seed=SEED)
    assert got[0] == again[0] and got[1] == again[1] and got[3] == again[3]
    worst = 0.0
    for it, ((gm, ge), (om, oe, cond)) in enumerate(zip(got[3], ref[3])):
        # both sides' FP64 error of every point (1e-12 of its conditioning
        # scale), plus rounding of the sums themselves
        bound = 2e-12 * cond + 1e-12 * (abs(om) + oe) if kind == "quad" else 1e-6 * oe
        worst = max(worst, abs(gm - om) / bound)
        print("  it %d device %.10e +- %.3e oracle %.10e +- %.3e |diff| / bound %.2e (relative %.1e)" % (
            it, gm, ge, om, oe, abs(gm - om) / bound, abs(gm - om) / (abs(om) + oe)), flush=True)
        assert abs(ge - oe) <= bound + 1e-10 * oe
    print("  sigma device %.10e +- %.3e (chi2/dof %.2f) oracle %.10e +- %.3e; worst |diff| / bound %.2e" % (
        got[0], got[1], got[2], ref[0], ref[1], worst), flush=True)
    assert worst <= 1.0
    assert abs(got[0] - ref[0]) < 1e-6 * ref[1]
    mixed = gpu.integrate_subtracted(real, rs, n, niter, nadapt, stream, "mixed", seed=SEED)
    print("  mixed %.10e +- %.3e: |mixed - fp64| / error %.2e" % (mixed[0], mixed[1], abs(mixed[0] - got[0]) / got[1]),
          flush=True)
    assert abs(mixed[0] - got[0]) < 0.02 * got[1]


def test_integrate_full_size(gpu, orc):
    """2^20 points per iteration, 10 iterations: the benchmark's launch
    configuration."""
    n, niter, nadapt = 1 << 20, 10, 3
    print("integrate gg_ttg full size", flush=True)
    a = gpu.integrate_subtracted("gg_ttg", 600.0, n, niter, nadapt, 330, "fp64", seed=SEED)
    b = gpu.integrate_subtracted("gg_ttg", 600.0, n, niter, nadapt, 330, "fp64", seed=SEED)
    assert a == b
    print("  sigma %.8e +- %.3e chi2/dof %.2f; iteration errors %s" % (
        a[0], a[1], a[2], " ".join("%.2e" % e for _, e in a[3])), flush=True)
    assert math.isfinite(a[0]) and a[1] > 0 and a[2] < 3
    assert a[3][-1][1] < a[3][0][1]           # the adapted grid beats the uniform one
    small = gpu.integrate_subtracted("gg_ttg", 600.0, 5000, 4, 2, 301, "fp64", seed=SEED)
    assert abs(a[0] - small[0]) < 4 * math.hypot(a[1], small[1])


def test_integrate_argument_errors(gpu):
    import paper_2503_07439_amd as nl
    bad = [dict(n=1), dict(n=(1 << 20) + 1), dict(niter=0), dict(niter=65), dict(nadapt=3, niter=3),
           dict(nadapt=-1), dict(rs=340.0), dict(rs=float("inf"))]
    for b in bad:
        args = dict(n=1000, niter=3, nadapt=1, rs=600.0)
        args.update(b)
        with pytest.raises(nl.NloError) as e:
            gpu.integrate_subtracted("gg_ttg", args["rs"], args["n"], args["niter"], args["nadapt"], 1, "fp64")
        assert e.value.status == 1, b
    with pytest.raises(nl.NloError) as e:
        gpu.integrate_subtracted("gg_ttg", 600.0, 1000, 3, 1, 1, "fp16")
    assert e.value.status == 5
    with pytest.raises(nl.NloError) as e:
        gpu.integrate_subtracted("gg_tt", 600.0, 1000, 3, 1, 1, "fp64")     # a Born process: no sectors
    assert e.value.status == 5
