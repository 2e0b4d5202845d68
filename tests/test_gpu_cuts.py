"""Device cuts (nlo_cut_mask, nlo_fks_cut_masks) and Algorithm 2's
regenerate-until-pass loop as stream compaction (nlo_generate_passing),
through the C ABI, against the oracle's cut predicates (oracle/cuts.py).

A cut decision is an integer decided by floating point: both sides take it in
FP64 with the same formulas, and the masks must agree bit for bit except on
events where the oracle finds a comparison within 1e-9 (relative) of a tie
(counted and printed; none may disagree elsewhere).  The compaction must
reproduce the batch recipe's candidates that pass, in candidate order, with
the exact trial count, and not depend on how the candidates were chunked."""
import math

import numpy as np
import pytest

from nlo_inputs.workloads import events, fks_variables
from oracle import cuts as oc

pytestmark = pytest.mark.gpu

OFF = 1e300
CUTS = {
    "ee_mumu": dict(jet_r=0.4, jet_ptmin=0.0, jet_ymax=OFF, njet_min=0, top_ptmin=0.0, top_ymax=OFF,
                    lep_ptmin=25.0, lep_ymax=1.5),
    "ee_uug": dict(jet_r=0.4, jet_ptmin=100.0, jet_ymax=1.5, njet_min=3, top_ptmin=0.0, top_ymax=OFF,
                   lep_ptmin=0.0, lep_ymax=OFF),
    "gg_tt": dict(jet_r=0.4, jet_ptmin=0.0, jet_ymax=OFF, njet_min=0, top_ptmin=100.0, top_ymax=2.0,
                  lep_ptmin=0.0, lep_ymax=OFF),
    "gg_ttg": dict(jet_r=0.5, jet_ptmin=40.0, jet_ymax=2.0, njet_min=1, top_ptmin=50.0, top_ymax=2.5,
                   lep_ptmin=0.0, lep_ymax=OFF),
    "gg_ttgg": dict(jet_r=0.6, jet_ptmin=40.0, jet_ymax=2.5, njet_min=2, top_ptmin=0.0, top_ymax=OFF,
                    lep_ptmin=0.0, lep_ymax=OFF),
}
RS = {"ee_mumu": 91.188, "ee_uug": 1000.0}


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _agree(dev, ref, hit, what):
    bad = (dev != ref) & ~hit
    print("%s: pass %.3f, ties %d, disagreements %d (all at ties: %s)" % (
        what, ref.astype(bool).mean() if ref.dtype == bool else (ref != 0).mean(), hit.sum(), (dev != ref).sum(),
        not bad.any()), flush=True)
    assert not bad.any()
    assert hit.mean() < 0.01


@pytest.mark.parametrize("proc", ["ee_mumu", "ee_uug", "gg_tt", "gg_ttg", "gg_ttgg"])
def test_cut_mask_matches_oracle(gpu, proc):
    import torch
    n = 1999
    mom, _ = events(proc, n, RS.get(proc, (400.0, 2000.0)), stream=501)
    ref, hit = oc.cut_mask(proc, mom, CUTS[proc])
    got = gpu.cut_mask(proc, torch.from_numpy(mom).cuda(), CUTS[proc])
    torch.cuda.synchronize()
    _agree(got.cpu().numpy().astype(bool), ref, hit, "cut mask " + proc)
    assert 0.05 < ref.mean() < 0.97


# (real, i, j, Born, sqrt(s), cuts): rapidity cuts make the beams' two collinear ends differ
FKS_CASES = [
    ("ee_uug", 4, 2, "ee_uu", 1000.0, dict(CUTS["ee_uug"], njet_min=2)),
    ("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0), dict(CUTS["gg_tt"], top_ymax=0.8)),
    ("uu_ttg", 4, -1, "uu_tt", (400.0, 2000.0), dict(CUTS["gg_tt"], top_ymax=0.8)),
    ("ug_ttu", 4, -1, "gg_tt", (400.0, 2000.0), dict(CUTS["gg_ttg"], njet_min=0, top_ymax=0.8)),
    ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0), CUTS["gg_ttg"]),
    ("gg_ttgg", 5, -1, "gg_ttg", (400.0, 2000.0), dict(CUTS["gg_ttg"], jet_ymax=1.0)),
]


@pytest.mark.parametrize("case", FKS_CASES, ids=["%s_%d_%d" % c[:3] for c in FKS_CASES])
def test_fks_cut_masks_match_oracle(gpu, orc, case):
    import torch
    real, i, j, born, rs, cuts = case
    n = 777
    mom, _ = events(born, n, rs, stream=502)
    xt, y, phi = fks_variables(n, stream=502, initial_state=j < 0)
    ref, hit = oc.fks_masks(orc, real, i, j, born, mom, xt, y, phi, cuts)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    got = gpu.fks_cut_masks(real, i, j, t(mom), t(xt), t(y), t(phi), cuts).cpu().numpy()
    for a, name in enumerate("BRSC"):
        _agree(got[a], ref[a], hit, "%s (%d,%d) mask %s" % (real, i, j, name))
    if real == "gg_ttgg" and j < 0:     # the two collinear ends differ somewhere on this set
        assert np.any((ref[3] & 4) != ((ref[3] & 8) >> 1))


def test_subtracted_reads_the_device_masks(gpu, orc):
    """nlo_subtracted with the device masks: each term zeroed exactly where its
    mask (for the beams, its collinear end) fails, W as with the oracle's
    masks; and near a collinear end the real mask agrees with that end's."""
    import torch
    real, i, j, born, rs, cuts = FKS_CASES[5]
    n = 600
    mom, _ = events(born, n, rs, stream=503)
    xt, y, phi = fks_variables(n, stream=503, initial_state=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    M, X, Y, P = t(mom), t(xt), t(y), t(phi)
    dm = gpu.fks_cut_masks(real, i, j, M, X, Y, P, cuts)
    ref, hit = oc.fks_masks(orc, real, i, j, born, mom, xt, y, phi, cuts)
    full = gpu.subtracted(real, i, j, M, X, Y, P, prec="fp64")
    got = gpu.subtracted(real, i, j, M, X, Y, P, prec="fp64", mask=dm)
    via_oracle = gpu.subtracted(real, i, j, M, X, Y, P, prec="fp64", mask=t(ref))
    torch.cuda.synchronize()
    m = dm.cpu().numpy()
    cp, cm = (m[3] & 4) != 0, (m[3] & 8) != 0
    g = {k: got[k].cpu().numpy() for k in ("born", "g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm", "W")}
    f = {k: full[k].cpu().numpy() for k in g}
    for key, keep in (("born", m[0] == 1), ("g_R", m[1] == 1), ("g_S", m[2] == 1), ("g_C", cp), ("g_Cm", cm),
                      ("g_SC", (m[2] == 1) & cp), ("g_SCm", (m[2] == 1) & cm)):
        assert np.all(g[key][~keep] == 0.0), key
        assert np.array_equal(g[key][keep], f[key][keep]), key
    same = ~hit
    assert np.array_equal(g["W"][same], via_oracle["W"].cpu().numpy()[same])
    # IR consistency: at 1 - |y| = 1e-10 the real point sits at the collinear end
    yy = np.where(y > 0, 1 - 1e-10, -1 + 1e-10)
    dn = gpu.fks_cut_masks(real, i, j, M, X, t(yy), P, cuts).cpu().numpy()
    end = np.where(yy > 0, (dn[3] & 4) != 0, (dn[3] & 8) != 0)
    _, hn = oc.fks_masks(orc, real, i, j, born, mom, xt, yy, phi, cuts)
    assert np.array_equal((dn[1] == 1)[~hn], end[~hn])


@pytest.mark.parametrize("proc", ["ee_mumu", "gg_tt", "gg_ttg"])
def test_generate_passing_matches_recipe(gpu, proc):
    """The outputs are the recipe's candidates that pass, in candidate order,
    and the trial count is one past the n-th of them."""
    import torch
    n, first = 1000, 12345
    rs = RS.get(proc, (400.0, 2000.0))
    mom, w, trials = gpu.generate_passing(proc, n, rs, 504, CUTS[proc], first=first)
    torch.cuda.synchronize()
    cand, cw = events(proc, trials + 200, rs, stream=504, first=first)
    ok, hit = oc.cut_mask(proc, cand, CUTS[proc])
    upto = np.nonzero(ok)[0]
    print("%s: acceptance %.3f, trials %d, ties among the candidates %d" % (proc, n / trials, trials, hit.sum()),
          flush=True)
    assert not hit[:trials].any()
    assert len(upto) >= n and upto[n - 1] + 1 == trials
    sel = upto[:n]
    scale = np.max(np.abs(cand[:, 0, sel]))
    assert np.allclose(mom.cpu().numpy(), cand[:, :, sel], rtol=0, atol=1e-12 * scale)
    assert np.allclose(w.cpu().numpy(), cw[sel], rtol=1e-12, atol=0)
    # a longer run starts with the same points (chunking does not matter)
    mom2, w2, t2 = gpu.generate_passing(proc, 3 * n, rs, 504, CUTS[proc], first=first)
    torch.cuda.synchronize()
    assert torch.equal(mom2[:, :, :n], mom) and torch.equal(w2[:n], w) and t2 > trials


def test_generate_passing_full_size(gpu):
    """2^20 passing g g -> t tbar g points over several chunks: every output
    passes the device cut mask, conserves momentum, and the first 4096 equal a
    short run's."""
    import torch
    n = 1 << 20
    mom, w, trials = gpu.generate_passing("gg_ttg", n, (400.0, 2000.0), 505, CUTS["gg_ttg"])
    torch.cuda.synchronize()
    print("gg_ttg 2^20 passing points: %d candidates (acceptance %.3f)" % (trials, n / trials), flush=True)
    assert trials > n and torch.all(w > 0)
    assert torch.all(gpu.cut_mask("gg_ttg", mom, CUTS["gg_ttg"]) == 1)
    tot = mom[2:].sum(dim=0) - mom[0] - mom[1]
    assert float(tot.abs().max()) < 1e-9 * 2000.0
    short, ws, ts = gpu.generate_passing("gg_ttg", 4096, (400.0, 2000.0), 505, CUTS["gg_ttg"])
    assert torch.equal(short, mom[:, :, :4096]) and ts < trials


def test_cross_section_over_the_cut_region(gpu, orc):
    """(1/trials) sum w |M|^2 / (2 s) over the passing points equals the
    oracle's plain Monte Carlo over all candidates with its cut mask."""
    import torch
    proc, n = "gg_tt", 4000
    mom, w, trials = gpu.generate_passing(proc, n, 800.0, 506, CUTS[proc])
    me = gpu.me2(proc, mom, "fp64")
    torch.cuda.synchronize()
    s = 800.0 ** 2
    dev = float((w * me).sum()) / (2 * s) / trials
    cand, cw = events(proc, trials, 800.0, stream=506)
    ok, _ = oc.cut_mask(proc, cand, CUTS[proc])
    ref = float(np.sum(cw[ok] * orc.me2(proc, np.ascontiguousarray(cand[:, :, ok])))) / (2 * s) / trials
    print("sigma over the cut region: device %.12e oracle %.12e" % (dev, ref), flush=True)
    assert abs(dev / ref - 1) < 1e-11


def test_cut_argument_errors(gpu):
    import torch
    import paper_2503_07439_amd as nl
    m = torch.zeros((4, 4, 8), dtype=torch.float64, device="cuda")
    for bad in (dict(jet_r=0.0), dict(jet_r=float("nan")), dict(njet_min=-1), dict(top_ptmin=float("nan"))):
        with pytest.raises(nl.NloError) as e:
            gpu.cut_mask("gg_tt", m, dict(CUTS["gg_tt"], **bad))
        assert e.value.status == 1
    z = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NloError) as e:
        gpu.fks_cut_masks("gg_ttg", 4, 2, m, z, z, z, CUTS["gg_tt"])
    assert e.value.status == 5
    # cuts nothing can pass: the loop gives up
    with pytest.raises(nl.NloError) as e:
        gpu.generate_passing("ee_mumu", 10, 91.188, 507, dict(CUTS["ee_mumu"], lep_ptmin=50.0))
    assert e.value.status == 1
    with pytest.raises(nl.NloError) as e:
        gpu.generate_passing("gg_tt", 10, (300.0, 400.0), 507, CUTS["gg_tt"])   # below 2 m_t
    assert e.value.status == 1
