"""Parity of the GPU FKS-subtracted real emission (through the C ABI) with
the FP64 oracle, event by event, on seeded Born points and radiation
variables with xi_tilde and 1-|y| log-uniform in [1e-6, 1].

The subtracted weight W is a difference of terms that each grow like
1/(xi (1-y)) near the limits, so its error is bounded relative to the
conditioning scale  D = (|g_R| + |g_S| + |g_C| + |g_SC| + ...)/(xi (1-y)).
Near the limits the real matrix element itself is ill-conditioned in FP64:
its smallest invariant (2 k_i.k_j for a final-state emitter, 2 p_a.k_i for
a beam) is of order xi (1-|y|) s but is formed from momentum components of
order sqrt(s), so any two FP64 codes agree on it, and on g_R, only to about
eps/kappa with kappa = xi (1-|y|).  Bounds:
  FP64 : terms g_X relative 1e-13/kappa;  |dW| <= 1e-13 D/kappa
  FP32 : |dW| <= 1e-4 D   (float amplitudes, FP64 denominators)
  MIXED: |dW| <= 1e-4 D, and the FP64-routed events as FP64
The plain relative error |dW|/|W| is printed for the record."""
import numpy as np
import pytest

from nlo_inputs.workloads import events, fks_variables

pytestmark = pytest.mark.gpu

SECTORS = [
    ("ee_uug", 4, 2, "ee_uu", 1000.0),
    ("ee_uug", 4, 3, "ee_uu", 1000.0),
    ("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0)),
    ("uu_ttg", 4, -1, "uu_tt", (400.0, 2000.0)),
    ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 5, 4, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 4, -1, "gg_ttg", (400.0, 2000.0)),
    ("gg_ttgg", 5, -1, "gg_ttg", (400.0, 2000.0)),
    ("ug_ttu", 4, -1, "gg_tt", (400.0, 2000.0)),      # quark FKS parton: Born flavour changes
]


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _inputs(real, j, born, rs, n, stream):
    mom, _ = events(born, n, rs, stream=stream)
    xt, y, phi = fks_variables(n, stream=stream, initial_state=(j < 0))
    return mom, xt, y, phi


def _gpu_run(gpu, real, i, j, mom, xt, y, phi, prec, mask=None, want_sum=False):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    res = gpu.subtracted(real, i, j, t(mom), t(xt), t(y), t(phi), prec=prec,
                         mask=None if mask is None else t(mask), want_real=True, want_sum=want_sum)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _scale(r, j):
    terms = np.abs(r["g_R"]) + np.abs(r["g_S"]) + np.abs(r["g_C"]) + np.abs(r["g_SC"])
    if j < 0:
        terms = terms + np.abs(r["g_Cm"]) + np.abs(r["g_SCm"])
        return terms / (r["xi"] * (1 - r["y"]) * (1 + r["y"]))
    return terms / (r["xi"] * (1 - r["y"]))


@pytest.mark.parametrize("real,i,j,born,rs", SECTORS)
def test_fks_fp64_parity(gpu, orc, real, i, j, born, rs):
    n = 400 if real != "gg_ttgg" else 96
    mom, xt, y, phi = _inputs(real, j, born, rs, n, 201)
    ref = orc.fks(real, i, j, mom, xt, y, phi, want_real=True)
    got = _gpu_run(gpu, real, i, j, mom, xt, y, phi, "fp64")
    scale = mom[0, 0] + mom[1, 0]
    assert np.max(np.abs(got["real_mom"] - ref["real_mom"])) < 1e-11 * scale.max()
    assert np.allclose(got["xi"], ref["xi"], rtol=1e-14)
    kappa = ref["xi"] * (1 - np.abs(ref["y"]))
    for key in ("born", "g_R", "g_S", "g_C", "g_SC") + (("g_Cm", "g_SCm") if j < 0 else ()):
        r = ref[key if key != "born" else "B"]
        zero = r == 0.0                       # e.g. no soft term for a quark FKS parton
        assert np.all(got[key][zero] == 0.0), key
        d = np.abs(got[key][~zero] - r[~zero]) / np.abs(r[~zero])
        if d.size:
            print(key, "max rel*kappa %.2e" % np.max(d * kappa[~zero]), flush=True)
        assert np.all(d <= 1e-13 / kappa[~zero]), key
    D = _scale(ref, j)
    dW = np.abs(got["W"] - ref["W"])
    print(real, i, j, "fp64 |dW|/D*kappa max %.2e, |dW|/|W| median %.2e max %.2e" % (
        np.max(dW / D * kappa), np.median(dW / np.abs(ref["W"])), np.max(dW / np.abs(ref["W"]))), flush=True)
    assert np.all(dW <= 1e-13 * D / kappa)
    assert np.all(got["status"] & 2)            # every event evaluated in FP64
    assert not np.any(got["status"] & 1)


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
@pytest.mark.parametrize("real,i,j,born,rs", SECTORS)
def test_fks_reduced_precision(gpu, orc, real, i, j, born, rs, prec):
    n = 400 if real != "gg_ttgg" else 96
    mom, xt, y, phi = _inputs(real, j, born, rs, n, 202)
    ref = orc.fks(real, i, j, mom, xt, y, phi)
    got = _gpu_run(gpu, real, i, j, mom, xt, y, phi, prec)
    D = _scale(ref, j)
    dW = np.abs(got["W"] - ref["W"])
    rel = dW / np.abs(ref["W"])
    routed = (got["status"] & 2) != 0
    print(real, i, j, prec, "routed %.2f |dW|/D max %.2e, |dW|/|W| median %.2e p99 %.2e" % (
        routed.mean(), np.max(dW / D), np.median(rel), np.quantile(rel, 0.99)), flush=True)
    assert np.all(dW <= 1e-4 * D)
    if prec == "mixed":
        dist = np.minimum(ref["xi"], 1 - np.abs(ref["y"]))
        kappa = ref["xi"] * (1 - np.abs(ref["y"]))
        assert np.array_equal(routed, dist < 1e-4)
        assert np.all(dW[routed] <= 1e-13 * D[routed] / kappa[routed])
    else:
        assert not np.any(routed)


def test_fks_masks_and_sum(gpu, orc):
    real, i, j, born, rs = SECTORS[2]
    n = 300
    mom, xt, y, phi = _inputs(real, j, born, rs, n, 203)
    rng = np.random.default_rng(9)
    mask = (rng.uniform(size=(4, n)) > 0.3).astype(np.uint8)
    full = _gpu_run(gpu, real, i, j, mom, xt, y, phi, "fp64")
    got = _gpu_run(gpu, real, i, j, mom, xt, y, phi, "fp64", mask=mask, want_sum=True)
    for a, key in ((0, "born"), (1, "g_R"), (2, "g_S"), (3, "g_C")):
        assert np.all(got[key][mask[a] == 0] == 0.0)
        assert np.array_equal(got[key][mask[a] == 1], full[key][mask[a] == 1])
    sc_ok = (mask[2] == 1) & (mask[3] == 1)
    assert np.all(got["g_SC"][~sc_ok] == 0.0)
    assert np.array_equal(((got["status"] & 4) != 0), ~np.all(mask == 1, axis=0))
    # fixed-order FP64 sum of W
    assert abs(got["w_sum"][0] - got["W"].sum()) <= 1e-12 * np.abs(got["W"]).sum()
    # repeated evaluation is bitwise identical (bucket order is not)
    again = _gpu_run(gpu, real, i, j, mom, xt, y, phi, "fp64", mask=mask, want_sum=True)
    assert np.array_equal(again["W"], got["W"]) and again["w_sum"][0] == got["w_sum"][0]


def test_fks_argument_errors(gpu):
    import torch
    import paper_2503_07439_amd as nl
    z = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = nl.nlo_fks_out()
    out.W = z.data_ptr()
    with pytest.raises(nl.NloError) as e:      # no such sector
        nl.nlo_subtracted(gpu.ctx, nl.proc_id("gg_ttg"), 4, 2, 1, 1, z.data_ptr(), z.data_ptr(), z.data_ptr(),
                          z.data_ptr(), 0, nl.NLO_FP64, out, 0)
    assert e.value.status == 5
    with pytest.raises(nl.NloError) as e:      # ld < n
        nl.nlo_subtracted(gpu.ctx, nl.proc_id("gg_ttg"), 4, -1, 4, 2, z.data_ptr(), z.data_ptr(), z.data_ptr(),
                          z.data_ptr(), 0, nl.NLO_FP64, out, 0)
    assert e.value.status == 1
    out.W = None
    with pytest.raises(nl.NloError) as e:      # W is required
        nl.nlo_subtracted(gpu.ctx, nl.proc_id("gg_ttg"), 4, -1, 1, 1, z.data_ptr(), z.data_ptr(), z.data_ptr(),
                          z.data_ptr(), 0, nl.NLO_FP64, out, 0)
    assert e.value.status == 1
    with pytest.raises(nl.NloError) as e:
        gpu.set_fks_threshold(2.0)
    assert e.value.status == 1


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("real,i,j,born,rs", [SECTORS[0], SECTORS[2], SECTORS[4], SECTORS[8]])
def test_fks_compact_masks_bitwise(gpu, real, i, j, born, rs, prec):
    """Compact mode (events failing the R cut skip the real |M|^2) gives
    bit for bit the results of the branch-free mode."""
    n = 500 if real != "gg_ttgg" else 120
    mom, xt, y, phi = _inputs(real, j, born, rs, n, 204)
    rng = np.random.default_rng(11)
    mask = (rng.uniform(size=(4, n)) > np.array([[0.1], [0.5], [0.1], [0.1]])).astype(np.uint8)
    ref = _gpu_run(gpu, real, i, j, mom, xt, y, phi, prec, mask=mask, want_sum=True)
    gpu.set_fks_mask_mode(True)
    try:
        got = _gpu_run(gpu, real, i, j, mom, xt, y, phi, prec, mask=mask, want_sum=True)
    finally:
        gpu.set_fks_mask_mode(False)
    for k in ("W", "xi", "born", "g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm", "status", "real_mom", "w_sum"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.all(got["g_R"][mask[1] == 0] == 0.0)
