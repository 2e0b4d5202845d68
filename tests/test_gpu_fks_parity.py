"""Parity of the GPU FKS-subtracted real emission (through the C ABI) with the
binary128 oracle, event by event, on seeded Born points and radiation
variables with xi_tilde and 1-|y| log-uniform in [1e-6, 1].

W = (g_R - counterterms) / kappa, kappa = xi (1-y) for a final-state emitter
and xi (1-y^2) for the beams, is a difference of terms that each grow like
1/kappa.  Its rounding error is bounded against the size of the terms it
cancels, D = sum|g_X| / kappa, with no further power of kappa:

  FP64 : every g_X within 1e-12 sum|g_X|;  |dW| <= 1e-12 (|W| + D).
         (Measured: at most 3.3e-13 sum|g_X|, the rounding of the real
         |M|^2; counterterms within 1.2e-13.)
  MIXED: FP32 where kappa >= 0.1, FP64 below: |dW| <= 1e-3 |W| on every
         FP32-routed event (measured <= 1.5e-5), the FP64 bound on the others;
         an FP32 event whose W comes out unresolved is evaluated again in
         FP64 (status bits 1 and 4), so MIXED flags bit 3 exactly where FP64
         does.
  FP32 : all events in FP32: |dW| <= 1e-3 D (FP32 is accurate only away
         from the limits; MIXED is the mode for near-singular sets).
Every event without status bit 3 (W resolved in its precision) is within
1e-3 |W|.  The sum of W is checked against the sum of the per-event bounds:
on these log-uniform sets it is dominated by the deepest events (|W| grows
like 1/sqrt(1-|y|)), where FP64 leaves W only about 1e-4 relative, so the
sum keeps about 1e-5 relative; its error is printed."""
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
IDS = ["%s_%d_%d" % s[:3] for s in SECTORS]
THR = 0.1                 # default MIXED routing threshold on kappa

_REF = {}


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _inputs(sector, n, stream, spread="log"):
    real, i, j, born, rs = sector
    mom, _ = events(born, n, rs, stream=stream)
    xt, y, phi = fks_variables(n, stream=stream, initial_state=(j < 0), spread=spread)
    return mom, xt, y, phi


def _ref(orc, sector, n, stream, spread="log"):
    """binary128 oracle on the sector's inputs (cached per module)"""
    key = (sector, n, stream, spread)
    if key not in _REF:
        real, i, j = sector[:3]
        mom, xt, y, phi = _inputs(sector, n, stream, spread)
        _REF[key] = orc.fks(real, i, j, mom, xt, y, phi, want_real=True, kind="quad")
    return _REF[key]


def _gpu_run(gpu, sector, mom, xt, y, phi, prec, mask=None, want_sum=False):
    import torch
    real, i, j = sector[:3]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    res = gpu.subtracted(real, i, j, t(mom), t(xt), t(y), t(phi), prec=prec,
                         mask=None if mask is None else t(mask), want_real=True, want_sum=want_sum)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _terms(r):
    return (np.abs(r["g_R"]) + np.abs(r["g_S"]) + np.abs(r["g_C"]) + np.abs(r["g_SC"])
            + np.abs(r["g_Cm"]) + np.abs(r["g_SCm"]))


def _kappa(r, j):
    return r["xi"] * ((1 - r["y"]) if j >= 0 else (1 - r["y"]) * (1 + r["y"]))


def _n(sector):
    return 96 if sector[0] == "gg_ttgg" else 400


@pytest.mark.parametrize("sector", SECTORS, ids=IDS)
def test_fks_fp64_parity(gpu, orc, sector):
    real, i, j = sector[:3]
    n = _n(sector)
    mom, xt, y, phi = _inputs(sector, n, 201)
    ref = _ref(orc, sector, n, 201)
    got = _gpu_run(gpu, sector, mom, xt, y, phi, "fp64")
    scale = mom[0, 0] + mom[1, 0]
    assert np.max(np.abs(got["real_mom"] - ref["real_mom"])) < 1e-11 * scale.max()
    assert np.allclose(got["xi"], ref["xi"], rtol=1e-14)
    terms = _terms(ref)
    for key in ("g_R", "g_S", "g_C", "g_SC") + (("g_Cm", "g_SCm") if j < 0 else ()):
        r = ref[key]
        zero = r == 0.0                       # e.g. no soft term for a quark FKS parton
        assert np.all(got[key][zero] == 0.0), key
        d = np.abs(got[key] - r) / terms
        print(key, "max |d|/sum|g| %.2e" % d.max(), flush=True)
        assert np.all(d <= 1e-12), key
    assert np.allclose(got["born"], ref["B"], rtol=1e-12, atol=0)
    D = terms / _kappa(ref, j)
    dW = np.abs(got["W"] - ref["W"])
    rel = dW / np.abs(ref["W"])
    unres = (got["status"] & 8) != 0
    print(real, i, j, "fp64 |dW|/D max %.2e; |dW|/|W| median %.2e max %.2e; unresolved %.3f" % (
        np.max(dW / D), np.median(rel), rel.max(), unres.mean()), flush=True)
    bound = 1e-12 * (np.abs(ref["W"]) + D)
    assert np.all(dW <= bound)
    assert np.all(rel[~unres] <= 1e-3)
    assert np.all(got["status"] & 2)            # every event evaluated in FP64
    assert not np.any(got["status"] & 1)


@pytest.mark.parametrize("sector", SECTORS, ids=IDS)
def test_fks_mixed_parity(gpu, orc, sector):
    real, i, j = sector[:3]
    n = _n(sector)
    mom, xt, y, phi = _inputs(sector, n, 201)
    ref = _ref(orc, sector, n, 201)
    got = _gpu_run(gpu, sector, mom, xt, y, phi, "mixed", want_sum=True)
    D = _terms(ref) / _kappa(ref, j)
    dW = np.abs(got["W"] - ref["W"])
    rel = dW / np.abs(ref["W"])
    routed = (got["status"] & 2) != 0
    redone = (got["status"] & 16) != 0
    unres = (got["status"] & 8) != 0
    kap = got["xi"] * ((1 - y) if j >= 0 else (1 - y) * (1 + y))
    # routing: FP64 exactly below the threshold (kappa as the kernel forms it
    # may differ in the last bit near the threshold), plus the re-evaluated
    near = np.abs(kap / THR - 1) < 1e-12
    assert np.array_equal((routed & ~redone)[~near], kap[~near] < THR)
    assert np.all(routed[redone]) and not np.any(redone & (kap < THR) & ~near)
    fp64 = _gpu_run(gpu, sector, mom, xt, y, phi, "fp64")
    assert np.array_equal(unres, (fp64["status"] & 8) != 0)
    assert np.array_equal(got["W"][routed], fp64["W"][routed])
    print(real, i, j, "mixed: routed %.3f (re-evaluated %.3f), FP32 |dW|/|W| max %.2e, unresolved %.3f, "
          "all |dW|/|W| p99.9 %.2e" % (routed.mean(), redone.mean(), rel[~routed].max() if np.any(~routed) else 0.0,
                                       unres.mean(), np.quantile(rel, 0.999)), flush=True)
    bound = np.where(routed, 1e-12 * (np.abs(ref["W"]) + D), 1e-3 * np.abs(ref["W"]))
    assert np.all(dW <= bound)
    assert np.all(rel[~unres] <= 1e-3)
    dsum = abs(got["w_sum"][0] - ref["W"].sum())
    print("   sum W relative error %.2e (of sum|W|)" % (dsum / np.abs(ref["W"]).sum()), flush=True)
    assert dsum <= bound.sum()
    assert not np.any(got["status"] & 1)


@pytest.mark.parametrize("sector", [SECTORS[0], SECTORS[2], SECTORS[4], SECTORS[6]], ids=lambda s: "%s_%d_%d" % s[:3])
def test_fks_mixed_parity_flat(gpu, orc, sector):
    """MIXED on radiation variables drawn flat over the radiation phase space,
    where most events sit away from the limits and run in FP32: the same
    bounds as on the stress sets (1e-3 |W| where FP32 resolves W, the FP64
    bound on the events routed to FP64 or evaluated again there)."""
    real, i, j = sector[:3]
    n = _n(sector)
    mom, xt, y, phi = _inputs(sector, n, 205, "flat")
    ref = _ref(orc, sector, n, 205, "flat")
    got = _gpu_run(gpu, sector, mom, xt, y, phi, "mixed", want_sum=True)
    D = _terms(ref) / _kappa(ref, j)
    dW = np.abs(got["W"] - ref["W"])
    rel = dW / np.abs(ref["W"])
    routed = (got["status"] & 2) != 0
    redone = (got["status"] & 16) != 0
    unres = (got["status"] & 8) != 0
    kap = got["xi"] * ((1 - y) if j >= 0 else (1 - y) * (1 + y))
    near = np.abs(kap / THR - 1) < 1e-12
    assert np.array_equal((routed & ~redone)[~near], kap[~near] < THR)
    print(real, i, j, "flat mixed: routed %.3f (re-evaluated %.3f), FP32 |dW|/|W| max %.2e, |dW|/D max %.2e, "
          "unresolved %.3f" % (routed.mean(), redone.mean(), rel[~routed].max(), (dW / D)[~routed].max(),
                               unres.mean()), flush=True)
    assert routed.mean() < 0.5                  # most of a flat set runs in FP32
    assert not np.any(unres & ~routed)          # an unresolved FP32 W was evaluated again
    fp32_bound = np.where(unres, 1e-3 * D, 1e-3 * np.abs(ref["W"]))
    bound = np.where(routed, 1e-12 * (np.abs(ref["W"]) + D), fp32_bound)
    assert np.all(dW <= bound)
    assert np.all(rel[~unres] <= 1e-3)
    assert abs(got["w_sum"][0] - ref["W"].sum()) <= bound.sum()
    assert not np.any(got["status"] & 1)


@pytest.mark.parametrize("sector", SECTORS, ids=IDS)
def test_fks_fp32(gpu, orc, sector):
    real, i, j = sector[:3]
    n = _n(sector)
    mom, xt, y, phi = _inputs(sector, n, 201)
    ref = _ref(orc, sector, n, 201)
    got = _gpu_run(gpu, sector, mom, xt, y, phi, "fp32")
    D = _terms(ref) / _kappa(ref, j)
    dW = np.abs(got["W"] - ref["W"])
    rel = dW / np.abs(ref["W"])
    unres = (got["status"] & 8) != 0
    print(real, i, j, "fp32 |dW|/D max %.2e, unresolved %.3f" % (np.max(dW / D), unres.mean()), flush=True)
    assert np.all(dW <= 1e-3 * D)
    assert np.all(rel[~unres] <= 1e-3)
    assert not np.any(got["status"] & 2)


def test_fks_masks_and_sum(gpu, orc):
    sector = SECTORS[2]
    n = 300
    mom, xt, y, phi = _inputs(sector, n, 203)
    rng = np.random.default_rng(9)
    mask = (rng.uniform(size=(4, n)) > 0.3).astype(np.uint8)
    full = _gpu_run(gpu, sector, mom, xt, y, phi, "fp64")
    got = _gpu_run(gpu, sector, mom, xt, y, phi, "fp64", mask=mask, want_sum=True)
    for a, key in ((0, "born"), (1, "g_R"), (2, "g_S"), (3, "g_C")):
        assert np.all(got[key][mask[a] == 0] == 0.0)
        assert np.array_equal(got[key][mask[a] == 1], full[key][mask[a] == 1])
    sc_ok = (mask[2] == 1) & (mask[3] == 1)
    assert np.all(got["g_SC"][~sc_ok] == 0.0)
    assert np.array_equal(((got["status"] & 4) != 0), ~np.all(mask == 1, axis=0))
    # fixed-order FP64 sum of W
    assert abs(got["w_sum"][0] - got["W"].sum()) <= 1e-12 * np.abs(got["W"]).sum()
    # repeated evaluation is bitwise identical (bucket order is not)
    again = _gpu_run(gpu, sector, mom, xt, y, phi, "fp64", mask=mask, want_sum=True)
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


@pytest.mark.parametrize("spread", ["log", "flat"])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("sector", [SECTORS[0], SECTORS[2], SECTORS[4], SECTORS[8]], ids=lambda s: "%s_%d_%d" % s[:3])
def test_fks_compact_masks_bitwise(gpu, sector, prec, spread):
    """Compact mode (events failing the R cut skip the real |M|^2) gives
    bit for bit the results of the branch-free mode, also where MIXED
    evaluates FP32 events again in FP64 (frequent on the flat sets)."""
    n = 500 if sector[0] != "gg_ttgg" else 120
    mom, xt, y, phi = _inputs(sector, n, 204, spread)
    rng = np.random.default_rng(11)
    mask = (rng.uniform(size=(4, n)) > np.array([[0.1], [0.5], [0.1], [0.1]])).astype(np.uint8)
    ref = _gpu_run(gpu, sector, mom, xt, y, phi, prec, mask=mask, want_sum=True)
    gpu.set_fks_mask_mode(True)
    try:
        got = _gpu_run(gpu, sector, mom, xt, y, phi, prec, mask=mask, want_sum=True)
    finally:
        gpu.set_fks_mask_mode(False)
    for k in ("W", "xi", "born", "g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm", "status", "real_mom", "w_sum"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.all(got["g_R"][mask[1] == 0] == 0.0)
