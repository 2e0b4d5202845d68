"""FKS subtraction at the full sizes of the FKS workloads, in the
precisions they are specified in (MIXED and FP64), one call per sector over
the whole set: a strided sample of events matches the binary128 oracle to
the bounds of the parity tests (test_gpu_fks_parity), every W is finite, and
MIXED routes exactly the events with kappa < 0.1 to FP64.

  g g -> t tbar g g, sector (4, 5) and (4, beams): 2^18 Born points
  e+e- -> u ubar g, sector (4, 2): 2^16 Born points
"""
import numpy as np
import pytest

from nlo_inputs.workloads import events, fks_variables

pytestmark = pytest.mark.gpu

CASES = [("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0), 1 << 18),
         ("gg_ttgg", 4, -1, "gg_ttg", (400.0, 2000.0), 1 << 18),
         ("ee_uug", 4, 2, "ee_uu", 1000.0, 1 << 16)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("real,i,j,born,rs,n", CASES)
def test_fks_full_size_sampled(gpu, orc, real, i, j, born, rs, n):
    import torch
    mom, _ = events(born, n, rs, stream=42)
    xt, y, phi = fks_variables(n, stream=42, initial_state=j < 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    M, X, Y, P = t(mom), t(xt), t(y), t(phi)
    idx = np.arange(0, n, n // 64) + 5
    ref = orc.fks(real, i, j, np.ascontiguousarray(mom[:, :, idx]), xt[idx], y[idx], phi[idx], kind="quad")
    terms = sum(np.abs(ref[k]) for k in ("g_R", "g_S", "g_C", "g_SC", "g_Cm", "g_SCm"))
    omy = (1 - ref["y"]) if j >= 0 else (1 - ref["y"]) * (1 + ref["y"])
    kappa = ref["xi"] * omy
    D = terms / kappa
    for prec in ("mixed", "fp64"):
        res = gpu.subtracted(real, i, j, M, X, Y, P, prec=prec)
        torch.cuda.synchronize()
        W = res["W"].cpu().numpy()
        st = res["status"].cpu().numpy()
        assert np.all(np.isfinite(W)) and not np.any(st & 1)
        dW = np.abs(W[idx] - ref["W"])
        routed = (st[idx] & 2) != 0
        unres = (st[idx] & 8) != 0
        fp64_bound = 1e-12 * (np.abs(ref["W"]) + D)
        if prec == "fp64":
            assert np.all(routed)
            assert np.all(dW <= fp64_bound)
        else:
            redone = (st[idx] & 16) != 0
            assert np.array_equal(routed & ~redone, kappa < 0.1)
            assert np.all(dW[~routed] <= 1e-3 * np.abs(ref["W"][~routed]))
            assert np.all(dW[routed] <= fp64_bound[routed])
        assert np.all(dW[~unres] <= 1e-3 * np.abs(ref["W"][~unres]))
        print(real, i, j, prec, "n", n, "routed %.3f unresolved %.4f" % (((st & 2) != 0).mean(), ((st & 8) != 0).mean()),
              flush=True)


def test_mixed_buckets_bitwise(gpu):
    """MIXED at 2^18 events (FP32 bucket, then one FP64 launch over the FP64
    bucket and the re-evaluation list): every event's W equals, bit for bit,
    its value from the all-FP64 call (routed or re-evaluated events) or the
    all-FP32 call (the others); exactly the FP32 events with an unresolved or
    non-finite W are re-evaluated; the result is the same on a second call;
    and the fixed-order sum of W equals the sum of those W."""
    import torch
    real, i, j, born, rs, n = "gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0), 1 << 18
    mom, _ = events(born, n, rs, stream=43)
    xt, y, phi = fks_variables(n, stream=43, initial_state=True, spread="flat")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    M, X, Y, P = t(mom), t(xt), t(y), t(phi)
    got = {}
    for prec in ("mixed", "fp64", "fp32"):
        r = gpu.subtracted(real, i, j, M, X, Y, P, prec=prec, want_sum=True)
        torch.cuda.synchronize()
        got[prec] = {k: r[k].cpu().numpy() for k in ("W", "status", "w_sum", "xi")}
    routed = (got["mixed"]["status"] & 2) != 0
    assert 0.1 < routed.mean() < 0.5
    expect = np.where(routed, got["fp64"]["W"], got["fp32"]["W"])
    assert np.array_equal(got["mixed"]["W"], expect)
    # the FP32 events whose W came out unresolved were evaluated again in FP64
    redone = (got["mixed"]["status"] & 16) != 0
    kap = got["mixed"]["xi"] * (1 - y) * (1 + y)
    near = np.abs(kap / 0.1 - 1) < 1e-12
    expect_redo = (kap >= 0.1) & ((got["fp32"]["status"] & 9) != 0)
    assert np.array_equal(redone[~near], expect_redo[~near])
    assert np.array_equal(got["mixed"]["status"] & 8, got["fp64"]["status"] & 8)
    print("re-evaluated in FP64: %.4f of the events" % redone.mean(), flush=True)
    again = gpu.subtracted(real, i, j, M, X, Y, P, prec="mixed", want_sum=True)
    torch.cuda.synchronize()
    assert np.array_equal(again["W"].cpu().numpy(), got["mixed"]["W"])
    assert again["w_sum"].cpu().numpy()[0] == got["mixed"]["w_sum"][0]
    W = got["mixed"]["W"]
    assert abs(got["mixed"]["w_sum"][0] - W.sum()) <= 1e-12 * np.abs(W).sum()
