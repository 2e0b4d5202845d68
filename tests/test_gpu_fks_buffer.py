"""Buffered FKS evaluation (nlo_fks_buffer_*, through the C ABI): events
pushed in uneven pieces join a real-emission queue and a counterterm queue by
their cuts, each queue is evaluated on its own terms when it holds enough
events, and after the flush every slot holds the subtracted weight W of
nlo_subtracted with the same masks, within 1e-12 (|W| + D) (the two-part sum
rounds differently; in MIXED, on the events that the direct call evaluates
again in FP64, within the FP32 rounding bound), and bit for bit the same
whatever the push pattern."""
import numpy as np
import pytest

from nlo_inputs.workloads import events, fks_variables

pytestmark = pytest.mark.gpu

CASES = [("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0), "fp64", 6000),
         ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0), "mixed", 3000),
         ("ee_uug", 4, 2, "ee_uu", 1000.0, "fp64", 6000),
         ("ug_ttu", 4, -1, "gg_tt", (400.0, 2000.0), "mixed", 4000)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _masks(n, beams, seed):
    rng = np.random.default_rng(seed)
    m = (rng.uniform(size=(4, n)) < 0.7).astype(np.uint8)
    if beams:       # the two collinear ends separately
        m[3] = 2 | 4 * (rng.uniform(size=n) < 0.7) | 8 * (rng.uniform(size=n) < 0.7)
    return m


def _run_buffer(gpu, case, mom, xt, y, phi, mask, pieces, threshold):
    import torch
    real, i, j, born, rs, prec, n = case
    w = torch.zeros(n, dtype=torch.float64, device="cuda")
    buf = gpu.fks_buffer(real, i, j, prec, threshold, w)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    try:
        lo = 0
        for p in pieces:
            hi = min(n, lo + p)
            sl = slice(lo, hi)
            buf.push(t(mom[:, :, sl]), t(xt[sl]), t(y[sl]), t(phi[sl]), t(mask[:, sl]),
                     t(np.arange(lo, hi, dtype=np.uint32)))
            lo = hi
        assert lo == n
        buf.flush()
        torch.cuda.synchronize()
    finally:
        buf.close()
    return w.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=["%s_%d_%d_%s" % (c[0], c[1], c[2], c[5]) for c in CASES])
def test_buffer_matches_subtracted(gpu, case):
    import torch
    real, i, j, born, rs, prec, n = case
    mom, _ = events(born, n, rs, stream=801)
    xt, y, phi = fks_variables(n, stream=801, initial_state=j < 0)
    mask = _masks(n, j < 0, 802)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    gpu.reserve(n)
    d = gpu.subtracted(real, i, j, t(mom), t(xt), t(y), t(phi), prec=prec, mask=t(mask))
    torch.cuda.synchronize()
    d = {k: v.cpu().numpy() for k, v in d.items()}
    kap = d["xi"] * (1 - y) * ((1 + y) if j < 0 else 1.0)
    D = sum(np.abs(d[k]) for k in ("g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm")) / kap
    a = _run_buffer(gpu, case, mom, xt, y, phi, mask, [1000, 37, 2500, 900, 1, 4096, 10000], 1024)
    b = _run_buffer(gpu, case, mom, xt, y, phi, mask, [n], 700)
    den = np.abs(d["W"]) + D
    off = den == 0                      # every term masked: W = 0 on both sides
    assert np.all(a[off] == 0.0) and np.all(d["W"][off] == 0.0)
    # MIXED evaluates an FP32 event again in FP64 when W, the difference of
    # its real and counterterm parts, is not resolved (status bit 4).  The
    # queues evaluate the two parts apart, each resolved on its own, so they
    # keep FP32 there: on those events the two differ by up to the FP32
    # rounding bound 32 eps_32 (1 + 1/sqrt(1-|y|)) D.
    redone = (d["status"] & 16) != 0
    c32 = 32 * 2.0 ** -24 * (1 + 1 / np.sqrt(1 - np.abs(y)))
    bound = np.where(redone, c32 * D, 1e-12 * den)
    dW = np.abs(a - d["W"])
    r = dW[~off] / den[~off]
    print("%s (%d,%d) %s: %d events all masked; max |dW| / (|W| + D) %.2e on the %d events the direct call did "
          "not re-evaluate" % (real, i, j, prec, off.sum(), r[~redone[~off]].max(), (~redone).sum()), flush=True)
    assert np.all(dW[~off] <= bound[~off])
    assert np.array_equal(a, b)


def test_buffer_argument_errors(gpu):
    import torch
    import paper_2503_07439_amd as nl
    w = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NloError) as e:
        gpu.fks_buffer("gg_ttg", 4, 2, "fp64", 64, w)
    assert e.value.status == 5
    with pytest.raises(nl.NloError) as e:
        gpu.fks_buffer("gg_ttg", 4, -1, "fp64", 0, w)
    assert e.value.status == 1
    with pytest.raises(nl.NloError) as e:
        gpu.fks_buffer("gg_ttg", 4, -1, "fp16", 64, w)
    assert e.value.status == 5
