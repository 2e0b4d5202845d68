"""nlo_subtracted_static (no allocation: its workspace is a static device
array) against nlo_subtracted (the context workspace), through the C ABI:
the same per-event results bit for bit, on two calls in a row with the
second smaller (the array keeps the first call's contents), in MIXED and
FP64; a call beyond the array's 65536 events fails before any launch."""
import numpy as np
import pytest

from nlo_inputs.workloads import events, fks_variables

pytestmark = pytest.mark.gpu

FIELDS = ("W", "xi", "born", "g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm")


def _static_call(nl, ctx, sector, M, X, Y, P, prec):
    import torch
    real, i, j = sector
    n = M.shape[2]
    res = {k: torch.full((n,), -7.0, dtype=torch.float64, device="cuda") for k in FIELDS}
    res["status"] = torch.zeros(n, dtype=torch.uint8, device="cuda")
    out = nl.nlo_fks_out()
    for k in FIELDS:
        setattr(out, k, res[k].data_ptr())
    out.status = res["status"].data_ptr()
    nl.nlo_subtracted_static(ctx.ctx, nl.proc_id(real), i, j, n, n, M.data_ptr(), X.data_ptr(), Y.data_ptr(),
                             P.data_ptr(), 0, nl.PREC[prec], out, ctx._stream())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.mark.parametrize("sector,born,rs", [((4, -1), "gg_tt", (400.0, 2000.0)), ((4, 5), "gg_ttg", (400.0, 2000.0))],
                         ids=["gg_ttg_beams", "gg_ttgg_4_5"])
def test_static_matches_workspace_entry_point(sector, born, rs):
    import torch
    import paper_2503_07439_amd as nl
    real = "gg_ttg" if born == "gg_tt" else "gg_ttgg"
    ctx = nl.Context()
    try:
        for n, stream in ((3000, 301), (700, 302)):          # second call smaller
            mom, _ = events(born, n, rs, stream=stream)
            xt, y, phi = fks_variables(n, stream=stream, initial_state=sector[1] < 0)
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
            M, X, Y, P = t(mom), t(xt), t(y), t(phi)
            for prec in ("mixed", "fp64"):
                ref = ctx.subtracted(real, sector[0], sector[1], M, X, Y, P, prec=prec)
                torch.cuda.synchronize()
                ref = {k: v.cpu().numpy() for k, v in ref.items()}
                got = _static_call(nl, ctx, (real,) + sector, M, X, Y, P, prec)
                for k in FIELDS + ("status",):
                    assert np.array_equal(got[k], ref[k]), (n, prec, k)
                assert np.all(np.isfinite(got["W"]))
    finally:
        ctx.close()


def test_static_rejects_oversize():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    try:
        z = torch.zeros(8, dtype=torch.float64, device="cuda")
        out = nl.nlo_fks_out()
        out.W = z.data_ptr()
        n = 65537
        with pytest.raises(nl.NloError) as e:
            nl.nlo_subtracted_static(ctx.ctx, nl.proc_id("gg_ttg"), 4, -1, n, n, z.data_ptr(), z.data_ptr(),
                                     z.data_ptr(), z.data_ptr(), 0, nl.NLO_MIXED, out, 0)
        assert e.value.status == 1 and "static scratch" in str(e.value)
    finally:
        ctx.close()
