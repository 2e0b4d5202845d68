"""One graph launch for an uneven mix of Born, real and subtracted items
(different processes and FKS sectors, event counts log-uniform): every
replay of the captured graph equals the direct per-item calls bit for bit,
with eager work and synchronisation between replays."""
import numpy as np
import pytest

from nlo_inputs.philox import uniforms
from nlo_inputs.workloads import events, fks_variables

pytestmark = pytest.mark.gpu

# (kind, process, fks pair, Born process for subtracted items, precision)
MIX = [
    ("me2", "gg_tt", None, None, "mixed"),
    ("me2", "gg_ttg", None, None, "mixed"),
    ("me2", "uu_ttg", None, None, "fp64"),
    ("me2", "ug_ttu", None, None, "mixed"),
    ("sub", "gg_ttg", (4, -1), "gg_tt", "mixed"),
    ("sub", "uu_ttg", (4, -1), "uu_tt", "fp64"),
    ("sub", "ee_uug", (4, 2), "ee_uu", "mixed"),
    ("me2", "gg_ttg", None, None, "fp16"),
]


def _mix(seed_stream, lo=3.0, hi=4.3):
    import torch
    import paper_2503_07439_amd as nl
    u = uniforms(7439, seed_stream, np.arange(len(MIX)), 0)[:, 0]
    counts = np.floor(10.0 ** (lo + (hi - lo) * u)).astype(np.int64)
    items, bufs, direct = [], [], []
    for k, ((kind, proc, pair, born, prec), n) in enumerate(zip(MIX, counts)):
        n = int(n)
        rs = 1000.0 if proc.startswith("ee") else (400.0, 2000.0)
        it = nl.nlo_work_item()
        it.proc_id = nl.proc_id(proc)
        it.n = n
        it.ld = n
        it.prec = nl.PREC[prec]
        if kind == "me2":
            mom = torch.from_numpy(events(proc, n, rs, stream=300 + k)[0]).cuda()
            out = torch.zeros(n, dtype=torch.float64, device="cuda")
            it.kind = nl.NLO_ITEM_ME2
            it.mom = mom.data_ptr()
            it.me2 = out.data_ptr()
            bufs.append((mom, out))
            direct.append(("me2", proc, mom, prec, out))
        else:
            mom = torch.from_numpy(events(born, n, rs, stream=300 + k)[0]).cuda()
            xt, y, phi = (torch.from_numpy(np.ascontiguousarray(a)).cuda()
                          for a in fks_variables(n, stream=300 + k, initial_state=pair[1] < 0))
            W = torch.zeros(n, dtype=torch.float64, device="cuda")
            wsum = torch.zeros(1, dtype=torch.float64, device="cuda")
            it.kind = nl.NLO_ITEM_SUBTRACTED
            it.fks_i, it.fks_j = pair
            it.mom, it.xi_tilde, it.y, it.phi = mom.data_ptr(), xt.data_ptr(), y.data_ptr(), phi.data_ptr()
            it.fks_out.W = W.data_ptr()
            it.fks_out.w_sum = wsum.data_ptr()
            bufs.append((mom, xt, y, phi, W, wsum))
            direct.append(("sub", proc, (pair, mom, xt, y, phi), prec, (W, wsum)))
        items.append(it)
    return items, bufs, direct, counts


def test_graph_batch_matches_direct_calls(orc):
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    items, bufs, direct, counts = _mix(401)
    # direct per-item results
    ref = []
    for kind, proc, args, prec, out in direct:
        if kind == "me2":
            ref.append(ctx.me2(proc, args, prec).clone())
        else:
            pair, mom, xt, y, phi = args
            r = ctx.subtracted(proc, pair[0], pair[1], mom, xt, y, phi, prec=prec, want_sum=True)
            ref.append((r["W"].clone(), r["w_sum"].clone()))
    torch.cuda.synchronize()
    plan = nl.nlo_batch_plan(ctx.ctx, items, 4)
    try:
        stream = torch.cuda.current_stream().cuda_stream
        for rep in range(3):
            for _, out in [(d, d[4]) for d in direct]:
                if isinstance(out, tuple):
                    out[0].zero_(); out[1].zero_()
                else:
                    out.zero_()
            nl.nlo_batch_run(plan, stream)
            torch.cuda.synchronize()
            for (kind, proc, args, prec, out), r in zip(direct, ref):
                if kind == "me2":     # an FP16 item may hold non-finite events: compare them too
                    assert torch.equal(out.isnan(), r.isnan()), (rep, proc)
                    assert torch.equal(torch.nan_to_num(out), torch.nan_to_num(r)), (rep, proc)
                else:
                    assert torch.equal(out[0], r[0]) and torch.equal(out[1], r[1]), (rep, proc)
            # eager work between replays
            _ = ctx.me2("gg_tt", bufs[0][0], "fp64")
            torch.cuda.synchronize()
    finally:
        nl.nlo_plan_destroy(plan)
        ctx.close()
    print("mix counts", counts.tolist(), flush=True)


def test_batch_plan_argument_errors():
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    try:
        it = nl.nlo_work_item()
        it.kind = nl.NLO_ITEM_SUBTRACTED
        it.proc_id = nl.proc_id("gg_ttg")
        it.fks_i, it.fks_j = 4, 3          # no such sector
        it.n = it.ld = 1
        with pytest.raises(nl.NloError) as e:
            nl.nlo_batch_plan(ctx.ctx, [it])
        assert e.value.status == 5
        it.kind = 7
        with pytest.raises(nl.NloError) as e:
            nl.nlo_batch_plan(ctx.ctx, [it])
        assert e.value.status == 1
        with pytest.raises(nl.NloError) as e:
            nl.nlo_batch_plan(ctx.ctx, [], 99)
        assert e.value.status == 1
    finally:
        ctx.close()


def test_autotune_keeps_results(orc):
    """The autotuner picks a valid configuration and results stay exact."""
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    try:
        mom, _ = events("gg_ttg", 1 << 14, (400.0, 2000.0), stream=410)
        m = torch.from_numpy(mom).cuda()
        for prec in ("fp64", "mixed"):
            (block, mode, sched), ns = ctx.autotune("gg_ttg", m, prec)
            print("gg_ttg %s tuned: block %d, colour unit %d, schedule %d, %.3f ns/event" % (prec, block, mode, sched, ns),
                  flush=True)
            assert block in (64, 128, 192, 256) and mode in (1, 2) and sched in (0, 1) and ns > 0
            assert nl.nlo_get_kernel_config(ctx.ctx, nl.proc_id("gg_ttg"), nl.PREC[prec]) == (block, mode, sched)
            out = ctx.me2("gg_ttg", m, prec)
            torch.cuda.synchronize()
            r = np.abs(out.cpu().numpy()[:256] / orc.me2("gg_ttg", mom[:, :, :256]) - 1)
            assert np.all(r < (1e-11 if prec == "fp64" else 1e-3))
    finally:
        ctx.close()


def _oracle_w_bound(orc, proc, pair, mom, xt, y, phi, idx, prec):
    """binary128 W on the sampled events and the per-event bound of the
    parity tests: |dW| <= 1e-12 (|W| + D) in FP64; MIXED adds 1e-3 |W| for
    its FP32-routed events"""
    r = orc.fks(proc, pair[0], pair[1], np.ascontiguousarray(mom[:, :, idx]), xt[idx], y[idx], phi[idx], kind="quad")
    kap = r["xi"] * (1 - r["y"]) * ((1 + r["y"]) if pair[1] < 0 else 1.0)
    D = sum(np.abs(r[k]) for k in ("g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm")) / kap
    bound = 1e-12 * (np.abs(r["W"]) + D) + (1e-3 * np.abs(r["W"]) if prec == "mixed" else 0.0)
    return r["W"], bound


def test_autotuned_mix_against_oracle(orc):
    """Every item of the mix autotuned on its own events (block size and
    colour unit; per-sector real and counterterm blocks), planned into one
    graph: the graph equals the tuned direct calls bit for bit, and a strided
    sample of every item matches the oracle (|M|^2: FP64 1e-11, MIXED 1e-5,
    FP16 median 2e-3; W: against binary128 within the parity tests' bound)."""
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    items, bufs, direct, counts = _mix(402)
    try:
        tuned = []
        for kind, proc, args, prec, out in direct:
            if kind == "me2":
                tuned.append(ctx.autotune(proc, args, prec)[0])
            else:
                pair, mom, xt, y, phi = args
                tuned.append(ctx.autotune_subtracted(proc, pair[0], pair[1], mom, xt, y, phi, prec)[0])
        print("tuned configurations", tuned, flush=True)
        ref = []
        for kind, proc, args, prec, out in direct:
            if kind == "me2":
                ref.append(ctx.me2(proc, args, prec).clone())
            else:
                pair, mom, xt, y, phi = args
                ref.append(ctx.subtracted(proc, pair[0], pair[1], mom, xt, y, phi, prec=prec)["W"].clone())
        ctx.reserve(int(counts.max()))
        plan = nl.nlo_batch_plan(ctx.ctx, items, 4)
        try:
            nl.nlo_batch_run(plan, torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
        finally:
            nl.nlo_plan_destroy(plan)
        for k, ((kind, proc, args, prec, out), r) in enumerate(zip(direct, ref)):
            got = (out if kind == "me2" else out[0]).cpu().numpy()
            assert np.array_equal(np.nan_to_num(got), np.nan_to_num(r.cpu().numpy())), (k, proc)
            n = got.size
            idx = np.unique(np.linspace(0, n - 1, min(n, 64 if kind == "sub" else 128)).astype(np.int64))
            if kind == "me2":
                mom = args.cpu().numpy()
                rel = np.abs(got[idx] / orc.me2(proc, np.ascontiguousarray(mom[:, :, idx])) - 1)
                print("item %d %s %s: median %.2e max %.2e" % (k, proc, prec, np.median(rel), rel.max()), flush=True)
                if prec == "fp64":
                    assert np.all(rel < 1e-11)
                elif prec == "mixed":
                    assert np.all(rel < 1e-5)
                else:
                    assert np.median(rel) < 2e-3
            else:
                pair, mom, xt, y, phi = (a.cpu().numpy() if hasattr(a, "cpu") else a for a in args)
                w, bound = _oracle_w_bound(orc, proc, pair, mom, xt, y, phi, idx, prec)
                dw = np.abs(got[idx] - w)
                print("item %d %s %s W: max |dW|/bound %.2e" % (k, proc, prec, np.max(dw / bound)), flush=True)
                assert np.all(dw <= bound)
    finally:
        ctx.close()


def test_tuning_cache_roundtrip(tmp_path):
    """Autotune results merge into a JSON cache keyed by device, runtime and
    build; a new context applies exactly the entries of its own key; a
    malformed file is rejected and changes nothing."""
    import json
    import torch
    import paper_2503_07439_amd as nl
    path = str(tmp_path / "tuning.json")
    a, b = nl.Context(), nl.Context()
    try:
        assert a.tuning_cache(path) == 0                       # no file yet: empty cache
        m = torch.from_numpy(events("gg_tt", 1 << 14, (400.0, 2000.0), stream=420)[0]).cuda()
        cfg_me2, _ = a.autotune("gg_tt", m, "mixed")
        mom, _ = events("ee_uu", 1 << 12, 1000.0, stream=421)
        xt, y, phi = (torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in fks_variables(1 << 12, stream=421))
        cfg_fks, _ = a.autotune_subtracted("ee_uug", 4, 2, torch.from_numpy(mom).cuda(), xt, y, phi, "fp64")
        doc = json.load(open(path))
        assert doc["format"] == "nlome-tuning-1" and len(doc["entries"]) == 2
        e_me2 = [e for e in doc["entries"] if e["kind"] == "me2"][0]
        e_fks = [e for e in doc["entries"] if e["kind"] == "subtracted"][0]
        for e in (e_me2, e_fks):
            assert e["arch"].startswith("gfx950") and e["cus"] > 0 and e["runtime"] > 0 and len(e["build"]) == 16
        assert (e_me2["proc"], e_me2["prec"], e_me2["block"], e_me2["colour_mode"], e_me2["schedule"]) == (
            "gg_tt", "mixed", *cfg_me2)
        assert (e_fks["proc"], e_fks["i"], e_fks["j"], e_fks["prec"]) == ("ee_uug", 4, 2, "fp64")
        assert (e_fks["real_block"], e_fks["colour_mode"], e_fks["ct_block"]) == cfg_fks
        # tuning again replaces the entry of the same key
        a.autotune("gg_tt", m, "mixed")
        assert len(json.load(open(path))["entries"]) == 2
        # a foreign key is kept in the file but not applied
        doc["entries"].append(dict(e_me2, arch="gfx000", block=64, proc="gg_ttg"))
        json.dump(doc, open(path, "w"))
        b.set_kernel_config("gg_tt", "mixed", 64, 1)
        assert b.tuning_cache(path) == 2
        assert b.kernel_config("gg_tt", "mixed") == tuple(cfg_me2)
        assert b.fks_config("ee_uug", 4, 2, "fp64") == tuple(cfg_fks)
        assert b.kernel_config("gg_ttg", "mixed") == (256, 0, 0)
        # a malformed file: error, nothing applied
        bad = str(tmp_path / "bad.json")
        open(bad, "w").write('{"format": "nlome-tuning-1", "entries": [{"kind": "me2", "block": }]}')
        with pytest.raises(nl.NloError) as e:
            b.tuning_cache(bad)
        assert e.value.status == 1
        assert b.kernel_config("gg_tt", "mixed") == tuple(cfg_me2)
    finally:
        a.close()
        b.close()
