"""Throughput benchmark: helicity- and colour-summed gg -> t tbar g |M|^2 on
one MI355X, mixed precision (FP32 amplitudes, FP64 prologue and helicity sum,
colour contraction on the vector ALU; the matrix-core variant is timed
beside it) against the plain FP64 GPU path, with the relative error of every
event against the FP64 result and of a sample against the FP64 CPU oracle.

One step = one nlo_me2 call over the whole batch (2^22 RAMBO events, m_t =
173 GeV, sqrt(s_hat) uniform in [400, 2000] GeV), inputs resident in HBM.
Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-mix] [--no-configs] [--no-fks]
                    [--prec mixed|fp32|fp64]

Beside the headline it times: the other |M|^2 configurations at their sizes
(e+e- -> mu+mu- 2^14, e+e- -> u ubar g 2^20, g g -> t tbar 2^22), g g -> t
tbar g g at 2^20 in every precision, the subtracted weight on the FKS stress
sets (MIXED against FP64, routed fraction, errors), an uneven mix of Born,
real and subtracted items as one captured-graph launch against per-item calls
("batch_mix"), the subtracted real emission integrated by VEGAS on the
device (2^20 points per iteration, g g -> t tbar g and e+e- -> u ubar g), and
the FP64 oracle on the host cores (cpu_baseline, which also holds the
binary128 oracle's check of the subtracted weights).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gg→tt̄g |M|^2 events/s (hel+colour summed) mixed vs FP64, at stated rel err"
# MI355X vector ALU peaks, TFLOP/s: FP32 and FP64 published; packed FP16 is
# 256 CUs x 4 SIMDs x 16 lanes x 2 (pair) x 2 (FMA) x 2.4 GHz; BF16 has no
# native arithmetic here and runs at the single-issue FP32 rate
PEAK = {"fp32": 157.3, "fp64": 78.6, "fp16": 157.3, "bf16": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # untimed steps before the timed ones: the clocks settle within about
    # 50 ms of sustained load (headline: 1.53 ms per step after 3 warm-up
    # steps, 1.43 after 50, 1.43 over 200 timed steps)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="gg_ttg_400_2000")
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp32", "fp64", "fp16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    ap.add_argument("--events", type=int, default=0, help="override the batch size")
    ap.add_argument("--no-mix", action="store_true", help="skip the batched-mix leg")
    ap.add_argument("--no-half", action="store_true", help="skip the FP16 leg")
    ap.add_argument("--no-gen", action="store_true", help="skip the device phase-space generation leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the other |M|^2 configurations and gg->ttgg")
    ap.add_argument("--no-fks", action="store_true", help="skip the subtracted-weight legs")
    ap.add_argument("--no-integrate", action="store_true", help="skip the device integration leg")
    ap.add_argument("--no-mask-study", action="store_true", help="skip the cut-mask study")
    ap.add_argument("--no-probe", action="store_true", help="skip the attainable-FMA probe")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (calibrates the HBM byte counters)")
    return ap.parse_args()


def timed(ctx, proc, mom, out, prec, steps, warmup):
    """Average duration of one launch, with HIP events on the launch stream."""
    import torch
    for _ in range(warmup):
        ctx.me2(proc, mom, prec, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        ctx.me2(proc, mom, prec, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def timed_fn(fn, steps, warmup=1):
    """Average duration of fn() (launches on the current stream), HIP events."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def device_batch(ctx, proc, n, rs, stream):
    """The batch recipe's points generated on the device (Philox + RAMBO;
    bit-identical to the host recipe, see the phase-space tests)."""
    lo, hi = rs if isinstance(rs, tuple) else (rs, rs)
    mom, _ = ctx.phase_space(proc, n, (lo, hi), stream)
    return mom


def kernel_name(ctx, proc, prec):
    if prec in ("fp16", "bf16"):
        return "k_me2_pair<%s, %s>" % (proc, "f16x2" if prec == "fp16" else "bf16x2")
    sched = ctx.kernel_config(proc, prec)[2]
    if prec == "fp64":
        return "k_me2_valu<%s, double, %d>" % (proc, sched)
    return "k_me2_mfma<%s>" % proc if ctx.colour_unit(proc, prec) == "mfma" else "k_me2_valu<%s, float, %d>" % (
        proc, sched)


def flops_per_event(proc):
    with open(os.path.join(ROOT, "paper_2503_07439_amd", "flops.json")) as f:
        return json.load(f)[proc]["nested_flops_per_event_folded"]


def configs_leg(ctx, steps):
    """The other |M|^2 configurations at their sizes: time per batch, events/s,
    vector-ALU and HBM fractions (FP64 and the mixed path)."""
    from nlo_inputs.workloads import CONFIGS
    rows = []
    for name in ("ee_mumu_91", "ee_uug_1000", "gg_tt_400_2000"):
        proc, n, rs, stream = CONFIGS[name]
        mom = device_batch(ctx, proc, n, rs, stream)
        npart = mom.shape[0]
        fl = flops_per_event(proc)
        for prec in ("mixed", "fp64"):
            ms = timed_fn(lambda: ctx.me2(proc, mom, prec), steps)
            eps = n / (ms * 1e-3)
            rows.append({"workload": name, "precision": prec, "events": n, "ms": ms, "events_per_s": eps,
                         "valu_frac": fl * eps / 1e12 / PEAK["fp64" if prec == "fp64" else "fp32"],
                         "hbm_frac": (32 * npart + 8) * eps / 8e12, "kernel": kernel_name(ctx, proc, prec)})
        del mom
    return rows


def gg_ttgg_leg(ctx, steps):
    """g g -> t tbar g g, 2^20 points: every amplitude precision, with the
    error against the FP64 GPU result (median, p99.9, summed)."""
    import torch
    from nlo_inputs.workloads import CONFIGS
    proc, n, rs, stream = CONFIGS["gg_ttgg_400_2000"]
    mom = device_batch(ctx, proc, n, rs, stream)
    fl = flops_per_event(proc)
    ctx.reserve(n)
    res, rows = {}, []
    for prec in ("fp64", "mixed", "fp16", "bf16"):
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        ms = timed_fn(lambda: ctx.me2(proc, mom, prec, out=out), max(2, steps))
        res[prec] = out
        row = {"precision": prec, "ms": ms, "events_per_s": n / (ms * 1e-3), "kernel": kernel_name(ctx, proc, prec),
               "valu_frac": fl * n / (ms * 1e-3) / 1e12 / PEAK["fp64" if prec == "fp64" else
                                                              ("fp32" if prec == "mixed" else prec)]}
        if prec != "fp64":
            rel = (out / res["fp64"] - 1).abs().cpu().numpy()
            row["rel_err_vs_gpu_fp64"] = {"median": float(np.median(rel)), "p99_9": float(np.quantile(rel, 0.999)),
                                          "max": float(rel.max()),
                                          "summed": abs(float(out.sum()) / float(res["fp64"].sum()) - 1)}
        rows.append(row)
    del mom, res
    return {"workload": "gg_ttgg_400_2000", "events": n, "flops_per_event": fl, "rows": rows}


# FKS stress sets: Born points, xi_tilde and 1-|y| log-uniform in [1e-6, 1]
# IR-safe cuts of the event loop (the paper defines none): jets by anti-kT
# with R = 0.5, pT >= 40 GeV, |y| <= 2; tops pT >= 50 GeV, |y| <= 2.5
GEN_CUTS = {"gg_ttg": dict(jet_r=0.5, jet_ptmin=40.0, jet_ymax=2.0, njet_min=1, top_ptmin=50.0, top_ymax=2.5)}

FKS_SETS = [("ee_uug", 4, 2, "ee_uu", 1000.0, 1 << 16), ("gg_ttg", 4, -1, "gg_tt", (400.0, 2000.0), 1 << 20),
            ("gg_ttgg", 4, 5, "gg_ttg", (400.0, 2000.0), 1 << 18)]


def fks_leg(ctx, steps):
    """The subtracted weight on the FKS stress sets (radiation variables
    log-uniform towards the limits) and on the same Born points with flat
    radiation variables: MIXED against FP64 time, the fraction MIXED routes to
    FP64, the fraction whose W its precision does not resolve to 1e-3 (status
    bit 3), and MIXED's error against FP64 on every event.  Returns the rows
    and the stress sets' inputs/outputs for the oracle sample."""
    import torch
    from nlo_inputs.workloads import events, fks_variables
    rows, keep = [], []
    for (real, i, j, born, rs, n), spread in [(s, "log") for s in FKS_SETS] + [(s, "flat") for s in FKS_SETS]:
        mom_np, _ = events(born, n, rs, stream=42)
        xt_np, y_np, phi_np = fks_variables(n, stream=42, initial_state=j < 0, spread=spread)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        M, X, Y, P = t(mom_np), t(xt_np), t(y_np), t(phi_np)
        ctx.reserve(n)
        out, ms = {}, {}
        for prec in ("mixed", "fp64", "fp32"):
            ms[prec] = timed_fn(lambda: ctx.subtracted(real, i, j, M, X, Y, P, prec=prec), steps)
            r = ctx.subtracted(real, i, j, M, X, Y, P, prec=prec)
            torch.cuda.synchronize()
            out[prec] = {k: r[k].cpu().numpy() for k in ("W", "status")}
        st = out["mixed"]["status"]
        rel = np.abs(out["mixed"]["W"] / out["fp64"]["W"] - 1)
        rows.append({"sector": "%s (%d,%s)" % (real, i, j if j >= 0 else "beams"), "events": n,
                     "radiation_variables": {"log": "log-uniform stress set", "flat": "flat"}[spread],
                     "ms_mixed": ms["mixed"], "ms_fp64": ms["fp64"], "ms_fp32": ms["fp32"],
                     "mixed_speedup_vs_fp64": ms["fp64"] / ms["mixed"],
                     "routed_to_fp64": float(((st & 2) != 0).mean()),
                     "reevaluated_in_fp64": float(((st & 16) != 0).mean()),
                     "unresolved_mixed": float(((st & 8) != 0).mean()),
                     "unresolved_fp64": float(((out["fp64"]["status"] & 8) != 0).mean()),
                     "mixed_rel_err_vs_gpu_fp64": {"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
                                                   "p99_9": float(np.quantile(rel, 0.999)), "max": float(rel.max())}})
        if spread == "log":
            keep.append((real, i, j, mom_np, xt_np, y_np, phi_np, out))
        del M, X, Y, P
    return rows, keep


INTEGRATE_SETS = [("gg_ttg", 600.0), ("ee_uug", 1000.0)]


def integrate_leg(ctx):
    """The subtracted real emission integrated over its phase space on the
    device (VEGAS, 2^20 points per iteration, 10 iterations, the first 3 only
    adapting the grid; summed over the FKS sectors): wall time of one whole
    call (it ends with a stream synchronisation), FP64 and MIXED."""
    rows = []
    n, niter, nadapt = 1 << 20, 10, 3
    for real, rs in INTEGRATE_SETS:
        for prec in ("fp64", "mixed"):
            ctx.integrate_subtracted(real, rs, n, niter, nadapt, 330, prec)      # warm-up
            t = time.perf_counter()
            sig, err, chi, its = ctx.integrate_subtracted(real, rs, n, niter, nadapt, 330, prec)
            dt = time.perf_counter() - t
            rows.append({"process": real, "sqrt_s_born_GeV": rs, "precision": prec, "points_per_iteration": n,
                         "iterations": niter, "adapt_only": nadapt, "s_per_call": dt,
                         "ms_per_iteration": dt * 1e3 / niter, "points_per_s": n * niter / dt,
                         "sigma_pb": sig, "error_pb": err, "chi2_dof": chi,
                         "first_iteration_error_pb": its[0][1], "last_iteration_error_pb": its[-1][1]})
            if real == "ee_uug":
                # the complete NLO correction from device pieces: the Born-proportional
                # virtual + integrated counterterms and this subtracted real emission
                mom, w = ctx.phase_space("ee_uu", n, rs, 331)
                b, vi = ctx.virtual_integrated("ee_uu", mom, prec)
                alpha = 1.0 / 132.507
                sig_b = 3 * (2.0 / 3.0) ** 2 * 4 * math.pi * alpha ** 2 / (3 * rs * rs) * 0.3893793721e9
                rows[-1]["nlo_k_factor_minus_1"] = float((w * vi).sum() / (w * b).sum()) + sig / sig_b
                rows[-1]["nlo_k_factor_error"] = err / sig_b
                rows[-1]["alpha_s_over_pi"] = 0.118 / math.pi
    return rows


def mix_leg(ctx, steps):
    """An uneven mix of Born, real and subtracted items (MIXED precision):
    one captured-graph launch of the whole mix against the same items issued
    one call after another on the stream, with the default launch
    configurations and after autotuning every item on its own events."""
    import torch
    import paper_2503_07439_amd as nl
    from nlo_inputs.workloads import MIX_ITEMS, MIX_STREAM, events, fks_variables, mix_counts
    counts = mix_counts()
    items, keep, calls = [], [], []
    stream = torch.cuda.current_stream().cuda_stream
    for k, ((kind, proc, pair, born), n) in enumerate(zip(MIX_ITEMS, counts)):
        n = int(n)
        it = nl.nlo_work_item()
        it.proc_id, it.n, it.ld, it.prec = nl.proc_id(proc), n, n, nl.NLO_MIXED
        if kind == "me2":
            mom = torch.from_numpy(events(proc, n, (400.0, 2000.0), stream=MIX_STREAM + k)[0]).cuda()
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            it.kind, it.mom, it.me2 = nl.NLO_ITEM_ME2, mom.data_ptr(), out.data_ptr()
            keep += [mom, out]
            calls.append(lambda it=it: nl.nlo_me2(ctx.ctx, it.proc_id, it.n, it.ld, it.mom, it.me2, it.prec, stream))
        else:
            mom = torch.from_numpy(events(born, n, (400.0, 2000.0), stream=MIX_STREAM + k)[0]).cuda()
            xt, y, phi = (torch.from_numpy(np.ascontiguousarray(a)).cuda()
                          for a in fks_variables(n, stream=MIX_STREAM + k, initial_state=pair[1] < 0))
            W = torch.empty(n, dtype=torch.float64, device="cuda")
            wsum = torch.empty(1, dtype=torch.float64, device="cuda")
            it.kind, (it.fks_i, it.fks_j) = nl.NLO_ITEM_SUBTRACTED, pair
            it.mom, it.xi_tilde, it.y, it.phi = mom.data_ptr(), xt.data_ptr(), y.data_ptr(), phi.data_ptr()
            it.fks_out.W, it.fks_out.w_sum = W.data_ptr(), wsum.data_ptr()
            keep += [mom, xt, y, phi, W, wsum]
            calls.append(lambda it=it: nl.nlo_subtracted(ctx.ctx, it.proc_id, it.fks_i, it.fks_j, it.n, it.ld, it.mom,
                                                         it.xi_tilde, it.y, it.phi, None, it.prec, it.fks_out, stream))
        items.append(it)
    ctx.reserve(int(counts.max()))     # the direct calls share the context workspace

    def timed_pair():
        """(graph ms, direct ms) with the context's current configurations"""
        plan = nl.nlo_batch_plan(ctx.ctx, items, 4)
        out = []
        try:
            for fn in (lambda: nl.nlo_batch_run(plan, stream), lambda: [c() for c in calls]):
                for _ in range(2):
                    fn()
                torch.cuda.synchronize()
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record()
                for _ in range(steps):
                    fn()
                t1.record()
                torch.cuda.synchronize()
                out.append(t0.elapsed_time(t1) / steps)
        finally:
            nl.nlo_plan_destroy(plan)
        return out

    default_graph, default_direct = timed_pair()
    # autotune every item on its own events, then plan again
    tuned = []
    for k, ((kind, proc, pair, born), it) in enumerate(zip(MIX_ITEMS, items)):
        if kind == "me2":
            mom = keep[[i for i, x in enumerate(keep) if x.data_ptr() == it.mom][0]]
            cfg, ns = ctx.autotune(proc, mom, "mixed")
        else:
            find = lambda ptr: keep[[i for i, x in enumerate(keep) if x.data_ptr() == ptr][0]]
            cfg, ns = ctx.autotune_subtracted(proc, pair[0], pair[1], find(it.mom), find(it.xi_tilde), find(it.y),
                                              find(it.phi), "mixed")
        tuned.append({"item": k, "config": list(cfg), "ns_per_event": ns})
    graph, direct = timed_pair()
    total = int(counts.sum())
    return {"items": [[k, p, list(q) if q else None, int(c)] for (k, p, q, _), c in zip(MIX_ITEMS, counts)],
            "events": total, "precision": "mixed", "graph_ms": graph, "direct_ms": direct,
            "graph_events_per_s": total / (graph * 1e-3), "graph_speedup": direct / graph,
            "default_config_graph_ms": default_graph, "default_config_direct_ms": default_direct,
            "autotuned": tuned}


def mask_study(ctx, steps):
    """Wasted compute of branch-free cut masks (every term evaluated, failed
    ones zeroed) against compact masks (events failing the R cut skip the
    real |M|^2, events failing every Born-level cut skip the Born amplitudes)
    and against the cut-class buffer (16 calls of 2^14 events each, too few
    to fill the chip on their own; a real and a counterterm queue, each
    evaluated when it holds 2^16 events), for several pass fractions of the R
    cut and of the S and C cuts together."""
    import torch
    from nlo_inputs.philox import uniforms
    from nlo_inputs.workloads import events, fks_variables
    n, piece = 1 << 18, 1 << 14
    mom, _ = events("gg_ttg", n, (400.0, 2000.0), stream=42)
    xt, y, phi = fks_variables(n, stream=42)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    M, X, Y, P = t(mom), t(xt), t(y), t(phi)
    slots = t(np.arange(n, dtype=np.uint32))
    u = uniforms(7439, 43, np.arange(n, dtype=np.uint64), 0)
    w = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.reserve(n)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps

    rows = []
    for r_pass, ct_pass in ((1.0, 1.0), (0.5, 1.0), (0.25, 1.0), (0.5, 0.5), (1.0, 0.25)):
        mask = np.zeros((4, n), dtype=np.uint8)
        mask[0] = 1
        mask[1] = (u[:, 0] < r_pass).astype(np.uint8)
        mask[2] = mask[3] = (u[:, 1] < ct_pass).astype(np.uint8)
        tm = t(mask)
        ms = {}
        for mode in (False, True):
            ctx.set_fks_mask_mode(mode)
            ms["compact" if mode else "branch_free"] = timed(
                lambda: ctx.subtracted("gg_ttgg", 4, 5, M, X, Y, P, prec="mixed", mask=tm))
        # the same 16 small calls one after another, compact, without buffering
        pieces = [(M[:, :, k:k + piece].contiguous(), X[k:k + piece], Y[k:k + piece], P[k:k + piece],
                   tm[:, k:k + piece].contiguous()) for k in range(0, n, piece)]
        ms["per_call"] = timed(lambda: [ctx.subtracted("gg_ttgg", 4, 5, a, b, c, d, prec="mixed", mask=e)
                                        for a, b, c, d, e in pieces])
        ctx.set_fks_mask_mode(False)
        buf = ctx.fks_buffer("gg_ttgg", 4, 5, "mixed", 4 * piece, w)

        def buffered():
            for k in range(0, n, piece):
                sl = slice(k, k + piece)
                buf.push(M[:, :, sl].contiguous(), X[sl], Y[sl], P[sl], tm[:, sl].contiguous(), slots[sl])
            buf.flush()

        try:
            ms["buffered"] = timed(buffered)
        finally:
            buf.close()
        rows.append({"r_pass": r_pass, "ct_pass": ct_pass, "branch_free_ms": ms["branch_free"],
                     "compact_ms": ms["compact"], "buffered_16_calls_ms": ms["buffered"],
                     "compact_16_calls_ms": ms["per_call"],
                     "wasted_fraction_branch_free": 1 - ms["compact"] / ms["branch_free"]})
    return {"sector": "gg_ttgg (4,5)", "events": n, "precision": "mixed", "buffer_pieces": n // piece, "rows": rows}


def attainable_fma():
    """Attainable vector FMA throughput of this device (TFLOP/s, FP32 and
    FP64) from the probe library: 2048 blocks of 256 threads, eight
    independent FMA chains per thread, timed with HIP events on the current
    stream.  The published peaks assume the 2.4 GHz engine clock; this is
    what the vector ALU delivers at the clock it runs."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2503_07439_amd", "libnlome_probe.so"))
    lib.nlo_probe_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    blocks, iters = 2048, 20000
    res = {}
    for prec, dt in ((0, torch.float32), (1, torch.float64)):
        out = torch.empty(blocks * 256, dtype=dt, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream

        def run():
            rc = lib.nlo_probe_fma(prec, blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream))
            if rc != 0:
                raise RuntimeError("FMA probe launch failed (%d)" % rc)
        ms = timed_fn(run, 5, warmup=2)
        res["fp32" if prec == 0 else "fp64"] = blocks * 256 * 16.0 * iters / (ms * 1e-3) / 1e12
    return {"fp32_tflops": res["fp32"], "fp64_tflops": res["fp64"],
            "probe": "2048 x 256 threads, 8 independent FMA chains each, 20000 iterations"}


def measured_counters(kernel):
    """The machine-readable record of the committed rocprofv3 counter passes
    of the headline kernel (dict), or None when the kernel sources or compile
    flags (build.py) have changed since the counters were taken, or for
    another kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gg_ttg_2p22_counters.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("traffic:"):
            rec = dict(kv.split("=", 1) for kv in line[len("traffic:"):].split())
    h = hashlib.sha256()
    for f in ("csrc/generated/gg_ttg.hpp", "csrc/kernels.hpp", "csrc/helas.hpp", "csrc/launch.hpp", "build.py"):
        with open(os.path.join(ROOT, "paper_2503_07439_amd", f), "rb") as fh:
            h.update(fh.read())
    if not rec or rec.get("sources") != h.hexdigest()[:16] or rec.get("kernel") != kernel.replace(" ", ""):
        return None
    return rec


def measured_traffic(kernel, n):
    """HBM bytes per launch from the counter passes (FETCH_SIZE and
    WRITE_SIZE, calibrated against a copy kernel), scaled to n events, or
    None (see measured_counters)."""
    rec = measured_counters(kernel)
    if rec is None:
        return None
    return (int(rec["fetch_bytes"]) + int(rec["write_bytes"])) * n / int(rec["events"])


def host_info():
    """Cores and CPU model of the host running the baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity": aff, "cpu_model": model}


def cpu_baseline(proc, mom_full, target_s=12.0, target_1_s=3.0, fks_keep=None):
    """The FP64 oracle, built for this host (g++ -O3 -march=native, no
    fast-math), on a bounded sample of the same workload (the first events of
    the batch): with every core this process may use (at most 16, the box's
    CPU share) and with one thread."""
    import oracle
    oracle.build_native()
    oracle.set_params()
    hi = host_info()
    threads = oracle.threads()
    probe = 16384        # large enough that thread start-up does not bias the rate
    t = time.perf_counter()
    oracle.me2(proc, mom_full[:, :, :probe], nthreads=threads, kind="native")
    rate = probe / (time.perf_counter() - t)
    n = int(min(mom_full.shape[2], max(probe, rate * target_s)))
    t = time.perf_counter()
    ref = oracle.me2(proc, np.ascontiguousarray(mom_full[:, :, :n]), nthreads=threads, kind="native")
    dt = time.perf_counter() - t
    n1 = int(min(n, max(256, rate / threads * target_1_s)))
    t = time.perf_counter()
    oracle.me2(proc, np.ascontiguousarray(mom_full[:, :, :n1]), nthreads=1, kind="native")
    dt1 = time.perf_counter() - t
    fks = []
    for real, i, j, mom_np, xt, y, phi, out in fks_keep or []:
        n_all = mom_np.shape[2]
        m = {"gg_ttgg": 96, "gg_ttg": 512}.get(real, 1024)
        idx = np.arange(0, n_all, n_all // m) + 3
        t = time.perf_counter()
        q = oracle.fks(real, i, j, np.ascontiguousarray(mom_np[:, :, idx]), xt[idx], y[idx], phi[idx],
                       nthreads=threads, kind="quad")
        dtq = time.perf_counter() - t
        terms = sum(np.abs(q[k]) for k in ("g_R", "g_S", "g_C", "g_SC", "g_Cm", "g_SCm"))
        kap = q["xi"] * ((1 - q["y"]) if j >= 0 else (1 - q["y"]) * (1 + q["y"]))
        row = {"sector": "%s (%d,%s)" % (real, i, j if j >= 0 else "beams"), "sample": "%d strided events" % len(idx),
               "oracle_binary128_events_per_s": len(idx) / dtq}
        for prec in ("mixed", "fp64"):
            dW = np.abs(out[prec]["W"][idx] - q["W"])
            rel = dW / np.abs(q["W"])
            row[prec] = {"rel_err": {"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
                                     "max": float(rel.max())},
                         "max_dW_over_D": float(np.max(dW * kap / terms)),
                         "rel_err_unflagged_max": float(rel[(out[prec]["status"][idx] & 8) == 0].max())}
        fks.append(row)
    return ref, {"value": n / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
                 "sample": "first %d events of the batch, %.1f s (FP64 oracle: colour-ordered recursion, "
                           "std::thread over events, g++ -O3 -march=native)" % (n, dt),
                 "one_thread": {"value": n1 / dt1, "unit": "events/s", "sample": "first %d events, %.1f s" % (n1, dt1)},
                 "host": hi, "fks_w_vs_binary128_oracle": fks}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (requested --gpus %d); events shard "
              "trivially across GPUs, see the design notes" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2503_07439_amd as nl
    from nlo_inputs.workloads import CONFIGS, config_events

    proc, nfull, rs, stream = CONFIGS[args.workload]
    n = args.events or nfull
    t = time.perf_counter()
    mom_np, _ = config_events(args.workload, n=n)
    print("inputs: %d %s events generated in %.1f s" % (n, proc, time.perf_counter() - t), file=sys.stderr, flush=True)
    ctx = nl.Context()
    if args.copy_probe_mib:
        a = torch.ones(args.copy_probe_mib << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    mom = torch.from_numpy(mom_np).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    info = ctx.info(proc)

    ms = timed(ctx, proc, mom, out, args.prec, args.steps, args.warmup)
    res = out.clone()
    print("%s %s: %.3f ms per step" % (proc, args.prec, ms), file=sys.stderr, flush=True)

    fp64 = None
    if not args.no_fp64 and args.prec != "fp64":
        out64 = torch.empty_like(out)
        ms64 = timed(ctx, proc, mom, out64, "fp64", max(10, args.steps // 2), 3)
        rel = (res / out64 - 1).abs().cpu().numpy()
        sum_rel = abs(float(res.sum()) / float(out64.sum()) - 1)
        fp64 = {"ms_per_step": ms64, "events_per_s": n / (ms64 * 1e-3), "speedup_mixed_vs_fp64": ms64 / ms,
                "rel_err_vs_gpu_fp64": {"median": float(np.median(rel)), "p99_9": float(np.quantile(rel, 0.999)),
                                        "max": float(rel.max()), "summed": sum_rel}}
        print("fp64: %.3f ms per step" % ms64, file=sys.stderr, flush=True)

    # the same batch generated on the device (Philox + RAMBO), alone and
    # followed by the |M|^2 launch: the event loop without host inputs
    gen = None
    if not args.no_gen and args.prec == "mixed":
        gmom = torch.empty_like(mom)
        gw = torch.empty(n, dtype=torch.float64, device="cuda")
        lo, hi = rs if isinstance(rs, tuple) else (rs, rs)
        pid = nl.proc_id(proc)

        def generate():
            nl.nlo_phase_space(ctx.ctx, pid, n, n, 7439, stream, 0, float(lo), float(hi), gmom.data_ptr(),
                               gw.data_ptr(), torch.cuda.current_stream().cuda_stream)

        def both():
            generate()
            ctx.me2(proc, gmom, "mixed", out=out)

        gms = {}
        for name, fn in (("generate", generate), ("generate_and_me2", both)):
            fn()
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(max(3, args.steps // 4)):
                fn()
            t1.record()
            torch.cuda.synchronize()
            gms[name] = t0.elapsed_time(t1) / max(3, args.steps // 4)
        same = bool(torch.allclose(gmom, mom, rtol=0, atol=1e-12 * float(hi)))
        gen = {"ms_generate": gms["generate"], "ms_generate_and_me2": gms["generate_and_me2"],
               "events_per_s_generate_and_me2": n / (gms["generate_and_me2"] * 1e-3),
               "same_points_as_host_batch": same}
        print("device generation: %.3f ms, with |M|^2 %.3f ms" % (gms["generate"], gms["generate_and_me2"]),
              file=sys.stderr, flush=True)
        if proc in GEN_CUTS:
            # Algorithm 2 on the device: the cut mask of the batch, and n
            # points that pass the cuts by regenerating candidates (stream
            # compaction; the call returns the candidate count, so it ends
            # with a synchronisation: wall time per call)
            cuts = GEN_CUTS[proc]
            ms_mask = timed_fn(lambda: ctx.cut_mask(proc, gmom, cuts), max(3, args.steps // 4))
            pass_frac = float(ctx.cut_mask(proc, gmom, cuts).double().mean())
            ctx.generate_passing(proc, n, rs, 7, cuts)
            torch.cuda.synchronize()
            reps = 3
            t = time.perf_counter()
            for _ in range(reps):
                pm, pw, trials = ctx.generate_passing(proc, n, rs, 7, cuts)
            ms_pass = (time.perf_counter() - t) * 1e3 / reps

            def loop():
                pm, pw, _ = ctx.generate_passing(proc, n, rs, 7, cuts)
                ctx.me2(proc, pm, "mixed", out=out)
                torch.cuda.synchronize()
            loop()
            t = time.perf_counter()
            for _ in range(reps):
                loop()
            ms_loop = (time.perf_counter() - t) * 1e3 / reps
            gen.update({"cuts": cuts, "ms_cut_mask": ms_mask, "pass_fraction": pass_frac,
                        "ms_generate_passing": ms_pass, "candidates_per_passing_event": trials / n,
                        "ms_generate_passing_and_me2": ms_loop,
                        "passing_events_per_s": n / (ms_loop * 1e-3)})
            print("cuts: mask %.3f ms (pass %.3f), %d passing points %.3f ms, with |M|^2 %.3f ms" % (
                ms_mask, pass_frac, n, ms_pass, ms_loop), file=sys.stderr, flush=True)
            del pm, pw
        del gmom, gw

    # FP16 amplitudes (FP32 pass for near-pole events) on the same batch, for the record
    half = None
    if not args.no_half and args.prec == "mixed" and fp64 is not None:
        out16 = torch.empty_like(out)
        ms16 = timed(ctx, proc, mom, out16, "fp16", max(3, args.steps // 4), 1)
        rel = (out16 / out64 - 1).abs().cpu().numpy()
        half = {"precision": "fp16", "ms_per_step": ms16, "events_per_s": n / (ms16 * 1e-3),
                "speedup_vs_mixed": ms / ms16,
                "rel_err_vs_gpu_fp64": {"median": float(np.median(rel)), "p99_9": float(np.quantile(rel, 0.999)),
                                        "max": float(rel.max()),
                                        "summed": abs(float(out16.sum()) / float(out64.sum()) - 1)}}
        print("fp16: %.3f ms per step" % ms16, file=sys.stderr, flush=True)
        del out16

    # the other colour-contraction unit, for the record
    other = None
    if args.prec == "mixed":
        unit_now = ctx.colour_unit(proc, "mixed")
        ctx.set_kernel_config(proc, "mixed", 256, 2 if unit_now == "valu" else 1)
        other_unit = ctx.colour_unit(proc, "mixed")
        ms_o = timed(ctx, proc, mom, out, "mixed", max(3, args.steps // 4), 1)
        ctx.set_kernel_config(proc, "mixed", 256, 0)
        other = {"colour_unit": other_unit, "kernel": "k_me2_mfma<%s>" % proc if other_unit == "mfma" else
                 "k_me2_valu<%s, float, 0>" % proc, "ms_per_step": ms_o, "events_per_s": n / (ms_o * 1e-3)}
        print("other colour unit: %.3f ms per step" % ms_o, file=sys.stderr, flush=True)

    # algorithmic flops per event: exact count of the generated source of the
    # nested helicity schedule the kernels run (amplitudes + colour
    # contraction), with operations on literal constants folded away
    with open(os.path.join(ROOT, "paper_2503_07439_amd", "flops.json")) as f:
        fl = json.load(f)[proc]
    flops_event = fl["nested_flops_per_event_folded"]
    att = None if args.no_probe else attainable_fma()
    if att is not None:
        print("attainable FMA: fp32 %.1f TFLOP/s, fp64 %.1f TFLOP/s" % (att["fp32_tflops"], att["fp64_tflops"]),
              file=sys.stderr, flush=True)
    achieved = flops_event * n / (ms * 1e-3) / 1e12
    peak = PEAK[args.prec if args.prec in PEAK else "fp32"]
    kernel = kernel_name(ctx, proc, args.prec)
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(kernel, n), "kernel": kernel,
                "flops_per_event": flops_event, "flops_per_event_as_written": fl["nested_flops_per_event"],
                "bytes_per_event": 32 * info.npart + 8}
    if args.prec in ("mixed", "fp32"):
        # packed FP32 instructions are not generated (compiler flag), so the
        # single-issue vector FP32 rate is the attainable ceiling
        roofline["frac_of_unpacked_fp32_peak"] = achieved / PEAK["fp64"]
        # the executed FP32 flops from the counters (the algorithmic count keeps
        # common subexpressions that the compiler removes, so its rate can pass
        # the single-issue ceiling)
        rec = measured_counters(kernel)
        if rec is not None and "fp32_flops_per_event" in rec:
            ex = float(rec["fp32_flops_per_event"]) * n / (ms * 1e-3) / 1e12
            roofline["executed_fp32_flops_per_event"] = float(rec["fp32_flops_per_event"])
            roofline["executed_fp32_tflops"] = ex
            roofline["executed_frac_of_unpacked_fp32_peak"] = ex / PEAK["fp64"]
            if att is not None:
                roofline["executed_frac_of_attainable_fp32_fma"] = ex / att["fp32_tflops"]

    study = None if args.no_mask_study else mask_study(ctx, 2)

    others = None
    if not args.no_configs:
        others = configs_leg(ctx, max(3, args.steps // 4))
        print("configs: " + ", ".join("%s %s %.3f ms" % (r["workload"], r["precision"], r["ms"]) for r in others),
              file=sys.stderr, flush=True)
    ttgg = None
    if not args.no_configs:
        ttgg = gg_ttgg_leg(ctx, 3)
        print("gg_ttgg 2^20: " + ", ".join("%s %.2f ms" % (r["precision"], r["ms"]) for r in ttgg["rows"]),
              file=sys.stderr, flush=True)
    fks_rows, fks_keep = None, None
    if not args.no_fks:
        fks_rows, fks_keep = fks_leg(ctx, 3)
        print("fks: " + ", ".join("%s mixed %.2f ms fp64 %.2f ms routed %.3f" % (
            r["sector"], r["ms_mixed"], r["ms_fp64"], r["routed_to_fp64"]) for r in fks_rows), file=sys.stderr, flush=True)

    integ = None
    if not args.no_integrate:
        integ = integrate_leg(ctx)
        print("integrate: " + ", ".join("%s %s %.1f ms/iteration" % (r["process"], r["precision"], r["ms_per_iteration"])
                                        for r in integ), file=sys.stderr, flush=True)

    mix = None
    if not args.no_mix:
        mix = mix_leg(ctx, max(3, args.steps // 4))
        print("mix: graph %.3f ms, direct %.3f ms" % (mix["graph_ms"], mix["direct_ms"]), file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        ref, cpu = cpu_baseline(proc, mom_np, fks_keep=fks_keep)
        k = ref.shape[0]
        r = np.abs(res[:k].cpu().numpy() / ref - 1)
        cpu["rel_err_of_gpu_%s_on_sample" % args.prec] = {
            "median": float(np.median(r)), "p99_9": float(np.quantile(r, 0.999)), "max": float(r.max()),
            "summed": abs(float(res[:k].sum().item()) / float(ref.sum()) - 1)}

    line = {
        "metric": METRIC, "value": n / (ms * 1e-3), "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp16": "f16", "bf16": "bf16"}.get(args.prec, "f32"),
        "data": "synthetic",
        "config": {"workload": args.workload, "process": info.name.decode(), "events": n,
                   "sqrt_s_hat_GeV": list(rs) if isinstance(rs, tuple) else rs, "m_top_GeV": 173.0,
                   "precision": args.prec, "diagrams": info.ndiagrams, "colour_flows": info.ncolour,
                   "helicities": info.ngood_hel},
        "roofline": roofline, "attainable_valu_peak": att, "cpu_baseline": cpu, "fp64_gpu": fp64,
        "other_colour_unit": other,
        "half_precision": half, "device_generation": gen, "batch_mix": mix, "mask_study": study,
        "other_configs": others, "gg_ttgg_2p20": ttgg, "fks_subtracted": fks_rows, "integrated_subtracted": integ,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
