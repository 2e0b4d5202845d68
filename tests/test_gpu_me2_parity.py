"""Parity of the HIP |M|^2 path (through the C ABI) with the FP64 oracle,
element by element on the same seeded inputs.

Tolerances (relative, per event), set a few times above what was measured:
  FP64           : median 1e-14 (measured <= 3.0e-15), every event within
                   1e-13 + 2e-15 c, where c = max over leg pairs of
                   E_a E_b / |p_a.p_b| is the conditioning of the smallest
                   pairwise invariant, which both codes form from O(sqrt s)
                   momentum components (measured max 1.2e-12, u g -> t tbar u)
  FP32 / MIXED   : median 1e-6 (measured <= 4.0e-7), every event 1e-5
                   (measured <= 2.3e-6): float amplitudes and colour
                   contraction, FP64 prologue and helicity sum
"""
import numpy as np
import pytest

from nlo_inputs.workloads import events

pytestmark = pytest.mark.gpu

PROCS = ["ee_mumu", "ee_uu", "ee_uug", "gg_tt", "uu_tt", "gg_ttg", "uu_ttg", "ug_ttu", "gg_ttgg"]


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    assert torch.cuda.is_available()
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _rs(proc):
    return 1000.0 if proc.startswith("ee") else (400.0, 2000.0)


def _cond(mom):
    """max over leg pairs of E_a E_b / |p_a.p_b|"""
    n = mom.shape[0]
    c = np.zeros(mom.shape[2])
    for a in range(n):
        for b in range(a + 1, n):
            pa, pb = mom[a], mom[b]
            dot = pa[0] * pb[0] - pa[1] * pb[1] - pa[2] * pb[2] - pa[3] * pb[3]
            c = np.maximum(c, pa[0] * pb[0] / np.abs(dot))
    return c


def _run(gpu, proc, mom, prec, block=None, colour_mode=0):
    import torch
    if block is not None:
        gpu.set_kernel_config(proc, prec, block, colour_mode)
    m = torch.from_numpy(np.ascontiguousarray(mom)).cuda()
    out = gpu.me2(proc, m, prec)
    torch.cuda.synchronize()
    if block is not None:
        gpu.set_kernel_config(proc, prec, 256, 0)
    return out.cpu().numpy()


@pytest.mark.parametrize("proc", PROCS)
def test_fp64_parity(gpu, orc, proc):
    # several blocks plus a ragged tail
    n = 1000 if proc != "gg_ttgg" else 333
    mom, _ = events(proc, n, _rs(proc), stream=101)
    ref = orc.me2(proc, mom)
    got = _run(gpu, proc, mom, "fp64")
    r = np.abs(got / ref - 1)
    bound = 1e-13 + 2e-15 * _cond(mom)
    print(proc, "fp64 median %.2e max %.2e max r/bound %.2f" % (np.median(r), r.max(), np.max(r / bound)), flush=True)
    assert np.median(r) <= 1e-14
    assert np.all(r <= bound)


@pytest.mark.parametrize("prec,mode", [("fp32", 1), ("mixed", 2)])
@pytest.mark.parametrize("proc", PROCS)
def test_fp32_parity(gpu, orc, proc, prec, mode):
    n = 1000 if proc != "gg_ttgg" else 333
    mom, _ = events(proc, n, _rs(proc), stream=102)
    ref = orc.me2(proc, mom)
    got = _run(gpu, proc, mom, prec, block=256, colour_mode=mode)
    r = np.abs(got / ref - 1)
    print(proc, prec, "median %.2e max %.2e" % (np.median(r), r.max()), flush=True)
    assert np.median(r) <= 1e-6
    assert np.all(r <= 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("proc", ["gg_ttg", "gg_ttgg"])
def test_alternative_schedule_parity(gpu, orc, proc, prec):
    """The alternative helicity schedule (the other lazy depth) against the
    oracle, to the bars of the default one."""
    import paper_2503_07439_amd as nl
    assert gpu.info(proc).nschedules == 2
    n = 1000 if proc != "gg_ttgg" else 333
    mom, _ = events(proc, n, _rs(proc), stream=105)
    ref = orc.me2(proc, mom)
    gpu.set_kernel_config(proc, prec, 256, 1, 1)
    try:
        import torch
        m = torch.from_numpy(np.ascontiguousarray(mom)).cuda()
        got = gpu.me2(proc, m, prec).cpu().numpy()
    finally:
        gpu.set_kernel_config(proc, prec, 256, 0, 0)
    r = np.abs(got / ref - 1)
    print(proc, prec, "schedule 1: median %.2e max %.2e" % (np.median(r), r.max()), flush=True)
    if prec == "fp64":
        assert np.median(r) <= 1e-14 and np.all(r <= 1e-13 + 2e-15 * _cond(mom))
    else:
        assert np.median(r) <= 1e-6 and np.all(r <= 1e-5)
    with pytest.raises(nl.NloError) as e:
        gpu.set_kernel_config("gg_tt", prec, 256, 1, 1)        # one schedule only
    assert e.value.status == 5


@pytest.mark.parametrize("block", [64, 128, 192])
def test_launch_shapes_bitwise_fp64(gpu, block):
    """FP64 results do not depend on the launch shape (bitwise)."""
    proc = "gg_ttg"
    mom, _ = events(proc, 777, _rs(proc), stream=103)
    a = _run(gpu, proc, mom, "fp64")
    b = _run(gpu, proc, mom, "fp64", block=block, colour_mode=1)
    assert np.array_equal(a, b)


def test_edge_cases(gpu, orc):
    import torch
    import paper_2503_07439_amd as nl
    proc = "gg_tt"
    # n = 0 is a no-op
    m = torch.zeros((4, 4, 1), dtype=torch.float64, device="cuda")
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    nl.nlo_me2(gpu.ctx, nl.proc_id(proc), 0, 1, m.data_ptr(), out.data_ptr(), nl.NLO_FP64, 0)
    torch.cuda.synchronize()
    assert out.item() == -1.0
    # single event, ld > n (strided batch), and a one-lane MFMA wave
    mom, _ = events(proc, 5, _rs(proc), stream=104)
    big = np.zeros((4, 4, 9))
    big[:, :, :5] = mom
    m = torch.from_numpy(big).cuda()
    for prec in ("fp64", "mixed"):
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        gpu.me2(proc, m, prec, out=out)
        torch.cuda.synchronize()
        ref = orc.me2(proc, mom[:, :, :1])
        assert abs(out.item() / ref[0] - 1) < (1e-11 if prec == "fp64" else 1e-4)
    # host-detected argument errors return before any launch
    with pytest.raises(nl.NloError) as e:
        nl.nlo_me2(gpu.ctx, 99, 1, 1, m.data_ptr(), out.data_ptr(), nl.NLO_FP64, 0)
    assert e.value.status == 2
    with pytest.raises(nl.NloError) as e:
        nl.nlo_me2(gpu.ctx, 3, 4, 2, m.data_ptr(), out.data_ptr(), nl.NLO_FP64, 0)
    assert e.value.status == 1
    with pytest.raises(nl.NloError) as e:
        nl.nlo_me2(gpu.ctx, 3, 1, 1, 0, out.data_ptr(), nl.NLO_FP64, 0)
    assert e.value.status == 1
    with pytest.raises(nl.NloError) as e:
        nl.nlo_me2(gpu.ctx, 3, 1, 1, m.data_ptr(), out.data_ptr(), 7, 0)   # no such precision
    assert e.value.status == 1
    # launch shapes beyond the kernels' launch bounds are rejected on the host
    for bad in (0, 32, 320, 512, 1024):
        with pytest.raises(nl.NloError) as e:
            nl.nlo_set_kernel_config(gpu.ctx, 3, nl.NLO_FP64, bad, 1)
        assert e.value.status == 1


def test_full_size_sampled_gg_ttg(gpu, orc):
    """The headline workload at its full size (2^22 events, the benchmark's
    launch configuration): every event is finite and positive, and a strided
    sample of 512 events matches the oracle."""
    import torch
    from nlo_inputs.workloads import config_events
    mom, _ = config_events("gg_ttg_400_2000")
    m = torch.from_numpy(mom).cuda()
    for prec, tol in (("mixed", 1e-3), ("fp64", 1e-11)):
        out = gpu.me2("gg_ttg", m, prec)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert np.all(np.isfinite(o)) and np.all(o > 0)
        idx = np.linspace(0, mom.shape[2] - 1, 512).astype(np.int64)
        ref = orc.me2("gg_ttg", mom[:, :, idx])
        r = np.abs(o[idx] / ref - 1)
        print("full size", prec, "median", np.median(r), "max", r.max(), flush=True)
        assert np.all(r < tol)


def test_me2_checked_status(gpu, orc):
    """nlo_me2_checked: the same |M|^2 as nlo_me2 and a per-event status --
    bit1 on an event with a non-finite momentum (bit0 follows from its
    result), nothing on good events."""
    import torch
    proc = "gg_ttg"
    mom, _ = events(proc, 300, (400.0, 2000.0), stream=120)
    mom[3, 2, 17] = np.nan
    mom[2, 0, 42] = np.inf
    m = torch.from_numpy(mom).cuda()
    ref = gpu.me2(proc, m, "fp64")
    got, st = gpu.me2_checked(proc, m, "fp64")
    torch.cuda.synchronize()
    ref, got, st = ref.cpu().numpy(), got.cpu().numpy(), st.cpu().numpy()
    good = np.ones(300, bool)
    good[[17, 42]] = False
    assert np.array_equal(got[good], ref[good])
    assert np.all(st[good] == 0)
    assert np.all(st[~good] & 2)
    assert np.allclose(got[good], orc.me2(proc, mom[:, :, good]), rtol=1e-12)


def test_reserve_and_colour_unit(gpu):
    """Evaluation calls never allocate: one that needs more workspace than
    nlo_reserve provided fails with NLO_EINVAL and launches nothing; after
    nlo_reserve it runs.  nlo_colour_unit reports the automatic unit (vector
    ALU) and an explicit override."""
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    try:
        mom = torch.from_numpy(events("gg_tt", 64, (400.0, 2000.0), stream=121)[0]).cuda()
        out = torch.empty(64, dtype=torch.float64, device="cuda")
        with pytest.raises(nl.NloError) as e:
            nl.nlo_me2(ctx.ctx, nl.proc_id("gg_tt"), 64, 64, mom.data_ptr(), out.data_ptr(), nl.NLO_FP16, 0)
        assert e.value.status == 1 and "nlo_reserve" in str(e.value)
        nl.nlo_reserve(ctx.ctx, 64)
        nl.nlo_me2(ctx.ctx, nl.proc_id("gg_tt"), 64, 64, mom.data_ptr(), out.data_ptr(), nl.NLO_FP16, 0)
        torch.cuda.synchronize()
        assert torch.all(torch.isfinite(out))
        for p in ("gg_ttg", "gg_ttgg"):
            assert ctx.colour_unit(p, "mixed") == "valu" and ctx.colour_unit(p, "fp64") == "valu"
        ctx.set_kernel_config("gg_ttg", "mixed", 256, 2)
        assert ctx.colour_unit("gg_ttg", "mixed") == "mfma"
    finally:
        ctx.close()
