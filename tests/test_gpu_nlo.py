"""The Born-proportional virtual + integrated counterterms of e+e- -> u ubar
(nlo_virtual_integrated, through the C ABI) against the oracle
(oracle/nlo.py), and the complete NLO cross section assembled from device
pieces: sigma_B (1 + (V+I)/B) + the subtracted real emission integrated on
the device (nlo_integrate_subtracted, both FKS sectors, 2^20 points x 10
iterations) = sigma_B (1 + alpha_s / pi) within 4 standard errors."""
import math

import numpy as np
import pytest

from nlo_inputs.workloads import events
from oracle import nlo

pytestmark = pytest.mark.gpu

ALPHA, ALPHA_S = 1.0 / 132.507, 0.118
GEV2_PB = 0.3893793721e9


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2503_07439_amd as nl
    ctx = nl.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def test_virtual_integrated_matches_oracle(gpu, orc):
    import torch
    mom, _ = events("ee_uu", 1001, 1000.0, stream=701)
    b_ref, vi_ref = nlo.virtual_integrated(orc, mom)
    m = torch.from_numpy(mom).cuda()
    for prec, tol in (("fp64", 1e-13), ("mixed", 1e-5)):
        b, vi = gpu.virtual_integrated("ee_uu", m, prec)
        torch.cuda.synchronize()
        b, vi = b.cpu().numpy(), vi.cpu().numpy()
        assert np.all(np.abs(b / b_ref - 1) < tol) and np.all(np.abs(vi / vi_ref - 1) < tol), prec
        assert np.allclose(vi / b, nlo.vi_coefficient(ALPHA_S), rtol=1e-15, atol=0)


def test_nlo_k_factor_on_device(gpu):
    import torch
    rs, n = 1000.0, 1 << 20
    s = rs * rs
    mom, w = gpu.phase_space("ee_uu", n, rs, 702)
    b, vi = gpu.virtual_integrated("ee_uu", mom, "fp64")
    sig_b_mc = float((w * b).sum()) / n / (2 * s) * GEV2_PB
    sig_vi = float((w * vi).sum()) / n / (2 * s) * GEV2_PB
    sig_b = 3 * (2.0 / 3.0) ** 2 * 4 * math.pi * ALPHA ** 2 / (3 * s) * GEV2_PB     # closed form
    sig_r, err_r, chi2, _ = gpu.integrate_subtracted("ee_uug", rs, 1 << 20, 10, 3, 703, "fp64")
    k = 1 + sig_vi / sig_b_mc + sig_r / sig_b
    print("sigma_B %.8f pb (MC %.8f), (V+I)/B %.6f, sigma_R^sub %.9f +- %.2e pb (chi2/dof %.2f); "
          "K - 1 = %.7f +- %.7f, alpha_s/pi = %.7f" % (sig_b, sig_b_mc, sig_vi / sig_b_mc, sig_r, err_r, chi2, k - 1,
                                                      err_r / sig_b, ALPHA_S / math.pi), flush=True)
    assert abs(sig_b_mc / sig_b - 1) < 5e-3
    assert abs(k - 1 - ALPHA_S / math.pi) < 4 * err_r / sig_b
    assert err_r / sig_b < 1e-3 * ALPHA_S / math.pi


def test_virtual_integrated_argument_errors(gpu):
    import torch
    import paper_2503_07439_amd as nl
    m = torch.zeros((4, 4, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NloError) as e:
        gpu.virtual_integrated("gg_tt", m)
    assert e.value.status == 5
    with pytest.raises(nl.NloError) as e:
        gpu.virtual_integrated("ee_uu", m, "fp16")
    assert e.value.status == 5
