"""The generated amplitude code, built for the host, against the oracle.

The GPU kernels run the generator's per-process code: a nested helicity
schedule that sums one helicity of each reversed pair (doubled), takes the
gluons in their linear polarisations and contracts colour through the
Cholesky factor.  Compiled here for the CPU (hipcc, host only) and evaluated
per event, it must give the oracle's |M|^2, which sums every helicity in the
helicity basis with its own colour algebra: in double to 1e-11 per event, in
float to 1e-5 at the median and 1e-3 per event.  This catches a generator
mistake without a GPU; the GPU parity tests check the kernels themselves.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from nlo_inputs.workloads import PROCESSES, events
from physics import ALPHA, ALPHA_S, M_TOP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_07439_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def host_bin(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    if not os.path.exists(os.path.join(CSRC, "generated", "gg_ttg.hpp")):
        pytest.skip("generated code not present (run the build)")
    out = str(tmp_path_factory.mktemp("host_me2") / "host_me2")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-O1", "--offload-host-only", "-std=c++17",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), "-x", "hip",
           os.path.join(ROOT, "tests", "host_me2.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _run(host_bin, tmp_path, proc, mom, prec):
    n = mom.shape[2]
    src, dst = str(tmp_path / "mom.bin"), str(tmp_path / "out.bin")
    np.ascontiguousarray(mom, dtype=np.float64).tofile(src)
    subprocess.run([host_bin, proc, str(n), str(prec), str(mom.shape[0]), src, dst,
                    repr(ALPHA_S), repr(ALPHA), repr(M_TOP)], check=True, timeout=300)
    return np.fromfile(dst)


@pytest.mark.parametrize("proc", list(PROCESSES))
def test_generated_code_on_host_matches_oracle(orc, host_bin, tmp_path, proc):
    rs = 1000.0 if proc.startswith("ee") else (400.0, 2000.0)
    n = 96 if proc != "gg_ttgg" else 32
    mom, _ = events(proc, n, rs, stream=17)
    ref = orc.me2(proc, mom)
    assert np.all(ref > 0)
    d = _run(host_bin, tmp_path, proc, mom, 0)
    assert np.max(np.abs(d / ref - 1)) < 1e-11
    f = np.abs(_run(host_bin, tmp_path, proc, mom, 1) / ref - 1)
    assert np.median(f) < 1e-5 and f.max() < 1e-3
