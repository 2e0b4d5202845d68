"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path
(``paper_2503_07439_amd``) and never imports it.

Thin ctypes wrapper around ``liboracle.so`` (built from ``oracle.cpp`` with
g++).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
# "double": IEEE double.  "quad": IEEE binary128 (__float128), the reference
# for the subtracted weight near the soft and collinear limits, where the
# weight keeps about log10(1/(xi (1-y))) fewer digits than the arithmetic.
_SO = {"double": os.path.join(_HERE, "liboracle.so"), "quad": os.path.join(_HERE, "liboracle_q.so"),
       "native": os.path.join(_HERE, "liboracle_native.so")}
_FLAGS = {"double": [], "quad": ["-DORACLE_QUAD"]}
_LIBS = {"double": [], "quad": ["-lquadmath"]}

PROCS = ["ee_mumu", "ee_uu", "ee_uug", "gg_tt", "uu_tt", "gg_ttg", "uu_ttg", "ug_ttu", "gg_ttgg"]


def build(verbose=False, kinds=("double", "quad")):
    """Compile the oracle (plain g++ -O3, no fast-math) in double and in
    binary128; the two builds run concurrently."""
    procs = []
    for k in kinds:
        tmp = _SO[k] + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread"] + _FLAGS[k] + ["-o", tmp, _SRC] + _LIBS[k]
        if verbose:
            print(" ".join(cmd))
        procs.append((subprocess.Popen(cmd), tmp, _SO[k]))
    for p, tmp, so in procs:
        if p.wait() != 0:
            raise RuntimeError("oracle build failed")
        os.replace(tmp, so)


def build_native():
    """The double build for this host's instruction set (-O3 -march=native,
    no fast-math), for timing the oracle as a CPU baseline.  Built on the host
    that runs it, every time (the instruction set differs between hosts)."""
    path = _SO["native"]
    tmp = path + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O3", "-march=native", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)
    _lib.pop("native", None)
    return path


_lib = {}


def _declare(L):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    L.orc_me2.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.c_int]
    L.orc_me2_hel.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, dp, ctypes.c_int]
    L.orc_me2_brute.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_int, dp, ctypes.c_int]
    L.orc_flows.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp, dp]
    L.orc_colour_matrix.argtypes = [ctypes.c_int, dp]
    L.orc_wavefunction.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp]
    L.orc_set_params.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.orc_proc_info.argtypes = [ctypes.c_int, ip, ip, dp, dp, ip, ip]
    return L


_params = None


def lib(kind="double"):
    """The loaded oracle library of the given arithmetic ("double", "quad")."""
    if kind not in _lib:
        if not os.path.exists(_SO[kind]):
            build_native() if kind == "native" else build(kinds=(kind,))
        _lib[kind] = _declare(ctypes.CDLL(_SO[kind]))
        if _params is not None:
            _lib[kind].orc_set_params(*_params)
    return _lib[kind]


def threads():
    """Worker threads for the oracle: the host's cores, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pid(proc):
    return PROCS.index(proc)


def set_params(alpha=1.0 / 132.507, alpha_s=0.118, m_top=173.0):
    global _params
    _params = (alpha, alpha_s, m_top)
    for L in _lib.values():
        L.orc_set_params(alpha, alpha_s, m_top)


def proc_info(proc):
    a, b = ctypes.c_int(), ctypes.c_int()
    c, d = ctypes.c_double(), ctypes.c_double()
    e, f = ctypes.c_int(), ctypes.c_int()
    lib().orc_proc_info(pid(proc), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                        ctypes.byref(e), ctypes.byref(f))
    return dict(npart=a.value, ncolour=b.value, avg=c.value, ident=d.value, a_pow=e.value, as_pow=f.value)


def me2(proc, mom, nthreads=8, kind="double"):
    """mom: [npart, 4, n] float64 (SoA).  Returns |M|^2 [n]."""
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    out = np.empty(n)
    rc = lib(kind).orc_me2(pid(proc), n, n, _dp(mom), _dp(out), nthreads)
    assert rc == 0
    return out


def me2_hel(proc, mom, nthreads=8):
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    nh = 1 << mom.shape[0]
    out = np.empty((nh, n))
    rc = lib().orc_me2_hel(pid(proc), n, n, _dp(mom), _dp(out), nthreads)
    assert rc == 0
    return out


def me2_brute(proc, mom, hel=-1, nthreads=8):
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    out = np.empty(n)
    rc = lib().orc_me2_brute(pid(proc), n, n, _dp(mom), hel, _dp(out), nthreads)
    assert rc == 0
    return out


def flows(proc, p_aos, hel, override_leg=-1, override_vec=None):
    """Colour-flow (or diagram) amplitudes for one event p_aos [npart, 4]."""
    p = np.ascontiguousarray(p_aos, dtype=np.float64)
    nc = proc_info(proc)["ncolour"]
    out = np.empty(2 * nc)
    ov = np.zeros(8)
    if override_vec is not None:
        ov[0::2] = np.real(override_vec)
        ov[1::2] = np.imag(override_vec)
    rc = lib().orc_flows(pid(proc), _dp(p), hel, override_leg, _dp(ov), _dp(out))
    assert rc == 0
    return out[0::2] + 1j * out[1::2]


def colour_matrix(proc):
    nc = proc_info(proc)["ncolour"]
    out = np.empty(2 * nc * nc)
    lib().orc_colour_matrix(pid(proc), _dp(out))
    return (out[0::2] + 1j * out[1::2]).reshape(nc, nc)


def wavefunction(proc, p_aos, leg, lam):
    p = np.ascontiguousarray(p_aos, dtype=np.float64)
    out = np.empty(8)
    lib().orc_wavefunction(pid(proc), _dp(p), leg, lam, _dp(out))
    return out[0::2] + 1j * out[1::2]


FKS_FIELDS = ["xi", "y", "g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm", "W", "me2_R", "B", "S", "jac", "dsig"]


def fks(real_proc, i, j, born_mom, xi_tilde, y, phi, nthreads=None, want_real=False, kind="double"):
    """FKS-subtracted real emission for pair (i, j) (j = -1: initial state).
    Returns dict of arrays (FKS_FIELDS) and optionally the real momenta.
    kind="quad" evaluates every step in binary128 (outputs rounded to double)."""
    L = lib(kind)
    if nthreads is None:
        nthreads = threads()
    f = L.orc_fks
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [ctypes.POINTER(ctypes.c_double)] * 6 + [ctypes.c_int]
    born_mom = np.ascontiguousarray(born_mom, dtype=np.float64)
    n = born_mom.shape[2]
    xi_tilde = np.ascontiguousarray(np.broadcast_to(xi_tilde, (n,)), dtype=np.float64)
    y = np.ascontiguousarray(np.broadcast_to(y, (n,)), dtype=np.float64)
    phi = np.ascontiguousarray(np.broadcast_to(phi, (n,)), dtype=np.float64)
    out = np.empty((n, 14))
    nreal = born_mom.shape[0] + 1
    real = np.empty((nreal, 4, n)) if want_real else None
    rc = f(pid(real_proc), i, j, n, _dp(born_mom), _dp(xi_tilde), _dp(y), _dp(phi), _dp(out),
           _dp(real) if want_real else ctypes.POINTER(ctypes.c_double)(), nthreads)
    assert rc == 0, rc
    res = {k: out[:, q].copy() for q, k in enumerate(FKS_FIELDS)}
    if want_real:
        res["real_mom"] = real
    return res


def fks_map(real_proc, i, j, born_mom, xi_tilde, y, phi, nthreads=None, kind="double"):
    """The FKS map of pair (i, j) without matrix elements: (xi, jac, real momenta
    SoA [nreal][4][n]), jac as in fks()."""
    L = lib(kind)
    if nthreads is None:
        nthreads = threads()
    f = L.orc_fks_map
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [ctypes.POINTER(ctypes.c_double)] * 6 + [ctypes.c_int]
    born_mom = np.ascontiguousarray(born_mom, dtype=np.float64)
    n = born_mom.shape[2]
    bc = lambda a: np.ascontiguousarray(np.broadcast_to(a, (n,)), dtype=np.float64)
    xi_tilde, y, phi = bc(xi_tilde), bc(y), bc(phi)
    out = np.empty((n, 2))
    real = np.empty((born_mom.shape[0] + 1, 4, n))
    rc = f(pid(real_proc), i, j, n, _dp(born_mom), _dp(xi_tilde), _dp(y), _dp(phi), _dp(out), _dp(real), nthreads)
    assert rc == 0, rc
    return out[:, 0].copy(), out[:, 1].copy(), real


def born_correlations(proc, mom):
    L = lib()
    f = L.orc_born_correlations
    f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    nl = ctypes.c_int()
    B = np.empty(n)
    Bkl = np.empty(n * 64)
    rc = f(pid(proc), n, _dp(mom), _dp(B), _dp(Bkl), ctypes.byref(nl))
    assert rc == 0
    k = nl.value
    return B, Bkl[:n * k * k].reshape(n, k, k)


def sector_functions(real_proc, real_mom):
    L = lib()
    f = L.orc_sector_functions
    f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_int)]
    real_mom = np.ascontiguousarray(real_mom, dtype=np.float64)
    n = real_mom.shape[2]
    out = np.empty(n * 8)
    k = ctypes.c_int()
    assert f(pid(real_proc), n, _dp(real_mom), _dp(out), ctypes.byref(k)) == 0
    return out[:n * k.value].reshape(n, k.value)


def born_spin_correlated(proc, mom, leg, eperp):
    L = lib()
    f = L.orc_born_spin_correlated
    f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    n = mom.shape[2]
    ep = np.ascontiguousarray(np.broadcast_to(eperp, (n, 4)), dtype=np.float64)
    out = np.empty(n)
    assert f(pid(proc), n, _dp(mom), leg, _dp(ep), _dp(out)) == 0
    return out


def rambo(sqrt_s, masses, u):
    """RAMBO from the uniforms u [n, nfin, 4] (cos theta, phi, two for the
    energy per particle) at per-event sqrt_s [n].  Returns (p [n, nfin, 4]
    with components E, px, py, pz in the final-state rest frame, weight [n])."""
    L = lib()
    f = L.orc_rambo
    f.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    sqrt_s = np.ascontiguousarray(sqrt_s, dtype=np.float64)
    masses = np.ascontiguousarray(masses, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n, nfin = u.shape[0], u.shape[1]
    p = np.empty((n, nfin, 4))
    w = np.empty(n)
    assert f(nfin, _dp(masses), n, _dp(sqrt_s), _dp(u), _dp(p), _dp(w)) == 0
    return p, w
