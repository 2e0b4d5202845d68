"""Seeded synthetic workloads: process kinematics and the batch recipes.

Every event is a pure function of (seed, stream, event index) through the
counter-based Philox generator, so any sub-range of a workload can be
regenerated on its own.  Momenta are returned in the structure-of-arrays
layout ``mom[particle, component, event]`` (float64, GeV, components
E, px, py, pz), incoming particles first along +z and -z in the partonic
centre-of-mass frame.
"""
import math
import numpy as np

from .philox import uniforms
from .rambo import rambo

SEED = 7439
M_TOP = 173.0

# name -> (incoming particle names, outgoing particle names)
PROCESSES = {
    "ee_mumu": (("e-", "e+"), ("mu-", "mu+")),
    "ee_uu": (("e-", "e+"), ("u", "u~")),
    "ee_uug": (("e-", "e+"), ("u", "u~", "g")),
    "gg_tt": (("g", "g"), ("t", "t~")),
    "uu_tt": (("u", "u~"), ("t", "t~")),
    "gg_ttg": (("g", "g"), ("t", "t~", "g")),
    "uu_ttg": (("u", "u~"), ("t", "t~", "g")),
    "ug_ttu": (("u", "g"), ("t", "t~", "u")),
    "gg_ttgg": (("g", "g"), ("t", "t~", "g", "g")),
}


def mass(name, m_top=M_TOP):
    return m_top if name in ("t", "t~") else 0.0


def npart(proc):
    i, o = PROCESSES[proc]
    return len(i) + len(o)


def _sqrt_s(n, seed, stream, first, sqrt_s):
    if np.isscalar(sqrt_s):
        return np.full(n, float(sqrt_s))
    lo, hi = sqrt_s
    u = uniforms(seed, stream, np.arange(first, first + n), 64)[:, 0]
    return lo + (hi - lo) * u


def events(proc, n, sqrt_s, seed=SEED, stream=0, first=0, m_top=M_TOP):
    """RAMBO events for ``proc``; sqrt_s is a number or a (lo, hi) range drawn
    uniformly per event.  Returns (mom [npart, 4, n], weight [n])."""
    inc, out = PROCESSES[proc]
    nf = len(out)
    ev = np.arange(first, first + n, dtype=np.uint64)
    u = np.empty((n, nf, 4))
    for k in range(nf):
        u[:, k, 0:2] = uniforms(seed, stream, ev, 2 * k)
        u[:, k, 2:4] = uniforms(seed, stream, ev, 2 * k + 1)
    rs = _sqrt_s(n, seed, stream, first, sqrt_s)
    p, w = rambo(rs, [mass(x, m_top) for x in out], u)
    mom = np.empty((nf + 2, 4, n))
    h = 0.5 * rs
    mom[0, 0], mom[0, 1], mom[0, 2], mom[0, 3] = h, 0.0, 0.0, h
    mom[1, 0], mom[1, 1], mom[1, 2], mom[1, 3] = h, 0.0, 0.0, -h
    mom[2:] = np.transpose(p, (1, 2, 0))
    return mom, w


def fks_variables(n, seed=SEED, stream=0, first=0, initial_state=False, spread="log"):
    """FKS radiation variables (xi_tilde, y, phi) with xi_tilde and 1-|y|
    log-uniform in [1e-6, 1] (spread "log", the stress sets that crowd the
    soft and collinear limits; y >= 0), or xi_tilde and y uniform in (0, 1)
    and (-1, 1) (spread "flat", plain sampling of the radiation phase space),
    and phi uniform in [0, 2pi).  For an initial-state sector y takes a random
    sign."""
    ev = np.arange(first, first + n, dtype=np.uint64)
    u1 = uniforms(seed, stream, ev, 65)
    u2 = uniforms(seed, stream, ev, 66)
    if spread == "log":
        xi_t = 10.0 ** (-6.0 * u1[:, 0])
        omy = 10.0 ** (-6.0 * u1[:, 1])
    elif spread == "flat":
        xi_t = 1.0 - u1[:, 0]
        omy = (1.0 if initial_state else 2.0) * (1.0 - u1[:, 1])
    else:
        raise ValueError("spread must be 'log' or 'flat'")
    y = 1.0 - omy
    if initial_state:
        y = np.where(u2[:, 1] < 0.5, y, -y)
    phi = 2.0 * math.pi * u2[:, 0]
    return xi_t, y, phi


def to_aos(mom):
    """[npart, 4, n] -> [n, npart, 4] (contiguous)."""
    return np.ascontiguousarray(np.transpose(mom, (2, 0, 1)))


# Batch recipes: (process, number of events, sqrt_s or range, stream)
CONFIGS = {
    "ee_mumu_91": ("ee_mumu", 1 << 14, 91.188, 1),
    "ee_uug_1000": ("ee_uug", 1 << 20, 1000.0, 2),
    "gg_tt_400_2000": ("gg_tt", 1 << 22, (400.0, 2000.0), 31),
    "gg_ttg_400_2000": ("gg_ttg", 1 << 22, (400.0, 2000.0), 32),
    "gg_ttgg_400_2000": ("gg_ttgg", 1 << 20, (400.0, 2000.0), 41),
}


def config_events(name, n=None, first=0):
    proc, nfull, rs, stream = CONFIGS[name]
    return events(proc, nfull if n is None else n, rs, stream=stream, first=first)


# Uneven mix of Born, real and subtracted items for one batched launch:
# (kind, process, FKS pair (i, j; j = -1 both beams), Born process), each item
# with floor(10^U(3, 6)) events drawn from the seed; momenta with sqrt(s_hat)
# uniform in [400, 2000] GeV, stream MIX_STREAM + item index.
MIX_ITEMS = [
    ("me2", "gg_tt", None, None),
    ("me2", "uu_tt", None, None),
    ("me2", "gg_ttg", None, None),
    ("me2", "uu_ttg", None, None),
    ("me2", "ug_ttu", None, None),
    ("sub", "gg_ttg", (4, -1), "gg_tt"),
    ("sub", "uu_ttg", (4, -1), "uu_tt"),
    ("sub", "ug_ttu", (4, -1), "gg_tt"),
]
MIX_STREAM = 50


def mix_counts(lo=3.0, hi=6.0, seed=SEED, stream=MIX_STREAM):
    u = uniforms(seed, stream, np.arange(len(MIX_ITEMS)), 0)[:, 0]
    return np.floor(10.0 ** (lo + (hi - lo) * u)).astype(np.int64)
