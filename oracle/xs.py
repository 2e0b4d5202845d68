"""Reference partonic cross sections -- ORACLE, TEST INFRASTRUCTURE ONLY (the
same rules as the rest of oracle/: only tests/, the smoke check and the
benchmark's CPU-baseline leg use it).

sigma(sqrt_s) of a 2 -> 2 process by Gauss-Legendre quadrature of the
oracle's |M|^2 over the scattering angle, sigma = (1/(2s)) (beta/(16 pi))
int |M|^2 dcos(theta) (two-body phase space beta/(8 pi) with the azimuth
integrated), and by plain Monte Carlo over the oracle's RAMBO points."""
import math

import numpy as np

from nlo_inputs.philox import uniforms

GEV2_PB = 0.3893793721e9


def two_body_momenta(rs, cos_t, m3, m4):
    n = cos_t.shape[0]
    s = rs * rs
    p = math.sqrt((s - (m3 + m4) ** 2) * (s - (m3 - m4) ** 2)) / (2 * rs)
    e3 = math.sqrt(m3 * m3 + p * p)
    e4 = math.sqrt(m4 * m4 + p * p)
    sin_t = np.sqrt(1 - cos_t ** 2)
    mom = np.zeros((4, 4, n))
    mom[0, 0], mom[0, 3] = rs / 2, rs / 2
    mom[1, 0], mom[1, 3] = rs / 2, -rs / 2
    mom[2, 0], mom[2, 1], mom[2, 3] = e3, p * sin_t, p * cos_t
    mom[3, 0], mom[3, 1], mom[3, 3] = e4, -p * sin_t, -p * cos_t
    return mom, 2 * p / rs


def sigma_quadrature(orc, proc, rs, m3, m4, order=64):
    x, wq = np.polynomial.legendre.leggauss(order)
    mom, beta = two_body_momenta(rs, x, m3, m4)
    me2 = orc.me2(proc, mom)
    return GEV2_PB / (2 * rs * rs) * beta / (16 * math.pi) * float(np.dot(wq, me2))


def sigma_mc(orc, proc, rs, masses, n, stream, seed=7439, ident=1.0):
    ev = np.arange(n, dtype=np.uint64)
    nf = len(masses)
    u = np.empty((n, nf, 4))
    for k in range(nf):
        u[:, k, 0:2] = uniforms(seed, stream, ev, 2 * k)
        u[:, k, 2:4] = uniforms(seed, stream, ev, 2 * k + 1)
    p, w = orc.rambo(np.full(n, rs), masses, u)
    mom = np.empty((nf + 2, 4, n))
    mom[0, 0], mom[0, 1], mom[0, 2], mom[0, 3] = rs / 2, 0.0, 0.0, rs / 2
    mom[1, 0], mom[1, 1], mom[1, 2], mom[1, 3] = rs / 2, 0.0, 0.0, -rs / 2
    mom[2:] = np.transpose(p, (1, 2, 0))
    f = w * orc.me2(proc, mom) * ident * GEV2_PB / (2 * rs * rs)
    return f.mean(), f.std(ddof=1) / math.sqrt(n), f
