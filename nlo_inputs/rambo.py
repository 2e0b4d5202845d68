"""RAMBO phase-space generator (Kleiss, Stirling, Ellis, Comput. Phys. Commun.
40 (1986) 359), vectorised over events, with the massive rescaling step.

Input generator only: it turns seeded uniforms into four-momenta and carries
no matrix-element arithmetic.  Both the oracle and the GPU path read the
arrays it writes.
"""
import math
import numpy as np


def massless_volume(nfin, s):
    """Lorentz-invariant massless n-body phase-space volume, (2pi)^(4-3n) included."""
    n = nfin
    return ((2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2)
            / (math.factorial(n - 1) * math.factorial(n - 2)))


def rambo(sqrt_s, masses, u):
    """sqrt_s: [N]; masses: length nfin; u: [N, nfin, 4] uniforms in (0,1).

    Returns (p [N, nfin, 4] with components (E, px, py, pz) in the frame where
    the final state is at rest, weight [N]).
    """
    sqrt_s = np.asarray(sqrt_s, dtype=np.float64)
    masses = np.asarray(masses, dtype=np.float64)
    nfin = masses.shape[0]
    # 1. isotropic massless momenta with energy density q0 exp(-q0)
    c = 2.0 * u[..., 0] - 1.0
    phi = 2.0 * math.pi * u[..., 1]
    q0 = -np.log(u[..., 2] * u[..., 3])
    st = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    q = np.stack([q0, q0 * st * np.cos(phi), q0 * st * np.sin(phi), q0 * c], axis=-1)
    # 2. conformal transformation to total momentum (sqrt_s, 0)
    Q = q.sum(axis=1)
    M = np.sqrt(Q[:, 0] ** 2 - Q[:, 1] ** 2 - Q[:, 2] ** 2 - Q[:, 3] ** 2)
    b = -Q[:, 1:] / M[:, None]
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    x = sqrt_s / M
    bq = np.einsum('nk,nik->ni', b, q[..., 1:])
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gam[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (q[..., 1:] + b[:, None, :] * q[..., 0:1]
                                     + (a[:, None] * bq)[..., None] * b[:, None, :])
    # The conformal boost amplifies rounding when gamma is large (nearly
    # collinear q's), leaving E != |p| and sum p != 0 at the 1e-12 level.
    # Project back: remove the residual three-momentum, put every momentum on
    # its massless shell and rescale to the exact total energy.  The shift is
    # of the order of the rounding error, so the distribution is unchanged.
    p[..., 1:] -= p[..., 1:].sum(axis=1, keepdims=True) / nfin
    pabs = np.sqrt((p[..., 1:] ** 2).sum(axis=-1))
    r = sqrt_s / pabs.sum(axis=1)
    p[..., 1:] *= r[:, None, None]
    p[..., 0] = pabs * r[:, None]
    w = np.full(sqrt_s.shape, 1.0) * massless_volume(nfin, 1.0) * sqrt_s ** (2 * (nfin - 2))
    if not np.any(masses > 0):
        return p, w
    # 3. massive rescaling: solve sum_i sqrt(m_i^2 + xi^2 E_i^2) = sqrt_s by Newton
    E = p[..., 0]
    m2 = masses[None, :] ** 2
    xi = np.sqrt(np.maximum(1e-30, 1.0 - (masses.sum() / sqrt_s) ** 2))
    for _ in range(50):
        ek = np.sqrt(m2 + (xi[:, None] * E) ** 2)
        f = ek.sum(axis=1) - sqrt_s
        fp = (xi[:, None] * E * E / ek).sum(axis=1)
        step = f / fp
        xi = xi - step
        if np.all(np.abs(f) <= 1e-14 * sqrt_s):
            break
    k = np.empty_like(p)
    k[..., 1:] = xi[:, None, None] * p[..., 1:]
    k[..., 0] = np.sqrt(m2 + (xi[:, None] * E) ** 2)
    kabs = np.sqrt(k[..., 1] ** 2 + k[..., 2] ** 2 + k[..., 3] ** 2)
    w = (w * (kabs.sum(axis=1) / sqrt_s) ** (2 * nfin - 3)
         * np.prod(kabs / k[..., 0], axis=1)
         * sqrt_s / (kabs ** 2 / k[..., 0]).sum(axis=1))
    return k, w
