"""VEGAS adaptive Monte Carlo and the subtracted real-emission cross section --
ORACLE, TEST INFRASTRUCTURE ONLY (the same rules as the rest of oracle/: only
tests/, the smoke check and the benchmark's CPU-baseline leg use it).

Monte Carlo integration estimates an integral by the mean of the integrand at
random points (the paper's "Monte-Carlo integration" section); VEGAS (Lepage,
J. Comput. Phys. 27 (1978) 192) importance-samples each variable separately
on an adaptive grid.  Written here from the published algorithm, in plain
numpy and in the order of its steps:

  map:    a uniform u in [0, 1) picks bin b = floor(u NB) of a variable's grid,
          the point is x = e_b + (u NB - b)(e_{b+1} - e_b), and the point's
          weight gains the factor NB (e_{b+1} - e_b);
  refine: per variable, d_b = sum over the iteration's points in bin b of
          (f w)^2; smooth d_b with its neighbours (two-point averages at the
          ends); with D = sum d_b, compress r_b = ((1 - d_b/D) / ln(D/d_b))^alpha;
          place the new edges so that each new bin holds sum r_b / NB of r,
          r_b spread evenly over old bin b;
  result: per iteration the mean and its standard error; the iterations from
          nadapt on combined with inverse-variance weights, and their chi^2.

The integrand of `subtracted_cross_section` is the oracle's dsig (the
subtracted weight with the map's phase-space factor in every term, see
oracle.cpp) summed over the FKS sectors of a real process, at Born points
from the oracle's RAMBO, in pb."""
import math

import numpy as np

from nlo_inputs.philox import uniforms

CONV_PB = 0.3893793721e9          # GeV^-2 -> pb
NBINS = 50
ALPHA = 1.5


class Grid:
    def __init__(self, ndim, nbins=NBINS):
        self.nb = nbins
        self.edges = np.tile(np.linspace(0.0, 1.0, nbins + 1), (ndim, 1))

    def map(self, u):
        """u [n, D] -> x [n, D], weight [n], bin [n, D]"""
        n, D = u.shape
        x = np.empty_like(u)
        w = np.ones(n)
        bins = np.empty((n, D), dtype=np.int64)
        for d in range(D):
            t = u[:, d] * self.nb
            b = np.minimum(t.astype(np.int64), self.nb - 1)
            lo = self.edges[d, b]
            wd = self.edges[d, b + 1] - lo
            x[:, d] = lo + (t - b) * wd
            w *= self.nb * wd
            bins[:, d] = b
        return x, w, bins

    def refine(self, f, bins, alpha=ALPHA):
        nb = self.nb
        for d in range(self.edges.shape[0]):
            h = np.zeros(nb)
            for b in range(nb):
                h[b] = np.sum((f[bins[:, d] == b]) ** 2)
            sm = np.empty(nb)
            sm[0] = 0.5 * (h[0] + h[1])
            for b in range(1, nb - 1):
                sm[b] = (h[b - 1] + h[b] + h[b + 1]) / 3.0
            sm[nb - 1] = 0.5 * (h[nb - 2] + h[nb - 1])
            tot = sm.sum()
            if not tot > 0:
                continue
            r = np.zeros(nb)
            for b in range(nb):
                a = sm[b] / tot
                if a <= 0:
                    r[b] = 0.0
                elif a >= 1:
                    r[b] = 1.0
                else:
                    r[b] = ((1 - a) / (-math.log(a))) ** alpha
            if not r.sum() > 0:
                continue
            old = self.edges[d].copy()
            share = r.sum() / nb
            new = np.empty(nb + 1)
            new[0], new[nb] = 0.0, 1.0
            b, acc = 0, 0.0
            for k in range(1, nb):
                target = k * share
                while b < nb - 1 and acc + r[b] < target:
                    acc += r[b]
                    b += 1
                frac = (target - acc) / r[b] if r[b] > 0 else 0.0
                new[k] = old[b] + frac * (old[b + 1] - old[b])
            self.edges[d] = new


def uniforms_block(seed, stream, first, n, ndim):
    """u [n, ndim]: point k at counter first + k, variable d from slot d // 2"""
    ev = np.arange(first, first + n, dtype=np.uint64)
    cols = []
    for s in range((ndim + 1) // 2):
        cols.append(uniforms(seed, stream, ev, s))
    return np.concatenate(cols, axis=1)[:, :ndim]


def integrate(func, ndim, n, niter, nadapt, seed, stream):
    """VEGAS: func(x [n, ndim]) -> f [n], or (f, scale) with a per-point
    rounding scale of f.  A non-finite f counts as zero.  Returns (mean,
    error, chi2_dof, per-iteration [(mean, error)]), each iteration with a
    third entry, the mean of the weighted scale, when func gives one."""
    grid = Grid(ndim)
    its = []
    for it in range(niter):
        u = uniforms_block(seed, stream, it * n, n, ndim)
        x, w, bins = grid.map(u)
        r = func(x)
        f = (r[0] if isinstance(r, tuple) else r) * w
        f = np.where(np.isfinite(f), f, 0.0)
        mean = f.sum() / n
        var = max(0.0, (f * f).sum() / n - mean * mean) / (n - 1)
        its.append((mean, math.sqrt(var)) + ((float(np.sum(r[1] * w)) / n,) if isinstance(r, tuple) else ()))
        if it + 1 < niter:
            grid.refine(f, bins)
    keep = [(m, e) for m, e, *_ in its[nadapt:] if e > 0]
    sw = sum(1 / e ** 2 for _, e in keep)
    res = sum(m / e ** 2 for m, e in keep) / sw if sw > 0 else its[-1][0]
    chi = sum((m - res) ** 2 / e ** 2 for m, e in keep)
    dof = len(keep) - 1
    return res, (1 / math.sqrt(sw) if sw > 0 else 0.0), (chi / dof if dof > 0 else 0.0), its


def subtracted_integrand(orc, real, sectors, born, sqrt_s_born, masses, kind="double", with_scale=False):
    """x [n, 4 nf + 3] -> f [n]: conv * w_RAMBO * 4 pi * sum_sectors dsig at the
    Born point RAMBO makes of the first 4 nf variables and xi_tilde = x, y = 2x - 1,
    phi = 2 pi x from the last three.

    with_scale: also the conditioning scale of f, the same factors times
    xi_max max(j, j(0, y)) sum_X |g_X| / (2 s_B kappa) per sector (kappa =
    xi (1-y), or xi (1-y^2) for the beams): an FP64 evaluation of f is exact
    to about 1e-12 of it (the subtracted weight's own bound), however
    strongly the terms of dsig cancel."""
    nf = len(masses)
    sb = sqrt_s_born ** 2
    j0 = sb / (64 * math.pi ** 3)

    def f(x):
        n = x.shape[0]
        u = np.ascontiguousarray(x[:, :4 * nf].reshape(n, nf, 4))
        p, wb = orc.rambo(np.full(n, sqrt_s_born), np.asarray(masses, float), u)
        mom = np.empty((nf + 2, 4, n))
        h = 0.5 * sqrt_s_born
        mom[0] = np.array([[h], [0.0], [0.0], [h]])
        mom[1] = np.array([[h], [0.0], [0.0], [-h]])
        mom[2:] = np.transpose(p, (1, 2, 0))
        xt, y, phi = x[:, 4 * nf], 2 * x[:, 4 * nf + 1] - 1, 2 * math.pi * x[:, 4 * nf + 2]
        tot, scale = np.zeros(n), np.zeros(n)
        for i, j in sectors:
            r = orc.fks(real, i, j, mom, xt, y, phi, kind=kind)
            tot += r["dsig"]
            if with_scale:
                g = sum(np.abs(r[k]) for k in ("g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm"))
                kap = r["xi"] * (1 - y) * ((1 + y) if j < 0 else 1.0)
                xmax = r["xi"] / xt
                scale += xmax * np.maximum(r["jac"] / xmax, j0) * g / (2 * sb * kap)
        c = CONV_PB * wb * (2 * 2 * math.pi)
        return (c * tot, c * scale) if with_scale else c * tot
    return f
