"""Phase-space cuts of the event loop -- ORACLE, TEST INFRASTRUCTURE ONLY (the
same rules as the rest of oracle/: only tests/, the smoke check and the
benchmark's CPU-baseline leg use it).

The paper's Algorithm 2 applies a cut predicate passCuts(a, p) to every
contribution a in {Born, real, soft, collinear} at its own kinematics and
regenerates points until at least one passes; the paper defines no cuts.  The
reading implemented here (IR safe, so that the subtraction still cancels):

  jets: the final-state massless coloured partons clustered by the anti-kT
        algorithm with radius R in the (rapidity, azimuth) plane, E-scheme
        recombination; a jet counts when pT >= jet_ptmin and |y| <= jet_ymax,
        and an event needs at least njet_min counted jets.  A parton with
        pT = 0 (exactly along the beam) is not clustered.
  tops: every top quark needs pT >= top_ptmin and |y| <= top_ymax.
  leptons: every charged lepton needs pT >= lep_ptmin and |y| <= lep_ymax.

Plain Python loops, one event at a time, written from the definitions.  Every
comparison that decides the result is also checked for a near tie (the two
sides within `margin` relatively); `margin_hit` reports such events, whose
decision may legitimately differ in another implementation's rounding."""
import math

import numpy as np

# final-state leg classes per process (final-state index 0 = the first outgoing leg)
LEGS = {
    "ee_mumu": "ll", "ee_uu": "qq", "ee_uug": "qqq", "gg_tt": "tt", "uu_tt": "tt",
    "gg_ttg": "ttq", "uu_ttg": "ttq", "ug_ttu": "ttq", "gg_ttgg": "ttqq",
}

FIELDS = ("jet_r", "jet_ptmin", "jet_ymax", "njet_min", "top_ptmin", "top_ymax", "lep_ptmin", "lep_ymax")


def rapidity(p):
    """y = 1/2 ln((E + pz) / (E - pz)), from E +- |pz| and the transverse mass
    so that no difference of nearly equal numbers is taken"""
    e, px, py, pz = p
    mt2 = (e - abs(pz)) * (e + abs(pz)) if e > abs(pz) else 0.0
    pt2 = px * px + py * py
    mt2 = max(mt2, pt2)           # massless (or rounding): the transverse momentum itself
    if mt2 <= 0.0:
        return math.copysign(math.inf, pz)
    return math.copysign(math.log((e + abs(pz)) / math.sqrt(mt2)), pz)


def pt(p):
    return math.hypot(p[1], p[2])


def delta_r2(a, b):
    dphi = math.atan2(a[2], a[1]) - math.atan2(b[2], b[1])
    while dphi > math.pi:
        dphi -= 2 * math.pi
    while dphi < -math.pi:
        dphi += 2 * math.pi
    dy = rapidity(a) - rapidity(b)
    return dy * dy + dphi * dphi


class _Tie:
    def __init__(self, margin):
        self.margin = margin
        self.hit = False

    def le(self, a, b):
        if abs(a - b) <= self.margin * max(abs(a), abs(b)):
            self.hit = True
        return a <= b

    def lt(self, a, b):
        if abs(a - b) <= self.margin * max(abs(a), abs(b)):
            self.hit = True
        return a < b


def anti_kt(partons, R, tie):
    """jets (4-vectors) from a list of parton 4-vectors"""
    objs = [np.asarray(p, dtype=float) for p in partons if pt(p) > 0.0]
    jets = []
    while objs:
        # the smallest of d_iB = 1/pT_i^2 and d_ij = min(1/pT_i^2, 1/pT_j^2) dR_ij^2 / R^2,
        # the first one in list order on an exact tie
        cand = []
        for i, a in enumerate(objs):
            cand.append((1.0 / pt(a) ** 2, i, -1))
            for j in range(i + 1, len(objs)):
                b = objs[j]
                cand.append((min(1.0 / pt(a) ** 2, 1.0 / pt(b) ** 2) * delta_r2(a, b) / (R * R), i, j))
        best, bi, bj = cand[0]
        for d, i, j in cand[1:]:
            if d < best:
                best, bi, bj = d, i, j
        # a near tie decides the outcome unless both distances are beam
        # distances (the minimal beam distances become jets in either order)
        for d, i, j in cand:
            if (i, j) != (bi, bj) and not (j < 0 and bj < 0):
                tie.lt(d, best)
        if bj < 0:
            jets.append(objs.pop(bi))
        else:
            merged = objs[bi] + objs[bj]
            objs = [o for k, o in enumerate(objs) if k not in (bi, bj)] + [merged]
    return jets


def event_pass(final, legs, cuts, margin=1e-9):
    """(pass, margin_hit) for one event: final = final-state 4-vectors in leg
    order, legs = their classes ('q' massless parton, 't' top, 'l' lepton)"""
    tie = _Tie(margin)
    ok = True
    for p, c in zip(final, legs):
        if c == "t":
            ok &= tie.le(cuts["top_ptmin"], pt(p)) and tie.le(abs(rapidity(p)), cuts["top_ymax"])
        elif c == "l":
            ok &= tie.le(cuts["lep_ptmin"], pt(p)) and tie.le(abs(rapidity(p)), cuts["lep_ymax"])
    jets = anti_kt([p for p, c in zip(final, legs) if c == "q"], cuts["jet_r"], tie)
    count = sum(1 for j in jets if tie.le(cuts["jet_ptmin"], pt(j)) and tie.le(abs(rapidity(j)), cuts["jet_ymax"]))
    ok &= count >= cuts["njet_min"]
    return bool(ok), tie.hit


def cut_mask(proc, mom, cuts, margin=1e-9):
    """mom SoA [npart][4][n] -> (pass [n] bool, margin_hit [n] bool)"""
    legs = LEGS[proc]
    nin = mom.shape[0] - len(legs)
    n = mom.shape[2]
    ok = np.zeros(n, bool)
    hit = np.zeros(n, bool)
    for e in range(n):
        final = [mom[nin + k, :, e] for k in range(len(legs))]
        ok[e], hit[e] = event_pass(final, legs, cuts, margin)
    return ok, hit


def fks_masks(orc, real, i, j, born, born_mom, xi_tilde, y, phi, cuts, margin=1e-9):
    """The four mask bytes of an FKS sector, as the kernels read them, from
    the kinematics of each term: B and S at the Born point (the soft limit adds
    a zero-energy parton, which is not clustered); R at the real point of the
    map; C at the map's collinear end(s): for a final-state emitter y = 1,
    where i and j are collinear and merge (so C = B); for the beams y = +1 and
    y = -1 separately, encoded as 2 | 4 (y = +1 passes) | 8 (y = -1 passes).
    Returns (mask [4][n] uint8, margin_hit [n])."""
    n = born_mom.shape[2]
    okb, hb = cut_mask(born, born_mom, cuts, margin)
    _, _, realm = orc.fks_map(real, i, j, born_mom, xi_tilde, y, phi)
    okr, hr = cut_mask(real, realm, cuts, margin)
    mask = np.zeros((4, n), np.uint8)
    mask[0] = okb
    mask[1] = okr
    mask[2] = okb
    hit = hb | hr
    if j >= 0:
        mask[3] = okb
    else:
        _, _, rp = orc.fks_map(real, i, j, born_mom, xi_tilde, np.ones(n), phi)
        _, _, rm = orc.fks_map(real, i, j, born_mom, xi_tilde, -np.ones(n), phi)
        okp, hp = cut_mask(real, rp, cuts, margin)
        okm, hm = cut_mask(real, rm, cuts, margin)
        mask[3] = 2 | (okp * 4) | (okm * 8)
        hit |= hp | hm
    return mask, hit
