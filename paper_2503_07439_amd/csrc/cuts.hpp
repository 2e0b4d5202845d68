// Phase-space cuts of the event loop (the paper's Algorithm 2 applies a cut
// predicate to every contribution at its own kinematics; the paper defines no
// cuts).  The cuts here are infrared safe, so that the subtraction still
// cancels: jets are the final-state massless coloured partons clustered by
// the anti-kT algorithm (radius R in rapidity and azimuth, four-momentum
// recombination); a jet counts when pT >= jet_ptmin and |y| <= jet_ymax, and
// an event needs at least njet_min of them; every top quark needs
// pT >= top_ptmin and |y| <= top_ymax, every charged lepton pT >= lep_ptmin
// and |y| <= lep_ymax.  A parton exactly along the beam (pT = 0) is not
// clustered.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "nlome.h"

namespace nlo {

// final-state leg classes: bit k = final-state leg k (the first outgoing leg is 0)
struct CutLegs {
  unsigned light, top, lep;
};

__device__ __forceinline__ double cut_pt(const double* p) { return sqrt(p[1] * p[1] + p[2] * p[2]); }

// y = 1/2 ln((E + pz)/(E - pz)) from E + |pz| and the transverse mass, so that
// no difference of nearly equal numbers enters
__device__ __forceinline__ double cut_rapidity(const double* p) {
  const double apz = fabs(p[3]);
  double mt2 = p[0] > apz ? (p[0] - apz) * (p[0] + apz) : 0.0;
  mt2 = fmax(mt2, p[1] * p[1] + p[2] * p[2]);
  if (mt2 <= 0.0) return copysign(HUGE_VAL, p[3]);
  return copysign(log((p[0] + apz) / sqrt(mt2)), p[3]);
}

__device__ __forceinline__ double cut_dr2(const double* a, const double* b) {
  double dphi = atan2(a[2], a[1]) - atan2(b[2], b[1]);
  while (dphi > M_PI) dphi -= 2.0 * M_PI;
  while (dphi < -M_PI) dphi += 2.0 * M_PI;
  const double dy = cut_rapidity(a) - cut_rapidity(b);
  return dy * dy + dphi * dphi;
}

// The cut decision for one event: fin[k] = final-state momentum k (NF legs)
template <int NF>
__device__ bool cut_pass(const double (&fin)[NF][4], const CutLegs& legs, const nlo_cuts& c) {
  bool ok = true;
  double obj[NF][4];
  int ord[NF], nobj = 0;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const double pt = cut_pt(fin[k]), ay = fabs(cut_rapidity(fin[k]));
    if ((legs.top >> k) & 1u) ok = ok && c.top_ptmin <= pt && ay <= c.top_ymax;
    if ((legs.lep >> k) & 1u) ok = ok && c.lep_ptmin <= pt && ay <= c.lep_ymax;
    if (((legs.light >> k) & 1u) && pt > 0.0) {
      for (int m = 0; m < 4; ++m) obj[nobj][m] = fin[k][m];
      ord[nobj] = nobj;
      ++nobj;
    }
  }
  // anti-kT: repeatedly the smallest of d_iB = 1/pT_i^2 and
  // d_ij = min(1/pT_i^2, 1/pT_j^2) dR_ij^2 / R^2; a beam distance makes i a
  // jet, a pair distance merges i and j into a new object at the end of the
  // list (the list order breaks exact ties)
  const double r2 = c.jet_r * c.jet_r;
  int njet = 0, live = nobj;
  while (live > 0) {
    double best = 0.0;
    int bi = -1, bj = -1;
    for (int a = 0; a < live; ++a) {
      const double* pa = obj[ord[a]];
      const double ia = 1.0 / (pa[1] * pa[1] + pa[2] * pa[2]);
      if (bi < 0 || ia < best) {
        best = ia;
        bi = a;
        bj = -1;
      }
      for (int b = a + 1; b < live; ++b) {
        const double* pb = obj[ord[b]];
        const double ib = 1.0 / (pb[1] * pb[1] + pb[2] * pb[2]);
        const double d = fmin(ia, ib) * cut_dr2(pa, pb) / r2;
        if (d < best) {
          best = d;
          bi = a;
          bj = b;
        }
      }
    }
    if (bj < 0) {
      const double* pj = obj[ord[bi]];
      if (c.jet_ptmin <= cut_pt(pj) && fabs(cut_rapidity(pj)) <= c.jet_ymax) ++njet;
      for (int a = bi; a + 1 < live; ++a) ord[a] = ord[a + 1];
      --live;
    } else {
      // the merged object reuses the slot of i; the list loses i and j and
      // gains the merged object at its end
      const int si = ord[bi], sj = ord[bj];
      for (int m = 0; m < 4; ++m) obj[si][m] += obj[sj][m];
      int w = 0;
      for (int a = 0; a < live; ++a)
        if (a != bi && a != bj) ord[w++] = ord[a];
      ord[w++] = si;
      live = w;
    }
  }
  return ok && njet >= c.njet_min;
}

}  // namespace nlo
