// FKS-subtracted real emission on the GPU (the paper's FKS subtraction and
// the branch-free evaluation of Born, real, soft and collinear terms per
// phase-space point, with masks applied afterwards).
//
// Per FKS sector (real process R, Born process B, FKS pair (I, J), J < 0 for
// the initial state) three launches:
//  1. k_fks_map (FP64): Born momenta + (xi_tilde, y, phi) -> real momenta,
//     written to a workspace in bucket order (FP32 bucket from the front,
//     FP64 bucket from the back) with the inverse permutation;
//  2. the |M|^2 kernels of R on each bucket, each in its own precision;
//  3. k_fks_born (per bucket, T = float or double): recomputes the FP64
//     kinematics, evaluates B, the colour-linked Borns B_kl (from the
//     helicity-summed density of the flow vector) and the spin-correlated Born
//     with the emitter polarisation replaced by the transverse unit vector,
//     then assembles the counterterms and the subtracted weight in FP64.
//
// Reading of the conventions (the paper leaves them open):
//   xi = 2 k_i^0/sqrt(s_R); y = cos(k_i, k_j) (final J) or cos(k_i, beam 1);
//   phi = azimuth about the emitter measured from the (emitter, z) plane.
//   FSR: xi_max = 1 - M_rec^2/s; recoilers boosted along the emitter axis.
//   ISR: xi_max = 1 - s_B/s_cap (sqrt(s_cap) = 4000 GeV), s_R = s_B/(1-xi),
//        Born final state pure-boosted to K = p1 + p2 - k_i.
//   f(xi,y) = xi^2 (1-y) |M_R|^2 S  (FSR),  xi^2 (1-y^2) |M_R|^2 S  (ISR)
//   W_FSR = [f - f(0,y) - f(xi,1) + f(0,1)] / (xi (1-y))
//   W_ISR = [f - f(0,y) - (1+y)/2 (f(xi,1)-f(0,1)) - (1-y)/2 (f(xi,-1)-f(0,-1))] / (xi (1-y^2))
//   Sector functions S = (h_IJ/d_IJ)/sum_pairs(h/d), d = xi_k xi_l (1-y_kl)
//   or xi_k (1-y_k^2) for the beams, h = xi_l/(xi_k+xi_l) for gluon pairs.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "cuts.hpp"
#include "helas.hpp"
#include "launch.hpp"

namespace nlo {

constexpr double FKS_SCAP = 4000.0 * 4000.0;   // notional hadronic s for the ISR xi_max
constexpr double FKS_CF = 4.0 / 3.0, FKS_CA = 3.0;

struct FksKin {
  double xi, y, sqs_b, sb, sqs_r;
  double nh[3];   // direction of parton I (soft limit)
  double ep[3];   // transverse unit vector of the collinear limit
  double ejc, z;  // FSR: E_J at y = 1 and its momentum fraction there
  double omz;     // FSR: 1 - z = E_I / E_J(Born), formed without cancellation
  double ei, ej;  // energies of partons I and J (FSR), or of I and of each beam (ISR)
  double ejb;     // FSR: energy of the Born emitter
  double xmax;    // xi_max
};

__device__ __forceinline__ double d3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ __forceinline__ double mink(const double* a, const double* b) {
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

// unit vectors orthogonal to kh: e1 in the plane of kh and z, e2 = kh x e1
__device__ __forceinline__ void fks_perp(const double* kh, double* e1, double* e2) {
  const double st = sqrt(kh[0] * kh[0] + kh[1] * kh[1]);
  const double ct = kh[2];
  const double cp = st > 0.0 ? kh[0] / st : 1.0, sp = st > 0.0 ? kh[1] / st : 0.0;
  e1[0] = ct * cp; e1[1] = ct * sp; e1[2] = -st;
  e2[0] = -sp; e2[1] = cp; e2[2] = 0.0;
}

// The Born point is on shell and conserves momentum by definition.  An input
// rounded to double does neither exactly (at the 1e-16 level), and the real
// emission meets its counterterms only as closely as it does, which would
// leave a term of that size over xi (1-y) in W.  So the final-state
// three-momenta are shifted by a common amount to sum to zero, every energy
// is put on its mass shell, and the beams (along +-z in the partonic frame)
// carry half the total energy each.
template <class S>
__device__ __forceinline__ void fks_project_born(double (&kb)[S::NB][4], double mt) {
  using BP = typename S::Born;
  constexpr int NF = S::NB - 2;
  double res[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 2; k < S::NB; ++k)
#pragma unroll
    for (int m = 0; m < 3; ++m) res[m] += kb[k][1 + m];
  double etot = 0.0;
#pragma unroll
  for (int k = 2; k < S::NB; ++k) {
#pragma unroll
    for (int m = 0; m < 3; ++m) kb[k][1 + m] -= res[m] / NF;
    const double m2 = ((BP::TOP_LEGS >> k) & 1u) ? mt * mt : 0.0;
    kb[k][0] = sqrt(d3(kb[k] + 1, kb[k] + 1) + m2);
    etot += kb[k][0];
  }
  kb[0][0] = 0.5 * etot; kb[0][1] = 0.0; kb[0][2] = 0.0; kb[0][3] = 0.5 * etot;
  kb[1][0] = 0.5 * etot; kb[1][1] = 0.0; kb[1][2] = 0.0; kb[1][3] = -0.5 * etot;
}

// real kinematics of one event
template <class S>
__device__ void fks_map(const double (&kb)[S::NB][4], double xit, double y, double phi, double (&kr)[S::NR][4],
                        FksKin& K) {
  K.y = y;
  K.sqs_b = kb[0][0] + kb[1][0];
  K.sb = K.sqs_b * K.sqs_b;
  const double sy = sqrt((1.0 - y) * (1.0 + y));
  double cphi, sphi;
  sincos(phi, &sphi, &cphi);
  if constexpr (S::J >= 0) {
    const double* kj = kb[S::JB];
    const double sq = K.sqs_b;
    const double rec[4] = {sq - kj[0], -kj[1], -kj[2], -kj[3]};
    const double mrec2 = mink(rec, rec);
    const double xi = xit * (1.0 - mrec2 / K.sb);
    const double ei = 0.5 * xi * sq;
    const double ej = (K.sb - mrec2 - 2.0 * sq * ei) / (2.0 * sq - 2.0 * ei * (1.0 - y));
    const double kabs = sqrt(ei * ei + ej * ej + 2.0 * ei * ej * y);
    const double kjabs = sqrt(d3(kj + 1, kj + 1));
    const double kh[3] = {kj[1] / kjabs, kj[2] / kjabs, kj[3] / kjabs};
    double e1[3], e2[3];
    fks_perp(kh, e1, e2);
    const double cti = (ei + ej * y) / kabs, sti = ej * sy / kabs;
    double kid[3];
    for (int m = 0; m < 3; ++m) {
      K.ep[m] = cphi * e1[m] + sphi * e2[m];
      kid[m] = cti * kh[m] + sti * K.ep[m];
      K.nh[m] = y * kh[m] + sy * K.ep[m];
    }
    // recoil: light-cone component E + p.u along u = -kh scaled by rho
    const double rho = (sq - ei - ej + kabs) / (sq - kj[0] + kjabs);
#pragma unroll
    for (int r = 0; r < S::NR; ++r) {
      if (r == S::I) {
        kr[r][0] = ei;
        for (int m = 0; m < 3; ++m) kr[r][1 + m] = ei * kid[m];
      } else if (r == S::J) {
        kr[r][0] = ej;
        for (int m = 0; m < 3; ++m) kr[r][1 + m] = kabs * kh[m] - ei * kid[m];
      } else {
        const double* p = kb[S::BMAP[r]];
        if (r < 2) {
          for (int m = 0; m < 4; ++m) kr[r][m] = p[m];
        } else {
          const double pl = -d3(p + 1, kh);
          const double pp = p[0] + pl, pm = p[0] - pl;
          const double e2n = 0.5 * (rho * pp + pm / rho), pl2 = 0.5 * (rho * pp - pm / rho);
          kr[r][0] = e2n;
          for (int m = 0; m < 3; ++m) kr[r][1 + m] = p[1 + m] - (pl2 - pl) * kh[m];
        }
      }
    }
    K.xi = xi;
    K.sqs_r = sq;
    K.ejc = kj[0] - ei;
    K.z = K.ejc / kj[0];
    K.omz = ei / kj[0];
    K.ei = ei;
    K.ej = ej;
    K.ejb = kj[0];
    K.xmax = 1.0 - mrec2 / K.sb;
  } else {
    const double xi = xit * (1.0 - K.sb / FKS_SCAP);
    const double sr = K.sb / (1.0 - xi);
    const double sqr = sqrt(sr);
    const double ei = 0.5 * xi * sqr;
    K.nh[0] = sy * cphi; K.nh[1] = sy * sphi; K.nh[2] = y;
    K.ep[0] = cphi; K.ep[1] = sphi; K.ep[2] = 0.0;
    // pure boost from the Born rest frame to K = p1 + p2 - k_i (K^2 = s_B)
    const double Kv[4] = {sqr - ei, -ei * K.nh[0], -ei * K.nh[1], -ei * K.nh[2]};
    const double M = K.sqs_b;
#pragma unroll
    for (int r = 0; r < S::NR; ++r) {
      if (r == 0 || r == 1) {
        kr[r][0] = 0.5 * sqr; kr[r][1] = 0.0; kr[r][2] = 0.0; kr[r][3] = r == 0 ? 0.5 * sqr : -0.5 * sqr;
      } else if (r == S::I) {
        kr[r][0] = ei;
        for (int m = 0; m < 3; ++m) kr[r][1 + m] = ei * K.nh[m];
      } else {
        const double* p = kb[S::BMAP[r]];
        const double bp = (Kv[1] * p[1] + Kv[2] * p[2] + Kv[3] * p[3]) / M;
        kr[r][0] = (Kv[0] * p[0]) / M + bp;
        const double f = p[0] / M + bp / (Kv[0] + M);
        for (int m = 0; m < 3; ++m) kr[r][1 + m] = p[1 + m] + f * Kv[1 + m];
      }
    }
    K.xi = xi;
    K.sqs_r = sqr;
    K.ejc = 0.0;
    K.z = 0.0;
    K.omz = 0.0;
    K.ei = ei;
    K.ej = 0.5 * sqr;
    K.ejb = 0.0;
    K.xmax = 1.0 - K.sb / FKS_SCAP;
  }
}

// Pairwise invariants 2 q_a.q_b (all momenta incoming) of the FKS pair, from
// the radiation variables: a final-state pair gives 2 k_I.k_J = 2 E_I E_J (1-y);
// the beams give -2 p_1.k_I = -2 E_1 E_I (1-y) and -2 p_2.k_I = -2 E_2 E_I (1+y).
// Formed from the rounded real momenta these invariants would carry a relative
// error of about eps/(xi (1-|y|)), which the real |M|^2 inherits.
template <class S>
__device__ __forceinline__ void fks_pair_invariants(const FksKin& K, double& v0, double& v1) {
  if constexpr (S::J >= 0) {
    v0 = 2.0 * K.ei * K.ej * (1.0 - K.y);
    v1 = 0.0;
  } else {
    v0 = -2.0 * K.ej * K.ei * (1.0 - K.y);
    v1 = -2.0 * K.ej * K.ei * (1.0 + K.y);
  }
}

// sector function of the pair (I, J) at the real point; the FKS pair's angle
// is the radiation variable y itself
template <class S>
__device__ double fks_sector(const double (&k)[S::NR][4], double sqs, double y) {
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int q = 0; q < S::NPAIR; ++q) {
    const int a = S::PI[q], b = S::PJ[q];
    const double xa = 2.0 * k[a][0] / sqs;
    const double pa = sqrt(d3(k[a] + 1, k[a] + 1));
    double t;
    if (b < 0) {
      const double ya = (S::J < 0 && a == S::I) ? y : k[a][3] / pa;
      t = 1.0 / (xa * (1.0 - ya) * (1.0 + ya));
    } else {
      const double xb = 2.0 * k[b][0] / sqs;
      const double pb = sqrt(d3(k[b] + 1, k[b] + 1));
      const bool pair = S::J >= 0 && ((a == S::I && b == S::J) || (a == S::J && b == S::I));
      const double yab = pair ? y : d3(k[a] + 1, k[b] + 1) / (pa * pb);
      const double h = (S::GLUON[a] && S::GLUON[b]) ? xb / (xa + xb) : 1.0;
      t = h / (xa * xb * (1.0 - yab));
    }
    den += t;
    if (a == S::I && b == S::J) num = t;
  }
  return num / den;
}

// its soft limit: parton I along nh, the others at their Born momenta
template <class S>
__device__ double fks_sector_soft(const double (&kb)[S::NB][4], const double* nh, double sqs_b, double yv) {
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int q = 0; q < S::NPAIR; ++q) {
    if (S::PI[q] != S::I) continue;
    const int b = S::PJ[q];
    double t;
    if (b < 0) {
      t = 1.0 / ((1.0 - nh[2]) * (1.0 + nh[2]));
    } else {
      const double* p = kb[S::BMAP[b]];
      // the soft direction makes the angle y with the emitter by construction
      const double y = b == S::J ? yv : d3(nh, p + 1) / sqrt(d3(p + 1, p + 1));
      t = 1.0 / ((2.0 * p[0] / sqs_b) * (1.0 - y));
    }
    den += t;
    if (b == S::J) num = t;
  }
  return num / den;
}

// ---------------------------------------------------------------------------
// launch arguments
// ---------------------------------------------------------------------------
struct FksArgs {
  int64_t n, ld;                       // events, leading dimension of the caller's arrays
  const double* born;                  // [NB][4][ld]
  const double *xit, *y, *phi;         // [n]
  const uint8_t* mask;                 // [4][ld] for B, R, S, C or null
  double* real;                        // workspace [NR][4][n], bucket order
  double* pinv;                        // workspace [2][n], bucket order: the FKS pair invariants
  double* me2r;                        // workspace [n], bucket order
  unsigned* inv;                       // workspace [n]: bucket position -> event
  unsigned* cnt;                       // workspace [8]: FP32 and FP64 bucket sizes, then the same
                                       // for the events whose real emission is skipped, then the
                                       // length of redo
  unsigned* skip_inv;                  // workspace [n]: skipped events (compact mode), FP32 from
                                       // the front, FP64 from the back
  unsigned* redo;                      // workspace [n] (MIXED): positions of FP32 events whose W
                                       // came out unresolved or non-finite, evaluated again in
                                       // FP64: bucket positions from the front (cnt[4]), skipped-
                                       // list positions from the back (cnt[5])
  int compact;                         // 1: events failing the R cut skip the real |M|^2
  double thr;                          // route to FP64 when kappa = xi (1-y) (final-state J) or
                                       // xi (1-y^2) (beams) is below thr
  int mode;                            // 0: all FP32, 1: all FP64, 2: route
  double scale_b, g2, mt;
  double scale_bm;                     // coupling x average factor of the y -> -1 Born (quark FKS parton)
  double *xi_out, *born_out, *gR, *gS, *gC, *gCm, *gSC, *gSCm, *W;   // [n], any may be null but W
  double *dsig, *jac;                  // [n] or null
  uint8_t* status;                     // [n] or null
  double* real_out;                    // [NR][4][ld] (event order) or null
};

// the Born point of event e, projected on shell (fks_project_born)
template <class S>
__device__ __forceinline__ void load_born(const FksArgs& a, int64_t e, double (&kb)[S::NB][4]) {
#pragma unroll
  for (int k = 0; k < S::NB; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) kb[k][m] = a.born[(k * 4 + m) * a.ld + e];
  fks_project_born<S>(kb, a.mt);
}

static __global__ void k_fks_zero(unsigned* cnt) {
  if (threadIdx.x < 8) cnt[threadIdx.x] = 0u;
}

// 1. map and route.  Every event goes to the FP32 or the FP64 bucket; in
// compact mode an event whose R cut fails goes to the skipped list instead,
// so the real |M|^2 is not evaluated for it (its counterterms still are).
template <class S>
__global__ __launch_bounds__(NLO_MAX_BLOCK) void k_fks_map(FksArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = e < a.n;
  double kb[S::NB][4], kr[S::NR][4];
  FksKin K;
  bool f64 = false, skip = false;
  if (act) {
    load_born<S>(a, e, kb);
    fks_map<S>(kb, a.xit[e], a.y[e], a.phi[e], kr, K);
    // W = (g_R - counterterms) / kappa cancels by about 1/kappa, so the FP32
    // rounding of the real |M|^2 reaches W amplified by that much
    const double kappa = S::J >= 0 ? K.xi * (1.0 - K.y) : K.xi * ((1.0 - K.y) * (1.0 + K.y));
    f64 = (a.mode == 1) || (a.mode == 2 && !(kappa >= a.thr));
    skip = a.compact && a.mask && !a.mask[1 * a.ld + e];
  }
  // positions in the four lists (FP32, FP64, and the two of events that
  // skip the real |M|^2): wave ballots, then one atomic per list and block
  const unsigned long long m32 = __ballot(act && !f64 && !skip), m64 = __ballot(act && f64 && !skip);
  const unsigned long long s32 = __ballot(act && !f64 && skip), s64 = __ballot(act && f64 && skip);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lower = lane ? (~0ull >> (64 - lane)) : 0ull;
  unsigned b32, b64, c32, c64;
  if (a.mode == 1 && !a.compact) {
    // every event in the FP64 list, in event order from the back: no atomics
    b32 = c32 = c64 = 0u;
    b64 = (unsigned)((int64_t)blockIdx.x * blockDim.x + wave * 64);
    if (e == 0) a.cnt[1] = (unsigned)a.n;
  } else {
    __shared__ unsigned wc[NLO_MAX_BLOCK / 64][4], wb[NLO_MAX_BLOCK / 64][4];
    const int nw = (int)(blockDim.x + 63) >> 6;
    if (lane == 0) {
      wc[wave][0] = (unsigned)__popcll(m32);
      wc[wave][1] = (unsigned)__popcll(m64);
      wc[wave][2] = (unsigned)__popcll(s32);
      wc[wave][3] = (unsigned)__popcll(s64);
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      const int l = threadIdx.x;
      unsigned tot = 0u;
      for (int w = 0; w < nw; ++w) tot += wc[w][l];
      unsigned base = tot ? atomicAdd(&a.cnt[l], tot) : 0u;
      for (int w = 0; w < nw; ++w) {
        wb[w][l] = base;
        base += wc[w][l];
      }
    }
    __syncthreads();
    b32 = wb[wave][0];
    b64 = wb[wave][1];
    c32 = wb[wave][2];
    c64 = wb[wave][3];
  }
  if (!act) return;
  if (skip) {
    const int64_t pos = f64 ? a.n - 1 - (int64_t)(c64 + __popcll(s64 & lower)) : (int64_t)(c32 + __popcll(s32 & lower));
    a.skip_inv[pos] = (unsigned)e;
  } else {
    const int64_t pos = f64 ? a.n - 1 - (int64_t)(b64 + __popcll(m64 & lower)) : (int64_t)(b32 + __popcll(m32 & lower));
    a.inv[pos] = (unsigned)e;
#pragma unroll
    for (int k = 0; k < S::NR; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) a.real[(k * 4 + m) * a.n + pos] = kr[k][m];
    double v0, v1;
    fks_pair_invariants<S>(K, v0, v1);
    a.pinv[pos] = v0;
    a.pinv[a.n + pos] = v1;
  }
  if (a.real_out) {
#pragma unroll
    for (int k = 0; k < S::NR; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) a.real_out[(k * 4 + m) * a.ld + e] = kr[k][m];
  }
}

// spin-correlated Born: leg LEG's polarisation replaced by (0, ep), summed
// over the other helicities.  The real vector is its own conjugate, so
// reversing all the other helicities leaves the colour-summed square
// unchanged (as for |M|^2): with HEL_SYM = 2 one more leg (PIN) is held at
// bit 0 and the sum doubled.
template <class BP, int LEG, class T>
__device__ double born_spin(const typename BP::template Pre<T>& s, const double* ep, T mt) {
  constexpr int PIN = LEG == 0 ? 1 : 0;
  const w4<T> ov = {{cx<T>{T(0), T(0)}, cx<T>{T(ep[0]), T(0)}, cx<T>{T(ep[1]), T(0)}, cx<T>{T(ep[2]), T(0)}}};
  double acc = 0.0;
#pragma unroll 1
  for (int h = 0; h < BP::NHEL; ++h) {
    if ((h >> (BP::NPART - 1 - LEG)) & 1) continue;
    if (BP::HEL_SYM == 2 && ((h >> (BP::NPART - 1 - PIN)) & 1)) continue;
    cx<T> J[BP::NFLOW];
    BP::template amplitudes<T, LEG>(s, h, mt, J, &ov);
    acc += (double)BP::colour_sum(J);
  }
  return acc * BP::HEL_SYM;
}

// Algorithm-2 masks (a failed cut zeroes its contribution after evaluation),
// the subtracted weight and the per-event outputs
template <class S>
__device__ __forceinline__ void fks_store(const FksArgs& a, int which, int64_t pos, int64_t e, double B, double gR,
                                          double gS, double gC, double gCm, double gSC, double gSCm, const FksKin& K) {
  const double xi = K.xi, y = K.y;
  // which & 1: evaluated in FP64 (buckets 1, 3 and the redo lists 5, 7)
  uint8_t st = (which & 1) ? (which >= 5 ? 2 | 16 : 2) : 0;
  double Bo = B;
  if (a.mask) {
    const bool mB = a.mask[0 * a.ld + e], mR = a.mask[1 * a.ld + e], mS = a.mask[2 * a.ld + e];
    // C byte: non-zero = passes; with bit 1 set, bits 2 and 3 give the y = +1
    // and y = -1 ends of the beams separately
    const uint8_t mC = a.mask[3 * a.ld + e];
    const bool cp = (mC & 2) ? (mC & 4) != 0 : mC != 0, cm = (mC & 2) ? (mC & 8) != 0 : mC != 0;
    if (!mB) Bo = 0.0;
    if (!mR) gR = 0.0;
    if (!mS) gS = 0.0;
    if (!cp) gC = 0.0;
    if (!cm) gCm = 0.0;
    if (!mS || !cp) gSC = 0.0;
    if (!mS || !cm) gSCm = 0.0;
    if (!(mB && mR && mS && cp && (S::J >= 0 || cm))) st |= 4;
  }
  double W;
  if constexpr (S::J >= 0) {
    W = (gR - gS - gC + gSC) / (xi * (1.0 - y));
  } else {
    W = (gR - gS - 0.5 * (1.0 + y) * (gC - gSC) - 0.5 * (1.0 - y) * (gCm - gSCm)) / (xi * (1.0 - y) * (1.0 + y));
  }
  if (!isfinite(W)) st |= 1;
  // bit 3: W not resolved in its working precision.  W cancels terms of
  // size D = sum|g_X| / kappa, and its rounding error is measured against D:
  // within 1e-12 D with the FP64 real |M|^2 (measured against the binary128
  // oracle: at most 3.3e-13 D), within 32 eps_32 (1 + 1/sqrt(1-|y|)) D with
  // the FP32 one (the collinear spinor products lose digits like
  // 1/sqrt(1-|y|)).  Set when that bound exceeds 1e-3 |W|.
  {
    const double kap = S::J >= 0 ? xi * (1.0 - y) : xi * ((1.0 - y) * (1.0 + y));
    const double D = (fabs(gR) + fabs(gS) + fabs(gC) + fabs(gCm) + fabs(gSC) + fabs(gSCm)) / kap;
    const double c = (which & 1) ? 1e-12 : 32.0 * 0x1p-24 * (1.0 + 1.0 / sqrt(1.0 - fabs(y)));
    if (!(c * D <= 1e-3 * fabs(W))) st |= 8;
  }
  // MIXED: an FP32 event whose W is unresolved or not finite goes on the redo
  // list (wave-aggregated append; the FP64 pass overwrites every output of
  // the event): bucket positions from the front, skipped ones from the back
  if ((which == 0 || which == 2) && a.mode == 2) {
    const bool redo = (st & 9) != 0;
    const unsigned long long m = __ballot(redo);
    if (m) {
      const int lane = __lane_id();
      const int leader = __ffsll((long long)m) - 1;
      unsigned base = 0u;
      if (lane == leader) base = atomicAdd(&a.cnt[which == 0 ? 4 : 5], (unsigned)__popcll(m));
      base = __shfl(base, leader);
      const int64_t k = (int64_t)base + __popcll(m & ((1ull << lane) - 1ull));
      if (redo) a.redo[which == 0 ? k : a.n - 1 - k] = (unsigned)pos;
    }
  }
  a.W[e] = W;
  if (a.dsig || a.jac) {
    // the map's phase-space factor at the event and at the limits each term
    // stands for (final state: j(0,y) = j(0,1) = j0, j(xi,1) = z j0; beams:
    // j = j0 / (1 - xi) wherever xi is kept, j0 at xi = 0)
    const double j0 = K.sb / (64.0 * M_PI * M_PI * M_PI);
    double jr, num;
    if constexpr (S::J >= 0) {
      jr = j0 * (K.ej / K.ejb) / (1.0 - 0.5 * xi * (1.0 - y));
      num = (jr * gR - j0 * gS - K.z * j0 * gC + j0 * gSC) / (xi * (1.0 - y));
    } else {
      jr = j0 / (1.0 - xi);
      num = (jr * (gR - 0.5 * (1.0 + y) * gC - 0.5 * (1.0 - y) * gCm)
             - j0 * (gS - 0.5 * (1.0 + y) * gSC - 0.5 * (1.0 - y) * gSCm)) / (xi * (1.0 - y) * (1.0 + y));
    }
    if (a.dsig) a.dsig[e] = K.xmax * num / (2.0 * K.sb);
    if (a.jac) a.jac[e] = K.xmax * jr;
  }
  if (a.xi_out) a.xi_out[e] = xi;
  if (a.born_out) a.born_out[e] = Bo;
  if (a.gR) a.gR[e] = gR;
  if (a.gS) a.gS[e] = gS;
  if (a.gC) a.gC[e] = gC;
  if (a.gCm) a.gCm[e] = gCm;
  if (a.gSC) a.gSC[e] = gSC;
  if (a.gSCm) a.gSCm[e] = gSCm;
  if (a.status) a.status[e] = st;
}

// helicity- and colour-summed |M|^2 of a Born (without its average factor)
template <class BP, class T>
__device__ __forceinline__ double born_sum(const double (&kb)[BP::NPART][4], double mt) {
  typename BP::template Pre<T> s;
  BP::prologue(kb, s, mt);
  double acc = 0.0;
  BP::helicity_sum(s, T(mt), [&](const cx<T> (&J)[BP::NFLOW]) { acc += (double)BP::colour_sum(J); });
  return acc * BP::HEL_SYM;   // the sum covers one of each pair (h, -h)
}

// Quark FKS parton from the initial state (e.g. u g -> t tbar u with the
// final u): a soft quark is not singular, so g_S = g_SC = 0; at y -> +1 the
// incoming quark of beam 1 turns into a gluon entering the Born (P_gq with its
// spin correlation, C_F [x B + 4 (1-x)/x B_perp]); at y -> -1 the gluon of
// beam 2 turns into an antiquark (P_qg = T_R [x^2 + (1-x)^2] B of the other
// Born).  Real and Born are averaged over their own initial states, so the
// unpolarised kernels apply without a ratio of spin x colour states.
template <class S, class T>
__device__ __forceinline__ void fks_quark_isr(const FksArgs& a, int which, int64_t pos, int64_t e,
                                              const double (&kb)[S::NB][4], const FksKin& K, double S_real) {
  using BP = typename S::Born;
  using BM = typename S::BornM;
  const double xi = K.xi, y = K.y, g2 = a.g2, x = 1.0 - xi;
  typename BP::template Pre<T> sp;
  BP::prologue(kb, sp, a.mt);
  double bp = 0.0;
  BP::helicity_sum(sp, T(a.mt), [&](const cx<T> (&J)[BP::NFLOW]) { bp += (double)BP::colour_sum(J); });
  const double Bplus = bp * BP::HEL_SYM * a.scale_b;
  const double Bperp = born_spin<BP, 0, T>(sp, K.ep, T(a.mt)) * a.scale_b;
  const double Bminus = born_sum<BM, T>(kb, a.mt) * a.scale_bm;
  const double Pp = FKS_CF * (x * Bplus + 4.0 * xi / x * Bperp);
  const double Pm = 0.5 * (x * x + xi * xi) * Bminus;
  const bool skipped = which == 2 || which == 3 || which == 7;
  const double gR = skipped ? 0.0 : xi * xi * (1.0 - y) * (1.0 + y) * a.me2r[pos] * S_real;
  fks_store<S>(a, which, pos, e, Bplus, gR, 0.0, 8.0 * xi * g2 / K.sb * Pp, 8.0 * xi * g2 / K.sb * Pm, 0.0, 0.0, K);
}

// 3. Born correlations, counterterms and subtracted weight for one bucket
template <class S, class T>
__global__ __launch_bounds__(NLO_MAX_BLOCK) void k_fks_born(FksArgs a, int launch) {
  using BP = typename S::Born;
  // launch: 0 / 1 the FP32 / FP64 bucket of evaluated real emissions, 2 / 3
  // the FP32 / FP64 part of the skipped list (no real |M|^2: its R cut
  // failed); MIXED, in FP64: 9 the FP64 bucket, then the FP32-bucket
  // positions on the redo list, 11 the FP64 part of the skipped list, then
  // the skipped positions on the redo list.  Each event is evaluated and
  // stored as `which`: 0 to 3 as above, 5 / 7 a re-evaluated bucket /
  // skipped event.
  int which = launch;
  int64_t pos;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (launch == 9 || launch == 11) {
    const int64_t c = a.cnt[launch == 9 ? 1 : 3];
    if (i < c) {
      pos = a.n - c + i;
      which = launch == 9 ? 1 : 3;
    } else {
      const int64_t j = i - c;
      if (j >= (int64_t)a.cnt[launch == 9 ? 4 : 5]) return;
      pos = a.redo[launch == 9 ? j : a.n - 1 - j];
      which = launch == 9 ? 5 : 7;
    }
  } else {
    const bool back = launch & 1;
    const int64_t lo = back ? a.n - (int64_t)a.cnt[launch] : 0;
    const int64_t hi = back ? a.n : (int64_t)a.cnt[launch];
    pos = lo + i;
    if (pos >= hi) return;
  }
  const bool skipped = which == 2 || which == 3 || which == 7;
  const int64_t e = skipped ? a.skip_inv[pos] : a.inv[pos];
  double kb[S::NB][4], kr[S::NR][4];
  FksKin K;
  load_born<S>(a, e, kb);
  fks_map<S>(kb, a.xit[e], a.y[e], a.phi[e], kr, K);
  const double S_real = fks_sector<S>(kr, K.sqs_r, K.y);
  if constexpr (S::QUARK_I) {
    fks_quark_isr<S, T>(a, which, pos, e, kb, K, S_real);
    return;
  } else {
  // compact mode: an event none of whose Born-level terms (B, S, C) passes
  // its cut skips the Born amplitudes; the masks would zero them anyway, so
  // the outputs are those of the branch-free evaluation bit for bit
  if (a.compact && a.mask) {
    const uint8_t mC = a.mask[3 * a.ld + e];
    const bool cany = (mC & 2) ? (mC & 12) != 0 : mC != 0;
    if (!a.mask[0 * a.ld + e] && !a.mask[2 * a.ld + e] && !cany) {
      const double me2r = skipped ? 0.0 : a.me2r[pos];
      const double gR = S::J >= 0 ? K.xi * K.xi * (1.0 - K.y) * me2r * S_real
                                  : K.xi * K.xi * (1.0 - K.y) * (1.0 + K.y) * me2r * S_real;
      fks_store<S>(a, which, pos, e, 0.0, gR, 0.0, 0.0, 0.0, 0.0, 0.0, K);
      return;
    }
  }

  // Born: |M|^2 and the helicity-summed density Re(J_u J_v^*) of the flow
  // vector, over the nested schedule of the |M|^2 kernels.  Both sums are
  // unchanged by reversing every helicity (J -> phase J^*) and by summing a
  // leg over any orthonormal basis of its states, so the schedule's half of
  // the helicities (doubled) and its linear gluon polarisations apply.
  typename BP::template Pre<T> s;
  BP::prologue(kb, s, a.mt);
  double rho[BP::NRHO];
#pragma unroll
  for (int q = 0; q < BP::NRHO; ++q) rho[q] = 0.0;
  double bsum = 0.0;
  BP::helicity_sum(s, T(a.mt), [&](const cx<T> (&J)[BP::NFLOW]) {
    bsum += (double)BP::colour_sum(J);
    int q = 0;
#pragma unroll
    for (int u = 0; u < BP::NFLOW; ++u)
#pragma unroll
      for (int v = u; v < BP::NFLOW; ++v, ++q) rho[q] += (double)(J[u].r * J[v].r + J[u].i * J[v].i);
  });
#pragma unroll
  for (int q = 0; q < BP::NRHO; ++q) rho[q] *= BP::HEL_SYM;
  double bkl[BP::NCL][BP::NCL];
  BP::colour_corr(rho, bkl);
  const double B = bsum * BP::HEL_SYM * a.scale_b;
  // eikonal factor -sum_kl (p_k.p_l)/((p_k.n)(p_l.n)) B_kl with n = (1, nh).
  // The soft direction makes the angle y with the emitter (or beam 1), so
  // there p.n = E (1 -+ y) exactly; from the components it would lose
  // digits as 1/(1-|y|).
  const double n4[4] = {1.0, K.nh[0], K.nh[1], K.nh[2]};
  double pn[BP::NCL];
#pragma unroll
  for (int k = 0; k < BP::NCL; ++k) {
    const int leg = BP::CLEG[k];
    const double* pk = kb[leg];
    if (S::J >= 0 && leg == S::JB) pn[k] = pk[0] * (1.0 - K.y);
    else if (S::J < 0 && leg == 0) pn[k] = pk[0] * (1.0 - K.y);
    else if (S::J < 0 && leg == 1) pn[k] = pk[0] * (1.0 + K.y);
    else pn[k] = mink(pk, n4);
  }
  // p_k.p_k is the nominal m_k^2 (zero for a massless parton): formed from
  // the components it would leave rounding over (p_k.n)^2 ~ (1-y)^2
  double eik = 0.0;
#pragma unroll
  for (int k = 0; k < BP::NCL; ++k)
#pragma unroll
    for (int l = 0; l < BP::NCL; ++l) {
      const double* pk = kb[BP::CLEG[k]];
      const double* pl = kb[BP::CLEG[l]];
      const double pkl = k != l ? mink(pk, pl) : (((BP::TOP_LEGS >> BP::CLEG[k]) & 1u) ? a.mt * a.mt : 0.0);
      eik -= pkl / (pn[k] * pn[l]) * bkl[k][l] * a.scale_b;
    }
  const double Ss = fks_sector_soft<S>(kb, K.nh, K.sqs_b, K.y);
  const double xi = K.xi, y = K.y, g2 = a.g2;
  const double me2r = skipped ? 0.0 : a.me2r[pos];
  double gR, gS, gC, gCm = 0.0, gSC, gSCm = 0.0;
  if constexpr (S::J >= 0) {
    gR = xi * xi * (1.0 - y) * me2r * S_real;
    gS = (1.0 - y) * 4.0 / K.sb * g2 * eik * Ss;
    const double z = K.z, omz = K.omz;
    const double Sc = S::J_GLUON && S::GLUON[S::I] ? z : 1.0;
    double P, Cj;
    if constexpr (S::J_GLUON) {
      const double Bp = born_spin<BP, S::JB, T>(s, K.ep, T(a.mt)) * a.scale_b;
      P = 2.0 * FKS_CA * ((z / omz + omz / z) * B + 2.0 * z * omz * Bp);
      Cj = FKS_CA;
    } else {
      P = FKS_CF * (1.0 + z * z) / omz * B;
      Cj = FKS_CF;
    }
    gC = 2.0 * xi * g2 / (K.sqs_b * K.ejc) * P * Sc;
    gSC = 8.0 * g2 * Cj / K.sb * B;
  } else {
    gR = xi * xi * (1.0 - y) * (1.0 + y) * me2r * S_real;
    gS = (1.0 - y) * (1.0 + y) * 4.0 / K.sb * g2 * eik * Ss;
    const double x = 1.0 - xi;
    double Pp, Pm, Cp, Cm;
    if constexpr (S::BEAM_GLUON0) {
      const double Bp = born_spin<BP, 0, T>(s, K.ep, T(a.mt)) * a.scale_b;
      Pp = 2.0 * FKS_CA * ((x / xi + x * xi) * B + 2.0 * xi / x * Bp);
      Cp = FKS_CA;
    } else {
      Pp = FKS_CF * (1.0 + x * x) / xi * B;
      Cp = FKS_CF;
    }
    if constexpr (S::BEAM_GLUON1) {
      const double Bp = born_spin<BP, 1, T>(s, K.ep, T(a.mt)) * a.scale_b;
      Pm = 2.0 * FKS_CA * ((x / xi + x * xi) * B + 2.0 * xi / x * Bp);
      Cm = FKS_CA;
    } else {
      Pm = FKS_CF * (1.0 + x * x) / xi * B;
      Cm = FKS_CF;
    }
    gC = 8.0 * xi * g2 / K.sb * Pp;
    gCm = 8.0 * xi * g2 / K.sb * Pm;
    gSC = 16.0 * g2 * Cp / K.sb * B;
    gSCm = 16.0 * g2 * Cm / K.sb * B;
  }
  fks_store<S>(a, which, pos, e, B, gR, gS, gC, gCm, gSC, gSCm, K);
  }
}

// Fixed-order FP64 sum of x[0, n): block b of FKS_SUM_PARTS reduces its
// contiguous share into part[b] (strided per thread, then a tree), and one
// block adds the parts the same way.  The order depends on n only, so the sum
// is reproducible bit for bit.
constexpr int FKS_SUM_PARTS = 512;

static __global__ __launch_bounds__(256) void k_sum_part(int64_t n, const double* __restrict__ x,
                                                         double* __restrict__ part) {
  __shared__ double t[256];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += x[i];
  t[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) t[threadIdx.x] += t[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = t[0];
}

static __global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double t[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < FKS_SUM_PARTS; i += blockDim.x) s += part[i];
  t[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) t[threadIdx.x] += t[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = t[0];
}

// ---------------------------------------------------------------------------
// cut masks of an FKS sector: every term at its own kinematics
// ---------------------------------------------------------------------------
struct FksCutArgs {
  int64_t n, ld;
  const double* born;              // [NB][4][ld]
  const double *xit, *y, *phi;     // [n]
  double mt;
  nlo_cuts cuts;
  uint8_t* mask;                   // [4][ld]: B, R, S, C
};

template <class P, int NF>
__device__ __forceinline__ CutLegs cut_legs_of() {
  constexpr unsigned all = (1u << NF) - 1u;
  const unsigned top = (P::TOP_LEGS >> 2) & all, lep = (P::LEP_LEGS >> 2) & all;
  return CutLegs{all & ~top & ~lep, top, lep};
}

// B and S at the Born point as given (the soft limit adds a zero-energy
// parton, which is not clustered); R at the real point of the map; C at the
// map's collinear end(s): a final-state emitter's y = 1 point has i and j
// collinear, which the jet algorithm merges back into the Born jet (C = B);
// for the beams the y = +1 and y = -1 points are evaluated and encoded as
// 2 | 4 (y = +1 passes) | 8 (y = -1 passes).
template <class S>
__global__ __launch_bounds__(256) void k_fks_cuts(FksCutArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n) return;
  constexpr int NBF = S::NB - 2, NRF = S::NR - 2;
  double kb[S::NB][4], fb[NBF][4], fr[NRF][4], kr[S::NR][4];
#pragma unroll
  for (int k = 0; k < S::NB; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) kb[k][m] = a.born[(k * 4 + m) * a.ld + e];
#pragma unroll
  for (int k = 0; k < NBF; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) fb[k][m] = kb[k + 2][m];
  const bool pb = cut_pass<NBF>(fb, cut_legs_of<typename S::Born, NBF>(), a.cuts);
  fks_project_born<S>(kb, a.mt);
  const CutLegs lr = cut_legs_of<typename S::Real, NRF>();
  auto real_pass = [&](double y) {
    FksKin K;
    fks_map<S>(kb, a.xit[e], y, a.phi[e], kr, K);
#pragma unroll
    for (int k = 0; k < NRF; ++k)
#pragma unroll
      for (int m = 0; m < 4; ++m) fr[k][m] = kr[k + 2][m];
    return cut_pass<NRF>(fr, lr, a.cuts);
  };
  const bool pr = real_pass(a.y[e]);
  uint8_t c;
  if constexpr (S::J >= 0) {
    c = pb;
  } else {
    c = (uint8_t)(2u | (real_pass(1.0) ? 4u : 0u) | (real_pass(-1.0) ? 8u : 0u));
  }
  a.mask[0 * a.ld + e] = pb;
  a.mask[1 * a.ld + e] = pr;
  a.mask[2 * a.ld + e] = pb;
  a.mask[3 * a.ld + e] = c;
}

template <class S>
hipError_t launch_fks_cuts(const FksCutArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_fks_cuts<S>), dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <class S>
hipError_t launch_fks_map(const FksArgs& a, int block, hipStream_t st) {
  hipLaunchKernelGGL(k_fks_zero, dim3(1), dim3(64), 0, st, a.cnt);
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL((k_fks_map<S>), dim3((unsigned)grid), dim3(block), 0, st, a);
  return hipGetLastError();
}

template <class S, class T>
hipError_t launch_fks_born(const FksArgs& a, int launch, int block, hipStream_t st) {
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL((k_fks_born<S, T>), dim3((unsigned)grid), dim3(block), 0, st, a, launch);
  return hipGetLastError();
}

}  // namespace nlo
