// On-device phase-space generation: the random numbers, RAMBO points and FKS
// radiation variables of a batch, produced where the matrix elements are
// evaluated (the paper's event loop draws phase-space points per event;
// keeping that step on the device removes the host round trip).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), a
// counter-based generator, so every draw is a pure function of
// (seed, stream, event index, slot) whatever the launch shape.  Key =
// (seed, stream), counter = (event low word, event high word, slot, 0); the
// four output words give two doubles of 53 random bits each, offset by half a
// unit of the last place so that log(u) is finite.  Slot layout of an event
// (the batch recipe): 2k and 2k+1 for final-state particle k, 64 for
// sqrt(s_hat), 65 and 66 for the FKS variables.
//
// Phase space: RAMBO (Kleiss, Stirling and Ellis) in the partonic
// centre-of-mass frame, beams along +z and -z, with the projection of the
// conformal transformation's rounding and the Newton rescaling for massive
// final states.  One event per lane, all in FP64.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "cuts.hpp"
#include "phase_space.hpp"

namespace nlo {

struct philox_out { uint32_t w[4]; };

__device__ __forceinline__ philox_out philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                     uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   // round multipliers
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   // Weyl key increments
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return {{c0, c1, c2, c3}};
}

// two uniforms in (0, 1) for (event, slot)
__device__ __forceinline__ void uniform2(uint32_t seed, uint32_t stream, uint64_t e, uint32_t slot, double& a,
                                         double& b) {
  const philox_out o = philox4x32_10((uint32_t)e, (uint32_t)(e >> 32), slot, 0u, seed, stream);
  const uint64_t ia = ((uint64_t)(o.w[0] >> 5) << 26) | (o.w[1] >> 6);
  const uint64_t ib = ((uint64_t)(o.w[2] >> 5) << 26) | (o.w[3] >> 6);
  const double s = 1.0 / 9007199254740992.0;   // 2^-53
  a = ((double)ia + 0.5) * s;
  b = ((double)ib + 0.5) * s;
}

__global__ __launch_bounds__(256) void k_uniforms(int64_t n, uint32_t seed, uint32_t stream, uint64_t first,
                                                  uint32_t slot, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a, b;
  uniform2(seed, stream, first + (uint64_t)i, slot, a, b);
  out[2 * i] = a;
  out[2 * i + 1] = b;
}

// One RAMBO point from 4 NF uniforms per event (u[k] = cos theta, phi and
// the two uniforms of the energy of particle k): momenta p[k] in the partonic
// centre-of-mass frame at sqrt(s) = rs, and the phase-space weight w (the
// volume for massless particles, times the massive correction).
template <int NF>
__device__ void rambo_point(const double (&u)[NF][4], double rs, const double* mass, double (&p)[NF][4], double& w) {
  // isotropic massless momenta, energy density q0 exp(-q0)
  double q[NF][4], Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const double c = 2.0 * u[k][0] - 1.0, ph = 2.0 * M_PI * u[k][1];
    const double en = -log(u[k][2] * u[k][3]);
    const double st = sqrt(fmax(0.0, 1.0 - c * c));
    double sp, cp;
    sincos(ph, &sp, &cp);
    q[k][0] = en; q[k][1] = en * st * cp; q[k][2] = en * st * sp; q[k][3] = en * c;
#pragma unroll
    for (int m = 0; m < 4; ++m) Q[m] += q[k][m];
  }
  // boost by -Q/M and scale by sqrt_s/M: total momentum (sqrt_s, 0)
  const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double bx = -Q[1] / M, by = -Q[2] / M, bz = -Q[3] / M;
  const double g = Q[0] / M, al = 1.0 / (1.0 + g), x = rs / M;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const double bq = bx * q[k][1] + by * q[k][2] + bz * q[k][3];
    p[k][0] = x * (g * q[k][0] + bq);
    p[k][1] = x * (q[k][1] + bx * q[k][0] + al * bq * bx);
    p[k][2] = x * (q[k][2] + by * q[k][0] + al * bq * by);
    p[k][3] = x * (q[k][3] + bz * q[k][0] + al * bq * bz);
  }
  // remove the rounding the transformation leaves: zero total three-momentum,
  // massless shells, exact total energy
  double r3[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int m = 0; m < 3; ++m) r3[m] += p[k][1 + m];
  double pa[NF], tot = 0.0;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
#pragma unroll
    for (int m = 0; m < 3; ++m) p[k][1 + m] -= r3[m] / NF;
    pa[k] = sqrt(p[k][1] * p[k][1] + p[k][2] * p[k][2] + p[k][3] * p[k][3]);
    tot += pa[k];
  }
  const double sc = rs / tot;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
#pragma unroll
    for (int m = 0; m < 3; ++m) p[k][1 + m] *= sc;
    p[k][0] = pa[k] * sc;
  }
  // massless volume (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!)
  w = pow(2.0 * M_PI, 4 - 3 * NF) * pow(0.5 * M_PI, NF - 1);
#pragma unroll
  for (int k = 2; k <= NF - 1; ++k) w /= k;
#pragma unroll
  for (int k = 2; k <= NF - 2; ++k) w /= k;
  w *= pow(rs, 2 * (NF - 2));
  double msum = 0.0;
  bool massive = false;
#pragma unroll
  for (int k = 0; k < NF; ++k) { msum += mass[k]; massive = massive || mass[k] > 0.0; }
  if (massive) {
    // common factor xi on the three-momenta with sum_k sqrt(m_k^2 + xi^2 E_k^2) = sqrt_s
    double xi = sqrt(fmax(1e-30, 1.0 - (msum / rs) * (msum / rs)));
    for (int it = 0; it < 50; ++it) {
      double f = -rs, fp = 0.0;
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        const double ek = sqrt(mass[k] * mass[k] + xi * xi * p[k][0] * p[k][0]);
        f += ek;
        fp += xi * p[k][0] * p[k][0] / ek;
      }
      xi -= f / fp;
      if (fabs(f) <= 1e-14 * rs) break;
    }
    double ksum = 0.0, kprod = 1.0, k2e = 0.0;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const double k0 = sqrt(mass[k] * mass[k] + xi * xi * p[k][0] * p[k][0]);
#pragma unroll
      for (int m = 0; m < 3; ++m) p[k][1 + m] *= xi;
      p[k][0] = k0;
      const double ka = sqrt(p[k][1] * p[k][1] + p[k][2] * p[k][2] + p[k][3] * p[k][3]);
      ksum += ka;
      kprod *= ka / k0;
      k2e += ka * ka / k0;
    }
    w *= pow(ksum / rs, 2 * NF - 3) * kprod * rs / k2e;
  }
}

// beams along +z and -z, then the final state, into mom[(particle 4 + mu) ld + i]
template <int NF>
__device__ __forceinline__ void store_event(const double (&p)[NF][4], double rs, double* mom, int64_t ld, int64_t i) {
  const double h = 0.5 * rs;
  const double beams[2][4] = {{h, 0.0, 0.0, h}, {h, 0.0, 0.0, -h}};
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int m = 0; m < 4; ++m) mom[(b * 4 + m) * ld + i] = beams[b][m];
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) mom[((k + 2) * 4 + m) * ld + i] = p[k][m];
}

// the batch recipe's point of event e: sqrt(s_hat) from slot 64, particle k
// from slots 2k and 2k + 1
template <int NF>
__device__ __forceinline__ void recipe_point(uint32_t seed, uint32_t stream, uint64_t e, double rs_lo, double rs_hi,
                                             const double* mass, double (&p)[NF][4], double& w, double& rs) {
  double u0, u1;
  uniform2(seed, stream, e, 64, u0, u1);
  rs = rs_lo + (rs_hi - rs_lo) * u0;
  double u[NF][4];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    uniform2(seed, stream, e, 2 * k, u[k][0], u[k][1]);
    uniform2(seed, stream, e, 2 * k + 1, u[k][2], u[k][3]);
  }
  rambo_point<NF>(u, rs, mass, p, w);
}

template <int NF>
__global__ __launch_bounds__(256) void k_rambo(PsArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double p[NF][4], w, rs;
  recipe_point<NF>(a.seed, a.stream, a.first + (uint64_t)i, a.rs_lo, a.rs_hi, a.mass, p, w, rs);
  store_event<NF>(p, rs, a.mom, a.ld, i);
  if (a.weight) a.weight[i] = w;
}

// ---------------------------------------------------------------------------
// cuts (cuts.hpp) on batches, and Algorithm 2's regenerate-until-pass loop as
// stream compaction
// ---------------------------------------------------------------------------
template <int NF>
__global__ __launch_bounds__(256) void k_cut_mask(int64_t n, int64_t ld, int nin, const double* __restrict__ mom,
                                                  CutLegs legs, nlo_cuts cuts, uint8_t* __restrict__ pass) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double fin[NF][4];
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) fin[k][m] = mom[((nin + k) * 4 + m) * ld + e];
  pass[e] = cut_pass<NF>(fin, legs, cuts) ? 1 : 0;
}

// passing candidates of this block's 256 (wave ballots, waves in order):
// returns the candidate's rank among them, or -1 if it fails
__device__ __forceinline__ int block_rank(bool ok, unsigned* total) {
  __shared__ unsigned wcnt[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(ok);
  if (lane == 0) wcnt[wave] = (unsigned)__popcll(m);
  __syncthreads();
  unsigned before = 0u;
  for (int w = 0; w < wave; ++w) before += wcnt[w];
  if (total) *total = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
  const unsigned long long lower = lane ? (~0ull >> (64 - lane)) : 0ull;
  return ok ? (int)(before + (unsigned)__popcll(m & lower)) : -1;
}

// pass 1: how many of each block's 256 candidates pass
template <int NF>
__global__ __launch_bounds__(256) void k_gen_count(GenArgs a) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool ok = false;
  if (c < a.m) {
    double p[NF][4], w, rs;
    recipe_point<NF>(a.seed, a.stream, a.first + (uint64_t)c, a.rs_lo, a.rs_hi, a.mass, p, w, rs);
    ok = cut_pass<NF>(p, a.legs, a.cuts);
  }
  unsigned tot;
  (void)block_rank(ok, &tot);
  if (threadIdx.x == 0) a.bcount[blockIdx.x] = tot;
}

// exclusive scan of the block counts in block order (one block of 256
// threads: each thread owns a contiguous run of blocks), and the total
__global__ __launch_bounds__(256) void k_gen_scan(int nblocks, const unsigned* __restrict__ bcount,
                                                  unsigned* __restrict__ boff, unsigned* __restrict__ total) {
  __shared__ unsigned part[256];
  const int t = threadIdx.x, per = (nblocks + 255) / 256;
  const int lo = t * per, hi = lo + per < nblocks ? lo + per : nblocks;
  unsigned s = 0u;
  for (int b = lo; b < hi; ++b) s += bcount[b];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    unsigned run = 0u;
    for (int k = 0; k < 256; ++k) {
      const unsigned v = part[k];
      part[k] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  unsigned run = part[t];
  for (int b = lo; b < hi; ++b) {
    boff[b] = run;
    run += bcount[b];
  }
}

// pass 2: regenerate, and write the passing candidates at their ranks (those
// below the target); the n-th passing candidate records the trial count
template <int NF>
__global__ __launch_bounds__(256) void k_gen_scatter(GenArgs a) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool ok = false;
  double p[NF][4], w = 0.0, rs = 0.0;
  if (c < a.m) {
    recipe_point<NF>(a.seed, a.stream, a.first + (uint64_t)c, a.rs_lo, a.rs_hi, a.mass, p, w, rs);
    ok = cut_pass<NF>(p, a.legs, a.cuts);
  }
  const int r = block_rank(ok, nullptr);
  if (r < 0) return;
  const int64_t rank = a.have + (int64_t)a.boff[blockIdx.x] + r;
  if (rank >= a.n) return;
  store_event<NF>(p, rs, a.mom, a.ld, rank);
  if (a.weight) a.weight[rank] = w;
  if (rank == a.n - 1) *a.trials = a.first + (uint64_t)c + 1 - a.first0;
}

// FKS radiation variables: xi_tilde and 1 - |y| log-uniform in [1e-6, 1],
// phi uniform in [0, 2 pi); a random sign of y for initial-state sectors
__global__ __launch_bounds__(256) void k_fks_variables(int64_t n, uint32_t seed, uint32_t stream, uint64_t first,
                                                       int initial_state, double* __restrict__ xit,
                                                       double* __restrict__ y, double* __restrict__ phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t e = first + (uint64_t)i;
  double a0, a1, b0, b1;
  uniform2(seed, stream, e, 65, a0, a1);
  uniform2(seed, stream, e, 66, b0, b1);
  xit[i] = pow(10.0, -6.0 * a0);
  const double yy = 1.0 - pow(10.0, -6.0 * a1);
  y[i] = (initial_state && !(b1 < 0.5)) ? -yy : yy;
  phi[i] = 2.0 * M_PI * b0;
}

// ---------------------------------------------------------------------------
// VEGAS adaptive Monte Carlo (Lepage's algorithm): every integration variable
// has its own grid of VEGAS_BINS bins on [0, 1); a uniform u selects bin
// b = floor(u NB) and the point x = edge_b + (u NB - b) (edge_{b+1} - edge_b),
// with weight NB (edge_{b+1} - edge_b).  After an iteration each bin's
// accumulated (f w)^2 sets the new edges: smoothed with its neighbours,
// compressed as ((1 - d/D) / ln(D/d))^alpha, and redistributed so that every
// new bin holds the same share.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_vegas_init(int D, double* __restrict__ edges, unsigned* zero) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *zero = 0u;
  if (i >= D * (VEGAS_BINS + 1)) return;
  edges[i] = (double)(i % (VEGAS_BINS + 1)) / VEGAS_BINS;
}

// the points of one iteration: D = 4 NF Born uniforms (RAMBO) + xi_tilde, y, phi
template <int NF>
__global__ __launch_bounds__(256) void k_vegas_points(VegasArgs a) {
  constexpr int D = 4 * NF + 3;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t e = a.first + (uint64_t)i;
  double x[D + 1];
  double wg = 1.0;
#pragma unroll
  for (int s = 0; s < (D + 1) / 2; ++s) {
    double v[2];
    uniform2(a.seed, a.stream, e, (uint32_t)s, v[0], v[1]);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int d = 2 * s + c;
      if (d >= D) break;
      const double t = v[c] * VEGAS_BINS;
      int b = (int)t;
      if (b > VEGAS_BINS - 1) b = VEGAS_BINS - 1;
      const double lo = a.edges[d * (VEGAS_BINS + 1) + b], wd = a.edges[d * (VEGAS_BINS + 1) + b + 1] - lo;
      x[d] = lo + (t - b) * wd;
      wg *= VEGAS_BINS * wd;
      a.bins[(int64_t)d * a.n + i] = (uint8_t)b;
    }
  }
  double u[NF][4];
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) u[k][m] = x[4 * k + m];
  double p[NF][4], wb;
  rambo_point<NF>(u, a.rs, a.mass, p, wb);
  store_event<NF>(p, a.rs, a.mom, a.n, i);
  a.xit[i] = x[4 * NF];
  a.y[i] = 2.0 * x[4 * NF + 1] - 1.0;
  a.phi[i] = 2.0 * M_PI * x[4 * NF + 2];
  a.w[i] = wb * wg * (2.0 * 2.0 * M_PI);   // dy = 2 du, dphi = 2 pi du
}

// f = scale * w * sum over sectors of dsig; a non-finite sum (an exactly
// singular point, measure zero) counts as zero and is counted
__global__ __launch_bounds__(256) void k_vegas_f(int64_t n, int nsec, const double* __restrict__ dsig,
                                                 const double* __restrict__ w, double scale, double* __restrict__ f,
                                                 unsigned* __restrict__ dropped) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nsec; ++k) s += dsig[(int64_t)k * n + i];
  double v = scale * w[i] * s;
  if (!isfinite(v)) {
    v = 0.0;
    atomicAdd(dropped, 1u);
  }
  f[i] = v;
}

// per-block sums of f^2 per (variable, bin), in a fixed order: block b takes a
// contiguous share of the points.  Thread t serves variable d = t / 16 and
// every 16th point of the share from t mod 16 on, adding each into its own
// column of an LDS histogram in point order; at the end the 16 columns of a
// variable are added in column order.  Rows are padded to 257 doubles so
// that the column sums, one bin per lane, fall into different banks.
constexpr int VEGAS_HIST_SUB = 256 / VEGAS_MAX_DIM;
__global__ __launch_bounds__(256) void k_vegas_hist_partial(int64_t n, int D, const double* __restrict__ f,
                                                            const uint8_t* __restrict__ bins,
                                                            double* __restrict__ part) {
  constexpr int ROW = 257;
  __shared__ double hist[VEGAS_BINS * ROW];
  const int t = threadIdx.x, d = t / VEGAS_HIST_SUB, sub = t % VEGAS_HIST_SUB;
  for (int b = 0; b < VEGAS_BINS; ++b) hist[b * ROW + t] = 0.0;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  if (d < D) {
    const uint8_t* bd = bins + (int64_t)d * n;
#pragma unroll 4
    for (int64_t j = lo + sub; j < hi; j += VEGAS_HIST_SUB) {
      const double fj = f[j];
      hist[bd[j] * ROW + t] += fj * fj;
    }
  }
  __syncthreads();
  const int pairs = D * VEGAS_BINS;
  for (int q = t; q < pairs; q += 256) {
    const int dq = q / VEGAS_BINS, b = q % VEGAS_BINS;
    double acc = 0.0;
    for (int c = 0; c < VEGAS_HIST_SUB; ++c) acc += hist[b * ROW + dq * VEGAS_HIST_SUB + c];
    part[(int64_t)blockIdx.x * pairs + q] = acc;
  }
}

// fold[s][q] = sum of part[b][q] over the VEGAS_HIST_BLOCKS / VEGAS_HIST_SEG
// blocks b of segment s, in block order within four interleaved chains
__global__ __launch_bounds__(256) void k_vegas_hist_fold(int pairs, const double* __restrict__ part,
                                                         double* __restrict__ fold) {
  constexpr int PER = VEGAS_HIST_BLOCKS / VEGAS_HIST_SEG;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= VEGAS_HIST_SEG * pairs) return;
  const int seg = i / pairs, q = i % pairs;
  const double* p = part + (int64_t)seg * PER * pairs + q;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < PER; ++k) a[k & 3] += p[(int64_t)k * pairs];
  fold[i] = (a[0] + a[1]) + (a[2] + a[3]);
}

// New grid of variable d = blockIdx.x from the folded histograms: lane b
// adds bin b over the segments (in order), smooths it with its neighbours
// and compresses it; lane 0 forms the running sums in bin order; lane k
// places new edge k.
__global__ __launch_bounds__(64) void k_vegas_refine(int D, double alpha, const double* __restrict__ fold,
                                                     double* __restrict__ edges) {
  constexpr int NB = VEGAS_BINS;
  __shared__ double h[NB], sm[NB], r[NB], cum[NB + 1], old[NB + 1], tot_s[2];
  const int d = blockIdx.x, b = threadIdx.x;
  const int pairs = D * NB;
  double* ed = edges + d * (NB + 1);
  if (b < NB) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < VEGAS_HIST_SEG; ++k) a[k & 3] += fold[(int64_t)k * pairs + d * NB + b];
    h[b] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  if (b <= NB) old[b] = ed[b];
  __syncthreads();
  // smoothing with the neighbours (two-point averages at the ends)
  if (b < NB) {
    sm[b] = b == 0 ? 0.5 * (h[0] + h[1])
                   : (b == NB - 1 ? 0.5 * (h[NB - 2] + h[NB - 1]) : (h[b - 1] + h[b] + h[b + 1]) / 3.0);
  }
  __syncthreads();
  if (b == 0) {
    double t = 0.0;
    for (int c = 0; c < NB; ++c) t += sm[c];
    tot_s[0] = t;
  }
  __syncthreads();
  const double tot = tot_s[0];
  if (!(tot > 0.0)) return;                  // nothing to adapt to: keep the grid
  if (b < NB) {
    const double a = sm[b] / tot;
    r[b] = a <= 0.0 ? 0.0 : (a >= 1.0 ? 1.0 : pow((1.0 - a) / (-log(a)), alpha));
  }
  __syncthreads();
  if (b == 0) {
    double c = 0.0;
    cum[0] = 0.0;
    for (int q = 0; q < NB; ++q) {
      c += r[q];
      cum[q + 1] = c;
    }
    tot_s[1] = c;
  }
  __syncthreads();
  const double rsum = tot_s[1];
  if (!(rsum > 0.0)) return;
  // edge k: the first old bin q (at most NB - 1) whose running sum reaches
  // k rsum / NB, entered by the fraction of its own r that is still missing
  if (b >= 1 && b < NB) {
    const double target = b * (rsum / NB);
    int q = 0;
    while (q < NB - 1 && cum[q + 1] < target) ++q;
    const double frac = r[q] > 0.0 ? (target - cum[q]) / r[q] : 0.0;
    ed[b] = old[q] + frac * (old[q + 1] - old[q]);
  }
  if (b == 0) ed[0] = 0.0;
  if (b == NB) ed[NB] = 1.0;
}

hipError_t launch_vegas_init(int D, double* edges, unsigned* zero, hipStream_t st) {
  hipLaunchKernelGGL(k_vegas_init, dim3((D * (VEGAS_BINS + 1) + 255) / 256), dim3(256), 0, st, D, edges, zero);
  return hipGetLastError();
}

hipError_t launch_vegas_points(int nfin, const VegasArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
  switch (nfin) {
    case 2: hipLaunchKernelGGL(k_vegas_points<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_vegas_points<3>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vegas_update(int64_t n, int D, int nsec, const double* dsig, const double* w, double scale,
                               double* f, unsigned* dropped, const uint8_t* bins, double* part, double* xs_part,
                               double* acc, bool refine, double alpha, double* edges, hipStream_t st) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_vegas_f, dim3((unsigned)grid), dim3(256), 0, st, n, nsec, dsig, w, scale, f, dropped);
  hipError_t e = launch_xs_sums(n, f, nullptr, 1.0, xs_part, acc, true, st);
  if (e != hipSuccess || !refine) return e;
  hipLaunchKernelGGL(k_vegas_hist_partial, dim3(VEGAS_HIST_BLOCKS), dim3(256), 0, st, n, D, (const double*)f, bins,
                     part);
  const int pairs = D * VEGAS_BINS;
  double* fold = part + (int64_t)VEGAS_HIST_BLOCKS * pairs;
  hipLaunchKernelGGL(k_vegas_hist_fold, dim3((VEGAS_HIST_SEG * pairs + 255) / 256), dim3(256), 0, st, pairs,
                     (const double*)part, fold);
  hipLaunchKernelGGL(k_vegas_refine, dim3(D), dim3(64), 0, st, D, alpha, (const double*)fold, edges);
  return hipGetLastError();
}

// Monte Carlo sums of f = scale * w * me2 over a chunk, in a fixed order:
// block b reduces its contiguous share into part[b] = (sum f, sum f^2); one
// block then adds the parts, in order, to acc.
constexpr int XS_BLOCKS = 512;

__global__ __launch_bounds__(256) void k_xs_partial(int64_t n, const double* __restrict__ w,
                                                    const double* __restrict__ me2, double scale,
                                                    double* __restrict__ part) {
  __shared__ double s1[256], s2[256];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  double a = 0.0, b = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double f = scale * w[i] * (me2 ? me2[i] : 1.0);
    a += f;
    b += f * f;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      s1[threadIdx.x] += s1[threadIdx.x + k];
      s2[threadIdx.x] += s2[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ __launch_bounds__(256) void k_xs_final(int nparts, const double* __restrict__ part, double* acc,
                                                  int reset) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      s1[threadIdx.x] += s1[threadIdx.x + k];
      s2[threadIdx.x] += s2[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] = (reset ? 0.0 : acc[0]) + s1[0];
    acc[1] = (reset ? 0.0 : acc[1]) + s2[0];
  }
}

hipError_t launch_xs_sums(int64_t n, const double* w, const double* me2, double scale, double* part, double* acc,
                          bool reset, hipStream_t st) {
  hipLaunchKernelGGL(k_xs_partial, dim3(XS_BLOCKS), dim3(256), 0, st, n, w, me2, scale, part);
  hipLaunchKernelGGL(k_xs_final, dim3(1), dim3(256), 0, st, XS_BLOCKS, (const double*)part, acc, reset ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_uniforms(int64_t n, uint32_t seed, uint32_t stream, uint64_t first, uint32_t slot, double* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_uniforms, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, seed, stream, first, slot,
                     out);
  return hipGetLastError();
}

hipError_t launch_rambo(int nfin, const PsArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
  switch (nfin) {
    case 2: hipLaunchKernelGGL(k_rambo<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_rambo<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_rambo<4>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cut_mask(int nfin, int64_t n, int64_t ld, int nin, const double* mom, const CutLegs& legs,
                           const nlo_cuts& cuts, uint8_t* pass, hipStream_t st) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (nfin) {
    case 2: hipLaunchKernelGGL(k_cut_mask<2>, grid, block, 0, st, n, ld, nin, mom, legs, cuts, pass); break;
    case 3: hipLaunchKernelGGL(k_cut_mask<3>, grid, block, 0, st, n, ld, nin, mom, legs, cuts, pass); break;
    case 4: hipLaunchKernelGGL(k_cut_mask<4>, grid, block, 0, st, n, ld, nin, mom, legs, cuts, pass); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_generate_chunk(int nfin, const GenArgs& a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.m + 255) / 256);
  const dim3 grid(nb), block(256);
  switch (nfin) {
    case 2: hipLaunchKernelGGL(k_gen_count<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_gen_count<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_gen_count<4>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_gen_scan, dim3(1), dim3(256), 0, st, (int)nb, (const unsigned*)a.bcount, a.boff, a.total);
  switch (nfin) {
    case 2: hipLaunchKernelGGL(k_gen_scatter<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_gen_scatter<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_gen_scatter<4>, grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_fks_variables(int64_t n, uint32_t seed, uint32_t stream, uint64_t first, int initial_state,
                                double* xit, double* y, double* phi, hipStream_t st) {
  hipLaunchKernelGGL(k_fks_variables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, seed, stream, first,
                     initial_state, xit, y, phi);
  return hipGetLastError();
}

}  // namespace nlo
