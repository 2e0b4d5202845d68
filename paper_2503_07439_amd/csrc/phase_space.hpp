// Launchers of the on-device phase-space generator (phase_space.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "cuts.hpp"

namespace nlo {

struct PsArgs {
  int64_t n, ld;
  uint32_t seed, stream;
  uint64_t first;            // index of the batch's first event
  double rs_lo, rs_hi;       // sqrt(s_hat) uniform in [rs_lo, rs_hi] (equal: fixed)
  double mass[8];            // final-state masses
  double* mom;               // [nfin + 2][4][ld]
  double* weight;            // [n] RAMBO weight, or null
};

// Algorithm 2's regenerate-until-pass loop, one chunk of m candidates:
// candidates first .. first + m - 1 of the batch recipe; the passing ones get
// ranks have, have + 1, ... in candidate order, and those below n are written
// to mom/weight at their rank; the candidate of rank n - 1 writes
// *trials = its counter + 1 - first0; *total = this chunk's passing count
constexpr int64_t GEN_CHUNK = (int64_t)1 << 20;
struct GenArgs {
  int64_t n, ld, m, have;
  uint32_t seed, stream;
  uint64_t first, first0;
  double rs_lo, rs_hi;
  double mass[8];
  CutLegs legs;
  nlo_cuts cuts;
  unsigned *bcount, *boff, *total;   // [m / 256], [m / 256], [1]
  uint64_t* trials;
  double *mom, *weight;
};

hipError_t launch_uniforms(int64_t n, uint32_t seed, uint32_t stream, uint64_t first, uint32_t slot, double* out,
                           hipStream_t st);
hipError_t launch_cut_mask(int nfin, int64_t n, int64_t ld, int nin, const double* mom, const CutLegs& legs,
                           const nlo_cuts& cuts, uint8_t* pass, hipStream_t st);
hipError_t launch_generate_chunk(int nfin, const GenArgs& a, hipStream_t st);
hipError_t launch_rambo(int nfin, const PsArgs& a, hipStream_t st);
hipError_t launch_fks_variables(int64_t n, uint32_t seed, uint32_t stream, uint64_t first, int initial_state,
                                double* xit, double* y, double* phi, hipStream_t st);

// VEGAS adaptive integration over the Born RAMBO uniforms and xi_tilde, y, phi
constexpr int VEGAS_BINS = 50;
constexpr int VEGAS_MAX_DIM = 16;       // 4 per Born final-state particle (at most 3) + 3
constexpr int VEGAS_HIST_BLOCKS = 1024;  // blocks of the histogram pass
constexpr int VEGAS_HIST_SEG = 32;       // their partial sums folded in 32 segments

struct VegasArgs {
  int64_t n;
  uint32_t seed, stream;
  uint64_t first;            // counter of the iteration's first point
  double rs;                 // Born sqrt(s_hat)
  double mass[8];            // Born final-state masses
  const double* edges;       // [D][VEGAS_BINS + 1]
  double* mom;               // Born momenta [NF + 2][4][n]
  double *w, *xit, *y, *phi; // [n]: RAMBO weight x grid weight x 4 pi, radiation variables
  uint8_t* bins;             // [D][n]
};

// uniform grids, and *zero = 0
hipError_t launch_vegas_init(int D, double* edges, unsigned* zero, hipStream_t st);
hipError_t launch_vegas_points(int nfin, const VegasArgs& a, hipStream_t st);
// f = scale w sum_s dsig[s]; (sum f, sum f^2) into acc; with refine, the
// per-bin sums of f^2 (part: (VEGAS_HIST_BLOCKS + VEGAS_HIST_SEG) x D x
// VEGAS_BINS doubles) and the new grid
hipError_t launch_vegas_update(int64_t n, int D, int nsec, const double* dsig, const double* w, double scale,
                               double* f, unsigned* dropped, const uint8_t* bins, double* part, double* xs_part,
                               double* acc, bool refine, double alpha, double* edges, hipStream_t st);

// fixed-order sums (sum f, sum f^2) of f = scale * w * me2 over n events,
// added to acc[0..1] (or replacing them when reset); part: 2 * 512 doubles;
// me2 may be null (then f = scale * w)
constexpr int64_t XS_PART_DOUBLES = 2 * 512;
hipError_t launch_xs_sums(int64_t n, const double* w, const double* me2, double scale, double* part, double* acc,
                          bool reset, hipStream_t st);

}  // namespace nlo
