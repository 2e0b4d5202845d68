// Launchers of the on-device phase-space generator (phase_space.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

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

hipError_t launch_uniforms(int64_t n, uint32_t seed, uint32_t stream, uint64_t first, uint32_t slot, double* out,
                           hipStream_t st);
hipError_t launch_rambo(int nfin, const PsArgs& a, hipStream_t st);
hipError_t launch_fks_variables(int64_t n, uint32_t seed, uint32_t stream, uint64_t first, int initial_state,
                                double* xit, double* y, double* phi, hipStream_t st);

// fixed-order sums (sum f, sum f^2) of f = scale * w * me2 over n events,
// added to acc[0..1] (or replacing them when reset); part: 2 * 512 doubles
constexpr int64_t XS_PART_DOUBLES = 2 * 512;
hipError_t launch_xs_sums(int64_t n, const double* w, const double* me2, double scale, double* part, double* acc,
                          bool reset, hipStream_t st);

}  // namespace nlo
