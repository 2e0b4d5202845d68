// Per-event status of an |M|^2 batch (nlo_me2_checked) and small elementwise
// steps: launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nlo {

// status[e] = bit0 if me2[e] is not a finite non-negative number, bit1 if a
// momentum component of event e is not finite
hipError_t launch_me2_status(int64_t n, int64_t ld, int npart, const double* mom, const double* me2,
                             uint8_t* status, hipStream_t st);

// status[list[i]] |= bit for i < *cnt (a device-side event list of at most n)
hipError_t launch_mark_list(int64_t n, const unsigned* cnt, const unsigned* list, uint8_t bit, uint8_t* status,
                            hipStream_t st);

// out[e] = c * in[e] for e < n
hipError_t launch_scale(int64_t n, const double* in, double c, double* out, hipStream_t st);

}  // namespace nlo
