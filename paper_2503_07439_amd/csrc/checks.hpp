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

// Class queues of the buffered FKS evaluation (nlo_fks_buffer): event e of a
// push (its inputs at e of arrays with leading dimension ld) joins the real
// queue (class 0) if its R cut passes and the counterterm queue (class 1) if
// any of its S and C cuts passes; positions from one atomic per class and
// block on cnt[0..1]; each queue holds the Born momenta [nb*4][cap], the
// radiation variables, the output slot and its mask bytes [4][cap] (the
// class's own terms only)
struct FksQueue {
  double* born;
  double *xit, *y, *phi;
  unsigned* slot;
  uint8_t* mask;
};
hipError_t launch_queue_push(int64_t n, int64_t ld, int nb, const double* born, const double* xit, const double* y,
                             const double* phi, const uint8_t* mask, const unsigned* slot, FksQueue q0, FksQueue q1,
                             int64_t cap, unsigned* cnt, hipStream_t st);
// out[slot[k]] += w[k] for k < m
hipError_t launch_queue_scatter(int64_t m, const unsigned* slot, const double* w, double* out, hipStream_t st);
// cnt[c] = 0
hipError_t launch_queue_reset(unsigned* cnt, int c, hipStream_t st);

// out[e] = c * in[e] for e < n
hipError_t launch_scale(int64_t n, const double* in, double c, double* out, hipStream_t st);

}  // namespace nlo
