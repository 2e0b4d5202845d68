// Per-event status of an |M|^2 batch (nlo_me2_checked).  The |M|^2 kernels
// are compiled without the IEEE NaN/infinity rules, so the tests here read
// the exponent bits instead of calling isfinite (this unit keeps full IEEE
// semantics anyway).
#include "checks.hpp"

namespace nlo {

__device__ __forceinline__ bool finite_bits(double x) {
  return ((unsigned long long)__double_as_longlong(x) & 0x7ff0000000000000ull) != 0x7ff0000000000000ull;
}

__global__ __launch_bounds__(256) void k_me2_status(int64_t n, int64_t ld, int npart, const double* __restrict__ mom,
                                                    const double* __restrict__ me2, uint8_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  uint8_t s = 0;
  const double v = me2[e];
  if (!finite_bits(v) || !(v >= 0.0)) s |= 1;
  for (int k = 0; k < 4 * npart; ++k)
    if (!finite_bits(mom[(int64_t)k * ld + e])) s |= 2;
  status[e] = s;
}

__global__ __launch_bounds__(256) void k_mark_list(int64_t n, const unsigned* __restrict__ cnt,
                                                   const unsigned* __restrict__ list, uint8_t bit,
                                                   uint8_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i >= (int64_t)cnt[0]) return;
  status[list[i]] |= bit;
}

hipError_t launch_me2_status(int64_t n, int64_t ld, int npart, const double* mom, const double* me2,
                             uint8_t* status, hipStream_t st) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_me2_status, dim3((unsigned)grid), dim3(256), 0, st, n, ld, npart, mom, me2, status);
  return hipGetLastError();
}

hipError_t launch_mark_list(int64_t n, const unsigned* cnt, const unsigned* list, uint8_t bit, uint8_t* status,
                            hipStream_t st) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_mark_list, dim3((unsigned)grid), dim3(256), 0, st, n, cnt, list, bit, status);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_scale(int64_t n, const double* __restrict__ in, double c,
                                               double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = c * in[e];
}

hipError_t launch_scale(int64_t n, const double* in, double c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, c, out);
  return hipGetLastError();
}

}  // namespace nlo
