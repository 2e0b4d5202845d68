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

__global__ __launch_bounds__(256) void k_queue_push(int64_t n, int64_t ld, int nb, const double* __restrict__ born,
                                                    const double* __restrict__ xit, const double* __restrict__ y,
                                                    const double* __restrict__ phi, const uint8_t* __restrict__ mask,
                                                    const unsigned* __restrict__ slot, FksQueue q0, FksQueue q1,
                                                    int64_t cap, unsigned* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = e < n;
  bool r = false, c = false;
  uint8_t mS = 1, mC = 1;
  if (act) {
    r = !mask || mask[1 * ld + e];
    if (mask) {
      mS = mask[2 * ld + e];
      mC = mask[3 * ld + e];
    }
    c = mS || ((mC & 2) ? (mC & 12) != 0 : mC != 0);
  }
  // positions: wave ballots, one atomic per class and block
  __shared__ unsigned wc[4][2], wb[4][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long br = __ballot(r), bc = __ballot(c);
  if (lane == 0) {
    wc[wave][0] = (unsigned)__popcll(br);
    wc[wave][1] = (unsigned)__popcll(bc);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int k = threadIdx.x, nw = (int)(blockDim.x + 63) >> 6;
    unsigned tot = 0u;
    for (int w = 0; w < nw; ++w) tot += wc[w][k];
    unsigned base = tot ? atomicAdd(&cnt[k], tot) : 0u;
    for (int w = 0; w < nw; ++w) {
      wb[w][k] = base;
      base += wc[w][k];
    }
  }
  __syncthreads();
  if (!act) return;
  const unsigned long long lower = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int k = 0; k < 2; ++k) {
    const bool in = k == 0 ? r : c;
    if (!in) continue;
    const FksQueue& q = k == 0 ? q0 : q1;
    const int64_t pos = (int64_t)wb[wave][k] + __popcll((k == 0 ? br : bc) & lower);
    for (int m = 0; m < nb * 4; ++m) q.born[m * cap + pos] = born[m * ld + e];
    q.xit[pos] = xit[e];
    q.y[pos] = y[e];
    q.phi[pos] = phi[e];
    q.slot[pos] = slot[e];
    q.mask[0 * cap + pos] = 0;
    q.mask[1 * cap + pos] = k == 0 ? 1 : 0;
    q.mask[2 * cap + pos] = k == 0 ? 0 : mS;
    q.mask[3 * cap + pos] = k == 0 ? 2 : mC;   // class 0: both collinear ends fail
  }
}

__global__ __launch_bounds__(256) void k_queue_scatter(int64_t m, const unsigned* __restrict__ slot,
                                                       const double* __restrict__ w, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) out[slot[k]] += w[k];
}

__global__ void k_queue_reset(unsigned* cnt, int c) {
  if (threadIdx.x == 0) cnt[c] = 0u;
}

hipError_t launch_queue_push(int64_t n, int64_t ld, int nb, const double* born, const double* xit, const double* y,
                             const double* phi, const uint8_t* mask, const unsigned* slot, FksQueue q0, FksQueue q1,
                             int64_t cap, unsigned* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_queue_push, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ld, nb, born, xit, y,
                     phi, mask, slot, q0, q1, cap, cnt);
  return hipGetLastError();
}

hipError_t launch_queue_scatter(int64_t m, const unsigned* slot, const double* w, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_queue_scatter, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, slot, w, out);
  return hipGetLastError();
}

hipError_t launch_queue_reset(unsigned* cnt, int c, hipStream_t st) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, cnt, c);
  return hipGetLastError();
}

}  // namespace nlo
