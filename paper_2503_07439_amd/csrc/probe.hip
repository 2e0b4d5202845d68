// Attainable vector-ALU FMA throughput of the device: a measurement aid for
// the benchmark's roofline (the published peaks assume the peak engine
// clock), not part of the library's interface.  Each thread runs eight
// independent FMA chains; the result is written so that the chains are kept.
#include <hip/hip_runtime.h>

namespace {

template <class T>
__global__ __launch_bounds__(256) void k_fma_chains(int iters, T b, T c, T* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  T a0 = T(g & 1023) * T(1e-3), a1 = a0 + T(1), a2 = a0 + T(2), a3 = a0 + T(3);
  T a4 = a0 + T(4), a5 = a0 + T(5), a6 = a0 + T(6), a7 = a0 + T(7);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
    a0 = a0 * b + c;
    a1 = a1 * b + c;
    a2 = a2 * b + c;
    a3 = a3 * b + c;
    a4 = a4 * b + c;
    a5 = a5 * b + c;
    a6 = a6 * b + c;
    a7 = a7 * b + c;
  }
  out[g] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

}  // namespace

// blocks x 256 threads, iters iterations of 8 FMAs (16 flops) per thread;
// out holds blocks x 256 values of the precision (0 = FP32, 1 = FP64).
// Returns the HIP launch status.
extern "C" int nlo_probe_fma(int precision, int blocks, int iters, void* out, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (blocks <= 0 || iters <= 0 || !out) return (int)hipErrorInvalidValue;
  if (precision == 0)
    hipLaunchKernelGGL(k_fma_chains<float>, dim3(blocks), dim3(256), 0, s, iters, 1.0000001f, 1e-7f, (float*)out);
  else
    hipLaunchKernelGGL(k_fma_chains<double>, dim3(blocks), dim3(256), 0, s, iters, 1.0000000001, 1e-12, (double*)out);
  return (int)hipGetLastError();
}
