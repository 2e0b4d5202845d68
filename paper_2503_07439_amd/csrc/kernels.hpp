// Kernel templates shared by the per-process translation units.
//
// One event per lane.  Per event: coalesced load of the structure-of-arrays
// FP64 momenta, a helicity-independent FP64 prologue (external-state data,
// internal momenta, propagator denominators), then a loop over the
// structurally non-zero helicities -- nested per leg, so that every
// Feynman-diagram sub-current is evaluated once per helicity assignment of
// its own legs and reused by the inner loops -- accumulates the colour-flow
// vector J, contracts
// J^dagger C J with the constant colour matrix and adds the result to an FP64
// per-event sum.  The colour contraction runs either on the vector ALU
// (Cholesky form |L^T Re J|^2 + |L^T Im J|^2) or on the matrix cores: each
// wave stages its 64 J vectors in LDS and multiplies the [128 x nc] block
// (real and imaginary rows) by L with v_mfma_f32_16x16x4f32.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "helas.hpp"
#include "launch.hpp"

namespace nlo {
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <class P>
__device__ __forceinline__ void load_event(const double* __restrict__ mom, int64_t ld, int64_t e,
                                           double (&p)[P::NPART][4]) {
#pragma unroll
  for (int k = 0; k < P::NPART; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) p[k][m] = mom[(k * 4 + m) * ld + e];
}

// ---------------------------------------------------------------------------
// vector-ALU kernel: any arithmetic type T
// ---------------------------------------------------------------------------
// event range of a launch: all of [0, n), or one bucket of a bucketed batch
__device__ __forceinline__ void event_range(int64_t n, const unsigned* cnt, int which, int64_t& lo, int64_t& hi) {
  lo = 0;
  hi = n;
  if (which == 0) hi = cnt[0];
  else if (which == 1) lo = n - (int64_t)cnt[1];
}

template <class P, class T>
__global__ __launch_bounds__(NLO_MAX_BLOCK) void k_me2_valu(int64_t n, int64_t ld, const double* __restrict__ mom,
                                                  double* __restrict__ out, double scale, double mt,
                                                  const unsigned* cnt, int which) {
  int64_t lo, hi;
  event_range(n, cnt, which, lo, hi);
  const int64_t e = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= hi) return;
  double p[P::NPART][4];
  load_event<P>(mom, ld, e, p);
  typename P::template Pre<T> s;
  P::prologue(p, s, mt);
  double acc = 0.0;
  P::helicity_sum(s, T(mt), [&](const cx<T> (&J)[P::NFLOW]) { acc += (double)P::colour_sum(J); });
  out[e] = acc * scale;
}

// ---------------------------------------------------------------------------
// matrix-core kernel: float amplitudes, colour contraction on MFMA
// ---------------------------------------------------------------------------
template <class P>
struct MfmaShape {
  static constexpr int NF = P::NFLOW;
  static constexpr int KP = (NF + 3) / 4 * 4;   // contraction length padded to the MFMA K=4
  static constexpr int KS = KP / 4;             // K steps
  static constexpr int NT = (NF + 15) / 16;     // 16-wide output tiles
  static constexpr int STR = KP + 1;            // LDS row stride (odd: spreads banks)
  static constexpr int WAVE_FLOATS = 128 * STR; // 64 real rows + 64 imaginary rows
};

template <class P>
__global__ __launch_bounds__(NLO_MAX_BLOCK) void k_me2_mfma(int64_t n, int64_t ld, const double* __restrict__ mom,
                                                  double* __restrict__ out, double scale, double mt,
                                                  const unsigned* cnt, int which) {
  using S = MfmaShape<P>;
  extern __shared__ float smem[];
  int64_t lo, hi;
  event_range(n, cnt, which, lo, hi);
  const int64_t b0 = lo + (int64_t)blockIdx.x * blockDim.x;
  if (b0 >= hi) return;   // block-uniform: the barriers below see every wave
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float* buf = smem + wave * S::WAVE_FLOATS;
  const int64_t e = b0 + threadIdx.x;
  // every lane of a wave takes part in the MFMA; lanes past the end reuse the
  // last event and do not store
  const int64_t ec = e < hi ? e : hi - 1;
  double p[P::NPART][4];
  load_event<P>(mom, ld, ec, p);
  typename P::template Pre<float> s;
  P::prologue(p, s, mt);

  // B fragments: B[k][c] = L[k][c] = LT[c][k]; lane supplies k = 4 ks + lane/16, c = 16 nt + lane%16
  float bfrag[S::KS][S::NT];
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < S::NT; ++nt) {
      const int k = 4 * ks + (lane >> 4), c = 16 * nt + (lane & 15);
      bfrag[ks][nt] = (k < S::NF && c < S::NF) ? P::LT[c][k] : 0.0f;
    }
  // zero the padding columns once
#pragma unroll
  for (int j = S::NF; j < S::KP; ++j) {
    buf[lane * S::STR + j] = 0.0f;
    buf[(64 + lane) * S::STR + j] = 0.0f;
  }
  float acc[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[t][r] = 0.0f;

  P::helicity_sum(s, float(mt), [&](const cx<float> (&J)[P::NFLOW]) {
    __syncthreads();   // the previous helicity's fragment reads are complete
#pragma unroll
    for (int j = 0; j < S::NF; ++j) {
      buf[lane * S::STR + j] = J[j].r;
      buf[(64 + lane) * S::STR + j] = J[j].i;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      floatx4 d[S::NT];
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt) d[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < S::KS; ++ks) {
        // A[i][k]: lane supplies row i = lane%16 of tile t, column k = 4 ks + lane/16
        const float a = buf[(16 * t + (lane & 15)) * S::STR + 4 * ks + (lane >> 4)];
#pragma unroll
        for (int nt = 0; nt < S::NT; ++nt) d[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bfrag[ks][nt], d[nt], 0, 0, 0);
      }
      // D[i][c]: lane holds rows i = 4 (lane/16) + r, column c = lane%16
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] += d[nt][r] * d[nt][r];
    }
  });
  // sum the squares over the 16 columns held by lanes with equal lane/16
  double rs[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = acc[t][r];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      rs[t][r] = v;
    }
  __syncthreads();
  double* rows = reinterpret_cast<double*>(buf);   // 128 doubles fit in the wave's staging area
  if ((lane & 15) == 0) {
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) rows[16 * t + 4 * (lane >> 4) + r] = rs[t][r];
  }
  __syncthreads();
  if (e < hi) out[e] = (rows[lane] + rows[64 + lane]) * scale;
}

template <class P>
constexpr size_t mfma_smem_bytes(int block) {
  return (size_t)(block / 64) * MfmaShape<P>::WAVE_FLOATS * sizeof(float);
}

// launch one variant; returns the HIP launch status
template <class P, int VARIANT>
hipError_t launch_me2(const LaunchArgs& a) {
  const int64_t grid = (a.n + a.block - 1) / a.block;
  if constexpr (VARIANT == VAR_F64) {
    hipLaunchKernelGGL((k_me2_valu<P, double>), dim3((unsigned)grid), dim3(a.block), 0, a.stream, a.n, a.ld, a.mom,
                       a.out, a.scale, a.mt, a.cnt, a.which);
  } else if constexpr (VARIANT == VAR_F32) {
    hipLaunchKernelGGL((k_me2_valu<P, float>), dim3((unsigned)grid), dim3(a.block), 0, a.stream, a.n, a.ld, a.mom,
                       a.out, a.scale, a.mt, a.cnt, a.which);
  } else {
    hipLaunchKernelGGL((k_me2_mfma<P>), dim3((unsigned)grid), dim3(a.block), mfma_smem_bytes<P>(a.block), a.stream,
                       a.n, a.ld, a.mom, a.out, a.scale, a.mt, a.cnt, a.which);
  }
  return hipGetLastError();
}

}  // namespace nlo
