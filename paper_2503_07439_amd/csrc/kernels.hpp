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
#include <type_traits>
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
// (which = 0: [0, cnt[0]), 1: [n - cnt[1], n)); which = 2 (vector-ALU
// kernels only) takes the events listed in list[0, cnt[0]) instead, and
// which = 3 (FP64 vector-ALU kernel) [n - cnt[1], n) followed by the events
// listed in list[0, cnt[4])
__device__ __forceinline__ void event_range(int64_t n, const unsigned* cnt, int which, int64_t& lo, int64_t& hi) {
  lo = 0;
  hi = n;
  if (which == 0) hi = cnt[0];
  else if (which == 1) lo = n - (int64_t)cnt[1];
}

// pair invariants of an FKS real emission: ovp carries the leg pairs, ovv
// the per-event values ([2][ld], same event index as the momenta) or null
__device__ __forceinline__ PairOv pair_ov(const PairOv& ovp, const double* __restrict__ ovv, int64_t ld, int64_t e) {
  PairOv ov = ovp;
  if (ovv) {
    ov.v0 = ovv[e];
    ov.v1 = ovv[ld + e];
  } else {
    ov.a0 = -1;
  }
  return ov;
}

template <class P, class T, int SCHED = 0>
__global__ __launch_bounds__(NLO_MAX_BLOCK)
__attribute__((amdgpu_waves_per_eu(std::is_same<T, float>::value && SCHED == 0 ? P::WAVES_F32 : 1)))
void k_me2_valu(int64_t n, int64_t ld, const double* __restrict__ mom,
                                                  double* __restrict__ out, double scale, double mt,
                                                  const unsigned* cnt, int which, const unsigned* list,
                                                  PairOv ovp, const double* __restrict__ ovv) {
  int64_t e;
  if (which == 2) {               // the events listed in list[0, cnt[0])
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)cnt[0]) return;
    e = list[i];
  } else if (std::is_same<T, double>::value && which == 3) {
    // the FP64 bucket [n - cnt[1], n), then the events listed in list[0, cnt[4])
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c1 = cnt[1];
    if (i < c1) {
      e = n - c1 + i;
    } else {
      if (i - c1 >= (int64_t)cnt[4]) return;
      e = list[i - c1];
    }
  } else {
    int64_t lo, hi;
    event_range(n, cnt, which, lo, hi);
    e = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= hi) return;
  }
  double p[P::NPART][4];
  load_event<P>(mom, ld, e, p);
  typename P::template Pre<T> s;
  P::prologue(p, s, mt, pair_ov(ovp, ovv, ld, e));
  double acc = 0.0;
  P::template helicity_sum_sched<SCHED>(s, T(mt), [&](const cx<T> (&J)[P::NFLOW]) {
    acc += (double)P::colour_sum(J);
  });
  out[e] = acc * (P::HEL_SYM * scale);   // the sum covers one of each pair (h, -h)
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
__global__ __launch_bounds__(NLO_MAX_BLOCK) __attribute__((amdgpu_waves_per_eu(P::WAVES_F32)))
void k_me2_mfma(int64_t n, int64_t ld, const double* __restrict__ mom,
                                                  double* __restrict__ out, double scale, double mt,
                                                  const unsigned* cnt, int which, PairOv ovp,
                                                  const double* __restrict__ ovv) {
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
  P::prologue(p, s, mt, pair_ov(ovp, ovv, ld, ec));

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
  if (e < hi) out[e] = (rows[lane] + rows[64 + lane]) * (P::HEL_SYM * scale);
}

// ---------------------------------------------------------------------------
// half-width kernels: FP16 or BF16 amplitudes, two events per lane
// ---------------------------------------------------------------------------
// The amplitude arithmetic runs on packed pairs (one event in each half of a
// 32-bit register), so one instruction serves two events.  Momenta and the top
// mass are divided by sqrt(s_hat) in FP64 first, making every input
// dimensionless and O(1): |M|^2 of N external particles has mass dimension
// 2(4 - N), so |M|^2(p) = s_hat^(4 - N) |M|^2(p / sqrt(s_hat)), and that factor
// is applied in FP64 at the end.  J is widened to FP32 and the colour
// contraction and helicity sum accumulate in FP32 / FP64.

// Largest propagator denominator handled in half width, in units of 1/s_hat.
// Beyond it an event is close to a soft or collinear pole, where Feynman-gauge
// diagrams cancel against each other by orders of magnitude: an 11-bit (FP16)
// or 8-bit (BF16) significand leaves no correct digit there.  Such events are
// listed and evaluated again in FP32 by a second launch.
constexpr int HALF_MAX_DEN_LOG2 = 14;

// loads one event, divides momenta and mass by sqrt(s_hat) and runs the FP64
// prologue on them; then scales the external wavefunctions down by 2^-b with
// b from the largest propagator denominator: intermediate currents grow
// roughly like the largest 1/(p^2 - m^2) on their tree, and this keeps them
// below the FP16 maximum while the rest stay well above its smallest normal
// number.  Returns 1 / sqrt(s_hat); f receives the FP64 factor that restores
// |M|^2, s_hat^(4 - N) 2^(2b); safe is false when the event needs FP32.
template <class P>
__device__ __forceinline__ double scaled_prologue(const double* __restrict__ mom, int64_t ld, int64_t e, double mt,
                                                  typename P::template Pre<float>& s, double& f, bool& safe) {
  double p[P::NPART][4];
  load_event<P>(mom, ld, e, p);
  double q[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) q[m] = p[0][m] + p[1][m];
  const double r = 1.0 / sqrt(q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3]);
#pragma unroll
  for (int k = 0; k < P::NPART; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) p[k][m] *= r;
  P::prologue(p, s, mt * r);
  float dmax = 1.0f;
#pragma unroll
  for (int k = 0; k < P::NDEN; ++k) dmax = fmaxf(dmax, fabsf(s.den[k]));
  int ex;
  (void)frexpf(dmax, &ex);            // dmax < 2^ex (ex = 0 for an infinite dmax)
  safe = dmax <= 3.0e38f && ex <= HALF_MAX_DEN_LOG2;   // an infinite denominator is not safe
  const int b = safe ? ex + 4 : 0;    // 16x headroom below the largest denominator
  P::scale_legs(s, b);
  f = ldexp(1.0, 2 * b);
#pragma unroll
  for (int k = 4; k < P::NPART; ++k) f *= r * r;   // s_hat^(4 - N)
  return r;
}

template <class P, class V2>
__global__ __launch_bounds__(NLO_MAX_BLOCK) __attribute__((amdgpu_waves_per_eu(P::WAVES_F32)))
void k_me2_pair(int64_t n, int64_t ld, const double* __restrict__ mom,
                                                  double* __restrict__ out, double scale, double mt,
                                                  const unsigned* cnt, int which, unsigned* fb_list,
                                                  unsigned* fb_cnt) {
  using Pf = typename P::template Pre<float>;
  using Pv = typename P::template Pre<V2>;
  static_assert(sizeof(V2) == sizeof(float) && sizeof(Pf) == sizeof(Pv), "pre-computed data must be all scalars");
  constexpr int NW = sizeof(Pf) / sizeof(float);
  int64_t lo, hi;
  event_range(n, cnt, which, lo, hi);
  // a block covers 2 * blockDim events: lanes take e and e + blockDim (both coalesced)
  const int64_t e0 = lo + (int64_t)blockIdx.x * 2 * blockDim.x + threadIdx.x;
  if (e0 >= hi) return;
  const int64_t e1 = e0 + blockDim.x;
  const bool has1 = e1 < hi;
  Pf a, b;
  double f[2], r[2];
  bool safe0, safe1;
  r[0] = scaled_prologue<P>(mom, ld, e0, mt, a, f[0], safe0);
  r[1] = scaled_prologue<P>(mom, ld, has1 ? e1 : e0, mt, b, f[1], safe1);
  {
    // append the events that need FP32 to the fallback list (wave-aggregated)
    const bool l0 = !safe0, l1 = has1 && !safe1;
    const unsigned long long m0 = __ballot(l0), m1 = __ballot(l1);
    if (m0 | m1) {
      const int lane = threadIdx.x & 63;
      const unsigned long long lower = lane ? (~0ull >> (64 - lane)) : 0ull;
      unsigned base = 0;
      if (lane == 0) base = atomicAdd(fb_cnt, (unsigned)(__popcll(m0) + __popcll(m1)));
      base = __shfl(base, 0);
      if (l0) fb_list[base + __popcll(m0 & lower)] = (unsigned)e0;
      if (l1) fb_list[base + __popcll(m0) + __popcll(m1 & lower)] = (unsigned)e1;
    }
  }
  // pack: one rounding from FP32 per element, both events in one instruction
  Pv s;
  const float* af = reinterpret_cast<const float*>(&a);
  const float* bf = reinterpret_cast<const float*>(&b);
  V2* sv = reinterpret_cast<V2*>(&s);
#pragma unroll
  for (int k = 0; k < NW; ++k) {   // element by element (a packed f32x2 conversion
    V2 t;                           // trips the compiler's instruction selection
    t[0] = af[k];                   // when NaNs and signed zeros are not honoured)
    t[1] = bf[k];
    sv[k] = t;
  }
  const V2 mtv = __builtin_convertvector(f32x2{float(mt * r[0]), float(mt * r[1])}, V2);
  double acc0 = 0.0, acc1 = 0.0;
  P::helicity_sum(s, mtv, [&](const cx<V2> (&J)[P::NFLOW]) {
    cx<float> J0[P::NFLOW], J1[P::NFLOW];
#pragma unroll
    for (int j = 0; j < P::NFLOW; ++j) {
      J0[j] = cx<float>{(float)J[j].r[0], (float)J[j].i[0]};
      J1[j] = cx<float>{(float)J[j].r[1], (float)J[j].i[1]};
    }
    acc0 += (double)P::colour_sum(J0);
    acc1 += (double)P::colour_sum(J1);
  });
  out[e0] = acc0 * f[0] * (P::HEL_SYM * scale);
  if (has1) out[e1] = acc1 * f[1] * (P::HEL_SYM * scale);
}

template <class P>
constexpr size_t mfma_smem_bytes(int block) {
  return (size_t)(block / 64) * MfmaShape<P>::WAVE_FLOATS * sizeof(float);
}

static __global__ void k_fb_zero(unsigned* c) {
  if (threadIdx.x == 0) *c = 0u;
}

// launch one variant; returns the HIP launch status
template <class P, int VARIANT>
hipError_t launch_me2(const LaunchArgs& a) {
  const int64_t grid = (a.n + a.block - 1) / a.block;
  if constexpr (VARIANT == VAR_F64 || VARIANT == VAR_F64_ALT) {
    constexpr int SCHED = VARIANT == VAR_F64_ALT ? 1 : 0;
    hipLaunchKernelGGL((k_me2_valu<P, double, SCHED>), dim3((unsigned)grid), dim3(a.block), 0, a.stream, a.n, a.ld,
                       a.mom, a.out, a.scale, a.mt, a.cnt, a.which, a.list, a.ovp, a.ovv);
  } else if constexpr (VARIANT == VAR_F32 || VARIANT == VAR_F32_ALT) {
    constexpr int SCHED = VARIANT == VAR_F32_ALT ? 1 : 0;
    hipLaunchKernelGGL((k_me2_valu<P, float, SCHED>), dim3((unsigned)grid), dim3(a.block), 0, a.stream, a.n, a.ld,
                       a.mom, a.out, a.scale, a.mt, a.cnt, a.which, a.list, a.ovp, a.ovv);
  } else if constexpr (VARIANT == VAR_F16 || VARIANT == VAR_BF16) {
    // half-width pass over all events, then FP32 over the listed ones
    using V2 = typename std::conditional<VARIANT == VAR_F16, f16x2, bf16x2>::type;
    const int64_t grid2 = (a.n + 2 * a.block - 1) / (2 * a.block);
    hipLaunchKernelGGL(k_fb_zero, dim3(1), dim3(64), 0, a.stream, a.fb_cnt);
    hipLaunchKernelGGL((k_me2_pair<P, V2>), dim3((unsigned)grid2), dim3(a.block), 0, a.stream, a.n, a.ld, a.mom,
                       a.out, a.scale, a.mt, a.cnt, a.which, a.fb_list, a.fb_cnt);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    // the FP32 kernel lives in the process's FP32 unit (one instantiation per
    // kernel across the library)
    if (!a.fb_launch) return hipErrorInvalidValue;
    LaunchArgs f = a;
    f.cnt = a.fb_cnt;
    f.which = 2;
    f.list = a.fb_list;
    return a.fb_launch(f);
  } else {
    hipLaunchKernelGGL((k_me2_mfma<P>), dim3((unsigned)grid), dim3(a.block), mfma_smem_bytes<P>(a.block), a.stream,
                       a.n, a.ld, a.mom, a.out, a.scale, a.mt, a.cnt, a.which, a.ovp, a.ovv);
  }
  return hipGetLastError();
}

}  // namespace nlo
