// Launch descriptors shared by the C ABI and the per-process kernel units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "helas.hpp"

// largest block the kernels are compiled for (their __launch_bounds__)
#define NLO_MAX_BLOCK 256

namespace nlo {

// kernel variants of one process: FP64 vector ALU, FP32 vector ALU, FP32 with
// the colour contraction on the matrix cores, FP16 and BF16 amplitudes on
// packed pairs of events, and FP64 / FP32 with the alternative helicity
// schedule (the other lazy depth; processes without one repeat 0 and 1)
enum { VAR_F64 = 0, VAR_F32 = 1, VAR_MFMA = 2, VAR_F16 = 3, VAR_BF16 = 4, VAR_F64_ALT = 5, VAR_F32_ALT = 6,
       NVAR = 7 };

struct LaunchArgs {
  int64_t n, ld;
  const double* mom;
  double* out;
  double scale;   // average factor x coupling powers
  double mt;
  int block;
  hipStream_t stream;
  // optional device-side event range (bucketed FKS evaluation): which = -1
  // all of [0, n); 0: [0, cnt[0]); 1: [n - cnt[1], n)
  const unsigned* cnt = nullptr;
  int which = -1;
  // which = 2: the events listed in list[0, cnt[0]) (vector-ALU variants);
  // which = 3 (FP64 vector-ALU variant): [n - cnt[1], n), then the events
  // listed in list[0, cnt[4])
  const unsigned* list = nullptr;
  // FP16 / BF16 variants: workspace for the list of events evaluated again in
  // FP32 (fb_list: n entries, fb_cnt: one counter), and the FP32 launcher of
  // the same process that evaluates them
  unsigned* fb_list = nullptr;
  unsigned* fb_cnt = nullptr;
  hipError_t (*fb_launch)(const LaunchArgs&) = nullptr;
  // FKS real emission (FP32 / FP64 / MFMA variants): the legs of up to two
  // pairwise invariants and their exact per-event values ovv[2][ld] (or null)
  PairOv ovp{};
  const double* ovv = nullptr;
};

struct ProcStatic {
  const char* name;
  int npart, nin, nflow, nhel, ngood, ndiag, nterm, ncur, gs_pow, e_pow;
  double avg, ident;
  unsigned top_legs;   // bit k set: leg k is a top quark (mass m_t), else massless
  unsigned lep_legs;   // bit k set: leg k is a charged lepton
};

typedef hipError_t (*me2_launcher)(const LaunchArgs&);

}  // namespace nlo
