// Host build of the generated per-process amplitude code: the nested
// helicity schedule and colour sum that the GPU kernels run, evaluated per
// event on the CPU in double or float.  Used by test_host_generated_me2.py to
// compare the generator's output with the oracle without a GPU.
//
//   host_me2 <process> <n> <prec 0=double 1=float> <npart> <mom.bin> <out.bin> <alpha_s> <alpha> <m_top>
//
// mom.bin: [npart][4][n] doubles (SoA); out.bin: n doubles, |M|^2 with the
// initial-state average and the couplings applied.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "helas.hpp"
#include "generated/ee_mumu.hpp"
#include "generated/ee_uu.hpp"
#include "generated/ee_uug.hpp"
#include "generated/gg_tt.hpp"
#include "generated/uu_tt.hpp"
#include "generated/gg_ttg.hpp"
#include "generated/uu_ttg.hpp"
#include "generated/ug_ttu.hpp"
#include "generated/gg_ttgg.hpp"

using namespace nlo;

template <class P, class T>
static void run(int n, const double* mom, double* out, double mt, double gs2, double e2) {
  const double scale = P::AVG * std::pow(gs2, P::GS_POW) * std::pow(e2, P::E_POW);
  for (int e = 0; e < n; ++e) {
    double p[P::NPART][4];
    for (int k = 0; k < P::NPART; ++k)
      for (int m = 0; m < 4; ++m) p[k][m] = mom[(k * 4 + m) * (size_t)n + e];
    typename P::template Pre<T> s;
    P::prologue(p, s, mt);
    double acc = 0.0;
    P::helicity_sum(s, T(mt), [&](const cx<T> (&J)[P::NFLOW]) { acc += (double)P::colour_sum(J); });
    out[e] = acc * P::HEL_SYM * scale;
  }
}

template <class P>
static bool dispatch(const char* name, int n, int prec, const double* mom, double* out, double mt, double gs2,
                     double e2) {
  if (std::strcmp(name, P::NAME) != 0) return false;
  if (prec == 0)
    run<P, double>(n, mom, out, mt, gs2, e2);
  else
    run<P, float>(n, mom, out, mt, gs2, e2);
  return true;
}

int main(int argc, char** argv) {
  if (argc != 10) {
    std::fprintf(stderr, "usage: host_me2 proc n prec npart mom.bin out.bin alpha_s alpha m_top\n");
    return 2;
  }
  const char* name = argv[1];
  const int n = std::atoi(argv[2]), prec = std::atoi(argv[3]), npart = std::atoi(argv[4]);
  const double gs2 = 4.0 * M_PI * std::atof(argv[7]), e2 = 4.0 * M_PI * std::atof(argv[8]), mt = std::atof(argv[9]);
  std::vector<double> mom((size_t)npart * 4 * n), out(n);
  FILE* f = std::fopen(argv[5], "rb");
  if (!f || std::fread(mom.data(), sizeof(double), mom.size(), f) != mom.size()) return 3;
  std::fclose(f);
  const bool ok = dispatch<ee_mumu>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<ee_uu>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<ee_uug>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<gg_tt>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<uu_tt>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<gg_ttg>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<uu_ttg>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<ug_ttu>(name, n, prec, mom.data(), out.data(), mt, gs2, e2) ||
                  dispatch<gg_ttgg>(name, n, prec, mom.data(), out.data(), mt, gs2, e2);
  if (!ok) return 4;
  f = std::fopen(argv[6], "wb");
  if (!f || std::fwrite(out.data(), sizeof(double), n, f) != (size_t)n) return 5;
  std::fclose(f);
  return 0;
}
