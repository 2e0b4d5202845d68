// Host-side operation count of the generated amplitude code: instantiates each
// process's per-helicity body and colour contraction with a scalar type that
// counts additions and multiplications (an FMA counts as two, a sign flip as
// none).  The code is straight-line, so the count is exact and independent of
// the event.  Prints one JSON object: per process, flops per helicity of the
// amplitude body and of the colour contraction, and the number of helicities.
#include <cstdio>
#include "generated/index.hpp"

namespace nlo {
struct Cnt {
  static long long add, mul;
  Cnt() = default;
  constexpr Cnt(double) {}
  explicit operator double() const { return 0.0; }
};
long long Cnt::add = 0, Cnt::mul = 0;
inline Cnt operator+(Cnt, Cnt) { ++Cnt::add; return {}; }
inline Cnt operator-(Cnt, Cnt) { ++Cnt::add; return {}; }
inline Cnt operator*(Cnt, Cnt) { ++Cnt::mul; return {}; }
inline Cnt operator-(Cnt) { return {}; }
inline Cnt& operator+=(Cnt& a, Cnt) { ++Cnt::add; return a; }
}  // namespace nlo
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

template <class P>
void count(const char* sep) {
  typename P::template Pre<Cnt> s{};
  cx<Cnt> J[P::NFLOW];
  Cnt::add = Cnt::mul = 0;
  P::amplitudes(s, 0, Cnt(0), J);
  long long amp = Cnt::add + Cnt::mul;
  Cnt::add = Cnt::mul = 0;
  (void)P::colour_sum(J);
  long long col = Cnt::add + Cnt::mul;
  // the nested helicity schedule the kernels run: whole helicity sum per event
  Cnt::add = Cnt::mul = 0;
  long long nbody = 0;
  P::helicity_sum(s, Cnt(0), [&](const cx<Cnt> (&Jn)[P::NFLOW]) { (void)P::colour_sum(Jn); ++nbody; });
  long long nested = Cnt::add + Cnt::mul;
  printf("%s\"%s\": {\"amp_flops_per_hel\": %lld, \"colour_flops_per_hel\": %lld, \"ngood\": %d, \"nflow\": %d, "
         "\"nested_flops_per_event\": %lld, \"nested_bodies\": %lld}",
         sep, P::NAME, amp, col, P::NGOOD, P::NFLOW, nested, nbody);
}

int main() {
  printf("{");
  count<ee_mumu>("");
  count<ee_uu>(", ");
  count<ee_uug>(", ");
  count<gg_tt>(", ");
  count<uu_tt>(", ");
  count<gg_ttg>(", ");
  count<uu_ttg>(", ");
  count<ug_ttu>(", ");
  count<gg_ttgg>(", ");
  printf("}\n");
  return 0;
}
