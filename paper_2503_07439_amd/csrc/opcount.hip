// Host-side operation count of the generated amplitude code: instantiates each
// process's per-helicity body and colour contraction with a scalar type that
// counts additions and multiplications (an FMA counts as two, a sign flip as
// none).  The code is straight-line, so the count is exact and independent of
// the event.  Prints one JSON object: per process, flops per helicity of the
// amplitude body and of the colour contraction, the number of helicities and
// the whole nested helicity sum per event, each both as written and with the
// operations on literal constants (0, +-1, constant-only) folded away.
#include <cstdio>
#include "generated/index.hpp"

namespace nlo {
// A value is either data (unknown at compile time) or a literal constant.
// Two counts are kept: every operation as written, and only those a compiler
// cannot fold away -- operations between constants, products with 0 or +-1
// and sums with 0 are free in the folded count.
struct Cnt {
  static long long add, mul, fadd, fmul;
  bool known = false;
  double v = 0.0;
  Cnt() = default;
  constexpr Cnt(double x) : known(true), v(x) {}
  explicit operator double() const { return v; }
  static Cnt data() { return Cnt(); }
};
long long Cnt::add = 0, Cnt::mul = 0, Cnt::fadd = 0, Cnt::fmul = 0;
inline Cnt operator+(Cnt a, Cnt b) {
  ++Cnt::add;
  if (a.known && b.known) return Cnt(a.v + b.v);
  if (a.known && a.v == 0.0) return b;
  if (b.known && b.v == 0.0) return a;
  ++Cnt::fadd;
  return {};
}
inline Cnt operator-(Cnt a) { return a.known ? Cnt(-a.v) : a; }
inline Cnt operator-(Cnt a, Cnt b) {
  ++Cnt::add;
  if (a.known && b.known) return Cnt(a.v - b.v);
  if (b.known && b.v == 0.0) return a;
  if (a.known && a.v == 0.0) return -b;
  ++Cnt::fadd;
  return {};
}
inline Cnt operator*(Cnt a, Cnt b) {
  ++Cnt::mul;
  if (a.known && b.known) return Cnt(a.v * b.v);
  if ((a.known && a.v == 0.0) || (b.known && b.v == 0.0)) return Cnt(0.0);
  if (a.known && (a.v == 1.0 || a.v == -1.0)) return a.v > 0 ? b : -b;
  if (b.known && (b.v == 1.0 || b.v == -1.0)) return b.v > 0 ? a : -a;
  ++Cnt::fmul;
  return {};
}
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
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

static void reset() { Cnt::add = Cnt::mul = Cnt::fadd = Cnt::fmul = 0; }
static long long written() { return Cnt::add + Cnt::mul; }
static long long folded() { return Cnt::fadd + Cnt::fmul; }

template <class P>
void count(const char* sep) {
  typename P::template Pre<Cnt> s{};          // event data: unknown values
  const Cnt mt = Cnt::data();
  cx<Cnt> J[P::NFLOW];
  reset();
  P::amplitudes(s, 0, mt, J);
  long long amp = written(), amp_f = folded();
  reset();
  (void)P::colour_sum(J);
  long long col = written(), col_f = folded();
  // the nested helicity schedule the kernels run: whole helicity sum per event
  reset();
  long long nbody = 0;
  P::helicity_sum(s, mt, [&](const cx<Cnt> (&Jn)[P::NFLOW]) { (void)P::colour_sum(Jn); ++nbody; });
  printf("%s\"%s\": {\"amp_flops_per_hel\": %lld, \"colour_flops_per_hel\": %lld, \"ngood\": %d, \"nflow\": %d, "
         "\"nested_flops_per_event\": %lld, \"nested_bodies\": %lld, \"amp_flops_per_hel_folded\": %lld, "
         "\"colour_flops_per_hel_folded\": %lld, \"nested_flops_per_event_folded\": %lld}",
         sep, P::NAME, amp, col, P::NGOOD, P::NFLOW, written(), nbody, amp_f, col_f, folded());
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
