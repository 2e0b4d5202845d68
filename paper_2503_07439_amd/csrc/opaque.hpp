// An optimisation barrier for one register value: the compiler must assume
// the value changed at this point, although no instruction is emitted.  The
// generated helicity sums use it to keep a computation inside the loop it
// was written in (loop-invariant code motion would otherwise hoist it).
#pragma once
#include <type_traits>
#include "helas.hpp"

namespace nlo {
template <class T> NLO_HD void opaque(T& x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#else
  (void)x;
#endif
}
// a copy of a value behind the barrier
template <class T> NLO_HD T oval(T x) {
  opaque(x);
  return x;
}
// a copy of a momentum behind the barrier (every component)
template <class T> NLO_HD r4<T> oq(const r4<T>& q) {
  r4<T> r = q;
#pragma unroll
  for (int m = 0; m < 4; ++m) opaque(r.v[m]);
  return r;
}
// momentum of a leg set from its slot: in FP64 summed from the external
// momenta in slots L... (each read through the barrier, summed left to right),
// in other types the stored slot through the barrier
template <class T, int... L> NLO_HD r4<T> qlegs(const r4<T>* Q, int slot) {
  if constexpr (std::is_same<T, double>::value) {
    r4<T> r;
#pragma unroll
    for (int m = 0; m < 4; ++m) r.v[m] = (... + oval(Q[L].v[m]));
    return r;
  } else {
    return oq(Q[slot]);
  }
}
// a copy of a wavefunction behind the barrier (every component)
template <class T> NLO_HD w4<T> ow(const w4<T>& w) {
  w4<T> r = w;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    opaque(r.c[m].r);
    opaque(r.c[m].i);
  }
  return r;
}
}  // namespace nlo
