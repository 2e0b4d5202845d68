// An optimisation barrier for one register value: the compiler must assume
// the value changed at this point, although no instruction is emitted.  The
// generated helicity sums use it to keep a computation inside the loop it
// was written in (loop-invariant code motion would otherwise hoist it).
#pragma once
#include "helas.hpp"

namespace nlo {
template <class T> NLO_HD void opaque(T& x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#else
  (void)x;
#endif
}
}  // namespace nlo
