// Kernel instances: shallow water with bathymetry (eq. swe_canonical).
#include "registry.h"

namespace aderdg {
static Instance<Swe, 2, 1> s2_1(3, false);
static Instance<Swe, 2, 2> s2_2(3, false);
static Instance<Swe, 2, 3> s2_3(3, true);
static Instance<Swe, 2, 4> s2_4(3, false);
static Instance<Swe, 2, 5> s2_5(3, true);
static Instance<Swe, 2, 6> s2_6(3, true);
}  // namespace aderdg
