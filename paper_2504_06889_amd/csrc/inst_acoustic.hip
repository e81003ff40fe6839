// Kernel instances: linear acoustics (eq. acoustic and its 3-D extension).
#include "registry.h"

namespace aderdg {
static Instance<Acoustic<2>, 2, 0> a2_0(0, false);
static Instance<Acoustic<2>, 2, 1> a2_1(0, false);
static Instance<Acoustic<2>, 2, 2> a2_2(0, false);
static Instance<Acoustic<2>, 2, 3> a2_3(0, true);
static Instance<Acoustic<2>, 2, 4> a2_4(0, false);
static Instance<Acoustic<2>, 2, 5> a2_5(0, true);
}  // namespace aderdg
