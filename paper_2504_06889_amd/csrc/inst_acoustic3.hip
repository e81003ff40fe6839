// Kernel instances: linear acoustics in 3-D.
#include "registry.h"

namespace aderdg {
static Instance<Acoustic<3>, 3, 1> a3_1(0, false);
static Instance<Acoustic<3>, 3, 2> a3_2(0, true);
static Instance<Acoustic<3>, 3, 3> a3_3(0, false);
static Instance<Acoustic<3>, 3, 5> a3_5(0, true);
}  // namespace aderdg
