// Kernel instances: compressible Euler equations (2-D and 3-D).
#include "registry.h"

namespace aderdg {
static Instance<Euler<2>, 2, 0> u2_0(2, false);
static Instance<Euler<2>, 2, 2> u2_2(2, false);
static Instance<Euler<2>, 2, 3> u2_3(2, true);
static Instance<Euler<2>, 2, 5> u2_5(2, true);
static Instance<Euler<3>, 3, 1> u3_1(2, false);
static Instance<Euler<3>, 3, 2> u3_2(2, true);
static Instance<Euler<3>, 3, 4> u3_4(2, true);
}  // namespace aderdg
