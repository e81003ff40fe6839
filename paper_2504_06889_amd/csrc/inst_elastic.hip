// Kernel instances: linear elastic waves (eq. equations_of_motion, 2-D and 3-D).
#include "registry.h"

namespace aderdg {
static Instance<Elastic<2>, 2, 2> e2_2(1, false);
static Instance<Elastic<2>, 2, 3> e2_3(1, false);
static Instance<Elastic<2>, 2, 5> e2_5(1, true);
static Instance<Elastic<3>, 3, 1> e3_1(1, false);
static Instance<Elastic<3>, 3, 2> e3_2(1, true);
}  // namespace aderdg
