// Kernel instances: 3-D elastic waves at order 3 and 5.
#include "registry.h"

namespace aderdg {
static Instance<Elastic<3>, 3, 3> e3_3(1, false);
static Instance<Elastic<3>, 3, 5> e3_5(1, true);
}  // namespace aderdg
