// Host-side basis construction (see basis.hip).
#pragma once
#include "common.h"

namespace aderdg {
void gauss_legendre01(int n, double *x, double *w);
bool build_basis(int n, DevBasis &B);
double lagrange_value(int n, const double *xi, int j, double x);
float round_prec(int p, double v);
}  // namespace aderdg
