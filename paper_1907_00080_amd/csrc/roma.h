// roma.h - the 3-point kernel of Roma, Peskin & Berger (J. Comput. Phys. 1999),
// used as the IB delta function on the 3 nearest nodes per axis (Sec. 2.2),
// and its first two derivatives.  Plain C++ so host code can use it too.
#pragma once
#include <math.h>

#if defined(__HIPCC__)
#define LBIB_HD __host__ __device__ inline
#else
#define LBIB_HD inline
#endif

namespace lbib {

// One square root, of the argument of whichever piece applies (the same
// values as evaluating the pieces separately, without a divergent branch).
LBIB_HD double roma_phi(double r) {
  const double a = fabs(r);
  const bool inner = a <= 0.5;
  const double b = 1.0 - a;
  const double s = 1.0 - 3.0 * b * b;
  const double q = sqrt(inner ? 1.0 - 3.0 * a * a : (s > 0.0 ? s : 0.0));
  if (inner) return (1.0 + q) * (1.0 / 3.0);
  if (a <= 1.5) return (5.0 - 3.0 * a - q) * (1.0 / 6.0);
  return 0.0;
}

LBIB_HD double roma_dphi(double r) {
  double a = fabs(r);
  if (a <= 0.5) return -r / sqrt(1.0 - 3.0 * r * r);
  if (a < 1.5) {
    double b = 1.0 - a;
    double v = -0.5 - b / (2.0 * sqrt(1.0 - 3.0 * b * b));
    return r > 0 ? v : -v;
  }
  return 0.0;
}

// Second derivative: -(1 - 3 r^2)^(-3/2) on the inner piece and
// (1 - 3 (1 - |r|)^2)^(-3/2) / 2 on the outer one; phi is C1, so this jumps
// at |r| = 1/2 and 3/2.
LBIB_HD double roma_ddphi(double r) {
  double a = fabs(r);
  if (a <= 0.5) {
    double s = 1.0 - 3.0 * r * r;
    return -1.0 / (s * sqrt(s));
  }
  if (a < 1.5) {
    double b = 1.0 - a;
    double s = 1.0 - 3.0 * b * b;
    return 0.5 / (s * sqrt(s));
  }
  return 0.0;
}

}  // namespace lbib
