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

// The three weights of a point on the nodes next to it along one axis,
// w[a] = phi(d + a - 1) with d = (nearest node) - (point) in (-1/2, 1/2],
// and (D) their derivatives dw[a] = phi'(d + a - 1).  All six share the
// square root q = sqrt(1 - 3 d^2): the middle node is on the inner piece,
// the outer two at |r| = 1 -+ d, where 1 - |r| = +-d, on the outer piece:
// phi(d - 1) = (2 + 3d - q)/6, phi(d) = (1 + q)/3, phi(d + 1) = (2 - 3d - q)/6,
// phi'(d - 1) = 1/2 + d/(2q), phi'(d) = -d/q, phi'(d + 1) = -1/2 + d/(2q).
template <bool D>
LBIB_HD void roma_weights3(double d, double w[3], double dw[3]) {
  const double q = sqrt(1.0 - 3.0 * d * d);
  w[0] = (2.0 + 3.0 * d - q) * (1.0 / 6.0);
  w[1] = (1.0 + q) * (1.0 / 3.0);
  w[2] = (2.0 - 3.0 * d - q) * (1.0 / 6.0);
  if (D) {
    const double h = d / q;
    dw[0] = 0.5 + 0.5 * h;
    dw[1] = -h;
    dw[2] = -0.5 + 0.5 * h;
  }
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
