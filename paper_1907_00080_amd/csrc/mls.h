// mls.h - moving-least-squares shape functions on the 3x3 stencil of a
// point (Sec. 2.2, Immersed Boundary Treatment: the reconstruction the paper
// uses to exchange data between the lattice and the Lagrangian chain;
// Sec. 2.3: nine nodes in a square of side 2.6 dx).
//
// Linear basis p = (1, x - X, y - Y) fitted by weighted least squares to the
// nodes (cx + a - 1, cy + b - 1), a, b = 0..2, c = floor(X + 1/2), with a
// tensor-product weight W_ab = w(x_a - X) w(y_b - Y) of support half-width
// h; rows beyond a wall carry no weight.  With the moment matrix
// A = sum W p p^T, gamma = A^{-1} e1 and the shape functions are
// phi_ab = W_ab gamma . p_ab.  Their derivatives with respect to the point
// follow the element-free Galerkin form (basis centre held fixed):
// gamma_X = A^{-1} (e2 - A_X gamma), dphi/dX = W gamma_X . p + W_X gamma . p.
//
// The weight is a tensor product, so every entry of A (and of A_X, A_Y) is a
// product of two one-axis moments S_k = sum_a w_a d_a^k: the 3x3 system is
// assembled from 6 + 6 sums instead of 9 outer products, and solved by its
// cofactors (A is symmetric positive definite).  A point with fewer than two
// stencil rows inside the support (only next to a wall) drops the y term of
// the basis: its third row and column of A become those of the identity.
#pragma once
#include "lbib_dev.h"

namespace lbib {

constexpr double kGaussAlpha = 0.4;   // Gaussian weight: exp(-(s / alpha)^2), s = |r| / h

// One-axis weight w(r) and dw/dr.  Roma: the kernel itself (support 3/2).
// Cubic spline (s = |r| / h): 2/3 - 4 s^2 + 4 s^3 for s <= 1/2,
// 4/3 (1 - s)^3 for 1/2 < s < 1.  Gaussian shifted to vanish at s = 1:
// (e^{-(s/a)^2} - e^{-1/a^2}) / (1 - e^{-1/a^2}).  Zero for s >= 1.
__device__ __forceinline__ double mls_weight(double r, int kind, double h, double& dw) {
  if (kind == LBIB_MLS_WEIGHT_ROMA) {
    dw = roma_dphi(r);
    return roma_phi(r);
  }
  const double s = fabs(r) / h;
  const double sg = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) / h;
  if (s >= 1.0) {
    dw = 0.0;
    return 0.0;
  }
  if (kind == LBIB_MLS_WEIGHT_CUBIC) {
    if (s <= 0.5) {
      dw = (-8.0 * s + 12.0 * s * s) * sg;
      return 2.0 / 3.0 - 4.0 * s * s + 4.0 * s * s * s;
    }
    const double t = 1.0 - s;
    dw = -4.0 * t * t * sg;
    return 4.0 / 3.0 * t * t * t;
  }
  const double e1 = exp(-1.0 / (kGaussAlpha * kGaussAlpha));
  const double g = exp(-(s / kGaussAlpha) * (s / kGaussAlpha));
  dw = -2.0 * s / (kGaussAlpha * kGaussAlpha) * g / (1.0 - e1) * sg;
  return (g - e1) / (1.0 - e1);
}

// The instance uses the MLS transfer (LBIB_TRANSFER_MLS).
__device__ __forceinline__ bool use_mls(const LatDev& L) { return L.transfer == LBIB_TRANSFER_MLS; }

// Shape functions ph[3 b + a] of the point (X, Y) and, when GRAD, their
// derivatives with respect to X (px) and Y (py).
template <bool GRAD>
__device__ __forceinline__ void mls_shape(const LatDev& L, double X, double Y, double ph[9],
                                          double px[9], double py[9]) {
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  const bool pery = L.periodic_y != 0;
  const int kind = L.mls_weight;
  const double h = L.mls_h;
  double dx[3], dy[3], wx[3], dwx[3], wy[3], dwy[3];
  // unrolled: the six weights are independent, and only kernels launched
  // for the MLS transfer hold this code
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dx[a] = (cxr + (a - 1)) - X;
    dy[a] = (cyr + (a - 1)) - Y;
    wx[a] = mls_weight(dx[a], kind, h, dwx[a]);
    wy[a] = mls_weight(dy[a], kind, h, dwy[a]);
  }
  int rows_in = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const double ry = cyr + (b - 1);
    const bool valid = pery || (ry >= 0.0 && ry < (double)L.ny);
    wy[b] = valid ? wy[b] : 0.0;
    dwy[b] = valid ? dwy[b] : 0.0;
    rows_in += (valid && fabs(dy[b]) / h < 1.0) ? 1 : 0;
  }
  const double ky = rows_in >= 2 ? 1.0 : 0.0;
#pragma unroll
  for (int b = 0; b < 3; ++b) dy[b] *= ky;      // the basis' y component
  double Sx0 = 0, Sx1 = 0, Sx2 = 0, Sy0 = 0, Sy1 = 0, Sy2 = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Sx0 += wx[a];
    Sx1 += wx[a] * dx[a];
    Sx2 += wx[a] * dx[a] * dx[a];
    Sy0 += wy[a];
    Sy1 += wy[a] * dy[a];
    Sy2 += wy[a] * dy[a] * dy[a];
  }
  const double a00 = Sx0 * Sy0, a01 = Sx1 * Sy0, a02 = Sx0 * Sy1;
  const double a11 = Sx2 * Sy0, a12 = Sx1 * Sy1, a22 = Sx0 * Sy2 + (1.0 - ky);
  // cofactors of the symmetric matrix; A^{-1} = C / det
  const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
  const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
  const double idet = 1.0 / (a00 * c00 + a01 * c01 + a02 * c02);
  const double g0 = c00 * idet, g1 = c01 * idet, g2 = c02 * idet;
  double gx0 = 0, gx1 = 0, gx2 = 0, gy0 = 0, gy1 = 0, gy2 = 0;
  if (GRAD) {
    double Tx0 = 0, Tx1 = 0, Tx2 = 0, Ty0 = 0, Ty1 = 0, Ty2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Tx0 += dwx[a];
      Tx1 += dwx[a] * dx[a];
      Tx2 += dwx[a] * dx[a] * dx[a];
      Ty0 += dwy[a];
      Ty1 += dwy[a] * dy[a];
      Ty2 += dwy[a] * dy[a] * dy[a];
    }
    // A_X = -(T^x S^y products), A_Y = -(S^x T^y products); r = e - A_. gamma
    const double rx0 = (Tx0 * Sy0) * g0 + (Tx1 * Sy0) * g1 + (Tx0 * Sy1) * g2;
    const double rx1 = 1.0 + (Tx1 * Sy0) * g0 + (Tx2 * Sy0) * g1 + (Tx1 * Sy1) * g2;
    const double rx2 = (Tx0 * Sy1) * g0 + (Tx1 * Sy1) * g1 + (Tx0 * Sy2) * g2;
    const double ry0 = (Sx0 * Ty0) * g0 + (Sx1 * Ty0) * g1 + (Sx0 * Ty1) * g2;
    const double ry1 = (Sx1 * Ty0) * g0 + (Sx2 * Ty0) * g1 + (Sx1 * Ty1) * g2;
    const double ry2 = ky + (Sx0 * Ty1) * g0 + (Sx1 * Ty1) * g1 + (Sx0 * Ty2) * g2;
    gx0 = (c00 * rx0 + c01 * rx1 + c02 * rx2) * idet;
    gx1 = (c01 * rx0 + c11 * rx1 + c12 * rx2) * idet;
    gx2 = (c02 * rx0 + c12 * rx1 + c22 * rx2) * idet;
    gy0 = (c00 * ry0 + c01 * ry1 + c02 * ry2) * idet;
    gy1 = (c01 * ry0 + c11 * ry1 + c12 * ry2) * idet;
    gy2 = (c02 * ry0 + c12 * ry1 + c22 * ry2) * idet;
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double W = wx[a] * wy[b];
      const double gp = g0 + g1 * dx[a] + g2 * dy[b];
      ph[3 * b + a] = W * gp;
      if (GRAD) {
        px[3 * b + a] = W * (gx0 + gx1 * dx[a] + gx2 * dy[b]) - dwx[a] * wy[b] * gp;
        py[3 * b + a] = W * (gy0 + gy1 * dx[a] + gy2 * dy[b]) - wx[a] * dwy[b] * gp;
      }
    }
  }
}

}  // namespace lbib
