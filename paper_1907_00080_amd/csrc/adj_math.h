// adj_math.h - local reverse-mode derivatives (vector-Jacobian products) of
// the pieces of one LB-IB time step, float64.  Each *_vjp function takes the
// forward inputs and the adjoint of the forward outputs, and returns the
// adjoint of the inputs, for the exact arithmetic of the forward formula
// written next to it.  Plain C++ (host and device).
//
// Pieces (paper sections):
//   collide     forced BGK collision with Guo's source and half-force
//               velocity (Sec. 2.1, Eqs. BGK, feq, ForcingTerm)
//   star        pre-forcing moments rho*, u* of the streamed populations
//   strain      element spring force (Eq. strainFor)
//   bend        bending forces at one vertex (Eq. bendFor)
//   area        area-penalty element load (Eq. areaFor)
//   spring      adhesion spring element load (Eq. adhFor)
//   hydro       probe pressure and viscous element load (Eqs. hydroForP,
//               hydroForNu)
//   rigid       summed load and torque, BDF2 velocity update and rigid
//               vertex motion (Eqs. linearVelRig, angularVelRig)
#pragma once
#include <math.h>

#include "roma.h"

namespace lbib {
namespace adj {

LBIB_HD int qex(int i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); }
LBIB_HD int qey(int i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); }
LBIB_HD double qw(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

// ------------------------------------------------------------------ collide
// h: pulled populations shifted by the rest weights (h = f - w); F: Eulerian
// force; omega = 1/tau, pre = 1 - 1/(2 tau).  Outputs h* and u.
LBIB_HD void collide_fwd(const double h[9], double Fx, double Fy, double omega, double pre,
                         double hs[9], double& ux, double& uy) {
  double drho = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; ++i) {
    drho += h[i];
    jx += qex(i) * h[i];
    jy += qey(i) * h[i];
  }
  const double rho = 1.0 + drho;
  ux = (jx + 0.5 * Fx) / rho;
  uy = (jy + 0.5 * Fy) / rho;
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    const double ex = qex(i), ey = qey(i), w = qw(i);
    const double eu = ex * ux + ey * uy;
    const double heq = w * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    const double src = pre * w * ((3.0 * (ex - ux) + 9.0 * eu * ex) * Fx + (3.0 * (ey - uy) + 9.0 * eu * ey) * Fy);
    hs[i] = h[i] + omega * (heq - h[i]) + src;
  }
}

// a: adjoint of h*; (uhx, uhy): adjoint of u.  Returns the adjoint of h in
// hh and of F in (Fhx, Fhy).
LBIB_HD void collide_vjp(const double h[9], double Fx, double Fy, double omega, double pre,
                         const double a[9], double uhx, double uhy, double hh[9], double& Fhx,
                         double& Fhy) {
  double drho = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; ++i) {
    drho += h[i];
    jx += qex(i) * h[i];
    jy += qey(i) * h[i];
  }
  const double rho = 1.0 + drho;
  const double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
  const double uu = ux * ux + uy * uy;
  double dr = 0.0, rh = 0.0, uxh = uhx, uyh = uhy, fxh = 0.0, fyh = 0.0;
  for (int i = 0; i < 9; ++i) {
    const double ex = qex(i), ey = qey(i), w = qw(i), ai = a[i];
    const double eu = ex * ux + ey * uy;
    const double Q = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
    const double ow = omega * ai * w;
    dr += ow;                                        // heq: w drho
    rh += ow * Q;                                    // heq: w rho Q(u)
    uxh += ow * rho * (3.0 * ex + 9.0 * eu * ex - 3.0 * ux);
    uyh += ow * rho * (3.0 * ey + 9.0 * eu * ey - 3.0 * uy);
    const double pw = ai * pre * w;
    const double eF = ex * Fx + ey * Fy;
    uxh += pw * (-3.0 * Fx + 9.0 * eF * ex);         // source: d/du
    uyh += pw * (-3.0 * Fy + 9.0 * eF * ey);
    fxh += pw * (3.0 * (ex - ux) + 9.0 * eu * ex);   // source: d/dF
    fyh += pw * (3.0 * (ey - uy) + 9.0 * eu * ey);
  }
  // u = (j + F/2) / rho
  const double jxh = uxh / rho, jyh = uyh / rho;
  fxh += 0.5 * uxh / rho;
  fyh += 0.5 * uyh / rho;
  rh -= (uxh * ux + uyh * uy) / rho;
  dr += rh;                                          // rho = 1 + drho
  for (int i = 0; i < 9; ++i) hh[i] = (1.0 - omega) * a[i] + dr + qex(i) * jxh + qey(i) * jyh;
  Fhx = fxh;
  Fhy = fyh;
}

// ------------------------------------------------------------------ star
// rho* = 1 + sum h, u* = (sum h e + g/2) / rho*: adjoint of h from the
// adjoints of rho*, u* (added to hh).
LBIB_HD void star_vjp(double rho, double ux, double uy, double rh, double uxh, double uyh,
                      double hh[9]) {
  const double jxh = uxh / rho, jyh = uyh / rho;
  const double r = rh - (uxh * ux + uyh * uy) / rho;
  for (int i = 0; i < 9; ++i) hh[i] += r + qex(i) * jxh + qey(i) * jyh;
}

// ------------------------------------------------------------------ geometry
// t = d / |d|, len = |d|: adjoint of d from those of t and len (added).
LBIB_HD void unit_vjp(double dx, double dy, double thx, double thy, double lenh, double& dhx,
                      double& dhy) {
  const double len = sqrt(dx * dx + dy * dy);
  const double tx = dx / len, ty = dy / len;
  const double tt = thx * tx + thy * ty;
  dhx += (thx - tt * tx) / len + lenh * tx;
  dhy += (thy - tt * ty) / len + lenh * ty;
}

// ------------------------------------------------------------------ strain
// Element d = x_{l+1} - x_l: s = ks (len - l0) t is added to vertex l and
// subtracted from vertex l+1.
LBIB_HD void strain_fwd(double dx, double dy, double l0, double ks, double& sx, double& sy) {
  const double len = sqrt(dx * dx + dy * dy);
  const double c = ks * (len - l0) / len;
  sx = c * dx;
  sy = c * dy;
}

// shx, shy: adjoint of s (= F^_l - F^_{l+1}).  Adds to dh and ksh.
LBIB_HD void strain_vjp(double dx, double dy, double l0, double ks, double shx, double shy,
                        double& dhx, double& dhy, double& ksh) {
  const double len = sqrt(dx * dx + dy * dy);
  const double c = 1.0 - l0 / len;
  const double ds = dx * shx + dy * shy;
  const double k3 = l0 / (len * len * len);
  dhx += ks * (c * shx + k3 * ds * dx);
  dhy += ks * (c * shy + k3 * ds * dy);
  ksh += c * ds;
}

// ------------------------------------------------------------------ bend
// Vertex u with left element dL = x_u - x_{u-1} and right element
// dR = x_{u+1} - x_u: signed turning angle th = atan2(tL x tR, tL . tR),
// n = normalize(nL + nR) with n = (t_y, -t_x), a = kb (th - th0);
// F_{u-1} += a lR/(lL+lR) n, F_u -= a n, F_{u+1} += a lL/(lL+lR) n (Eq. bendFor,
// lever rule: each neighbour's share is the far edge's length, so the three
// forces exert no net moment).
LBIB_HD void bend_fwd(double dLx, double dLy, double dRx, double dRy, double th0, double kb,
                      double Fm[2], double Fu[2], double Fp[2]) {
  const double lL = sqrt(dLx * dLx + dLy * dLy), lR = sqrt(dRx * dRx + dRy * dRy);
  const double tLx = dLx / lL, tLy = dLy / lL, tRx = dRx / lR, tRy = dRy / lR;
  const double th = atan2(tLx * tRy - tLy * tRx, tLx * tRx + tLy * tRy);
  const double nsx = tLy + tRy, nsy = -tLx - tRx;
  const double nn = sqrt(nsx * nsx + nsy * nsy);
  const double nx = nsx / nn, ny = nsy / nn;
  const double a = kb * (th - th0);
  const double wL = lR / (lL + lR), wR = lL / (lL + lR);
  Fm[0] = a * wL * nx; Fm[1] = a * wL * ny;
  Fu[0] = -a * nx;     Fu[1] = -a * ny;
  Fp[0] = a * wR * nx; Fp[1] = a * wR * ny;
}

// Given the adjoints of the three vertex forces: adds the adjoints of dL, dR
// and kb.
LBIB_HD void bend_vjp(double dLx, double dLy, double dRx, double dRy, double th0, double kb,
                      const double Fhm[2], const double Fhu[2], const double Fhp[2], double dLh[2],
                      double dRh[2], double& kbh) {
  const double lL = sqrt(dLx * dLx + dLy * dLy), lR = sqrt(dRx * dRx + dRy * dRy);
  const double tLx = dLx / lL, tLy = dLy / lL, tRx = dRx / lR, tRy = dRy / lR;
  const double cr = tLx * tRy - tLy * tRx, dt = tLx * tRx + tLy * tRy;
  const double th = atan2(cr, dt);
  const double nsx = tLy + tRy, nsy = -tLx - tRx;
  const double nn = sqrt(nsx * nsx + nsy * nsy);
  const double nx = nsx / nn, ny = nsy / nn;
  const double a = kb * (th - th0);
  const double S = lL + lR, wL = lR / S, wR = lL / S;
  const double Gx = wL * Fhm[0] - Fhu[0] + wR * Fhp[0];
  const double Gy = wL * Fhm[1] - Fhu[1] + wR * Fhp[1];
  const double ah = nx * Gx + ny * Gy;
  const double nhx = a * Gx, nhy = a * Gy;
  const double wLh = a * (nx * Fhm[0] + ny * Fhm[1]);
  const double wRh = a * (nx * Fhp[0] + ny * Fhp[1]);
  kbh += (th - th0) * ah;
  const double thh = kb * ah;
  const double r2 = cr * cr + dt * dt;
  const double crh = thh * dt / r2, dth = -thh * cr / r2;
  double tLhx = crh * tRy + dth * tRx, tLhy = -crh * tRx + dth * tRy;
  double tRhx = -crh * tLy + dth * tLx, tRhy = crh * tLx + dth * tLy;
  // n = ns / |ns|, ns = (tLy + tRy, -tLx - tRx)
  const double nd = nhx * nx + nhy * ny;
  const double nshx = (nhx - nd * nx) / nn, nshy = (nhy - nd * ny) / nn;
  tLhx -= nshy; tLhy += nshx;
  tRhx -= nshy; tRhy += nshx;
  const double S2 = S * S;
  // wL = lR / S, wR = lL / S
  const double lLh = -wLh * (lR / S2) + wRh * (lR / S2);
  const double lRh = wLh * (lL / S2) - wRh * (lL / S2);
  unit_vjp(dLx, dLy, tLhx, tLhy, lLh, dLh[0], dLh[1]);
  unit_vjp(dRx, dRy, tRhx, tRhy, lRh, dRh[0], dRh[1]);
}

// ------------------------------------------------------------------ area
// Element load F = kappa (d_y, -d_x) = kappa len n, kappa = ka p_ref (1 - A/A0);
// shared half and half by the element's vertices.  Given its adjoint Fh:
// adds the adjoint of d and returns the element's share of kappa^.
LBIB_HD double area_vjp(double dx, double dy, double kappa, double Fhx, double Fhy, double& dhx,
                        double& dhy) {
  dhx += -kappa * Fhy;
  dhy += kappa * Fhx;
  return Fhx * dy - Fhy * dx;
}

// ------------------------------------------------------------------ spring
// Element load F = sigma (y - y_eq) n, n = (t_y, -t_x), y the bond length
// from the centroid c to the receptor, with (ddx, ddy) = d y / d c.
// Adds the adjoints of d (element vector), c and sigma.
LBIB_HD void spring_fwd(double dx, double dy, double y, double sigma, double y_eq, double& Fx,
                        double& Fy) {
  const double len = sqrt(dx * dx + dy * dy);
  const double k = sigma * (y - y_eq);
  Fx = k * (dy / len);
  Fy = k * (-dx / len);
}

LBIB_HD void spring_vjp(double dx, double dy, double y, double ddx, double ddy, double sigma,
                        double y_eq, double Fhx, double Fhy, double& dhx, double& dhy,
                        double& chx, double& chy, double& sigh) {
  const double len = sqrt(dx * dx + dy * dy);
  const double nx = dy / len, ny = -dx / len;
  const double nF = nx * Fhx + ny * Fhy;
  sigh += (y - y_eq) * nF;
  const double yh = sigma * nF;
  chx += yh * ddx;
  chy += yh * ddy;
  const double k = sigma * (y - y_eq);
  const double nhx = k * Fhx, nhy = k * Fhy;
  unit_vjp(dx, dy, -nhy, nhx, 0.0, dhx, dhy);
}

// ------------------------------------------------------------------ hydro
// Element load from the probe state: pressure pr = (rho - 1)/3, velocity
// gradient g = (du/dx, du/dy, dv/dx, dv/dy), tau = nu (g + g^T):
//   F = (-pr n + tau n) len.
LBIB_HD void hydro_fwd(double pr, const double g[4], double nu, double nx, double ny, double len,
                       double& Fx, double& Fy) {
  const double txx = 2.0 * nu * g[0], tyy = 2.0 * nu * g[3], txy = nu * (g[1] + g[2]);
  Fx = (-pr * nx + txx * nx + txy * ny) * len;
  Fy = (-pr * ny + txy * nx + tyy * ny) * len;
}

// Adjoints of pr, g, n and len (added) from that of F.
LBIB_HD void hydro_vjp(double pr, const double g[4], double nu, double nx, double ny, double len,
                       double Fhx, double Fhy, double& prh, double gh[4], double& nhx, double& nhy,
                       double& lenh) {
  const double txx = 2.0 * nu * g[0], tyy = 2.0 * nu * g[3], txy = nu * (g[1] + g[2]);
  lenh += Fhx * (-pr * nx + txx * nx + txy * ny) + Fhy * (-pr * ny + txy * nx + tyy * ny);
  prh += -len * (Fhx * nx + Fhy * ny);
  const double txxh = len * Fhx * nx, tyyh = len * Fhy * ny, txyh = len * (Fhx * ny + Fhy * nx);
  nhx += len * (Fhx * (-pr + txx) + Fhy * txy);
  nhy += len * (Fhx * txy + Fhy * (-pr + tyy));
  gh[0] += 2.0 * nu * txxh;
  gh[3] += 2.0 * nu * tyyh;
  gh[1] += nu * txyh;
  gh[2] += nu * txyh;
}

// ------------------------------------------------------------------ rigid
// Rigid particle (Sec. 2.3, Eqs. linearVelRig, angularVelRig).  Its summed
// load and torque, element by element: F_tot += f, M_tot += r x f with the
// arm r = c - x_c from the reference point to the element centroid.  Given
// the adjoints (Fh, Mh) of the sums: adds the adjoints of f and of r.
LBIB_HD void rigid_load_vjp(double rx, double ry, double fx, double fy, double Fhx, double Fhy,
                            double Mh, double& fhx, double& fhy, double& rhx, double& rhy) {
  fhx += Fhx - Mh * ry;
  fhy += Fhy + Mh * rx;
  rhx += Mh * fy;
  rhy += -Mh * fx;
}

// Velocity update v' = 2/3 (2 v - v_prev / 2 + r / m), or v' = v + r / m on
// the first step (BDF2 in time, forward Euler to start; r the summed load
// or torque, m the mass or moment of inertia).  Given the adjoint of v':
// adds those of v and v_prev and returns that of r.
LBIB_HD double bdf2_vjp(bool first, double m, double vh_new, double& vh, double& vph) {
  if (first) {
    vh += vh_new;
    return vh_new / m;
  }
  vh += (4.0 / 3.0) * vh_new;
  vph += (-1.0 / 3.0) * vh_new;
  return (2.0 / 3.0) * vh_new / m;
}

// Vertex of a rigid particle after the step: X' = x_c' + R(theta') r0 and
// the rigid-body velocity there, U_k = U' + Omega' x (X' - x_c').
LBIB_HD void rigid_vertex_fwd(double r0x, double r0y, double xc, double yc, double th, double Ux,
                              double Uy, double Om, double X[2], double Uk[2]) {
  const double cs = cos(th), sn = sin(th);
  const double relx = r0x * cs - r0y * sn, rely = r0x * sn + r0y * cs;
  X[0] = xc + relx;
  X[1] = yc + rely;
  Uk[0] = Ux - Om * rely;
  Uk[1] = Uy + Om * relx;
}

// Given the adjoints of X' (xh) and of U_k (uh) at a vertex with arm
// rel = R(theta') r0: adds those of x_c' (ch), theta' (thh), U' (Uh) and
// Omega' (Omh).
LBIB_HD void rigid_vertex_vjp(double relx, double rely, double Om, double xhx, double xhy,
                              double uhx, double uhy, double ch[2], double& thh, double Uh[2],
                              double& Omh) {
  ch[0] += xhx;
  ch[1] += xhy;
  Uh[0] += uhx;
  Uh[1] += uhy;
  Omh += -uhx * rely + uhy * relx;
  // adjoint of rel: from X' directly and through Omega' x rel
  const double rhx = xhx + Om * uhy, rhy = xhy - Om * uhx;
  thh += -rhx * rely + rhy * relx;   // d rel / d theta = (-rel_y, rel_x)
}

}  // namespace adj
}  // namespace lbib
