// Test-only C wrappers around the local derivative functions of the adjoint
// (compiled on the host with g++ by tests/test_adj_math.py).
#include "adj_math.h"

using namespace lbib;
using namespace lbib::adj;

extern "C" {
double t_phi(double r) { return roma_phi(r); }
double t_dphi(double r) { return roma_dphi(r); }
double t_ddphi(double r) { return roma_ddphi(r); }

void t_collide_fwd(const double* h, double Fx, double Fy, double omega, double pre, double* out) {
  collide_fwd(h, Fx, Fy, omega, pre, out, out[9], out[10]);
}
void t_collide_vjp(const double* h, double Fx, double Fy, double omega, double pre, const double* a,
                   double uhx, double uhy, double* out) {
  collide_vjp(h, Fx, Fy, omega, pre, a, uhx, uhy, out, out[9], out[10]);
}
void t_star_vjp(double rho, double ux, double uy, double rh, double uxh, double uyh, double* hh) {
  for (int i = 0; i < 9; ++i) hh[i] = 0.0;
  star_vjp(rho, ux, uy, rh, uxh, uyh, hh);
}
void t_strain_fwd(double dx, double dy, double l0, double ks, double* s) { strain_fwd(dx, dy, l0, ks, s[0], s[1]); }
void t_strain_vjp(double dx, double dy, double l0, double ks, double shx, double shy, double* out) {
  out[0] = out[1] = out[2] = 0.0;
  strain_vjp(dx, dy, l0, ks, shx, shy, out[0], out[1], out[2]);
}
void t_bend_fwd(const double* d, double th0, double kb, double* F) {
  bend_fwd(d[0], d[1], d[2], d[3], th0, kb, F, F + 2, F + 4);
}
void t_bend_vjp(const double* d, double th0, double kb, const double* Fh, double* out) {
  for (int i = 0; i < 5; ++i) out[i] = 0.0;
  bend_vjp(d[0], d[1], d[2], d[3], th0, kb, Fh, Fh + 2, Fh + 4, out, out + 2, out[4]);
}
void t_spring_vjp(double dx, double dy, double y, double ddx, double ddy, double sigma, double y_eq,
                  double Fhx, double Fhy, double* out) {
  for (int i = 0; i < 5; ++i) out[i] = 0.0;
  spring_vjp(dx, dy, y, ddx, ddy, sigma, y_eq, Fhx, Fhy, out[0], out[1], out[2], out[3], out[4]);
}
void t_hydro_fwd(double pr, const double* g, double nu, double nx, double ny, double len, double* F) {
  hydro_fwd(pr, g, nu, nx, ny, len, F[0], F[1]);
}
void t_hydro_vjp(double pr, const double* g, double nu, double nx, double ny, double len, double Fhx,
                 double Fhy, double* out) {
  for (int i = 0; i < 8; ++i) out[i] = 0.0;
  hydro_vjp(pr, g, nu, nx, ny, len, Fhx, Fhy, out[0], out + 1, out[5], out[6], out[7]);
}
void t_spring_fwd(double dx, double dy, double y, double sigma, double y_eq, double* F) {
  spring_fwd(dx, dy, y, sigma, y_eq, F[0], F[1]);
}
void t_rigid_load_vjp(double rx, double ry, double fx, double fy, double Fhx, double Fhy, double Mh,
                      double* out) {
  for (int i = 0; i < 4; ++i) out[i] = 0.0;
  rigid_load_vjp(rx, ry, fx, fy, Fhx, Fhy, Mh, out[0], out[1], out[2], out[3]);
}
double t_bdf2_vjp(int first, double m, double vh_new, double* out) {
  out[0] = out[1] = 0.0;
  return bdf2_vjp(first != 0, m, vh_new, out[0], out[1]);
}
void t_rigid_vertex_fwd(double r0x, double r0y, const double* s, double* out) {
  rigid_vertex_fwd(r0x, r0y, s[0], s[1], s[2], s[3], s[4], s[5], out, out + 2);
}
void t_rigid_vertex_vjp(double relx, double rely, double Om, const double* xh, const double* uh,
                        double* out) {
  for (int i = 0; i < 6; ++i) out[i] = 0.0;
  double ch[2] = {0.0, 0.0}, Uh[2] = {0.0, 0.0};
  rigid_vertex_vjp(relx, rely, Om, xh[0], xh[1], uh[0], uh[1], ch, out[2], Uh, out[5]);
  out[0] = ch[0];
  out[1] = ch[1];
  out[3] = Uh[0];
  out[4] = Uh[1];
}
void t_area_vjp(double dx, double dy, double kappa, double Fhx, double Fhy, double* out) {
  out[0] = out[1] = 0.0;
  out[2] = area_vjp(dx, dy, kappa, Fhx, Fhy, out[0], out[1]);
}
}
