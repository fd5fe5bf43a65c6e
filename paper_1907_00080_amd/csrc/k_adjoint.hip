// k_adjoint.hip - reverse sweep of one LB-IB time step (discrete adjoint).
//
// Forward step n (bond topology frozen; order as in the forward kernels):
//   f_pre = pull(h^n)                       streaming, halfway bounce-back
//   rho*, u* = moments of f_pre, u* = (j + g/2)/rho*
//   RBC:   F_k = membrane forces at X^n                    (Sec. 2.2)
//   soft:  F_el = probe loads(rho*, u*) + springs,          (Sec. 2.2, 2.3)
//          X^{n+1} = X + U0 + Fv/(2 m_v), U0 = interp(u*, X),
//          F_k = 2 (X^{n+1} - X - U0) ds_k
//   rigid: F_tot, M_tot from the element loads, U', Omega' by BDF2, the
//          reference point and angle moved, X^{n+1} = x_c' + R(theta') r0,
//          F_k = 2 (U' + Omega' x (X^{n+1} - x_c') - U0) ds_k
//          (Eqs. linearVelRig, angularVelRig)
//   F_E = g + sum_k F_k delta(x - X_k)                     spreading
//   h^{n+1}, u = collide(f_pre, F_E)                       (Sec. 2.1)
//   RBC:   X^{n+1} = 2/3 (2 X^n - X^{n-1}/2 + interp(u, X^n))  (Eq. kinematicPos;
//          forward Euler on the first step)
// The kernels below apply the transposed Jacobian of this map to the
// adjoint state (h^, X^, X^_prev, and the rigid particles' state) in reverse
// order, and accumulate the derivatives with respect to each body's k_s, k_b
// and bond constant sigma.
// All adjoint arithmetic is float64; the forward data of step n come from
// the segment store of the checkpointed recomputation.
//
// Scatter-form terms (the spreading of the stored marker forces, the
// transpose of an interpolation or of a probe evaluation) add into dense
// fields of exact two-word fixed-point accumulators (value = hi 2^-24 +
// lo 2^-72): each contribution is rounded once to the 2^-72 grid and the
// sums are exact integer sums, so they do not depend on the order of the
// atomics and the gradient is bitwise reproducible from run to run.
#include "adj_math.h"
#include "lbib_dev.h"

namespace lbib {

namespace {

// 3x3 stencil of a point with kernel weights and their derivatives
// (weights are phi(node - X); rows beyond the walls are marked invalid).
struct Stencil {
  int col[3], row[3];
  bool ok[3];
  double wx[3], dwx[3], ddwx[3], wy[3], dwy[3], ddwy[3];
};

__device__ inline void stencil_at(const LatDev& L, double X, double Y, bool second, Stencil& s) {
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  const bool pery = L.periodic_y != 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double rx = cxr + (a - 1);
    s.col[a] = wrap_i((int)rx, L.nx);
    s.wx[a] = roma_phi(rx - X);
    s.dwx[a] = roma_dphi(rx - X);
    s.ddwx[a] = second ? roma_ddphi(rx - X) : 0.0;
    const double ry = cyr + (a - 1);
    int row = (int)ry;
    bool ok = true;
    if (pery) row = wrap_i(row, L.ny);
    else ok = row >= 0 && row < L.ny;
    s.row[a] = row;
    s.ok[a] = ok;
    s.wy[a] = roma_phi(ry - Y);
    s.dwy[a] = roma_dphi(ry - Y);
    s.ddwy[a] = second ? roma_ddphi(ry - Y) : 0.0;
  }
}

__device__ inline int wrap_idx(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

constexpr int kAdjThreads = 256;

// Adds v to the accumulator entry k.  v is split into a coarse part, an
// integer multiple of 2^-24 (v rounded to that grid, exact as a double),
// and the exact remainder, |r| <= 2^-25, rounded to a multiple of 2^-72;
// each part is added to its own 64-bit integer word.  Integer sums are
// exact in any order; the atomics return nothing, so none waits.  Range: a
// term of magnitude 2^30 or more (or not finite) is refused and flagged, so
// the coarse word holds sums of up to 2^9 such terms and the fine word
// (|r 2^72| <= 2^47 per term) of up to 2^16 terms without overflow.
__device__ inline void acc_add(const AccField& f, long long k, double v, int* bad) {
  if (!(fabs(v) < 0x1p30)) {   // also NaN
    atomicOr(bad, 1);
    return;
  }
  const double c = rint(v * 0x1p24);       // integer valued, |c| < 2^54
  const double r = v - c * 0x1p-24;        // exact
  const long long hi = (long long)c, lo = __double2ll_rn(r * 0x1p72);
  if (hi != 0) __hip_atomic_fetch_add(&f.hi[k], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (lo != 0) __hip_atomic_fetch_add(&f.lo[k], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double acc_get(const AccField& f, long long k) {
  return double(f.hi[k]) * 0x1p-24 + double(f.lo[k]) * 0x1p-72;
}

__device__ inline void acc_clear(const AccField& f, long long k) {
  f.hi[k] = 0;
  f.lo[k] = 0;
}

// Sums K values over the workgroup in a fixed order (wave_sum within each
// wave, then the waves in turn): every thread gets the totals.
template <int K>
__device__ inline void block_sum(double v[K], double (*s)[kAdjThreads / 64]) {
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double x = wave_sum(v[k]);
    if (lane == 0) s[k][w] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) x += s[k][i];
    v[k] = x;
  }
  __syncthreads();
}

// Bond geometry of element l of a particle (Eq. adhFor): for a bonded ligand
// element, the bond length y from the centroid (cx, cy) to its receptor and
// (ddx, ddy) = dy/dc.  Returns false for an element without a bond.
template <typename T>
__device__ inline bool bond_geometry(const Ptrs<T>& p, const LatDev& L, const BodyDev* Bp, int l,
                                     double cx, double cy, double& yl, double& ddx, double& ddy) {
  if (Bp->lig_stride <= 0 || l % Bp->lig_stride != 0) return false;
  const int r = p.l2r[Bp->lig_base + l / Bp->lig_stride];
  if (r < 0) return false;
  const int wall = r < L.n_rec0 ? 0 : 1;
  const double xr = p.rec_x[L.rec_base + r];
  const double cxw = cx - L.nx * floor(cx / L.nx);
  double dx = xr - cxw;
  if (dx > 0.5 * L.nx) dx -= L.nx;
  else if (dx < -0.5 * L.nx) dx += L.nx;
  const double yw = wall == 0 ? -0.5 : L.ny - 0.5;
  const double dy = cy - yw;
  yl = sqrt(dx * dx + dy * dy);
  ddx = -dx / yl;
  ddy = dy / yl;
  return true;
}

// Probe load of an element (centroid c, outward normal n, length len) read
// at q = c + 1.2 n, its ordinate clamped into the fluid (Eqs. hydroForP,
// hydroForNu, from rho*, u* in mom).  Returns the load in (pfx, pfy); given
// its adjoint (Fhx, Fhy), adds the adjoints of c, n and len and scatters
// those of rho*, u* into Rh.
__device__ inline void probe_adjoint(const LatDev& L, const AdjPtrs& a, double cx, double cy,
                                     double nxl, double nyl, double len, double nu, double Fhx,
                                     double Fhy, double& pfx, double& pfy, double& Chx, double& Chy,
                                     double& nhx, double& nhy, double& lenh) {
  const long long N = L.plane;
  const double* mom = a.mom;
  const double qx = cx + 1.2 * nxl;
  const double qy_raw = cy + 1.2 * nyl;
  double qy = qy_raw;
  bool clamped = false;
  if (!L.periodic_y) {
    qy = fmin(fmax(qy_raw, 0.5), L.ny - 1.5);
    clamped = qy != qy_raw;
  }
  Stencil s;
  stencil_at(L, qx, qy, true, s);
  double rq = 0.0, g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int bb = 0; bb < 3; ++bb) {
    if (!s.ok[bb]) continue;
    for (int c = 0; c < 3; ++c) {
      const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
      const double w = s.wx[c] * s.wy[bb];
      const double r0 = mom[node], us = mom[N + node], vs = mom[2 * N + node];
      rq += r0 * w;
      g[0] -= us * s.dwx[c] * s.wy[bb];
      g[1] -= us * s.wx[c] * s.dwy[bb];
      g[2] -= vs * s.dwx[c] * s.wy[bb];
      g[3] -= vs * s.wx[c] * s.dwy[bb];
    }
  }
  const double pr = (rq - 1.0) * (1.0 / 3.0);
  adj::hydro_fwd(pr, g, nu, nxl, nyl, len, pfx, pfy);
  double prh = 0.0, gh[4] = {0.0, 0.0, 0.0, 0.0}, nh2x = 0.0, nh2y = 0.0;
  adj::hydro_vjp(pr, g, nu, nxl, nyl, len, Fhx, Fhy, prh, gh, nh2x, nh2y, lenh);
  const double rqh = prh * (1.0 / 3.0);
  double qhx = 0.0, qhy = 0.0;
  for (int bb = 0; bb < 3; ++bb) {
    if (!s.ok[bb]) continue;
    for (int c = 0; c < 3; ++c) {
      const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
      const double wx = s.wx[c], wy = s.wy[bb], dwx = s.dwx[c], dwy = s.dwy[bb];
      const double ddwx = s.ddwx[c], ddwy = s.ddwy[bb];
      const double r0 = mom[node], us = mom[N + node], vs = mom[2 * N + node];
      qhx += -rqh * r0 * dwx * wy + gh[0] * us * ddwx * wy + gh[1] * us * dwx * dwy +
             gh[2] * vs * ddwx * wy + gh[3] * vs * dwx * dwy;
      qhy += -rqh * r0 * wx * dwy + gh[0] * us * dwx * dwy + gh[1] * us * wx * ddwy +
             gh[2] * vs * dwx * dwy + gh[3] * vs * wx * ddwy;
    }
  }
  // the scatter last: no load waits behind its atomics
  for (int bb = 0; bb < 3; ++bb) {
    if (!s.ok[bb]) continue;
    for (int c = 0; c < 3; ++c) {
      const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
      const double wx = s.wx[c], wy = s.wy[bb], dwx = s.dwx[c], dwy = s.dwy[bb];
      acc_add(a.Rh, node, rqh * wx * wy, a.bad);
      acc_add(a.Rh, N + node, -gh[0] * dwx * wy - gh[1] * wx * dwy, a.bad);
      acc_add(a.Rh, 2 * N + node, -gh[2] * dwx * wy - gh[3] * wx * dwy, a.bad);
    }
  }
  if (clamped) qhy = 0.0;
  Chx += qhx;
  Chy += qhy;
  nhx += nh2x + 1.2 * qhx;
  nhy += nh2y + 1.2 * qhy;
}

}  // namespace

// --------------------------------------------------------------- markers
// Every marker: (a) spreading of its stored force into the Eulerian IB force
// of step n (without g); (b) X^n gets the adjoint carried by
// X_prev^{n+1} = X^n; (c) red cells: reverse of the kinematic BDF2 / Euler
// update, whose interpolation of the stored velocity u^n scatters into the
// adjoint of u.
// One marker per row of 16 lanes: lane j < 9 of the row takes stencil node
// (j / 3, j % 3), its atomics and its share of the interpolation gradient;
// the row's sum (xor butterfly, the same value in every lane) goes to lane 0,
// which writes the marker's outputs.  Every lane of the row takes part in the
// sums, also where the marker index is past the end.
template <typename T>
__device__ inline void marker_adjoint(const Ptrs<T>& p, const AdjPtrs& a, int gm, int j) {
  const bool live = gm < p.nm_total;
  const LatDev L = p.lat[0];
  const long long N = L.plane;
  double gx = 0.0, gy = 0.0;
  const int bb = j / 3, c = j - 3 * (j / 3);
  bool mine = false, rbc = false;
  long long node = 0;
  double w = 0.0, fx = 0.0, fy = 0.0, ux = 0.0, uy = 0.0, xa = 0.0, ya = 0.0, dx = 0.0, dy = 0.0;
  if (live) {
    const int kind = p.minfo[gm] & 3;
    rbc = kind == kRBC;
    const double X = a.x[gm], Y = a.y[gm];
    // every load before the first atomic: a load issued behind pending
    // atomics waits for all of them
    fx = a.fx[gm];
    fy = a.fy[gm];
    xa = a.xa[gm];
    ya = a.ya[gm];
    dx = a.xma[gm];
    dy = a.yma[gm];
    const double c3 = a.first ? 1.0 : 2.0 / 3.0;
    ux = rbc ? c3 * xa : 0.0;
    uy = rbc ? c3 * ya : 0.0;
    // this lane's node of the 3x3 stencil (the weights as stencil_at takes them)
    const double rx = floor(X + 0.5) + (c - 1), ry = floor(Y + 0.5) + (bb - 1);
    int row = (int)ry;
    bool ok = true;
    if (L.periodic_y != 0) row = wrap_i(row, L.ny);
    else ok = row >= 0 && row < L.ny;
    mine = j < 9 && ok;
    if (mine) {
      const double wx = roma_phi(rx - X), dwx = roma_dphi(rx - X);
      const double wy = roma_phi(ry - Y), dwy = roma_dphi(ry - Y);
      node = (long long)row * L.pitch + wrap_i((int)rx, L.nx);
      w = wx * wy;
      if (rbc) {
        const T* U = (const T*)a.u;
        const double uu = ux * double(U[node]) + uy * double(U[N + node]);
        gx = -uu * dwx * wy;
        gy = -uu * wx * dwy;
      }
    }
  }
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) {
    gx += __shfl_xor(gx, m, 16);
    gy += __shfl_xor(gy, m, 16);
  }
  if (mine) {
    acc_add(a.FE, node, fx * w, a.bad);
    acc_add(a.FE, N + node, fy * w, a.bad);
    if (rbc) {
      acc_add(a.Uh, node, ux * w, a.bad);
      acc_add(a.Uh, N + node, uy * w, a.bad);
    }
  }
  if (!live || j != 0) return;
  const double c1 = a.first ? 1.0 : 4.0 / 3.0, c2 = a.first ? 0.0 : -1.0 / 3.0;
  if (rbc) {
    dx += c1 * xa + gx;
    dy += c1 * ya + gy;
    a.xma[gm] = c2 * xa;
    a.yma[gm] = c2 * ya;
  } else {
    a.xma[gm] = 0.0;
    a.yma[gm] = 0.0;
  }
  a.dirx[gm] = dx;
  a.diry[gm] = dy;
}

// --------------------------------------------------------------- collide
// Per node: reverse of the forced collision; adjoint of the pulled
// populations and of the Eulerian force.
template <typename T>
__global__ void ka_collide(Ptrs<T> p, AdjPtrs a) {
  const LatDev L = p.lat[0];
  const long long N = L.plane;
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const unsigned un = (unsigned)node, pitch = (unsigned)L.pitch;
  const int x = (int)(un % pitch), y = (int)(un / pitch);
  if (x >= L.nx) return;   // row padding
  const T* H = (const T*)a.h;
  double h[kQ], ah[kQ], hh[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    int xs = wrap_idx(x - ex(i), L.nx);
    int ys = y - ey(i);
    const bool out = ys < 0 || ys >= L.ny;
    ys = wrap_idx(ys, L.ny);
    const long long src = (out && !L.periodic_y) ? opp(i) * N + node : i * N + (long long)ys * L.pitch + xs;
    h[i] = double(H[src]);
    ah[i] = a.ha[i * N + node];
  }
  const double Fx = L.gx + acc_get(a.FE, node), Fy = L.gy + acc_get(a.FE, N + node);
  const double omega = L.omega, pre = L.pre;
  double Fhx, Fhy;
  adj::collide_vjp(h, Fx, Fy, omega, pre, ah, acc_get(a.Uh, node), acc_get(a.Uh, N + node), hh, Fhx,
                   Fhy);
#pragma unroll
  for (int i = 0; i < kQ; ++i) a.fph[i * N + node] = hh[i];
  a.FEh[node] = Fhx;
  a.FEh[N + node] = Fhy;
  // pre-forcing moments rho*, u* (probe and particle-vertex interpolation)
  double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += h[i];
    jx += ex(i) * h[i];
    jy += ey(i) * h[i];
  }
  const double rho = 1.0 + drho;
  a.mom[node] = rho;
  a.mom[N + node] = (jx + 0.5 * L.gx) / rho;
  a.mom[2 * N + node] = (jy + 0.5 * L.gy) / rho;
  // this node's accumulators are consumed: clear them for the next step
  // (rho^*, u^* are filled by the body kernel that follows)
  acc_clear(a.FE, node);
  acc_clear(a.FE, N + node);
  acc_clear(a.Uh, node);
  acc_clear(a.Uh, N + node);
  acc_clear(a.Rh, node);
  acc_clear(a.Rh, N + node);
  acc_clear(a.Rh, 2 * N + node);
}

// --------------------------------------------------------------- bodies
// Rigid particle (Sec. 2.3, Eqs. linearVelRig, angularVelRig), forward step:
//   f_e = probe load + adhesion spring of element e at X^n;
//   F_tot = sum f_e, M_tot = sum (c_e - x_c) x f_e;
//   U', Omega' by BDF2 (forward Euler on the first step);
//   x_c' = x_c + U', theta' = theta + Omega', X' = x_c' + R(theta') r0;
//   F_k = 2 (U_k - U0_k) ds_k, U_k = U' + Omega' x (X'_k - x_c'),
//   U0 = interp(u*, X^n), spread at X^n.
// Its reverse: the adjoint of X' (per vertex) and of the state after the
// step (rig) give those of the loads, of X^n (per vertex, out), of sigma and
// of the state before the step (rig, out).  X^n itself was formed from the
// state by the previous step, whose reverse maps its adjoint onto it.
template <typename T>
__device__ void rigid_adjoint(const Ptrs<T>& p, const AdjPtrs& a, int b,
                              double (*s_red)[kAdjThreads / 64]) {
  const BodyDev* Bp = p.body + b;
  const BodyDev& S0 = a.body0[b];   // state before the step
  const BodyDev& S1 = a.body1[b];   // after it
  const int nv = Bp->nv, v0 = Bp->v0;
  const LatDev L = p.lat[0];
  const long long N = L.plane;
  const double nu = (L.tau - 0.5) / 3.0, sigma = Bp->sigma;
  const int t = threadIdx.x, nt = blockDim.x;
  const double* X = a.x + v0;
  const double* Y = a.y + v0;
  const double* mom = a.mom;
  double* R = a.rig + 9 * b;
  double rin[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) rin[k] = R[k];
  const bool first = a.first != 0;

  // ---- vertices: adjoint of the spread force F_k, through U_k to the
  // state after the step, through U0 to u*, and of X^n by the spreading
  // weights and by U0's interpolation weights
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // x_c'^ (2), theta'^, U'^ (2), Omega'^
  for (int v = t; v < nv; v += nt) {
    const int gm = v0 + v;
    const int vp = v + 1 == nv ? 0 : v + 1, vm = v == 0 ? nv - 1 : v - 1;
    const double lr = sqrt((X[vp] - X[v]) * (X[vp] - X[v]) + (Y[vp] - Y[v]) * (Y[vp] - Y[v]));
    const double ll = sqrt((X[v] - X[vm]) * (X[v] - X[vm]) + (Y[v] - Y[vm]) * (Y[v] - Y[vm]));
    const double ds = 0.5 * (ll + lr);
    Stencil s;
    stencil_at(L, X[v], Y[v], false, s);
    const double Fx = a.fx[gm], Fy = a.fy[gm];
    double fhx = 0.0, fhy = 0.0, gx = 0.0, gy = 0.0, U0x = 0.0, U0y = 0.0;
    for (int bb = 0; bb < 3; ++bb) {
      if (!s.ok[bb]) continue;
      for (int c = 0; c < 3; ++c) {
        const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
        const double w = s.wx[c] * s.wy[bb];
        const double ex_ = a.FEh[node], ey_ = a.FEh[N + node];
        fhx += ex_ * w;
        fhy += ey_ * w;
        U0x += mom[N + node] * w;
        U0y += mom[2 * N + node] * w;
        const double sf = Fx * ex_ + Fy * ey_;
        gx -= sf * s.dwx[c] * s.wy[bb];
        gy -= sf * s.wx[c] * s.dwy[bb];
      }
    }
    const double relx = a.xn[gm] - S1.xc, rely = a.yn[gm] - S1.yc;
    const double Ukx = S1.U[0] + S1.Om * (-rely), Uky = S1.U[1] + S1.Om * relx;
    const double dsh = 2.0 * ((Ukx - U0x) * fhx + (Uky - U0y) * fhy);
    const double uhx = 2.0 * ds * fhx, uhy = 2.0 * ds * fhy;   // adjoint of U_k; U0 gets minus it
    double g2x = 0.0, g2y = 0.0;
    for (int bb = 0; bb < 3; ++bb) {
      if (!s.ok[bb]) continue;
      for (int c = 0; c < 3; ++c) {
        const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
        const double uu = -uhx * mom[N + node] - uhy * mom[2 * N + node];
        g2x -= uu * s.dwx[c] * s.wy[bb];
        g2y -= uu * s.wx[c] * s.dwy[bb];
      }
    }
    const double xa = a.xa[gm], ya = a.ya[gm], dirx = a.dirx[gm], diry = a.diry[gm];
    const double Om1 = S1.Om;
    // the scatter after every load of this vertex
    for (int bb = 0; bb < 3; ++bb) {
      if (!s.ok[bb]) continue;
      for (int c = 0; c < 3; ++c) {
        const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
        const double w = s.wx[c] * s.wy[bb];
        acc_add(a.Rh, N + node, -uhx * w, a.bad);
        acc_add(a.Rh, 2 * N + node, -uhy * w, a.bad);
      }
    }
    double ch[2] = {0.0, 0.0}, Uh[2] = {0.0, 0.0}, thh = 0.0, Omh = 0.0;
    adj::rigid_vertex_vjp(relx, rely, Om1, xa, ya, uhx, uhy, ch, thh, Uh, Omh);
    acc[0] += ch[0];
    acc[1] += ch[1];
    acc[2] += thh;
    acc[3] += Uh[0];
    acc[4] += Uh[1];
    acc[5] += Omh;
    a.dirx[gm] = dirx + gx + g2x;
    a.diry[gm] = diry + gy + g2y;
    a.dsh[gm] = dsh;
  }
  block_sum<6>(acc, s_red);   // barriers also publish the vertex pass

  // ---- the state: x_c' = x_c + U', theta' = theta + Omega', BDF2
  const double xch[2] = {rin[0] + acc[0], rin[1] + acc[1]};
  const double thh = rin[2] + acc[2];
  const double Uh1[2] = {rin[3] + acc[3] + xch[0], rin[4] + acc[4] + xch[1]};
  const double Omh1 = rin[7] + acc[5] + thh;
  double Uh0[2] = {rin[5], rin[6]}, Umh0[2] = {0.0, 0.0}, Omh0 = rin[8], Ommh0 = 0.0;
  const double Fh[2] = {adj::bdf2_vjp(first, Bp->mass, Uh1[0], Uh0[0], Umh0[0]),
                        adj::bdf2_vjp(first, Bp->mass, Uh1[1], Uh0[1], Umh0[1])};
  const double Mh = adj::bdf2_vjp(first, Bp->inertia, Omh1, Omh0, Ommh0);

  // ---- elements: loads into F_tot and M_tot (arms from x_c of the state
  // before the step)
  double arm[3] = {0.0, 0.0, 0.0};   // x_c^ (2) from the arms, sigma^
  for (int l = t; l < nv; l += nt) {
    const int gl = v0 + l;
    const int lp = l + 1 == nv ? 0 : l + 1;
    const double dx = X[lp] - X[l], dy = Y[lp] - Y[l];
    const double len = sqrt(dx * dx + dy * dy);
    const double cx = 0.5 * (X[l] + X[lp]), cy = 0.5 * (Y[l] + Y[lp]);
    const double nxl = dy / len, nyl = -dx / len;
    const double rx = cx - S0.xc, ry = cy - S0.yc;
    // adjoint of f_e (it needs only the arm; the arm's needs f_e, below)
    double Fex = 0.0, Fey = 0.0, rhx = 0.0, rhy = 0.0;
    adj::rigid_load_vjp(rx, ry, 0.0, 0.0, Fh[0], Fh[1], Mh, Fex, Fey, rhx, rhy);
    double Dhx = 0.0, Dhy = 0.0, Chx = 0.0, Chy = 0.0;
    double lenh = 0.5 * (a.dsh[gl] + a.dsh[v0 + lp]);
    double fex = 0.0, fey = 0.0;
    double yl, ddx, ddy;
    if (bond_geometry(p, L, Bp, l, cx, cy, yl, ddx, ddy)) {
      adj::spring_fwd(dx, dy, yl, sigma, L.y_eq, fex, fey);
      adj::spring_vjp(dx, dy, yl, ddx, ddy, sigma, L.y_eq, Fex, Fey, Dhx, Dhy, Chx, Chy, arm[2]);
    }
    double pfx, pfy, nhx = 0.0, nhy = 0.0;
    probe_adjoint(L, a, cx, cy, nxl, nyl, len, nu, Fex, Fey, pfx, pfy, Chx, Chy, nhx, nhy, lenh);
    fex += pfx;
    fey += pfy;
    // adjoint of the arm r = c - x_c: to the centroid and to x_c
    double fdx = 0.0, fdy = 0.0;
    adj::rigid_load_vjp(rx, ry, fex, fey, 0.0, 0.0, Mh, fdx, fdy, rhx, rhy);
    Chx += rhx;
    Chy += rhy;
    arm[0] -= rhx;
    arm[1] -= rhy;
    adj::unit_vjp(dx, dy, -nhy, nhx, 0.0, Dhx, Dhy);
    adj::unit_vjp(dx, dy, 0.0, 0.0, lenh, Dhx, Dhy);
    a.Dx[gl] = Dhx;
    a.Dy[gl] = Dhy;
    a.Cx[gl] = Chx;
    a.Cy[gl] = Chy;
  }
  block_sum<3>(arm, s_red);

  // ---- vertices: gather the element terms into the adjoint of X^n
  for (int v = t; v < nv; v += nt) {
    const int gm = v0 + v;
    const int vm = v == 0 ? nv - 1 : v - 1;
    a.xa[gm] = a.dirx[gm] + a.Dx[v0 + vm] - a.Dx[gm] + 0.5 * (a.Cx[gm] + a.Cx[v0 + vm]);
    a.ya[gm] = a.diry[gm] + a.Dy[v0 + vm] - a.Dy[gm] + 0.5 * (a.Cy[gm] + a.Cy[v0 + vm]);
  }
  if (t == 0) {
    R[0] = xch[0] + arm[0];
    R[1] = xch[1] + arm[1];
    R[2] = thh;
    R[3] = Uh0[0];
    R[4] = Uh0[1];
    R[5] = Umh0[0];
    R[6] = Umh0[1];
    R[7] = Omh0;
    R[8] = Ommh0;
    a.grad[3 * b + 2] += arm[2];
  }
}

// One workgroup per body.
template <typename T>
__global__ __launch_bounds__(kAdjThreads) void ka_body(Ptrs<T> p, AdjPtrs a) {
  __shared__ double s_red[6][kAdjThreads / 64];
  const int b = blockIdx.x;
  const BodyDev* Bp = p.body + b;
  const int kind = Bp->kind, nv = Bp->nv, v0 = Bp->v0;
  if (kind == kRigid) {
    rigid_adjoint(p, a, b, s_red);
    return;
  }
  const LatDev L = p.lat[0];
  const long long N = L.plane;
  const bool pery = L.periodic_y != 0;
  const double nu = (L.tau - 0.5) / 3.0;
  const double ks = Bp->ks, kb = Bp->kb, ka = Bp->ka, p_ref = Bp->p_ref, A0 = Bp->A0;
  const double mv = Bp->mv, sigma = Bp->sigma;
  const int t = threadIdx.x, nt = blockDim.x;
  const double* X = a.x + v0;
  const double* Y = a.y + v0;
  const double* mom = a.mom;

  // ---- phase A (vertices): spread adjoint; soft Verlet / coupling chain
  double shoe = 0.0;
  for (int v = t; v < nv; v += nt) {
    const int gm = v0 + v;
    const int vp = v + 1 == nv ? 0 : v + 1, vm = v == 0 ? nv - 1 : v - 1;
    shoe += X[v] * Y[vp] - X[vp] * Y[v];
    Stencil s;
    stencil_at(L, X[v], Y[v], false, s);
    const double Fx = a.fx[gm], Fy = a.fy[gm];
    double fhx = 0.0, fhy = 0.0, gx = 0.0, gy = 0.0;
    for (int bb = 0; bb < 3; ++bb) {
      if (!s.ok[bb]) continue;
      for (int c = 0; c < 3; ++c) {
        const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
        const double w = s.wx[c] * s.wy[bb];
        const double ex_ = a.FEh[node], ey_ = a.FEh[N + node];
        fhx += ex_ * w;
        fhy += ey_ * w;
        const double sf = Fx * ex_ + Fy * ey_;
        gx -= sf * s.dwx[c] * s.wy[bb];
        gy -= sf * s.wx[c] * s.dwy[bb];
      }
    }
    double dxv = a.dirx[gm] + gx, dyv = a.diry[gm] + gy;
    double fvx = fhx, fvy = fhy, dsh = 0.0;
    if (kind == kSoft) {
      const double xa = a.xa[gm], ya = a.ya[gm];
      const double lr = sqrt((X[vp] - X[v]) * (X[vp] - X[v]) + (Y[vp] - Y[v]) * (Y[vp] - Y[v]));
      const double ll = sqrt((X[v] - X[vm]) * (X[v] - X[vm]) + (Y[v] - Y[vm]) * (Y[v] - Y[vm]));
      const double ds = 0.5 * (ll + lr);
      // U0 = interp(u*, X) and its adjoint (= the adjoint of X^{n+1})
      double U0x = 0.0, U0y = 0.0, g2x = 0.0, g2y = 0.0;
      for (int bb = 0; bb < 3; ++bb) {
        if (!s.ok[bb]) continue;
        for (int c = 0; c < 3; ++c) {
          const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
          const double w = s.wx[c] * s.wy[bb];
          const double us = mom[N + node], vs = mom[2 * N + node];
          U0x += us * w;
          U0y += vs * w;
          const double uu = xa * us + ya * vs;
          g2x -= uu * s.dwx[c] * s.wy[bb];
          g2y -= uu * s.wx[c] * s.dwy[bb];
        }
      }
      const double xnv = a.xn[gm], ynv = a.yn[gm], Xv = X[v], Yv = Y[v];
      // the scatter after every load of this vertex
      for (int bb = 0; bb < 3; ++bb) {
        if (!s.ok[bb]) continue;
        for (int c = 0; c < 3; ++c) {
          const long long node = (long long)s.row[bb] * L.pitch + s.col[c];
          const double w = s.wx[c] * s.wy[bb];
          acc_add(a.Rh, N + node, xa * w, a.bad);
          acc_add(a.Rh, 2 * N + node, ya * w, a.bad);
        }
      }
      const double xn1h = xa + 2.0 * ds * fhx, yn1h = ya + 2.0 * ds * fhy;
      dxv += xa + g2x;
      dyv += ya + g2y;
      fvx = 0.5 * xn1h / mv;
      fvy = 0.5 * yn1h / mv;
      dsh = 2.0 * ((xnv - Xv - U0x) * fhx + (ynv - Yv - U0y) * fhy);
    }
    a.dirx[gm] = dxv;
    a.diry[gm] = dyv;
    a.fvx[gm] = fvx;
    a.fvy[gm] = fvy;
    a.dsh[gm] = dsh;
  }
  {
    double v1[1] = {shoe};
    block_sum<1>(v1, s_red);   // barriers also publish phase A
    shoe = v1[0];
  }
  const double area = 0.5 * shoe;
  const double kappa = ka * (1.0 - area / A0) * p_ref;

  // ---- phase B (elements l: v -> v+1) and bending (vertices)
  double ksh = 0.0, kbh = 0.0, sigh = 0.0, kaph = 0.0;
  for (int l = t; l < nv; l += nt) {
    const int gl = v0 + l;
    const int lp = l + 1 == nv ? 0 : l + 1, lm = l == 0 ? nv - 1 : l - 1;
    const double dx = X[lp] - X[l], dy = Y[lp] - Y[l];
    const double len = sqrt(dx * dx + dy * dy);
    const double f0x = a.fvx[gl], f0y = a.fvy[gl], f1x = a.fvx[v0 + lp], f1y = a.fvy[v0 + lp];
    double Dhx = 0.0, Dhy = 0.0, Chx = 0.0, Chy = 0.0, lenh = 0.0;
    adj::strain_vjp(dx, dy, p.l0[gl], ks, f0x - f1x, f0y - f1y, Dhx, Dhy, ksh);
    const double Fex = 0.5 * (f0x + f1x), Fey = 0.5 * (f0y + f1y);   // element-load adjoint
    kaph += adj::area_vjp(dx, dy, kappa, Fex, Fey, Dhx, Dhy);
    // bending operands (vertex l: left element lm, right element l), read
    // before the probe's scatter
    const double dLx = X[l] - X[lm], dLy = Y[l] - Y[lm];
    const double Fhm[2] = {a.fvx[v0 + lm], a.fvy[v0 + lm]};
    const double th0 = p.th0[gl];
    if (kind == kSoft) {
      lenh += 0.5 * (a.dsh[gl] + a.dsh[v0 + lp]);
      const double cx = 0.5 * (X[l] + X[lp]), cy = 0.5 * (Y[l] + Y[lp]);
      const double nxl = dy / len, nyl = -dx / len;
      // adhesion spring on a bonded ligand element
      double yl, ddx, ddy;
      if (bond_geometry(p, L, Bp, l, cx, cy, yl, ddx, ddy))
        adj::spring_vjp(dx, dy, yl, ddx, ddy, sigma, L.y_eq, Fex, Fey, Dhx, Dhy, Chx, Chy, sigh);
      double pfx, pfy, nhx = 0.0, nhy = 0.0;
      probe_adjoint(L, a, cx, cy, nxl, nyl, len, nu, Fex, Fey, pfx, pfy, Chx, Chy, nhx, nhy, lenh);
      // n = (t_y, -t_x)
      adj::unit_vjp(dx, dy, -nhy, nhx, 0.0, Dhx, Dhy);
    }
    adj::unit_vjp(dx, dy, 0.0, 0.0, lenh, Dhx, Dhy);
    a.Dx[gl] = Dhx;
    a.Dy[gl] = Dhy;
    a.Cx[gl] = Chx;
    a.Cy[gl] = Chy;
    // bending at vertex l
    const double Fhu[2] = {f0x, f0y};
    const double Fhp[2] = {f1x, f1y};
    double dLh[2] = {0.0, 0.0}, dRh[2] = {0.0, 0.0};
    adj::bend_vjp(dLx, dLy, dx, dy, th0, kb, Fhm, Fhu, Fhp, dLh, dRh, kbh);
    a.BLx[gl] = dLh[0];
    a.BLy[gl] = dLh[1];
    a.BRx[gl] = dRh[0];
    a.BRy[gl] = dRh[1];
  }
  double v4[4] = {ksh, kbh, sigh, kaph};
  block_sum<4>(v4, s_red);
  const double Ah = -v4[3] * ka * p_ref / A0;

  // ---- phase D (vertices): gather element terms into the adjoint of X^n
  for (int v = t; v < nv; v += nt) {
    const int gm = v0 + v;
    const int vp = v + 1 == nv ? 0 : v + 1, vm = v == 0 ? nv - 1 : v - 1;
    // element l = v-1 ends at v (+d^), element v starts at v (-d^)
    const double Dmx = a.Dx[v0 + vm] + a.BRx[v0 + vm] + a.BLx[gm];
    const double Dmy = a.Dy[v0 + vm] + a.BRy[v0 + vm] + a.BLy[gm];
    const double Dvx = a.Dx[gm] + a.BRx[gm] + a.BLx[v0 + vp];
    const double Dvy = a.Dy[gm] + a.BRy[gm] + a.BLy[v0 + vp];
    double xh = a.dirx[gm] + Dmx - Dvx + 0.5 * (a.Cx[gm] + a.Cx[v0 + vm]);
    double yh = a.diry[gm] + Dmy - Dvy + 0.5 * (a.Cy[gm] + a.Cy[v0 + vm]);
    xh += Ah * 0.5 * (Y[vp] - Y[vm]);
    yh += Ah * 0.5 * (X[vm] - X[vp]);
    a.xa[gm] = xh;
    a.ya[gm] = yh;
  }
  if (t == 0) {
    a.grad[3 * b + 0] += v4[0];
    a.grad[3 * b + 1] += v4[1];
    a.grad[3 * b + 2] += v4[2];
  }
}

// --------------------------------------------------------------- stream
// Reverse of the pull streaming: h^_j(y) = f^_j(y + e_j), or, where the pull
// bounced at a wall, f^_{opp(j)}(y).  f^ includes the pre-forcing moment
// terms of rho*, u*.
template <typename T>
__device__ inline void stream_adjoint(const Ptrs<T>& p, const AdjPtrs& a, long long node) {
  const LatDev L = p.lat[0];
  const long long N = L.plane;
  if (node >= N) return;
  const unsigned un = (unsigned)node, pitch = (unsigned)L.pitch;
  const int x = (int)(un % pitch), y = (int)(un / pitch);
  if (x >= L.nx) return;   // row padding
#pragma unroll
  for (int j = 0; j < kQ; ++j) {
    int xs = wrap_idx(x + ex(j), L.nx), ys = y + ey(j);
    int i = j;
    long long src;
    if ((ys < 0 || ys >= L.ny) && !L.periodic_y) {
      src = node;
      i = opp(j);
    } else {
      ys = wrap_idx(ys, L.ny);
      src = (long long)ys * L.pitch + xs;
    }
    const double rho = a.mom[src], us = a.mom[N + src], vs = a.mom[2 * N + src];
    const double rh = acc_get(a.Rh, src), uh = acc_get(a.Rh, N + src), vh = acc_get(a.Rh, 2 * N + src);
    const double ir = 1.0 / rho;
    const double r = rh - (uh * us + vh * vs) * ir;
    a.ha[j * N + node] = a.fph[i * N + src] + r + (ex(i) * uh + ey(i) * vh) * ir;
  }
}

// Four markers to a 64-lane workgroup, a row of 16 lanes each.
template <typename T>
__global__ void ka_marker(Ptrs<T> p, AdjPtrs a) {
  marker_adjoint(p, a, (int)blockIdx.x * 4 + (int)(threadIdx.x >> 4), (int)(threadIdx.x & 15));
}

template <typename T>
__global__ void ka_stream(Ptrs<T> p, AdjPtrs a) {
  stream_adjoint(p, a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// Reverse streaming of step s (workgroups [0, gn)) together with the marker
// kernel of step s - 1 (the rest): independent data, one launch.
template <typename T>
__global__ void ka_stream_marker(Ptrs<T> p, AdjPtrs as, AdjPtrs am, int gn) {
  const int b = blockIdx.x;
  if (b < gn) stream_adjoint(p, as, (long long)b * blockDim.x + threadIdx.x);
  else marker_adjoint(p, am, (b - gn) * 4 + (int)(threadIdx.x >> 4), (int)(threadIdx.x & 15));
}

// --------------------------------------------------------------- copies
// Several device-to-device copies in one launch, one row of the grid per
// copy: 16-byte words where both ends are 16-byte aligned, the remaining
// 4-byte words after them (sizes are whole 4-byte words).
__global__ void ka_copy(CopyList c) {
  const int r = blockIdx.y;
  if (r >= c.n) return;
  const unsigned long long n = c.bytes[r] >> 2;
  const unsigned long long k0 = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long st = (unsigned long long)gridDim.x * blockDim.x;
  unsigned long long done = 0;
  if ((((unsigned long long)c.src[r] | (unsigned long long)c.dst[r]) & 15) == 0) {
    const uint4* s = (const uint4*)c.src[r];
    uint4* d = (uint4*)c.dst[r];
    const unsigned long long n4 = n >> 2;
    for (unsigned long long k = k0; k < n4; k += st) d[k] = s[k];
    done = n4 << 2;
  }
  const unsigned* s = (const unsigned*)c.src[r];
  unsigned* d = (unsigned*)c.dst[r];
  for (unsigned long long k = done + k0; k < n; k += st) d[k] = s[k];
}

// Set the adjoint seed / clear accumulators: out[k] = v for k < n.
__global__ void ka_fill(double* out, long long n, double v) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    out[k] = v;
}

// ------------------------------------------------------------------ launchers
// Reverse sweep over the steps of a segment, last to first: the marker
// kernel of step s runs inside the previous launch (the reverse streaming of
// step s + 1), so a step costs three launches.
template <typename T>
void launch_adjoint_segment(const Ptrs<T>& p, const AdjPtrs* a, int n, long long N, hipStream_t s) {
  const int nm = p.nm_total;
  // one wave per workgroup (a small lattice still reaches every compute
  // unit); four markers to a workgroup
  constexpr int kNodeThreads = 64;
  const unsigned gn = (unsigned)((N + kNodeThreads - 1) / kNodeThreads), gm = (unsigned)((nm + 3) / 4);
  // FE, Uh (and Rh) start each step cleared: by the previous reverse step's
  // collide kernel, or by the fill before the first one
  if (nm > 0) hipLaunchKernelGGL(ka_marker<T>, dim3(gm), dim3(kNodeThreads), 0, s, p, a[n - 1]);
  for (int k = n - 1; k >= 0; --k) {
    hipLaunchKernelGGL(ka_collide<T>, dim3(gn), dim3(kNodeThreads), 0, s, p, a[k]);
    if (p.nbody_total > 0)
      hipLaunchKernelGGL(ka_body<T>, dim3(p.nbody_total), dim3(kAdjThreads), 0, s, p, a[k]);
    if (k > 0 && nm > 0)
      hipLaunchKernelGGL(ka_stream_marker<T>, dim3(gn + gm), dim3(kNodeThreads), 0, s, p, a[k], a[k - 1],
                         (int)gn);
    else
      hipLaunchKernelGGL(ka_stream<T>, dim3(gn), dim3(kNodeThreads), 0, s, p, a[k]);
  }
}

void launch_copies(const CopyList& c, hipStream_t s) {
  if (c.n <= 0) return;
  unsigned long long mx = 0;
  for (int r = 0; r < c.n; ++r) mx = std::max(mx, c.bytes[r] >> 4);
  const unsigned gx = (unsigned)std::min<unsigned long long>((mx + 255) / 256, 1024ull);
  hipLaunchKernelGGL(ka_copy, dim3(std::max(gx, 1u), c.n), dim3(256), 0, s, c);
}

void launch_fill(double* out, long long n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(ka_fill, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), 0,
                     s, out, n, v);
}

template void launch_adjoint_segment<float>(const Ptrs<float>&, const AdjPtrs*, int, long long, hipStream_t);
template void launch_adjoint_segment<double>(const Ptrs<double>&, const AdjPtrs*, int, long long, hipStream_t);

}  // namespace lbib
