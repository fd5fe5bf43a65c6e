// k_lagrangian.hip - Lagrangian side of the LB-IB step (gfx950), float64.
//
// Per time step n (the order is the one used throughout the library):
//   k_body        first one workgroup per lattice instance:
//                   - bond kinetics: rupture pass, then formation pass in
//                     ascending ligand order (Sec. 2.2 Wall-Particle Interaction),
//                     with Philox4x32-10 uniforms keyed by (step, ligand).
//                 then one workgroup per body:
//                   - membrane strain, bending and area forces (Eqs. strainFor,
//                     bendFor, areaFor), adhesion springs (Eq. adhFor);
//                   - particles: probe pressure/viscous loads (Eqs. hydroForP,
//                     hydroForNu) from the pre-forcing fluid state, soft Verlet
//                     position update (Eqs. newtonSoft, verletPos) or rigid BDF2
//                     (Eqs. linearVelRig, angularVelRig), weak-coupling force.
//   (the fused lattice kernel runs here)
//   k_advance     one lane per marker: red cells by the kinematic IB
//                 (Eq. kinematicPos), particles adopt their new positions;
//                 the stencil of the new position (centre node floor(X + 1/2)
//                 and the 3+3 weights of the Roma 3-point kernel) is stored
//                 and the marker joins the bins of every lattice tile that
//                 stencil overlaps, for the next step's fused kernel.
#include "lbib_dev.h"
#include "mls.h"

namespace lbib {

// ------------------------------------------------------------------ helpers
// Populations at a node after streaming, before forcing (walls: bounce-back).
template <typename T>
__device__ inline void pull_node(const T* A, long long N, int nx, int ny, int pitch, bool pery, int x,
                                 int y, T hv[kQ]) {
  const long long node = (long long)y * pitch + x;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    int xs = x - ex(i);
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    int ys = y - ey(i);
    const bool out = ys < 0 || ys >= ny;
    ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
    const long long src = (out && !pery) ? opp(i) * N + node : i * N + (long long)ys * pitch + xs;
    hv[i] = A[src];
  }
}

// Velocity walls: a wall node of the pre-forcing state takes the drive as its
// force (the step's IB forces are not known yet).
template <typename T>
__device__ __forceinline__ void wall_fill_drive(const LatDev& L, int y, T hv[kQ]) {
  if (L.wall_mode == 1 && !L.periodic_y && (y == 0 || y == L.ny - 1))
    zou_he_fill(hv, y == 0, T(y == 0 ? L.u_wall_lo : L.u_wall_hi), T(L.gx), T(L.gy));
}

template <typename T>
__device__ inline void pulled_moments(const T* A, const LatDev& L, long long N, int x, int y,
                                      double& drho, double& jx, double& jy) {
  drho = 0.0; jx = 0.0; jy = 0.0;
  T hv[kQ];
  pull_node(A, N, L.nx, L.ny, L.pitch, L.periodic_y != 0, x, y, hv);
  wall_fill_drive(L, y, hv);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const double h = double(hv[i]);
    drho += h;
    jx += ex(i) * h;
    jy += ey(i) * h;
  }
}

// rho*, u* of the pre-forcing state: u* = (sum f e + g/2) / rho*.
template <typename T>
__device__ inline void node_star(const T* A, const LatDev& L, int x, int y, double& rho,
                                 double& ux, double& uy) {
  const long long N = L.plane;
  double drho, jx, jy;
  pulled_moments(A, L, N, x, y, drho, jx, jy);
  rho = 1.0 + drho;
  ux = (jx + 0.5 * L.gx) / rho;
  uy = (jy + 0.5 * L.gy) / rho;
}

// MLS interpolant of rho*, u* at a point and (GRAD) its gradient (the MLS
// shape functions and their derivatives), from the node values fetch(x, row,
// rho, ux, uy) (x unwrapped; row wrapped on a periodic lattice, else
// clamped: a row beyond a wall has weight zero, so it reads the wall row,
// inside the lattice and any cache of the point's nodes).
template <bool GRAD, typename Fetch>
__device__ __forceinline__ void interp_mls(const LatDev& L, double X, double Y, Fetch fetch,
                                           double& rho, double& ux, double& uy, double g[4]) {
  double ph[9], px[9], py[9];
  mls_shape<GRAD>(L, X, Y, ph, px, py);
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  rho = 0; ux = 0; uy = 0;
  g[0] = g[1] = g[2] = g[3] = 0;
  const bool pery = L.periodic_y != 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    int row = (int)(cyr + (b - 1));
    row = pery ? row : min(max(row, 0), L.ny - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double r, u, v;
      fetch((int)(cxr + (a - 1)), row, r, u, v);
      const double w = ph[3 * b + a];
      rho += r * w;
      ux += u * w;
      uy += v * w;
      if (GRAD) {
        g[0] += u * px[3 * b + a];
        g[1] += u * py[3 * b + a];
        g[2] += v * px[3 * b + a];
        g[3] += v * py[3 * b + a];
      }
    }
  }
}

// Kernel (or, with MLS compiled in and selected, MLS) interpolant of rho*,
// u* at a point and (optionally) its gradient.  MLS = false compiles the
// kernel weights only: the latency-bound kernels of runs without the MLS
// transfer carry none of its code (their instruction fetches grow with the
// code they hold).
template <bool MLS, typename T>
__device__ inline void interp_star(const T* A, const LatDev& L, double X, double Y, bool grad,
                                   double& rho, double& ux, double& uy, double g[4]) {
  if (MLS && use_mls(L)) {
    auto fetch = [&](int xr, int row, double& r, double& u, double& v) {
      node_star(A, L, wrap_i(xr, L.nx), L.periodic_y ? wrap_i(row, L.ny) : row, r, u, v);
    };
    if (grad) interp_mls<true>(L, X, Y, fetch, rho, ux, uy, g);
    else interp_mls<false>(L, X, Y, fetch, rho, ux, uy, g);
    return;
  }
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  rho = 0; ux = 0; uy = 0;
  g[0] = g[1] = g[2] = g[3] = 0;  // du/dx, du/dy, dv/dx, dv/dy
  const bool pery = L.periodic_y != 0;
  double wxa[3], dwxa[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    wxa[a] = roma_phi((cxr + (a - 1)) - X);
    dwxa[a] = grad ? roma_dphi((cxr + (a - 1)) - X) : 0.0;
  }
  for (int b = 0; b < 3; ++b) {
    const double ry = cyr + (b - 1);
    int row = (int)ry;
    if (pery) row = wrap_i(row, L.ny);
    else if (row < 0 || row >= L.ny) continue;
    const double wy = roma_phi(ry - Y), dwy = grad ? roma_dphi(ry - Y) : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double rx = cxr + (a - 1);
      const int col = wrap_i((int)rx, L.nx);
      const double wx = wxa[a], dwx = dwxa[a];
      double r, u, v;
      node_star(A, L, col, row, r, u, v);
      rho += r * wx * wy;
      ux += u * wx * wy;
      uy += v * wx * wy;
      if (grad) {
        g[0] -= u * dwx * wy;
        g[1] -= u * wx * dwy;
        g[2] -= v * dwx * wy;
        g[3] -= v * wx * dwy;
      }
    }
  }
}

// rho*, u* of the nodes in a box [bx0, bx0 + bw) x [by0, by0 + bh) cached in
// LDS (x unwrapped; rows wrapped for a periodic lattice).  Same interpolant
// as interp_star, read from the cache.  The cache holds the density's
// deviation rho* - 1, not rho*: in float32, rho* itself (about 1 + 1e-4)
// would keep only the leading digits of the deviation that the probe
// pressure cs^2 (rho* - 1) is made of.
template <typename T>
struct StarCache {
  const T* c;   // 3 values per node: rho - 1, ux, uy
  int bx0, by0, bw, bh;
};

template <bool MLS, typename T>
__device__ inline void interp_cached(const StarCache<T>& C, const LatDev& L, double X, double Y,
                                     bool grad, double& rho, double& ux, double& uy, double g[4]) {
  if (MLS && use_mls(L)) {
    auto fetch = [&](int xr, int row, double& r, double& u, double& v) {
      const int k = 3 * ((row - C.by0) * C.bw + (xr - C.bx0));
      r = 1.0 + double(C.c[k]);
      u = double(C.c[k + 1]);
      v = double(C.c[k + 2]);
    };
    if (grad) interp_mls<true>(L, X, Y, fetch, rho, ux, uy, g);
    else interp_mls<false>(L, X, Y, fetch, rho, ux, uy, g);
    return;
  }
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  rho = 0; ux = 0; uy = 0;
  g[0] = g[1] = g[2] = g[3] = 0;
  const bool pery = L.periodic_y != 0;
  double wxa[3], dwxa[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    wxa[a] = roma_phi((cxr + (a - 1)) - X);
    dwxa[a] = grad ? roma_dphi((cxr + (a - 1)) - X) : 0.0;
  }
  for (int b = 0; b < 3; ++b) {
    const double ry = cyr + (b - 1);
    const int row = (int)ry;
    if (!pery && (row < 0 || row >= L.ny)) continue;
    const double wy = roma_phi(ry - Y), dwy = grad ? roma_dphi(ry - Y) : 0.0;
    const int kr = (row - C.by0) * C.bw;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double rx = cxr + (a - 1);
      const double wx = wxa[a], dwx = dwxa[a];
      const int k = 3 * (kr + ((int)rx - C.bx0));
      const double r = 1.0 + double(C.c[k]), u = double(C.c[k + 1]), v = double(C.c[k + 2]);
      rho += r * wx * wy;
      ux += u * wx * wy;
      uy += v * wx * wy;
      if (grad) {
        g[0] -= u * dwx * wy;
        g[1] -= u * wx * dwy;
        g[2] -= v * dwx * wy;
        g[3] -= v * wx * dwy;
      }
    }
  }
}

__device__ inline double wrap_x(double cx, int nx) { return cx - nx * floor(cx / nx); }

__device__ inline double min_image(double xr, double cxw, int nx) {
  double d = xr - cxw;
  if (d > 0.5 * nx) d -= nx;
  else if (d < -0.5 * nx) d += nx;
  return d;
}

// Bond length between element centroid c and receptor (xr, wall).
__device__ inline double bond_len(double cx, double cy, double xr, int wall, const LatDev& L) {
#pragma clang fp contract(off)
  const double dx = min_image(xr, wrap_x(cx, L.nx), L.nx);
  const double yw = wall == 0 ? L.y_wall_lo : L.y_wall_hi;
  const double dy = cy - yw;
  return sqrt(dx * dx + dy * dy);
}

// Block-wide exclusive scan of one int per thread (blockDim <= 1024).
__device__ inline int block_exclusive_scan(int v, int* s_tmp) {
  const int t = threadIdx.x, n = blockDim.x;
  s_tmp[t] = v;
  __syncthreads();
  for (int off = 1; off < n; off <<= 1) {
    int add = t >= off ? s_tmp[t - off] : 0;
    __syncthreads();
    s_tmp[t] += add;
    __syncthreads();
  }
  int incl = s_tmp[t];
  __syncthreads();
  return incl - v;
}

// ---------------------------------------------------------------- marker bins
// Register marker gm in every tile its 3x3 stencil overlaps (centre cx, cy).
// Three consecutive columns (rows) touch at most three tiles (a ragged last
// tile can be one column wide), so a marker joins at most nine bins.  Slots
// come from wave-aggregated atomics: a run of adjacent lanes that hit the
// same tile (neighbours along a membrane) shares one atomic.  A full bin drops the
// registration and counts it in *overflow (the fused kernel then poisons
// that tile's force so the watchdog reports it).
template <int TX, int TY, int R>
__device__ inline void register_markers(int* cnt, int* bin, int cap, int* overflow, const LatDev& L,
                                        const int* gm, const int* cx, const int* cy,
                                        const bool* active) {
  const bool pery = L.periodic_y != 0;
  const int nx = L.nx, ny = L.ny;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int key[R][9], leader[R][9], rank[R][9], gcount[R][9];
  unsigned used = 0;   // slots some lane of the wave uses (bit r * 9 + s9; wave-uniform)
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // tile column and row of each stencil offset; an offset whose tile an
    // earlier offset already reached adds no slot (fixed indices only, so
    // the lists stay in registers)
    int tc[3], tr[3];
    bool okc[3], okr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int c = cx[r] + a - 1;
      c = c < 0 ? c + nx : (c >= nx ? c - nx : c);
      tc[a] = c / TX;
      okc[a] = active[r];
      int rr = cy[r] + a - 1;
      bool ok = active[r];
      if (pery) rr = rr < 0 ? rr + ny : (rr >= ny ? rr - ny : rr);
      else ok = ok && rr >= 0 && rr < ny;
      tr[a] = ok ? rr / TY : -1;
      okr[a] = ok;
    }
    bool vc[3], vr[3];
    vc[0] = okc[0];
    vc[1] = okc[1] && tc[1] != tc[0];
    vc[2] = okc[2] && tc[2] != tc[0] && tc[2] != tc[1];
    vr[0] = okr[0];
    vr[1] = okr[1] && !(okr[0] && tr[1] == tr[0]);
    vr[2] = okr[2] && !(okr[0] && tr[2] == tr[0]) && !(okr[1] && tr[2] == tr[1]);
    // 1. group the lanes of every slot by tile, no memory traffic: a run of
    //    adjacent lanes with the same tile (neighbouring markers) is one
    //    group; a tile met in several runs gets one group per run
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9) {
      const int i = s9 / 3, j = s9 % 3;
      const bool has = vr[i] && vc[j];
      const int k = has ? L.tile_base + tr[i] * L.ntx + tc[j] : -1;
      key[r][s9] = k;
      leader[r][s9] = lane;
      rank[r][s9] = 0;
      gcount[r][s9] = 0;
      const unsigned long long hasm = __ballot(has);
      if (hasm == 0ull) continue;
      used |= 1u << (r * 9 + s9);
      const int kprev = __shfl_up(k, 1);
      const unsigned long long heads = __ballot(has && (lane == 0 || kprev != k));
      const unsigned long long le = lt | (1ull << lane);
      const unsigned long long mine = heads & le;
      const int ld = mine ? 63 - __clzll((long long)mine) : lane;
      leader[r][s9] = ld;
      rank[r][s9] = lane - ld;
      const unsigned long long brk = (heads | ~hasm) & ~le;   // lanes after this one that end the run
      const int next = brk ? __ffsll((long long)brk) - 1 : 64;
      gcount[r][s9] = has && lane == ld ? next - lane : 0;
    }
  }
  // 2. every group leader reserves its slots; the atomics of all markers,
  //    groups and slots are in flight together
  int base[R][9];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9)
      base[r][s9] = (used >> (r * 9 + s9) & 1u) && gcount[r][s9] > 0
                        ? atomicAdd(&cnt[key[r][s9]], gcount[r][s9]) : 0;
  // 3. positions and stores
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9) {
      if (!(used >> (r * 9 + s9) & 1u)) continue;
      const int b = __shfl(base[r][s9], leader[r][s9]);
      if (key[r][s9] >= 0) {
        const int pos = b + rank[r][s9];
        if (pos < cap) bin[(long long)key[r][s9] * cap + pos] = gm[r];
        else atomicAdd(overflow, 1);
      }
    }
}

// One marker per lane.
template <int TX, int TY>
__device__ inline void register_marker(int* cnt, int* bin, int cap, int* overflow, const LatDev& L,
                                       int gm, int cx, int cy, bool active) {
  register_markers<TX, TY, 1>(cnt, bin, cap, overflow, L, &gm, &cx, &cy, &active);
}

// ---------------------------------------------------------------- stencils
// Stencil of a marker at (X, Y): centre node floor(X + 1/2) (column wrapped,
// row wrapped on a periodic lattice, else kept raw so rows beyond the walls
// can be recognised) and the weights of its 3x3 nodes: the Roma kernel
// along each axis (zero for rows beyond the walls), or the MLS shape
// functions.
template <bool MLS = true, typename T>
__device__ inline void marker_stencil(const Ptrs<T>& p, const LatDev& L, int gm, double X, double Y,
                                      int& ocx, int& ocy) {
  const int nm = p.nm_total;
  const bool pery = L.periodic_y != 0;
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  if (MLS && use_mls(L)) {
    double ph[9];
    mls_shape<false>(L, X, Y, ph, nullptr, nullptr);
#pragma unroll
    for (int k = 0; k < 9; ++k) p.wx[k * nm + gm] = ph[k];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p.wx[a * nm + gm] = roma_phi((cxr + (a - 1)) - X);
      const double ry = cyr + (a - 1);
      const bool valid = pery || (ry >= 0.0 && ry < (double)L.ny);
      p.wy[a * nm + gm] = valid ? roma_phi(ry - Y) : 0.0;
    }
  }
  ocx = wrap_i((int)cxr, L.nx);
  ocy = pery ? wrap_i((int)cyr, L.ny) : (int)fmin(fmax(cyr, -4.0), (double)(L.ny + 3));
  p.cx[gm] = ocx;
  p.cy[gm] = ocy;
}

// Stencils of all markers from their current positions (after set-up or
// after positions were overwritten from the host).
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_stencil(Ptrs<T> p) {
  const int gm = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = gm < p.nm_total;
  const int g = active ? gm : 0;
  const LatDev& L = p.lat[p.minfo[g] >> 2];
  int cx = 0, cy = 0;
  if (active) marker_stencil(p, L, gm, p.x[gm], p.y[gm], cx, cy);
  register_marker<TX, TY>(p.cnt_cur, p.bin_cur, p.bin_cap, p.overflow, L, gm, cx, cy, active);
}

// LDS cache of rho*, u* per particle: sized by the host from the particles'
// extent (between 16 KB and 96 KB; the body kernel's static LDS is ~41 KB)

// ---------------------------------------------------------------- advance
// Kinematic IB update of a red-cell vertex (Eq. kinematicPos): the velocity
// of the step, interpolated at X^n with the stencil stored for X^n, then
// BDF2 (forward Euler on the first step).
// Split in two so that a lane handling several vertices issues every load
// of all of them before it waits: first the stencil and X^{n-1} (needed by
// BDF2 only, loaded unconditionally), then the velocity gather.
// MLS = false: the Roma kernel's per-axis weights (the layout the kernels
// without MLS keep: a wider one costs them register spills); MLS = true: nine
// slots, the Roma weights in 0..5 (wx then wy) or the nine MLS weights.
template <bool MLS> struct RbcAdv;
template <> struct RbcAdv<false> {
  int cx, cy;
  double wx[3], wy[3];
  double xm, ym;
};
template <> struct RbcAdv<true> {
  int cx, cy;
  double ph[9];
  double xm, ym;
};

template <bool MLS, typename T>
__device__ inline void rbc_adv_load(const Ptrs<T>& p, const LatDev& L, int gm, RbcAdv<MLS>& a) {
  const int nm = p.nm_total;
  a.cx = p.cx[gm];
  a.cy = p.cy[gm];
  if constexpr (MLS) {
    // one load per slot from the array the transfer uses (fixed slots, no
    // branch around the writes, so the struct stays in registers)
    const bool mls = use_mls(L);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double* src = (mls || k < 3) ? p.wx + k * nm : p.wy + (k - 3) * nm;
      a.ph[k] = src[gm];
    }
#pragma unroll
    for (int k = 6; k < 9; ++k) a.ph[k] = mls ? p.wx[k * nm + gm] : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.wx[k] = p.wx[k * nm + gm];
      a.wy[k] = p.wy[k * nm + gm];
    }
  }
  a.xm = p.xm[gm];
  a.ym = p.ym[gm];
}

template <bool MLS, typename T>
__device__ inline void rbc_adv_finish(const Ptrs<T>& p, const LatDev& L, const RbcAdv<MLS>& in, double X,
                                      double Y, bool first, double& xn, double& yn) {
  const long long N = L.plane;
  const T* U = p.U + 2 * L.node_base;
  const int cx = in.cx, cy = in.cy;
  double ux = 0.0, uy = 0.0;
  // a row beyond a wall has weight exactly zero: it reads a clamped row and
  // adds zeros, so all 18 loads are independent of control flow
#pragma unroll
  for (int b2 = 0; b2 < 3; ++b2) {
    int row = cy + b2 - 1;
    if (L.periodic_y) row = wrap_i(row, L.ny);
    else row = min(max(row, 0), L.ny - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int col = wrap_i(cx + a - 1, L.nx);
      double w;
      if constexpr (MLS) w = use_mls(L) ? in.ph[3 * b2 + a] : in.ph[a] * in.ph[3 + b2];
      else w = in.wx[a] * in.wy[b2];
      const long long node = (long long)row * L.pitch + col;
      ux += double(U[node]) * w;
      uy += double(U[N + node]) * w;
    }
  }
  if (first) {
    xn = X + ux;
    yn = Y + uy;
  } else {
    xn = (2.0 / 3.0) * (2.0 * X - 0.5 * in.xm + ux);
    yn = (2.0 / 3.0) * (2.0 * Y - 0.5 * in.ym + uy);
  }
}

template <bool MLS, typename T>
__device__ inline void advance_rbc(const Ptrs<T>& p, const LatDev& L, int gm, double X, double Y,
                                   bool first, double& xn, double& yn) {
  RbcAdv<MLS> a;
  rbc_adv_load<MLS>(p, L, gm, a);
  rbc_adv_finish<MLS>(p, L, a, X, Y, first, xn, yn);
}

// ---------------------------------------------------------------- k_bonds
template <typename T>
__device__ __forceinline__ void bonds_kinetics(Ptrs<T>& p, const LatDev& L, int inst, long long n,
                                               int nx, int ny, int* s_tmp, int& s_nelig) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // bond kinetics (Sec. 2.2): rupture then formation
  if (L.n_lig == 0 || L.freeze) return;
  __syncthreads();
  if (tid == 0) s_nelig = 0;
  __syncthreads();
  const double y_cr = L.y_cr;
  unsigned long long ties = 0;
  // (a) rupture (independent per bond) and formation eligibility
  for (int l0 = 0; l0 < L.n_lig; l0 += nt) {
    const int l = l0 + tid;
    int flag = 0;
    if (l < L.n_lig) {
      const int gl = L.lig_base + l;
      const int va = p.lig_va[gl], vb = p.lig_vb[gl];
      // particle positions X^n: xn (equal to x once a step has ended; while
      // the merged step kernel runs, its particle workgroups copy xn into x)
      const double cx = 0.5 * (p.xn[va] + p.xn[vb]);
      const double cy = 0.5 * (p.yn[va] + p.yn[vb]);
      const int r = p.l2r[gl];
      if (r >= 0) {
        const int wall = r < L.n_rec0 ? 0 : 1;
        const double yl = bond_len(cx, cy, p.rec_x[L.rec_base + r], wall, L);
        const double sig = p.lig_sigma[gl], sts = L.sigma_ts_frac * sig;
        const double dy = yl - L.y_eq;
        const double kr = L.kr0_dt * exp((sig - sts) * dy * dy / (2.0 * L.kbt));
        const double P = 1.0 - exp(-kr);
        const double u = philox_uniform(L.seed, n, l, 1, L.instance);
        ties += fabs(u - P) < 1e-12;
        if (u < P) {
          p.l2r[gl] = -1;
          p.r2l[L.rec_base + r] = -1;
        }
      } else {
        const double d0 = cy - L.y_wall_lo, d1 = L.y_wall_hi - cy;
        const int wall = d0 <= d1 ? 0 : 1;
        const double d = wall == 0 ? d0 : d1;
        if (d < y_cr) flag = 1 + wall;
      }
    }
    // ordered compaction of eligible ligands (ascending ligand id)
    const int pos = block_exclusive_scan(flag ? 1 : 0, s_tmp);
    const int base = s_nelig;
    if (flag) p.lig_flag[L.lig_base + base + pos] = (l << 1) | (flag - 1);
    __syncthreads();
    if (tid == nt - 1) s_nelig = base + pos + (flag ? 1 : 0);
    __syncthreads();
  }
  // (b) formation, sequential over the eligible ligands in ascending order
  if (tid == 0) {
    const int ne = s_nelig;
    for (int q = 0; q < ne; ++q) {
      const int code = p.lig_flag[L.lig_base + q];
      const int l = code >> 1, wall = code & 1;
      const int gl = L.lig_base + l;
      const int va = p.lig_va[gl], vb = p.lig_vb[gl];
      const double cx = 0.5 * (p.xn[va] + p.xn[vb]);
      const double cy = 0.5 * (p.yn[va] + p.yn[vb]);
      const int nr = wall == 0 ? L.n_rec0 : L.n_rec1;
      if (nr == 0) continue;
      const int roff = wall == 0 ? 0 : L.n_rec0;
      const double* xs = p.rec_x + L.rec_base + roff;
      const int* taken = p.r2l + L.rec_base + roff;
      const double cxw = wrap_x(cx, nx);
      // first receptor at or right of cxw (receptors strictly increasing)
      int lo = 0, hi = nr;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (xs[mid] < cxw) lo = mid + 1; else hi = mid;
      }
      // merge the rightward and leftward sequences by their own distances;
      // each receptor is met first at its minimum-image distance
      int ir = lo % nr, il = (lo - 1 + nr) % nr;
      int best = -1;
      for (int it = 0; it < 2 * nr && best < 0; ++it) {
        double dr = xs[ir] - cxw;
        if (dr < 0) dr += nx;
        double dl = cxw - xs[il];
        if (dl < 0) dl += nx;
        // oracle's minimum image: equal to the smaller of the two one-sided
        // distances; ties between the two sides go to the lower index
        bool take_r = dr < dl || (dr == dl && ir <= il);
        int cand = take_r ? ir : il;
        if (taken[cand] < 0) {
          best = cand;
        } else if (take_r) {
          ir = (ir + 1) % nr;
        } else {
          il = (il - 1 + nr) % nr;
        }
      }
      if (best < 0) continue;
      const double yl = bond_len(cx, cy, xs[best], wall, L);
      const double sig = p.lig_sigma[gl], sts = L.sigma_ts_frac * sig;
      const double dy = yl - L.y_eq;
      const double kf = L.kf0_dt * exp(-sts * dy * dy / (2.0 * L.kbt));
      const double P = 1.0 - exp(-kf);
      const double u = philox_uniform(L.seed, n, l, 0, L.instance);
      ties += fabs(u - P) < 1e-12;
      if (u < P) {
        p.l2r[gl] = roff + best;
        p.r2l[L.rec_base + roff + best] = gl;
      }
    }
  }
  if (ties) atomicAdd(&p.ties[inst], ties);
}

// Step bookkeeping and bond kinetics of one lattice instance (the first
// workgroups of the body kernel).  Ends by raising the instance's flag that
// particle workgroups wait for before they read the bond table.
template <typename T>
__device__ __forceinline__ void bonds_impl(Ptrs<T>& p, int inst, int* s_tmp, int* s_nelig_p) {
  int& s_nelig = *s_nelig_p;
  const LatDev& L = p.lat[inst];
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long n = p.step_next[inst];
  __syncthreads();
  if (tid == 0) {
    p.step_cur[inst] = n;
    p.step_next[inst] = n + 1;
    p.step_slot[inst] = n;
  }
  if (inst == 0 && tid == 0) {
    // the other slot was last used by the previous step, whose kernels have
    // all finished: clear it for the next step
    for (int i = 0; i < p.ninst; ++i) {
      p.fmax_next[i] = 0ull;
      p.bond_flag_next[i] = 0;
    }
  }
  const int ny = L.ny, nx = L.nx;
  bonds_kinetics(p, L, inst, n, nx, ny, s_tmp, s_nelig);
  // publish: every lane's writes, then the flag
  __threadfence();
  __syncthreads();
  if (tid == 0) __hip_atomic_store(&p.bond_flag[inst], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}



// ---------------------------------------------------------------- k_body
// Block reduction (fixed tree order) of NV values per thread slot.
// Block sum of NV values per lane in a fixed order (butterfly inside each
// wave, then the wave sums in wave order): deterministic.
constexpr int kBodyThreads = 256;
constexpr int kSpinMax = 1 << 22;   // bounded wait for the bond flag (~0.2 s)
template <int NV>
__device__ inline void block_sum(double (*s)[kBodyThreads / 64], double* v) {
  const int t = threadIdx.x, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((t & 63) == 0) s[k][t >> 6] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = 0.0;
    for (int w = 0; w < nw; ++w) x += s[k][w];
    v[k] = x;
  }
  __syncthreads();
}

// max that propagates NaN (fmax drops it)
__device__ inline double fmax_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// Largest |F| a body hands to the fluid, folded into the instance maximum
// (non-negative doubles order like their bit patterns; NaN and Inf sort above
// every finite value, so a broken force shows up as a non-finite maximum).
__device__ inline void record_fmax(unsigned long long* slot, double m, double (*s)[kBodyThreads / 64]) {
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_xor(m, o);
    m = (other > m || other != other) ? other : m;
  }
  if ((threadIdx.x & 63) == 0 && m != 0.0) atomicMax(slot, (unsigned long long)__double_as_longlong(m));
}

constexpr int kVmax = kSmallBody;

// SMALL: the body's per-vertex scratch lives in LDS (sm); otherwise in the
// workspace.  A template parameter, so every access has a known address space.
template <typename T, bool SMALL, int TX, int TY, bool ADV, bool MLS>
__device__ __forceinline__ void body_impl(Ptrs<T>& p, int b, int cache_nodes, double (*sm)[kVmax],
                                          double (*s_red)[kBodyThreads / 64], double* s_rigid, int* s_box,
                                          unsigned char* s_dyn, double (*s_uv)[kBodyThreads / 2]) {
  BodyDev* Bp = p.body + b;
  const int kind = Bp->kind, nv = Bp->nv, v0 = Bp->v0, inst = Bp->inst;
  const double ks = Bp->ks, kb = Bp->kb, ka = Bp->ka, p_ref = Bp->p_ref, A0 = Bp->A0;
  const double mv = Bp->mv, sigma = Bp->sigma;
  const int lig_stride = Bp->lig_stride, lig_base = Bp->lig_base;
  const LatDev& L = p.lat[inst];
  const int t = threadIdx.x, nt = kBodyThreads;   // the launch's block size
  const T* A = p.A + 9 * L.node_base;
  const double nu = (L.tau - 0.5) / 3.0;
  const bool pery = L.periodic_y != 0;
  // rest data of this lane's vertices (a small body has at most kPre per
  // lane), requested now so that the loads are in flight during the work
  // before their use
  constexpr int kPre = (kVmax + kBodyThreads - 1) / kBodyThreads;
  double pre_th0[kPre], pre_l0[kPre], pre_l0m[kPre], pre_rep[kPre];
  // vertex repulsion (Eq. repFor): summed magnitudes from the repulsion
  // kernel, which runs before this one (never in the merged form)
  const bool rep = !ADV && L.rep_coeff > 0.0;
  if constexpr (SMALL) {
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int v = t + j * nt < nv ? t + j * nt : 0;
      const int vm = v == 0 ? nv - 1 : v - 1;
      const bool soft = kind != kRigid;
      pre_th0[j] = soft ? p.th0[v0 + v] : 0.0;
      pre_l0[j] = soft ? p.l0[v0 + v] : 0.0;
      pre_l0m[j] = soft ? p.l0[v0 + vm] : 0.0;
      pre_rep[j] = rep ? p.frep[v0 + v] : 0.0;
    }
  }
  // per-vertex scratch: LDS for small bodies, workspace otherwise
  const double* X = SMALL ? sm[0] : p.x + v0;
  const double* Y = SMALL ? sm[1] : p.y + v0;
  double* S_len = SMALL ? sm[2] : p.s_len + v0;
  double* S_nx = SMALL ? sm[3] : p.s_nx + v0;
  double* S_ny = SMALL ? sm[4] : p.s_ny + v0;
  double* S_bc = SMALL ? sm[5] : p.s_bc + v0;
  double* S_bnx = SMALL ? sm[6] : p.s_bnx + v0;
  double* S_bny = SMALL ? sm[7] : p.s_bny + v0;
  double* S_fex = SMALL ? sm[8] : p.s_fex + v0;
  double* S_fey = SMALL ? sm[9] : p.s_fey + v0;
  // ---- end of the previous step (merged form) for this body's vertices:
  // X^n from the kinematic update (red cells) or the particle dynamics,
  // stencils, and the bins of this step's fused kernel; two vertices per
  // lane, their loads and bin reservations in flight together.  Particles
  // also take the bounding box of X^n for their LDS cache from here.
  int mnx = 0x7fffffff, mxx = -0x7fffffff, mny = 0x7fffffff, mxy = -0x7fffffff;
  if (ADV) {
    const bool first_prev = p.step_prev[inst] == 0;
    constexpr int R = 2;
    for (int base0 = 0; base0 < nv; base0 += R * nt) {
      int gmv[R], ncx[R], ncy[R];
      bool act[R];
      double xo[R], yo[R], xn[R], yn[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int v = base0 + r * nt + t;
        act[r] = v < nv;
        gmv[r] = v0 + (act[r] ? v : 0);
        xo[r] = p.x[gmv[r]];
        yo[r] = p.y[gmv[r]];
      }
      if (kind == kRBC) {
        RbcAdv<MLS> ra[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rbc_adv_load<MLS>(p, L, gmv[r], ra[r]);
#pragma unroll
        for (int r = 0; r < R; ++r)
          rbc_adv_finish<MLS>(p, L, ra[r], xo[r], yo[r], first_prev, xn[r], yn[r]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          xn[r] = p.xn[gmv[r]];
          yn[r] = p.yn[gmv[r]];
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        ncx[r] = 0;
        ncy[r] = 0;
        if (act[r]) {
          p.xm[gmv[r]] = xo[r];
          p.ym[gmv[r]] = yo[r];
          p.x[gmv[r]] = xn[r];
          p.y[gmv[r]] = yn[r];
          if constexpr (SMALL) {
            sm[0][base0 + r * nt + t] = xn[r];
            sm[1][base0 + r * nt + t] = yn[r];
          }
          marker_stencil<MLS>(p, L, gmv[r], xn[r], yn[r], ncx[r], ncy[r]);
          if (kind != kRBC) {
            mnx = min(mnx, (int)floor(xn[r]) - 4); mxx = max(mxx, (int)ceil(xn[r]) + 4);
            mny = min(mny, (int)floor(yn[r]) - 4); mxy = max(mxy, (int)ceil(yn[r]) + 4);
          }
        }
      }
      register_markers<TX, TY, R>(p.cnt_cur, p.bin_cur, p.bin_cap, p.overflow, L, gmv, ncx, ncy, act);
    }
  }

  // ---- particles: LDS cache of rho*, u* over the box of nodes their vertex
  // and probe stencils can reach: the vertex bounding box of X^n widened by
  // 4 nodes (probe 1.2 along the normal, stencil reach 1.5, one node of
  // margin).  Boxes larger than the cache fall back to direct evaluation.
  bool cached = false;
  StarCache<T> C{(const T*)s_dyn, 0, 0, 0, 0};
  if (kind != kRBC) {
    if (!ADV) {
      for (int v = t; v < nv; v += nt) {
        const double xv = p.x[v0 + v], yv = p.y[v0 + v];
        mnx = min(mnx, (int)floor(xv) - 4); mxx = max(mxx, (int)ceil(xv) + 4);
        mny = min(mny, (int)floor(yv) - 4); mxy = max(mxy, (int)ceil(yv) + 4);
      }
    }
    // wave reductions first: only one lane per wave touches the LDS words
    for (int o = 32; o > 0; o >>= 1) {
      mnx = min(mnx, __shfl_xor(mnx, o)); mxx = max(mxx, __shfl_xor(mxx, o));
      mny = min(mny, __shfl_xor(mny, o)); mxy = max(mxy, __shfl_xor(mxy, o));
    }
    if (t == 0) { s_box[0] = 0x7fffffff; s_box[1] = -0x7fffffff; s_box[2] = 0x7fffffff; s_box[3] = -0x7fffffff; }
    __syncthreads();
    if ((t & 63) == 0) {
      atomicMin(&s_box[0], mnx); atomicMax(&s_box[1], mxx);
      atomicMin(&s_box[2], mny); atomicMax(&s_box[3], mxy);
    }
    __syncthreads();
    int by0 = s_box[2], by1 = s_box[3];
    if (!pery) { by0 = max(by0, 0); by1 = min(by1, L.ny - 1); }
    const int bw = s_box[1] - s_box[0] + 1, bh = by1 - by0 + 1;
    if (bw > 0 && bh > 0 && (long long)bw * bh <= cache_nodes) {
      cached = true;
      C.bx0 = s_box[0]; C.by0 = by0; C.bw = bw; C.bh = bh;
      const int nbox = bw * bh;
      const long long Nn = L.plane;
      T* cw = (T*)s_dyn;
      constexpr int NB = 4;   // nodes per lane per batch: 36 loads in flight
      T hv[NB][kQ];
      for (int k0 = 0; k0 < nbox; k0 += NB * nt) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const int k = k0 + q * nt + t;
          const int kk = k < nbox ? k : 0;
          const int col = wrap_i(C.bx0 + kk % bw, L.nx);
          int row = by0 + kk / bw;
          if (pery) row = wrap_i(row, L.ny);
          pull_node(A, Nn, L.nx, L.ny, L.pitch, pery, col, row, hv[q]);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const int k = k0 + q * nt + t;
          if (k >= nbox) continue;
          if (L.wall_mode == 1) {   // velocity walls: wall rows take the drive as force
            int row = by0 + k / bw;
            if (pery) row = wrap_i(row, L.ny);
            wall_fill_drive(L, row, hv[q]);
          }
          double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
          for (int i = 0; i < kQ; ++i) {
            const double h = double(hv[q][i]);
            drho += h;
            jx += ex(i) * h;
            jy += ey(i) * h;
          }
          const double r = 1.0 + drho;
          cw[3 * k] = T(drho);
          cw[3 * k + 1] = T((jx + 0.5 * L.gx) / r);
          cw[3 * k + 2] = T((jy + 0.5 * L.gy) / r);
        }
      }
    }
  }
  __syncthreads();   // positions, stencils and cache visible to the workgroup

  if (SMALL && !ADV) {
    // (the merged form wrote X^n into LDS as it computed it)
    for (int v = t; v < nv; v += nt) {
      sm[0][v] = p.x[v0 + v];
      sm[1][v] = p.y[v0 + v];
    }
    __syncthreads();
  }

  // pass 1: element geometry (element v joins v -> v+1), bending data, area
  double shoe = 0.0;
  auto pass1 = [&](int v, double th0v) {
    const int vp = v + 1 == nv ? 0 : v + 1, vm = v == 0 ? nv - 1 : v - 1;
    const double xv = X[v], yv = Y[v], xp = X[vp], yp = Y[vp], xm = X[vm], ym = Y[vm];
    const double dxr = xp - xv, dyr = yp - yv;
    const double lr = sqrt(dxr * dxr + dyr * dyr);
    const double txr = dxr / lr, tyr = dyr / lr;
    const double dxl = xv - xm, dyl = yv - ym;
    const double ll = sqrt(dxl * dxl + dyl * dyl);
    const double txl = dxl / ll, tyl = dyl / ll;
    S_len[v] = lr;
    S_nx[v] = tyr;
    S_ny[v] = -txr;
    if (kind != kRigid || rep) {
      // vertex normal (bending; also the direction of the repulsion)
      const double nsx = tyl + tyr, nsy = -txl - txr;
      const double nn = sqrt(nsx * nsx + nsy * nsy);
      S_bnx[v] = nsx / nn;
      S_bny[v] = nsy / nn;
    }
    if (kind != kRigid) {
      const double cr = txl * tyr - tyl * txr;
      const double dt = txl * txr + tyl * tyr;
      const double th = atan2(cr, dt);
      S_bc[v] = kb * (th - th0v);
    }
    shoe += xv * yp - xp * yv;
  };
  if constexpr (SMALL) {
#pragma unroll
    for (int j = 0; j < kPre; ++j)
      if (t + j * nt < nv) pass1(t + j * nt, pre_th0[j]);
  } else {
    for (int v = t; v < nv; v += nt) pass1(v, p.th0[v0 + v]);
  }
  double area = shoe;
  block_sum<1>(s_red, &area);   // its barriers also publish the scratch
  area *= 0.5;

  // particles read the bond table (and rigid ones the step counter) written
  // by this instance's bond workgroup: wait for its flag (bounded spin; the
  // bond workgroups have the lowest ids, so they are always dispatched)
  bool first = false;
  if (kind != kRBC) {
    if (t == 0) {
      int it = 0;
      while (__hip_atomic_load(&p.bond_flag[inst], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
             it < kSpinMax) {
        __builtin_amdgcn_s_sleep(2);
        ++it;
      }
      if (it == kSpinMax) atomicAdd(p.spin_timeouts, 1);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    first = p.step_cur[inst] == 0;
  }

  // A particle of at most nt/2 vertices: the upper half of the lanes (other
  // waves, so other SIMDs) interpolates the fluid velocity at the vertices
  // while the lower half runs the probes, instead of after the particle's
  // update; the values are the same, read back from LDS.
  const bool vel_early = SMALL && kind != kRBC && nv <= nt / 2;
  if (vel_early && t >= nt / 2 && t - nt / 2 < nv) {
    const int v = t - nt / 2;
    double rho, ux, uy, g[4];
    if (cached) interp_cached<MLS>(C, L, X[v], Y[v], false, rho, ux, uy, g);
    else interp_star<MLS>(A, L, X[v], Y[v], false, rho, ux, uy, g);
    s_uv[0][v] = ux;
    s_uv[1][v] = uy;
  }
  // pass 2: element loads (area penalty, adhesion springs, probe stresses)
  for (int l = t; l < nv; l += nt) {
    const int lp = l + 1 == nv ? 0 : l + 1;
    const double len = S_len[l], nxl = S_nx[l], nyl = S_ny[l];
    double fex = 0.0, fey = 0.0;
    if (kind != kRigid) {
      const double c = ka * (1.0 - area / A0) * p_ref * len;
      fex += c * nxl;
      fey += c * nyl;
    }
    if (kind != kRBC) {
      const double cx = 0.5 * (X[l] + X[lp]), cy = 0.5 * (Y[l] + Y[lp]);
      // adhesion spring on a bonded ligand element
      if (lig_stride > 0 && l % lig_stride == 0) {
        const int gl = lig_base + l / lig_stride;
        const int r = p.l2r[gl];
        if (r >= 0) {
          const int wall = r < L.n_rec0 ? 0 : 1;
          const double yl = bond_len(cx, cy, p.rec_x[L.rec_base + r], wall, L);
          const double sp = sigma * (yl - L.y_eq);
          fex += sp * nxl;
          fey += sp * nyl;
        }
      }
      // probe 1.2 dx along the outward normal, kept inside the fluid
      const double qx = cx + 1.2 * nxl;
      double qy = cy + 1.2 * nyl;
      if (!pery) qy = fmin(fmax(qy, 0.5), L.ny - 1.5);
      double rho, ux, uy, g[4];
      if (cached) interp_cached<MLS>(C, L, qx, qy, true, rho, ux, uy, g);
      else interp_star<MLS>(A, L, qx, qy, true, rho, ux, uy, g);
      const double pr = (rho - 1.0) * (1.0 / 3.0);
      const double txx = 2.0 * nu * g[0], tyy = 2.0 * nu * g[3], txy = nu * (g[1] + g[2]);
      fex += (-pr * nxl + txx * nxl + txy * nyl) * len;
      fey += (-pr * nyl + txy * nxl + tyy * nyl) * len;
    }
    S_fex[l] = fex;
    S_fey[l] = fey;
  }
  __syncthreads();

  if (kind == kRigid) {
    const double xc0 = Bp->xc, yc0 = Bp->yc;
    double r3[3] = {0.0, 0.0, 0.0};
    auto rigid_sum = [&](int l, double sv) {
      const int lp = l + 1 == nv ? 0 : l + 1;
      const double fex = S_fex[l], fey = S_fey[l];
      const double cx = 0.5 * (X[l] + X[lp]) - xc0, cy = 0.5 * (Y[l] + Y[lp]) - yc0;
      r3[0] += fex;
      r3[1] += fey;
      r3[2] += cx * fey - cy * fex;
      if (rep) {
        // repulsion at vertex l, along its inward normal; lever X_l - X_c
        const double frx = -sv * S_bnx[l], fry = -sv * S_bny[l];
        r3[0] += frx;
        r3[1] += fry;
        r3[2] += (X[l] - xc0) * fry - (Y[l] - yc0) * frx;
        p.frep[v0 + l] = 0.0;   // applied: the next step's repulsion kernel rewrites it
      }
    };
    if constexpr (SMALL) {
#pragma unroll
      for (int j = 0; j < kPre; ++j)
        if (t + j * nt < nv) rigid_sum(t + j * nt, pre_rep[j]);
    } else {
      for (int l = t; l < nv; l += nt) rigid_sum(l, rep ? p.frep[v0 + l] : 0.0);
    }
    block_sum<3>(s_red, r3);
    if (t == 0) {
      double U[2], Om;
      for (int k = 0; k < 2; ++k) {
        const double a = r3[k] / Bp->mass;
        U[k] = first ? Bp->U[k] + a : (2.0 / 3.0) * (2.0 * Bp->U[k] - 0.5 * Bp->Um[k] + a);
      }
      const double al = r3[2] / Bp->inertia;
      Om = first ? Bp->Om + al : (2.0 / 3.0) * (2.0 * Bp->Om - 0.5 * Bp->Omm + al);
      Bp->Um[0] = Bp->U[0]; Bp->Um[1] = Bp->U[1];
      Bp->U[0] = U[0]; Bp->U[1] = U[1];
      Bp->Omm = Bp->Om; Bp->Om = Om;
      const double xc = xc0 + U[0], yc = yc0 + U[1], th = Bp->theta + Om;
      Bp->xc = xc; Bp->yc = yc; Bp->theta = th;
      s_rigid[0] = U[0]; s_rigid[1] = U[1]; s_rigid[2] = Om;
      s_rigid[3] = xc; s_rigid[4] = yc; s_rigid[5] = th;
    }
    __syncthreads();
    double fm = 0.0;
    const double U0 = s_rigid[0], U1 = s_rigid[1], Om = s_rigid[2];
    const double xc = s_rigid[3], yc = s_rigid[4], th = s_rigid[5];
    const double c = cos(th), sn = sin(th);
    for (int v = t; v < nv; v += nt) {
      const int gm = v0 + v, vm = v == 0 ? nv - 1 : v - 1;
      const double rx = p.r0x[gm], ry = p.r0y[gm];
      const double xn = xc + (rx * c + ry * (-sn));
      const double yn = yc + (rx * sn + ry * c);
      const double relx = xn - xc, rely = yn - yc;
      const double ukx = U0 + Om * (-rely), uky = U1 + Om * relx;
      double rho, ux, uy, g[4];
      if (vel_early) {
        ux = s_uv[0][v];
        uy = s_uv[1][v];
      } else if (cached) {
        interp_cached<MLS>(C, L, X[v], Y[v], false, rho, ux, uy, g);
      } else {
        interp_star<MLS>(A, L, X[v], Y[v], false, rho, ux, uy, g);
      }
      const double ds = 0.5 * (S_len[vm] + S_len[v]);
      p.xn[gm] = xn;
      p.yn[gm] = yn;
      const double fx = (2.0 * (ukx - ux)) * ds, fy = (2.0 * (uky - uy)) * ds;
      p.fx[gm] = fx;
      p.fy[gm] = fy;
      fm = fmax_nan(fm, fmax_nan(fabs(fx), fabs(fy)));
    }
    record_fmax(p.fmax_bits + inst, fm, s_red);
    return;
  }

  // membrane vertex forces: strain + bending + shared element loads
  double fm = 0.0;
  auto vertex_force = [&](int v, double l0v, double l0m, double sv) {
    const int gm = v0 + v;
    const int vm = v == 0 ? nv - 1 : v - 1, vp = v + 1 == nv ? 0 : v + 1;
    const int vmm = vm == 0 ? nv - 1 : vm - 1;
    // strain: element v pulls v along +t, element v-1 pulls v along -t
    const double lr = S_len[v], ll = S_len[vm];
    const double sr = ks * (lr - l0v);
    const double sl = ks * (ll - l0m);
    // tangents from normals: t = (-n_y, n_x)
    double fx = sr * (-S_ny[v]) - sl * (-S_ny[vm]);
    double fy = sr * S_nx[v] - sl * S_nx[vm];
    // bending at v-1 (v is its right vertex), v, v+1 (v is its left vertex);
    // Eq. bendFor with the lever rule: a neighbour's share is the length of
    // the edge on the far side of the bent vertex over the two lengths (the
    // symbols' defining sentence), so the three forces exert no net moment
    {
      const double c = S_bc[vm];
      const double fr = S_len[vmm] / (S_len[vmm] + S_len[vm]);
      fx += c * fr * S_bnx[vm];
      fy += c * fr * S_bny[vm];
    }
    {
      const double c = S_bc[v];
      fx -= c * S_bnx[v];
      fy -= c * S_bny[v];
    }
    {
      const double c = S_bc[vp];
      const double fl = S_len[vp] / (S_len[v] + S_len[vp]);
      fx += c * fl * S_bnx[vp];
      fy += c * fl * S_bny[vp];
    }
    fx += 0.5 * S_fex[v] + 0.5 * S_fex[vm];
    fy += 0.5 * S_fey[v] + 0.5 * S_fey[vm];
    if (rep) {
      fx -= sv * S_bnx[v];
      fy -= sv * S_bny[v];
      p.frep[gm] = 0.0;   // applied: the next step's repulsion kernel rewrites it
    }
    if (kind == kRBC) {
      p.fx[gm] = fx;
      p.fy[gm] = fy;
      fm = fmax_nan(fm, fmax_nan(fabs(fx), fabs(fy)));
    } else {
      double rho, ux, uy, g[4];
      if (vel_early) {
        ux = s_uv[0][v];
        uy = s_uv[1][v];
      } else if (cached) {
        interp_cached<MLS>(C, L, X[v], Y[v], false, rho, ux, uy, g);
      } else {
        interp_star<MLS>(A, L, X[v], Y[v], false, rho, ux, uy, g);
      }
      const double xn = X[v] + ux + 0.5 * fx / mv;
      const double yn = Y[v] + uy + 0.5 * fy / mv;
      // velocity imposed by the weak coupling: the vertex displacement of the
      // step (the second-order velocity of Eq. verletVel turns the coupling
      // into a marginally stable feedback that grows next to walls)
      const double Ux = xn - X[v], Uy = yn - Y[v];
      const double ds = 0.5 * (ll + lr);
      p.xn[gm] = xn;
      p.yn[gm] = yn;
      const double ffx = (2.0 * (Ux - ux)) * ds, ffy = (2.0 * (Uy - uy)) * ds;
      p.fx[gm] = ffx;
      p.fy[gm] = ffy;
      fm = fmax_nan(fm, fmax_nan(fabs(ffx), fabs(ffy)));
    }
  };
  if constexpr (SMALL) {
#pragma unroll
    for (int j = 0; j < kPre; ++j)
      if (t + j * nt < nv) vertex_force(t + j * nt, pre_l0[j], pre_l0m[j], pre_rep[j]);
  } else {
    for (int v = t; v < nv; v += nt) {
      const int vm = v == 0 ? nv - 1 : v - 1;
      vertex_force(v, p.l0[v0 + v], p.l0[v0 + vm], rep ? p.frep[v0 + v] : 0.0);
    }
  }
  record_fmax(p.fmax_bits + inst, fm, s_red);
}

// Workgroups [0, ninst): bond kinetics of each instance; then one workgroup
// per body: membrane forces, particle loads and motion.  ADV: the body's
// vertices first finish the previous step (merged step kernel).  SMALL_ONLY:
// every body has at most kVmax vertices (the host knows), so only the LDS
// form of the body code is compiled in: a smaller kernel, fewer instruction
// fetches on its serial path.  The merged form is only launched that way.
template <typename T, int TX, int TY, bool ADV, bool SMALL_ONLY, bool MLS>
__global__ __launch_bounds__(kBodyThreads) void k_body(Ptrs<T> p, int cache_nodes) {
  static_assert(SMALL_ONLY || !ADV, "the merged step form needs small bodies");
  __shared__ double s_red[3][kBodyThreads / 64];
  __shared__ double s_rigid[6];
  __shared__ int s_box[4];
  __shared__ double sm[10][kVmax];   // x, y, len, nx, ny, bc, bnx, bny, fex, fey
  __shared__ double s_uv[2][kBodyThreads / 2];   // fluid velocity at a small particle's vertices
  __shared__ int s_tmp[kBodyThreads];
  __shared__ int s_nelig;
  extern __shared__ unsigned char s_dyn[];
  // the other bin set (last read two steps ago) starts its next use empty
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < p.ntile_total; t += gridDim.x * blockDim.x)
    p.cnt_next[t] = 0;
  if ((int)blockIdx.x < p.ninst) {
    bonds_impl(p, blockIdx.x, s_tmp, &s_nelig);
    return;
  }
  const int b = blockIdx.x - p.ninst;
  if (SMALL_ONLY || p.body[b].nv <= kVmax)
    body_impl<T, true, TX, TY, ADV, MLS>(p, b, cache_nodes, sm, s_red, s_rigid, s_box, s_dyn, s_uv);
  else
    body_impl<T, false, TX, TY, false, MLS>(p, b, cache_nodes, sm, s_red, s_rigid, s_box, s_dyn, s_uv);
}

// Ends a run of steps: every marker moves to X^{n+1} (red cells by the
// kinematic update, particles adopt the positions of their dynamics) and
// joins the bins the next step's fused kernel reads.  Inside a run the body
// workgroups of the next step may do this for their own vertices.
template <typename T, int TX, int TY, bool MLS>
__device__ __forceinline__ void advance_impl(Ptrs<T>& p) {
  const int gm0 = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = gm0 < p.nm_total;
  const int gm = active ? gm0 : p.nm_total - 1;   // idle lanes shadow the last marker
  const int info = p.minfo[gm];          // (instance << 2) | body kind
  const int kind = info & 3;
  // the instance is almost always the same across a wave: then make it a
  // scalar so the lattice descriptor comes through scalar loads
  int inst = info >> 2;
  const int inst0 = __builtin_amdgcn_readfirstlane(inst);
  if (__ballot(inst != inst0) == 0ull) inst = inst0;
  const LatDev& L = p.lat[inst];
  const bool first = p.step_cur[inst] == 0;
  const double X = p.x[gm], Y = p.y[gm];
  double xn, yn;
  if (kind == kRBC) {
    advance_rbc<MLS>(p, L, gm, X, Y, first, xn, yn);
  } else {
    xn = p.xn[gm];
    yn = p.yn[gm];
  }
  int ncx = 0, ncy = 0;
  if (active) {
    p.xm[gm] = X;
    p.ym[gm] = Y;
    p.x[gm] = xn;
    p.y[gm] = yn;
    // stencil of the new position, used by the next step's spreading and
    // interpolation (this lane has finished reading the old one)
    marker_stencil<MLS>(p, L, gm, xn, yn, ncx, ncy);
  }
  // join the bins the next step's fused kernel reads (all lanes take part
  // in the wave-aggregated registration)
  register_marker<TX, TY>(p.cnt_next, p.bin_next, p.bin_cap, p.overflow, L, gm, ncx, ncy, active);
}

// Marker advance and new stencils: kernel weights only, or with the MLS
// transfer compiled in (launched when an instance uses it).
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_advance(Ptrs<T> p) { advance_impl<T, TX, TY, false>(p); }

template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_advance_mls(Ptrs<T> p) { advance_impl<T, TX, TY, true>(p); }

// ------------------------------------------------------------------ launchers
#define LBIB_TILE_DISPATCH(a, KERNEL, ...)                                                   \
  do {                                                                                     \
    if ((a).tile_x == 64 && (a).tile_y == 4) hipLaunchKernelGGL((KERNEL<T, 64, 4>), __VA_ARGS__);          \
    else if ((a).tile_x == 128 && (a).tile_y == 2) hipLaunchKernelGGL((KERNEL<T, 128, 2>), __VA_ARGS__);   \
    else if ((a).tile_x == 32 && (a).tile_y == 8) hipLaunchKernelGGL((KERNEL<T, 32, 8>), __VA_ARGS__);     \
    else hipLaunchKernelGGL((KERNEL<T, 256, 1>), __VA_ARGS__);                             \
  } while (0)

template <typename T>
void launch_stencil(const Ptrs<T>& p, const StepArgs& a, hipStream_t s) {
  if (p.nm_total == 0) return;
  LBIB_TILE_DISPATCH(a, k_stencil, dim3((p.nm_total + 255) / 256), dim3(256), 0, s, p);
}

template <typename T>
void launch_lagrangian(const Ptrs<T>& p, const StepArgs& a, hipStream_t s, bool advance_first) {
  const int cache_nodes = a.body_cache_bytes / (3 * (int)sizeof(T));
  const dim3 grid(p.ninst + p.nbody_total), block(kBodyThreads);
  const unsigned lds = (unsigned)a.body_cache_bytes;
  // advance_first (the merged form) is only requested when every body is
  // small: the engine resolves the step form from the same limit
  const bool small = a.max_nv <= kVmax;
#define LBIB_BODY(TXv, TYv, M)                                                                     \
  do {                                                                                          \
    if (advance_first) hipLaunchKernelGGL((k_body<T, TXv, TYv, true, true, M>), grid, block, lds, s, p, cache_nodes); \
    else if (small) hipLaunchKernelGGL((k_body<T, TXv, TYv, false, true, M>), grid, block, lds, s, p, cache_nodes); \
    else hipLaunchKernelGGL((k_body<T, TXv, TYv, false, false, M>), grid, block, lds, s, p, cache_nodes); \
  } while (0)
#define LBIB_BODY_T(M)                                                                             \
  do {                                                                                          \
    if (a.tile_x == 64 && a.tile_y == 4) LBIB_BODY(64, 4, M);                                   \
    else if (a.tile_x == 128 && a.tile_y == 2) LBIB_BODY(128, 2, M);                            \
    else if (a.tile_x == 32 && a.tile_y == 8) LBIB_BODY(32, 8, M);                              \
    else LBIB_BODY(256, 1, M);                                                                  \
  } while (0)
  if (a.any_mls) LBIB_BODY_T(true);
  else LBIB_BODY_T(false);
#undef LBIB_BODY_T
#undef LBIB_BODY
}

template <typename T>
void launch_advance(const Ptrs<T>& p, const StepArgs& a, hipStream_t s) {
  if (p.nm_total == 0) return;
  if (a.any_mls) LBIB_TILE_DISPATCH(a, k_advance_mls, dim3((p.nm_total + 255) / 256), dim3(256), 0, s, p);
  else LBIB_TILE_DISPATCH(a, k_advance, dim3((p.nm_total + 255) / 256), dim3(256), 0, s, p);
}
#undef LBIB_TILE_DISPATCH

template void launch_lagrangian<float>(const Ptrs<float>&, const StepArgs&, hipStream_t, bool);
template void launch_lagrangian<double>(const Ptrs<double>&, const StepArgs&, hipStream_t, bool);
template void launch_advance<float>(const Ptrs<float>&, const StepArgs&, hipStream_t);
template void launch_advance<double>(const Ptrs<double>&, const StepArgs&, hipStream_t);
template void launch_stencil<float>(const Ptrs<float>&, const StepArgs&, hipStream_t);
template void launch_stencil<double>(const Ptrs<double>&, const StepArgs&, hipStream_t);

}  // namespace lbib
