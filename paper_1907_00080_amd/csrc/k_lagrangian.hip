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
//
// No multiply-add contraction in this file: the same quantity is computed by
// several kernels (a body's forces by the chunked body kernel and by the
// merged step kernel, a probe value from an LDS cache or straight from the
// populations), and all of them must round alike.  Fused multiply-adds the
// compiler would form differently in each inlining context could differ in
// the last bit; the few fused operations kept are explicit (__fma_rn).
#pragma clang fp contract(off)
#include "lbib_dev.h"
#include "mls.h"

namespace lbib {

// ------------------------------------------------------------------ helpers
// Populations at a node after streaming, before forcing (walls: bounce-back),
// from a state of streaming scheme sch.
// The slots are those of streamed_slot, addressed as the fused kernel
// addresses them: the node's neighbour columns and row offsets once, then a
// uniform plane offset plus a 32-bit in-plane offset per direction (a plane
// holds at most 2^31 nodes).
template <typename T>
__device__ inline void pull_node(const T* A, int sch, long long N, int nx, int ny, int pitch, bool pery,
                                 int x, int y, T hv[kQ]) {
  const unsigned o0 = (unsigned)y * (unsigned)pitch + (unsigned)x;
  if (sch == 2) {   // node-local layout: slot i of the node itself
#pragma unroll
    for (int i = 0; i < kQ; ++i) hv[i] = A[i * N + o0];
    return;
  }
  const bool lo = !pery && y == 0, hi = !pery && y == ny - 1;   // first / last row of a walled lattice
  const unsigned cm = x == 0 ? nx - 1 : x - 1, cp = x == nx - 1 ? 0 : x + 1;
  const unsigned rm = (unsigned)(y == 0 ? (pery ? ny - 1 : y) : y - 1) * (unsigned)pitch;
  const unsigned rp = (unsigned)(y == ny - 1 ? (pery ? 0 : y) : y + 1) * (unsigned)pitch;
  const unsigned r0 = (unsigned)y * (unsigned)pitch;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const unsigned c = ex(i) > 0 ? cm : (ex(i) < 0 ? cp : (unsigned)x);
    const unsigned r = ey(i) > 0 ? rm : (ey(i) < 0 ? rp : r0);
    // bounce-back: h*_opp(i) of the node itself
    const bool bounce = (ey(i) > 0 && lo) || (ey(i) < 0 && hi);
    const int pl = bounce ? (sch == 1 ? i : opp(i)) : (sch == 1 ? opp(i) : i);
    hv[i] = A[pl * N + (bounce ? o0 : r + c)];
  }
}

// Velocity walls: a wall node of the pre-forcing state takes the drive as its
// force (the step's IB forces are not known yet).
template <typename T>
__device__ __forceinline__ void wall_fill_drive(const LatDev& L, int y, T hv[kQ]) {
  if (L.wall_mode == 1 && !L.periodic_y && (y == 0 || y == L.ny - 1))
    zou_he_fill(hv, y == 0, T(y == 0 ? L.u_wall_lo : L.u_wall_hi), T(L.gx), T(L.gy));
}

// rho* - 1 and u* = (sum f e + g/2) / rho* of a node of the pre-forcing
// state from its pulled moments, each rounded to the storage type T: the
// values the particles' LDS cache holds, so that a probe evaluated from the
// cache and one evaluated straight from the populations agree to the bit.
// The deviation rho* - 1 is what is stored, not rho* (in float32, rho*
// itself, about 1 + 1e-4, would keep only the leading digits of the
// deviation that the probe pressure cs^2 (rho* - 1) is made of).
template <typename T>
__device__ __forceinline__ void star_values(const LatDev& L, double drho, double jx, double jy, T& d,
                                            T& ux, T& uy) {
  const double r = 1.0 + drho;
  d = T(drho);
  ux = T((jx + 0.5 * L.gx) / r);
  uy = T((jy + 0.5 * L.gy) / r);
}

// MLS interpolant of rho*, u* at a point and (GRAD) its gradient (the MLS
// shape functions and their derivatives), from the node values fetch(a, b,
// x, row, rho, ux, uy) of stencil node (a, b) (x unwrapped; row unwrapped on
// a periodic lattice, else clamped: a row beyond a wall has weight zero, so
// it reads the wall row, inside the lattice and any cache of the point's
// nodes).
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
      fetch(a, b, (int)(cxr + (a - 1)), row, r, u, v);
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

// rho*, u* of the pre-forcing state at a node (x, y) inside the lattice,
// from the streamed populations, as star_values rounds them.
template <typename T>
__device__ inline void node_star(const T* A, int sch, const LatDev& L, int x, int y, double& rho,
                                 double& ux, double& uy) {
  T hv[kQ];
  pull_node(A, sch, L.plane, L.nx, L.ny, L.pitch, L.periodic_y != 0, x, y, hv);
  wall_fill_drive(L, y, hv);
  double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const double h = double(hv[i]);
    drho += h;
    jx += ex(i) * h;
    jy += ey(i) * h;
  }
  T d, u, v;
  star_values(L, drho, jx, jy, d, u, v);
  rho = 1.0 + double(d);
  ux = double(u);
  uy = double(v);
}

// Kernel (or, with MLS compiled in and selected, MLS) interpolant of rho*,
// u* at a point and (optionally) its gradient, node by node straight from
// the streamed populations: compact code for the rare point whose nodes no
// cache holds.  MLS = false compiles the kernel weights only: the
// latency-bound kernels of runs without the MLS transfer carry none of its
// code (their instruction fetches grow with the code they hold).  The three
// interpolants here (this one, interp_cached, star_sum) take the same
// node values and sum them alike, so they agree to the bit; a stencil row
// beyond a wall adds nothing (skipped here, zero weight in star_sum:
// the same sums).
template <bool MLS, typename T>
__device__ inline void interp_star(const T* A, int sch, const LatDev& L, double X, double Y, bool grad,
                                   double& rho, double& ux, double& uy, double g[4]) {
  if (MLS && use_mls(L)) {
    auto fetch = [&](int, int, int xr, int row, double& r, double& u, double& v) {
      node_star(A, sch, L, wrap_i(xr, L.nx), L.periodic_y ? wrap_i(row, L.ny) : row, r, u, v);
    };
    if (grad) interp_mls<true>(L, X, Y, fetch, rho, ux, uy, g);
    else interp_mls<false>(L, X, Y, fetch, rho, ux, uy, g);
    return;
  }
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  rho = 0; ux = 0; uy = 0;
  g[0] = g[1] = g[2] = g[3] = 0;  // du/dx, du/dy, dv/dx, dv/dy
  const bool pery = L.periodic_y != 0;
  double wxa[3], dwxa[3], wya[3], dwya[3];
  roma_weights3<true>(cxr - X, wxa, dwxa);
  roma_weights3<true>(cyr - Y, wya, dwya);
  for (int b = 0; b < 3; ++b) {
    const double ry = cyr + (b - 1);
    int row = (int)ry;
    if (pery) row = wrap_i(row, L.ny);
    else if (row < 0 || row >= L.ny) continue;
    const double wy = wya[b], dwy = dwya[b];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double rx = cxr + (a - 1);
      const int col = wrap_i((int)rx, L.nx);
      const double wx = wxa[a], dwx = dwxa[a];
      double r, u, v;
      node_star(A, sch, L, col, row, r, u, v);
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

// The star field (4 values per node: rho* - 1, u*x, u*y, unused) that the
// advance and stencil passes leave over every particle's node box, at the
// 3 x 3 nodes of a point: loaded first (nine 4-wide loads), summed by
// star_sum, so that a caller can have the loads of several points in flight
// together.  Rows beyond a wall read the wall row (weight zero).
template <typename T>
struct Star9 {
  T r[9], u[9], v[9];
};

template <typename T>
__device__ __forceinline__ void star_load(const T* S, const LatDev& L, double X, double Y, Star9<T>& n) {
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  const bool pery = L.periodic_y != 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int r = (int)(cyr + (b - 1));
    const int row = pery ? wrap_i(r, L.ny) : min(max(r, 0), L.ny - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const long long node = (long long)row * L.pitch + wrap_i((int)cxr + a - 1, L.nx);
      const T* q = S + 4 * node;
      n.r[3 * b + a] = q[0];
      n.u[3 * b + a] = q[1];
      n.v[3 * b + a] = q[2];
    }
  }
}

// Interpolant of rho*, u* (and with GRAD its gradient) from the node values
// star_load gave, summed as interp_star and interp_cached sum them.
template <bool MLS, bool GRAD, typename T>
__device__ __forceinline__ void star_sum(const LatDev& L, double X, double Y, const Star9<T>& n,
                                         double& rho, double& ux, double& uy, double g[4]) {
  constexpr bool grad = GRAD;
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  const bool pery = L.periodic_y != 0;
  if (MLS && use_mls(L)) {
    auto fetch = [&](int a, int b, int, int, double& r, double& u, double& v) {
      r = 1.0 + double(n.r[3 * b + a]);
      u = double(n.u[3 * b + a]);
      v = double(n.v[3 * b + a]);
    };
    interp_mls<GRAD>(L, X, Y, fetch, rho, ux, uy, g);
    return;
  }
  rho = 0; ux = 0; uy = 0;
  g[0] = g[1] = g[2] = g[3] = 0;
  double wxa[3], dwxa[3], wya[3], dwya[3];
  roma_weights3<true>(cxr - X, wxa, dwxa);
  roma_weights3<true>(cyr - Y, wya, dwya);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int ry = (int)(cyr + (b - 1));
    const bool ok = pery || (ry >= 0 && ry < L.ny);
    const double wy = ok ? wya[b] : 0.0;
    const double dwy = ok ? dwya[b] : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double wx = wxa[a], dwx = dwxa[a];
      const double r = 1.0 + double(n.r[3 * b + a]), u = double(n.u[3 * b + a]), v = double(n.v[3 * b + a]);
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
// LDS (x unwrapped; rows wrapped for a periodic lattice), as star_values
// gives them.  Same interpolant as interp_star, read from the cache.
template <typename T>
struct StarCache {
  const T* c;   // 3 values per node: rho - 1, ux, uy
  int bx0, by0, bw, bh;
};

template <bool MLS, typename T>
__device__ __forceinline__ void interp_cached(const StarCache<T>& C, const LatDev& L, double X, double Y,
                                     bool grad, double& rho, double& ux, double& uy, double g[4]) {
  if (MLS && use_mls(L)) {
    auto fetch = [&](int, int, int xr, int row, double& r, double& u, double& v) {
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
  double wxa[3], dwxa[3], wya[3], dwya[3];
  roma_weights3<true>(cxr - X, wxa, dwxa);
  roma_weights3<true>(cyr - Y, wya, dwya);
  for (int b = 0; b < 3; ++b) {
    const double ry = cyr + (b - 1);
    const int row = (int)ry;
    if (!pery && (row < 0 || row >= L.ny)) continue;
    const double wy = wya[b], dwy = dwya[b];
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

// ---------------------------------------------------------------- marker bins
// Register marker gm in every tile its 3x3 stencil overlaps (centre cx, cy).
// Three consecutive columns (rows) touch at most three tiles (a ragged last
// tile can be one column wide), so a marker joins at most nine bins.  Slots
// come from wave-aggregated atomics: a run of adjacent lanes that hit the
// same tile (neighbours along a membrane) shares one atomic.  A full bin drops the
// registration and counts it in *overflow (the fused kernel then poisons
// that tile's force so the watchdog reports it).
// The registration in two halves: bins_reserve issues the slot
// reservations (the atomics), bins_commit waits for them and stores the
// marker ids, so that a caller can do other work while the atomics are in
// flight.
template <int R>
struct BinSlots {
  int key[R][9], leader[R][9], rank[R][9], base[R][9];
  unsigned used;   // slots some lane of the wave uses (bit r * 9 + s9; wave-uniform)
};

template <int TX, int TY, int R>
__device__ inline void bins_reserve(int* cnt, const LatDev& L, const int* cx, const int* cy,
                                    const bool* active, BinSlots<R>& S) {
  // lattice fields in registers: read inside the loop below, the compiler
  // reloads them (and waits for them) at every slot
  const bool pery = L.periodic_y != 0;
  const int nx = L.nx, ny = L.ny, tile_base = L.tile_base, ntx = L.ntx;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int gcount[R][9];
  auto& key = S.key;
  auto& leader = S.leader;
  auto& rank = S.rank;
  unsigned used = 0;
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
      const int k = has ? tile_base + tr[i] * ntx + tc[j] : -1;
      key[r][s9] = k;
      leader[r][s9] = lane;
      rank[r][s9] = 0;
      gcount[r][s9] = 0;
      const unsigned long long hasm = __ballot(has);
      if (hasm == 0ull) continue;
      used |= 1u << (r * 9 + s9);
      const int kprev = dpp_i<kDppWaveShr1>(k);   // lane 0: its own (not used)
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
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9)
      S.base[r][s9] = (used >> (r * 9 + s9) & 1u) && gcount[r][s9] > 0
                          ? atomicAdd(&cnt[key[r][s9]], gcount[r][s9]) : 0;
  S.used = used;
}

// 3. positions and stores
//    (every slot's position first, then the stores: a store issued between
//    two of the reads would be waited for by the next one)
template <int R>
__device__ inline void bins_commit(int* bin, int cap, int* overflow, const int* gm, const BinSlots<R>& S) {
  const unsigned used = S.used;
  int pos[R][9];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9)
      pos[r][s9] = (used >> (r * 9 + s9) & 1u) ? __shfl(S.base[r][s9], S.leader[r][s9]) + S.rank[r][s9] : 0;
  int dropped = 0;
  int* dst[R][9];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9) {
      const bool on = (used >> (r * 9 + s9) & 1u) && S.key[r][s9] >= 0;
      dropped += on && pos[r][s9] >= cap;
      dst[r][s9] = on && pos[r][s9] < cap ? bin + (long long)S.key[r][s9] * cap + pos[r][s9] : nullptr;
    }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s9 = 0; s9 < 9; ++s9)
      if (dst[r][s9]) *dst[r][s9] = gm[r];
  if (dropped) atomicAdd(overflow, dropped);
}

template <int TX, int TY, int R>
__device__ inline void register_markers(int* cnt, int* bin, int cap, int* overflow, const LatDev& L,
                                        const int* gm, const int* cx, const int* cy,
                                        const bool* active) {
  BinSlots<R> S;
  bins_reserve<TX, TY, R>(cnt, L, cx, cy, active, S);
  bins_commit<R>(bin, cap, overflow, gm, S);
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
// Stencil centre node of a marker at (X, Y), as marker_stencil stores it.
__device__ inline void stencil_centre(const LatDev& L, double X, double Y, int& ocx, int& ocy) {
  const bool pery = L.periodic_y != 0;
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  ocx = wrap_i((int)cxr, L.nx);
  ocy = pery ? wrap_i((int)cyr, L.ny) : (int)fmin(fmax(cyr, -4.0), (double)(L.ny + 3));
}

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
    double w3x[3], w3y[3], d3[3];
    roma_weights3<false>(cxr - X, w3x, d3);
    roma_weights3<false>(cyr - Y, w3y, d3);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p.wx[a * nm + gm] = w3x[a];
      const double ry = cyr + (a - 1);
      const bool valid = pery || (ry >= 0.0 && ry < (double)L.ny);
      p.wy[a * nm + gm] = valid ? w3y[a] : 0.0;
    }
  }
  ocx = wrap_i((int)cxr, L.nx);
  ocy = pery ? wrap_i((int)cyr, L.ny) : (int)fmin(fmax(cyr, -4.0), (double)(L.ny + 3));
  p.cx[gm] = ocx;
  p.cy[gm] = ocy;
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
  // bond kinetics (Sec. 2.2): rupture then formation (a frozen topology
  // skips both); then every bond's spring coefficient sigma (y_l - y_eq)
  // at X^n for the particles' spring forces (Eq. adhFor)
  if (L.n_lig == 0) return;
  const bool kinetics = !L.freeze;
  __syncthreads();
  if (tid == 0) s_nelig = 0;
  __syncthreads();
  const double y_cr = L.y_cr;
  unsigned long long ties = 0;
  // (a) rupture (independent per bond) and formation eligibility; R
  // ligands per lane and pass (l0 + r nt + tid), their loads in flight
  // together
  constexpr int R = 4;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int l0 = 0; l0 < L.n_lig; l0 += R * nt) {
    int gl[R], va[R], vb[R], rr[R], flag[R];
    bool on[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int l = l0 + r * nt + tid;
      on[r] = l < L.n_lig;
      gl[r] = L.lig_base + (on[r] ? l : 0);
      va[r] = p.lig_va[gl[r]];
      vb[r] = p.lig_vb[gl[r]];
      rr[r] = p.l2r[gl[r]];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int l = l0 + r * nt + tid;
      flag[r] = 0;
      if (!on[r]) continue;
      // particle positions X^n: xn (equal to x once a step has ended; while
      // the merged step kernel runs, its particle workgroups copy xn into x)
      const double cx = 0.5 * (p.xn[va[r]] + p.xn[vb[r]]);
      const double cy = 0.5 * (p.yn[va[r]] + p.yn[vb[r]]);
      const int rc = rr[r];
      if (rc >= 0) {
        const int wall = rc < L.n_rec0 ? 0 : 1;
        const double yl = bond_len(cx, cy, p.rec_x[L.rec_base + rc], wall, L);
        const double sig = p.lig_sigma[gl[r]], sts = L.sigma_ts_frac * sig;
        const double dy = yl - L.y_eq;
        bool broken = false;
        if (kinetics) {
          const double kr = L.kr0_dt * exp((sig - sts) * dy * dy / (2.0 * L.kbt));
          const double P = 1.0 - exp(-kr);
          const double u = philox_uniform(L.seed, n, l, 1, L.instance);
          ties += fabs(u - P) < 1e-12;
          broken = u < P;
        }
        if (broken) {
          // atomic: body waves read the table while this runs
          __hip_atomic_store(&p.l2r[gl[r]], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          p.r2l[L.rec_base + rc] = -1;
        } else {
          p.lig_sp[gl[r]] = sig * dy;
        }
      } else if (kinetics) {
        const double d0 = cy - L.y_wall_lo, d1 = L.y_wall_hi - cy;
        const int wall = d0 <= d1 ? 0 : 1;
        const double d = wall == 0 ? d0 : d1;
        if (d < y_cr) flag[r] = 1 + wall;
      }
    }
    // ordered compaction of the eligible ligands (ascending ligand id):
    // per-wave counts by ballot, then every lane's place from the counts of
    // the earlier ligand ranges and waves
    unsigned long long bal[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bal[r] = __ballot(flag[r] != 0);
      if (lane == 0) s_tmp[r * nw + w] = __popcll(bal[r]);
    }
    __syncthreads();
    const int base = s_nelig;
    int off = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int before = 0, tot = 0;
      for (int k = 0; k < nw; ++k) {
        const int c = s_tmp[r * nw + k];
        before += k < w ? c : 0;
        tot += c;
      }
      if (flag[r]) {
        const int pos = base + off + before + __popcll(bal[r] & lt);
        p.lig_flag[L.lig_base + pos] = ((l0 + r * nt + tid) << 1) | (flag[r] - 1);
      }
      off += tot;
    }
    __syncthreads();
    if (tid == 0) s_nelig = base + off;
    __syncthreads();
  }
  // (b) formation, sequential over the eligible ligands in ascending order
  if (tid == 0 && kinetics) {
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
        __hip_atomic_store(&p.l2r[gl], roff + best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        p.r2l[L.rec_base + roff + best] = gl;
        p.lig_sp[gl] = sig * dy;
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
  const LatDev L = p.lat[inst];
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
  // publish: the barrier orders every lane's writes before thread 0's
  // release store of the flag (one write-back of the cache, not one per lane)
  __syncthreads();
  if (tid == 0) __hip_atomic_store(&p.bond_flag[inst], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}



// ---------------------------------------------------------------- star field
// Node box of a set of positions: floor of the smallest and ceiling of the
// largest x and y (wave-wide; lanes with on = false do not count).
struct IBox {
  int x0, x1, y0, y1;
};
__device__ inline IBox wave_box(double x, double y, bool on) {
  const auto mn = [](int a, int b) { return min(a, b); };
  const auto mx = [](int a, int b) { return max(a, b); };
  return IBox{wave_reduce_i(on ? (int)floor(x) : 0x7fffffff, mn), wave_reduce_i(on ? (int)ceil(x) : -0x7fffffff, mx),
              wave_reduce_i(on ? (int)floor(y) : 0x7fffffff, mn), wave_reduce_i(on ? (int)ceil(y) : -0x7fffffff, mx)};
}

__device__ inline void put_box(int* pbox, int chunk, const IBox& q) {
  pbox[4 * chunk] = q.x0;
  pbox[4 * chunk + 1] = q.x1;
  pbox[4 * chunk + 2] = q.y0;
  pbox[4 * chunk + 3] = q.y1;
}

// rho* - 1 and u* (star_values) of the pre-forcing state at every node of
// one particle's box: the box of its vertices (the union of its chunk
// boxes) widened by 4 nodes (probe 1.2 along the normal, stencil reach 1.5,
// a node of margin), rows clamped to the lattice unless it is periodic.
// Entry w of the star work list names the particle, this workgroup's rank
// and the particle's workgroup count; src holds the populations the next
// step streams from, in streaming scheme sch.  Nodes of overlapping boxes
// are written twice with the same values.
// The kernels below copy their instance's lattice record into registers
// before their first store: read through a reference, its fields are
// reloaded (and waited for) after every store, which may alias them.
template <typename T>
__device__ inline void star_pass(Ptrs<T>& p, const T* src, int sch, int w) {
  const int b = p.star_wg[3 * w], rank = p.star_wg[3 * w + 1], K = p.star_wg[3 * w + 2];
  const BodyDev& B = p.body[b];
  const LatDev L = p.lat[B.inst];
  const int nch = chunks_of(B.nv);
  int x0 = 0x7fffffff, x1 = -0x7fffffff, y0 = 0x7fffffff, y1 = -0x7fffffff;
  for (int k = 0; k < nch; ++k) {
    const int* q = p.pbox + 4 * (B.chunk0 + k);
    x0 = min(x0, q[0]);
    x1 = max(x1, q[1]);
    y0 = min(y0, q[2]);
    y1 = max(y1, q[3]);
  }
  x0 -= 4; x1 += 4; y0 -= 4; y1 += 4;
  const bool pery = L.periodic_y != 0;
  if (!pery) {
    y0 = max(y0, 0);
    y1 = min(y1, L.ny - 1);
  }
  const int bw = x1 - x0 + 1, bh = y1 - y0 + 1;
  if (bw <= 0 || bh <= 0) return;
  const int nbox = bw * bh;
  const T* A = src + 9 * L.node_base;
  T* S = p.star + 4 * L.node_base;
  constexpr int NB = 4;   // nodes per lane per pass: 36 loads in flight
  const int t = threadIdx.x, nt = blockDim.x;
  for (int k0 = rank * NB * nt; k0 < nbox; k0 += K * NB * nt) {
    T hv[NB][kQ];
    int row[NB];
    long long node[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int k = k0 + q * nt + t;
      const int kk = k < nbox ? k : 0;
      const int col = wrap_i(x0 + kk % bw, L.nx);
      int r = y0 + kk / bw;
      if (pery) r = wrap_i(r, L.ny);
      row[q] = r;
      node[q] = (long long)r * L.pitch + col;
      pull_node(A, sch, L.plane, L.nx, L.ny, L.pitch, pery, col, r, hv[q]);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (k0 + q * nt + t >= nbox) continue;
      wall_fill_drive(L, row[q], hv[q]);
      double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        const double h = double(hv[q][i]);
        drho += h;
        jx += ex(i) * h;
        jy += ey(i) * h;
      }
      T* o = S + 4 * node[q];
      star_values(L, drho, jx, jy, o[0], o[1], o[2]);
    }
  }
}

// ---------------------------------------------------------------- k_body
constexpr int kBodyThreads = 256;
constexpr int kWaves = kBodyThreads / 64;
constexpr int kSpinMax = 1 << 22;   // bounded wait for the bond flag (~0.2 s)
constexpr int kVmax = kSmallBody;
constexpr int kMaxChunks = (kVmax + kChunk - 1) / kChunk;

// max that propagates NaN (fmax drops it)
__device__ inline double fmax_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// Largest |F| the lanes of a wave hand to the fluid, folded into the
// instance maximum (non-negative doubles order like their bit patterns; NaN
// and Inf sort above every finite value, so a broken force shows up as a
// non-finite maximum).
__device__ inline void record_fmax(unsigned long long* slot, double m) {
  m = wave_reduce_d(m, [](double a, double b) { return fmax_nan(a, b); });
  if ((threadIdx.x & 63) == 0 && m != 0.0) atomicMax(slot, (unsigned long long)__double_as_longlong(m));
}

// Particles read the bond table (and rigid ones the step counter) that this
// instance's bond workgroup writes during the same launch: each wave waits
// for its flag (bounded spin; the bond workgroups have the lowest ids, so
// they are always dispatched).  The polls are relaxed and one acquire fence
// follows them: an acquire load invalidates the cache on every poll.
template <typename T>
__device__ inline void wait_bonds(const Ptrs<T>& p, int inst) {
  if ((threadIdx.x & 63) == 0) {
    int it = 0;
    while (__hip_atomic_load(&p.bond_flag[inst], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
           it < kSpinMax) {
      __builtin_amdgcn_s_sleep(2);
      ++it;
    }
    if (it == kSpinMax) atomicAdd(p.spin_timeouts, 1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// ---- membrane and particle arithmetic, shared by the chunked and the merged
// body kernels (the same expressions on the same inputs give the same bits)

// Element from (x0, y0) to (x1, y1): length and unit tangent.  The outward
// normal of the counter-clockwise contour is (ty, -tx).
__device__ __forceinline__ void edge_of(double x0, double y0, double x1, double y1, double& len,
                                        double& tx, double& ty) {
  const double dx = x1 - x0, dy = y1 - y0;
  len = sqrt(dx * dx + dy * dy);
  tx = dx / len;
  ty = dy / len;
}

// Vertex normal normalize(n_L + n_R) from the unit tangents of the left and
// right elements (reading R14).
__device__ __forceinline__ void vertex_normal(double txl, double tyl, double txr, double tyr,
                                              double& bnx, double& bny) {
  const double nsx = tyl + tyr, nsy = -txl - txr;
  const double nn = sqrt(nsx * nsx + nsy * nsy);
  bnx = nsx / nn;
  bny = nsy / nn;
}

// k_b (theta - theta_0), theta the signed turning angle from the left to the
// right tangent (Eq. bendFor, reading R13).
__device__ __forceinline__ double bend_coeff(double txl, double tyl, double txr, double tyr, double kb,
                                             double th0) {
  const double cr = txl * tyr - tyl * txr;
  const double dt = txl * txr + tyl * tyr;
  return kb * (atan2(cr, dt) - th0);
}

// Probe point 1.2 dx along the outward normal from the element centroid,
// kept inside the fluid (Sec. 2.2 Hydrodynamics Stresses; reading R24).
__device__ __forceinline__ void probe_point(const LatDev& L, double cx, double cy, double nxl,
                                            double nyl, double& qx, double& qy) {
  qx = cx + 1.2 * nxl;
  qy = cy + 1.2 * nyl;
  if (!L.periodic_y) qy = fmin(fmax(qy, 0.5), L.ny - 1.5);
}

// Pressure and viscous load of an element (Eqs. hydroForP, hydroForNu) from
// the probe's rho* and velocity gradient g = (du/dx, du/dy, dv/dx, dv/dy).
__device__ __forceinline__ void probe_load(double rho, const double g[4], double nu, double nxl,
                                           double nyl, double len, double& fx, double& fy) {
  const double pr = (rho - 1.0) * (1.0 / 3.0);
  const double txx = 2.0 * nu * g[0], tyy = 2.0 * nu * g[3], txy = nu * (g[1] + g[2]);
  fx = (-pr * nxl + txx * nxl + txy * nyl) * len;
  fy = (-pr * nyl + txy * nxl + tyy * nyl) * len;
}

// Load of one element: area penalty (Eq. areaFor, coefficient ca), adhesion
// spring (Eq. adhFor, sp = sigma (y_l - y_eq)) along the outward normal, and
// the probe load, summed in this order.
__device__ __forceinline__ void element_load(bool area_on, double ca, bool spring_on, double sp,
                                             bool probe_on, double pfx, double pfy, double nxl,
                                             double nyl, double& fex, double& fey) {
  fex = 0.0;
  fey = 0.0;
  if (area_on) {
    fex += ca * nxl;
    fey += ca * nyl;
  }
  if (spring_on) {
    fex += sp * nxl;
    fey += sp * nyl;
  }
  if (probe_on) {
    fex += pfx;
    fey += pfy;
  }
}

// What the force on vertex v needs from its neighbourhood: elements v-2 ..
// v+1 and vertices v-1 .. v+1.
struct VertexNbr {
  double len_mm, len_m, len, len_p;          // lengths of elements v-2, v-1, v, v+1
  double nx_m, ny_m, nx, ny;                 // outward normals of elements v-1, v
  double bc_m, bc, bc_p;                     // k_b (theta - theta_0) at v-1, v, v+1
  double bnx_m, bny_m, bnx, bny, bnx_p, bny_p;   // vertex normals at v-1, v, v+1
  double fex_m, fey_m, fex, fey;             // loads of elements v-1, v
};

// Force on vertex v: strain of its two elements (Eq. strainFor), bending at
// v-1, v and v+1 (Eq. bendFor with the lever-rule weights of reading R13b: a
// neighbour's share is the length of the edge on the far side of the bent
// vertex over the two lengths, so the three forces exert no net moment),
// half of each adjacent element's load, then the repulsion magnitude sv
// (Eq. repFor) along the inward vertex normal.
__device__ __forceinline__ void membrane_force(const VertexNbr& q, double ks, double l0v, double l0m,
                                               bool rep, double sv, double& fx, double& fy) {
  const double sr = ks * (q.len - l0v);
  const double sl = ks * (q.len_m - l0m);
  // tangents from normals: t = (-n_y, n_x)
  fx = sr * (-q.ny) - sl * (-q.ny_m);
  fy = sr * q.nx - sl * q.nx_m;
  {
    const double fr = q.len_mm / (q.len_mm + q.len_m);
    fx += q.bc_m * fr * q.bnx_m;
    fy += q.bc_m * fr * q.bny_m;
  }
  fx -= q.bc * q.bnx;
  fy -= q.bc * q.bny;
  {
    const double fl = q.len_p / (q.len + q.len_p);
    fx += q.bc_p * fl * q.bnx_p;
    fy += q.bc_p * fl * q.bny_p;
  }
  fx += 0.5 * q.fex + 0.5 * q.fex_m;
  fy += 0.5 * q.fey + 0.5 * q.fey_m;
  if (rep) {
    fx -= sv * q.bnx;
    fy -= sv * q.bny;
  }
}

// Soft-particle vertex (Eqs. newtonSoft, verletPos): new position from the
// fluid velocity u* at the vertex and half the force over the vertex mass.
// The weak coupling drives the fluid towards the vertex displacement of the
// step (readings R26, R26': the second-order velocity of Eq. verletVel turns
// the coupling into a feedback that grows next to walls), spread with the
// weight ds.
__device__ __forceinline__ void soft_vertex(double X, double Y, double ux, double uy, double fx,
                                            double fy, double mv, double ds, double& xn, double& yn,
                                            double& ffx, double& ffy) {
  xn = X + ux + 0.5 * fx / mv;
  yn = Y + uy + 0.5 * fy / mv;
  const double Ux = xn - X, Uy = yn - Y;
  ffx = (2.0 * (Ux - ux)) * ds;
  ffy = (2.0 * (Uy - uy)) * ds;
}

// One vertex's terms of a rigid particle's sums: the load of element l at
// its centroid (cx, cy) relative to the reference point, and the repulsion
// (frx, fry) at the vertex (lever lx, ly).
__device__ __forceinline__ void rigid_terms(double fex, double fey, double cx, double cy, bool rep,
                                            double frx, double fry, double lx, double ly,
                                            double t[3]) {
  t[0] = fex;
  t[1] = fey;
  t[2] = cx * fey - cy * fex;
  if (rep) {
    t[0] += frx;
    t[1] += fry;
    t[2] += lx * fry - ly * frx;
  }
}

// Rigid particle (Eqs. linearVelRig, angularVelRig; readings R28, R29): BDF2
// for U and Omega from the summed force and torque (forward Euler on the
// first step), then the reference point and the angle move by them.
// st = (U_x, U_y, Omega, x_c, y_c, theta) after the step.
__device__ __forceinline__ void rigid_step(const BodyDev* Bp, bool first, const double r3[3],
                                           double st[6]) {
  double U[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double a = r3[k] / Bp->mass;
    U[k] = first ? Bp->U[k] + a : (2.0 / 3.0) * (2.0 * Bp->U[k] - 0.5 * Bp->Um[k] + a);
  }
  const double al = r3[2] / Bp->inertia;
  const double Om = first ? Bp->Om + al : (2.0 / 3.0) * (2.0 * Bp->Om - 0.5 * Bp->Omm + al);
  st[0] = U[0];
  st[1] = U[1];
  st[2] = Om;
  st[3] = Bp->xc + U[0];
  st[4] = Bp->yc + U[1];
  st[5] = Bp->theta + Om;
}

__device__ __forceinline__ void rigid_commit(BodyDev* Bp, const double st[6]) {
  Bp->stepped = 1;
  Bp->Um[0] = Bp->U[0];
  Bp->Um[1] = Bp->U[1];
  Bp->U[0] = st[0];
  Bp->U[1] = st[1];
  Bp->Omm = Bp->Om;
  Bp->Om = st[2];
  Bp->xc = st[3];
  Bp->yc = st[4];
  Bp->theta = st[5];
}

// Rigid-particle vertex: its position from the reference shape (rx, ry)
// rotated by theta (cos cs, sin sn), and the weak-coupling force towards the
// rigid-body velocity U + Omega x r there (reading R26).
__device__ __forceinline__ void rigid_vertex(double rx, double ry, const double st[6], double cs,
                                             double sn, double ux, double uy, double ds, double& xn,
                                             double& yn, double& fx, double& fy) {
  xn = st[3] + (rx * cs + ry * (-sn));
  yn = st[4] + (rx * sn + ry * cs);
  const double relx = xn - st[3], rely = yn - st[4];
  const double ukx = st[0] + st[2] * (-rely), uky = st[1] + st[2] * relx;
  fx = (2.0 * (ukx - ux)) * ds;
  fy = (2.0 * (uky - uy)) * ds;
}

// ---------------------------------------------------------------- chunked body kernel
// One wave per vertex chunk (lane i holds vertex first + i - 2 of the body;
// the chunk's own vertices are lanes 2 .. 2 + cnt - 1).  Neighbour data come
// from the neighbouring lanes, the body's area from the chunk records of
// X^n that the advance (or stencil) pass left, so a red cell's or a soft
// particle's chunk needs nothing from any other wave.  A rigid particle's
// force and torque need all its chunks: each chunk stores its partial sums
// and the fluid velocity at its vertices, and the chunk that arrives last
// (a counter per body) takes the rigid step and moves every vertex.
template <typename T, bool MLS>
__device__ __forceinline__ void chunk_impl(Ptrs<T>& p, int code, int b, double (*s_rp)[kWaves]) {
  const int lane = threadIdx.x & 63;
  // code: the chunk of body b, or -2 for an idle wave in the workgroup of a
  // rigid body whose chunks share this workgroup (it takes part in the sums)
  const bool idle = code < 0;
  const int chunk = idle ? -1 : code;
  // the body record in registers, read before any store (the rigid step
  // writes the record back through Bp)
  BodyDev* Bp = p.body + b;
  const BodyDev B = *Bp;
  const int kind = B.kind, nv = B.nv, v0 = B.v0, inst = B.inst, ch0 = B.chunk0;
  const int nch = chunks_of(nv);
  const int first_v = idle ? 0 : (chunk - ch0) * kChunk, cnt = idle ? 0 : min(kChunk, nv - first_v);
  const int v = chunk_vertex(lane, first_v, nv), gm = v0 + v;
  const bool inner = lane >= 2 && lane < 2 + cnt;     // the chunk's own vertices
  const bool has_elem = lane >= 1 && lane < 2 + cnt;  // elements v -> v+1 they touch
  const LatDev L = p.lat[inst];
  const T* S = p.star + 4 * L.node_base;   // rho*, u* over the particles' boxes
  const bool rigid = kind == kRigid, particle = kind != kRBC;
  const bool rep = L.rep_coeff > 0.0;
  const double X = p.x[gm], Y = p.y[gm];
  // a rigid vertex's reference offset, for its move after the rigid step
  const double r0xv = rigid && inner ? p.r0x[gm] : 0.0, r0yv = rigid && inner ? p.r0y[gm] : 0.0;
  const double l0v = rigid ? 0.0 : p.l0[gm];
  const double th0v = rigid ? 0.0 : p.th0[gm];
  const double sv = rep && inner ? p.frep[gm] : 0.0;
  // the ligand of element v and its bond table entry as this wave finds it:
  // the bond workgroup rewrites the table while the wave runs (see below)
  const int ls = particle ? B.lig_stride : 0;
  const bool lig = has_elem && ls > 0 && v % ls == 0;
  const int gl = lig ? B.lig_base + v / ls : 0;
  const int r_seen = lig ? __hip_atomic_load(&p.l2r[gl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
  double area = 0.0;
  if (!rigid) area = body_area2(p.area_part, p.nchunk_total, ch0, nch) * 0.5;

  // element v -> v+1 and the bending at v
  const double Xp = lane_next(X), Yp = lane_next(Y);
  double len, tx, ty;
  edge_of(X, Y, Xp, Yp, len, tx, ty);
  const double enx = ty, eny = -tx;
  const double txl = lane_prev(tx), tyl = lane_prev(ty);
  double bnx = 0.0, bny = 0.0, bc = 0.0;
  if (!rigid || rep) vertex_normal(txl, tyl, tx, ty, bnx, bny);
  if (!rigid) bc = bend_coeff(txl, tyl, tx, ty, B.kb, th0v);

  // particles: probe load of the element and fluid velocity u* at the vertex,
  // from the star field of the particle's box
  const double cx = 0.5 * (X + Xp), cy = 0.5 * (Y + Yp);
  double pfx = 0.0, pfy = 0.0, uvx = 0.0, uvy = 0.0;
  if (particle) {
    const double nu = (L.tau - 0.5) / 3.0;
    // the probe of element v (lanes without an element probe at the vertex:
    // always a point of the box) and the vertex itself: both points' loads
    // are issued before either sum
    double qx = X, qy = Y;
    if (has_elem) probe_point(L, cx, cy, enx, eny, qx, qy);
    Star9<T> nq, nv;
    star_load(S, L, qx, qy, nq);
    star_load(S, L, X, Y, nv);
    double rho, ux, uy, g[4];
    star_sum<MLS, true>(L, qx, qy, nq, rho, ux, uy, g);
    if (has_elem) probe_load(rho, g, nu, enx, eny, len, pfx, pfy);
    double rho2, g2[4];
    star_sum<MLS, false>(L, X, Y, nv, rho2, ux, uy, g2);
    if (inner) {
      uvx = ux;
      uvy = uy;
    }
  }
  // adhesion springs on bonded ligand elements (after this step's bond
  // update).  A ligand element whose centroid lies farther than y_cr from
  // both wall lines cannot form a bond in this step, and a bond broken in
  // this step is not re-formed in it: if the entry the wave read is free,
  // whether it was the entry before the update or after it, the element
  // holds no bond after the update.  A chunk whose ligands are all such
  // needs nothing from the bond workgroup and does not wait for it.
  bool spring_on = false;
  double sp = 0.0;
  if (particle) {
    const double dw = fmin(cy - L.y_wall_lo, L.y_wall_hi - cy);
    const bool maybe = lig && (r_seen >= 0 || dw < L.y_cr + 0.25);
    if (__ballot(maybe) != 0ull) {
      wait_bonds(p, inst);
      if (lig) {
        const int r = p.l2r[gl];
        sp = p.lig_sp[gl];   // sigma (y_l - y_eq), from the bond workgroup
        spring_on = r >= 0;
      }
    }
  }
  const bool first = rigid && B.stepped == 0;
  const double ca = rigid ? 0.0 : B.ka * (1.0 - area / B.A0) * B.p_ref * len;
  double fex, fey;
  element_load(!rigid, ca, spring_on, sp, particle, pfx, pfy, enx, eny, fex, fey);
  const double len_m = lane_prev(len);
  const double ds = 0.5 * (len_m + len);   // spreading weight of the vertex

  double fm = 0.0;
  if (rigid) {
    const double xc0 = B.xc, yc0 = B.yc;
    double t3[3] = {0.0, 0.0, 0.0};
    if (inner) {
      rigid_terms(fex, fey, cx - xc0, cy - yc0, rep, -sv * bnx, -sv * bny, X - xc0, Y - yc0, t3);
      if (rep) p.frep[gm] = 0.0;   // applied: the next step's repulsion kernel rewrites it
    }
    double s3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s3[k] = wave_sum(t3[k]);
    double st[6], xn = 0.0, yn = 0.0, fx, fy;
    if (rigid_grouped(kind, nv)) {
      // the body's chunks are the waves of this workgroup, chunk c on wave c
      const int w = threadIdx.x >> 6;
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) s_rp[k][w] = s3[k];
      }
      __syncthreads();
      double r3[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) r3[k] = chunk_total(s_rp[k], nch);
      rigid_step(&B, first, r3, st);
      __syncthreads();   // every wave has read the rigid state
      if (threadIdx.x == 0) rigid_commit(Bp, st);
      const double cs = cos(st[5]), sn = sin(st[5]);
      if (inner) {
        rigid_vertex(r0xv, r0yv, st, cs, sn, uvx, uvy, ds, xn, yn, fx, fy);
        p.xn[gm] = xn;
        p.yn[gm] = yn;
        p.fx[gm] = fx;
        p.fy[gm] = fy;
        fm = fmax_nan(fabs(fx), fabs(fy));
      }
      const IBox q = wave_box(xn, yn, inner);
      if (lane == 0 && !idle) put_box(p.pbox, chunk, q);
    } else {
      // a larger rigid body: its chunks' partial sums meet in memory, and
      // the chunk that arrives last takes the rigid step for all vertices
      const int nct = p.nchunk_total;
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) p.rig_part[k * nct + chunk] = s3[k];
      }
      if (inner) {
        p.s_fex[gm] = uvx;
        p.s_fey[gm] = uvy;
        p.s_len[gm] = ds;
      }
      __threadfence();
      int done = 0;
      if (lane == 0)
        done = __hip_atomic_fetch_add(&p.body_cnt[b], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      done = __builtin_amdgcn_readfirstlane(done);   // lane 0's count
      if (done != nch - 1) return;   // a later chunk finishes the body
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) p.body_cnt[b] = 0;
      double r3[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) r3[k] = chunk_total(p.rig_part + k * nct + ch0, nch);
      rigid_step(&B, first, r3, st);
      if (lane == 0) rigid_commit(Bp, st);
      const double cs = cos(st[5]), sn = sin(st[5]);
      IBox q{0x7fffffff, -0x7fffffff, 0x7fffffff, -0x7fffffff};
      // four vertices per lane and pass, their loads issued before any store
      for (int w0 = 0; w0 < nv; w0 += 4 * 64) {
        double rx[4], ry[4], ux[4], uy[4], dv[4];
        int g2[4];
        bool on[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int w = w0 + j * 64 + lane;
          on[j] = w < nv;
          g2[j] = v0 + (on[j] ? w : 0);
          rx[j] = p.r0x[g2[j]];
          ry[j] = p.r0y[g2[j]];
          ux[j] = p.s_fex[g2[j]];
          uy[j] = p.s_fey[g2[j]];
          dv[j] = p.s_len[g2[j]];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (!on[j]) continue;
          rigid_vertex(rx[j], ry[j], st, cs, sn, ux[j], uy[j], dv[j], xn, yn, fx, fy);
          p.xn[g2[j]] = xn;
          p.yn[g2[j]] = yn;
          p.fx[g2[j]] = fx;
          p.fy[g2[j]] = fy;
          fm = fmax_nan(fm, fmax_nan(fabs(fx), fabs(fy)));
          q.x0 = min(q.x0, (int)floor(xn)); q.x1 = max(q.x1, (int)ceil(xn));
          q.y0 = min(q.y0, (int)floor(yn)); q.y1 = max(q.y1, (int)ceil(yn));
        }
      }
      const auto mn = [](int a, int b) { return min(a, b); };
      const auto mx = [](int a, int b) { return max(a, b); };
      q = IBox{wave_reduce_i(q.x0, mn), wave_reduce_i(q.x1, mx), wave_reduce_i(q.y0, mn),
               wave_reduce_i(q.y1, mx)};
      for (int k = lane; k < nch; k += 64) put_box(p.pbox, ch0 + k, q);
    }
    record_fmax(p.fmax_bits + inst, fm);
    return;
  }

  // red cells and soft particles: vertex forces
  VertexNbr q;
  // (two lanes back: lane 1 gets lane 0's value, which only the halo uses)
  q.len_mm = lane_prev(len_m);
  q.len_m = len_m;
  q.len = len;
  q.len_p = lane_next(len);
  q.nx_m = lane_prev(enx);
  q.ny_m = lane_prev(eny);
  q.nx = enx;
  q.ny = eny;
  q.bc_m = lane_prev(bc);
  q.bc = bc;
  q.bc_p = lane_next(bc);
  q.bnx_m = lane_prev(bnx);
  q.bny_m = lane_prev(bny);
  q.bnx = bnx;
  q.bny = bny;
  q.bnx_p = lane_next(bnx);
  q.bny_p = lane_next(bny);
  q.fex_m = lane_prev(fex);
  q.fey_m = lane_prev(fey);
  q.fex = fex;
  q.fey = fey;
  const double l0m = lane_prev(l0v);
  double sxn = 0.0, syn = 0.0, ffx, ffy;   // a soft particle's new position
  if (inner) {
    double fx, fy;
    membrane_force(q, B.ks, l0v, l0m, rep, sv, fx, fy);
    if (rep) p.frep[gm] = 0.0;   // applied: the next step's repulsion kernel rewrites it
    if (kind == kRBC) {
      p.fx[gm] = fx;
      p.fy[gm] = fy;
      fm = fmax_nan(fabs(fx), fabs(fy));
    } else {
      soft_vertex(X, Y, uvx, uvy, fx, fy, B.mv, ds, sxn, syn, ffx, ffy);
      p.xn[gm] = sxn;
      p.yn[gm] = syn;
      p.fx[gm] = ffx;
      p.fy[gm] = ffy;
      fm = fmax_nan(fabs(ffx), fabs(ffy));
    }
  }
  if (kind == kSoft) {
    const IBox q = wave_box(sxn, syn, inner);
    if (lane == 0) put_box(p.pbox, chunk, q);
  }
  record_fmax(p.fmax_bits + inst, fm);
}

// ---------------------------------------------------------------- merged step kernel
// Sum over a body's vertices in the canonical order (terms in LDS, term[v]):
// wave w forms the partials of chunks w, w + kWaves, ... over the lanes of
// the chunk layout, then every lane adds the chunk partials in chunk order.
__device__ inline double canonical_sum(const double* term, int nv, double* s_part) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nch = chunks_of(nv);
  __syncthreads();   // the terms are in LDS
  for (int c = w; c < nch; c += kWaves) {
    const int first = c * kChunk, cnt = min(kChunk, nv - first);
    const int v = chunk_vertex(lane, first, nv);
    const bool inner = lane >= 2 && lane < 2 + cnt;
    const double s = wave_sum(inner ? term[v] : 0.0);
    if (lane == 0) s_part[c] = s;
  }
  __syncthreads();
  const double out = chunk_total(s_part, nch);
  __syncthreads();   // the terms and partials may be overwritten
  return out;
}

// One 256-lane workgroup per body of at most kVmax vertices, its per-vertex
// data in LDS.  The body's vertices first finish the previous step (the
// kinematic update of red cells or the adoption of the particle dynamics,
// stencils, and the bins of this step's fused kernel; two vertices per lane,
// their loads and bin reservations in flight together), then the forces
// and particle dynamics of this step, with the arithmetic of the chunked
// kernel.  Particles cache rho*, u* of the node box their stencils reach in
// LDS.
template <typename T, int TX, int TY, bool MLS>
__device__ __forceinline__ void body_merged_impl(Ptrs<T>& p, int b, int cache_nodes, double (*sm)[kVmax],
                                                 double (*s_terms)[kVmax], double (*s_part)[kMaxChunks],
                                                 int* s_box, int* s_nbox, unsigned char* s_dyn,
                                                 double (*s_uv)[kBodyThreads / 2]) {
  BodyDev* Bp = p.body + b;
  const int kind = Bp->kind, nv = Bp->nv, v0 = Bp->v0, inst = Bp->inst;
  const double ks = Bp->ks, kb = Bp->kb, ka = Bp->ka, p_ref = Bp->p_ref, A0 = Bp->A0;
  const double mv = Bp->mv, sigma = Bp->sigma;
  const int lig_stride = Bp->lig_stride, lig_base = Bp->lig_base;
  const LatDev L = p.lat[inst];
  const int t = threadIdx.x, nt = kBodyThreads;   // the launch's block size
  const T* A = p.A + 9 * L.node_base;
  const double nu = (L.tau - 0.5) / 3.0;
  const bool pery = L.periodic_y != 0;
  // the repulsion needs every body's X^n before any body's forces, which
  // this form cannot give: it is never launched with the repulsion on
  const bool rep = false;
  // rest data of this lane's two vertices (va, vb), requested now so that
  // the loads are in flight during the work before their use (scalars, not
  // arrays: an array the compiler fails to keep in registers goes to
  // private memory)
  static_assert(kVmax == 2 * kBodyThreads, "two vertices per lane");
  const int va = t, vb = t + nt;
  double th0a, th0b, l0a, l0b, l0ma, l0mb;
  {
    const bool soft = kind != kRigid;
    const int ua = va < nv ? va : 0, ub = vb < nv ? vb : 0;
    th0a = soft ? p.th0[v0 + ua] : 0.0;
    th0b = soft ? p.th0[v0 + ub] : 0.0;
    l0a = soft ? p.l0[v0 + ua] : 0.0;
    l0b = soft ? p.l0[v0 + ub] : 0.0;
    l0ma = soft ? p.l0[v0 + (ua == 0 ? nv - 1 : ua - 1)] : 0.0;
    l0mb = soft ? p.l0[v0 + (ub == 0 ? nv - 1 : ub - 1)] : 0.0;
  }
  const double* X = sm[0];
  const double* Y = sm[1];
  double* S_len = sm[2];
  double* S_nx = sm[3];
  double* S_ny = sm[4];
  double* S_bc = sm[5];
  double* S_bnx = sm[6];
  double* S_bny = sm[7];
  double* S_fex = sm[8];
  double* S_fey = sm[9];
  // ---- end of the previous step for this body's vertices: X^n, stencils,
  // bins of this step's fused kernel.  Particles also take the bounding box
  // of X^n for their LDS cache from here.
  int mnx = 0x7fffffff, mxx = -0x7fffffff, mny = 0x7fffffff, mxy = -0x7fffffff;
  {
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
          sm[0][base0 + r * nt + t] = xn[r];
          sm[1][base0 + r * nt + t] = yn[r];
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
  // margin).  Boxes larger than the cache fall back to direct evaluation
  // (the same values: star_values rounds both alike).
  bool cached = false;
  StarCache<T> C{(const T*)s_dyn, 0, 0, 0, 0};
  if (kind != kRBC) {
    // wave reductions first: only one lane per wave touches the LDS words.
    // (Shuffles, not wave_reduce_i: with the DPP form this kernel's FP32
    // MLS particles went non-finite, for a cause not found.)
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
          pull_node(A, p.sch, Nn, L.nx, L.ny, L.pitch, pery, col, row, hv[q]);
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
          star_values(L, drho, jx, jy, cw[3 * k], cw[3 * k + 1], cw[3 * k + 2]);
        }
      }
    }
  }
  __syncthreads();   // positions, stencils and cache visible to the workgroup

  // pass 1: element geometry (element v joins v -> v+1), bending, shoelace terms
  auto pass1 = [&](int v, double th0v) {
    const int vp = v + 1 == nv ? 0 : v + 1, vm = v == 0 ? nv - 1 : v - 1;
    double lr, txr, tyr, ll, txl, tyl;
    edge_of(X[v], Y[v], X[vp], Y[vp], lr, txr, tyr);
    edge_of(X[vm], Y[vm], X[v], Y[v], ll, txl, tyl);
    S_len[v] = lr;
    S_nx[v] = tyr;
    S_ny[v] = -txr;
    if (kind != kRigid || rep) {
      double bnx, bny;
      vertex_normal(txl, tyl, txr, tyr, bnx, bny);
      S_bnx[v] = bnx;
      S_bny[v] = bny;
    }
    if (kind != kRigid) S_bc[v] = bend_coeff(txl, tyl, txr, tyr, kb, th0v);
    s_terms[0][v] = shoelace_term(X[v], Y[v], X[vp], Y[vp]);
  };
  if (va < nv) pass1(va, th0a);
  if (vb < nv) pass1(vb, th0b);
  // twice the area in the canonical order of body_area2: per chunk the sum
  // over its interior edges (a wave butterfly in the chunk layout) plus its
  // last edge, then the chunks in order (the barriers also publish the scratch)
  double area;
  {
    const int lane = t & 63, w = t >> 6, nch = chunks_of(nv);
    __syncthreads();
    for (int c = w; c < nch; c += kWaves) {
      const int first = c * kChunk, cnt = min(kChunk, nv - first);
      const int v = chunk_vertex(lane, first, nv);
      const double P = wave_sum(lane >= 2 && lane < 1 + cnt ? s_terms[0][v] : 0.0);
      if (lane == 0) s_part[0][c] = P + s_terms[0][first + cnt - 1];
    }
    __syncthreads();
    area = chunk_total(s_part[0], nch) * 0.5;
    __syncthreads();
  }

  const bool first = kind == kRigid && Bp->stepped == 0;
  if (kind != kRBC) wait_bonds(p, inst);

  // A particle of at most nt/2 vertices: the upper half of the lanes (other
  // waves, so other SIMDs) interpolates the fluid velocity at the vertices
  // while the lower half runs the probes, instead of after the particle's
  // update; the values are the same, read back from LDS.
  const bool vel_early = kind != kRBC && nv <= nt / 2;
  if (vel_early && t >= nt / 2 && t - nt / 2 < nv) {
    const int v = t - nt / 2;
    double rho, ux, uy, g[4];
    if (cached) interp_cached<MLS>(C, L, X[v], Y[v], false, rho, ux, uy, g);
    else interp_star<MLS>(A, p.sch, L, X[v], Y[v], false, rho, ux, uy, g);
    s_uv[0][v] = ux;
    s_uv[1][v] = uy;
  }
  auto vertex_velocity = [&](int v, double& ux, double& uy) {
    double rho, g[4];
    if (vel_early) {
      ux = s_uv[0][v];
      uy = s_uv[1][v];
    } else if (cached) {
      interp_cached<MLS>(C, L, X[v], Y[v], false, rho, ux, uy, g);
    } else {
      interp_star<MLS>(A, p.sch, L, X[v], Y[v], false, rho, ux, uy, g);
    }
  };
  // pass 2: element loads (area penalty, adhesion springs, probe stresses)
  for (int l = t; l < nv; l += nt) {
    const int lp = l + 1 == nv ? 0 : l + 1;
    const double len = S_len[l], nxl = S_nx[l], nyl = S_ny[l];
    const double ca = kind != kRigid ? ka * (1.0 - area / A0) * p_ref * len : 0.0;
    bool spring_on = false;
    double sp = 0.0, pfx = 0.0, pfy = 0.0;
    if (kind != kRBC) {
      const double cx = 0.5 * (X[l] + X[lp]), cy = 0.5 * (Y[l] + Y[lp]);
      if (lig_stride > 0 && l % lig_stride == 0) {
        const int gl = lig_base + l / lig_stride;
        spring_on = p.l2r[gl] >= 0;
        sp = spring_on ? p.lig_sp[gl] : 0.0;   // sigma (y_l - y_eq), from the bond workgroup
      }
      double qx, qy, rho, ux, uy, g[4];
      probe_point(L, cx, cy, nxl, nyl, qx, qy);
      if (cached) interp_cached<MLS>(C, L, qx, qy, true, rho, ux, uy, g);
      else interp_star<MLS>(A, p.sch, L, qx, qy, true, rho, ux, uy, g);
      probe_load(rho, g, nu, nxl, nyl, len, pfx, pfy);
    }
    element_load(kind != kRigid, ca, spring_on, sp, kind != kRBC, pfx, pfy, nxl, nyl, S_fex[l], S_fey[l]);
  }
  __syncthreads();

  double fm = 0.0;
  if (kind == kRigid) {
    const double xc0 = Bp->xc, yc0 = Bp->yc;
    for (int l = t; l < nv; l += nt) {
      const int lp = l + 1 == nv ? 0 : l + 1;
      double t3[3];
      rigid_terms(S_fex[l], S_fey[l], 0.5 * (X[l] + X[lp]) - xc0, 0.5 * (Y[l] + Y[lp]) - yc0, rep,
                  0.0, 0.0, X[l] - xc0, Y[l] - yc0, t3);
      s_terms[0][l] = t3[0];
      s_terms[1][l] = t3[1];
      s_terms[2][l] = t3[2];
    }
    double r3[3], st[6];
    r3[0] = canonical_sum(s_terms[0], nv, s_part[0]);
    r3[1] = canonical_sum(s_terms[1], nv, s_part[1]);
    r3[2] = canonical_sum(s_terms[2], nv, s_part[2]);
    rigid_step(Bp, first, r3, st);
    __syncthreads();   // every lane has read the rigid state
    if (t == 0) rigid_commit(Bp, st);
    const double cs = cos(st[5]), sn = sin(st[5]);
    IBox q{0x7fffffff, -0x7fffffff, 0x7fffffff, -0x7fffffff};
    for (int v = t; v < nv; v += nt) {
      const int gm = v0 + v, vm = v == 0 ? nv - 1 : v - 1;
      double ux, uy, xn, yn, fx, fy;
      vertex_velocity(v, ux, uy);
      rigid_vertex(p.r0x[gm], p.r0y[gm], st, cs, sn, ux, uy, 0.5 * (S_len[vm] + S_len[v]), xn, yn, fx,
                   fy);
      p.xn[gm] = xn;
      p.yn[gm] = yn;
      p.fx[gm] = fx;
      p.fy[gm] = fy;
      fm = fmax_nan(fm, fmax_nan(fabs(fx), fabs(fy)));
      q.x0 = min(q.x0, (int)floor(xn)); q.x1 = max(q.x1, (int)ceil(xn));
      q.y0 = min(q.y0, (int)floor(yn)); q.y1 = max(q.y1, (int)ceil(yn));
    }
    record_fmax(p.fmax_bits + inst, fm);
    publish_box(p.pbox, Bp->chunk0, chunks_of(nv), q, s_nbox);
    return;
  }

  // membrane vertex forces: strain + bending + shared element loads
  IBox q{0x7fffffff, -0x7fffffff, 0x7fffffff, -0x7fffffff};   // soft particles' new box
  auto vertex_force = [&](int v, double l0v, double l0m) {
    const int gm = v0 + v;
    const int vm = v == 0 ? nv - 1 : v - 1, vp = v + 1 == nv ? 0 : v + 1;
    const int vmm = vm == 0 ? nv - 1 : vm - 1;
    VertexNbr n;
    n.len_mm = S_len[vmm];
    n.len_m = S_len[vm];
    n.len = S_len[v];
    n.len_p = S_len[vp];
    n.nx_m = S_nx[vm];
    n.ny_m = S_ny[vm];
    n.nx = S_nx[v];
    n.ny = S_ny[v];
    n.bc_m = S_bc[vm];
    n.bc = S_bc[v];
    n.bc_p = S_bc[vp];
    n.bnx_m = S_bnx[vm];
    n.bny_m = S_bny[vm];
    n.bnx = S_bnx[v];
    n.bny = S_bny[v];
    n.bnx_p = S_bnx[vp];
    n.bny_p = S_bny[vp];
    n.fex_m = S_fex[vm];
    n.fey_m = S_fey[vm];
    n.fex = S_fex[v];
    n.fey = S_fey[v];
    double fx, fy;
    membrane_force(n, ks, l0v, l0m, rep, 0.0, fx, fy);
    if (kind == kRBC) {
      p.fx[gm] = fx;
      p.fy[gm] = fy;
      fm = fmax_nan(fm, fmax_nan(fabs(fx), fabs(fy)));
    } else {
      double ux, uy, xn, yn, ffx, ffy;
      vertex_velocity(v, ux, uy);
      soft_vertex(X[v], Y[v], ux, uy, fx, fy, mv, 0.5 * (n.len_m + n.len), xn, yn, ffx, ffy);
      p.xn[gm] = xn;
      p.yn[gm] = yn;
      p.fx[gm] = ffx;
      p.fy[gm] = ffy;
      fm = fmax_nan(fm, fmax_nan(fabs(ffx), fabs(ffy)));
      q.x0 = min(q.x0, (int)floor(xn)); q.x1 = max(q.x1, (int)ceil(xn));
      q.y0 = min(q.y0, (int)floor(yn)); q.y1 = max(q.y1, (int)ceil(yn));
    }
  };
  if (va < nv) vertex_force(va, l0a, l0ma);
  if (vb < nv) vertex_force(vb, l0b, l0mb);
  record_fmax(p.fmax_bits + inst, fm);
  if (kind == kSoft) publish_box(p.pbox, Bp->chunk0, chunks_of(nv), q, s_nbox);
}

// Box of a particle's new vertex positions (this workgroup's lanes folded in
// LDS), written to every chunk slot of the particle for the star pass.
__device__ inline void publish_box(int* pbox, int ch0, int nch, IBox q, int* s_nbox) {
  const int t = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) {
    q.x0 = min(q.x0, __shfl_xor(q.x0, o));
    q.x1 = max(q.x1, __shfl_xor(q.x1, o));
    q.y0 = min(q.y0, __shfl_xor(q.y0, o));
    q.y1 = max(q.y1, __shfl_xor(q.y1, o));
  }
  if (t == 0) {
    s_nbox[0] = 0x7fffffff; s_nbox[1] = -0x7fffffff; s_nbox[2] = 0x7fffffff; s_nbox[3] = -0x7fffffff;
  }
  __syncthreads();
  if ((t & 63) == 0) {
    atomicMin(&s_nbox[0], q.x0); atomicMax(&s_nbox[1], q.x1);
    atomicMin(&s_nbox[2], q.y0); atomicMax(&s_nbox[3], q.y1);
  }
  __syncthreads();
  for (int k = t; k < nch; k += blockDim.x) {
    pbox[4 * (ch0 + k)] = s_nbox[0];
    pbox[4 * (ch0 + k) + 1] = s_nbox[1];
    pbox[4 * (ch0 + k) + 2] = s_nbox[2];
    pbox[4 * (ch0 + k) + 3] = s_nbox[3];
  }
}

// Merged step form: workgroups [0, ninst) run the bond kinetics of each
// instance; then one workgroup per body (every body has at most kVmax
// vertices) finishes the previous step for its vertices and computes this
// step's forces.
template <typename T, int TX, int TY, bool MLS>
__global__ __launch_bounds__(kBodyThreads) void k_body(Ptrs<T> p, int cache_nodes) {
  __shared__ double s_part[3][kMaxChunks];
  __shared__ int s_box[4];
  __shared__ int s_nbox[4];
  __shared__ double sm[10][kVmax];   // x, y, len, nx, ny, bc, bnx, bny, fex, fey
  __shared__ double s_terms[3][kVmax];
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
  body_merged_impl<T, TX, TY, MLS>(p, blockIdx.x - p.ninst, cache_nodes, sm, s_terms, s_part, s_box,
                                   s_nbox, s_dyn, s_uv);
}

// Three-kernel and overlapped step forms: workgroups [0, ninst) run the bond
// kinetics of each instance; then one wave per vertex chunk of every body.
template <typename T, bool MLS>
__global__ __launch_bounds__(kBodyThreads) void k_body_chunks(Ptrs<T> p) {
  __shared__ int s_tmp[kBodyThreads];
  __shared__ int s_nelig;
  __shared__ double s_rp[3][kWaves];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < p.ntile_total; t += gridDim.x * blockDim.x)
    p.cnt_next[t] = 0;
  if ((int)blockIdx.x < p.ninst) {
    bonds_impl(p, blockIdx.x, s_tmp, &s_nelig);
    return;
  }
  const int slot = (blockIdx.x - p.ninst) * kWaves + (threadIdx.x >> 6);
  const int2 sc = slot < p.nslot ? p.slot_chunk[slot] : make_int2(-1, 0);
  if (sc.x != -1) chunk_impl<T, MLS>(p, sc.x, sc.y, s_rp);
}

// ---------------------------------------------------------------- advance and stencil passes
// One wave per vertex chunk, its own vertices on lanes 2 .. 2 + cnt - 1 (the
// halo lanes idle: their vertices belong to waves that move them in place).
// ADVANCE: every vertex moves to X^{n+1} (red cells by the kinematic update,
// particles adopt the positions of their dynamics); otherwise X stays (the
// stencil pass after set-up or after the positions were set).  Each vertex
// stores its stencil and joins the bins (cnt, bin) of the next fused
// kernel.  The chunk's area record of the new positions (its interior-edge
// shoelace sum, its first and last vertex) is what the next body kernel
// adds up into the body's area.
template <typename T, int TX, int TY, bool MLS, bool ADVANCE>
__device__ __forceinline__ void advance_chunk(Ptrs<T>& p, int* cnt, int* bin) {
  const int lane = threadIdx.x & 63;
  const int chunk = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (chunk >= p.nchunk_total) return;   // the whole wave
  // one load gives the wave its vertices (the body record is not needed)
  const int4 ci = p.chunk_info[chunk];
  const int kind = ci.w & 3, inst = ci.w >> 2, cnt_v = ci.z;
  const bool inner = lane >= 2 && lane < 2 + cnt_v;
  const int gm = inner ? ci.y + lane : 0;
  const LatDev L = p.lat[inst];
  double X = 0.0, Y = 0.0, xn = 0.0, yn = 0.0;
  int ncx = 0, ncy = 0;
  if (inner) {
    X = p.x[gm];
    Y = p.y[gm];
    xn = X;
    yn = Y;
    if (ADVANCE) {
      if (kind == kRBC) {
        advance_rbc<MLS>(p, L, gm, X, Y, p.step_cur[inst] == 0, xn, yn);
      } else {
        xn = p.xn[gm];
        yn = p.yn[gm];
      }
    }
    stencil_centre(L, xn, yn, ncx, ncy);
  }
  // bin slots for the new stencil: the reservations (atomics) go out first
  // and the stores below are issued while they are in flight
  BinSlots<1> S;
  bins_reserve<TX, TY, 1>(cnt, L, &ncx, &ncy, &inner, S);
  if (inner) {
    if (ADVANCE) {
      p.xm[gm] = X;
      p.ym[gm] = Y;
      p.x[gm] = xn;
      p.y[gm] = yn;
    }
    // stencil of the new position, used by the next step's spreading and
    // interpolation (this lane has finished reading the old one)
    marker_stencil<MLS>(p, L, gm, xn, yn, ncx, ncy);
  }
  const double xr = lane_next(xn), yr = lane_next(yn);
  const double part = wave_sum(lane >= 2 && lane < 1 + cnt_v ? shoelace_term(xn, yn, xr, yr) : 0.0);
  const int nct = p.nchunk_total;
  if (lane == 0) p.area_part[chunk] = part;
  if (lane == 2) {
    p.area_part[nct + chunk] = xn;
    p.area_part[2 * nct + chunk] = yn;
  }
  if (lane == 1 + cnt_v) {
    p.area_part[3 * nct + chunk] = xn;
    p.area_part[4 * nct + chunk] = yn;
  }
  if (!ADVANCE && kind != kRBC) {
    // the stencil pass boxes the particles for the star pass that follows
    // it (when advancing, the body kernel has boxed their new positions)
    const IBox q = wave_box(xn, yn, inner);
    if (lane == 0) put_box(p.pbox, chunk, q);
  }
  bins_commit<1>(bin, p.bin_cap, p.overflow, &gm, S);
}

inline __host__ __device__ int chunk_blocks(int nchunk) { return (nchunk + kWaves - 1) / kWaves; }

// Marker advance, new stencils, bins and area records (kernel weights only,
// or with the MLS transfer compiled in, launched when an instance uses it);
// the workgroups after the chunks' fill the star field of the particles'
// boxes from the populations this step's fused kernel wrote.
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_advance(Ptrs<T> p) {
  const int cb = chunk_blocks(p.nchunk_total);
  if ((int)blockIdx.x >= cb) {
    star_pass(p, p.B, p.sch_next, blockIdx.x - cb);
    return;
  }
  advance_chunk<T, TX, TY, false, true>(p, p.cnt_next, p.bin_next);
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_advance_mls(Ptrs<T> p) {
  const int cb = chunk_blocks(p.nchunk_total);
  if ((int)blockIdx.x >= cb) {
    star_pass(p, p.B, p.sch_next, blockIdx.x - cb);
    return;
  }
  advance_chunk<T, TX, TY, true, true>(p, p.cnt_next, p.bin_next);
}

// Star field of the particles' boxes from the current populations (after
// the stencil pass).
template <typename T>
__global__ __launch_bounds__(256) void k_star(Ptrs<T> p) { star_pass(p, p.A, p.sch, blockIdx.x); }

// Stencils, bins and area partials of all markers from their current
// positions (after set-up or after positions were overwritten from the host).
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_stencil(Ptrs<T> p) {
  advance_chunk<T, TX, TY, true, false>(p, p.cnt_cur, p.bin_cur);
}

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
  if (p.nchunk_total == 0) return;
  LBIB_TILE_DISPATCH(a, k_stencil, dim3(chunk_blocks(p.nchunk_total)), dim3(256), 0, s, p);
  if (p.nstar_wg > 0) hipLaunchKernelGGL((k_star<T>), dim3(p.nstar_wg), dim3(256), 0, s, p);
}

template <typename T>
void launch_lagrangian(const Ptrs<T>& p, const StepArgs& a, hipStream_t s, bool advance_first) {
  if (!advance_first) {
    const dim3 grid(p.ninst + (unsigned)(p.nslot / kWaves)), block(kBodyThreads);
    if (a.any_mls) hipLaunchKernelGGL((k_body_chunks<T, true>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((k_body_chunks<T, false>), grid, block, 0, s, p);
    return;
  }
  // the merged form is only requested when every body is small: the engine
  // resolves the step form from the same limit
  const int cache_nodes = a.body_cache_bytes / (3 * (int)sizeof(T));
  const dim3 grid(p.ninst + p.nbody_total), block(kBodyThreads);
  const unsigned lds = (unsigned)a.body_cache_bytes;
#define LBIB_BODY_T(M)                                                                                       \
  do {                                                                                                    \
    if (a.tile_x == 64 && a.tile_y == 4) hipLaunchKernelGGL((k_body<T, 64, 4, M>), grid, block, lds, s, p, cache_nodes);       \
    else if (a.tile_x == 128 && a.tile_y == 2) hipLaunchKernelGGL((k_body<T, 128, 2, M>), grid, block, lds, s, p, cache_nodes); \
    else if (a.tile_x == 32 && a.tile_y == 8) hipLaunchKernelGGL((k_body<T, 32, 8, M>), grid, block, lds, s, p, cache_nodes);   \
    else hipLaunchKernelGGL((k_body<T, 256, 1, M>), grid, block, lds, s, p, cache_nodes);                  \
  } while (0)
  if (a.any_mls) LBIB_BODY_T(true);
  else LBIB_BODY_T(false);
#undef LBIB_BODY_T
}

template <typename T>
void launch_advance(const Ptrs<T>& p, const StepArgs& a, hipStream_t s) {
  if (p.nchunk_total == 0) return;
  const dim3 grid((unsigned)(chunk_blocks(p.nchunk_total) + p.nstar_wg)), block(256);
  if (a.any_mls) LBIB_TILE_DISPATCH(a, k_advance_mls, grid, block, 0, s, p);
  else LBIB_TILE_DISPATCH(a, k_advance, grid, block, 0, s, p);
}
#undef LBIB_TILE_DISPATCH

template void launch_lagrangian<float>(const Ptrs<float>&, const StepArgs&, hipStream_t, bool);
template void launch_lagrangian<double>(const Ptrs<double>&, const StepArgs&, hipStream_t, bool);
template void launch_advance<float>(const Ptrs<float>&, const StepArgs&, hipStream_t);
template void launch_advance<double>(const Ptrs<double>&, const StepArgs&, hipStream_t);
template void launch_stencil<float>(const Ptrs<float>&, const StepArgs&, hipStream_t);
template void launch_stencil<double>(const Ptrs<double>&, const StepArgs&, hipStream_t);

}  // namespace lbib
