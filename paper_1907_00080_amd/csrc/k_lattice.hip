// k_lattice.hip - fused D2Q9 collide-and-stream with gathered IB spreading (gfx950).
//
// One workgroup owns one TX x TY tile of nodes (one node per lane).  Per node:
//   1. Eulerian force F = g + sum_k F_k delta(x - X_k) (Sec. 2.2 spreading):
//      gathered from the tile's bin of markers whose 3x3 stencil overlaps it
//      (filled by the previous step's marker advance),
//      accumulated in LDS in 64-bit fixed point (order independent, hence
//      deterministic, and free of global atomics).  Tiles with an empty bin
//      skip this and use F = g.
//   2. Streaming h_i(x) <- h*_i(x - e_i), x periodic, halfway bounce-back
//      at y = -1/2 and ny - 1/2 (Sec. 3 walls; Eq. BGK streaming part):
//      pulled from a second buffer (SCH 0), or in place in one buffer by
//      the neighbour pass (SCH 1) and the node-local pass (SCH 2), which
//      alternate (slot layouts: streamed_slot in lbib_dev.h).
//   3. rho = 1 + sum h, u = (sum h e + F/2)/rho, BGK relaxation towards the
//      equilibrium of Eq. (feq) plus Guo's source of Eq. (ForcingTerm):
//      h* = h + (h_eq - h)/tau + (1 - 1/(2 tau)) w_i [3(e-u) + 9(e.u)e].F
//   4. Store h*, and u on touched tiles (interpolation input of the markers).
// Populations are stored shifted by their rest weights (h = f - w) so that
// float32 keeps the small deviations of the low-Mach flows accurately.
//
// Workgroup -> tile mapping is XCD aware: consecutive workgroups go to the 8
// XCDs in turn, and the tiles are cut into 8 * kXcdBands equal bands of
// consecutive tiles, XCD k taking bands k, k + 8, ...  Within a band the
// rows that neighbouring tiles share stay in one XCD's L2; two bands per XCD
// instead of one spread each XCD's share over the lattice, so that the tiles
// with IB force (which cluster where the bodies are) and the lattice regions
// even out between XCDs (measured faster on the 6667 x 667 capillary, the
// same on 2000 x 200; more bands gained no more).
//
// No multiply-add contraction in this file: the kernel is instantiated per
// streaming form, tile and cache hint, and every instantiation must round
// alike (fused multiply-adds formed differently per instantiation differ in
// the last bit).  The collision writes its multiply-adds explicitly.
#pragma clang fp contract(off)
#include <algorithm>

#include "lbib_dev.h"

namespace lbib {

constexpr int kCap = 256;  // lanes per workgroup = nodes per tile
constexpr int kXcdBands = 2;   // bands of tiles per XCD

// mode bits: 1 = record which tiles carried IB force (touched), 2 = clear the
// bin counts this launch consumed; mode >> 2 selects tiles: 0 all, 1 only
// those without registered markers, 2 only those with.  mode = 0
// (measurement launches): the bins are left in place and the caller points
// U at a spare buffer, so the simulation state is untouched.
// Adds the markers of a tile's bin (entries lane, lane + kCap, ...) to the
// tile's fixed-point force accumulators.  Stencil weights: the Roma kernel's
// per-axis products (MLS = false) or the nine MLS weights; the transfer is
// chosen per instance outside the loop, so each loop is straight-line code.
template <bool MLS, int TX, int TY, typename T>
__device__ __forceinline__ void spread_entries(const Ptrs<T>& p, const int* bin, int M, int lane,
                                               double sc, int x0, int y0, int nx, int ny, bool pery,
                                               unsigned long long* s_ax, unsigned long long* s_ay) {
  const int nm = p.nm_total;
  for (int j = lane; j < M; j += kCap) {
    const int m = bin[j];
    const int cx = p.cx[m], cy = p.cy[m];
    const double fx = p.fx[m] * sc, fy = p.fy[m] * sc;
    double wxa[3], wyb[3], ph[9];
    if constexpr (MLS) {
#pragma unroll
      for (int k = 0; k < 9; ++k) ph[k] = p.wx[k * nm + m];
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        wxa[k] = p.wx[k * nm + m];
        wyb[k] = p.wy[k * nm + m];
      }
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      int row = cy + b - 1;
      if (pery) row = wrap_i(row, ny);
      const int ly = row - y0;
      if (ly < 0 || ly >= TY) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int lx = wrap_i(cx + a - 1, nx) - x0;
        if (lx < 0 || lx >= TX) continue;
        const double w = MLS ? ph[3 * b + a] : wxa[a] * wyb[b];
        atomicAdd(&s_ax[ly * TX + lx], (unsigned long long)__double2ll_rn(fx * w));
        atomicAdd(&s_ay[ly * TX + lx], (unsigned long long)__double2ll_rn(fy * w));
      }
    }
  }
}

// NT bit 0: the population loads carry the non-temporal hint.  Pull
// streaming is a permutation of the nodes, so every population is read
// exactly once per step and its cache line is worth nothing to this kernel
// afterwards; measured on one lattice the hint gains a few per cent, on
// batches of many small lattices it loses.  NT bit 1: the population stores
// carry it too, which measured faster on a lattice whose populations stay in
// the last-level cache and much slower on one larger than it.  The host
// chooses per context.
// One tile, the g-th of the launch's virtual grid of 8 * kXcdBands * band
// workgroups (band = tiles per band): g mod 8 is the XCD the hardware gives
// workgroup g, whose (g / 8)-th workgroup takes the tiles of its bands in
// order.  Returns early (every lane, or a lane outside the lattice after the
// workgroup's last barrier).
template <typename T, int TX, int TY, int NT, int SCH>
__device__ __forceinline__ void lb_tile(Ptrs<T>& p, int g, int ntiles_total, int band, int mode) {
  static_assert(TX * TY == kCap, "one lane per LDS slot");
  const int q = (g >> 3) / band, r = (g >> 3) - q * band;
  const int tile = (q * 8 + (g & 7)) * band + r;
  if (tile >= ntiles_total) return;
  const int cls = mode >> 2;
  if (cls != 0 && (cls == 1) == (p.cnt_cur[tile] > 0)) return;   // the other launch's tile
  // a single lattice needs no lookup: its parameters are the first load
  const int inst = p.ninst == 1 ? 0 : p.tile_inst[tile];
  // by value: the fields are read once, before the stores below (through a
  // reference they are re-read, and waited for, after every store)
  const LatDev L = p.lat[inst];
  const int nx = L.nx, ny = L.ny, ntx = L.ntx, pitch = L.pitch;
  const bool pery = L.periodic_y != 0;
  const int local = tile - L.tile_base;
  const int tx = local % ntx, ty = local / ntx;
  const int lane = threadIdx.x;
  const int x = tx * TX + (lane % TX);
  const int y = ty * TY + (lane / TX);
  const bool inside = x < nx && y < ny;

  // ---- pull streaming with halfway bounce-back, issued first so that the
  // population loads are in flight while the tile's IB force is gathered.
  // Addresses: one uniform pointer per population plane plus a 32-bit
  // element offset inside the plane (a plane holds at most 2^31 nodes).
  const long long N = L.plane;
  // two buffers (SCH 0): A and B never alias; in place (SCH 1, 2) the one
  // array is accessed through F only
  const T* __restrict__ A = p.A + 9 * L.node_base;
  T* __restrict__ B = p.B + 9 * L.node_base;
  T* const F = p.B + 9 * L.node_base;
  const unsigned o0 = (unsigned)y * (unsigned)pitch + (unsigned)x;
  // neighbour columns (periodic) and rows: periodic rows wrap, otherwise a
  // row beyond a wall is replaced by the node's own row and the lanes
  // concerned take the bounced value instead (lo / hi: the node lies on the
  // first / last row of a walled lattice)
  const bool lo = !pery && y == 0, hi = !pery && y == ny - 1;
  const unsigned cm = x == 0 ? nx - 1 : x - 1, cp = x == nx - 1 ? 0 : x + 1;
  const unsigned rm = (unsigned)(y == 0 ? (pery ? ny - 1 : y) : y - 1) * (unsigned)pitch;
  const unsigned rp = (unsigned)(y == ny - 1 ? (pery ? 0 : y) : y + 1) * (unsigned)pitch;
  const unsigned r0 = (unsigned)y * (unsigned)pitch;
  T h[kQ];
  if (inside) {
    // all nine loads issued back to back; the bounced values of the wall
    // rows are fetched afterwards (uniform per wave when a wave is one row)
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      if constexpr (SCH == 2) {
        h[i] = F[i * N + o0];   // node-local pass: slot i of the node itself
      } else {
        const unsigned c = ex(i) > 0 ? cm : (ex(i) < 0 ? cp : (unsigned)x);
        const unsigned r = ey(i) > 0 ? rm : (ey(i) < 0 ? rp : r0);
        if constexpr (SCH == 0) {
          const T* src = A + i * N + (r + c);
          h[i] = (NT & 1) ? __builtin_nontemporal_load(src) : *src;
        } else {
          h[i] = F[opp(i) * N + (r + c)];
        }
      }
    }
    if constexpr (SCH != 2) {
      if (lo || hi) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
          if ((ey(i) > 0 && lo) || (ey(i) < 0 && hi))
            h[i] = SCH == 0 ? A[opp(i) * N + o0] : F[i * N + o0];   // h*_opp(i) of the node
        }
      }
    }
  }

  // ---- Eulerian force: drive plus the markers whose stencil overlaps this tile.
  // Contributions F_k w_a w_b are accumulated in LDS as 64-bit fixed-point
  // integers: integer addition is associative, so the sum at every node is
  // the same whatever order the lanes add in (deterministic, no global
  // atomics).  The scale 2^S is chosen per tile from the largest force of the
  // instance and the bin size so the accumulator cannot overflow:
  // |sum| <= M * max|F| < 2^61.
  const int Mreg = p.cnt_cur[tile];
  const bool full = Mreg > p.bin_cap;          // registrations were dropped
  const int M = full ? p.bin_cap : Mreg;
  const int* bin = p.bin_cur + (long long)tile * p.bin_cap;
  T Fx = T(L.gx), Fy = T(L.gy);
  if (M > 0) {
    __shared__ unsigned long long s_ax[kCap], s_ay[kCap];
    // largest |F| any body of this instance handed to the fluid this step
    // (recorded by the body kernel); non-finite means a broken force
    const double fmax_t = __longlong_as_double((long long)p.fmax_bits[inst]);
    s_ax[lane] = 0ull;
    s_ay[lane] = 0ull;
    __syncthreads();
    if (full || !isfinite(fmax_t)) {
      Fx = Fy = T(NAN);
    } else if (fmax_t > 0.0) {
      int e;
      frexp(fmax_t * (double)M, &e);
      const double sc = ldexp(1.0, 61 - e);
      const int x0 = tx * TX, y0 = ty * TY;
      if (L.transfer == LBIB_TRANSFER_MLS)
        spread_entries<true, TX, TY>(p, bin, M, lane, sc, x0, y0, nx, ny, pery, s_ax, s_ay);
      else
        spread_entries<false, TX, TY>(p, bin, M, lane, sc, x0, y0, nx, ny, pery, s_ax, s_ay);
      __syncthreads();
      const double isc = 1.0 / sc;
      Fx = T(L.gx + (double)(long long)s_ax[lane] * isc);
      Fy = T(L.gy + (double)(long long)s_ay[lane] * isc);
    }
  }
  if (lane == 0) {
    // every lane has read the count: clear it for the next use of this set
    if ((mode & 2) && Mreg > 0) p.cnt_cur[tile] = 0;
    if (mode & 1) p.touched[tile] = Mreg > 0;
  }
  if (!inside) return;
  // velocity walls: the populations from beyond the wall, set now that the
  // node's force is known (the pull above loaded placeholders)
  if (L.wall_mode == 1 && !pery && (y == 0 || y == ny - 1))
    zou_he_fill(h, y == 0, T(y == 0 ? L.u_wall_lo : L.u_wall_hi), Fx, Fy);

  // ---- moments and forced BGK collision, written with explicit
  // multiply-adds (the same rounding in every instantiation)
  const T drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
  const T rho = T(1) + drho;
  const T jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
  const T jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
  T inv_rho;
  if constexpr (sizeof(T) == 4) inv_rho = __builtin_amdgcn_rcpf(rho);   // hardware reciprocal, 1 ulp
  else inv_rho = T(1) / rho;
  const T ux = fma(T(0.5), Fx, jx) * inv_rho;
  const T uy = fma(T(0.5), Fy, jy) * inv_rho;
  // per node: 3u, 3/2 |u|^2 and u.F; per workgroup: the relaxation weights
  const T ux3 = T(3) * ux, uy3 = T(3) * uy;
  const T uu15 = T(1.5) * fma(ux, ux, uy * uy);
  const T uF = fma(ux, Fx, uy * Fy);
  const T omega = T(L.omega);
  const T keep = T(1) - omega;
  const T pre3 = T(3) * T(L.pre);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    // h* = (1 - 1/tau) h + w/tau (drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u^2))
    //      + 3 (1 - 1/(2 tau)) w (3 (e.u)(e.F) + e.F - u.F)
    // (Guo's source [3 (e - u) + 9 (e.u) e].F regrouped); the zero and unit
    // components of e_i are folded by hand, since IEEE rules keep the
    // compiler from dropping 0 * u
    T q, s;
    if (ex(i) == 0 && ey(i) == 0) {
      q = fma(-rho, uu15, drho);
      s = -uF;
    } else {
      const T eu3 = ex(i) == 0 ? T(ey(i)) * uy3
                  : (ey(i) == 0 ? T(ex(i)) * ux3 : T(ex(i)) * ux3 + T(ey(i)) * uy3);
      const T eF = ex(i) == 0 ? T(ey(i)) * Fy
                 : (ey(i) == 0 ? T(ex(i)) * Fx : T(ex(i)) * Fx + T(ey(i)) * Fy);
      q = fma(rho, fma(eu3, fma(T(0.5), eu3, T(1)), -uu15), drho);
      s = fma(eu3, eF, eF - uF);
    }
    const T hn = fma(keep, h[i], fma(omega * wq<T>(i), q, (pre3 * wq<T>(i)) * s));
    if constexpr (SCH == 0) {
      T* dst = B + i * N + o0;
      if (NT & 2) __builtin_nontemporal_store(hn, dst);
      else *dst = hn;
    } else if constexpr (SCH == 2) {
      F[opp(i) * N + o0] = hn;
    } else {
      // neighbour pass: slot i of x + e_i, or slot opp(i) of the node when
      // x + e_i lies beyond a wall.  Every store depends on all nine loads
      // above, and no other node of the step touches these slots.
      if ((ey(i) > 0 && hi) || (ey(i) < 0 && lo)) {
        F[opp(i) * N + o0] = hn;
      } else {
        const unsigned c = ex(i) > 0 ? cp : (ex(i) < 0 ? cm : (unsigned)x);
        const unsigned r = ey(i) > 0 ? rp : (ey(i) < 0 ? rm : r0);
        F[i * N + (r + c)] = hn;
      }
    }
  }
  if (M > 0) {
    T* U = p.U + 2 * L.node_base;
    U[o0] = ux;
    U[N + o0] = uy;
  }
}

// One workgroup per tile (the default launch).
template <typename T, int TX, int TY, int NT, int SCH>
__global__ __launch_bounds__(TX * TY) void k_lb_fused(Ptrs<T> p, int ntiles_total, int band, int mode) {
  lb_tile<T, TX, TY, NT, SCH>(p, blockIdx.x, ntiles_total, band, mode);
}

// Persistent launch: a fixed grid (a multiple of 8 workgroups, sized by the
// host as a number of workgroups per CU) walks the virtual grid with stride
// gridDim.x, so workgroup b keeps to the tiles of XCD b mod 8.  The barrier
// between tiles frees the LDS accumulators for the next one.
template <typename T, int TX, int TY, int NT>
__global__ __launch_bounds__(TX * TY) void k_lb_persistent(Ptrs<T> p, int ntiles_total, int band, int mode) {
  const int gtot = 8 * kXcdBands * band;
  for (int g = blockIdx.x; g < gtot; g += gridDim.x) {
    lb_tile<T, TX, TY, NT, 0>(p, g, ntiles_total, band, mode);
    __syncthreads();
  }
}

// Physical fields of the last step from its post-collision populations:
// collision conserves mass, so rho = 1 + sum h*; the forced BGK step leaves
// a post-collision momentum sum h* e = rho u + F/2, so where F is the uniform
// drive alone rho u = sum h* e - g/2.  Touched tiles take u from the velocity
// buffer written by the fused kernel (their F includes the IB forces).
// Outputs are dense [y][x] arrays of nx * ny values.
template <typename T>
__global__ void k_fields(Ptrs<T> p, int inst, int TX, int TY, double* rho_o, double* ux_o,
                         double* uy_o) {
  const LatDev& L = p.lat[inst];
  const long long N = L.plane;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)L.nx * L.ny) return;
  const int x = (int)(k % L.nx), y = (int)(k / L.nx);
  const long long node = (long long)y * L.pitch + x;
  const T* A = p.A + 9 * L.node_base;  // A holds the newest post-collision populations
  double h[kQ];
  for (int i = 0; i < kQ; ++i) h[i] = double(A[post_slot(p.sch, i, x, y, L.nx, L.ny, L.pitch, L.periodic_y != 0, N)]);
  double drho = 0, jx = 0, jy = 0;
  for (int i = 0; i < kQ; ++i) {
    drho += h[i];
    jx += ex(i) * h[i];
    jy += ey(i) * h[i];
  }
  const double rho = 1.0 + drho;
  // touched tile: the fused kernel applied IB forces there in the last step
  const bool touched = p.touched[L.tile_base + (y / TY) * L.ntx + (x / TX)] != 0;
  double ux, uy;
  if (touched) {
    const T* U = p.U + 2 * L.node_base;
    ux = double(U[node]);
    uy = double(U[N + node]);
  } else {
    ux = (jx - 0.5 * L.gx) / rho;
    uy = (jy - 0.5 * L.gy) / rho;
  }
  if (rho_o) rho_o[k] = rho;
  if (ux_o) ux_o[k] = ux;
  if (uy_o) uy_o[k] = uy;
}

// Deterministic two-pass reduction of mass, momentum, min rho, max |u| and
// non-finite count over all nodes of all instances (diagnostics/watchdog).
// Pass 1: fixed tree per workgroup into red[6 * block]; pass 2 in order.
template <typename T>
__global__ __launch_bounds__(256) void k_diag1(Ptrs<T> p, long long nodes_total, double* part) {
  __shared__ double s[6][256];
  const int t = threadIdx.x;
  double m = 0, px = 0, py = 0, rmin = 1e300, umax = 0, bad = 0;
  for (long long g = (long long)blockIdx.x * 256 + t; g < nodes_total; g += (long long)gridDim.x * 256) {
    // locate instance: linear scan is fine for diagnostics (few instances)
    int inst = 0;
    while (inst + 1 < p.ninst && p.lat[inst + 1].node_base <= g) ++inst;
    const LatDev& L = p.lat[inst];
    const long long N = L.plane;
    const long long node = g - L.node_base;
    if (node % L.pitch >= L.nx) continue;   // row padding
    const int x = (int)(node % L.pitch), y = (int)(node / L.pitch);
    const T* A = p.A + 9 * L.node_base;
    double drho = 0, jx = 0, jy = 0;
    bool fin = true;
    for (int i = 0; i < kQ; ++i) {
      double v = double(A[post_slot(p.sch, i, x, y, L.nx, L.ny, L.pitch, L.periodic_y != 0, N)]);
      fin &= isfinite(v);
      drho += v;
      jx += ex(i) * v;
      jy += ey(i) * v;
    }
    const double rho = 1.0 + drho;
    // momentum of the post-collision state minus the drive's half force;
    // exact for nodes without IB force, diagnostic elsewhere
    const double rux = jx - 0.5 * L.gx, ruy = jy - 0.5 * L.gy;
    if (!fin) { bad += 1; continue; }
    m += rho;
    px += rux;
    py += ruy;
    rmin = fmin(rmin, rho);
    umax = fmax(umax, sqrt(rux * rux + ruy * ruy) / rho);
  }
  s[0][t] = m; s[1][t] = px; s[2][t] = py; s[3][t] = rmin; s[4][t] = umax; s[5][t] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      s[0][t] += s[0][t + w]; s[1][t] += s[1][t + w]; s[2][t] += s[2][t + w];
      s[3][t] = fmin(s[3][t], s[3][t + w]); s[4][t] = fmax(s[4][t], s[4][t + w]);
      s[5][t] += s[5][t + w];
    }
    __syncthreads();
  }
  if (t == 0)
    for (int k = 0; k < 6; ++k) part[6 * blockIdx.x + k] = s[k][0];
}

__global__ void k_diag2(const double* part, int nblk, double* out) {
  if (threadIdx.x != 0) return;
  double m = 0, px = 0, py = 0, rmin = 1e300, umax = 0, bad = 0;
  for (int b = 0; b < nblk; ++b) {
    m += part[6 * b]; px += part[6 * b + 1]; py += part[6 * b + 2];
    rmin = fmin(rmin, part[6 * b + 3]); umax = fmax(umax, part[6 * b + 4]); bad += part[6 * b + 5];
  }
  out[0] = m; out[1] = px; out[2] = py; out[3] = rmin; out[4] = umax; out[5] = bad;
}

// Populations of instance `inst` between the state in p.A (scheme p.sch) and
// a buffer in scheme-0 order (every node's h*_i in slot i): to = 1 copies the
// state into buf, to = 0 writes buf into the state.  Row padding is left
// alone.
template <typename T>
__global__ void k_canon(Ptrs<T> p, int inst, T* buf, int to) {
  const LatDev& L = p.lat[inst];
  const long long N = L.plane;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)L.nx * L.ny) return;
  const int x = (int)(k % L.nx), y = (int)(k / L.nx);
  const long long node = (long long)y * L.pitch + x;
  T* A = p.A + 9 * L.node_base;
  T* C = buf + 9 * L.node_base;
  const bool pery = L.periodic_y != 0;
  for (int i = 0; i < kQ; ++i) {
    const long long s = post_slot(p.sch, i, x, y, L.nx, L.ny, L.pitch, pery, N);
    if (to) C[i * N + node] = A[s];
    else A[s] = C[i * N + node];
  }
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_lb_fused(const Ptrs<T>& p, const StepArgs& a, hipStream_t s, int mode,
                     hipEvent_t ev0, hipEvent_t ev1) {
  const int band = (a.ntiles_total + 8 * kXcdBands - 1) / (8 * kXcdBands);
  const int vgrid = 8 * kXcdBands * band;
  // persistent: wpc workgroups per CU, a multiple of 8, at most the virtual
  // grid; two-buffer streaming only
  const bool persist = a.lb_wpc > 0 && p.sch == 0;
  const int pgrid = std::min(vgrid, 8 * ((a.lb_wpc * a.n_cu + 7) / 8));
  dim3 grid(persist ? pgrid : vgrid), block(kCap);
  // the optional events are bound to the dispatch itself, so their elapsed
  // time is the kernel's execution time and not that of separate markers
#define LBIB_LB1(KERNEL, ...)                                                                    \
  hipExtLaunchKernelGGL((KERNEL<T, __VA_ARGS__>), grid, block, 0, s, ev0, ev1, 0, p,             \
                        a.ntiles_total, band, mode)
#define LBIB_LB(TXv, TYv)                                                                        \
  do {                                                                                          \
    if (p.sch == 1) LBIB_LB1(k_lb_fused, TXv, TYv, 0, 1);                                       \
    else if (p.sch == 2) LBIB_LB1(k_lb_fused, TXv, TYv, 0, 2);                                  \
    else if (persist) {                                                                         \
      if (a.nt_mode == 3) LBIB_LB1(k_lb_persistent, TXv, TYv, 3);                               \
      else if (a.nt_mode == 1) LBIB_LB1(k_lb_persistent, TXv, TYv, 1);                          \
      else LBIB_LB1(k_lb_persistent, TXv, TYv, 0);                                              \
    } else {                                                                                    \
      if (a.nt_mode == 3) LBIB_LB1(k_lb_fused, TXv, TYv, 3, 0);                                 \
      else if (a.nt_mode == 1) LBIB_LB1(k_lb_fused, TXv, TYv, 1, 0);                            \
      else LBIB_LB1(k_lb_fused, TXv, TYv, 0, 0);                                                \
    }                                                                                           \
  } while (0)
  if (a.tile_x == 64 && a.tile_y == 4) LBIB_LB(64, 4);
  else if (a.tile_x == 128 && a.tile_y == 2) LBIB_LB(128, 2);
  else if (a.tile_x == 32 && a.tile_y == 8) LBIB_LB(32, 8);
  else LBIB_LB(256, 1);
#undef LBIB_LB
#undef LBIB_LB1
}

template <typename T>
void launch_fields(const Ptrs<T>& p, const StepArgs& a, int inst, double* rho, double* ux,
                   double* uy, int nx, int ny, long long, hipStream_t s) {
  long long n = (long long)nx * ny;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(k_fields<T>, grid, block, 0, s, p, inst, a.tile_x, a.tile_y, rho, ux, uy);
}

template <typename T>
void launch_diag(const Ptrs<T>& p, const StepArgs&, long long nodes_total, double* out,
                 hipStream_t s) {
  const int nblk = 1024;
  hipLaunchKernelGGL(k_diag1<T>, dim3(nblk), dim3(256), 0, s, p, nodes_total, p.red);
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(64), 0, s, p.red, nblk, out);
}

template <typename T>
void launch_canon(const Ptrs<T>& p, int ninst, const long long* inst_nodes, T* buf, int to,
                  hipStream_t s) {
  for (int i = 0; i < ninst; ++i) {
    const unsigned g = (unsigned)((inst_nodes[i] + 255) / 256);
    if (g) hipLaunchKernelGGL(k_canon<T>, dim3(g), dim3(256), 0, s, p, i, buf, to);
  }
}
template void launch_canon<float>(const Ptrs<float>&, int, const long long*, float*, int, hipStream_t);
template void launch_canon<double>(const Ptrs<double>&, int, const long long*, double*, int, hipStream_t);

template void launch_lb_fused<float>(const Ptrs<float>&, const StepArgs&, hipStream_t, int,
                                     hipEvent_t, hipEvent_t);
template void launch_lb_fused<double>(const Ptrs<double>&, const StepArgs&, hipStream_t, int,
                                      hipEvent_t, hipEvent_t);
template void launch_fields<float>(const Ptrs<float>&, const StepArgs&, int, double*, double*,
                                   double*, int, int, long long, hipStream_t);
template void launch_fields<double>(const Ptrs<double>&, const StepArgs&, int, double*, double*,
                                    double*, int, int, long long, hipStream_t);
template void launch_diag<float>(const Ptrs<float>&, const StepArgs&, long long, double*, hipStream_t);
template void launch_diag<double>(const Ptrs<double>&, const StepArgs&, long long, double*, hipStream_t);

}  // namespace lbib
