// k_lagrangian.hip - Lagrangian side of the LB-IB step (gfx950), float64.
//
// Per time step n (the order is the one used throughout the library):
//   k_bin_bonds   one workgroup per lattice instance:
//                   - stencil of every marker: centre node floor(X + 1/2) and the
//                     3+3 weights of the Roma 3-point kernel;
//                   - marker bins per lattice tile (counting sort, each bin then
//                     ordered by marker id so spreading sums in a fixed order);
//                   - bond kinetics: rupture pass, then formation pass in
//                     ascending ligand order (Sec. 2.2 Wall-Particle Interaction),
//                     with Philox4x32-10 uniforms keyed by (step, ligand).
//   k_body        one workgroup per body:
//                   - membrane strain, bending and area forces (Eqs. strainFor,
//                     bendFor, areaFor), adhesion springs (Eq. adhFor);
//                   - particles: probe pressure/viscous loads (Eqs. hydroForP,
//                     hydroForNu) from the pre-forcing fluid state, soft Verlet
//                     position update (Eqs. newtonSoft, verletPos) or rigid BDF2
//                     (Eqs. linearVelRig, angularVelRig), weak-coupling force.
//   (the fused lattice kernel runs here)
//   k_advance     one lane per marker: red cells by the kinematic IB
//                 (Eq. kinematicPos), particles adopt their new positions.
#include "lbib_dev.h"

namespace lbib {

// ------------------------------------------------------------------ helpers
// Populations at a node after streaming, before forcing (walls: bounce-back).
template <typename T>
__device__ inline void pulled_moments(const T* A, long long N, int nx, int ny, bool pery, int x,
                                      int y, double& drho, double& jx, double& jy) {
  drho = 0.0; jx = 0.0; jy = 0.0;
  const long long node = (long long)y * nx + x;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    int xs = wrap_i(x - ex(i), nx);
    int ys = y - ey(i);
    double h;
    if (ys < 0 || ys >= ny) {
      if (pery) h = double(A[i * N + (long long)wrap_i(ys, ny) * nx + xs]);
      else h = double(A[opp(i) * N + node]);
    } else {
      h = double(A[i * N + (long long)ys * nx + xs]);
    }
    drho += h;
    jx += ex(i) * h;
    jy += ey(i) * h;
  }
}

// rho*, u* of the pre-forcing state: u* = (sum f e + g/2) / rho*.
template <typename T>
__device__ inline void node_star(const T* A, const LatDev& L, int x, int y, double& rho,
                                 double& ux, double& uy) {
  const long long N = (long long)L.nx * L.ny;
  double drho, jx, jy;
  pulled_moments(A, N, L.nx, L.ny, L.periodic_y != 0, x, y, drho, jx, jy);
  rho = 1.0 + drho;
  ux = (jx + 0.5 * L.gx) / rho;
  uy = (jy + 0.5 * L.gy) / rho;
}

// Kernel interpolant of rho*, u* at a point and (optionally) its gradient.
template <typename T>
__device__ inline void interp_star(const T* A, const LatDev& L, double X, double Y, bool grad,
                                   double& rho, double& ux, double& uy, double g[4]) {
  const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
  rho = 0; ux = 0; uy = 0;
  g[0] = g[1] = g[2] = g[3] = 0;  // du/dx, du/dy, dv/dx, dv/dy
  const bool pery = L.periodic_y != 0;
  for (int b = 0; b < 3; ++b) {
    const double ry = cyr + (b - 1);
    int row = (int)ry;
    if (pery) row = wrap_i(row, L.ny);
    else if (row < 0 || row >= L.ny) continue;
    const double wy = roma_phi(ry - Y), dwy = roma_dphi(ry - Y);
    for (int a = 0; a < 3; ++a) {
      const double rx = cxr + (a - 1);
      const int col = wrap_i((int)rx, L.nx);
      const double wx = roma_phi(rx - X), dwx = roma_dphi(rx - X);
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
  const double yw = wall == 0 ? -0.5 : L.ny - 0.5;
  const double dy = cy - yw;
  return sqrt(dx * dx + dy * dy);
}

__device__ inline double ligand_cx(const Ptrs<float>&, const double* x, int v0, int nv, int e) {
  return 0.5 * (x[v0 + e] + x[v0 + (e + 1) % nv]);
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

// ---------------------------------------------------------------- k_bin_bonds
template <typename T>
__global__ __launch_bounds__(1024) void k_bin_bonds(Ptrs<T> p, int TX, int TY) {
  __shared__ int s_tmp[1024];
  const int inst = blockIdx.x;
  const LatDev& L = p.lat[inst];
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long n = p.step_next[inst];
  __syncthreads();
  if (tid == 0) {
    p.step_cur[inst] = n;
    p.step_next[inst] = n + 1;
  }
  const int nx = L.nx, ny = L.ny, ntx = L.ntx;
  const bool pery = L.periodic_y != 0;
  const int ntiles = L.ntx * L.nty;
  int* cnt = p.bin_cnt + L.tile_base;
  int* off = p.bin_off + L.bin_base;
  const int nm = p.nm_total;
  for (int t = tid; t < ntiles; t += nt) cnt[t] = 0;
  __syncthreads();

  // 1. stencils and bin counts
  for (int m = tid; m < L.n_markers; m += nt) {
    const int gm = L.marker_base + m;
    const double X = p.x[gm], Y = p.y[gm];
    const double cxr = floor(X + 0.5), cyr = floor(Y + 0.5);
    for (int a = 0; a < 3; ++a) {
      p.wx[a * nm + gm] = roma_phi((cxr + (a - 1)) - X);
      const double ry = cyr + (a - 1);
      const bool valid = pery || (ry >= 0.0 && ry < (double)ny);
      p.wy[a * nm + gm] = valid ? roma_phi(ry - Y) : 0.0;
    }
    const int cx = wrap_i((int)cxr, nx);
    int cy;
    if (pery) cy = wrap_i((int)cyr, ny);
    else cy = (int)fmin(fmax(cyr, -4.0), (double)(ny + 3));
    p.cx[gm] = cx;
    p.cy[gm] = cy;
    const int tx = cx / TX;
    const int ty = min(max(cy, 0), ny - 1) / TY;
    atomicAdd(&cnt[ty * ntx + tx], 1);
  }
  __syncthreads();

  // 2. exclusive scan -> bin offsets (global marker ids); counts become cursors
  {
    const int chunk = (ntiles + nt - 1) / nt;
    const int lo = min(tid * chunk, ntiles), hi = min(lo + chunk, ntiles);
    int sum = 0;
    for (int t = lo; t < hi; ++t) sum += cnt[t];
    int run = block_exclusive_scan(sum, s_tmp) + L.marker_base;
    for (int t = lo; t < hi; ++t) {
      off[t] = run;
      run += cnt[t];
      cnt[t] = 0;
    }
    if (tid == nt - 1) off[ntiles] = L.marker_base + L.n_markers;
  }
  __syncthreads();

  // 3. scatter (arbitrary order inside a bin)
  for (int m = tid; m < L.n_markers; m += nt) {
    const int gm = L.marker_base + m;
    const int tx = p.cx[gm] / TX;
    const int ty = min(max(p.cy[gm], 0), ny - 1) / TY;
    const int key = ty * ntx + tx;
    const int pos = atomicAdd(&cnt[key], 1);
    p.bin_tmp[off[key] + pos] = gm;
  }
  __syncthreads();

  // 4. order every bin by marker id (rank by counting; ids are unique)
  {
    const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
    for (int base = wave * 64; base < ntiles; base += nwave * 64) {
      const int b = base + lane;
      int c = 0, s0 = 0;
      if (b < ntiles) {
        s0 = off[b];
        c = off[b + 1] - s0;
        if (c == 1) p.bin_idx[s0] = p.bin_tmp[s0];
      }
      unsigned long long mask = __ballot(c > 1);
      while (mask) {
        const int k = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const int bs = __shfl(s0, k), bc = __shfl(c, k);
        for (int i = lane; i < bc; i += 64) {
          const int id = p.bin_tmp[bs + i];
          int rank = 0;
          for (int j = 0; j < bc; ++j) rank += p.bin_tmp[bs + j] < id;
          p.bin_idx[bs + rank] = id;
        }
      }
    }
  }

  // 5. bond kinetics
  if (L.n_lig == 0 || L.freeze) return;
  __syncthreads();
  const double y_cr = L.y_cr;
  unsigned long long ties = 0;
  for (int l = tid; l < L.n_lig; l += nt) {
    const int gl = L.lig_base + l;
    const int b = p.lig_body[gl], e = p.lig_elem[gl];
    const BodyDev& Bd = p.body[b];
    const int v0 = Bd.v0, nv = Bd.nv;
    const double cx = 0.5 * (p.x[v0 + e] + p.x[v0 + (e + 1) % nv]);
    const double cy = 0.5 * (p.y[v0 + e] + p.y[v0 + (e + 1) % nv]);
    const int r = p.l2r[gl];
    int flag = 0;
    if (r >= 0) {
      const int wall = r < L.n_rec0 ? 0 : 1;
      const double yl = bond_len(cx, cy, p.rec_x[L.rec_base + r], wall, L);
      const double sig = Bd.sigma, sts = L.sigma_ts_frac * sig;
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
      const double d0 = cy + 0.5, d1 = (ny - 0.5) - cy;
      const int wall = d0 <= d1 ? 0 : 1;
      const double d = wall == 0 ? d0 : d1;
      if (d < y_cr) flag = 1 + wall;
    }
    p.lig_flag[gl] = flag;
  }
  __syncthreads();
  if (tid == 0) {
    for (int l = 0; l < L.n_lig; ++l) {
      const int gl = L.lig_base + l;
      const int flag = p.lig_flag[gl];
      if (!flag) continue;
      const int wall = flag - 1;
      const int b = p.lig_body[gl], e = p.lig_elem[gl];
      const BodyDev& Bd = p.body[b];
      const int v0 = Bd.v0, nv = Bd.nv;
      const double cx = 0.5 * (p.x[v0 + e] + p.x[v0 + (e + 1) % nv]);
      const double cy = 0.5 * (p.y[v0 + e] + p.y[v0 + (e + 1) % nv]);
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
      const double sig = Bd.sigma, sts = L.sigma_ts_frac * sig;
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

// ---------------------------------------------------------------- k_body
// Block reduction (fixed tree order) of NV values per thread slot.
template <int NV>
__device__ inline void block_sum(double (*s)[256], double* v) {
  const int t = threadIdx.x;
  for (int k = 0; k < NV; ++k) s[k][t] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < NV; ++k) s[k][t] += s[k][t + w];
    __syncthreads();
  }
  for (int k = 0; k < NV; ++k) v[k] = s[k][0];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_body(Ptrs<T> p) {
  __shared__ double s_red[3][256];
  __shared__ double s_rigid[6];
  const int b = blockIdx.x;
  BodyDev& Bd = p.body[b];
  const int kind = Bd.kind, nv = Bd.nv, v0 = Bd.v0, inst = Bd.inst;
  const LatDev& L = p.lat[inst];
  const bool first = p.step_cur[inst] == 0;
  const int t = threadIdx.x, nt = blockDim.x;
  const double* X = p.x + v0;
  const double* Y = p.y + v0;
  const T* A = p.A + 9 * L.node_base;
  const double nu = (L.tau - 0.5) / 3.0;

  // pass 1: element geometry (element v joins v -> v+1), bending data, area
  double shoe = 0.0;
  for (int v = t; v < nv; v += nt) {
    const int vp = v + 1 == nv ? 0 : v + 1, vm = v == 0 ? nv - 1 : v - 1;
    const double dxr = X[vp] - X[v], dyr = Y[vp] - Y[v];
    const double lr = sqrt(dxr * dxr + dyr * dyr);
    const double txr = dxr / lr, tyr = dyr / lr;
    const double dxl = X[v] - X[vm], dyl = Y[v] - Y[vm];
    const double ll = sqrt(dxl * dxl + dyl * dyl);
    const double txl = dxl / ll, tyl = dyl / ll;
    p.s_len[v0 + v] = lr;
    p.s_nx[v0 + v] = tyr;
    p.s_ny[v0 + v] = -txr;
    if (kind != kRigid) {
      const double cr = txl * tyr - tyl * txr;
      const double dt = txl * txr + tyl * tyr;
      const double th = atan2(cr, dt);
      const double nsx = tyl + tyr, nsy = -txl - txr;
      const double nn = sqrt(nsx * nsx + nsy * nsy);
      p.s_bc[v0 + v] = Bd.kb * (th - p.th0[v0 + v]);
      p.s_bnx[v0 + v] = nsx / nn;
      p.s_bny[v0 + v] = nsy / nn;
    }
    shoe += X[v] * Y[vp] - X[vp] * Y[v];
  }
  double area = shoe;
  block_sum<1>(s_red, &area);
  area *= 0.5;

  // pass 2: element loads (area penalty, adhesion springs, probe stresses)
  for (int l = t; l < nv; l += nt) {
    const int lp = l + 1 == nv ? 0 : l + 1;
    const double len = p.s_len[v0 + l], nxl = p.s_nx[v0 + l], nyl = p.s_ny[v0 + l];
    double fex = 0.0, fey = 0.0;
    if (kind != kRigid) {
      const double c = Bd.ka * (1.0 - area / Bd.A0) * Bd.p_ref * len;
      fex += c * nxl;
      fey += c * nyl;
    }
    if (kind != kRBC) {
      const double cx = 0.5 * (X[l] + X[lp]), cy = 0.5 * (Y[l] + Y[lp]);
      // adhesion spring on a bonded ligand element
      if (Bd.lig_stride > 0 && l % Bd.lig_stride == 0) {
        const int gl = Bd.lig_base + l / Bd.lig_stride;
        const int r = p.l2r[gl];
        if (r >= 0) {
          const int wall = r < L.n_rec0 ? 0 : 1;
          const double yl = bond_len(cx, cy, p.rec_x[L.rec_base + r], wall, L);
          const double s = Bd.sigma * (yl - L.y_eq);
          fex += s * nxl;
          fey += s * nyl;
        }
      }
      // probe 1.2 dx along the outward normal, kept inside the fluid
      const double qx = cx + 1.2 * nxl;
      double qy = cy + 1.2 * nyl;
      if (!L.periodic_y) qy = fmin(fmax(qy, 0.5), L.ny - 1.5);
      double rho, ux, uy, g[4];
      interp_star(A, L, qx, qy, true, rho, ux, uy, g);
      const double pr = (rho - 1.0) * (1.0 / 3.0);
      const double txx = 2.0 * nu * g[0], tyy = 2.0 * nu * g[3], txy = nu * (g[1] + g[2]);
      fex += (-pr * nxl + txx * nxl + txy * nyl) * len;
      fey += (-pr * nyl + txy * nxl + tyy * nyl) * len;
    }
    p.s_fex[v0 + l] = fex;
    p.s_fey[v0 + l] = fey;
  }
  __syncthreads();

  if (kind == kRigid) {
    double r3[3] = {0.0, 0.0, 0.0};
    for (int l = t; l < nv; l += nt) {
      const int lp = l + 1 == nv ? 0 : l + 1;
      const double fex = p.s_fex[v0 + l], fey = p.s_fey[v0 + l];
      const double cx = 0.5 * (X[l] + X[lp]) - Bd.xc, cy = 0.5 * (Y[l] + Y[lp]) - Bd.yc;
      r3[0] += fex;
      r3[1] += fey;
      r3[2] += cx * fey - cy * fex;
    }
    block_sum<3>(s_red, r3);
    if (t == 0) {
      double U[2], Om;
      for (int k = 0; k < 2; ++k) {
        const double a = r3[k] / Bd.mass;
        U[k] = first ? Bd.U[k] + a : (2.0 / 3.0) * (2.0 * Bd.U[k] - 0.5 * Bd.Um[k] + a);
      }
      const double al = r3[2] / Bd.inertia;
      Om = first ? Bd.Om + al : (2.0 / 3.0) * (2.0 * Bd.Om - 0.5 * Bd.Omm + al);
      Bd.Um[0] = Bd.U[0]; Bd.Um[1] = Bd.U[1];
      Bd.U[0] = U[0]; Bd.U[1] = U[1];
      Bd.Omm = Bd.Om; Bd.Om = Om;
      Bd.xc += U[0];
      Bd.yc += U[1];
      Bd.theta += Om;
      s_rigid[0] = U[0]; s_rigid[1] = U[1]; s_rigid[2] = Om;
      s_rigid[3] = Bd.xc; s_rigid[4] = Bd.yc; s_rigid[5] = Bd.theta;
    }
    __syncthreads();
    const double U0 = s_rigid[0], U1 = s_rigid[1], Om = s_rigid[2];
    const double xc = s_rigid[3], yc = s_rigid[4], th = s_rigid[5];
    const double c = cos(th), s = sin(th);
    for (int v = t; v < nv; v += nt) {
      const int gm = v0 + v, vm = v == 0 ? nv - 1 : v - 1;
      const double rx = p.r0x[gm], ry = p.r0y[gm];
      const double xn = xc + (rx * c + ry * (-s));
      const double yn = yc + (rx * s + ry * c);
      const double relx = xn - xc, rely = yn - yc;
      const double ukx = U0 + Om * (-rely), uky = U1 + Om * relx;
      double rho, ux, uy, g[4];
      interp_star(A, L, X[v], Y[v], false, rho, ux, uy, g);
      const double ds = 0.5 * (p.s_len[v0 + vm] + p.s_len[gm]);
      p.xn[gm] = xn;
      p.yn[gm] = yn;
      p.fx[gm] = (2.0 * (ukx - ux)) * ds;
      p.fy[gm] = (2.0 * (uky - uy)) * ds;
    }
    return;
  }

  // membrane vertex forces: strain + bending + shared element loads
  for (int v = t; v < nv; v += nt) {
    const int gm = v0 + v;
    const int vm = v == 0 ? nv - 1 : v - 1, vp = v + 1 == nv ? 0 : v + 1;
    const int vmm = vm == 0 ? nv - 1 : vm - 1;
    // strain: element v pulls v along +t, element v-1 pulls v along -t
    const double lr = p.s_len[gm], ll = p.s_len[v0 + vm];
    const double sr = Bd.ks * (lr - p.l0[gm]);
    const double sl = Bd.ks * (ll - p.l0[v0 + vm]);
    // tangents from normals: t = (-n_y, n_x)
    double fx = sr * (-p.s_ny[gm]) - sl * (-p.s_ny[v0 + vm]);
    double fy = sr * p.s_nx[gm] - sl * p.s_nx[v0 + vm];
    // bending at v-1 (v is its right vertex), v, v+1 (v is its left vertex)
    {
      const double c = p.s_bc[v0 + vm];
      const double fr = p.s_len[v0 + vm] / (p.s_len[v0 + vmm] + p.s_len[v0 + vm]);
      fx += c * fr * p.s_bnx[v0 + vm];
      fy += c * fr * p.s_bny[v0 + vm];
    }
    {
      const double c = p.s_bc[gm];
      fx -= c * p.s_bnx[gm];
      fy -= c * p.s_bny[gm];
    }
    {
      const double c = p.s_bc[v0 + vp];
      const double fl = p.s_len[gm] / (p.s_len[gm] + p.s_len[v0 + vp]);
      fx += c * fl * p.s_bnx[v0 + vp];
      fy += c * fl * p.s_bny[v0 + vp];
    }
    fx += 0.5 * p.s_fex[gm] + 0.5 * p.s_fex[v0 + vm];
    fy += 0.5 * p.s_fey[gm] + 0.5 * p.s_fey[v0 + vm];
    if (kind == kRBC) {
      p.fx[gm] = fx;
      p.fy[gm] = fy;
    } else {
      double rho, ux, uy, g[4];
      interp_star(A, L, X[v], Y[v], false, rho, ux, uy, g);
      const double xn = X[v] + ux + 0.5 * fx / Bd.mv;
      const double yn = Y[v] + uy + 0.5 * fy / Bd.mv;
      // velocity imposed by the weak coupling: the vertex displacement of the
      // step (the second-order velocity of Eq. verletVel turns the coupling
      // into a marginally stable feedback that grows next to walls)
      const double Ux = xn - X[v], Uy = yn - Y[v];
      const double ds = 0.5 * (ll + lr);
      p.xn[gm] = xn;
      p.yn[gm] = yn;
      p.fx[gm] = (2.0 * (Ux - ux)) * ds;
      p.fy[gm] = (2.0 * (Uy - uy)) * ds;
    }
  }
}

// ---------------------------------------------------------------- k_advance
template <typename T>
__global__ __launch_bounds__(256) void k_advance(Ptrs<T> p) {
  const int gm = blockIdx.x * blockDim.x + threadIdx.x;
  if (gm >= p.nm_total) return;
  const int b = p.mbody[gm];
  const int kind = p.body[b].kind;
  const int inst = p.body[b].inst;
  const LatDev& L = p.lat[inst];
  const bool first = p.step_cur[inst] == 0;
  const double X = p.x[gm], Y = p.y[gm];
  double xn, yn;
  if (kind == kRBC) {
    const long long N = (long long)L.nx * L.ny;
    const T* U = p.U + 2 * L.node_base;
    const int nm = p.nm_total;
    const int cx = p.cx[gm], cy = p.cy[gm];
    double ux = 0.0, uy = 0.0;
    for (int b2 = 0; b2 < 3; ++b2) {
      int row = cy + b2 - 1;
      if (L.periodic_y) row = wrap_i(row, L.ny);
      else if (row < 0 || row >= L.ny) continue;
      const double wy = p.wy[b2 * nm + gm];
      for (int a = 0; a < 3; ++a) {
        const int col = wrap_i(cx + a - 1, L.nx);
        const double w = p.wx[a * nm + gm] * wy;
        const long long node = (long long)row * L.nx + col;
        ux += double(U[node]) * w;
        uy += double(U[N + node]) * w;
      }
    }
    if (first) {
      xn = X + ux;
      yn = Y + uy;
    } else {
      xn = (2.0 / 3.0) * (2.0 * X - 0.5 * p.xm[gm] + ux);
      yn = (2.0 / 3.0) * (2.0 * Y - 0.5 * p.ym[gm] + uy);
    }
  } else {
    xn = p.xn[gm];
    yn = p.yn[gm];
  }
  p.xm[gm] = X;
  p.ym[gm] = Y;
  p.x[gm] = xn;
  p.y[gm] = yn;
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_lagrangian(const Ptrs<T>& p, const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_bonds<T>, dim3(p.ninst), dim3(1024), 0, s, p, a.tile_x, a.tile_y);
  if (p.nbody_total > 0) hipLaunchKernelGGL(k_body<T>, dim3(p.nbody_total), dim3(256), 0, s, p);
}

template <typename T>
void launch_advance(const Ptrs<T>& p, hipStream_t s) {
  if (p.nm_total == 0) return;
  hipLaunchKernelGGL(k_advance<T>, dim3((p.nm_total + 255) / 256), dim3(256), 0, s, p);
}

template void launch_lagrangian<float>(const Ptrs<float>&, const StepArgs&, hipStream_t);
template void launch_lagrangian<double>(const Ptrs<double>&, const StepArgs&, hipStream_t);
template void launch_advance<float>(const Ptrs<float>&, hipStream_t);
template void launch_advance<double>(const Ptrs<double>&, hipStream_t);

}  // namespace lbib
