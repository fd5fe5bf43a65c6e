// k_repulsion.hip - repulsion between vertices of different bodies (gfx950),
// Sec. 2.2 "Particle-Particle Interaction", Eq. (repFor).
//
// A vertex at distance d < r_c from a vertex of another body is pushed along
// its own inward normal with magnitude c sqrt(1 / d^5) (lattice units); the
// magnitudes of all such neighbours add.  This kernel computes the summed
// magnitude S_v of every vertex at X^n; the body kernel applies -S_v n_v with
// the vertex normal it computes anyway (red cells and soft particles add it to
// the vertex force, rigid particles to their force and torque).
//
// One workgroup per body.  The marker bins of the step (every marker is
// registered in the tiles its 3x3 stencil overlaps) serve as the cell list:
//   1. the body's bounding box gives the tile columns and rows that can hold
//      the stencil centre of a vertex within r_c of it;
//   2. the bins of those tiles are read in parallel; a marker is taken from
//      the bin of the tile that holds its stencil centre only (so once), if
//      it belongs to another body and lies within r_c of the box;
//   3. the accepted candidates are ranked in LDS by (x, marker id), a total
//      order independent of the order the bins were filled in, so every sum
//      below is taken in a fixed order (deterministic results);
//   4. each vertex binary-searches the x window [x - r_c, x + r_c] and adds
//      the candidates closer than r_c.
// Distances use the minimum image along x, and along y on a periodic lattice.
// Candidate lists that exceed their fixed capacity are truncated and counted
// in *overflow, which the host reports.
#include "lbib_dev.h"

namespace lbib {

constexpr int kRepThreads = 256;
constexpr int kRepCand = 1024;   // candidate vertices of other bodies per body
constexpr int kRepAxis = 1024;   // tile columns / rows considered per body

__device__ inline double min_image_n(double d, int n) { return d - n * rint(d / n); }

// Does the circular arc of `len` nodes starting at node a (mod n) meet the
// node interval [s, e] (0 <= s <= e < n)?
__device__ inline bool arc_meets(int a, int len, int s, int e, int n) {
  if (len >= n) return true;
  int ds = s - a;
  ds = ds < 0 ? ds + n : ds;
  if (ds < len) return true;          // the arc reaches s
  int da = a - s;
  da = da < 0 ? da + n : da;
  return da <= e - s;                 // the arc starts inside [s, e]
}

// Block-wide exclusive prefix sum of one value per lane: *excl gets the sum
// over the lanes before this one; returns the total (every lane).
__device__ inline int block_scan(int v, int* s_tmp, int* excl) {
  const int t = threadIdx.x, n = kRepThreads;
  s_tmp[t] = v;
  __syncthreads();
  for (int o = 1; o < n; o <<= 1) {
    const int u = t >= o ? s_tmp[t - o] : 0;
    __syncthreads();
    s_tmp[t] += u;
    __syncthreads();
  }
  *excl = s_tmp[t] - v;
  const int total = s_tmp[n - 1];
  __syncthreads();
  return total;
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(kRepThreads) void k_repulsion(Ptrs<T> p) {
  __shared__ int s_col[kRepAxis], s_row[kRepAxis];
  __shared__ int s_tmp[kRepThreads];
  __shared__ int s_off[kRepThreads + 1];
  __shared__ double s_x[kRepCand], s_y[kRepCand];     // candidates as accepted
  __shared__ int s_id[kRepCand];
  __shared__ double s_sx[kRepCand], s_sy[kRepCand];   // ranked by (x, id)
  __shared__ double s_red[4][kRepThreads / 64];

  const int b = blockIdx.x;
  const BodyDev& B = p.body[b];
  const int nv = B.nv, v0 = B.v0;
  const LatDev& L = p.lat[B.inst];
  const int t = threadIdx.x, nt = kRepThreads;
  if (!(L.rep_coeff > 0.0)) {
    for (int v = t; v < nv; v += nt) p.frep[v0 + v] = 0.0;
    return;
  }
  const double coeff = L.rep_coeff, rc = L.rep_cutoff;
  const int nx = L.nx, ny = L.ny, ntx = L.ntx, nty = L.nty;
  const bool pery = L.periodic_y != 0;

  // ---- 1. bounding box of X^n (a body's chain is continuous: unwrapped)
  double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
  for (int v = t; v < nv; v += nt) {
    const double xv = p.x[v0 + v], yv = p.y[v0 + v];
    bx0 = fmin(bx0, xv); bx1 = fmax(bx1, xv);
    by0 = fmin(by0, yv); by1 = fmax(by1, yv);
  }
  for (int o = 32; o > 0; o >>= 1) {
    bx0 = fmin(bx0, __shfl_xor(bx0, o)); bx1 = fmax(bx1, __shfl_xor(bx1, o));
    by0 = fmin(by0, __shfl_xor(by0, o)); by1 = fmax(by1, __shfl_xor(by1, o));
  }
  if ((t & 63) == 0) {
    s_red[0][t >> 6] = bx0; s_red[1][t >> 6] = bx1;
    s_red[2][t >> 6] = by0; s_red[3][t >> 6] = by1;
  }
  __syncthreads();
  for (int w = 0; w < nt / 64; ++w) {
    bx0 = fmin(bx0, s_red[0][w]); bx1 = fmax(bx1, s_red[1][w]);
    by0 = fmin(by0, s_red[2][w]); by1 = fmax(by1, s_red[3][w]);
  }
  const double xm = 0.5 * (bx0 + bx1), hw = 0.5 * (bx1 - bx0);
  const double ym = 0.5 * (by0 + by1), hh = 0.5 * (by1 - by0);

  // ---- 2. tile columns and rows that can hold the stencil centre of a
  // vertex within rc of the box (centre = nearest node: one node of margin)
  const int n0x = (int)floor(bx0 - rc) - 1, n1x = (int)ceil(bx1 + rc) + 1;
  const int n0y = (int)floor(by0 - rc) - 1, n1y = (int)ceil(by1 + rc) + 1;
  int ncol = 0, nrow = 0;
  {
    const int a = wrap_i(n0x, nx), len = n1x - n0x + 1;
    for (int c0 = 0; c0 < ntx; c0 += nt) {
      const int tc = c0 + t;
      const bool f = tc < ntx && arc_meets(a, len, tc * TX, min(tc * TX + TX, nx) - 1, nx);
      int pos;
      const int cnt = block_scan(f ? 1 : 0, s_tmp, &pos);
      if (f && ncol + pos < kRepAxis) s_col[ncol + pos] = tc;
      ncol += cnt;
    }
  }
  {
    const int a = pery ? wrap_i(n0y, ny) : 0;
    const int lo = max(n0y, 0), hi = min(n1y, ny - 1);
    for (int r0 = 0; r0 < nty; r0 += nt) {
      const int tr = r0 + t;
      bool f = false;
      if (tr < nty) {
        const int s = tr * TY, e = min(s + TY, ny) - 1;
        f = pery ? arc_meets(a, n1y - n0y + 1, s, e, ny) : (s <= hi && e >= lo);
      }
      int pos;
      const int cnt = block_scan(f ? 1 : 0, s_tmp, &pos);
      if (f && nrow + pos < kRepAxis) s_row[nrow + pos] = tr;
      nrow += cnt;
    }
  }
  __syncthreads();   // the last column and row entries
  if (ncol > kRepAxis || nrow > kRepAxis) {
    if (t == 0) atomicAdd(p.overflow, 1);
    ncol = min(ncol, kRepAxis);
    nrow = min(nrow, kRepAxis);
  }

  // ---- 3. candidates from the bins of those tiles, in chunks of nt tiles
  const int ntl = ncol * nrow;
  int nc = 0;   // accepted candidates
  for (int k0 = 0; k0 < ntl; k0 += nt) {
    const int k = k0 + t;
    int tile = -1, cnt = 0;
    if (k < ntl) {
      tile = L.tile_base + s_row[k / ncol] * ntx + s_col[k % ncol];
      cnt = min(p.cnt_cur[tile], p.bin_cap);
    }
    // entry offsets of the chunk's tiles
    int excl;
    const int E = block_scan(cnt, s_tmp, &excl);
    s_off[t] = excl;
    if (t == nt - 1) s_off[nt] = E;
    __syncthreads();
    for (int e0 = 0; e0 < E; e0 += nt) {
      const int e = e0 + t;
      bool keep = false;
      int m2 = 0;
      double x2 = 0.0, y2 = 0.0;
      if (e < E) {
        // tile of entry e: last i with s_off[i] <= e
        int lo = 0, hi = nt - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int kk = k0 + lo;
        const int tl = L.tile_base + s_row[kk / ncol] * ntx + s_col[kk % ncol];
        m2 = p.bin_cur[(long long)tl * p.bin_cap + (e - s_off[lo])];
        const int cx2 = p.cx[m2];
        const int cy2 = min(max(p.cy[m2], 0), ny - 1);   // a centre beyond a wall sits in the edge row
        const int home = L.tile_base + (cy2 / TY) * ntx + cx2 / TX;
        if (home == tl && p.mbody[m2] != b) {
          x2 = p.x[m2];
          y2 = p.y[m2];
          const double dxb = fabs(min_image_n(x2 - xm, nx)) - hw;
          const double dyb = fabs(pery ? min_image_n(y2 - ym, ny) : y2 - ym) - hh;
          keep = dxb < rc && dyb < rc;
          // x relative to the body: unwrapped next to its box
          x2 = xm + min_image_n(x2 - xm, nx);
        }
      }
      int pos;
      const int cnt2 = block_scan(keep ? 1 : 0, s_tmp, &pos);
      if (keep && nc + pos < kRepCand) {
        s_x[nc + pos] = x2;
        s_y[nc + pos] = y2;
        s_id[nc + pos] = m2;
      }
      nc += cnt2;
    }
  }
  if (nc > kRepCand) {
    if (t == 0) atomicAdd(p.overflow, 1);
    nc = kRepCand;
  }
  __syncthreads();

  // ---- 4. rank by (x, id): a fixed order for the sums
  for (int i = t; i < nc; i += nt) {
    const double xi = s_x[i];
    const int ii = s_id[i];
    int r = 0;
    for (int j = 0; j < nc; ++j) {
      const double xj = s_x[j];
      r += (xj < xi || (xj == xi && s_id[j] < ii)) ? 1 : 0;
    }
    s_sx[r] = xi;
    s_sy[r] = s_y[i];
  }
  __syncthreads();

  // ---- 5. per vertex: the close candidates of the x window, in rank order.
  // A body wider than half the lattice could see a candidate through both
  // images; it then scans all candidates with the minimum image per pair.
  const bool window = 2.0 * (hw + rc) + 2.0 < 0.5 * nx;
  for (int v = t; v < nv; v += nt) {
    const double xv = p.x[v0 + v], yv = p.y[v0 + v];
    int j0 = 0, j1 = nc;
    if (window) {
      int lo = 0, hi = nc;   // first candidate with x >= xv - rc
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_sx[mid] < xv - rc) lo = mid + 1; else hi = mid;
      }
      j0 = lo;
    }
    double S = 0.0;
    for (int j = j0; j < j1; ++j) {
      const double xj = s_sx[j];
      if (window && xj > xv + rc) break;
      const double dx = min_image_n(xj - xv, nx);
      const double dyr = s_sy[j] - yv;
      const double dy = pery ? min_image_n(dyr, ny) : dyr;
      const double d = sqrt(dx * dx + dy * dy);
      if (d < rc) {
        const double d2 = d * d;
        S += coeff * sqrt(1.0 / (d2 * d2 * d));
      }
    }
    p.frep[v0 + v] = S;
  }
}

template <typename T>
void launch_repulsion(const Ptrs<T>& p, const StepArgs& a, hipStream_t s) {
  if (p.nbody_total == 0) return;
  const dim3 grid(p.nbody_total), block(kRepThreads);
  if (a.tile_x == 64 && a.tile_y == 4) hipLaunchKernelGGL((k_repulsion<T, 64, 4>), grid, block, 0, s, p);
  else if (a.tile_x == 128 && a.tile_y == 2) hipLaunchKernelGGL((k_repulsion<T, 128, 2>), grid, block, 0, s, p);
  else if (a.tile_x == 32 && a.tile_y == 8) hipLaunchKernelGGL((k_repulsion<T, 32, 8>), grid, block, 0, s, p);
  else hipLaunchKernelGGL((k_repulsion<T, 256, 1>), grid, block, 0, s, p);
}

template void launch_repulsion<float>(const Ptrs<float>&, const StepArgs&, hipStream_t);
template void launch_repulsion<double>(const Ptrs<double>&, const StepArgs&, hipStream_t);

}  // namespace lbib
