// k_repulsion.hip - repulsion between vertices of different bodies (gfx950),
// Sec. 2.2 "Particle-Particle Interaction", Eq. (repFor).
//
// A vertex at distance d < r_c from a vertex of another body is pushed along
// its own inward normal with magnitude c sqrt(1 / d^5) (lattice units); the
// magnitudes of all such neighbours add.  This kernel computes the summed
// magnitude S_v of every vertex at X^n; the body kernel applies -S_v n_v with
// the vertex normal it computes anyway (red cells and soft particles add it to
// the vertex force, rigid particles to their force and torque) and clears S_v
// after use.
//
// One workgroup per chunk of kRepChunk consecutive vertices of a body (the
// host lists the chunks), so that a large body is spread over many
// workgroups and each looks at a small neighbourhood.  The marker bins of the
// step (every marker is registered in the tiles its 3x3 stencil overlaps)
// serve as the cell list:
//   1. the chunk's bounding box gives the tile columns and rows that can hold
//      the stencil centre of a vertex within r_c of it;
//   2. the bins of those tiles are read with all loads of a round in flight
//      together; a marker is taken from the bin of the tile that holds its
//      stencil centre only (so once), if it belongs to another body and lies
//      within r_c of the box;
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
constexpr int kRepCand = 512;      // candidate vertices of other bodies per chunk
constexpr int kRepTiles = 256;     // neighbour tiles per chunk (one lane each)
constexpr int kRepAxis = 64;       // tile columns / rows per chunk
constexpr int kRepPerLane = 4;     // bin entries per lane and round

__device__ inline double min_image_n(double d, int n) { return d - n * rint(d / n); }

// Block-wide exclusive prefix sum of one value per lane: *excl gets the sum
// over the lanes before this one; returns the total (every lane).  Scan
// inside each wave by shuffles, then across the waves' totals in LDS.
__device__ inline int block_scan(int v, int* s_wave, int* excl) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[w] = x;
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kRepThreads / 64; ++k) {
    const int s = s_wave[k];
    base += k < w ? s : 0;
    total += s;
  }
  *excl = base + x - v;
  __syncthreads();   // s_wave is reused by the next scan
  return total;
}

// Tiles along one axis whose nodes meet [n0, n1] (unwrapped node indices):
// wrapped on a periodic axis, clamped to [0, n) otherwise.  Distinct, in
// order of first meeting.  Returns the count (may exceed cap: then only the
// first cap are stored).
__device__ inline int axis_tiles(int n0, int n1, int n, int tw, bool periodic, int* out, int cap) {
  int k = 0;
  if (!periodic) {
    const int lo = max(n0, 0), hi = min(n1, n - 1);
    for (int tt = lo / tw; lo <= hi && tt <= hi / tw; ++tt) {
      if (k < cap) out[k] = tt;
      ++k;
    }
    return k;
  }
  if (n1 - n0 + 1 >= n) {
    const int nt = (n + tw - 1) / tw;
    for (int tt = 0; tt < nt; ++tt) {
      if (k < cap) out[k] = tt;
      ++k;
    }
    return k;
  }
  for (int m = n0; m <= n1;) {
    const int w = wrap_i(m, n);
    const int tt = w / tw;
    bool dup = false;
    for (int j = 0; j < min(k, cap); ++j) dup |= out[j] == tt;
    if (!dup) {
      if (k < cap) out[k] = tt;
      ++k;
    }
    m += min(tt * tw + tw, n) - w;   // to the first node of the next tile
  }
  return k;
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(kRepThreads) void k_repulsion(Ptrs<T> p, const int* chunks) {
  __shared__ int s_col[kRepAxis], s_row[kRepAxis];
  __shared__ int s_nc[2];
  __shared__ int s_tmp[kRepThreads / 64];
  __shared__ int s_off[kRepTiles + 1];
  __shared__ double s_x[kRepCand], s_y[kRepCand];     // candidates as accepted
  __shared__ int s_id[kRepCand];
  __shared__ double s_sx[kRepCand], s_sy[kRepCand];   // ranked by (x, id)
  __shared__ double s_box[4];

  // chunk record: body, first global vertex, vertex count, lattice instance
  const int* ck = chunks + 4 * blockIdx.x;
  const int b = ck[0], gv0 = ck[1], nvc = ck[2];
  const LatDev& L = p.lat[ck[3]];
  const int t = threadIdx.x, nt = kRepThreads;
  if (!(L.rep_coeff > 0.0)) return;   // the body kernel then reads the cleared zeros
  const double coeff = L.rep_coeff, rc = L.rep_cutoff;
  const int nx = L.nx, ny = L.ny, ntx = L.ntx;
  const bool pery = L.periodic_y != 0;

  // ---- 1. the chunk's vertices (one per lane of the first wave) and box
  const bool own = t < nvc;
  const int gv = gv0 + (own ? t : 0);
  const double xv = p.x[gv], yv = p.y[gv];
  if (t < 64) {
    double bx0 = own ? xv : 1e300, bx1 = own ? xv : -1e300;
    double by0 = own ? yv : 1e300, by1 = own ? yv : -1e300;
    {
      const auto mn = [](double a, double b) { return fmin(a, b); };
      const auto mx = [](double a, double b) { return fmax(a, b); };
      bx0 = wave_reduce_d(bx0, mn);
      bx1 = wave_reduce_d(bx1, mx);
      by0 = wave_reduce_d(by0, mn);
      by1 = wave_reduce_d(by1, mx);
    }
    if (t == 0) {
      s_box[0] = bx0; s_box[1] = bx1; s_box[2] = by0; s_box[3] = by1;
      // ---- 2. tiles that can hold the stencil centre (the nearest node) of
      // a vertex within rc of the box: one node of margin beyond rc
      const int nc = axis_tiles((int)floor(bx0 - rc) - 1, (int)ceil(bx1 + rc) + 1, nx, TX, true,
                                s_col, kRepAxis);
      const int nr = axis_tiles((int)floor(by0 - rc) - 1, (int)ceil(by1 + rc) + 1, ny, TY, pery,
                                s_row, kRepAxis);
      int ncol = min(nc, kRepAxis), nrow = min(nr, kRepAxis);
      if (nc > kRepAxis || nr > kRepAxis || ncol * nrow > kRepTiles) {
        atomicAdd(p.overflow, 1);
        nrow = min(nrow, kRepTiles / max(ncol, 1));
      }
      s_nc[0] = ncol;
      s_nc[1] = nrow;
    }
  }
  __syncthreads();
  const double xm = 0.5 * (s_box[0] + s_box[1]), hw = 0.5 * (s_box[1] - s_box[0]);
  const double ym = 0.5 * (s_box[2] + s_box[3]), hh = 0.5 * (s_box[3] - s_box[2]);
  const int ncol = s_nc[0], nrow = s_nc[1], ntl = ncol * nrow;

  // ---- 3. bin entry counts of those tiles (one tile per lane) and offsets
  int cnt = 0;
  if (t < ntl) cnt = min(p.cnt_cur[L.tile_base + s_row[t / ncol] * ntx + s_col[t % ncol]], p.bin_cap);
  int excl;
  const int E = block_scan(cnt, s_tmp, &excl);
  s_off[t] = excl;
  if (t == nt - 1) s_off[nt] = E;
  __syncthreads();

  // candidates, kRepPerLane entries per lane per round, loads issued together
  int ncand = 0;
  for (int e0 = 0; e0 < E; e0 += kRepPerLane * nt) {
    int m2[kRepPerLane], tl[kRepPerLane];
#pragma unroll
    for (int q = 0; q < kRepPerLane; ++q) {
      const int e = e0 + q * nt + t;
      m2[q] = -1;
      tl[q] = -1;
      if (e < E) {
        int lo = 0, hi = nt - 1;   // tile of entry e: last i with s_off[i] <= e
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        tl[q] = L.tile_base + s_row[lo / ncol] * ntx + s_col[lo % ncol];
        m2[q] = p.bin_cur[(long long)tl[q] * p.bin_cap + (e - s_off[lo])];
      }
    }
    int bd2[kRepPerLane];
    double x2[kRepPerLane], y2[kRepPerLane];
#pragma unroll
    for (int q = 0; q < kRepPerLane; ++q) {
      const int m = m2[q] >= 0 ? m2[q] : 0;
      bd2[q] = p.mbody[m];
      x2[q] = p.x[m];
      y2[q] = p.y[m];
    }
    bool keep[kRepPerLane];
    int nkeep = 0;
#pragma unroll
    for (int q = 0; q < kRepPerLane; ++q) {
      // home tile: the one holding the marker's stencil centre, the nearest
      // node (as the stencil takes it), a centre beyond a wall in the edge row
      const int cx2 = wrap_i((int)floor(x2[q] + 0.5), nx);
      const double fy = floor(y2[q] + 0.5);
      const int cy2 = pery ? wrap_i((int)fy, ny) : (int)fmin(fmax(fy, 0.0), (double)(ny - 1));
      const int home = L.tile_base + (cy2 / TY) * ntx + cx2 / TX;
      keep[q] = m2[q] >= 0 && home == tl[q] && bd2[q] != b;
      if (keep[q]) {
        const double dxb = fabs(min_image_n(x2[q] - xm, nx)) - hw;
        const double dyb = fabs(pery ? min_image_n(y2[q] - ym, ny) : y2[q] - ym) - hh;
        keep[q] = dxb < rc && dyb < rc;
      }
      nkeep += keep[q] ? 1 : 0;
    }
    int pos;
    const int added = block_scan(nkeep, s_tmp, &pos);
#pragma unroll
    for (int q = 0; q < kRepPerLane; ++q) {
      if (!keep[q]) continue;
      const int at = ncand + pos;
      ++pos;
      if (at < kRepCand) {
        s_x[at] = xm + min_image_n(x2[q] - xm, nx);   // unwrapped next to the box
        s_y[at] = y2[q];
        s_id[at] = m2[q];
      }
    }
    ncand += added;
  }
  if (ncand > kRepCand) {
    if (t == 0) atomicAdd(p.overflow, 1);
    ncand = kRepCand;
  }
  __syncthreads();

  // ---- 4. rank by (x, id): a fixed order for the sums
  for (int i = t; i < ncand; i += nt) {
    const double xi = s_x[i];
    const int ii = s_id[i];
    int r = 0;
    for (int j = 0; j < ncand; ++j) {
      const double xj = s_x[j];
      r += (xj < xi || (xj == xi && s_id[j] < ii)) ? 1 : 0;
    }
    s_sx[r] = xi;
    s_sy[r] = s_y[i];
  }
  __syncthreads();

  // ---- 5. per vertex: the close candidates of the x window, in rank order.
  // A box wider than about half the lattice could see a candidate through
  // both images; the vertex then scans all candidates with the minimum
  // image per pair.
  if (!own) return;
  const bool window = 2.0 * (hw + rc) + 2.0 < 0.5 * nx;
  const double xvr = xm + min_image_n(xv - xm, nx);
  int j0 = 0, j1 = ncand;
  if (window) {
    int lo = 0, hi = ncand;   // first candidate with x >= xv - rc
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_sx[mid] < xvr - rc) lo = mid + 1; else hi = mid;
    }
    j0 = lo;
    hi = ncand;               // first candidate with x > xv + rc
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_sx[mid] <= xvr + rc) lo = mid + 1; else hi = mid;
    }
    j1 = lo;
  }
  double S = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double dx = min_image_n(s_sx[j] - xvr, nx);
    const double dyr = s_sy[j] - yv;
    const double dy = pery ? min_image_n(dyr, ny) : dyr;
    const double d = sqrt(dx * dx + dy * dy);
    if (d < rc) {
      const double d2 = d * d;
      S += coeff * sqrt(1.0 / (d2 * d2 * d));
    }
  }
  p.frep[gv] = S;
}

template <typename T>
void launch_repulsion(const Ptrs<T>& p, const StepArgs& a, const int* chunks, int nchunk,
                      hipStream_t s) {
  if (nchunk == 0) return;
  const dim3 grid(nchunk), block(kRepThreads);
  if (a.tile_x == 64 && a.tile_y == 4)
    hipLaunchKernelGGL((k_repulsion<T, 64, 4>), grid, block, 0, s, p, chunks);
  else if (a.tile_x == 128 && a.tile_y == 2)
    hipLaunchKernelGGL((k_repulsion<T, 128, 2>), grid, block, 0, s, p, chunks);
  else if (a.tile_x == 32 && a.tile_y == 8)
    hipLaunchKernelGGL((k_repulsion<T, 32, 8>), grid, block, 0, s, p, chunks);
  else
    hipLaunchKernelGGL((k_repulsion<T, 256, 1>), grid, block, 0, s, p, chunks);
}

template void launch_repulsion<float>(const Ptrs<float>&, const StepArgs&, const int*, int, hipStream_t);
template void launch_repulsion<double>(const Ptrs<double>&, const StepArgs&, const int*, int,
                                       hipStream_t);

}  // namespace lbib
