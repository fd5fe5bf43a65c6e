// k_observe.hip - per-body observables of a run (gfx950): the quantities the
// paper reports for margination and adhesion (Sec. 3).
//
// One workgroup per body updates its record (lbib_body_obs) from the current
// state: centre of mass (mean of the vertex positions; vertices carry equal
// masses), flow region of the lateral position eta = (y_c + 1/2) / n_y
// (cell-free layer eta <= 0.2 or >= 0.8, bulk 0.3 <= eta <= 0.7, the
// intermediate zone between), the largest lateral displacement from the
// release position (the first observation), the centre-of-mass velocity
// over the interval since the previous observation and running sums of it,
// and the number of the body's ligands holding a bond (and that number at the
// first observation).  Sums run in a fixed order (strided lane sums, wave
// butterflies, waves in order), so observations are deterministic.
#include "lbib.h"
#include "lbib_dev.h"

namespace lbib {

constexpr int kObsThreads = 256;

template <typename T>
__global__ __launch_bounds__(kObsThreads) void k_observe(Ptrs<T> p, lbib_body_obs* obs, long long step) {
  __shared__ double s_sum[2][kObsThreads / 64];
  __shared__ int s_nb[kObsThreads / 64];
  const int b = blockIdx.x, t = threadIdx.x;
  const BodyDev& B = p.body[b];
  const int nv = B.nv, v0 = B.v0;
  const LatDev& L = p.lat[B.inst];
  double sx = 0.0, sy = 0.0;
  for (int v = t; v < nv; v += kObsThreads) {
    sx += p.x[v0 + v];
    sy += p.y[v0 + v];
  }
  int nb = 0;
  for (int l = t; l < B.n_lig; l += kObsThreads) nb += p.l2r[B.lig_base + l] >= 0 ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
    nb += __shfl_xor(nb, o);
  }
  if ((t & 63) == 0) {
    s_sum[0][t >> 6] = sx;
    s_sum[1][t >> 6] = sy;
    s_nb[t >> 6] = nb;
  }
  __syncthreads();
  if (t != 0) return;
  sx = 0.0;
  sy = 0.0;
  nb = 0;
  for (int w = 0; w < kObsThreads / 64; ++w) {
    sx += s_sum[0][w];
    sy += s_sum[1][w];
    nb += s_nb[w];
  }
  const double xc = sx / nv, yc = sy / nv;
  lbib_body_obs o = obs[b];
  if (o.n_obs == 0) {
    o.x0 = xc;
    o.y0 = yc;
    o.n_bonds0 = nb;
  } else {
    const long long dn = step - o.step_obs;
    if (dn > 0) {
      o.u_x = (xc - o.xc) / (double)dn;
      o.u_y = (yc - o.yc) / (double)dn;
      o.u_x_sum += o.u_x;
      o.u_y_sum += o.u_y;
    }
  }
  o.xc = xc;
  o.yc = yc;
  o.r_max = fmax(o.r_max, fabs(yc - o.y0));
  const double eta = (yc - L.y_wall_lo) / (L.y_wall_hi - L.y_wall_lo);
  o.region = (eta <= 0.2 || eta >= 0.8) ? LBIB_REGION_CFL
             : (eta >= 0.3 && eta <= 0.7) ? LBIB_REGION_BULK : LBIB_REGION_INTERMEDIATE;
  o.n_bonds = nb;
  o.n_obs += 1;
  o.step_obs = step;
  obs[b] = o;
}

template <typename T>
void launch_observe(const Ptrs<T>& p, lbib_body_obs* obs, long long step, hipStream_t s) {
  if (p.nbody_total == 0) return;
  hipLaunchKernelGGL(k_observe<T>, dim3(p.nbody_total), dim3(kObsThreads), 0, s, p, obs, step);
}

template void launch_observe<float>(const Ptrs<float>&, lbib_body_obs*, long long, hipStream_t);
template void launch_observe<double>(const Ptrs<double>&, lbib_body_obs*, long long, hipStream_t);

}  // namespace lbib
