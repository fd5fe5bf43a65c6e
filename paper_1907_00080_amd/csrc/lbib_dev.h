// lbib_dev.h - device-side data layout and helpers of the LB-IB library (gfx950).
//
// Layout in the caller's workspace (all float64 Lagrangian data, SoA):
//   populations  A, B : T[9][N] per instance, node = y*pitch + x with the
//                       row pitch nx rounded up to 64 elements (every row
//                       starts on a 256-byte boundary; columns x >= nx are
//                       padding that no kernel reads), N = pitch*ny,
//                       stored shifted by the rest weights: h_i = f_i - w_i
//   velocity     U    : T[2][N] per instance (written on touched tiles only)
//   markers           : x[Nm], y[Nm] (current), xm/ym (previous), xn/yn (next,
//                       particles), fx/fy (force handed to the fluid),
//                       per-marker stencil cx, cy (int) and its weights: the
//                       Roma kernel's wx[3], wy[3] (node (a, b) weighs
//                       wx[a] wy[b]), or with the MLS transfer the nine
//                       weights in wx[9] (node (a, b) at row 3 b + a)
//   bins              : per tile, the markers whose 3x3 stencil overlaps it
//                       (fixed capacity, two sets used alternately)
//   ligands           : l2r[NL] (-1 free), receptors rec_x[NR], r2l[NR]
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include "lbib.h"
#include "roma.h"
#include <stdint.h>

namespace lbib {

constexpr int kQ = 9;
// D2Q9 velocity set in the order of Eq. (GaussHermite).
__host__ __device__ constexpr int ex(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp axis");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp diag");

template <typename T>
__host__ __device__ constexpr T wq(int i) {
  return i == 0 ? T(4) / T(9) : (i <= 4 ? T(1) / T(9) : T(1) / T(36));
}

enum BodyKind : int { kRBC = 0, kSoft = 1, kRigid = 2 };

// ------------------------------------------------------------ streaming schemes
// Where the populations live (Ptrs::sch):
//   0  two buffers: A holds every node's post-collision h*_i(x) in slot i; a
//      step pulls from A and writes B (pull streaming, halfway bounce-back).
//   1  one buffer, in place, layout P: h*_i(x) sits in slot opp(i) of x.
//   2  one buffer, in place, layout S: the populations already streamed for
//      the coming step sit in their own slots, h_i(x) in slot i of x.
// In place, a step on layout P reads slot opp(i) of x - e_i and writes slot
// i of x + e_i (layout S); a step on layout S reads and writes node x only
// (slot i in, slot opp(i) out: layout P again).  Every slot is read and then
// written by one node of the step, so the update needs no second buffer, and
// a lattice of 160 MB of populations keeps its whole working set in the
// 256 MB last-level cache.  Where x - e_i (x + e_i) lies beyond a wall the
// population bounces back at x, as in scheme 0.
//
// Slot (index into the population array of the instance, N nodes per plane)
// of the population h_i that node (x, y) streams in for the coming step.
__host__ __device__ inline long long streamed_slot(int s, int i, int x, int y, int nx, int ny,
                                                   int pitch, bool pery, long long N) {
  const long long node = (long long)y * pitch + x;
  if (s == 2) return i * N + node;
  int xs = x - ex(i);
  xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
  int ys = y - ey(i);
  const bool out = ys < 0 || ys >= ny;
  ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
  // bounce-back: h*_opp(i) of the node itself
  if (out && !pery) return (s == 1 ? i : opp(i)) * N + node;
  return (s == 1 ? opp(i) : i) * N + (long long)ys * pitch + xs;
}

// Slot where the step that read a state of scheme s leaves h*_i of node
// (x, y) (scheme 0: in B).
__host__ __device__ inline long long post_store_slot(int s, int i, int x, int y, int nx, int ny,
                                                     int pitch, bool pery, long long N) {
  const long long node = (long long)y * pitch + x;
  if (s == 0) return i * N + node;
  if (s == 2) return opp(i) * N + node;
  int xd = x + ex(i);
  xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
  int yd = y + ey(i);
  const bool out = yd < 0 || yd >= ny;
  yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
  if (out && !pery) return opp(i) * N + node;   // bounced into h_opp(i) of the node
  return i * N + (long long)yd * pitch + xd;
}

// Slot holding the last post-collision h*_i of node (x, y) in a state of
// scheme s (the scheme the next step reads).
__host__ __device__ inline long long post_slot(int s, int i, int x, int y, int nx, int ny,
                                               int pitch, bool pery, long long N) {
  if (s == 2) return post_store_slot(1, i, x, y, nx, ny, pitch, pery, N);
  return (s == 1 ? opp(i) : i) * (N) + (long long)y * pitch + x;
}

// Row pitch of an instance's node arrays: nx rounded up to 64 elements.
// Rows that start on 256-byte boundaries keep a tile's row segment within
// whole cache lines; with unaligned rows every segment straddles one more
// line, which neighbouring tiles then fetch twice.
__host__ __device__ constexpr int row_pitch(int nx) { return (nx + 63) & ~63; }

// Per-instance lattice description (device copy).
struct LatDev {
  int nx, ny, periodic_y;
  int ntx, nty;          // tiles of the fused kernel / marker bins
  int tile_base;         // first global tile index of this instance
  int pitch;             // row pitch of the node arrays (row_pitch(nx))
  int marker_base, n_markers;
  int body_base, n_bodies;
  int lig_base, n_lig;
  int rec_base, n_rec0, n_rec1;
  int instance;
  long long node_base;   // first node of this instance (populations at 9*node_base)
  long long plane;       // nodes of one population plane: pitch * ny
  double tau, gx, gy;
  unsigned long long seed;
  double y_cr, y_eq, kf0_dt, kr0_dt, sigma_ts_frac, kbt;
  int freeze;
  int pad_;
  double rep_coeff, rep_cutoff;   // vertex repulsion (Eq. repFor); coeff 0: off
  int wall_mode;                  // 0 halfway bounce-back, 1 velocity walls on rows 0, ny-1
  int pad2_;
  double u_wall_lo, u_wall_hi;    // wall velocities along x (velocity walls)
  double y_wall_lo, y_wall_hi;    // wall positions: -1/2, ny-1/2 or 0, ny-1
  int transfer;                   // 0 Roma kernel, 1 moving least squares (LBIB_TRANSFER_*)
  int mls_weight;                 // MLS weight (LBIB_MLS_WEIGHT_*)
  double mls_h;                   // MLS support half-width (3/2 for the Roma weight)
  double omega, pre;              // 1/tau and 1 - 1/(2 tau), computed once on the host
};

// Per-body description and rigid-body state (device copy; rigid state mutable).
struct BodyDev {
  int kind, nv, v0, inst;   // v0: global index of vertex 0
  int lig_base, n_lig, lig_stride;
  int chunk0;               // global index of the body's first vertex chunk
  int stepped;              // rigid: 1 once the body has taken a step (BDF2 has a history)
  double ks, kb, ka, p_ref;
  double A0, mass, mv, inertia, sigma;
  double xc, yc, theta;     // rigid: reference point and angle
  double U[2], Um[2];       // rigid: velocity history
  double Om, Omm;           // rigid: angular velocity history
};

// Device pointers into the workspace.
// Velocity walls on the node rows 0 and ny - 1 (Zou and He; the paper's wall
// condition, Sec. 2.1): the populations of a wall node whose source lies
// beyond the wall are set so that the node's half-force velocity is the wall
// velocity (u_w, 0), i.e. its bare momentum is rho u_w - F/2 (F the node's
// force), its density following from the known populations, and the
// non-equilibrium parts of the normal pair bounced back.  On shifted
// populations h = f - w: the pairs' differences are those of f, and the
// weights of the known terms of the density sum to one.
template <typename T>
__device__ __forceinline__ void zou_he_fill(T h[9], bool bottom, T u_wall, T Fx, T Fy) {
  // both walls' candidates from the old values, then selects: no branch
  // around the array's writes, so it stays in registers
  const T d13 = h[1] - h[3];
  const T jy = -T(0.5) * Fy;
  const T known = bottom ? (h[4] + h[7] + h[8]) : (h[2] + h[5] + h[6]);
  const T rho = T(1) + h[0] + h[1] + h[3] + T(2) * known + (bottom ? -T(0.5) : T(0.5)) * Fy;
  const T jx = rho * u_wall - T(0.5) * Fx;
  const T n2 = h[4] + T(2.0 / 3.0) * jy;                             // bottom: 2 (+y)
  const T n5 = h[7] - T(0.5) * d13 + T(0.5) * jx + jy * T(1.0 / 6.0);  //         5 (+x+y)
  const T n6 = h[8] + T(0.5) * d13 - T(0.5) * jx + jy * T(1.0 / 6.0);  //         6 (-x+y)
  const T n4 = h[2] - T(2.0 / 3.0) * jy;                             // top: 4 (-y)
  const T n7 = h[5] + T(0.5) * d13 - T(0.5) * jx - jy * T(1.0 / 6.0);  //      7 (-x-y)
  const T n8 = h[6] - T(0.5) * d13 + T(0.5) * jx - jy * T(1.0 / 6.0);  //      8 (+x-y)
  h[2] = bottom ? n2 : h[2];
  h[5] = bottom ? n5 : h[5];
  h[6] = bottom ? n6 : h[6];
  h[4] = bottom ? h[4] : n4;
  h[7] = bottom ? h[7] : n7;
  h[8] = bottom ? h[8] : n8;
}

template <typename T>
struct Ptrs {
  LatDev* lat;
  BodyDev* body;
  T* A;  // populations read this step
  T* B;  // populations written this step (in place: A)
  int sch;        // streaming scheme of the state this step reads (see above)
  int sch_next;   // and of the state it leaves
  T* U;  // velocity of touched tiles
  double *x, *y, *xm, *ym, *xn, *yn, *fx, *fy;
  double *l0, *th0, *r0x, *r0y;
  int* mbody;
  int* minfo;            // per marker: (instance << 2) | body kind
  int *cx, *cy;
  double *wx, *wy;       // Roma kernel: wx[3][Nm], wy[3][Nm] per axis; MLS:
                         // wx[9][Nm], node (a, b) at row 3 b + a (one array
                         // for both keeps this argument block, and the
                         // registers holding it, as small as it was)
  double* frep;          // per marker: summed repulsion magnitude of this step
                         // (written by the repulsion kernel, cleared by the
                         // body kernel once applied)
  double *s_len, *s_nx, *s_ny, *s_bc, *s_bnx, *s_bny, *s_bfl, *s_fex, *s_fey;  // per-vertex scratch
  // marker bins of fixed capacity per tile, double buffered: the fused
  // kernel consumes (and clears) the current set while the marker advance
  // fills the other one for the next step
  int *cnt_cur, *cnt_next;   // registrations per tile
  int *bin_cur, *bin_next;   // [tile * bin_cap + k] = marker id
  int* touched;              // per tile: IB force applied in the last step
  int* overflow;             // registrations dropped because a bin was full
  // per-step slots (two sets used alternately, like the population buffers)
  unsigned long long* fmax_bits;  // per instance: bit pattern of max |F| this step
  int* bond_flag;            // per instance: bond update of this step done
  long long* step_slot;      // per instance: step number of this step
  unsigned long long* fmax_next;  // the other slots: cleared during this step
  int* bond_flag_next;
  long long* step_prev;      // step number of the previous step
  int* spin_timeouts;        // waits for a bond flag that hit their bound
  int bin_cap;
  int* tile_inst;
  int *lig_body, *lig_elem, *l2r, *r2l, *lig_flag;
  int *lig_va, *lig_vb;  // global vertex ids of a ligand element's two ends
  double* lig_sigma;     // bond spring constant of each ligand's body
  double* lig_sp;        // per ligand holding a bond: sigma (y_l - y_eq) at X^n (Eq. adhFor),
                         // written by the bond workgroup of the step
  double* rec_x;
  long long *step_next, *step_cur;   // per instance
  // vertex chunks (kChunk consecutive vertices of one body, one wave each)
  const int4* chunk_info;             // per chunk: body, global index of its first
                                      // vertex minus 2 (the marker of lane 0),
                                      // vertex count, kind | instance << 2
  // waves of the chunked body kernel: (chunk, body) each one takes (chunk
  // -1: none; -2: an idle wave in the workgroup of a rigid body whose
  // chunks, at most four, share one workgroup so that its force and torque
  // are summed in LDS)
  const int2* slot_chunk;
  int nslot;
  double* area_part;                  // per chunk [5][nchunk]: shoelace sum over its interior
                                      // edges, its first vertex (x, y), its last vertex (x, y)
  double* rig_part;                   // per chunk: rigid load partials [3][nchunk]
  int* body_cnt;                      // per body: chunks done (rigid finish), reset by the last
  // particles' star field: rho* - 1, u*x, u*y (and one unused slot) of the
  // pre-forcing state per node, written over each particle's node box by
  // the advance and stencil passes for the next body kernel
  T* star;                            // [4 * nodes]
  int* pbox;                          // per chunk of a particle: vertex box x0, x1, y0, y1
  const int* star_wg;                 // star work list: (body, rank, workgroups of the body)
  int nstar_wg;
  double* red;                        // reduction scratch
  unsigned long long* ties;           // per instance count of bond draws within 1e-12 of P
  int nm_total, nbody_total, ntile_total, ninst, nlig_total, nchunk_total;
};

// Vertex chunks.  A body's vertices are cut into chunks of kChunk
// consecutive vertices; chunk c of a body covers [kChunk c, kChunk c + cnt)
// and is handled by one 64-lane wave whose lane i holds vertex
// kChunk c + i - 2 (modulo nv): the two lanes on either side are the halo
// that strain and bending at the chunk's own ("inner") vertices need.  Every
// sum over a body's vertices (its area, the rigid loads) is taken the same
// way on every path: each chunk's inner terms summed over the 64 lanes by a
// fixed butterfly (wave_sum), then the chunk sums in chunk order
// (chunk_total), so all kernels and step forms give the same bits.
constexpr int kChunk = 60;
__host__ __device__ constexpr int chunks_of(int nv) { return (nv + kChunk - 1) / kChunk; }
// rigid bodies of at most this many chunks (one per wave of a 256-lane
// workgroup) are summed inside their workgroup
constexpr int kGroupChunks = 4;
__host__ __device__ constexpr bool rigid_grouped(int kind, int nv) {
  return kind == kRigid && chunks_of(nv) <= kGroupChunks;
}

__device__ __forceinline__ int chunk_vertex(int lane, int first, int nv) {
  int v = (first + lane - 2) % nv;   // first + lane - 2 >= -2
  return v < 0 ? v + nv : v;
}

// Value of a double held by lane l of the wave (l wave-uniform: two
// readlanes, no LDS traffic).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Cross-lane moves by DPP (a vector ALU move from another lane, a few cycles,
// where a shuffle through the LDS crossbar takes a round trip of about a
// hundred).  Every lane of the wave must be active: a lane reading an
// inactive one gets its own value back.  The moves are volatile asm so that
// the compiler keeps them where they are written (in converged code) and
// does not sink them into a branch that only some lanes take, such as the
// one where lane 0 stores a reduced value; each starts with the two wait
// states a DPP read of a just-written register needs.
constexpr int kDppWaveShl1 = 0x130;   // lane i reads lane i + 1 (lane 63 keeps its own)
constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i - 1 (lane 0 keeps its own)
constexpr int kDppRowRor8 = 0x128, kDppRowRor4 = 0x124, kDppRowRor2 = 0x122, kDppRowRor1 = 0x121;
#define LBIB_DPP_MOV(CTRLTXT) \
  asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 " CTRLTXT " row_mask:0xf bank_mask:0xf" : "+v"(r) : "v"(v))
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  int r = v;   // lanes whose source lies outside the wave keep their own value
  if constexpr (CTRL == kDppWaveShl1) LBIB_DPP_MOV("wave_shl:1");
  else if constexpr (CTRL == kDppWaveShr1) LBIB_DPP_MOV("wave_shr:1");
  else if constexpr (CTRL == kDppRowRor8) LBIB_DPP_MOV("row_ror:8");
  else if constexpr (CTRL == kDppRowRor4) LBIB_DPP_MOV("row_ror:4");
  else if constexpr (CTRL == kDppRowRor2) LBIB_DPP_MOV("row_ror:2");
  else if constexpr (CTRL == kDppRowRor1) LBIB_DPP_MOV("row_ror:1");
  else static_assert(CTRL == kDppWaveShl1, "unsupported DPP control");
  return r;
}
#undef LBIB_DPP_MOV
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// x of the next / previous lane, as __shfl_down(x, 1) / __shfl_up(x, 1)
__device__ __forceinline__ double lane_next(double x) { return dpp_d<kDppWaveShl1>(x); }
__device__ __forceinline__ double lane_prev(double x) { return dpp_d<kDppWaveShr1>(x); }

// Sum over the 64 lanes of a wave in one fixed order: within each 16-lane
// row, rotations by 8, 4, 2 and 1 lanes (each lane adds the value the
// rotation brings, so both lanes of a pair add the same two values and the
// row ends with the same bits in every lane), then the four row sums as
// (r0 + r1) + (r2 + r3).  Every lane gets the same bits.
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_d<kDppRowRor8>(x);
  x += dpp_d<kDppRowRor4>(x);
  x += dpp_d<kDppRowRor2>(x);
  x += dpp_d<kDppRowRor1>(x);
  return (readlane_d(x, 0) + readlane_d(x, 16)) + (readlane_d(x, 32) + readlane_d(x, 48));
}

// Reduction over the 64 lanes with an associative, commutative operation
// that rounds nothing (min, max), every lane getting the result.
template <typename Op>
__device__ __forceinline__ double wave_reduce_d(double v, Op op) {
  v = op(v, dpp_d<kDppRowRor8>(v));
  v = op(v, dpp_d<kDppRowRor4>(v));
  v = op(v, dpp_d<kDppRowRor2>(v));
  v = op(v, dpp_d<kDppRowRor1>(v));
  return op(op(readlane_d(v, 0), readlane_d(v, 16)), op(readlane_d(v, 32), readlane_d(v, 48)));
}
template <typename Op>
__device__ __forceinline__ int wave_reduce_i(int v, Op op) {
  v = op(v, dpp_i<kDppRowRor8>(v));
  v = op(v, dpp_i<kDppRowRor4>(v));
  v = op(v, dpp_i<kDppRowRor2>(v));
  v = op(v, dpp_i<kDppRowRor1>(v));
  return op(op(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
            op(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// s + x_0 + x_1 + ... + x_{m-1} in this order, x_j held by lane j (m <= 64;
// a rolled loop: this code runs once per chunk, and its instruction fetches
// cost more than the loop)
__device__ __forceinline__ double ordered_lane_sum(double s, double x, int m) {
#pragma unroll 1
  for (int j = 0; j < m; ++j) s += readlane_d(x, j);
  return s;
}

// Sum of a body's chunk partials in chunk order (part[k], k < nch; every
// lane of the wave gets the same bits).
__device__ __forceinline__ double chunk_total(const double* part, int nch) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int k0 = 0; k0 < nch; k0 += 64) {
    const double pv = k0 + lane < nch ? part[k0 + lane] : 0.0;
    s = ordered_lane_sum(s, pv, nch - k0 < 64 ? nch - k0 : 64);
  }
  return s;
}

// Shoelace term of the edge from (x0, y0) to (x1, y1): twice the signed area
// of the triangle it spans with the origin (its rounding fixed by the fma).
__device__ __forceinline__ double shoelace_term(double x0, double y0, double x1, double y1) {
  return __fma_rn(x0, y1, -(x1 * y0));
}

// Twice a body's signed area from its chunk records (the advance or stencil
// pass writes them): chunk k adds its interior-edge sum P_k and the edge
// from its last vertex to the first vertex of chunk k + 1 (cyclically),
// T_k = P_k + shoelace(last_k, first_k+1), and the T_k are added in chunk
// order.  A chunk's record never needs a vertex another wave moves.
__device__ __forceinline__ double body_area2(const double* rec, int nct, int ch0, int nch) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int k0 = 0; k0 < nch; k0 += 64) {
    const int k = k0 + lane;
    double tk = 0.0;
    if (k < nch) {
      const int kn = k + 1 == nch ? 0 : k + 1;
      tk = rec[ch0 + k] + shoelace_term(rec[3 * nct + ch0 + k], rec[4 * nct + ch0 + k],
                                        rec[nct + ch0 + kn], rec[2 * nct + ch0 + kn]);
    }
    s = ordered_lane_sum(s, tk, nch - k0 < 64 ? nch - k0 : 64);
  }
  return s;
}

__host__ __device__ inline int wrap_i(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// ------------------------------------------------------------ Philox4x32-10
// Salmon et al., SC'11: 10 rounds of multiply/xor with Weyl key schedule.
__device__ inline void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    unsigned lo0 = 0xD2511F53u * c[0];
    unsigned hi0 = __umulhi(0xD2511F53u, c[0]);
    unsigned lo1 = 0xCD9E8D57u * c[2];
    unsigned hi1 = __umulhi(0xCD9E8D57u, c[2]);
    unsigned n0 = hi1 ^ c[1] ^ k0;
    unsigned n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ inline double philox_uniform(unsigned long long seed, long long step, int lig,
                                        int purpose, int instance) {
  unsigned c[4] = {(unsigned)(step & 0xffffffffull), (unsigned)lig, (unsigned)purpose,
                   (unsigned)instance};
  philox4x32_10(c, (unsigned)(seed & 0xffffffffull), (unsigned)(seed >> 32));
  return (double)c[0] * (1.0 / 4294967296.0);
}

// ------------------------------------------------------------ adjoint
// Pointers of one reverse step (single lattice instance).  Forward data of
// step n come from the segment store; everything else is float64 adjoint
// state or per-step scratch.
// Scatter target of the adjoint: an exact accumulator per entry, the value
// at k being hi[k] 2^-24 + lo[k] 2^-72 (two signed 64-bit integer words, a
// coarse and a fine part of every term).  Integer addition is associative,
// so the sums do not depend on the order in which contributions arrive: the
// reverse sweep is bitwise reproducible.
struct AccField {
  long long* hi;
  long long* lo;
};

struct AdjPtrs {
  const void* h;                      // h^n (T[9][N])
  const double *x, *y;                // X^n
  const double *fx, *fy;              // marker forces of step n
  const double *xn, *yn;              // X^{n+1} of particles
  const void* u;                      // physical velocity u^n (T[2][N], valid where touched)
  int first;                          // step n is the first step
  double* ha;                         // [9][N] adjoint of h^{n+1} in, of h^n out
  double *xa, *ya;                    // adjoint of X^{n+1} in, of X^n out
  double *xma, *yma;                  // adjoint of X_prev^{n+1} in, of X_prev^n out
  double *fph, *FEh, *mom;            // [9N] [2N] [3N]
  AccField FE, Uh, Rh;                // [2N] [2N] [3N] scatter targets
  int* bad;                           // set by a scattered value that is not finite or
                                      // beyond the accumulator's range (|v| >= 2^30)
  double *dirx, *diry, *fvx, *fvy, *dsh, *Dx, *Dy, *Cx, *Cy, *BLx, *BLy, *BRx, *BRy;  // [nm]
  double* grad;                       // [nbody][3]: d/dks, d/dkb, d/dsigma
  const BodyDev *body0, *body1;       // bodies before and after step n (rigid state)
  double* rig;                        // [nbody][9] adjoint of a rigid particle's state
                                      // (x_c, y_c, theta, U, U_prev, Omega, Omega_prev):
                                      // after step n in, before it out
};

// Up to 24 device-to-device copies in one launch (sizes multiple of 4 bytes).
struct CopyList {
  int n;
  const char* src[24];
  char* dst[24];
  unsigned long long bytes[24];
};

template <typename T>
void launch_adjoint_segment(const Ptrs<T>& p, const AdjPtrs* a, int n, long long N, hipStream_t s);
void launch_copies(const CopyList& c, hipStream_t s);
void launch_fill(double* out, long long n, double v, hipStream_t s);

// ------------------------------------------------------------ launchers
// (defined in the kernel translation units, called by the host engine)
// Bodies with at most this many vertices keep their per-vertex scratch in the
// body kernel's LDS; the merged step form needs every body to be that small.
constexpr int kSmallBody = 512;

struct StepArgs {
  int tile_x, tile_y;
  int ntiles_total;
  int max_inst_tiles;   // largest tile count of any instance
  int body_cache_bytes; // LDS cache of rho*, u* per particle workgroup
  int max_nv;           // most vertices of any body
  int any_mls;          // some instance uses the MLS transfer
  int nt_mode;          // lattice kernel: non-temporal population loads (1), and stores (3)
  int lb_wpc;           // lattice kernel: 0 one workgroup per tile, else a persistent
                        // grid of this many workgroups per CU
  int n_cu;             // compute units of the device
};

template <typename T>
void launch_observe(const Ptrs<T>& p, lbib_body_obs* obs, long long step, hipStream_t s);

// The repulsion kernel's work unit: kRepChunk consecutive vertices of one
// body; the host lists the chunks as (body, first global vertex, vertex
// count, instance) records.
constexpr int kRepChunk = 16;
template <typename T>
void launch_repulsion(const Ptrs<T>& p, const StepArgs& a, const int* chunks, int nchunk,
                      hipStream_t s);
// Populations between the state (scheme p.sch, in p.A) and scheme-0 order in
// buf, per instance (inst_nodes[i] = nx * ny of instance i): to = 1 state ->
// buf, to = 0 buf -> state.
template <typename T>
void launch_canon(const Ptrs<T>& p, int ninst, const long long* inst_nodes, T* buf, int to,
                  hipStream_t s);
template <typename T>
void launch_lb_fused(const Ptrs<T>& p, const StepArgs& a, hipStream_t s, int mode = 3,
                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
void launch_fields(const Ptrs<T>& p, const StepArgs& a, int inst, double* rho, double* ux,
                   double* uy, int nx, int ny, long long node_base, hipStream_t s);
template <typename T>
void launch_diag(const Ptrs<T>& p, const StepArgs& a, long long nodes_total, double* out,
                 hipStream_t s);
template <typename T>
void launch_init_pop(const Ptrs<T>& p, const double* rho, const double* ux, const double* uy,
                     long long node_base, long long n, long long nodes_total, hipStream_t s);
template <typename T>
void launch_lagrangian(const Ptrs<T>& p, const StepArgs& a, hipStream_t s, bool advance_first);
template <typename T>
void launch_advance(const Ptrs<T>& p, const StepArgs& a, hipStream_t s);
template <typename T>
void launch_stencil(const Ptrs<T>& p, const StepArgs& a, hipStream_t s);

}  // namespace lbib
