// engine.hip - host side of the LB-IB library: set-up, workspace layout,
// step scheduling (plain launches or captured HIP graphs), readback, C ABI.
//
// One Engine holds one or more independent lattice instances that advance in
// lock-step with the same kernels (a single instance is the plain solver; a
// batch of uneven instances is a parameter sweep).  All device state lives in
// the caller-provided workspace; the engine never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include <cstddef>
#include "lbib.h"
#include "lbib_batch.h"
#include "lbib_dev.h"

using namespace lbib;

namespace {

struct BodyHost {
  lbib_body_desc d;
  std::vector<double> xy;
};

struct InstHost {
  lbib_lattice_desc lat{};
  std::vector<BodyHost> bodies;
  std::vector<double> rec[2];
  lbib_adhesion_desc adh{};
  double rep_coeff = 0.0, rep_cutoff = 2.0;   // vertex repulsion (Eq. repFor)
  int wall_mode = 0;                          // 0 halfway bounce-back, 1 velocity walls
  double u_wall_lo = 0.0, u_wall_hi = 0.0;
  int transfer = LBIB_TRANSFER_ROMA;           // lattice <-> marker transfer
  int mls_weight = LBIB_MLS_WEIGHT_CUBIC;
  double mls_h = 1.3;
  std::vector<double> rho0, ux0, uy0;
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Registrations one tile's bin holds: markers whose 3x3 stencil overlaps a
// TX x TY tile lie in its (TX+2) x (TY+2) halo; membranes with spacing of
// about one lattice unit put a few per halo column or row there.
int bin_capacity(int tx, int ty) { return std::max(1024, 16 * (tx + ty + 2)); }

bool valid_tile(int tx, int ty) {
  return (tx == 64 && ty == 4) || (tx == 128 && ty == 2) || (tx == 32 && ty == 8) ||
         (tx == 256 && ty == 1);
}

struct Layout {
  size_t lat, body, A, B, U;
  size_t x, y, xm, ym, xn, yn, fx, fy, l0, th0, r0x, r0y;
  size_t mbody, minfo, cx, cy, wx, wy, frep, rep_chunk, obs;
  size_t s[9];
  size_t cnt[2], bins[2], touched, overflow, fmax, bond_flag, step_slot, spin, Uspare, tile_inst;
  size_t lig_body, lig_elem, l2r, r2l, lig_flag, rec_x, lig_va, lig_vb, lig_sigma, lig_sp;
  size_t step_next, step_cur, ties, red;
  size_t chunk_info, area_part, rig_part, body_cnt, star, pbox, star_wg, slot_chunk;
  size_t total;
};

}  // namespace

struct lbib_ctx {
  std::vector<InstHost> inst;
  int dtype = LBIB_F32;
  int TX = 64, TY = 4;
  int phase = 0;  // 0 setup, 1 bound, 2 running
  // sizes
  int ninst = 0, nm = 0, nbody = 0, nlig = 0, nrec = 0, ntiles = 0;
  int nchunk = 0;              // vertex chunks of all bodies (kChunk vertices each)
  int nstar_wg = 0;            // workgroups of the star pass (particle node boxes)
  int nslot = 0;               // waves of the chunked body kernel (a multiple of 4)
  long long nodes = 0;
  std::vector<int> marker_base, body_base, lig_base, rec_base, tile_base;
  std::vector<long long> node_base;
  Layout L{};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int device = -1;            // device current at lbib_bind (the workspace's)
  long long step = 0;
  int parity = 0;  // 0: A holds the state; 1: B holds it
  bool watchdog = false;
  // total mass at set-up (or at the last set_state): the watchdog's drift
  // reference; NaN when a lattice has velocity walls (they exchange mass)
  double mass_ref = 0.0;
  double mass_tol = 1e-6;     // relative drift the watchdog accepts
  int graph_steps = 0;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::string err;
  bool is_batch = false;
  bool stencil_dirty = true;  // marker stencils/bins must be rebuilt from positions
  bool ktiming = false;       // bracket fused-kernel launches with events
  std::vector<std::pair<hipEvent_t, hipEvent_t>> kevents;
  int bin_cap = 1024;         // marker registrations per tile and bin set
  int body_cache = 16 * 1024; // LDS bytes of a particle workgroup's rho*, u* cache
  // how a step is launched (lbib_set_step_mode): 0 automatic, 1 three
  // kernels, 2 merged advance, 3 overlapped lattice tiles
  int step_mode = 0;
  // cache hints of the fused lattice kernel's population accesses
  // (lbib_set_cache_hints): -1 automatic, else the NT bits
  int cache_hints = -1;
  // launch form of the fused lattice kernel (lbib_set_lattice_launch): 0 one
  // workgroup per tile, else persistent with this many workgroups per CU
  int lb_wpc = 0;
  int n_cu = 256;             // compute units of the bound device
  // streaming (lbib_set_streaming): -1 automatic, 0 two buffers, 1 in place;
  // inplace is the resolved form (see streamed_slot in lbib_dev.h)
  int streaming = -1;
  bool inplace = false;
  bool merge_advance = true;  // resolved from step_mode and the bodies
  bool repulsion = false;     // some instance has the vertex repulsion on
  int nrep_chunk = 0;         // repulsion work units (kRepChunk vertices of a body)
  bool overlap = false;
  hipStream_t aux = nullptr;  // second stream of the overlapped form
  // streams of the adjoint's backward pass (segment recompute, reverse
  // sweep), created together so that they sit on different hardware queues
  hipStream_t adj_s[2] = {nullptr, nullptr};
  hipEvent_t ev_adj_start = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // adjoint window (single-instance contexts): caller-owned workspace
  char* aws = nullptr;
  size_t aws_bytes = 0;
  long long adjK = 0;         // window length the workspace was sized for
  int adjk = 0;               // checkpoint spacing
  bool adj_ready = false;     // a forward window has run since the last change
  std::vector<long long> ck_step;   // step of each checkpoint (last: end of window)
  // captured recompute of a segment, keyed by (steps, start parity, store),
  // and reverse sweep, keyed by (steps, store, segment starts at step 0)
  std::map<std::tuple<long long, int, int>, hipGraphExec_t> adj_graphs, adj_rgraphs;
  hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  std::vector<double> adj_y;        // marker ordinates at the end of the window
};

static std::string g_create_err;

namespace {

lbib_status fail(lbib_ctx* c, lbib_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, LBIB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

int elem_size(int dtype) { return dtype == LBIB_F64 ? 8 : 4; }

// Workgroups of the star pass for one particle: its node box at rest (the
// vertex extent widened by 4 nodes on each side) with 10 % spare for
// deformation, 1024 nodes per workgroup and pass (any larger box is still
// covered: the workgroups loop over it).
int star_workgroups(const BodyHost& b) {
  if (b.d.kind == LBIB_RBC_KINEMATIC) return 0;
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int v = 0; v < b.d.nv; ++v) {
    x0 = std::min(x0, b.xy[2 * v]); x1 = std::max(x1, b.xy[2 * v]);
    y0 = std::min(y0, b.xy[2 * v + 1]); y1 = std::max(y1, b.xy[2 * v + 1]);
  }
  const double nodes = std::ceil(x1 - x0 + 10.0) * std::ceil(y1 - y0 + 10.0) * 1.1;
  return std::max(1, (int)std::ceil(nodes / 1024.0));
}

void compute_sizes(lbib_ctx* c) {
  c->ninst = (int)c->inst.size();
  c->nm = c->nbody = c->nlig = c->nrec = c->ntiles = 0;
  c->nchunk = 0;
  c->nstar_wg = 0;
  int grouped = 0, grouped_chunks = 0;
  c->nrep_chunk = 0;
  c->nodes = 0;
  c->marker_base.clear(); c->body_base.clear(); c->lig_base.clear();
  c->rec_base.clear(); c->tile_base.clear(); c->node_base.clear();
  for (auto& I : c->inst) {
    c->marker_base.push_back(c->nm);
    c->body_base.push_back(c->nbody);
    c->lig_base.push_back(c->nlig);
    c->rec_base.push_back(c->nrec);
    c->tile_base.push_back(c->ntiles);
    c->node_base.push_back(c->nodes);
    for (auto& b : I.bodies) {
      c->nm += b.d.nv;
      c->nbody += 1;
      c->nrep_chunk += (b.d.nv + kRepChunk - 1) / kRepChunk;
      c->nchunk += chunks_of(b.d.nv);
      c->nstar_wg += star_workgroups(b);
      if (rigid_grouped(b.d.kind, b.d.nv)) {
        ++grouped;
        grouped_chunks += chunks_of(b.d.nv);
      }
      if (b.d.ligand_stride > 0) c->nlig += (b.d.nv + b.d.ligand_stride - 1) / b.d.ligand_stride;
    }
    c->nrec += (int)(I.rec[0].size() + I.rec[1].size());
    const int ntx = (I.lat.nx + c->TX - 1) / c->TX, nty = (I.lat.ny + c->TY - 1) / c->TY;
    c->ntiles += ntx * nty;
    c->nodes += (long long)row_pitch(I.lat.nx) * I.lat.ny;   // padded rows
  }
  const int packed = c->nchunk - grouped_chunks;
  c->nslot = (packed + kGroupChunks - 1) / kGroupChunks * kGroupChunks + kGroupChunks * grouped;
}

void compute_layout(lbib_ctx* c) {
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t o = cur;
    cur = align256(cur + std::max<size_t>(bytes, 8));
    return o;
  };
  Layout& L = c->L;
  const size_t es = elem_size(c->dtype);
  const size_t nm = std::max(c->nm, 1), nl = std::max(c->nlig, 1), nr = std::max(c->nrec, 1);
  L.lat = take(sizeof(LatDev) * c->ninst);
  L.body = take(sizeof(BodyDev) * std::max(c->nbody, 1));
  L.A = take(es * 9 * c->nodes);
  L.B = take(es * 9 * c->nodes);
  L.U = take(es * 2 * c->nodes);
  size_t* dbl[] = {&L.x, &L.y, &L.xm, &L.ym, &L.xn, &L.yn, &L.fx, &L.fy,
                   &L.l0, &L.th0, &L.r0x, &L.r0y};
  for (auto* o : dbl) *o = take(8 * nm);
  L.mbody = take(4 * nm);
  L.minfo = take(4 * nm);
  L.cx = take(4 * nm);
  L.cy = take(4 * nm);
  L.wx = take(8 * 9 * nm);   // 9 rows: the MLS weights; the Roma kernel uses 3
  L.wy = take(8 * 3 * nm);
  L.frep = take(8 * nm);
  L.obs = take(sizeof(lbib_body_obs) * (size_t)std::max(c->nbody, 1));
  L.rep_chunk = take(16 * (size_t)std::max(c->nrep_chunk, 1));
  for (auto& s : L.s) s = take(8 * nm);
  for (int k = 0; k < 2; ++k) {
    L.cnt[k] = take(4 * (size_t)c->ntiles);
    L.bins[k] = take(4 * (size_t)c->ntiles * c->bin_cap);
  }
  L.touched = take(4 * (size_t)c->ntiles);
  L.overflow = take(8);
  L.fmax = take(8 * 2 * (size_t)c->ninst);        // two slots, by step parity
  L.bond_flag = take(4 * 2 * (size_t)c->ninst);
  L.step_slot = take(8 * 2 * (size_t)c->ninst);
  L.spin = take(8);
  L.Uspare = take(es * 2 * c->nodes);   // velocity output of measurement launches
  L.tile_inst = take(4 * c->ntiles);
  L.lig_body = take(4 * nl);
  L.lig_elem = take(4 * nl);
  L.l2r = take(4 * nl);
  L.lig_flag = take(4 * nl);
  L.lig_va = take(4 * nl);
  L.lig_vb = take(4 * nl);
  L.lig_sigma = take(8 * nl);
  L.lig_sp = take(8 * nl);
  L.r2l = take(4 * nr);
  L.rec_x = take(8 * nr);
  L.step_next = take(8 * c->ninst);
  L.step_cur = take(8 * c->ninst);
  L.ties = take(8 * c->ninst);
  L.red = take(8 * (6 * 1024 + 64));
  const size_t nch = (size_t)std::max(c->nchunk, 1);
  L.chunk_info = take(16 * nch);
  L.area_part = take(8 * 5 * nch);
  L.rig_part = take(8 * 3 * nch);
  L.body_cnt = take(4 * (size_t)std::max(c->nbody, 1));
  L.star = take(es * 4 * (size_t)c->nodes);
  L.pbox = take(4 * 4 * nch);
  L.star_wg = take(4 * 3 * (size_t)std::max(c->nstar_wg, 1));
  L.slot_chunk = take(8 * (size_t)std::max(c->nslot, 1));
  L.total = cur;
}

template <typename T>
Ptrs<T> make_ptrs(const lbib_ctx* c) {
  const Layout& L = c->L;
  char* w = c->ws;
  Ptrs<T> p{};
  p.lat = (LatDev*)(w + L.lat);
  p.body = (BodyDev*)(w + L.body);
  T* a = (T*)(w + L.A);
  T* b = (T*)(w + L.B);
  if (c->inplace) {
    // one buffer; layout P (scheme 1) at even parity, S (scheme 2) at odd
    p.A = p.B = a;
    p.sch = 1 + c->parity;
    p.sch_next = 1 + (c->parity ^ 1);
  } else {
    p.A = c->parity == 0 ? a : b;
    p.B = c->parity == 0 ? b : a;
    p.sch = p.sch_next = 0;
  }
  p.U = (T*)(w + L.U);
  p.x = (double*)(w + L.x); p.y = (double*)(w + L.y);
  p.xm = (double*)(w + L.xm); p.ym = (double*)(w + L.ym);
  p.xn = (double*)(w + L.xn); p.yn = (double*)(w + L.yn);
  p.fx = (double*)(w + L.fx); p.fy = (double*)(w + L.fy);
  p.l0 = (double*)(w + L.l0); p.th0 = (double*)(w + L.th0);
  p.r0x = (double*)(w + L.r0x); p.r0y = (double*)(w + L.r0y);
  p.mbody = (int*)(w + L.mbody);
  p.minfo = (int*)(w + L.minfo);
  p.cx = (int*)(w + L.cx); p.cy = (int*)(w + L.cy);
  p.wx = (double*)(w + L.wx); p.wy = (double*)(w + L.wy);
  p.frep = (double*)(w + L.frep);
  double** sp[] = {&p.s_len, &p.s_nx, &p.s_ny, &p.s_bc, &p.s_bnx, &p.s_bny, &p.s_bfl, &p.s_fex, &p.s_fey};
  for (int k = 0; k < 9; ++k) *sp[k] = (double*)(w + L.s[k]);
  p.cnt_cur = (int*)(w + L.cnt[c->parity]);
  p.cnt_next = (int*)(w + L.cnt[c->parity ^ 1]);
  p.bin_cur = (int*)(w + L.bins[c->parity]);
  p.bin_next = (int*)(w + L.bins[c->parity ^ 1]);
  p.touched = (int*)(w + L.touched);
  p.overflow = (int*)(w + L.overflow);
  {
    const int cur = c->parity, oth = c->parity ^ 1;
    const size_t ni = (size_t)c->ninst;
    p.fmax_bits = (unsigned long long*)(w + L.fmax) + cur * ni;
    p.fmax_next = (unsigned long long*)(w + L.fmax) + oth * ni;
    p.bond_flag = (int*)(w + L.bond_flag) + cur * ni;
    p.bond_flag_next = (int*)(w + L.bond_flag) + oth * ni;
    p.step_slot = (long long*)(w + L.step_slot) + cur * ni;
    p.step_prev = (long long*)(w + L.step_slot) + oth * ni;
  }
  p.spin_timeouts = (int*)(w + L.spin);
  p.bin_cap = c->bin_cap;
  p.tile_inst = (int*)(w + L.tile_inst);
  p.lig_body = (int*)(w + L.lig_body);
  p.lig_elem = (int*)(w + L.lig_elem);
  p.l2r = (int*)(w + L.l2r);
  p.lig_flag = (int*)(w + L.lig_flag);
  p.lig_va = (int*)(w + L.lig_va);
  p.lig_vb = (int*)(w + L.lig_vb);
  p.lig_sigma = (double*)(w + L.lig_sigma);
  p.lig_sp = (double*)(w + L.lig_sp);
  p.r2l = (int*)(w + L.r2l);
  p.rec_x = (double*)(w + L.rec_x);
  p.step_next = (long long*)(w + L.step_next);
  p.step_cur = (long long*)(w + L.step_cur);
  p.ties = (unsigned long long*)(w + L.ties);
  p.red = (double*)(w + L.red);
  p.chunk_info = (const int4*)(w + L.chunk_info);
  p.area_part = (double*)(w + L.area_part);
  p.rig_part = (double*)(w + L.rig_part);
  p.body_cnt = (int*)(w + L.body_cnt);
  p.star = (T*)(w + L.star);
  p.pbox = (int*)(w + L.pbox);
  p.star_wg = (const int*)(w + L.star_wg);
  p.nstar_wg = c->nstar_wg;
  p.slot_chunk = (const int2*)(w + L.slot_chunk);
  p.nslot = c->nslot;
  p.nm_total = c->nm;
  p.nbody_total = c->nbody;
  p.ntile_total = c->ntiles;
  p.ninst = c->ninst;
  p.nlig_total = c->nlig;
  p.nchunk_total = c->nchunk;
  return p;
}

// LDS bytes for a particle workgroup's cache of rho*, u*: the node box that
// its vertex and probe stencils reach (extent + probe 1.2 + stencil 1 + margin
// 2 on each side), with 10 % spare for deformation; 16 KB to 96 KB.
int body_cache_bytes(const lbib_ctx* c) {
  const int es = elem_size(c->dtype);
  long long need = 0;
  for (auto& I : c->inst)
    for (auto& b : I.bodies) {
      if (b.d.kind == LBIB_RBC_KINEMATIC) continue;
      double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
      for (int v = 0; v < b.d.nv; ++v) {
        x0 = std::min(x0, b.xy[2 * v]); x1 = std::max(x1, b.xy[2 * v]);
        y0 = std::min(y0, b.xy[2 * v + 1]); y1 = std::max(y1, b.xy[2 * v + 1]);
      }
      const double pad = 2.0 * (1.2 + 1.0 + 2.0) + 2.0;
      const long long nodes = (long long)std::ceil(x1 - x0 + pad) * (long long)std::ceil(y1 - y0 + pad);
      need = std::max(need, nodes * 3 * es * 11 / 10);
    }
  const long long lo = 16 * 1024, hi = 96 * 1024;
  need = std::min(std::max(need, lo), hi);
  return (int)((need + 255) & ~255ll);
}

StepArgs step_args(const lbib_ctx* c) {
  StepArgs a;
  a.tile_x = c->TX;
  a.tile_y = c->TY;
  a.ntiles_total = c->ntiles;
  a.max_inst_tiles = 0;
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const int nt = ((c->inst[i].lat.nx + c->TX - 1) / c->TX) * ((c->inst[i].lat.ny + c->TY - 1) / c->TY);
    a.max_inst_tiles = std::max(a.max_inst_tiles, nt);
  }
  a.body_cache_bytes = c->body_cache;
  a.lb_wpc = c->lb_wpc;
  a.n_cu = c->n_cu;
  a.max_nv = 0;
  a.any_mls = 0;
  // automatic cache hints: non-temporal loads and stores on a single lattice
  // whose two population buffers stay well inside the 256 MB last-level cache
  // (28.8 MB measured), plain accesses otherwise (with 256-byte aligned rows
  // they measured as fast or faster on 320 MB, and on batches); the
  // autotuner times all three forms
  const double pop_bytes = 2.0 * 9.0 * (double)c->nodes * (double)elem_size(c->dtype);
  a.nt_mode = c->cache_hints >= 0 ? c->cache_hints
                                  : (c->ninst == 1 && pop_bytes <= 128.0 * 1024 * 1024 ? 3 : 0);
  for (auto& I : c->inst) {
    for (auto& b : I.bodies) a.max_nv = std::max(a.max_nv, b.d.nv);
    if (I.transfer == LBIB_TRANSFER_MLS) a.any_mls = 1;
  }
  return a;
}

// Stress-free state of a closed chain (host, float64).
void rest_state(const std::vector<double>& xy, int nv, std::vector<double>& l0,
                std::vector<double>& th0, double& A) {
  l0.resize(nv);
  th0.resize(nv);
  A = 0.0;
  for (int v = 0; v < nv; ++v) {
    const int vp = (v + 1) % nv, vm = (v + nv - 1) % nv;
    const double dxr = xy[2 * vp] - xy[2 * v], dyr = xy[2 * vp + 1] - xy[2 * v + 1];
    const double lr = std::sqrt(dxr * dxr + dyr * dyr);
    const double dxl = xy[2 * v] - xy[2 * vm], dyl = xy[2 * v + 1] - xy[2 * vm + 1];
    const double ll = std::sqrt(dxl * dxl + dyl * dyl);
    const double txr = dxr / lr, tyr = dyr / lr, txl = dxl / ll, tyl = dyl / ll;
    l0[v] = lr;
    th0[v] = std::atan2(txl * tyr - tyl * txr, txl * txr + tyl * tyr);
    A += xy[2 * v] * xy[2 * vp + 1] - xy[2 * vp] * xy[2 * v + 1];
  }
  A *= 0.5;
}

// Streaming scheme: in place when asked, or (automatic) when the one
// population buffer takes at most 192 MB, so that a step's whole working
// set stays in the 256 MB last-level cache; two buffers otherwise.
bool resolve_inplace(const lbib_ctx* c) {
  if (c->streaming >= 0) return c->streaming == 1;
  return (double)elem_size(c->dtype) * 9.0 * (double)c->nodes <= 192.0 * 1024 * 1024;
}

// nx * ny of every instance (the node counts of the conversion launches).
std::vector<long long> inst_nodes(const lbib_ctx* c) {
  std::vector<long long> n;
  for (auto& I : c->inst) n.push_back((long long)I.lat.nx * I.lat.ny);
  return n;
}

// In place: the state's populations between A (in the state's layout) and
// B in scheme-0 order; to = 1 copies A into B, to = 0 B into A.
template <typename T>
lbib_status canon_populations(lbib_ctx* c, int to) {
  const std::vector<long long> n = inst_nodes(c);
  launch_canon<T>(make_ptrs<T>(c), c->ninst, n.data(), (T*)(c->ws + c->L.B), to, c->stream);
  HIPCHK(c, hipGetLastError());
  return LBIB_OK;
}

lbib_status canon_any(lbib_ctx* c, int to) {
  return c->dtype == LBIB_F64 ? canon_populations<double>(c, to) : canon_populations<float>(c, to);
}

// The state's populations in scheme-0 order where state_regions points
// (before a save; in place they are staged in B) ...
lbib_status stage_state(lbib_ctx* c) { return c->inplace ? canon_any(c, 1) : LBIB_OK; }
// ... and back into the state's layout (after a restore).
lbib_status unstage_state(lbib_ctx* c) { return c->inplace ? canon_any(c, 0) : LBIB_OK; }

template <typename T>
lbib_status upload_all(lbib_ctx* c) {
  const Layout& L = c->L;
  hipStream_t s = c->stream;
  std::vector<LatDev> lat(c->ninst);
  std::vector<BodyDev> bodies(std::max(c->nbody, 1));
  const size_t nm = std::max(c->nm, 1);
  std::vector<double> x(nm), y(nm), l0(nm), th0(nm), r0x(nm, 0.0), r0y(nm, 0.0);
  std::vector<int> mbody(nm, 0), minfo(nm, 0);
  std::vector<int> tile_inst(std::max(c->ntiles, 1));
  std::vector<int> lig_body(std::max(c->nlig, 1)), lig_elem(std::max(c->nlig, 1));
  std::vector<int> lig_va(std::max(c->nlig, 1)), lig_vb(std::max(c->nlig, 1));
  std::vector<double> lig_sigma(std::max(c->nlig, 1), 0.0);
  std::vector<double> rec_x(std::max(c->nrec, 1));
  std::vector<int> chunk_info(4 * (size_t)std::max(c->nchunk, 1), 0);
  int bi = 0, li = 0, ci = 0;
  for (int i = 0; i < c->ninst; ++i) {
    InstHost& I = c->inst[i];
    LatDev& D = lat[i];
    std::memset(&D, 0, sizeof(D));
    D.nx = I.lat.nx; D.ny = I.lat.ny; D.periodic_y = I.lat.periodic_y;
    D.ntx = (D.nx + c->TX - 1) / c->TX;
    D.nty = (D.ny + c->TY - 1) / c->TY;
    D.tile_base = c->tile_base[i];
    D.pitch = row_pitch(D.nx);
    D.plane = (long long)D.pitch * D.ny;
    D.marker_base = c->marker_base[i];
    D.body_base = c->body_base[i];
    D.n_bodies = (int)I.bodies.size();
    D.lig_base = c->lig_base[i];
    D.rec_base = c->rec_base[i];
    D.n_rec0 = (int)I.rec[0].size();
    D.n_rec1 = (int)I.rec[1].size();
    D.instance = I.lat.instance;
    D.node_base = c->node_base[i];
    D.tau = I.lat.tau; D.gx = I.lat.gx; D.gy = I.lat.gy;
    D.omega = 1.0 / D.tau;
    D.pre = 1.0 - 0.5 / D.tau;
    D.seed = I.lat.seed;
    D.y_cr = I.adh.y_cr; D.y_eq = I.adh.y_eq; D.kf0_dt = I.adh.kf0_dt; D.kr0_dt = I.adh.kr0_dt;
    D.sigma_ts_frac = I.adh.sigma_ts_frac; D.kbt = I.adh.kbt; D.freeze = I.adh.freeze_topology;
    D.rep_coeff = I.rep_coeff; D.rep_cutoff = I.rep_cutoff;
    D.wall_mode = I.wall_mode;
    D.u_wall_lo = I.u_wall_lo; D.u_wall_hi = I.u_wall_hi;
    D.y_wall_lo = I.wall_mode == 1 ? 0.0 : -0.5;
    D.y_wall_hi = I.wall_mode == 1 ? I.lat.ny - 1.0 : I.lat.ny - 0.5;
    D.transfer = I.transfer;
    D.mls_weight = I.mls_weight;
    D.mls_h = I.mls_weight == LBIB_MLS_WEIGHT_ROMA ? 1.5 : I.mls_h;
    for (int t = 0; t < D.ntx * D.nty; ++t) tile_inst[D.tile_base + t] = i;
    int m = D.marker_base, nl = 0;
    for (auto& b : I.bodies) {
      BodyDev& B = bodies[bi];
      std::memset(&B, 0, sizeof(B));
      B.kind = b.d.kind; B.nv = b.d.nv; B.v0 = m; B.inst = i;
      B.ks = b.d.ks; B.kb = b.d.kb; B.ka = b.d.ka; B.p_ref = b.d.p_ref; B.sigma = b.d.sigma;
      B.lig_stride = b.d.ligand_stride;
      B.lig_base = D.lig_base + nl;
      B.chunk0 = ci;
      for (int k = 0; k < chunks_of(b.d.nv); ++k, ++ci) {
        const int first = k * kChunk;
        chunk_info[4 * ci] = bi;
        chunk_info[4 * ci + 1] = m + first - 2;
        chunk_info[4 * ci + 2] = std::min(kChunk, b.d.nv - first);
        chunk_info[4 * ci + 3] = b.d.kind | (i << 2);
      }
      std::vector<double> bl0, bth0;
      double A0;
      rest_state(b.xy, b.d.nv, bl0, bth0, A0);
      B.A0 = A0;
      B.mass = b.d.density_ratio * 1.0 * A0;
      B.mv = B.mass / b.d.nv;
      double xc = 0, yc = 0;
      for (int v = 0; v < b.d.nv; ++v) { xc += b.xy[2 * v]; yc += b.xy[2 * v + 1]; }
      xc /= b.d.nv; yc /= b.d.nv;
      double r2 = 0;
      for (int v = 0; v < b.d.nv; ++v) {
        x[m + v] = b.xy[2 * v];
        y[m + v] = b.xy[2 * v + 1];
        l0[m + v] = bl0[v];
        th0[m + v] = bth0[v];
        mbody[m + v] = bi;
        minfo[m + v] = (i << 2) | b.d.kind;
        if (b.d.kind == LBIB_PARTICLE_RIGID) {
          r0x[m + v] = b.xy[2 * v] - xc;
          r0y[m + v] = b.xy[2 * v + 1] - yc;
          r2 += r0x[m + v] * r0x[m + v] + r0y[m + v] * r0y[m + v];
        }
      }
      B.xc = xc; B.yc = yc; B.theta = 0.0;
      B.inertia = 0.5 * B.mass * (r2 / b.d.nv);
      if (b.d.ligand_stride > 0) {
        int k = 0;
        for (int e = 0; e < b.d.nv; e += b.d.ligand_stride, ++k) {
          lig_body[li] = bi;
          lig_elem[li] = e;
          lig_va[li] = m + e;
          lig_vb[li] = m + (e + 1) % b.d.nv;
          lig_sigma[li] = b.d.sigma;
          ++li;
        }
        B.n_lig = k;
        nl += k;
      }
      m += b.d.nv;
      ++bi;
    }
    D.n_markers = m - D.marker_base;
    D.n_lig = nl;
    for (int w = 0; w < 2; ++w)
      for (size_t k = 0; k < I.rec[w].size(); ++k)
        rec_x[D.rec_base + (w == 0 ? 0 : D.n_rec0) + k] = I.rec[w][k];
  }
  char* w = c->ws;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  HIPCHK(c, up(L.lat, lat.data(), sizeof(LatDev) * c->ninst));
  HIPCHK(c, up(L.body, bodies.data(), sizeof(BodyDev) * bodies.size()));
  HIPCHK(c, up(L.x, x.data(), 8 * nm));
  HIPCHK(c, up(L.y, y.data(), 8 * nm));
  HIPCHK(c, up(L.xm, x.data(), 8 * nm));
  HIPCHK(c, up(L.ym, y.data(), 8 * nm));
  HIPCHK(c, up(L.xn, x.data(), 8 * nm));
  HIPCHK(c, up(L.yn, y.data(), 8 * nm));
  HIPCHK(c, hipMemsetAsync(w + L.fx, 0, 8 * nm, s));
  HIPCHK(c, hipMemsetAsync(w + L.fy, 0, 8 * nm, s));
  HIPCHK(c, up(L.l0, l0.data(), 8 * nm));
  HIPCHK(c, up(L.th0, th0.data(), 8 * nm));
  HIPCHK(c, up(L.r0x, r0x.data(), 8 * nm));
  HIPCHK(c, up(L.r0y, r0y.data(), 8 * nm));
  HIPCHK(c, up(L.mbody, mbody.data(), 4 * nm));
  {
    // work units of the repulsion kernel: (body, first global vertex,
    // vertex count, instance) per chunk of kRepChunk vertices
    std::vector<int> chunks;
    for (int bb = 0; bb < c->nbody; ++bb)
      for (int v = 0; v < bodies[bb].nv; v += kRepChunk) {
        chunks.push_back(bb);
        chunks.push_back(bodies[bb].v0 + v);
        chunks.push_back(std::min(kRepChunk, bodies[bb].nv - v));
        chunks.push_back(bodies[bb].inst);
      }
    if (!chunks.empty()) HIPCHK(c, up(L.rep_chunk, chunks.data(), 4 * chunks.size()));
  }
  HIPCHK(c, up(L.minfo, minfo.data(), 4 * nm));
  const size_t nchk = chunk_info.size() / 4;
  HIPCHK(c, up(L.chunk_info, chunk_info.data(), 4 * chunk_info.size()));
  HIPCHK(c, hipMemsetAsync(w + L.area_part, 0, 8 * 5 * nchk, s));
  HIPCHK(c, hipMemsetAsync(w + L.rig_part, 0, 8 * 3 * nchk, s));
  HIPCHK(c, hipMemsetAsync(w + L.body_cnt, 0, 4 * (size_t)std::max(c->nbody, 1), s));
  HIPCHK(c, hipMemsetAsync(w + L.star, 0, (size_t)elem_size(c->dtype) * 4 * c->nodes, s));
  HIPCHK(c, hipMemsetAsync(w + L.pbox, 0, 4 * 4 * nchk, s));
  {
    // star work list: (body, rank, workgroups of the body) per workgroup
    std::vector<int> sw;
    for (int i = 0, bb = 0; i < c->ninst; ++i)
      for (auto& b : c->inst[i].bodies) {
        const int K = star_workgroups(b);
        for (int r = 0; r < K; ++r) {
          sw.push_back(bb);
          sw.push_back(r);
          sw.push_back(K);
        }
        ++bb;
      }
    if (!sw.empty()) HIPCHK(c, up(L.star_wg, sw.data(), 4 * sw.size()));
  }
  {
    // waves of the chunked body kernel, as (chunk, body): one workgroup per
    // grouped rigid body first (chunk c on wave c, idle waves -2), then the
    // chunks of the other particles and of the red cells, packed (the
    // particles' chains are the longer ones: they start first)
    std::vector<int> sl;
    for (int bb = 0; bb < c->nbody; ++bb)
      if (rigid_grouped(bodies[bb].kind, bodies[bb].nv))
        for (int k = 0; k < kGroupChunks; ++k) {
          sl.push_back(k < chunks_of(bodies[bb].nv) ? bodies[bb].chunk0 + k : -2);
          sl.push_back(bb);
        }
    for (int pass = 0; pass < 2; ++pass)
      for (int bb = 0; bb < c->nbody; ++bb) {
        const bool rbc = bodies[bb].kind == LBIB_RBC_KINEMATIC;
        if (rigid_grouped(bodies[bb].kind, bodies[bb].nv) || rbc != (pass == 1)) continue;
        for (int k = 0; k < chunks_of(bodies[bb].nv); ++k) {
          sl.push_back(bodies[bb].chunk0 + k);
          sl.push_back(bb);
        }
      }
    while (sl.size() % (2 * kGroupChunks)) {
      sl.push_back(-1);
      sl.push_back(0);
    }
    if ((int)sl.size() != 2 * c->nslot) return fail(c, LBIB_EINVAL, "internal: wave slot count");
    if (!sl.empty()) HIPCHK(c, up(L.slot_chunk, sl.data(), 4 * sl.size()));
  }
  HIPCHK(c, up(L.tile_inst, tile_inst.data(), 4 * tile_inst.size()));
  HIPCHK(c, up(L.lig_body, lig_body.data(), 4 * lig_body.size()));
  HIPCHK(c, up(L.lig_elem, lig_elem.data(), 4 * lig_elem.size()));
  HIPCHK(c, up(L.lig_va, lig_va.data(), 4 * lig_va.size()));
  HIPCHK(c, up(L.lig_vb, lig_vb.data(), 4 * lig_vb.size()));
  HIPCHK(c, up(L.lig_sigma, lig_sigma.data(), 8 * lig_sigma.size()));
  HIPCHK(c, hipMemsetAsync(w + L.lig_sp, 0, 8 * lig_sigma.size(), s));
  HIPCHK(c, hipMemsetAsync(w + L.l2r, 0xff, 4 * std::max(c->nlig, 1), s));
  HIPCHK(c, hipMemsetAsync(w + L.r2l, 0xff, 4 * std::max(c->nrec, 1), s));
  HIPCHK(c, up(L.rec_x, rec_x.data(), 8 * rec_x.size()));
  HIPCHK(c, hipMemsetAsync(w + L.step_next, 0, 8 * c->ninst, s));
  HIPCHK(c, hipMemsetAsync(w + L.step_cur, 0, 8 * c->ninst, s));
  HIPCHK(c, hipMemsetAsync(w + L.ties, 0, 8 * c->ninst, s));
  // marker bins: empty until the stencil pass before the first step
  for (int k = 0; k < 2; ++k) HIPCHK(c, hipMemsetAsync(w + L.cnt[k], 0, 4 * (size_t)c->ntiles, s));
  HIPCHK(c, hipMemsetAsync(w + L.touched, 0, 4 * (size_t)c->ntiles, s));
  HIPCHK(c, hipMemsetAsync(w + L.overflow, 0, 8, s));
  HIPCHK(c, hipMemsetAsync(w + L.frep, 0, 8 * nm, s));
  HIPCHK(c, hipMemsetAsync(w + L.obs, 0, sizeof(lbib_body_obs) * (size_t)std::max(c->nbody, 1), s));
  HIPCHK(c, hipMemsetAsync(w + L.fmax, 0, 8 * 2 * (size_t)c->ninst, s));
  HIPCHK(c, hipMemsetAsync(w + L.bond_flag, 0, 4 * 2 * (size_t)c->ninst, s));
  HIPCHK(c, hipMemsetAsync(w + L.step_slot, 0, 8 * 2 * (size_t)c->ninst, s));
  HIPCHK(c, hipMemsetAsync(w + L.spin, 0, 8, s));
  HIPCHK(c, hipStreamSynchronize(s));
  // populations: equilibrium of the initial fields, shifted by the weights
  for (int i = 0; i < c->ninst; ++i) {
    InstHost& I = c->inst[i];
    const int nx = I.lat.nx, pitch = row_pitch(nx);
    const long long N = (long long)pitch * I.lat.ny;
    std::vector<T> h(9 * N, T(0));   // row padding stays zero
    for (long long k = 0; k < (long long)nx * I.lat.ny; ++k) {
      const double rho = I.rho0.empty() ? 1.0 : I.rho0[k];
      const double ux = I.ux0.empty() ? 0.0 : I.ux0[k];
      const double uy = I.uy0.empty() ? 0.0 : I.uy0[k];
      const double uu = ux * ux + uy * uy;
      const long long node = (k / nx) * pitch + k % nx;
      for (int q = 0; q < 9; ++q) {
        const double eu = ex(q) * ux + ey(q) * uy;
        const double w8 = wq<double>(q);
        h[q * N + node] = T(w8 * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
      }
    }
    // two buffers: straight into A; in place: into B in scheme-0 order,
    // then into A in the state's layout
    HIPCHK(c, hipMemcpyAsync(w + (c->inplace ? L.B : L.A) + 9 * c->node_base[i] * sizeof(T), h.data(),
                             sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  c->parity = 0;
  if (c->inplace) {
    lbib_status st = canon_populations<T>(c, 0);
    if (st != LBIB_OK) return st;
  } else {
    HIPCHK(c, hipMemsetAsync(w + L.B, 0, sizeof(T) * 9 * c->nodes, s));
  }
  HIPCHK(c, hipMemsetAsync(w + L.U, 0, sizeof(T) * 2 * c->nodes, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->step = 0;
  c->stencil_dirty = true;
  return LBIB_OK;
}

// n steps.  With merge_advance, two kernels each: the Lagrangian kernel
// (which, after the first step, also finishes the previous step's marker
// advance for its own bodies) and the fused lattice kernel, and the last
// step ends with the marker advance of all markers.  Otherwise three kernels
// each: Lagrangian, fused lattice, marker advance.
// Step form of the context: three kernels (body, lattice, advance), the
// merged form (the body kernel finishes the previous step's advance; only
// when every body has <= kSmallBody vertices, where one round of the
// workgroup covers them), or the overlapped form (the lattice tiles without IB force
// on a second stream while the body kernel runs).  Automatic: merged when
// possible, else three kernels (measured faster than the overlapped form on
// the 2000 x 200 and 6667 x 667 capillaries and the 64-instance sweep).
// The vertex repulsion needs X^n of every body before any body's forces,
// which the merged form cannot give (there each body workgroup finishes its
// own advance): with the repulsion on, the merged form is not used.
void resolve_step_mode(lbib_ctx* c) {
  bool small_bodies = true;
  c->repulsion = false;
  for (auto& I : c->inst) {
    for (auto& b : I.bodies)
      if (b.d.nv > kSmallBody) small_bodies = false;
    if (I.rep_coeff > 0.0 && !I.bodies.empty()) c->repulsion = true;
  }
  int m = c->step_mode;
  if (m == 0) m = small_bodies && !c->repulsion ? 2 : 1;
  c->merge_advance = m == 2 && small_bodies && !c->repulsion;
  c->overlap = m == 3;
}

template <typename T>
void enqueue_steps(lbib_ctx* c, long long n) {
  const StepArgs a = step_args(c);
  if (c->overlap && !c->ktiming) {
    for (long long k = 0; k < n; ++k) {
      Ptrs<T> p = make_ptrs<T>(c);
      if (c->repulsion) launch_repulsion<T>(p, a, (const int*)(c->ws + c->L.rep_chunk), c->nrep_chunk, c->stream);
      (void)hipEventRecord(c->ev_fork, c->stream);
      (void)hipStreamWaitEvent(c->aux, c->ev_fork, 0);
      launch_lb_fused<T>(p, a, c->aux, 1 | (1 << 2));        // tiles without IB force
      (void)hipEventRecord(c->ev_join, c->aux);
      launch_lagrangian<T>(p, a, c->stream, false);
      launch_lb_fused<T>(p, a, c->stream, 1 | (2 << 2));     // tiles with IB force
      (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
      launch_advance<T>(p, a, c->stream);
      c->parity ^= 1;
    }
    return;
  }
  for (long long k = 0; k < n; ++k) {
    Ptrs<T> p = make_ptrs<T>(c);
    if (c->repulsion) launch_repulsion<T>(p, a, (const int*)(c->ws + c->L.rep_chunk), c->nrep_chunk, c->stream);
    launch_lagrangian<T>(p, a, c->stream, c->merge_advance && k > 0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->ktiming && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      launch_lb_fused<T>(p, a, c->stream, 3, e0, e1);
      c->kevents.emplace_back(e0, e1);
    } else {
      launch_lb_fused<T>(p, a, c->stream);
    }
    if (!c->merge_advance || k == n - 1) launch_advance<T>(p, a, c->stream);
    c->parity ^= 1;
  }
}

void drop_kevents(lbib_ctx* c) {
  for (auto& e : c->kevents) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  c->kevents.clear();
}

void drop_adjoint_graphs(lbib_ctx* c) {
  for (auto& kv : c->adj_graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : c->adj_rgraphs) (void)hipGraphExecDestroy(kv.second);
  c->adj_graphs.clear();
  c->adj_rgraphs.clear();
}

void drop_graphs(lbib_ctx* c) {
  for (auto& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

template <typename T>
lbib_status run_steps(lbib_ctx* c, long long n) {
  if (c->ktiming) {
    // measurement mode: plain launches with event pairs around the fused kernel
    if (c->stencil_dirty && n > 0) {
      HIPCHK(c, hipMemsetAsync(c->ws + c->L.cnt[c->parity], 0, 4 * (size_t)c->ntiles, c->stream));
      launch_stencil<T>(make_ptrs<T>(c), step_args(c), c->stream);
      c->stencil_dirty = false;
    }
    enqueue_steps<T>(c, n);
    c->step += n;
    HIPCHK(c, hipGetLastError());
    return LBIB_OK;
  }
  if (c->stencil_dirty && n > 0) {
    // rebuild the current bin set from the marker positions (eager, never
    // part of a captured graph)
    HIPCHK(c, hipMemsetAsync(c->ws + c->L.cnt[c->parity], 0, 4 * (size_t)c->ntiles, c->stream));
    launch_stencil<T>(make_ptrs<T>(c), step_args(c), c->stream);
    c->stencil_dirty = false;
  }
  const int G = c->graph_steps;
  if (G > 0) {
    while (n >= G) {
      int par = c->parity;
      if (!c->gexec[par]) {
        hipGraph_t graph;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        enqueue_steps<T>(c, G);
        HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
        c->parity = par;  // capture did not execute anything
        hipGraphExec_t ex_;
        hipError_t e = hipGraphInstantiate(&ex_, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(c, LBIB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        c->gexec[par] = ex_;
      }
      HIPCHK(c, hipGraphLaunch(c->gexec[par], c->stream));
      c->parity = par ^ (G & 1);
      c->step += G;
      n -= G;
    }
  }
  enqueue_steps<T>(c, n);
  c->step += n;
  HIPCHK(c, hipGetLastError());
  return LBIB_OK;
}

template <typename T>
lbib_status diag_impl(lbib_ctx* c, double out[6]) {
  Ptrs<T> p = make_ptrs<T>(c);
  double* dout = p.red + 6 * 1024;
  launch_diag<T>(p, step_args(c), c->nodes, dout, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(out, dout, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBIB_OK;
}

// Reference mass of the watchdog's drift check, from the current state.
lbib_status record_mass(lbib_ctx* c) {
  for (auto& I : c->inst)
    if (I.wall_mode != 0) {
      c->mass_ref = NAN;   // velocity walls exchange mass with the outside
      return LBIB_OK;
    }
  double d[6];
  lbib_status s = c->dtype == LBIB_F64 ? diag_impl<double>(c, d) : diag_impl<float>(c, d);
  if (s != LBIB_OK) return s;
  c->mass_ref = d[0];
  return LBIB_OK;
}

template <typename T>
lbib_status fields_impl(lbib_ctx* c, int inst, double* rho, double* ux, double* uy) {
  const InstHost& I = c->inst[inst];
  const long long N = (long long)I.lat.nx * I.lat.ny;
  Ptrs<T> p = make_ptrs<T>(c);
  // stage in the population buffer the state does not hold (two buffers: the
  // one the next step rewrites in full; in place: the spare)
  double* stage = c->inplace ? (double*)(c->ws + c->L.B) : (double*)p.B;
  launch_fields<T>(p, step_args(c), inst, stage, stage + N, stage + 2 * N, I.lat.nx, I.lat.ny,
                   c->node_base[inst], c->stream);
  HIPCHK(c, hipGetLastError());
  std::vector<double> tmp(3 * N);
  HIPCHK(c, hipMemcpyAsync(tmp.data(), stage, 3 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (rho) std::memcpy(rho, tmp.data(), N * sizeof(double));
  if (ux) std::memcpy(ux, tmp.data() + N, N * sizeof(double));
  if (uy) std::memcpy(uy, tmp.data() + 2 * N, N * sizeof(double));
  return LBIB_OK;
}

lbib_status check_body(lbib_ctx* c, int inst, int body) {
  if (inst < 0 || inst >= c->ninst) return fail(c, LBIB_EINVAL, "instance out of range");
  if (body < 0 || body >= (int)c->inst[inst].bodies.size()) return fail(c, LBIB_EINVAL, "body out of range");
  return LBIB_OK;
}

int body_v0(const lbib_ctx* c, int inst, int body) {
  int v = c->marker_base[inst];
  for (int k = 0; k < body; ++k) v += c->inst[inst].bodies[k].d.nv;
  return v;
}

// Dynamic-state regions saved by get_state.
std::vector<std::pair<size_t, size_t>> state_regions(const lbib_ctx* c) {
  const Layout& L = c->L;
  const size_t es = elem_size(c->dtype);
  const size_t nm = std::max(c->nm, 1), nl = std::max(c->nlig, 1), nr = std::max(c->nrec, 1);
  // in place, the state's populations travel in scheme-0 order through B
  // (staged by stage_state / unstage_state)
  const size_t Aoff = c->inplace ? L.B : (c->parity == 0 ? L.A : L.B);
  std::vector<std::pair<size_t, size_t>> r = {
      {Aoff, es * 9 * c->nodes}, {L.U, es * 2 * c->nodes},
      {L.body, sizeof(BodyDev) * std::max(c->nbody, 1)},
      {L.x, 8 * nm}, {L.y, 8 * nm}, {L.xm, 8 * nm}, {L.ym, 8 * nm}, {L.xn, 8 * nm}, {L.yn, 8 * nm},
      {L.fx, 8 * nm}, {L.fy, 8 * nm}, {L.cx, 4 * nm}, {L.cy, 4 * nm}, {L.wx, 72 * nm}, {L.wy, 24 * nm},
      {L.touched, 4 * (size_t)c->ntiles},
      {L.l2r, 4 * nl}, {L.r2l, 4 * nr}, {L.lig_sigma, 8 * nl}, {L.step_next, 8 * (size_t)c->ninst},
      {L.step_cur, 8 * (size_t)c->ninst}, {L.ties, 8 * (size_t)c->ninst}};
  return r;
}

struct StateHeader {
  uint64_t magic, bytes, step;
  int32_t dtype, ninst, nm, nbody, nlig, nrec, ntiles, pad;
  int64_t nodes;
};
constexpr uint64_t kMagic = 0x4c4249425354ull;  // "LBIBST"


// ------------------------------------------------------------ adjoint window
// Workspace of the adjoint: checkpoints of the dynamic state every k steps
// (plus the end of the window), a segment store with the forward data of k
// steps, and the float64 adjoint state and per-step scratch.
struct AdjLayout {
  size_t ck_bytes;
  int nseg, nck;
  size_t ck;
  size_t rec_bytes, r_h, r_x, r_y, r_fx, r_fy, r_xn, r_yn, r_u, r_b0, r_b1;
  size_t seg[2];   // two segment stores: recompute into one while the other is reversed
  size_t ha, fph, FE, FEh, mom, Uh, Rh, bad, xa, ya, xma, yma;
  size_t mk[13];
  size_t grad, rig;
  size_t total;
};

AdjLayout adj_layout(const lbib_ctx* c, long long K, int k) {
  AdjLayout A{};
  size_t cur = 0;
  auto take = [&](size_t b) {
    size_t o = cur;
    cur = align256(cur + std::max<size_t>(b, 8));
    return o;
  };
  for (auto& r : state_regions(c)) A.ck_bytes += align256(r.second);
  A.nseg = (int)((K + k - 1) / k);
  A.nck = A.nseg + 1;
  A.ck = take(A.ck_bytes * (size_t)A.nck);
  const size_t es = elem_size(c->dtype), nm = std::max(c->nm, 1);
  const size_t N = (size_t)c->nodes;
  size_t rb = 0;
  auto rt = [&](size_t b) {
    size_t o = rb;
    rb = align256(rb + std::max<size_t>(b, 8));
    return o;
  };
  A.r_h = rt(es * 9 * N);
  A.r_x = rt(8 * nm); A.r_y = rt(8 * nm);
  A.r_fx = rt(8 * nm); A.r_fy = rt(8 * nm);
  A.r_xn = rt(8 * nm); A.r_yn = rt(8 * nm);
  A.r_u = rt(es * 2 * N);
  // the bodies (rigid-particle state) before and after the step
  const size_t bb = sizeof(BodyDev) * (size_t)std::max(c->nbody, 1);
  A.r_b0 = rt(bb); A.r_b1 = rt(bb);
  A.rec_bytes = rb;
  A.seg[0] = take(rb * (size_t)k);
  A.seg[1] = take(rb * (size_t)k);
  A.ha = take(8 * 9 * N); A.fph = take(8 * 9 * N);
  // accumulators: a high and a low 64-bit word per entry (high words first)
  A.FE = take(32 * N); A.FEh = take(16 * N); A.mom = take(24 * N);
  A.Uh = take(32 * N); A.Rh = take(48 * N); A.bad = take(8);
  A.xa = take(8 * nm); A.ya = take(8 * nm); A.xma = take(8 * nm); A.yma = take(8 * nm);
  for (auto& o : A.mk) o = take(8 * nm);
  A.grad = take(24 * (size_t)std::max(c->nbody, 1));
  A.rig = take(72 * (size_t)std::max(c->nbody, 1));
  A.total = cur;
  return A;
}

AdjPtrs adj_ptrs(const lbib_ctx* c, const AdjLayout& A) {
  char* w = c->aws;
  AdjPtrs a{};
  a.ha = (double*)(w + A.ha); a.fph = (double*)(w + A.fph);
  const size_t N = (size_t)c->nodes;
  auto acc = [&](size_t off, size_t n) {
    return AccField{(long long*)(w + off), (long long*)(w + off + 8 * n)};
  };
  a.FE = acc(A.FE, 2 * N); a.Uh = acc(A.Uh, 2 * N); a.Rh = acc(A.Rh, 3 * N);
  a.FEh = (double*)(w + A.FEh); a.mom = (double*)(w + A.mom);
  a.bad = (int*)(w + A.bad);
  a.xa = (double*)(w + A.xa); a.ya = (double*)(w + A.ya);
  a.xma = (double*)(w + A.xma); a.yma = (double*)(w + A.yma);
  double** m[13] = {&a.dirx, &a.diry, &a.fvx, &a.fvy, &a.dsh, &a.Dx, &a.Dy,
                    &a.Cx, &a.Cy, &a.BLx, &a.BLy, &a.BRx, &a.BRy};
  for (int k = 0; k < 13; ++k) *m[k] = (double*)(w + A.mk[k]);
  a.grad = (double*)(w + A.grad);
  a.rig = (double*)(w + A.rig);
  return a;
}

// Save (or restore) the dynamic state to (from) checkpoint j.
void adj_checkpoint(lbib_ctx* c, const AdjLayout& A, int j, bool save) {
  char* base = c->aws + A.ck + (size_t)j * A.ck_bytes;
  if (save) (void)stage_state(c);
  CopyList cl{};
  size_t off = 0;
  for (auto& r : state_regions(c)) {
    if (cl.n == 24) {
      launch_copies(cl, c->stream);
      cl.n = 0;
    }
    cl.src[cl.n] = save ? c->ws + r.first : base + off;
    cl.dst[cl.n] = save ? base + off : c->ws + r.first;
    cl.bytes[cl.n] = r.second;
    ++cl.n;
    off += align256(r.second);
  }
  launch_copies(cl, c->stream);
  if (!save) (void)unstage_state(c);
}

lbib_status set_freeze(lbib_ctx* c, int32_t f) {
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.lat + offsetof(LatDev, freeze), &f, 4, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBIB_OK;
}

lbib_status adj_check_sizes(lbib_ctx* c) {
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "finalize_setup before binding an adjoint workspace");
  if (c->ninst != 1) return fail(c, LBIB_EINVAL, "the adjoint runs on single-lattice contexts");
  if (c->repulsion) return fail(c, LBIB_EINVAL, "the adjoint does not cover the vertex repulsion");
  if (c->inst[0].wall_mode != 0) return fail(c, LBIB_EINVAL, "the adjoint covers bounce-back walls only");
  if (c->inst[0].transfer != LBIB_TRANSFER_ROMA)
    return fail(c, LBIB_EINVAL, "the adjoint covers the Roma-kernel transfer only");
  return LBIB_OK;
}

lbib_status adj_check(lbib_ctx* c) {
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  if (c->ninst != 1) return fail(c, LBIB_EINVAL, "the adjoint runs on single-lattice contexts");
  if (c->repulsion) return fail(c, LBIB_EINVAL, "the adjoint does not cover the vertex repulsion");
  if (c->inst[0].wall_mode != 0) return fail(c, LBIB_EINVAL, "the adjoint covers bounce-back walls only");
  if (c->inst[0].transfer != LBIB_TRANSFER_ROMA)
    return fail(c, LBIB_EINVAL, "the adjoint covers the Roma-kernel transfer only");
  if (!c->aws) return fail(c, LBIB_ESTATE, "bind an adjoint workspace first");
  return LBIB_OK;
}

// J = mean over particle vertices of the distance to the nearer wall.
double wall_objective(const lbib_ctx* c, const std::vector<double>& y, std::vector<double>* dJdy) {
  const InstHost& I = c->inst[0];
  const double ny = I.lat.ny;
  int v = 0, np = 0;
  double s = 0.0;
  if (dJdy) dJdy->assign(y.size(), 0.0);
  for (auto& b : I.bodies) {
    if (b.d.kind != LBIB_RBC_KINEMATIC) np += b.d.nv;
  }
  for (auto& b : I.bodies) {
    for (int k = 0; k < b.d.nv; ++k, ++v) {
      if (b.d.kind == LBIB_RBC_KINEMATIC) continue;
      const double lo = y[v] + 0.5, hi = ny - 0.5 - y[v];
      s += lo <= hi ? lo : hi;
      if (dJdy) (*dJdy)[v] = (lo <= hi ? 1.0 : -1.0) / np;
    }
  }
  return np > 0 ? s / np : 0.0;
}

template <typename T>
lbib_status adjoint_forward_impl(lbib_ctx* c, double* J) {
  const AdjLayout A = adj_layout(c, c->adjK, c->adjk);
  const bool kt = c->ktiming;
  c->ktiming = false;
  lbib_status st = set_freeze(c, 1);
  if (st != LBIB_OK) return st;
  c->ck_step.assign(A.nck, 0);
  for (int j = 0; j < A.nseg; ++j) {
    c->ck_step[j] = c->step;
    adj_checkpoint(c, A, j, true);
    const long long n = std::min<long long>(c->adjk, c->adjK - (long long)j * c->adjk);
    st = run_steps<T>(c, n);
    if (st != LBIB_OK) return st;
  }
  c->ck_step[A.nseg] = c->step;
  adj_checkpoint(c, A, A.nseg, true);
  HIPCHK(c, hipGetLastError());
  c->adj_y.assign(std::max(c->nm, 1), 0.0);
  HIPCHK(c, hipMemcpyAsync(c->adj_y.data(), c->ws + c->L.y, 8 * (size_t)c->nm, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->adj_y.resize(c->nm);
  if (J) *J = wall_objective(c, c->adj_y, nullptr);
  st = set_freeze(c, c->inst[0].adh.freeze_topology);
  if (st != LBIB_OK) return st;
  c->ktiming = kt;
  c->adj_ready = true;
  return LBIB_OK;
}

// Recompute n steps from the restored state into segment store `buf`,
// keeping the forward data of each step (one copy launch per step, after its
// lattice kernel: the populations h^n are still in the read buffer, positions
// X^n, forces and particle positions X^{n+1} are set, u^n is written).
template <typename T>
void enqueue_recompute(lbib_ctx* c, const AdjLayout& A, int buf, long long n) {
  const long long N = c->nodes;
  const size_t es = elem_size(c->dtype), nmb = 8 * (size_t)c->nm;
  const size_t bb = sizeof(BodyDev) * (size_t)c->nbody;
  const StepArgs sa = step_args(c);
  char* seg = c->aws + A.seg[buf];
  if (bb > 0) {   // the bodies before the first step (later steps: after the previous one)
    CopyList cl{};
    cl.n = 1;
    cl.src[0] = c->ws + c->L.body;
    cl.dst[0] = seg + A.r_b0;
    cl.bytes[0] = bb;
    launch_copies(cl, c->stream);
  }
  for (long long s = 0; s < n; ++s) {
    char* rec = seg + (size_t)s * A.rec_bytes;
    Ptrs<T> p = make_ptrs<T>(c);
    launch_lagrangian<T>(p, sa, c->stream, c->merge_advance && s > 0);
    if (c->inplace) {
      // h^n in scheme-0 order, before the lattice kernel rewrites its buffer
      const long long nn = (long long)c->inst[0].lat.nx * c->inst[0].lat.ny;
      launch_canon<T>(p, 1, &nn, (T*)(rec + A.r_h), 1, c->stream);
    }
    launch_lb_fused<T>(p, sa, c->stream);
    CopyList cl{};
    const char* src[10] = {(const char*)p.A, (const char*)p.x, (const char*)p.y, (const char*)p.fx,
                           (const char*)p.fy, (const char*)p.xn, (const char*)p.yn, (const char*)p.U,
                           (const char*)p.body, (const char*)p.body};
    const size_t off[10] = {A.r_h, A.r_x, A.r_y, A.r_fx, A.r_fy, A.r_xn, A.r_yn, A.r_u, A.r_b1,
                            A.rec_bytes + A.r_b0};
    const size_t by[10] = {es * 9 * N, nmb, nmb, nmb, nmb, nmb, nmb, es * 2 * N, bb, bb};
    const int k0 = c->inplace ? 1 : 0;   // in place, h^n is stored already
    const int kn = bb == 0 ? 8 : (s + 1 < n ? 10 : 9);
    cl.n = kn - k0;
    for (int k = k0; k < kn; ++k) {
      cl.src[k - k0] = src[k];
      cl.dst[k - k0] = rec + off[k];
      cl.bytes[k - k0] = by[k];
    }
    launch_copies(cl, c->stream);
    if (!c->merge_advance || s == n - 1) launch_advance<T>(p, sa, c->stream);
    c->parity ^= 1;
  }
}

// Reverse sweep over the n steps held in segment store `buf`, on stream s.
template <typename T>
void enqueue_reverse(lbib_ctx* c, const AdjLayout& A, AdjPtrs a, int buf, long long n, bool first,
                     hipStream_t s) {
  std::vector<AdjPtrs> steps((size_t)n, a);
  for (long long k = 0; k < n; ++k) {
    const char* rec = c->aws + A.seg[buf] + (size_t)k * A.rec_bytes;
    AdjPtrs& q = steps[(size_t)k];
    q.h = rec + A.r_h;
    q.x = (const double*)(rec + A.r_x); q.y = (const double*)(rec + A.r_y);
    q.fx = (const double*)(rec + A.r_fx); q.fy = (const double*)(rec + A.r_fy);
    q.xn = (const double*)(rec + A.r_xn); q.yn = (const double*)(rec + A.r_yn);
    q.u = rec + A.r_u;
    q.body0 = (const BodyDev*)(rec + A.r_b0);
    q.body1 = (const BodyDev*)(rec + A.r_b1);
    q.first = first && k == 0;
  }
  launch_adjoint_segment<T>(make_ptrs<T>(c), steps.data(), (int)n, c->nodes, s);
}

// Capture `enqueue` on stream s once per key; return the executable graph.
template <typename F>
lbib_status cached_graph(lbib_ctx* c, std::map<std::tuple<long long, int, int>, hipGraphExec_t>& cache,
                         std::tuple<long long, int, int> key, hipStream_t s, F enqueue,
                         hipGraphExec_t* out) {
  auto it = cache.find(key);
  if (it == cache.end()) {
    hipGraph_t graph;
    HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue();
    HIPCHK(c, hipStreamEndCapture(s, &graph));
    hipGraphExec_t ex_;
    hipError_t e = hipGraphInstantiate(&ex_, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, LBIB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it = cache.emplace(key, ex_).first;
  }
  *out = it->second;
  return LBIB_OK;
}

template <typename T>
lbib_status adjoint_backward_impl(lbib_ctx* c, double dJ, double* grad) {
  const AdjLayout A = adj_layout(c, c->adjK, c->adjk);
  AdjPtrs a = adj_ptrs(c, A);
  const bool kt = c->ktiming;
  c->ktiming = false;
  lbib_status st = set_freeze(c, 1);
  if (st != LBIB_OK) return st;
  const long long N = c->nodes;
  const int nm = c->nm;
  launch_fill(a.ha, 9 * N, 0.0, c->stream);
  launch_fill(a.xa, nm, 0.0, c->stream);
  launch_fill(a.xma, nm, 0.0, c->stream);
  launch_fill(a.yma, nm, 0.0, c->stream);
  launch_fill(a.grad, 3 * (long long)std::max(c->nbody, 1), 0.0, c->stream);
  launch_fill(a.rig, 9 * (long long)std::max(c->nbody, 1), 0.0, c->stream);
  std::vector<double> seed;
  wall_objective(c, c->adj_y, &seed);
  for (auto& v : seed) v *= dJ;
  if (nm > 0)
    HIPCHK(c, hipMemcpyAsync(a.ya, seed.data(), 8 * (size_t)nm, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // accumulators and the range flag start at zero (0.0 has all bits clear)
  launch_fill((double*)a.FE.hi, 4 * N, 0.0, c->stream);
  launch_fill((double*)a.Uh.hi, 4 * N, 0.0, c->stream);
  launch_fill((double*)a.Rh.hi, 6 * N, 0.0, c->stream);
  launch_fill((double*)a.bad, 1, 0.0, c->stream);
  // segments from last to first on the adjoint's own two streams: the
  // recompute of segment j - 1 (first stream, in the role of the context's
  // stream for the loop) overlaps the reverse sweep of segment j (second
  // stream); stores alternate, and a store is refilled only after its
  // previous reverse sweep
  hipStream_t caller = c->stream;
  struct RestoreStream {   // every return below leaves the caller's stream in place
    lbib_ctx* c;
    hipStream_t s;
    ~RestoreStream() { c->stream = s; }
  } restore{c, caller};
  HIPCHK(c, hipEventRecord(c->ev_adj_start, caller));
  HIPCHK(c, hipStreamWaitEvent(c->adj_s[0], c->ev_adj_start, 0));
  c->stream = c->adj_s[0];
  hipStream_t rev = c->adj_s[1];
  for (int j = A.nseg - 1; j >= 0; --j) {
    const int buf = j & 1;
    if (j + 2 <= A.nseg - 1) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_rev[buf], 0));
    adj_checkpoint(c, A, j, false);
    c->step = c->ck_step[j];
    // marker bins of the restored positions (eager, outside the graphs)
    HIPCHK(c, hipMemsetAsync(c->ws + c->L.cnt[c->parity], 0, 4 * (size_t)c->ntiles, c->stream));
    launch_stencil<T>(make_ptrs<T>(c), step_args(c), c->stream);
    c->stencil_dirty = false;
    const long long n = std::min<long long>(c->adjk, c->adjK - (long long)j * c->adjk);
    const int par = c->parity, first = c->ck_step[j] == 0 ? 1 : 0;
    hipGraphExec_t gr, gv;
    st = cached_graph(c, c->adj_graphs, std::make_tuple(n, par, buf), c->stream,
                      [&] { enqueue_recompute<T>(c, A, buf, n); }, &gr);
    if (st != LBIB_OK) return st;
    c->parity = par;   // capture ran nothing
    st = cached_graph(c, c->adj_rgraphs, std::make_tuple(n, buf, first), rev,
                      [&] { enqueue_reverse<T>(c, A, a, buf, n, first != 0, rev); }, &gv);
    if (st != LBIB_OK) return st;
    HIPCHK(c, hipGraphLaunch(gr, c->stream));
    c->parity = par ^ (int)(n & 1);
    c->step += n;
    HIPCHK(c, hipEventRecord(c->ev_rec[buf], c->stream));
    HIPCHK(c, hipStreamWaitEvent(rev, c->ev_rec[buf], 0));
    HIPCHK(c, hipGraphLaunch(gv, rev));
    HIPCHK(c, hipEventRecord(c->ev_rev[buf], rev));
  }
  // the caller's stream resumes after both of the adjoint's streams
  c->stream = caller;
  HIPCHK(c, hipEventRecord(c->ev_adj_start, c->adj_s[0]));
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_adj_start, 0));
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_rev[0], 0));
  if (A.nseg > 1) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_rev[1], 0));
  HIPCHK(c, hipGetLastError());
  // leave the context at the end of the window
  adj_checkpoint(c, A, A.nseg, false);
  c->step = c->ck_step[A.nseg];
  c->stencil_dirty = true;
  std::vector<double> g(3 * (size_t)std::max(c->nbody, 1));
  int bad = 0;
  HIPCHK(c, hipMemcpyAsync(g.data(), a.grad, 8 * g.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&bad, a.bad, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (bad) {
    (void)set_freeze(c, c->inst[0].adh.freeze_topology);
    c->ktiming = kt;
    return fail(c, LBIB_EUNSTABLE, "adjoint: a scattered term was not finite or of magnitude 2^30 or more");
  }
  if (grad) std::memcpy(grad, g.data(), 8 * 3 * (size_t)c->nbody);
  st = set_freeze(c, c->inst[0].adh.freeze_topology);
  if (st != LBIB_OK) return st;
  c->ktiming = kt;
  return LBIB_OK;
}

}  // namespace

// =============================================================== C ABI
// ------------------------------------------------ allocation-free field readback
// Staging of lbib_get_fields_noalloc: a file-scope device array, of which
// every GPU the library runs on holds its own copy until the process ends.
// In host code its name is not a device address: the address of each
// device's copy comes from hipGetSymbolAddress, resolved once per device with
// that device current (at lbib_bind), and only that address is handed to
// kernels and copies.  Every call on a GPU shares that GPU's copy, so calls
// that overlap on one GPU race; each call writes all the entries it reads.
constexpr long long kFieldStageNodes = 1ll << 19;   // rho, ux, uy: 3 x 4 MiB
static __device__ __align__(256) double scratch[3 * kFieldStageNodes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's staging array (resolved once per device).
lbib_status resolve_scratch(lbib_ctx* c) {
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, LBIB_EINVAL, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (double*)ptr;
  }
  c->device = dev;
  return LBIB_OK;
}

template <typename T>
lbib_status fields_noalloc_impl(lbib_ctx* c, double* rho, double* ux, double* uy) {
  const InstHost& I = c->inst[0];
  const long long N = (long long)I.lat.nx * I.lat.ny;
  double* stage = g_scratch_ptr[c->device];
  launch_fields<T>(make_ptrs<T>(c), step_args(c), 0, stage, stage + kFieldStageNodes,
                   stage + 2 * kFieldStageNodes, I.lat.nx, I.lat.ny, c->node_base[0], c->stream);
  HIPCHK(c, hipGetLastError());
  double* dst[3] = {rho, ux, uy};
  for (int k = 0; k < 3; ++k)
    if (dst[k])
      HIPCHK(c, hipMemcpyAsync(dst[k], stage + k * kFieldStageNodes, (size_t)N * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBIB_OK;
}
}  // namespace

extern "C" {

uint32_t lbib_abi_version(void) { return LBIB_ABI_VERSION; }

const char* lbib_status_string(int32_t s) {
  switch (s) {
    case LBIB_OK: return "LBIB_OK";
    case LBIB_EINVAL: return "LBIB_EINVAL";
    case LBIB_ESTATE: return "LBIB_ESTATE";
    case LBIB_EHIP: return "LBIB_EHIP";
    case LBIB_ENOSPACE: return "LBIB_ENOSPACE";
    case LBIB_EUNSTABLE: return "LBIB_EUNSTABLE";
    default: return "LBIB_UNKNOWN";
  }
}

const char* lbib_last_error(const lbib_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

lbib_status lbib_create(const lbib_lattice_desc* d, lbib_ctx** out) {
  if (!d || !out) return fail(nullptr, LBIB_EINVAL, "NULL argument");
  if (d->nx < 1 || d->ny < 1) return fail(nullptr, LBIB_EINVAL, "nx and ny must be >= 1");
  if ((long long)row_pitch(d->nx) * d->ny > (1ll << 31)) return fail(nullptr, LBIB_EINVAL, "lattice too large");
  if (!(d->tau > 0.5) || !std::isfinite(d->tau)) return fail(nullptr, LBIB_EINVAL, "tau must be > 1/2");
  if (d->dtype != LBIB_F32 && d->dtype != LBIB_F64) return fail(nullptr, LBIB_EINVAL, "bad dtype");
  if (!std::isfinite(d->gx) || !std::isfinite(d->gy))
    return fail(nullptr, LBIB_EINVAL, "the body force must be finite");
  int tx = d->tile_x, ty = d->tile_y;
  if (tx == 0 && ty == 0) { tx = 64; ty = 4; }
  if (!valid_tile(tx, ty)) return fail(nullptr, LBIB_EINVAL, "unsupported tile shape");
  lbib_ctx* c = new lbib_ctx();
  c->dtype = d->dtype;
  c->TX = tx;
  c->TY = ty;
  c->bin_cap = bin_capacity(tx, ty);
  InstHost I;
  I.lat = *d;
  I.adh.y_cr = 0.0;  // no bonds unless set
  I.adh.y_eq = 0.0;
  I.adh.kbt = 1.0;
  c->inst.push_back(I);
  *out = c;
  return LBIB_OK;
}

lbib_status lbib_add_body(lbib_ctx* c, const lbib_body_desc* d, const double* xy, int32_t* id) {
  if (!c || !d || !xy) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "bodies can only be added during set-up");
  if (d->nv < 3) return fail(c, LBIB_EINVAL, "a body needs nv >= 3");
  if (d->kind < 0 || d->kind > 2) return fail(c, LBIB_EINVAL, "bad body kind");
  if (d->ligand_stride < 0) return fail(c, LBIB_EINVAL, "ligand_stride must be >= 0");
  if (d->kind == LBIB_RBC_KINEMATIC && d->ligand_stride > 0)
    return fail(c, LBIB_EINVAL, "ligands sit on particles only (red cells carry none)");
  if (d->kind != LBIB_RBC_KINEMATIC && !(d->density_ratio > 0 && std::isfinite(d->density_ratio)))
    return fail(c, LBIB_EINVAL, "particles need a finite density_ratio > 0");
  for (double v : {d->ks, d->kb, d->ka, d->p_ref, d->sigma})
    if (!(v >= 0) || !std::isfinite(v))
      return fail(c, LBIB_EINVAL, "ks, kb, ka, p_ref and sigma must be finite and >= 0");
  BodyHost b;
  b.d = *d;
  b.xy.assign(xy, xy + 2 * (size_t)d->nv);
  for (double v : b.xy)
    if (!std::isfinite(v)) return fail(c, LBIB_EINVAL, "non-finite vertex");
  std::vector<double> l0, th0;
  double A;
  rest_state(b.xy, d->nv, l0, th0, A);
  if (!(A > 0)) return fail(c, LBIB_EINVAL, "vertices must run counter-clockwise (positive area)");
  for (double l : l0)
    if (!(l > 0)) return fail(c, LBIB_EINVAL, "coincident consecutive vertices");
  auto& I = c->inst.back();
  if (id) *id = (int32_t)I.bodies.size();
  I.bodies.push_back(b);
  return LBIB_OK;
}

lbib_status lbib_set_receptors(lbib_ctx* c, int32_t wall, const double* x, int32_t n) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "receptors can only be set during set-up");
  if (wall != 0 && wall != 1) return fail(c, LBIB_EINVAL, "wall must be 0 or 1");
  if (n < 0 || (n > 0 && !x)) return fail(c, LBIB_EINVAL, "bad receptor array");
  auto& I = c->inst.back();
  for (int k = 0; k < n; ++k) {
    if (!(x[k] >= 0.0 && x[k] < I.lat.nx)) return fail(c, LBIB_EINVAL, "receptor x outside [0, nx)");
    if (k > 0 && !(x[k] > x[k - 1])) return fail(c, LBIB_EINVAL, "receptor x must increase strictly");
  }
  I.rec[wall].assign(x, x + n);
  return LBIB_OK;
}

lbib_status lbib_set_adhesion(lbib_ctx* c, const lbib_adhesion_desc* d) {
  if (!c || !d) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "adhesion can only be set during set-up");
  if (!(d->kbt > 0) || !(d->y_cr >= 0) || !(d->kf0_dt >= 0) || !(d->kr0_dt >= 0))
    return fail(c, LBIB_EINVAL, "bad adhesion parameters");
  for (double v : {d->y_cr, d->y_eq, d->kf0_dt, d->kr0_dt, d->sigma_ts_frac, d->kbt})
    if (!std::isfinite(v)) return fail(c, LBIB_EINVAL, "adhesion parameters must be finite");
  c->inst.back().adh = *d;
  return LBIB_OK;
}

lbib_status lbib_set_walls(lbib_ctx* c, int32_t mode, double u_lo, double u_hi) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "walls can only be set during set-up");
  auto& I = c->inst.back();
  if (mode != 0 && mode != 1) return fail(c, LBIB_EINVAL, "wall mode must be 0 or 1");
  if (!std::isfinite(u_lo) || !std::isfinite(u_hi) || std::fabs(u_lo) > 0.3 || std::fabs(u_hi) > 0.3)
    return fail(c, LBIB_EINVAL, "wall velocities must be finite and |u| <= 0.3");
  if (mode == 0 && (u_lo != 0.0 || u_hi != 0.0))
    return fail(c, LBIB_EINVAL, "moving walls need the velocity-wall mode");
  if (mode == 1 && (I.lat.periodic_y || I.lat.ny < 2))
    return fail(c, LBIB_EINVAL, "velocity walls need a walled lattice with ny >= 2");
  I.wall_mode = mode;
  I.u_wall_lo = u_lo;
  I.u_wall_hi = u_hi;
  return LBIB_OK;
}

lbib_status lbib_set_transfer(lbib_ctx* c, int32_t mode, int32_t weight, double half_width) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "the transfer can only be set during set-up");
  if (mode != LBIB_TRANSFER_ROMA && mode != LBIB_TRANSFER_MLS)
    return fail(c, LBIB_EINVAL, "transfer mode must be LBIB_TRANSFER_ROMA or LBIB_TRANSFER_MLS");
  if (weight != LBIB_MLS_WEIGHT_ROMA && weight != LBIB_MLS_WEIGHT_CUBIC && weight != LBIB_MLS_WEIGHT_GAUSS)
    return fail(c, LBIB_EINVAL, "unknown MLS weight");
  // a support above 1 keeps two nodes per axis inside it; up to 3/2 it lies
  // within the 3x3 nearest nodes
  if (weight != LBIB_MLS_WEIGHT_ROMA && !(half_width > 1.0 && half_width <= 1.5))
    return fail(c, LBIB_EINVAL, "MLS support half-width must be in (1, 1.5]");
  auto& I = c->inst.back();
  I.transfer = mode;
  I.mls_weight = weight;
  I.mls_h = weight == LBIB_MLS_WEIGHT_ROMA ? 1.5 : half_width;
  return LBIB_OK;
}

lbib_status lbib_set_repulsion(lbib_ctx* c, double coeff, double cutoff) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "repulsion can only be set during set-up");
  if (!std::isfinite(coeff) || coeff < 0.0) return fail(c, LBIB_EINVAL, "repulsion coefficient must be finite and >= 0");
  if (!std::isfinite(cutoff) || !(cutoff > 0.0) || cutoff > 16.0)
    return fail(c, LBIB_EINVAL, "repulsion cutoff must be in (0, 16]");
  c->inst.back().rep_coeff = coeff;
  c->inst.back().rep_cutoff = cutoff;
  return LBIB_OK;
}

lbib_status lbib_init_fields(lbib_ctx* c, const double* rho, const double* ux, const double* uy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 0 || c->is_batch) return fail(c, LBIB_ESTATE, "fields can only be initialised during set-up");
  auto& I = c->inst.back();
  const size_t N = (size_t)I.lat.nx * I.lat.ny;
  for (const double* a : {rho, ux, uy})
    if (a)
      for (size_t k = 0; k < N; ++k)
        if (!std::isfinite(a[k])) return fail(c, LBIB_EINVAL, "non-finite initial field");
  if (rho)
    for (size_t k = 0; k < N; ++k)
      if (!(rho[k] > 0)) return fail(c, LBIB_EINVAL, "initial density must be positive");
  I.rho0 = rho ? std::vector<double>(rho, rho + N) : std::vector<double>();
  I.ux0 = ux ? std::vector<double>(ux, ux + N) : std::vector<double>();
  I.uy0 = uy ? std::vector<double>(uy, uy + N) : std::vector<double>();
  return LBIB_OK;
}

lbib_status lbib_workspace_query(const lbib_ctx* cc, size_t* bytes) {
  lbib_ctx* c = const_cast<lbib_ctx*>(cc);
  if (!c || !bytes) return fail(c, LBIB_EINVAL, "NULL argument");
  compute_sizes(c);
  compute_layout(c);
  *bytes = c->L.total;
  return LBIB_OK;
}

lbib_status lbib_get_fields_noalloc(lbib_ctx* c, double* rho, double* ux, double* uy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  const long long N = (long long)c->inst[0].lat.nx * c->inst[0].lat.ny;
  if (N > kFieldStageNodes)
    return fail(c, LBIB_EINVAL, "lattice of " + std::to_string(N) + " nodes exceeds the " +
                                    std::to_string(kFieldStageNodes) +
                                    "-node staging of lbib_get_fields_noalloc (use lbib_get_fields)");
  if (c->device < 0 || c->device >= kMaxDevices || !g_scratch_ptr[c->device])
    return fail(c, LBIB_ESTATE, "staging array not resolved for this context's device");
  return c->dtype == LBIB_F64 ? fields_noalloc_impl<double>(c, rho, ux, uy)
                              : fields_noalloc_impl<float>(c, rho, ux, uy);
}

lbib_status lbib_bind(lbib_ctx* c, void* ws, size_t bytes, void* stream) {
  if (!c || !ws) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 0) return fail(c, LBIB_ESTATE, "already bound");
  if (((uintptr_t)ws) & 255) return fail(c, LBIB_EINVAL, "workspace must be 256-byte aligned");
  compute_sizes(c);
  compute_layout(c);
  if (bytes < c->L.total) return fail(c, LBIB_ENOSPACE, "workspace smaller than lbib_workspace_query");
  lbib_status rs = resolve_scratch(c);
  if (rs != LBIB_OK) return rs;
  int ncu = 0;
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  if (ncu > 0) c->n_cu = ncu;
  c->ws = (char*)ws;
  c->ws_bytes = bytes;
  c->stream = (hipStream_t)stream;
  if (!c->aux) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  c->phase = 1;
  return LBIB_OK;
}

lbib_status lbib_finalize_setup(lbib_ctx* c) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 1) return fail(c, LBIB_ESTATE, "bind a workspace before finalize_setup");
  c->body_cache = body_cache_bytes(c);
  resolve_step_mode(c);
  c->inplace = resolve_inplace(c);
  lbib_status s = c->dtype == LBIB_F64 ? upload_all<double>(c) : upload_all<float>(c);
  if (s != LBIB_OK) return s;
  s = record_mass(c);
  if (s != LBIB_OK) return s;
  c->phase = 2;
  return LBIB_OK;
}

lbib_status lbib_set_step_mode(lbib_ctx* c, int32_t mode) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (mode < 0 || mode > 3) return fail(c, LBIB_EINVAL, "step mode must be 0..3");
  c->step_mode = mode;
  if (c->phase == 2) {
    drop_graphs(c);
    drop_adjoint_graphs(c);
    resolve_step_mode(c);
  }
  return LBIB_OK;
}

lbib_status lbib_set_cache_hints(lbib_ctx* c, int32_t hints) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (hints != -1 && hints != 0 && hints != 1 && hints != 3)
    return fail(c, LBIB_EINVAL, "cache hints must be -1, 0, 1 or 3");
  if (hints != c->cache_hints) {
    drop_graphs(c);
    drop_adjoint_graphs(c);
  }
  c->cache_hints = hints;
  return LBIB_OK;
}

lbib_status lbib_set_lattice_launch(lbib_ctx* c, int32_t wgs_per_cu) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (wgs_per_cu != 0 && wgs_per_cu != 1 && wgs_per_cu != 2 && wgs_per_cu != 4 && wgs_per_cu != 8)
    return fail(c, LBIB_EINVAL, "lattice launch must be 0, 1, 2, 4 or 8 workgroups per CU");
  if (wgs_per_cu != c->lb_wpc) {
    drop_graphs(c);
    drop_adjoint_graphs(c);
  }
  c->lb_wpc = wgs_per_cu;
  return LBIB_OK;
}

lbib_status lbib_set_streaming(lbib_ctx* c, int32_t mode) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (mode < -1 || mode > 1) return fail(c, LBIB_EINVAL, "streaming must be -1, 0 or 1");
  c->streaming = mode;
  if (c->phase != 2) return LBIB_OK;
  const bool want = resolve_inplace(c);
  if (want == c->inplace) return LBIB_OK;
  // the populations through B in scheme-0 order (two buffers: the state's
  // buffer is A at even parity, B at odd), then into the new form
  const size_t bytes = elem_size(c->dtype) * 9 * (size_t)c->nodes;
  lbib_status st = LBIB_OK;
  if (c->inplace) st = canon_any(c, 1);
  else if (c->parity == 0) HIPCHK(c, hipMemcpyAsync(c->ws + c->L.B, c->ws + c->L.A, bytes,
                                                    hipMemcpyDeviceToDevice, c->stream));
  if (st != LBIB_OK) return st;
  c->inplace = want;
  if (c->inplace) st = canon_any(c, 0);
  else if (c->parity == 0) HIPCHK(c, hipMemcpyAsync(c->ws + c->L.A, c->ws + c->L.B, bytes,
                                                    hipMemcpyDeviceToDevice, c->stream));
  if (st != LBIB_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graphs(c);
  drop_adjoint_graphs(c);
  return LBIB_OK;
}

lbib_status lbib_get_streaming(const lbib_ctx* c, int32_t* inplace) {
  if (!c || !inplace) return fail(const_cast<lbib_ctx*>(c), LBIB_EINVAL, "NULL argument");
  *inplace = c->phase == 2 ? (c->inplace ? 1 : 0) : (int32_t)resolve_inplace(c);
  return LBIB_OK;
}

lbib_status lbib_get_lattice_launch(const lbib_ctx* c, int32_t* wgs_per_cu) {
  if (!c || !wgs_per_cu) return fail(const_cast<lbib_ctx*>(c), LBIB_EINVAL, "NULL argument");
  *wgs_per_cu = c->lb_wpc;
  return LBIB_OK;
}

lbib_status lbib_get_cache_hints(const lbib_ctx* cc, int32_t* hints) {
  lbib_ctx* c = const_cast<lbib_ctx*>(cc);
  if (!c || !hints) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase == 0) compute_sizes(c);
  *hints = step_args(c).nt_mode;
  return LBIB_OK;
}

lbib_status lbib_get_step_mode(const lbib_ctx* cc, int32_t* mode) {
  lbib_ctx* c = const_cast<lbib_ctx*>(cc);
  if (!c || !mode) return fail(c, LBIB_EINVAL, "NULL argument");
  *mode = c->phase == 2 ? (c->overlap ? 3 : (c->merge_advance ? 2 : 1)) : c->step_mode;
  return LBIB_OK;
}

lbib_status lbib_set_watchdog(lbib_ctx* c, int32_t on) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  c->watchdog = on != 0;
  return LBIB_OK;
}

lbib_status lbib_set_watchdog_mass_tolerance(lbib_ctx* c, double rel) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (!(rel >= 0.0) || !std::isfinite(rel)) return fail(c, LBIB_EINVAL, "tolerance must be finite and >= 0");
  c->mass_tol = rel;
  return LBIB_OK;
}

lbib_status lbib_set_graph_steps(lbib_ctx* c, int32_t steps) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (steps < 0 || (steps & 1)) return fail(c, LBIB_EINVAL, "graph steps must be even and >= 0");
  if (steps != c->graph_steps) drop_graphs(c);
  c->graph_steps = steps;
  return LBIB_OK;
}

lbib_status lbib_step(lbib_ctx* c, int64_t n) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "finalize_setup before stepping");
  if (n < 0) return fail(c, LBIB_EINVAL, "nsteps must be >= 0");
  lbib_status s = c->dtype == LBIB_F64 ? run_steps<double>(c, n) : run_steps<float>(c, n);
  if (s != LBIB_OK) return s;
  if (c->watchdog) {
    double d[6];
    s = c->dtype == LBIB_F64 ? diag_impl<double>(c, d) : diag_impl<float>(c, d);
    if (s != LBIB_OK) return s;
    if (d[5] > 0 || !(d[3] > 0))
      return fail(c, LBIB_EUNSTABLE, "watchdog: non-finite population or non-positive density");
    if (std::isfinite(c->mass_ref) && !(std::fabs(d[0] - c->mass_ref) <= c->mass_tol * c->mass_ref)) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "watchdog: total mass %.17g drifted from %.17g by more than %g relative",
                    d[0], c->mass_ref, c->mass_tol);
      return fail(c, LBIB_EUNSTABLE, msg);
    }
  }
  return LBIB_OK;
}

lbib_status lbib_get_fields(lbib_ctx* c, double* rho, double* ux, double* uy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  return c->dtype == LBIB_F64 ? fields_impl<double>(c, 0, rho, ux, uy)
                              : fields_impl<float>(c, 0, rho, ux, uy);
}

static lbib_status copy_marker_pair(lbib_ctx* c, int inst, int body, size_t ox, size_t oy, double* xy) {
  if (!c || !xy) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  lbib_status s = check_body(c, inst, body);
  if (s != LBIB_OK) return s;
  const int v0 = body_v0(c, inst, body), nv = c->inst[inst].bodies[body].d.nv;
  std::vector<double> a(nv), b(nv);
  HIPCHK(c, hipMemcpyAsync(a.data(), c->ws + ox + 8 * (size_t)v0, 8 * nv, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(b.data(), c->ws + oy + 8 * (size_t)v0, 8 * nv, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int v = 0; v < nv; ++v) {
    xy[2 * v] = a[v];
    xy[2 * v + 1] = b[v];
  }
  return LBIB_OK;
}

lbib_status lbib_get_markers(lbib_ctx* c, int32_t body, double* xy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  return copy_marker_pair(c, 0, body, c->L.x, c->L.y, xy);
}

lbib_status lbib_get_marker_forces(lbib_ctx* c, int32_t body, double* fxy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  return copy_marker_pair(c, 0, body, c->L.fx, c->L.fy, fxy);
}

lbib_status lbib_set_markers(lbib_ctx* c, int32_t body, const double* xy, const double* xyp) {
  if (!c || !xy) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  lbib_status s = check_body(c, 0, body);
  if (s != LBIB_OK) return s;
  const int v0 = body_v0(c, 0, body), nv = c->inst[0].bodies[body].d.nv;
  if (!xyp) xyp = xy;
  std::vector<double> a(nv), b(nv), am(nv), bm(nv);
  for (int v = 0; v < nv; ++v) {
    a[v] = xy[2 * v]; b[v] = xy[2 * v + 1];
    am[v] = xyp[2 * v]; bm[v] = xyp[2 * v + 1];
    if (!std::isfinite(a[v]) || !std::isfinite(b[v]) || !std::isfinite(am[v]) || !std::isfinite(bm[v]))
      return fail(c, LBIB_EINVAL, "non-finite marker position");
  }
  const size_t o = 8 * (size_t)v0;
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.x + o, a.data(), 8 * nv, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.y + o, b.data(), 8 * nv, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.xm + o, am.data(), 8 * nv, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.ym + o, bm.data(), 8 * nv, hipMemcpyHostToDevice, c->stream));
  // particles: X^n also in the slot their dynamics fill (read by the bond kinetics)
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.xn + o, a.data(), 8 * nv, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ws + c->L.yn + o, b.data(), 8 * nv, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->stencil_dirty = true;
  return LBIB_OK;
}

lbib_status lbib_num_ligands(const lbib_ctx* cc, int32_t* n) {
  lbib_ctx* c = const_cast<lbib_ctx*>(cc);
  if (!c || !n) return fail(c, LBIB_EINVAL, "NULL argument");
  int k = 0;
  for (auto& b : c->inst[0].bodies)
    if (b.d.ligand_stride > 0) k += (b.d.nv + b.d.ligand_stride - 1) / b.d.ligand_stride;
  *n = k;
  return LBIB_OK;
}

static lbib_status bonds_get(lbib_ctx* c, int inst, int32_t* l2r, int32_t* nb) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  if (inst < 0 || inst >= c->ninst) return fail(c, LBIB_EINVAL, "instance out of range");
  const int base = c->lig_base[inst];
  const int n = (inst + 1 < c->ninst ? c->lig_base[inst + 1] : c->nlig) - base;
  std::vector<int32_t> v(std::max(n, 1));
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(v.data(), c->ws + c->L.l2r + 4 * (size_t)base, 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  int cnt = 0;
  for (int k = 0; k < n; ++k) {
    if (v[k] >= 0) ++cnt;
    if (l2r) l2r[k] = v[k];
  }
  if (nb) *nb = cnt;
  return LBIB_OK;
}

lbib_status lbib_get_bonds(lbib_ctx* c, int32_t* l2r, int32_t* nb) { return bonds_get(c, 0, l2r, nb); }

lbib_status lbib_set_bonds(lbib_ctx* c, const int32_t* l2r) {
  if (!c || !l2r) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  const int n = c->ninst > 1 ? c->lig_base[1] : c->nlig;
  const int nr = (int)(c->inst[0].rec[0].size() + c->inst[0].rec[1].size());
  std::vector<int32_t> r2l(std::max(nr, 1), -1);
  for (int k = 0; k < n; ++k) {
    const int r = l2r[k];
    if (r < -1 || r >= nr) return fail(c, LBIB_EINVAL, "receptor index out of range");
    if (r >= 0) {
      if (r2l[r] >= 0) return fail(c, LBIB_EINVAL, "receptor bonded twice");
      r2l[r] = k;  // instance 0: global ligand id == local id
    }
  }
  if (n > 0)
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.l2r, l2r, 4 * n, hipMemcpyHostToDevice, c->stream));
  if (nr > 0)
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.r2l, r2l.data(), 4 * nr, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBIB_OK;
}

lbib_status lbib_get_state(lbib_ctx* c, void* blob, size_t* bytes) {
  if (!c || !bytes) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  auto regs = state_regions(c);
  size_t total = sizeof(StateHeader);
  for (auto& r : regs) total += r.second;
  if (!blob) {
    *bytes = total;
    return LBIB_OK;
  }
  if (*bytes < total) return fail(c, LBIB_EINVAL, "state buffer too small");
  StateHeader h{kMagic, total, (uint64_t)c->step, c->dtype, c->ninst, c->nm, c->nbody, c->nlig,
                c->nrec, c->ntiles, 0, c->nodes};
  lbib_status st = stage_state(c);
  if (st != LBIB_OK) return st;
  char* o = (char*)blob;
  std::memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  for (auto& r : regs) {
    HIPCHK(c, hipMemcpyAsync(o, c->ws + r.first, r.second, hipMemcpyDeviceToHost, c->stream));
    o += r.second;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *bytes = total;
  return LBIB_OK;
}

lbib_status lbib_set_state(lbib_ctx* c, const void* blob, size_t bytes) {
  if (!c || !blob) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  StateHeader h;
  if (bytes < sizeof(h)) return fail(c, LBIB_EINVAL, "state blob too small");
  std::memcpy(&h, blob, sizeof(h));
  if (h.magic != kMagic || h.bytes != bytes || h.dtype != c->dtype || h.ninst != c->ninst ||
      h.nm != c->nm || h.nbody != c->nbody || h.nlig != c->nlig || h.nrec != c->nrec ||
      h.ntiles != c->ntiles || h.nodes != c->nodes)
    return fail(c, LBIB_EINVAL, "state blob does not match this context");
  auto regs = state_regions(c);
  const char* o = (const char*)blob + sizeof(h);
  for (auto& r : regs) {
    HIPCHK(c, hipMemcpyAsync(c->ws + r.first, o, r.second, hipMemcpyHostToDevice, c->stream));
    o += r.second;
  }
  lbib_status st = unstage_state(c);
  if (st != LBIB_OK) return st;
  // the host copies of the body constants follow the restored records
  std::vector<BodyDev> bd(std::max(c->nbody, 1));
  HIPCHK(c, hipMemcpyAsync(bd.data(), c->ws + c->L.body, sizeof(BodyDev) * bd.size(),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0, b = 0; i < c->ninst; ++i)
    for (auto& B : c->inst[i].bodies) {
      B.d.ks = bd[b].ks;
      B.d.kb = bd[b].kb;
      B.d.sigma = bd[b].sigma;
      ++b;
    }
  c->step = (long long)h.step;
  c->stencil_dirty = true;   // marker bins are rebuilt from the restored positions
  c->adj_ready = false;
  return record_mass(c);
}

lbib_status lbib_diagnostics(lbib_ctx* c, lbib_diag* out) {
  if (!c || !out) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  double d[6];
  lbib_status s = c->dtype == LBIB_F64 ? diag_impl<double>(c, d) : diag_impl<float>(c, d);
  if (s != LBIB_OK) return s;
  out->step = c->step;
  out->mass = d[0];
  out->mom_x = d[1];
  out->mom_y = d[2];
  out->rho_min = d[3];
  out->u_max = d[4];
  out->nonfinite = (int64_t)d[5];
  int32_t nb = 0;
  int tot = 0;
  for (int i = 0; i < c->ninst; ++i) {
    s = bonds_get(c, i, nullptr, &nb);
    if (s != LBIB_OK) return s;
    tot += nb;
  }
  out->nbonds = tot;
  int32_t ovf = 0, spin = 0;
  HIPCHK(c, hipMemcpyAsync(&ovf, c->ws + c->L.overflow, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&spin, c->ws + c->L.spin, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->bin_overflow = ovf;
  out->sync_timeouts = spin;
  return LBIB_OK;
}

lbib_status lbib_observe(lbib_ctx* c) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  lbib_body_obs* o = (lbib_body_obs*)(c->ws + c->L.obs);
  if (c->dtype == LBIB_F64) launch_observe<double>(make_ptrs<double>(c), o, c->step, c->stream);
  else launch_observe<float>(make_ptrs<float>(c), o, c->step, c->stream);
  HIPCHK(c, hipGetLastError());
  return LBIB_OK;
}

lbib_status lbib_get_observations(lbib_ctx* c, lbib_body_obs* out) {
  if (!c || !out) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  if (c->nbody == 0) return LBIB_OK;
  HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.obs, sizeof(lbib_body_obs) * (size_t)c->nbody,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBIB_OK;
}

lbib_status lbib_reset_observations(lbib_ctx* c) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  HIPCHK(c, hipMemsetAsync(c->ws + c->L.obs, 0, sizeof(lbib_body_obs) * (size_t)std::max(c->nbody, 1),
                           c->stream));
  return LBIB_OK;
}

lbib_status lbib_time_lattice_kernel(lbib_ctx* c, int32_t reps, double* avg_ms) {
  if (!c || !avg_ms) return fail(c, LBIB_EINVAL, "NULL argument");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  if (c->step < 1 || c->stencil_dirty) return fail(c, LBIB_ESTATE, "needs one completed step");
  if (reps < 1) return fail(c, LBIB_EINVAL, "reps must be >= 1");
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  const StepArgs a = step_args(c);
  // in place the launches rewrite the state's own buffer: it is kept in B
  // meanwhile and put back afterwards
  lbib_status st = stage_state(c);
  if (st != LBIB_OK) return st;
  HIPCHK(c, hipEventRecord(e0, c->stream));
  // measurement launches: bins of the coming step are read but not consumed,
  // the velocity output goes to a spare buffer, populations to the spare set
  for (int r = 0; r < reps; ++r) {
    if (c->dtype == LBIB_F64) {
      Ptrs<double> p = make_ptrs<double>(c);
      p.U = (double*)(c->ws + c->L.Uspare);
      launch_lb_fused<double>(p, a, c->stream, 0);
    } else {
      Ptrs<float> p = make_ptrs<float>(c);
      p.U = (float*)(c->ws + c->L.Uspare);
      launch_lb_fused<float>(p, a, c->stream, 0);
    }
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  st = unstage_state(c);
  if (st != LBIB_OK) return st;
  HIPCHK(c, hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  return LBIB_OK;
}

lbib_status lbib_set_kernel_timing(lbib_ctx* c, int32_t on) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  c->ktiming = on != 0;
  drop_kevents(c);
  return LBIB_OK;
}

lbib_status lbib_get_kernel_timing(lbib_ctx* c, double* avg_ms, int64_t* launches) {
  if (!c || !avg_ms) return fail(c, LBIB_EINVAL, "NULL argument");
  double sum = 0.0;
  for (auto& e : c->kevents) {
    HIPCHK(c, hipEventSynchronize(e.second));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e.first, e.second));
    sum += ms;
  }
  *avg_ms = c->kevents.empty() ? 0.0 : sum / (double)c->kevents.size();
  if (launches) *launches = (int64_t)c->kevents.size();
  return LBIB_OK;
}

lbib_status lbib_get_step(const lbib_ctx* cc, int64_t* step) {
  lbib_ctx* c = const_cast<lbib_ctx*>(cc);
  if (!c || !step) return fail(c, LBIB_EINVAL, "NULL argument");
  *step = c->step;
  return LBIB_OK;
}

lbib_status lbib_destroy(lbib_ctx* c) {
  if (!c) return LBIB_OK;
  drop_graphs(c);
  drop_adjoint_graphs(c);
  for (int k = 0; k < 2; ++k) {
    if (c->ev_rec[k]) (void)hipEventDestroy(c->ev_rec[k]);
    if (c->ev_rev[k]) (void)hipEventDestroy(c->ev_rev[k]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  for (auto& st : c->adj_s)
    if (st) (void)hipStreamDestroy(st);
  if (c->ev_adj_start) (void)hipEventDestroy(c->ev_adj_start);
  drop_kevents(c);
  delete c;
  return LBIB_OK;
}


// ------------------------------------------------------------ adjoint window
lbib_status lbib_adjoint_workspace_query(const lbib_ctx* cc, int64_t nsteps, int32_t ckpt_every,
                                         size_t* bytes) {
  lbib_ctx* c = const_cast<lbib_ctx*>(cc);
  if (!c || !bytes) return fail(c, LBIB_EINVAL, "NULL argument");
  if (nsteps < 1 || ckpt_every < 1) return fail(c, LBIB_EINVAL, "nsteps and ckpt_every must be >= 1");
  lbib_status s = adj_check_sizes(c);
  if (s != LBIB_OK) return s;
  *bytes = adj_layout(c, nsteps, ckpt_every).total;
  return LBIB_OK;
}

lbib_status lbib_adjoint_bind(lbib_ctx* c, void* ws, size_t bytes, int64_t nsteps, int32_t ckpt_every) {
  if (!c || !ws) return fail(c, LBIB_EINVAL, "NULL argument");
  if (nsteps < 1 || ckpt_every < 1) return fail(c, LBIB_EINVAL, "nsteps and ckpt_every must be >= 1");
  if (((uintptr_t)ws) & 255) return fail(c, LBIB_EINVAL, "workspace must be 256-byte aligned");
  lbib_status s = adj_check_sizes(c);
  if (s != LBIB_OK) return s;
  if (bytes < adj_layout(c, nsteps, ckpt_every).total)
    return fail(c, LBIB_ENOSPACE, "adjoint workspace smaller than lbib_adjoint_workspace_query");
  drop_adjoint_graphs(c);   // they hold pointers into the previous workspace
  for (int k = 0; k < 2; ++k) {
    if (!c->ev_rec[k]) HIPCHK(c, hipEventCreateWithFlags(&c->ev_rec[k], hipEventDisableTiming));
    if (!c->ev_rev[k]) HIPCHK(c, hipEventCreateWithFlags(&c->ev_rev[k], hipEventDisableTiming));
  }
  if (!c->ev_adj_start) HIPCHK(c, hipEventCreateWithFlags(&c->ev_adj_start, hipEventDisableTiming));
  // the recompute and the reverse sweep overlap only on distinct hardware
  // queues; streams made one after the other get distinct queues, whereas
  // the caller's stream and the context's second stream may share one
  for (int k = 0; k < 2; ++k)
    if (!c->adj_s[k]) HIPCHK(c, hipStreamCreateWithFlags(&c->adj_s[k], hipStreamNonBlocking));
  c->aws = (char*)ws;
  c->aws_bytes = bytes;
  c->adjK = nsteps;
  c->adjk = ckpt_every;
  c->adj_ready = false;
  return LBIB_OK;
}

lbib_status lbib_adjoint_forward(lbib_ctx* c, double* J, int32_t* nbonds) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  lbib_status s = adj_check(c);
  if (s != LBIB_OK) return s;
  s = c->dtype == LBIB_F64 ? adjoint_forward_impl<double>(c, J) : adjoint_forward_impl<float>(c, J);
  if (s != LBIB_OK) return s;
  return bonds_get(c, 0, nullptr, nbonds);
}

lbib_status lbib_adjoint_backward(lbib_ctx* c, double dJ, double* grad) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  lbib_status s = adj_check(c);
  if (s != LBIB_OK) return s;
  if (!c->adj_ready) return fail(c, LBIB_ESTATE, "run lbib_adjoint_forward first");
  return c->dtype == LBIB_F64 ? adjoint_backward_impl<double>(c, dJ, grad)
                              : adjoint_backward_impl<float>(c, dJ, grad);
}

lbib_status lbib_set_body_params(lbib_ctx* c, int32_t body, double ks, double kb, double sigma) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  lbib_status s = check_body(c, 0, body);
  if (s != LBIB_OK) return s;
  if (!std::isfinite(ks) || !std::isfinite(kb) || !std::isfinite(sigma) || ks < 0 || kb < 0 || sigma < 0)
    return fail(c, LBIB_EINVAL, "body constants must be finite and >= 0");
  BodyHost& B = c->inst[0].bodies[body];
  B.d.ks = ks;
  B.d.kb = kb;
  B.d.sigma = sigma;
  const int gb = c->body_base[0] + body;
  char* bd = c->ws + c->L.body + sizeof(BodyDev) * (size_t)gb;
  const double v3[3] = {ks, kb, sigma};
  HIPCHK(c, hipMemcpyAsync(bd + offsetof(BodyDev, ks), &v3[0], 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(bd + offsetof(BodyDev, kb), &v3[1], 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(bd + offsetof(BodyDev, sigma), &v3[2], 8, hipMemcpyHostToDevice, c->stream));
  if (B.d.ligand_stride > 0) {
    int lb = c->lig_base[0];
    for (int k = 0; k < body; ++k) {
      const auto& o = c->inst[0].bodies[k].d;
      if (o.ligand_stride > 0) lb += (o.nv + o.ligand_stride - 1) / o.ligand_stride;
    }
    const int nl = (B.d.nv + B.d.ligand_stride - 1) / B.d.ligand_stride;
    std::vector<double> sg(nl, sigma);
    HIPCHK(c, hipMemcpyAsync(c->ws + c->L.lig_sigma + 8 * (size_t)lb, sg.data(), 8 * (size_t)nl,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->adj_ready = false;
  return LBIB_OK;
}

// ------------------------------------------------------------ batch (sweeps)
lbib_status lbib_batch_create(const lbib_ctx* const* insts, int32_t n, int32_t tile_x, int32_t tile_y,
                              lbib_ctx** out) {
  if (!insts || !out || n < 1) return fail(nullptr, LBIB_EINVAL, "bad batch arguments");
  int tx = tile_x, ty = tile_y;
  if (tx == 0 && ty == 0) { tx = 64; ty = 4; }
  if (!valid_tile(tx, ty)) return fail(nullptr, LBIB_EINVAL, "unsupported tile shape");
  const int dtype = insts[0] ? insts[0]->dtype : -1;
  for (int i = 0; i < n; ++i) {
    if (!insts[i]) return fail(nullptr, LBIB_EINVAL, "NULL instance");
    if (insts[i]->phase != 0 || insts[i]->is_batch || insts[i]->inst.size() != 1)
      return fail(nullptr, LBIB_ESTATE, "instances must be single-lattice contexts in set-up");
    if (insts[i]->dtype != dtype) return fail(nullptr, LBIB_EINVAL, "instances must share the dtype");
  }
  lbib_ctx* c = new lbib_ctx();
  c->dtype = dtype;
  c->TX = tx;
  c->TY = ty;
  c->bin_cap = bin_capacity(tx, ty);
  c->is_batch = true;
  for (int i = 0; i < n; ++i) c->inst.push_back(insts[i]->inst[0]);
  *out = c;
  return LBIB_OK;
}

lbib_status lbib_batch_size(const lbib_ctx* c, int32_t* n) {
  if (!c || !n) return LBIB_EINVAL;
  *n = (int32_t)c->inst.size();
  return LBIB_OK;
}

lbib_status lbib_batch_get_fields(lbib_ctx* c, int32_t inst, double* rho, double* ux, double* uy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  if (c->phase != 2) return fail(c, LBIB_ESTATE, "not running");
  if (inst < 0 || inst >= c->ninst) return fail(c, LBIB_EINVAL, "instance out of range");
  return c->dtype == LBIB_F64 ? fields_impl<double>(c, inst, rho, ux, uy)
                              : fields_impl<float>(c, inst, rho, ux, uy);
}

lbib_status lbib_batch_get_markers(lbib_ctx* c, int32_t inst, int32_t body, double* xy) {
  if (!c) return fail(c, LBIB_EINVAL, "NULL context");
  return copy_marker_pair(c, inst, body, c->L.x, c->L.y, xy);
}

lbib_status lbib_batch_get_bonds(lbib_ctx* c, int32_t inst, int32_t* l2r, int32_t* nb) {
  return bonds_get(c, inst, l2r, nb);
}

}  // extern "C"
