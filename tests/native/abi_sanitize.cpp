// Host-side exercise of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer over the library's host code (no GPU needed):
// argument validation of every set-up call, the phase rules, workspace
// sizing, batch creation, and a seeded stream of malformed inputs.  Each
// call must return the documented status; the sanitizers report any
// invalid memory access or undefined operation on the way (the process then
// exits non-zero).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "lbib.h"
#include "lbib_batch.h"

static int g_fail = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)

static lbib_lattice_desc lattice(int nx, int ny, int dtype = LBIB_F32) {
  lbib_lattice_desc d;
  std::memset(&d, 0, sizeof(d));
  d.nx = nx;
  d.ny = ny;
  d.tau = 1.0;
  d.dtype = dtype;
  d.seed = 7;
  return d;
}

static std::vector<double> circle(double cx, double cy, double r, int n, bool ccw = true) {
  std::vector<double> xy(2 * n);
  for (int k = 0; k < n; ++k) {
    const double a = (ccw ? 1.0 : -1.0) * 2.0 * M_PI * k / n;
    xy[2 * k] = cx + r * std::cos(a);
    xy[2 * k + 1] = cy + r * std::sin(a);
  }
  return xy;
}

static lbib_body_desc body(int kind, int nv) {
  lbib_body_desc b;
  std::memset(&b, 0, sizeof(b));
  b.kind = kind;
  b.nv = nv;
  b.ks = kind == LBIB_PARTICLE_RIGID ? 0.0 : 0.01;
  b.kb = 0.0;
  b.ka = 1.0;
  b.p_ref = 1.0 / 3.0;
  b.density_ratio = 1.1;
  b.sigma = kind == LBIB_RBC_KINEMATIC ? 0.0 : 1e-3;
  b.ligand_stride = kind == LBIB_RBC_KINEMATIC ? 0 : 2;
  return b;
}

static void test_create() {
  lbib_ctx* h = nullptr;
  lbib_lattice_desc d = lattice(64, 32);
  CHECK(lbib_create(nullptr, &h) == LBIB_EINVAL);
  CHECK(lbib_create(&d, nullptr) == LBIB_EINVAL);
  CHECK(lbib_last_error(nullptr) != nullptr && std::strlen(lbib_last_error(nullptr)) > 0);
  const int bad_nx[] = {0, -1};
  for (int v : bad_nx) {
    lbib_lattice_desc b = d;
    b.nx = v;
    CHECK(lbib_create(&b, &h) == LBIB_EINVAL);
  }
  {
    lbib_lattice_desc b = d;
    b.ny = 0;
    CHECK(lbib_create(&b, &h) == LBIB_EINVAL);
  }
  const double bad_tau[] = {0.5, 0.1, -1.0, std::numeric_limits<double>::quiet_NaN(),
                            std::numeric_limits<double>::infinity()};
  for (double t : bad_tau) {
    lbib_lattice_desc b = d;
    b.tau = t;
    CHECK(lbib_create(&b, &h) == LBIB_EINVAL);
  }
  {
    lbib_lattice_desc b = d;
    b.dtype = 7;
    CHECK(lbib_create(&b, &h) == LBIB_EINVAL);
  }
  {
    lbib_lattice_desc b = d;
    b.gx = std::numeric_limits<double>::quiet_NaN();
    CHECK(lbib_create(&b, &h) == LBIB_EINVAL);
  }
  CHECK(lbib_create(&d, &h) == LBIB_OK && h != nullptr);
  CHECK(lbib_destroy(h) == LBIB_OK);
  CHECK(lbib_destroy(nullptr) == LBIB_OK);
  for (int s = 0; s <= 5; ++s) CHECK(lbib_status_string(s) != nullptr);
  CHECK(lbib_status_string(99) != nullptr);
}

static void test_bodies_and_setup_calls() {
  lbib_ctx* h = nullptr;
  lbib_lattice_desc d = lattice(96, 48);
  CHECK(lbib_create(&d, &h) == LBIB_OK);
  int32_t id = -1;
  std::vector<double> ok = circle(30, 24, 5, 40), cw = circle(60, 24, 5, 40, false);
  lbib_body_desc b = body(LBIB_RBC_KINEMATIC, 40);
  CHECK(lbib_add_body(nullptr, &b, ok.data(), &id) == LBIB_EINVAL);
  CHECK(lbib_add_body(h, nullptr, ok.data(), &id) == LBIB_EINVAL);
  CHECK(lbib_add_body(h, &b, nullptr, &id) == LBIB_EINVAL);
  CHECK(lbib_add_body(h, &b, cw.data(), &id) == LBIB_EINVAL);   // clockwise contour
  {
    lbib_body_desc x = b;
    x.nv = 2;
    CHECK(lbib_add_body(h, &x, ok.data(), &id) == LBIB_EINVAL);
    x = b;
    x.kind = 9;
    CHECK(lbib_add_body(h, &x, ok.data(), &id) == LBIB_EINVAL);
    x = b;
    x.ks = -1.0;
    CHECK(lbib_add_body(h, &x, ok.data(), &id) == LBIB_EINVAL);
    x = b;
    x.ligand_stride = -3;
    CHECK(lbib_add_body(h, &x, ok.data(), &id) == LBIB_EINVAL);
    std::vector<double> nan = ok;
    nan[7] = std::numeric_limits<double>::quiet_NaN();
    CHECK(lbib_add_body(h, &b, nan.data(), &id) == LBIB_EINVAL);
  }
  CHECK(lbib_add_body(h, &b, ok.data(), &id) == LBIB_OK && id == 0);
  lbib_body_desc r = body(LBIB_PARTICLE_RIGID, 24), s = body(LBIB_PARTICLE_SOFT, 130);
  std::vector<double> pr = circle(60, 24, 3, 24), ps = circle(80, 20, 8, 130);
  CHECK(lbib_add_body(h, &r, pr.data(), &id) == LBIB_OK && id == 1);
  CHECK(lbib_add_body(h, &s, ps.data(), &id) == LBIB_OK && id == 2);

  std::vector<double> rec(96);
  for (int k = 0; k < 96; ++k) rec[k] = k;
  std::vector<double> unsorted = rec;
  std::swap(unsorted[3], unsorted[4]);
  std::vector<double> outside = {0.0, 100.0};
  CHECK(lbib_set_receptors(h, 0, nullptr, 3) == LBIB_EINVAL);
  CHECK(lbib_set_receptors(h, 2, rec.data(), 96) == LBIB_EINVAL);
  CHECK(lbib_set_receptors(h, 0, unsorted.data(), 96) == LBIB_EINVAL);
  CHECK(lbib_set_receptors(h, 1, outside.data(), 2) == LBIB_EINVAL);
  CHECK(lbib_set_receptors(h, 0, rec.data(), -1) == LBIB_EINVAL);
  CHECK(lbib_set_receptors(h, 0, rec.data(), 96) == LBIB_OK);
  CHECK(lbib_set_receptors(h, 1, rec.data(), 96) == LBIB_OK);

  lbib_adhesion_desc a;
  std::memset(&a, 0, sizeof(a));
  a.y_cr = 0.5;
  a.y_eq = 0.25;
  a.kf0_dt = 1e-3;
  a.kr0_dt = 1e-7;
  a.sigma_ts_frac = 0.5;
  a.kbt = 1.0;
  CHECK(lbib_set_adhesion(h, nullptr) == LBIB_EINVAL);
  {
    lbib_adhesion_desc x = a;
    x.kbt = 0.0;
    CHECK(lbib_set_adhesion(h, &x) == LBIB_EINVAL);
    x = a;
    x.y_cr = -1.0;
    CHECK(lbib_set_adhesion(h, &x) == LBIB_EINVAL);
    x = a;
    x.kf0_dt = std::numeric_limits<double>::quiet_NaN();
    CHECK(lbib_set_adhesion(h, &x) == LBIB_EINVAL);
  }
  CHECK(lbib_set_adhesion(h, &a) == LBIB_OK);
  CHECK(lbib_set_walls(h, 5, 0.0, 0.0) == LBIB_EINVAL);
  CHECK(lbib_set_walls(h, 1, 0.0, std::numeric_limits<double>::quiet_NaN()) == LBIB_EINVAL);
  CHECK(lbib_set_transfer(h, 4, 0, 1.3) == LBIB_EINVAL);
  CHECK(lbib_set_transfer(h, LBIB_TRANSFER_MLS, 9, 1.3) == LBIB_EINVAL);
  CHECK(lbib_set_transfer(h, LBIB_TRANSFER_MLS, LBIB_MLS_WEIGHT_CUBIC, 0.2) == LBIB_EINVAL);
  CHECK(lbib_set_transfer(h, LBIB_TRANSFER_MLS, LBIB_MLS_WEIGHT_CUBIC, 1.3) == LBIB_OK);
  CHECK(lbib_set_repulsion(h, -1.0, 2.0) == LBIB_EINVAL);
  CHECK(lbib_set_repulsion(h, 1e-5, 0.0) == LBIB_EINVAL);
  CHECK(lbib_set_repulsion(h, 1e-5, 2.0) == LBIB_OK);

  std::vector<double> rho(96 * 48, 1.0), ux(96 * 48, 0.0), uy(96 * 48, 0.0);
  CHECK(lbib_init_fields(h, rho.data(), ux.data(), uy.data()) == LBIB_OK);
  CHECK(lbib_init_fields(h, nullptr, nullptr, nullptr) == LBIB_OK);
  rho[5] = -1.0;
  CHECK(lbib_init_fields(h, rho.data(), ux.data(), uy.data()) == LBIB_EINVAL);

  // phases: running-phase calls are refused during set-up, with no effect
  double out[4];
  int32_t n = 0;
  int64_t st = -1;
  size_t bytes = 0;
  CHECK(lbib_step(h, 1) == LBIB_ESTATE);
  CHECK(lbib_finalize_setup(h) == LBIB_ESTATE);
  CHECK(lbib_get_fields(h, out, out, out) == LBIB_ESTATE);
  CHECK(lbib_get_markers(h, 0, out) == LBIB_ESTATE);
  CHECK(lbib_get_bonds(h, &n, &n) == LBIB_ESTATE);
  CHECK(lbib_get_state(h, nullptr, &bytes) == LBIB_ESTATE);
  CHECK(lbib_set_state(h, out, sizeof(out)) == LBIB_ESTATE);
  CHECK(lbib_observe(h) == LBIB_ESTATE);
  CHECK(lbib_set_body_params(h, 0, 0.1, 0.0, 0.0) == LBIB_ESTATE);
  CHECK(lbib_get_step(h, &st) == LBIB_OK && st == 0);
  CHECK(lbib_num_ligands(h, &n) == LBIB_OK && n == 12 + 65);

  // workspace: the size query, then bind's checks that come before any HIP call
  size_t nb = 0;
  CHECK(lbib_workspace_query(h, nullptr) == LBIB_EINVAL);
  CHECK(lbib_workspace_query(h, &nb) == LBIB_OK && nb > (size_t)96 * 48 * 9 * 4 * 2);
  CHECK(lbib_bind(h, nullptr, nb, nullptr) == LBIB_EINVAL);
  CHECK(lbib_bind(h, reinterpret_cast<void*>(4096 + 8), nb, nullptr) == LBIB_EINVAL);
  CHECK(lbib_bind(h, reinterpret_cast<void*>(4096), nb - 1, nullptr) == LBIB_ENOSPACE);
  CHECK(lbib_set_graph_steps(h, 3) == LBIB_EINVAL);
  CHECK(lbib_set_graph_steps(h, -2) == LBIB_EINVAL);
  CHECK(lbib_set_graph_steps(h, 4) == LBIB_OK);
  CHECK(lbib_set_step_mode(h, 7) == LBIB_EINVAL);
  CHECK(lbib_set_step_mode(h, 1) == LBIB_OK);
  CHECK(lbib_set_cache_hints(h, 2) == LBIB_EINVAL);
  CHECK(lbib_set_cache_hints(h, 3) == LBIB_OK);
  CHECK(lbib_set_watchdog_mass_tolerance(h, -1.0) == LBIB_EINVAL);
  size_t an = 0;
  CHECK(lbib_adjoint_workspace_query(h, 10, 5, &an) == LBIB_ESTATE);
  CHECK(lbib_last_error(h) != nullptr && std::strlen(lbib_last_error(h)) > 0);
  CHECK(lbib_destroy(h) == LBIB_OK);
}

static void test_workspace_sizes() {
  // larger lattices, more bodies and float64 all need more workspace
  size_t prev = 0;
  for (int s = 1; s <= 4; ++s) {
    for (int dt = 0; dt < 2; ++dt) {
      lbib_ctx* h = nullptr;
      lbib_lattice_desc d = lattice(64 * s, 32 * s, dt);
      CHECK(lbib_create(&d, &h) == LBIB_OK);
      for (int k = 0; k < s; ++k) {
        lbib_body_desc b = body(LBIB_RBC_KINEMATIC, 30 + 17 * k);
        std::vector<double> xy = circle(20.0 + 40.0 * k, 16.0 * s, 4.0, 30 + 17 * k);
        int32_t id;
        CHECK(lbib_add_body(h, &b, xy.data(), &id) == LBIB_OK);
      }
      size_t nb = 0;
      CHECK(lbib_workspace_query(h, &nb) == LBIB_OK);
      CHECK(nb > prev);
      prev = nb;
      lbib_destroy(h);
    }
  }
}

static void test_batch_rules() {
  lbib_ctx* a = nullptr;
  lbib_ctx* b = nullptr;
  lbib_ctx* c = nullptr;
  lbib_lattice_desc d1 = lattice(64, 32), d2 = lattice(80, 32), d3 = lattice(64, 32, LBIB_F64);
  CHECK(lbib_create(&d1, &a) == LBIB_OK && lbib_create(&d2, &b) == LBIB_OK &&
        lbib_create(&d3, &c) == LBIB_OK);
  lbib_ctx* out = nullptr;
  const lbib_ctx* mixed[2] = {a, c};
  const lbib_ctx* same[2] = {a, b};
  const lbib_ctx* hole[2] = {a, nullptr};
  CHECK(lbib_batch_create(nullptr, 2, 0, 0, &out) == LBIB_EINVAL);
  CHECK(lbib_batch_create(same, 0, 0, 0, &out) == LBIB_EINVAL);
  CHECK(lbib_batch_create(hole, 2, 0, 0, &out) == LBIB_EINVAL);
  CHECK(lbib_batch_create(mixed, 2, 0, 0, &out) == LBIB_EINVAL);
  CHECK(lbib_batch_create(same, 2, 48, 4, &out) == LBIB_EINVAL);   // no such tile
  CHECK(lbib_batch_create(same, 2, 0, 0, &out) == LBIB_OK && out != nullptr);
  int32_t n = 0;
  CHECK(lbib_batch_size(out, &n) == LBIB_OK && n == 2);
  size_t nb = 0;
  CHECK(lbib_workspace_query(out, &nb) == LBIB_OK && nb > 0);
  double buf[8];
  CHECK(lbib_batch_get_fields(out, 0, buf, buf, buf) == LBIB_ESTATE);
  CHECK(lbib_destroy(out) == LBIB_OK);
  lbib_destroy(a);
  lbib_destroy(b);
  lbib_destroy(c);
}

// Seeded malformed inputs: every call returns a status, none crashes.
static void test_seeded_malformed_inputs() {
  std::mt19937_64 rng(1907);
  std::uniform_real_distribution<double> U(-2.0, 2.0);
  const double specials[] = {0.0, -0.0, 1e308, -1e308, 5e-324, std::numeric_limits<double>::quiet_NaN(),
                             std::numeric_limits<double>::infinity()};
  for (int it = 0; it < 400; ++it) {
    lbib_lattice_desc d = lattice(1 + (int)(rng() % 300) - 20, 1 + (int)(rng() % 120) - 10,
                                  (int)(rng() % 3));
    d.tau = rng() % 5 == 0 ? specials[rng() % 7] : 0.5 + std::fabs(U(rng));
    d.periodic_y = (int)(rng() % 3) - 1;
    d.tile_x = (int)(rng() % 300);
    d.tile_y = (int)(rng() % 10);
    lbib_ctx* h = nullptr;
    const lbib_status s = lbib_create(&d, &h);
    CHECK(s == LBIB_OK || s == LBIB_EINVAL);
    if (s != LBIB_OK) continue;
    const int nb = (int)(rng() % 4);
    for (int k = 0; k < nb; ++k) {
      const int nv = (int)(rng() % 200) - 5;
      lbib_body_desc b = body((int)(rng() % 4), nv);
      b.ks = rng() % 7 == 0 ? specials[rng() % 7] : std::fabs(U(rng));
      b.ligand_stride = (int)(rng() % 5) - 1;
      std::vector<double> xy = circle(std::fabs(U(rng)) * d.nx, std::fabs(U(rng)) * d.ny,
                                      0.5 + std::fabs(U(rng)) * 10.0, nv > 0 ? nv : 1, rng() % 4 != 0);
      if (rng() % 5 == 0) xy[rng() % xy.size()] = specials[rng() % 7];
      int32_t id = -1;
      const lbib_status sb = lbib_add_body(h, &b, nv > 0 ? xy.data() : nullptr, &id);
      CHECK(sb == LBIB_OK || sb == LBIB_EINVAL);
    }
    std::vector<double> rec(1 + rng() % 64);
    for (size_t k = 0; k < rec.size(); ++k) rec[k] = k * std::fabs(U(rng)) * 3.0 - 2.0;
    const lbib_status sr = lbib_set_receptors(h, (int)(rng() % 3), rec.data(), (int32_t)rec.size());
    CHECK(sr == LBIB_OK || sr == LBIB_EINVAL);
    size_t bytes = 0;
    CHECK(lbib_workspace_query(h, &bytes) == LBIB_OK);
    CHECK(lbib_step(h, 1) == LBIB_ESTATE);
    CHECK(lbib_destroy(h) == LBIB_OK);
  }
}

int main() {
  test_create();
  test_bodies_and_setup_calls();
  test_workspace_sizes();
  test_batch_rules();
  test_seeded_malformed_inputs();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("abi_sanitize: all checks passed\n");
  return 0;
}
