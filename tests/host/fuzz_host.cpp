// Host-side fuzzing of the C ABI's validation, layout and batching code, built
// with AddressSanitizer and UndefinedBehaviorSanitizer for the host only and
// run on the CPU (no HIP call is reached: every case either fails validation,
// has an empty grid, passes NULL buffers, or is host-only by definition).
// Exits non-zero on any inconsistency; the sanitizers abort on memory errors
// and undefined behaviour.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "hweno.h"

static int failures = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);   \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static hweno_problem base(std::mt19937_64& g) {
  hweno_problem p;
  std::memset(&p, 0, sizeof p);
  std::uniform_int_distribution<int> small(-3, 40), pick(0, 9);
  p.dim = 1 + (int)(g() % 2);
  p.nx = small(g);
  p.ny = p.dim == 2 ? small(g) : 1;
  p.physics = (int)(g() % 4) - (pick(g) == 0 ? 1 : 0);
  p.dtype = (int)(g() % 3);
  p.bc_x = (int)(g() % 4);
  p.bc_y = (int)(g() % 4);
  p.characteristic = (int)(g() % 2);
  p.limiter_on = (int)(g() % 2);
  p.limiter_characteristic = (int)(g() % 3);
  std::uniform_real_distribution<double> u(-0.5, 2.0);
  p.dx = u(g);
  p.dy = u(g);
  p.gamma_gas = 1.0 + u(g);
  p.adv_speed[0] = u(g);
  p.adv_speed[1] = u(g);
  const double w0 = std::fabs(u(g)) + 0.01, w1 = std::fabs(u(g)) + 0.01, w2 = std::fabs(u(g)) + 0.01;
  const double s = pick(g) == 0 ? 1.0 : w0 + w1 + w2;
  p.lin_w[0] = w0 / s, p.lin_w[1] = w1 / s, p.lin_w[2] = w2 / s;
  p.lim_w[0] = 0.98, p.lim_w[1] = 0.01, p.lim_w[2] = 0.01;
  p.eps = pick(g) == 0 ? -1e-6 : 1e-6;
  p.cfl = pick(g) == 0 ? 0.0 : 0.6;
  if (pick(g) == 0) p.dx = NAN;
  if (pick(g) == 0) p.nx = 1 << 29;
  // edge descriptions (read when a bc is HWENO_BC_EDGES): kinds 0..3, splits and
  // states with the odd non-finite or non-physical value
  std::uniform_real_distribution<double> v(-1.0, 3.0);
  for (auto& e : p.edges) {
    e.kind[0] = (int)(g() % 4), e.kind[1] = (int)(g() % 4);
    for (double& x : e.split) x = pick(g) == 0 ? NAN : v(g);
    for (auto& st : e.state) {
      st[0] = 0.1 + std::fabs(v(g)), st[1] = v(g), st[2] = v(g), st[3] = 5.0 + v(g);
      if (pick(g) == 0) st[3] = -1.0;
    }
  }
  // the obstacle (solid cells i >= i_s, j < j_s): mostly absent, else anything
  if (pick(g) < 3) p.obstacle[0] = small(g), p.obstacle[1] = small(g);
  return p;
}

int main() {
  std::mt19937_64 g(12345);
  int valid = 0;
  for (int it = 0; it < 200000; ++it) {
    hweno_problem p = base(g);
    const hweno_status st = hweno_validate(&p);
    CHECK(st == HWENO_OK || st == HWENO_ERR_INVALID_ARG || st == HWENO_ERR_UNSUPPORTED);
    CHECK(std::strlen(hweno_last_error()) < 4096);
    CHECK(std::strlen(hweno_status_string(st)) > 0);
    const size_t ws = hweno_workspace_bytes(&p), wa = hweno_adjoint_workspace_bytes(&p);
    if (st != HWENO_OK) {
      CHECK(ws == 0 && wa == 0);
      // every entry point refuses an invalid problem before touching any pointer
      CHECK(hweno_rk3_step(&p, nullptr, nullptr, 0, 0.0, 0.0, nullptr, nullptr, nullptr) == st);
      CHECK(hweno_rhs(&p, nullptr, nullptr, nullptr, 1, nullptr) == st);
      CHECK(hweno_limit(&p, nullptr, nullptr, nullptr) == st);
      CHECK(hweno_rk3_steps(&p, nullptr, nullptr, 0, 3, 0.0, 0.0, nullptr, nullptr) == st);
      continue;
    }
    ++valid;
    const bool edges = p.bc_x == HWENO_BC_EDGES || (p.dim == 2 && p.bc_y == HWENO_BC_EDGES);
    CHECK(ws > 0 && ws % 256 == 0 && (edges ? wa == 0 : wa > 0));
    if (edges) {
      // the adjoint has no edge-described sides: refused before any pointer is read
      CHECK(hweno_rhs_adjoint(&p, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
            HWENO_ERR_UNSUPPORTED);
      CHECK(hweno_rk3_step_adjoint(&p, nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr) ==
            HWENO_ERR_UNSUPPORTED);
    }
    const bool empty = p.nx == 0 || (p.dim == 2 && p.ny == 0);
    // NULL buffers: refused, or nothing to do for an empty grid; never a HIP call
    const hweno_status s1 = hweno_rk3_step(&p, nullptr, nullptr, 0, 0.0, 0.0, nullptr, nullptr, nullptr);
    CHECK(empty ? s1 == HWENO_OK : s1 == HWENO_ERR_INVALID_ARG);
    const hweno_status s2 = hweno_rhs(&p, nullptr, nullptr, nullptr, 1, nullptr);
    CHECK(empty ? s2 == HWENO_OK : s2 == HWENO_ERR_INVALID_ARG);
    const hweno_status s3 = hweno_rk3_steps(&p, nullptr, nullptr, 0, 2, 0.0, 0.0, nullptr, nullptr);
    CHECK(empty ? s3 == HWENO_OK : s3 == HWENO_ERR_INVALID_ARG);
    CHECK(hweno_rk3_steps(&p, nullptr, nullptr, 0, -1, 0.0, 0.0, nullptr, nullptr) == HWENO_ERR_INVALID_ARG);
    CHECK(hweno_rk3_steps(&p, nullptr, nullptr, 0, 0, 0.0, 0.0, nullptr, nullptr) == HWENO_OK);
  }
  CHECK(valid > 1000);
  CHECK(hweno_validate(nullptr) == HWENO_ERR_INVALID_ARG);
  CHECK(std::strlen(hweno_status_string(-7)) > 0 && std::strlen(hweno_status_string(99)) > 0);

  // batching: random uneven instances, prepared and mapped on the host
  hweno_problem c;
  std::memset(&c, 0, sizeof c);
  c.dim = 2, c.nx = 1, c.ny = 1, c.physics = HWENO_EULER, c.dtype = HWENO_F32;
  c.characteristic = 1, c.limiter_on = 1, c.dx = c.dy = 1.0, c.gamma_gas = 1.4;
  c.lin_w[0] = c.lim_w[0] = 0.98, c.lin_w[1] = c.lim_w[1] = 0.01, c.lin_w[2] = c.lim_w[2] = 0.01;
  c.eps = 1e-6, c.cfl = 0.6;
  for (int it = 0; it < 2000; ++it) {
    const int n = 1 + (int)(g() % 40);
    std::vector<hweno_instance> inst(n);
    std::memset(inst.data(), 0, sizeof(hweno_instance) * n);
    for (auto& I : inst) {
      I.nx = 1 + (int)(g() % 300) - (g() % 50 == 0 ? 2 : 0);
      I.ny = 1 + (int)(g() % 300);
      I.bc_x = (int)(g() % 3), I.bc_y = (int)(g() % 3);
      I.dx = I.dy = 0.01;
    }
    int32_t total[HWENO_BATCH_VARIANTS] = {0, 0};
    const hweno_status st = hweno_batch_prepare(&c, inst.data(), n, total);
    if (st != HWENO_OK) {
      CHECK(st == HWENO_ERR_INVALID_ARG);
      continue;
    }
    for (int v = 0; v < HWENO_BATCH_VARIANTS; ++v) {
      std::vector<int32_t> map(total[v] + 1, -1);
      CHECK(hweno_batch_tile_map(inst.data(), n, v, map.data(), total[v]) == HWENO_OK);
      int32_t expect = 0;
      for (int q = 0; q < n; ++q) {
        CHECK(inst[q].tile_begin[v] == expect);
        for (int t = 0; t < inst[q].n_tiles[v]; ++t) CHECK(map[expect + t] == q);
        expect += inst[q].n_tiles[v];
      }
      CHECK(expect == total[v] && map[total[v]] == -1);
      // a map shorter than the tile count is refused
      if (total[v] > 1)
        CHECK(hweno_batch_tile_map(inst.data(), n, v, map.data(), total[v] - 1) != HWENO_OK);
    }
  }
  std::printf("host fuzz: %d valid problems, %d failures\n", valid, failures);
  return failures == 0 ? 0 : 1;
}
