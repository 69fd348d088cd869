// Host unit tests of the library's pure-host code (csrc/wfd_plan.cpp):
// position -> node mapping, the stability symbol, and the binomial checkpoint
// schedule that the gradient's backward sweep executes.  Built with g++ under
// the address and undefined-behaviour sanitizers by tests/test_host_cpp.py.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

#include "wfd_plan.h"

static int failures = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);          \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static wfd_grid grid() {
  wfd_grid g{};
  g.nx = 10, g.ny = 7, g.nz = 5;
  g.dx = 10.0, g.dy = 5.0, g.dz = 2.5;
  g.ox = -20.0, g.oy = 100.0, g.oz = 0.0;
  g.border = 3, g.dt = 1e-3, g.nt = 1;
  return g;
}

static bool node(const wfd_grid &g, double x, double y, double z, int ex, int ey, int ez) {
  const double p[3] = {x, y, z};
  int32_t ijk[3] = {-1, -1, -1};
  return wfd::map_position(g, p, ijk) && ijk[0] == ex && ijk[1] == ey && ijk[2] == ez;
}

static bool outside(const wfd_grid &g, double x, double y, double z) {
  const double p[3] = {x, y, z};
  int32_t ijk[3];
  return !wfd::map_position(g, p, ijk);
}

static void test_positions() {
  const wfd_grid g = grid();
  CHECK(node(g, -20.0, 100.0, 0.0, 3, 3, 3));          // the origin is model node 0
  CHECK(node(g, 5.0, 102.5, 1.25, 6, 4, 4));           // exact halves round up
  CHECK(node(g, 4.999, 102.499, 1.2499, 5, 3, 3));     // just below a half rounds down
  CHECK(node(g, -25.0, 97.5, -1.25, 3, 3, 3));         // half a cell before node 0: inside
  CHECK(outside(g, -25.0001, 100.0, 0.0));             // past it: outside
  CHECK(node(g, 74.999, 132.499, 11.249, 12, 9, 7));   // last nodes (9, 6, 4) + border
  CHECK(outside(g, 75.0, 100.0, 0.0));                 // rounds to node nx: outside
  CHECK(outside(g, 0.0, 132.5, 0.0));
  CHECK(outside(g, 0.0, 100.0, 11.25));
  CHECK(outside(g, std::nan(""), 100.0, 0.0));
  CHECK(outside(g, 0.0, std::numeric_limits<double>::infinity(), 0.0));
}

static void test_stability() {
  // the 1-D symbol of -D2 peaks at theta = pi with value 2048/315 (h = 1)
  CHECK(std::fabs(wfd::laplacian_symbol_max() - 2048.0 / 315.0) < 1e-14);
  wfd_grid g = grid();
  g.dx = g.dy = g.dz = 10.0;
  // constant density, equal spacing: Courant limit c dt / h < 2 / sqrt(3 * 2048 / 315)
  const double courant = 2.0 / std::sqrt(3.0 * 2048.0 / 315.0);
  g.dt = courant * 10.0 / 3000.0;
  CHECK(std::fabs(wfd::cfl_ratio(g, 3000.0, 0.0) - 1.0) < 1e-12);
  CHECK(std::fabs(wfd::cfl_ratio(g, 3000.0, -5.0) - 1.0) < 1e-12);  // negative m^2 ignored
  CHECK(wfd::cfl_ratio(g, 3000.0, 1e-3) > 1.0);
}

// Least forward steps by dynamic programming (independent of the closed form):
// consume l states in reverse with the first stored and c more slots.
static std::vector<std::vector<int64_t>> dp_costs(int lmax, int cmax) {
  std::vector<std::vector<int64_t>> F(lmax + 1, std::vector<int64_t>(cmax + 1, 0));
  for (int l = 2; l <= lmax; ++l) {
    F[l][0] = (int64_t)l * (l - 1) / 2;
    for (int c = 1; c <= cmax; ++c) {
      int64_t best = std::numeric_limits<int64_t>::max();
      for (int j = 1; j < l; ++j) {
        const int64_t v = j + F[l - j][c - 1] + F[j][c];
        if (v < best) best = v;
      }
      F[l][c] = best;
    }
  }
  return F;
}

// Execute a plan the way the gradient does: states available are the zero
// state 0, stored slots, the current state and the one before it.  Checks
// each action's precondition, the visit order nt .. 1, and returns the steps.
static int64_t execute(const std::vector<int32_t> &plan, int nt, int nsnap, bool &ok) {
  std::vector<int> slot(nsnap, -1);
  int cur = -1, prev = -1, next_visit = nt;
  int64_t steps = 0;
  ok = true;
  auto stored = [&](int s) {
    for (int v : slot)
      if (v == s) return true;
    return false;
  };
  if (plan.size() % 3) ok = false;
  for (size_t i = 0; ok && i + 3 <= plan.size(); i += 3) {
    const int op = plan[i], a = plan[i + 1], b = plan[i + 2];
    if (op == wfd::kAdvance) {
      if (!(a == 0 || a == cur || stored(a)) || b <= a || b > nt) ok = false;
      steps += b - a;
      prev = b - 1;
      cur = b;
    } else if (op == wfd::kStore) {
      if (a != cur || b < 0 || b >= nsnap || slot[b] != -1) ok = false;
      else slot[b] = a;
    } else if (op == wfd::kVisit) {
      if (a != next_visit || !(a == cur || a == prev || stored(a))) ok = false;
      --next_visit;
    } else if (op == wfd::kFree) {
      if (b < 0 || b >= nsnap || slot[b] != a) ok = false;
      else slot[b] = -1;
    } else {
      ok = false;
    }
  }
  if (next_visit != 0) ok = false;
  for (int v : slot)
    if (v != -1) ok = false;
  return steps;
}

static void test_checkpoint_plans() {
  const int lmax = 80, cmax = 12;
  const auto F = dp_costs(lmax, cmax);
  for (int l = 1; l <= lmax; ++l)
    for (int c = 0; c <= cmax; ++c) CHECK(wfd::checkpoint_cost(l, c) == F[l][c]);
  for (int nt = 1; nt < lmax; ++nt)
    for (int s = 1; s <= cmax; ++s) {
      std::vector<int32_t> plan;
      int64_t n = -1;
      wfd::build_checkpoint_plan(nt, s, plan, n);
      bool ok = false;
      const int64_t steps = execute(plan, nt, s, ok);
      CHECK(ok);
      CHECK(steps == n);
      CHECK(n == F[nt + 1][s]);
    }
  // the gradient workload: 1200 steps with 20 stored pairs.  The zero initial
  // state needs no slot, so this is the closed form t l - C(s + t, t - 1) for
  // l = 1201 states and s = 21 snapshots (t = 3): 3603 - 276 = 3327 steps, of
  // which 1200 are the recording sweep.
  std::vector<int32_t> plan;
  int64_t n = 0;
  wfd::build_checkpoint_plan(1200, 20, plan, n);
  bool ok = false;
  CHECK(execute(plan, 1200, 20, ok) == 3327 && ok && n == 3327);
}

int main() {
  test_positions();
  test_stability();
  test_checkpoint_plans();
  if (failures) {
    std::printf("%d FAILED\n", failures);
    return 1;
  }
  std::printf("ALL PASSED\n");
  return 0;
}
