// Host-only parts of the library: position -> node mapping, the stability
// check (ValidConditions) and the optimal checkpoint schedule used by the
// gradient's backward sweep.  No GPU code; unit-testable on any machine.
#include "wfd_plan.h"

#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

namespace wfd {

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
bool map_position(const wfd_grid &g, const double xyz[3], int32_t ijk[3]) {
  const int32_t n[3] = {g.nx, g.ny, g.nz};
  const double o[3] = {g.ox, g.oy, g.oz};
  const double h[3] = {g.dx, g.dy, g.dz};
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(xyz[d])) return false;
    const double f = std::floor((xyz[d] - o[d]) / h[d] + 0.5);
    if (f < 0.0 || f >= (double)n[d]) return false;
    ijk[d] = (int32_t)f + g.border;
  }
  return true;
}

// max over wavenumbers of the 1-D symbol of -d2/dx2 (h = 1): 2048 / 315.
double laplacian_symbol_max() {
  const double w[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
  double s = -w[0];
  for (int j = 1; j <= 4; ++j) s -= 2.0 * w[j] * ((j & 1) ? -1.0 : 1.0);
  return s;
}

double cfl_ratio(const wfd_grid &g, double vmax, double m2max) {
  const double lam =
      laplacian_symbol_max() * (1.0 / (g.dx * g.dx) + 1.0 / (g.dy * g.dy) + 1.0 / (g.dz * g.dz));
  const double m2 = m2max > 0.0 ? m2max : 0.0;
  return g.dt * g.dt * vmax * vmax * (lam + m2) / 4.0;
}

// ---------------------------------------------------------------------------
// optimal checkpointing (binomial schedule)
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kCap = int64_t(1) << 62;

// C(s + t, t), saturated at kCap.
int64_t binom(int64_t s, int64_t t) {
  if (s < 0 || t < 0) return 0;
  unsigned __int128 v = 1;
  for (int64_t i = 1; i <= t; ++i) {
    v = v * (unsigned __int128)(s + i) / (unsigned __int128)i;
    if (v > (unsigned __int128)kCap) return kCap;
  }
  return (int64_t)v;
}

}  // namespace

// Least forward steps to consume states x_{l-1} .. x_0 in reverse order when
// x_0 is stored and c more states may be stored at once.  Closed form of
// Griewank & Walther with s = c + 1 snapshots: t*l - C(s+t, t-1), t minimal
// with C(s+t, t) >= l.
int64_t checkpoint_cost(int64_t l, int64_t c) {
  if (l <= 1) return 0;
  if (c <= 0) return l * (l - 1) / 2;
  const int64_t s = c + 1;
  int64_t t = 1;
  while (binom(s, t) < l) ++t;
  return t * l - binom(s + 1, t - 1);
}

namespace {

struct PlanBuilder {
  std::vector<int32_t> out;
  std::vector<int32_t> free_slots;
  int64_t steps = 0;

  void emit(int32_t op, int32_t a, int32_t b) {
    out.push_back(op);
    out.push_back(a);
    out.push_back(b);
  }

  // Consume states x_{a+l-1} .. x_{a+1} (and x_a itself when visit_first) in
  // reverse order; x_a is available (stored, or the zero initial state), c
  // storage slots are free.
  void run(int32_t a, int64_t l, int64_t c, bool visit_a) {
    if (l <= 0) return;
    if (l == 1) {
      if (visit_a) emit(kVisit, a, 0);
      return;
    }
    if (c == 0) {
      for (int64_t j = l - 1; j >= 1; --j) {
        emit(kAdvance, a, (int32_t)(a + j));
        steps += j;
        emit(kVisit, (int32_t)(a + j), 0);
      }
      if (visit_a) emit(kVisit, a, 0);
      return;
    }
    // best first split
    int64_t best_j = 1, best = std::numeric_limits<int64_t>::max();
    for (int64_t j = 1; j < l; ++j) {
      const int64_t v = j + checkpoint_cost(l - j, c - 1) + checkpoint_cost(j, c);
      if (v <= best) {
        best = v;
        best_j = j;
      }
    }
    const int32_t m = (int32_t)(a + best_j);
    emit(kAdvance, a, m);
    steps += best_j;
    if (l - best_j == 1) {
      emit(kVisit, m, 0);  // consumed at once, no storage needed
    } else {
      const int32_t slot = free_slots.back();
      free_slots.pop_back();
      emit(kStore, m, slot);
      run(m, l - best_j, c - 1, true);
      emit(kFree, m, slot);
      free_slots.push_back(slot);
    }
    run(a, best_j, c, visit_a);
  }
};

}  // namespace

void build_checkpoint_plan(int32_t nt, int32_t n_snapshots, std::vector<int32_t> &actions,
                           int64_t &n_forward_steps) {
  PlanBuilder b;
  for (int32_t s = n_snapshots - 1; s >= 0; --s) b.free_slots.push_back(s);
  // states x_0 .. x_nt, x_0 = zero (free); visits nt .. 1
  b.run(0, (int64_t)nt + 1, n_snapshots, false);
  actions.swap(b.out);
  n_forward_steps = b.steps;
}

}  // namespace wfd
