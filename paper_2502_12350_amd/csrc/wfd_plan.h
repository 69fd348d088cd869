// Host-only helpers shared by the C ABI (wfd_api.cpp) and the plan code.
#pragma once

#include <cstdint>
#include <vector>

#include "wfd.h"

namespace wfd {

enum : int32_t { kAdvance = 0, kStore = 1, kVisit = 2, kFree = 3 };

// Padded-grid node (ix, iy, iz) of a position in metres: nearest node,
// round half up; false when outside the model.
bool map_position(const wfd_grid &g, const double xyz[3], int32_t ijk[3]);

double laplacian_symbol_max();
double cfl_ratio(const wfd_grid &g, double vmax, double m2max);

int64_t checkpoint_cost(int64_t l, int64_t c);
void build_checkpoint_plan(int32_t nt, int32_t n_snapshots, std::vector<int32_t> &actions,
                           int64_t &n_forward_steps);

}  // namespace wfd
