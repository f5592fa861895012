// md_setup.h -- host-side system construction shared by the MD engine.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hmd.h"

namespace hmd {

// One channel system as built on the host before upload.
struct HostSystem {
  double h = 0, g = 0;
  uint64_t seed = 0;
  double aw = 0, Lx = 0, Lz = 0;   // wall cube edge, snapped periodic extents
  int64_t nf = 0, nw = 0;          // fluid and wall atom counts
  std::vector<double> x, v;        // fluid, nf x 3 (atom id order)
  std::vector<double> xw;          // wall, nw x 3
  int nx = 0, ny = 0, nz = 0;      // fluid cell grid
  double wx = 0, wy = 0, wz = 0;   // cell widths
  double inv_x = 0, inv_y = 0, inv_z = 0;  // n_a / L_a
  int nbins = 0;                   // wall-normal profile bins
};

void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]);
// Cells are at least `wmin` wide (>= rc) in every direction.
int build_system(const hmd_md_params& P, double h, double g, uint64_t seed, double wmin, HostSystem& S,
                 std::string& err);
// Cell coordinate rule: floor(x * (n / L)) clamped to [0, n - 1].
int cell_coord(double x, double inv, int n);

}  // namespace hmd
