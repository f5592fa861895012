// md_setup.cpp -- host-side construction of one NEMD channel system:
// frozen wall lattice, fluid start lattice, Maxwell velocities, cell grid.
//
// Model (paper, Appendix A): LJ fluid between frozen FCC walls, periodic in
// x and z.  Start (Sec. 2.4): a lattice with zero mean velocity.  The
// readings used where the paper is silent (wall registry, lattice choice,
// random streams) are documented with the design notes; the formulas below
// are the definitions every implementation of this model has to share.
//
// Built with -ffp-contract=off so every expression rounds as written.
#include "md_setup.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hmd {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products mixed with the counter and a Weyl-sequence key.
void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {in[0], in[1], in[2], in[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    const uint64_t a = uint64_t(0xD2511F53u) * c[0];
    const uint64_t b = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t next[4] = {uint32_t(b >> 32) ^ c[1] ^ k[0], uint32_t(b),
                              uint32_t(a >> 32) ^ c[3] ^ k[1], uint32_t(a)};
    std::memcpy(c, next, sizeof(c));
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
  std::memcpy(out, c, sizeof(c));
}

namespace {

inline double open_unit(uint32_t r) { return (double(r) + 0.5) * (1.0 / 4294967296.0); }

struct Stack {
  int planes, mx, mz;
  double gap, ax, az;
};

// Among plane counts 1..floor(D/0.5)+1, pick the square-plane stack (planes
// shifted by half a spacing) with at least nf sites whose closest pair is
// farthest apart; ties keep the smaller plane count.
Stack pick_stack(int64_t nf, double Lx, double Lz, double D) {
  Stack best{1, 1, 1, 0.0, Lx, Lz};
  double best_d = -1.0;
  const int top = std::max(1, int(std::floor(D / 0.5)) + 1);
  for (int planes = 1; planes <= top; ++planes) {
    const double gap = planes > 1 ? D / double(planes - 1) : 0.0;
    const int64_t per_plane = (nf + planes - 1) / planes;
    const int mx = std::max(1, int(std::ceil(std::sqrt(double(per_plane) * Lx / Lz))));
    const int mz = std::max(1, int((per_plane + mx - 1) / mx));
    const double ax = Lx / double(mx), az = Lz / double(mz);
    double closest = std::min(ax, az);
    if (planes > 1) closest = std::min(closest, std::sqrt(0.25 * ax * ax + 0.25 * az * az + gap * gap));
    if (planes > 2) closest = std::min(closest, 2.0 * gap);
    if (closest > best_d) {
      best_d = closest;
      best = Stack{planes, mx, mz, gap, ax, az};
    }
  }
  return best;
}

}  // namespace

int build_system(const hmd_md_params& P, double h, double g, uint64_t seed, double wmin, HostSystem& S,
                 std::string& err) {
  if (!(h > 2.0 * P.delta) || !std::isfinite(h) || !std::isfinite(g)) {
    err = "channel height must exceed twice the start gap delta";
    return HMD_EINVAL;
  }
  // the thermostat may not act on the streamwise component: it would damp
  // the flow that is being measured
  if (!(P.rc > 0.0) || !(P.rho > 0.0) || !(P.rho_wall > 0.0) || !(P.dt > 0.0) || !(P.tau_T > 0.0) ||
      P.wall_layers < 0 || P.thermo_axis < 1 || P.thermo_axis > 2 || P.n_blocks < 0 || P.n_blocks == 1 ||
      P.n_blocks > 1024 || !(P.tile_alpha >= 0.0) || P.graph_chunk < 0 || (P.graph_chunk & 1) || !(P.bin_dy > 0.0) ||
      !(wmin >= P.rc)) {
    err = "invalid MD parameters (thermostat axis must be 1 or 2)";
    return HMD_EINVAL;
  }
  S = HostSystem{};
  S.h = h;
  S.g = g;
  S.seed = seed;
  S.aw = std::cbrt(4.0 / P.rho_wall);
  const int cubes_x = std::max(1, int(std::lround(P.Lx_nom / S.aw)));
  const int cubes_z = std::max(1, int(std::lround(P.Lz_nom / S.aw)));
  S.Lx = double(cubes_x) * S.aw;
  S.Lz = double(cubes_z) * S.aw;
  if (S.Lx < 3.0 * wmin || S.Lz < 3.0 * wmin) {
    err = "periodic extent must hold at least three cells";
    return HMD_EINVAL;
  }

  // Walls: layer k at y = -k a/2 (lower) and h + k a/2 (upper); sites
  // (p a/2, q a/2) with p + q + k even.
  const double half = 0.5 * S.aw;
  for (int side = 0; side < 2; ++side)
    for (int k = 0; k < P.wall_layers; ++k) {
      const double y = side == 0 ? -double(k) * half : h + double(k) * half;
      for (int q = 0; q < 2 * cubes_z; ++q)
        for (int p = 0; p < 2 * cubes_x; ++p)
          if (((p + q + k) & 1) == 0) {
            S.xw.push_back(double(p) * half);
            S.xw.push_back(y);
            S.xw.push_back(double(q) * half);
          }
    }
  S.nw = int64_t(S.xw.size() / 3);

  S.nf = P.n_fluid > 0 ? P.n_fluid : int64_t(std::llround(P.rho * S.Lx * S.Lz * h));
  if (S.nf < 1 || S.nf > (int64_t(1) << 30)) {
    err = "fluid atom count out of range";
    return HMD_EINVAL;
  }

  // Start lattice and the seed-keyed choice of nf of its sites.
  const Stack st = pick_stack(S.nf, S.Lx, S.Lz, h - 2.0 * P.delta);
  const int64_t sites = int64_t(st.planes) * st.mx * st.mz;
  std::vector<int64_t> pick(sites);
  for (int64_t i = 0; i < sites; ++i) pick[i] = i;
  const uint32_t key[2] = {uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32)};
  for (int64_t i = sites - 1; i > 0; --i) {
    const uint32_t ctr[4] = {uint32_t(i), 0u, 0u, 0u};
    uint32_t r[4];
    philox4x32_10(ctr, key, r);
    const int64_t j = int64_t((uint64_t(r[0]) * uint64_t(i + 1)) >> 32);
    std::swap(pick[i], pick[j]);
  }
  std::sort(pick.begin(), pick.begin() + S.nf);
  S.x.resize(3 * S.nf);
  S.v.resize(3 * S.nf);
  for (int64_t n = 0; n < S.nf; ++n) {
    const int64_t site = pick[n];
    const int i = int(site % st.mx), k = int((site / st.mx) % st.mz);
    const int plane = int(site / (int64_t(st.mx) * st.mz));
    const double shift = (plane & 1) ? 0.5 : 0.0;
    S.x[3 * n + 0] = (double(i) + shift) * st.ax;
    S.x[3 * n + 1] = st.planes > 1 ? P.delta + double(plane) * st.gap : 0.5 * h;
    S.x[3 * n + 2] = (double(k) + shift) * st.az;
  }

  // Maxwell velocities: Box-Muller on the draws of counter (n, 1, 0, 0).
  const double two_pi = 6.283185307179586;
  const double sd = std::sqrt(P.T0);
  for (int64_t n = 0; n < S.nf; ++n) {
    const uint32_t ctr[4] = {uint32_t(n), 1u, 0u, 0u};
    uint32_t r[4];
    philox4x32_10(ctr, key, r);
    const double ra = std::sqrt(-2.0 * std::log(open_unit(r[0])));
    const double ta = two_pi * open_unit(r[1]);
    const double rb = std::sqrt(-2.0 * std::log(open_unit(r[2])));
    const double tb = two_pi * open_unit(r[3]);
    S.v[3 * n + 0] = sd * (ra * std::cos(ta));
    S.v[3 * n + 1] = sd * (ra * std::sin(ta));
    S.v[3 * n + 2] = sd * (rb * std::cos(tb));
  }
  double mean[3] = {0.0, 0.0, 0.0};
  for (int64_t n = 0; n < S.nf; ++n)
    for (int a = 0; a < 3; ++a) mean[a] += S.v[3 * n + a];
  for (double& m : mean) m = m / double(S.nf);
  double sum_sq = 0.0;
  for (int64_t n = 0; n < S.nf; ++n) {
    for (int a = 0; a < 3; ++a) S.v[3 * n + a] = S.v[3 * n + a] - mean[a];
    const double* w = &S.v[3 * n];
    sum_sq += w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  }
  const double scale = std::sqrt(P.T0 / (sum_sq / (3.0 * double(S.nf))));
  for (double& w : S.v) w = w * scale;

  // Cell grid: widths >= wmin over [0,Lx) x [0,h) x [0,Lz).
  S.nx = int(std::floor(S.Lx / wmin));
  S.ny = std::max(1, int(std::floor(h / wmin)));
  S.nz = int(std::floor(S.Lz / wmin));
  S.wx = S.Lx / double(S.nx);
  S.wy = h / double(S.ny);
  S.wz = S.Lz / double(S.nz);
  S.inv_x = double(S.nx) / S.Lx;
  S.inv_y = double(S.ny) / h;
  S.inv_z = double(S.nz) / S.Lz;
  S.nbins = int(std::ceil(h / P.bin_dy));
  return HMD_OK;
}

int cell_coord(double x, double inv, int n) {
  const double t = std::floor(x * inv);
  if (!(t >= 0.0)) return 0;
  if (t >= double(n - 1)) return n - 1;
  return int(t);
}

}  // namespace hmd
