// startup.cpp -- start-up length of a fallback MD run (Alg. 1 "pseudoMD";
// Sec. 2.4): a 1-D Navier-Stokes solve of the channel with a Navier slip
// condition u = b du/dn at both walls,
//     du/dt = g* + nu d2u/dy2,  0 < y < h,
// from the steady profile of the prior run's body force g_in (g_in = 0 for a
// start from rest).  The deviation from the new steady profile lives in the
// symmetric modes cos(k_n (y - h/2)) with cot(k_n h / 2) = b k_n and decays as
// exp(-nu k_n^2 t); the start-up time is the first t at which the flow rate
// is within tol of its new steady value, relative to the larger of the old
// and new steady flow rates.  Host code, FP64.
#include "startup.h"

#include <cmath>
#include <vector>

namespace hmd {

namespace {

constexpr double kPi = 3.141592653589793;

// roots of cos z - c z sin z = 0, z = k h / 2, one in each ((n-1) pi, (n-1/2) pi]
double root(int n, double c) {
  double lo = double(n - 1) * kPi, hi = (double(n) - 0.5) * kPi;
  if (c == 0.0) return hi;
  if (n == 1) lo += 1e-15;
  double flo = std::cos(lo) - c * lo * std::sin(lo);
  for (int it = 0; it < 200; ++it) {
    const double m = 0.5 * (lo + hi);
    const double fm = std::cos(m) - c * m * std::sin(m);
    if ((fm > 0.0) == (flo > 0.0)) {
      lo = m;
      flo = fm;
    } else {
      hi = m;
    }
  }
  return 0.5 * (lo + hi);
}

}  // namespace

double steady_flow_rate(double h, double g, double nu, double b) {
  return g * h * h * h * (1.0 + 6.0 * b / h) / (12.0 * nu);
}

double startup_time(double h, double g_in, double g_new, double nu, double b, double tol, int n_modes) {
  const double dg = g_in - g_new, a = 0.5 * h;
  std::vector<double> cw(n_modes), rate(n_modes);
  for (int n = 1; n <= n_modes; ++n) {
    const double k = 2.0 * root(n, 2.0 * b / h) / h;
    const double s = std::sin(k * a), c = std::cos(k * a);
    const double phi_int = 2.0 * s / k;
    const double phi_sq = a + std::sin(2.0 * k * a) / (2.0 * k);
    const double x2 = 2.0 * a * a * s / k + 4.0 * a * c / (k * k) - 4.0 * s / (k * k * k);
    const double proj = (dg / (2.0 * nu)) * ((a * a + b * h) * phi_int - x2);
    cw[n - 1] = proj / phi_sq * phi_int;
    rate[n - 1] = nu * k * k;
  }
  auto dev = [&](double t) {
    double sum = 0.0;
    for (int n = 0; n < n_modes; ++n) sum += cw[n] * std::exp(-rate[n] * t);
    return std::fabs(sum);
  };
  const double target =
      tol * std::fmax(std::fabs(steady_flow_rate(h, g_in, nu, b)), std::fabs(steady_flow_rate(h, g_new, nu, b)));
  if (dev(0.0) <= target) return 0.0;
  double hi = 1.0 / rate[0];
  while (dev(hi) > target) hi *= 2.0;
  double lo = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double m = 0.5 * (lo + hi);
    if (dev(m) > target) lo = m;
    else hi = m;
  }
  return hi;
}

int64_t startup_steps(double t_s, double dt, int64_t n_min) {
  const int64_t n = int64_t(std::ceil(t_s / dt - 1e-9));
  return n > n_min ? n : n_min;
}

}  // namespace hmd
