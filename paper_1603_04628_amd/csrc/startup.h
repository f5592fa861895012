// startup.h -- start-up length of a fallback MD run (see startup.cpp).
#pragma once

#include <cstdint>

namespace hmd {

// Steady flow rate per unit span and unit density of the channel:
// g h^3 (1 + 6 b / h) / (12 nu).
double steady_flow_rate(double h, double g, double nu, double b);
// Start-up time of the 1-D channel flow with Navier slip b from the steady
// profile of body force g_in to that of g_new: the first t with
// |q(t) - q*| <= tol max(|q_in|, |q*|) (0 when already within it).
double startup_time(double h, double g_in, double g_new, double nu, double b, double tol, int n_modes = 200);
// Equilibration steps: ceil(t_s / dt), at least n_min.
int64_t startup_steps(double t_s, double dt, int64_t n_min);

}  // namespace hmd
