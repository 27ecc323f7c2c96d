// Stop rule of run_to_steady for FP32 runs (host code, no HIP).
#pragma once

// FP32 stop "at the rounding floor".  Near its fixed point an FP32 run's
// residual stops decaying at a noise level of ~1e-7 (rounding of the state
// between checks), while the slowest mode may still be far from settled: with
// a per-check decay factor lambda its remaining change is r lambda / (1 -
// lambda), e.g. ~1e-4 for lambda = 0.999 (a wide conduction-dominated
// cavity).  So the rule fires when
//   (a) the largest residual is <= 1e-6 and the last four checks set no new
//       minimum (the floor, not a slow decay, which keeps setting minima), and
//   (b) the slowest mode, extrapolated from the decade of decay just above
//       the floor (lambda from the last checks at 100x and at 10x the floor
//       value before the floor was reached), has fallen to a remaining
//       relative change of kFloorDist since the floor was reached (the first
//       check within 2x of the lowest residual: noise keeps setting slightly
//       lower minima, which must not restart the count).
// A run that shows no decade of decay above the floor (one that starts
// within 10x of it, such as a start from a nearly steady field) gives no
// measure of its slow mode; the rule then waits for lam_min, the per-check
// decay factor of the cavity's slowest diffusive mode (lf_slow_mode; 0: no
// wait).  A measured decay is kept as it is: at high Ra convection makes
// the slow modes decay many times faster than diffusion alone would (the
// 512^2 cavity at Ra 1e6: ~2e-5 per step measured, 2.3e-6 diffusive).
// h: the largest of the three residuals at each check, oldest first.
#include <math.h>
#include <vector>
static constexpr double kFloorDist = 2e-6;

// Per-check (K steps) decay factor of the slowest diffusive mode of an
// nx x ny cavity: the temperature mode of the lowest wavenumber its walls
// allow (pi / L between two fixed-temperature walls, pi / 2L with one, none
// along a direction without one) at rate alpha k^2, or the velocity mode of
// no-slip walls at rate nu pi^2 (1 / nx^2 + 1 / ny^2) (no wavenumber along a
// periodic direction), whichever decays more slowly.  tfix: W, E, S, N.
static inline double lf_slow_mode(double alpha, double nu, int nx, int ny, const int tfix[4],
                                  int xper, int yper, int K) {
  const double pi2 = 9.869604401089358;
  const double lx = (double)nx * nx, ly = (double)ny * ny;
  auto kk = [&](int a, int b, double l2) {
    return (a && b) ? pi2 / l2 : (a || b) ? 0.25 * pi2 / l2 : 0.0;
  };
  const double kt = (xper ? 0.0 : kk(tfix[0], tfix[1], lx)) + (yper ? 0.0 : kk(tfix[2], tfix[3], ly));
  const double kv = (xper ? 0.0 : pi2 / lx) + (yper ? 0.0 : pi2 / ly);
  double rate = nu * kv;
  if (kt > 0.0 && alpha * kt < rate) rate = alpha * kt;
  return rate > 0.0 ? exp(-(double)K * rate) : 0.0;
}

static inline bool lf_at_floor(const std::vector<double>& h, double lam_min = 0.0) {
  const size_t n = h.size();
  if (n < 6 || h[n - 1] > 1e-6) return false;
  size_t m = 0;  // the lowest residual so far
  for (size_t k = 1; k < n; ++k)
    if (h[k] < h[m]) m = k;
  if (m + 4 >= n) return false;
  const double fl = h[m];
  size_t m0 = 0;  // the floor was reached
  while (h[m0] > 2.0 * fl) ++m0;
  // the decade of decay above the floor: last check before m0 at >= 10x the
  // floor value, and the last check before that at >= 100x (or the first)
  size_t k2 = m0, k1 = 0;
  for (size_t k = m0; k-- > 0;)
    if (h[k] >= 10.0 * fl) {
      k2 = k;
      break;
    }
  double lam = 0.0;  // no decade above the floor: no measured slow mode
  if (k2 != m0) {
    for (size_t k = k2; k-- > 0;)
      if (h[k] >= 100.0 * fl) {
        k1 = k;
        break;
      }
    if (k1 != k2) lam = pow(h[k2] / h[k1], 1.0 / (double)(k2 - k1));
  }
  if (!(lam > 0.0)) lam = lam_min;
  if (!(lam > 0.0)) return true;  // no slow mode to wait for
  if (!(lam < 1.0 - 1e-6)) lam = 1.0 - 1e-6;
  const double rest = h[m0] * lam / (1.0 - lam);  // remaining change when the floor was reached
  if (rest <= kFloorDist) return true;
  const double need = log(kFloorDist / rest) / log(lam);  // further checks
  return (double)(n - 1 - m0) >= need;
}

