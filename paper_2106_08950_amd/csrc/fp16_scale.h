// fp16_scale.h -- host side: the automatic storage scale of FP16 populations.
#pragma once

#include <algorithm>
#include <cmath>

namespace dilbm {

// FP16 storage keeps g_i 2^k with g_i = S (f_i - w_i rho0).  The automatic choice is the
// largest k at which every equilibrium state with 0 < rho <= 2 rho0 and |u| <= 0.5 (the
// speeds a step accepts as stable) is stored at no more than half of FP16's largest
// finite value, 65504; the other half is headroom for the non-equilibrium part.  Over
// that range |g_i^eq| = S w_i |rho h_i - rho0| with h_i = 1 + 3 c.u + 4.5 (c.u)^2 -
// 1.5 u.u (the equilibrium of Eq. (2) over w_i rho) is largest at rho = 2 rho0 with u
// along c_i and |u| = 0.5, so c.u = |c_i| / 2; for the rest direction it is S w_0 rho0
// (at rest, or as rho -> 0).  A power-of-two scale changes no relative precision in
// FP16's normal range: larger k only keep the smallest deviations out of the subnormals.
// sw[n]: S w_i of the directions with |c_i|^2 = n, for n = 0 .. nmax.
inline int auto_fp16_scale_log2(const double *sw, int nmax, double rho0) {
  double m = sw[0];
  for (int n = 1; n <= nmax; ++n) {
    const double cu = 0.5 * std::sqrt((double)n);
    const double h = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * 0.25;
    m = std::max(m, sw[n] * (2.0 * h - 1.0));
  }
  const int k = (int)std::floor(std::log2(0.5 * 65504.0 / (m * rho0)));
  return std::min(24, std::max(0, k));
}

}  // namespace dilbm
