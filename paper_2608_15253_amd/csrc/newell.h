// Cell-averaged demagnetisation tensor in FP64 (device code).
//
// N_ab(R) = (1/V) int_cell int_cell G_ab(x - x') with the point-dipole kernel
// G_ab(r) = (delta_ab r^2 - 3 r_a r_b) / (4 pi r^5) (Newell, Williams & Dunlop
// 1993; the paper convolves with this tensor).  Near the source (scaled
// Chebyshev distance d <= 2) the closed form -- second differences over the 27
// corner offsets of Newell's functions f and g -- is evaluated directly.
// Beyond, where that form loses digits to cancellation, the equivalent
// triangle-weighted single integral int G(R + s) prod_a (D_a - |s_a|) ds / V
// is taken by tensor-product Gauss-Legendre quadrature split at s_a = 0, with
// n nodes per half interval: 10 (d < 5), 8 (d < 10), 6 (d < 40), 4 (d < 200),
// 3 beyond.  d = floor(max_a |o_a| D_a / max_a D_a).
#pragma once
#include "common.h"

namespace mmx {

struct GaussRules {      // nodes/weights on [-1, 1] for n = 3, 4, 6, 8, 10
  double x[5][10];
  double w[5][10];
};

__device__ inline double nw_asinh_ratio(double num, double den) {
  return den != 0.0 ? asinh(num / den) : 0.0;
}
__device__ inline double nw_atan_ratio(double num, double den) {
  return den != 0.0 ? atan(num / den) : 0.0;
}

__device__ inline double newell_f(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double t = 0.5 * y * (z2 - x2) * nw_asinh_ratio(y, sqrt(x2 + z2));
  t += 0.5 * z * (y2 - x2) * nw_asinh_ratio(z, sqrt(x2 + y2));
  t -= x * y * z * nw_atan_ratio(y * z, x * R);
  t += (2.0 * x2 - y2 - z2) * R / 6.0;
  return t;
}

__device__ inline double newell_g(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double t = x * y * z * nw_asinh_ratio(z, sqrt(x2 + y2));
  t += y / 6.0 * (3.0 * z2 - y2) * nw_asinh_ratio(x, sqrt(y2 + z2));
  t += x / 6.0 * (3.0 * z2 - x2) * nw_asinh_ratio(y, sqrt(x2 + z2));
  t -= z2 * z / 6.0 * nw_atan_ratio(x * y, z * R);
  t -= z * y2 / 2.0 * nw_atan_ratio(x * z, y * R);
  t -= z * x2 / 2.0 * nw_atan_ratio(y * z, x * R);
  t -= x * y * R / 3.0;
  return t;
}

template <bool G>
__device__ inline double second_difference(double X, double Y, double Z, double dx, double dy,
                                           double dz) {
  double acc = 0.0;
  for (int ex = -1; ex <= 1; ++ex)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ez = -1; ez <= 1; ++ez) {
        const double w = (ex == 0 ? 2.0 : -1.0) * (ey == 0 ? 2.0 : -1.0) * (ez == 0 ? 2.0 : -1.0);
        const double a = X + ex * dx, b = Y + ey * dy, c = Z + ez * dz;
        acc += w * (G ? newell_g(a, b, c) : newell_f(a, b, c));
      }
  return acc;
}

// out: xx, yy, zz, xy, xz, yz
__device__ inline void tensor_closed_form(double X, double Y, double Z, double dx, double dy,
                                          double dz, double out[6]) {
  const double pref = 1.0 / (4.0 * kPi * dx * dy * dz);
  out[0] = pref * second_difference<false>(X, Y, Z, dx, dy, dz);
  out[1] = pref * second_difference<false>(Y, X, Z, dy, dx, dz);
  out[2] = pref * second_difference<false>(Z, Y, X, dz, dy, dx);
  out[3] = pref * second_difference<true>(X, Y, Z, dx, dy, dz);
  out[4] = pref * second_difference<true>(X, Z, Y, dx, dz, dy);
  out[5] = pref * second_difference<true>(Y, Z, X, dy, dz, dx);
}

__device__ inline void tensor_quadrature(double X, double Y, double Z, double dx, double dy,
                                         double dz, int rule, int n, const GaussRules& g,
                                         double out[6]) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const double h[3] = {dx, dy, dz};
  // node s and weight (GL weight * half length * (h - |s|)) of node k on axis a
  auto node = [&](int a, int k, double& s, double& w) {
    const int i = k % n;
    const double sp = 0.5 * h[a] * (1.0 + g.x[rule][i]);
    s = (k < n) ? -sp : sp;
    w = 0.5 * h[a] * g.w[rule][i] * (h[a] - sp);
  };
  for (int i = 0; i < 2 * n; ++i) {
    double sx, wx;
    node(0, i, sx, wx);
    const double rx = X + sx;
    for (int j = 0; j < 2 * n; ++j) {
      double sy, wy;
      node(1, j, sy, wy);
      const double ry = Y + sy;
      const double wxy = wx * wy;
      for (int k = 0; k < 2 * n; ++k) {
        double sz, wz;
        node(2, k, sz, wz);
        const double rz = Z + sz;
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double inv = wxy * wz / (4.0 * kPi * r2 * r2 * sqrt(r2));
        acc[0] += (r2 - 3.0 * rx * rx) * inv;
        acc[1] += (r2 - 3.0 * ry * ry) * inv;
        acc[2] += (r2 - 3.0 * rz * rz) * inv;
        acc[3] -= 3.0 * rx * ry * inv;
        acc[4] -= 3.0 * rx * rz * inv;
        acc[5] -= 3.0 * ry * rz * inv;
      }
    }
  }
  const double iv = 1.0 / (dx * dy * dz);
  for (int c = 0; c < 6; ++c) out[c] = acc[c] * iv;
}

// Tensor at integer cell offset (ox, oy, oz), two-zone rule; adds w * N to acc.
__device__ inline void tensor_add(long ox, long oy, long oz, double dx, double dy, double dz,
                                  const GaussRules& g, double w, double acc[6]) {
  const double hmax = fmax(dx, fmax(dy, dz));
  const double rho = fmax(fabs((double)ox) * dx, fmax(fabs((double)oy) * dy,
                                                      fabs((double)oz) * dz)) / hmax;
  const long d = (long)floor(rho + 1e-9);
  double t[6];
  if (d <= 2) {
    tensor_closed_form(ox * dx, oy * dy, oz * dz, dx, dy, dz, t);
  } else {
    int rule, n;
    if (d < 5) { rule = 4; n = 10; }
    else if (d < 10) { rule = 3; n = 8; }
    else if (d < 40) { rule = 2; n = 6; }
    else if (d < 200) { rule = 1; n = 4; }
    else { rule = 0; n = 3; }
    tensor_quadrature(ox * dx, oy * dy, oz * dz, dx, dy, dz, rule, n, g, t);
  }
  for (int c = 0; c < 6; ++c) acc[c] += w * t[c];
}

}  // namespace mmx
