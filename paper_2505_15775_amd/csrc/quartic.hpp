// Exact line search along a direction: the quartic phi(t) = Lbar(R - t G) and
// its minimiser over t >= 0.
#pragma once

#include <math.h>

#include "kernels.hpp"

namespace almbm {

// phi(t) = k0 + k1 t + k2 t^2 + k3 t^3 + k4 t^4
__device__ inline double phi_eval(const double* k, double t) {
  return k[0] + t * (k[1] + t * (k[2] + t * (k[3] + t * k[4])));
}

__device__ inline double polish_cubic(double a, double b, double c, double d, double t) {
  for (int it = 0; it < 3; ++it) {
    const double f = ((a * t + b) * t + c) * t + d;
    const double fp = (3.0 * a * t + 2.0 * b) * t + c;
    if (fp == 0.0) break;
    const double tn = t - f / fp;
    if (!isfinite(tn)) break;
    t = tn;
  }
  return t;
}

// Real roots of a t^3 + b t^2 + c t + d (a != 0) by the depressed-cubic
// closed forms (Cardano for one real root, the trigonometric form for three),
// each refined by Newton steps on the original cubic.
__device__ inline int cubic_real_roots(double a, double b, double c, double d, double* out) {
  const double B = b / a, Cc = c / a, D = d / a;
  const double p = Cc - B * B / 3.0;
  const double q = 2.0 * B * B * B / 27.0 - B * Cc / 3.0 + D;
  const double disc = q * q / 4.0 + p * p * p / 27.0;
  int nr = 0;
  if (disc > 0.0) {
    const double s = sqrt(disc);
    const double A = -copysign(cbrt(fabs(q) / 2.0 + s), q);
    const double u = (A != 0.0) ? A - p / (3.0 * A) : 0.0;
    out[nr++] = u - B / 3.0;
  } else if (p == 0.0) {
    out[nr++] = -B / 3.0;
  } else {
    const double m = 2.0 * sqrt(-p / 3.0);
    double arg = 3.0 * q / (p * m);
    arg = fmin(1.0, fmax(-1.0, arg));
    const double th = acos(arg) / 3.0;
    for (int k = 0; k < 3; ++k) out[nr++] = m * cos(th - 2.0 * M_PI * k / 3.0) - B / 3.0;
  }
  for (int k = 0; k < nr; ++k) out[k] = polish_cubic(a, b, c, d, out[k]);
  return nr;
}

// argmin over t >= 0 of the quartic with coefficients k (smallest t on ties;
// 0 when phi is unbounded below along t >= 0).
__device__ inline double quartic_argmin(const double* k) {
  const double d3 = 4.0 * k[4], d2 = 3.0 * k[3], d1 = 2.0 * k[2], d0 = k[1];
  double roots[3];
  int nr = 0;
  if (d3 != 0.0) {
    if (d3 < 0.0) return 0.0;
    nr = cubic_real_roots(d3, d2, d1, d0, roots);
  } else if (d2 != 0.0) {
    if (d2 < 0.0) return 0.0;
    const double disc = d1 * d1 - 4.0 * d2 * d0;
    if (disc >= 0.0) {
      const double s = sqrt(disc);
      const double qq = -0.5 * (d1 + copysign(s, d1));
      if (qq != 0.0) {
        roots[nr++] = qq / d2;
        roots[nr++] = d0 / qq;
      } else {
        roots[nr++] = 0.0;
      }
    }
  } else if (d1 != 0.0) {
    if (d1 < 0.0) return 0.0;
    roots[nr++] = -d0 / d1;
  } else {
    return 0.0;
  }
  // sort ascending (at most three)
  for (int a = 0; a < nr; ++a)
    for (int b2 = a + 1; b2 < nr; ++b2)
      if (roots[b2] < roots[a]) {
        const double tmp = roots[a];
        roots[a] = roots[b2];
        roots[b2] = tmp;
      }
  double best_t = 0.0, best_v = phi_eval(k, 0.0);
  for (int a = 0; a < nr; ++a) {
    const double t = roots[a];
    if (!(t > 0.0)) continue;
    const double v = phi_eval(k, t);
    if (v < best_v) {
      best_t = t;
      best_v = v;
    }
  }
  return best_t;
}

// Quartic coefficients from the totals (tot[P_C0] must already include any -jJ part).
__device__ inline void quartic_coeffs(const double* tot, double sigma, double* k) {
  const double c0 = tot[P_C0], c1 = 2.0 * tot[P_GP], c2 = tot[P_C2];
  k[0] = c0 + tot[P_YBMA] + 0.5 * sigma * tot[P_EE];
  k[1] = -c1 + tot[P_YA1] - sigma * tot[P_EA1];
  k[2] = c2 - tot[P_YA2] + 0.5 * sigma * (tot[P_A1A1] + 2.0 * tot[P_EA2]);
  k[3] = -sigma * tot[P_A1A2];
  k[4] = 0.5 * sigma * tot[P_A2A2];
}

}  // namespace almbm
