// Dawson integral F(x) = exp(-x^2) int_0^x exp(t^2) dt in double precision.
//
// F solves F' = 1 - 2 x F, F(0) = 0.  Differentiating m times gives
// F^(m+1) = -2 x F^(m) - 2 m F^(m-1), so the Taylor coefficients
// c_m = F^(m)(x0)/m! about a node x0 obey
//   c_0 = F(x0), c_1 = 1 - 2 x0 c_0, c_{m+1} = (-2 x0 c_m - 2 c_{m-1})/(m+1).
// Node values F(n h), h = 1/16, n = 0..160, are produced on the host by
// marching this series from F(0) = 0 in long double (the ODE is stable
// forward: its homogeneous solution exp(-x^2) decays).  On the device,
// |x| < 10 uses the series about the nearest node (|x - x0| <= 1/32, 24
// terms); |x| >= 10 uses the asymptotic series
//   F(x) = 1/(2x) sum_n (2n-1)!! / (2 x^2)^n,
// whose 16th term is below 1e-18 at x = 10.
#pragma once
#include <hip/hip_runtime.h>

namespace m1 {

constexpr int kDawsonNodes = 161;           // x = 0 .. 10 step 1/16
constexpr double kDawsonStep = 1.0 / 16.0;
constexpr double kDawsonXMax = 10.0;

__host__ __device__ inline double dawson(double x, const double* nodes) {
  double ax = x < 0 ? -x : x;
  double r;
  if (ax < kDawsonXMax) {
    int n = (int)(ax * 16.0 + 0.5);
    double x0 = n * kDawsonStep;
    double d = ax - x0;
    double cm1 = nodes[n];
    double cm = 1.0 - 2.0 * x0 * cm1;
    double sum = cm1 + cm * d;
    double dp = d;
    for (int m = 1; m < 24; ++m) {
      double cn = (-2.0 * x0 * cm - 2.0 * cm1) / (m + 1);
      dp *= d;
      sum += cn * dp;
      cm1 = cm;
      cm = cn;
    }
    r = sum;
  } else {
    double u = 1.0 / (2.0 * ax * ax);
    double t = 1.0, s = 1.0;
    for (int n = 1; n < 16; ++n) {
      t *= (2 * n - 1) * u;
      s += t;
    }
    r = s / (2.0 * ax);
  }
  return x < 0 ? -r : r;
}

// Host: node table by marching the Taylor series in long double.
inline void dawson_nodes_host(double* out) {
  long double F = 0.0L;
  out[0] = 0.0;
  const long double h = 1.0L / 16.0L;
  for (int n = 1; n < kDawsonNodes; ++n) {
    long double x0 = (n - 1) * h;
    long double cm1 = F, cm = 1.0L - 2.0L * x0 * F;
    long double sum = cm1 + cm * h, hp = h;
    for (int m = 1; m < 60; ++m) {
      long double cn = (-2.0L * x0 * cm - 2.0L * cm1) / (m + 1);
      hp *= h;
      sum += cn * hp;
      cm1 = cm;
      cm = cn;
    }
    F = sum;
    out[n] = (double)F;
  }
}

}  // namespace m1
