// Compile-time trigonometry for FFT twiddle factors.
//
// cis_cos(e, n) and cis_sin(e, n) return cos and sin of 2*pi*e/n in double precision. The angle
// is reduced exactly in rational arithmetic to an octant (8e/n = q + r/n), so the Taylor series
// only ever sees |t| <= pi/4, where 14 terms are far below double rounding. Everything is
// constexpr so that the HIP kernels get the twiddles as immediate constants; the header has no
// HIP dependency so a host compiler can check it against the C library.
#pragma once

namespace hpm {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

// Octant reduction of 2*pi*e/n: 8e = q n + r with 0 <= r < n, t = (pi/4) r/n.
struct CosSin {
  double c, s;
};

constexpr CosSin cis(long e, long n) {
  e %= n;
  if (e < 0) e += n;
  const long q = (8 * e) / n;
  const long r = 8 * e - q * n;
  const double t = (kPi / 4.0) * (double(r) / double(n));
  const double u = (kPi / 4.0) * (double(n - r) / double(n));  // pi/4 - t, exactly reduced
  const double st = taylor_sin(t), ct = taylor_cos(t);
  const double su = taylor_sin(u), cu = taylor_cos(u);
  switch (q) {
    case 0: return {ct, st};
    case 1: return {su, cu};
    case 2: return {-st, ct};
    case 3: return {-cu, su};
    case 4: return {-ct, -st};
    case 5: return {-su, -cu};
    case 6: return {st, -ct};
    default: return {cu, -su};
  }
}

constexpr double cis_cos(long e, long n) { return cis(e, n).c; }
constexpr double cis_sin(long e, long n) { return cis(e, n).s; }

}  // namespace hpm
