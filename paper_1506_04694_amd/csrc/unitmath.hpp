// FP64 logarithm and sine/cosine of pi x for the arguments Box-Muller draws:
// u = (k + 1/2) 2^-32 in (0, 1) and x = 2 u in (0, 2).  No special cases
// (zero, negative, subnormal, infinite or NaN arguments never occur), so each
// is a short range reduction plus one polynomial, about a third of the
// general library functions' instructions.  Both are built from the
// mathematics, with errors of a few units in the last place (checked against
// 60-digit references by the CPU tests):
//
//  * log_unit: u = m 2^e with m in [sqrt(1/2), sqrt(2)); with f = m - 1 and
//    s = f / (2 + f), log m = 2 atanh s = 2 s (1 + s^2/3 + s^4/5 + ...);
//    |s| <= 3 - 2 sqrt(2) < 0.172, so the terms up to s^20/21 leave a
//    truncation below 3e-17 relative.
//  * sincospi_unit: x = q/2 + r with q = round(2x) and |r| <= 1/4 (exact, x is
//    a multiple of 2^-31), the Taylor series of sin(pi r) and cos(pi r) in r
//    (|pi r| <= pi/4: terms to r^17 and r^18 leave below 6e-17 relative), and
//    the quadrant q mod 4 picks signs and swaps.
//
// The functions are plain C++ on doubles (host and device), so the CPU tests
// compile this header as it is.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define MLMC_HD __host__ __device__
#else
#define MLMC_HD
#endif

namespace mlmc {

MLMC_HD inline double log_unit(double u) {
  int e;
  double m = frexp(u, &e);  // u = m 2^e, m in [1/2, 1)
  if (m < 0.7071067811865476) {
    m += m;
    e -= 1;
  }
  const double f = m - 1.0;  // exact: m and 1 are within a factor of 2
  const double s = f / (2.0 + f);
  const double z = s * s;
  // 1 + z/3 + z^2/5 + ... + z^10/21 (coefficients 1 / (2k + 1))
  double p = 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  const double lm = (s + s) + (s + s) * (z * p);  // 2 s (1 + z p)
  return (double)e * 0.6931471805599453 + lm;     // e ln 2 + log m
}

// sin(pi x) and cos(pi x) for x in [0, 2].
MLMC_HD inline void sincospi_unit(double x, double* sp, double* cp) {
  const double q = rint(x + x);
  const double r = x - 0.5 * q;  // exact, |r| <= 1/4
  const double z = r * r;
  // Taylor coefficients (-1)^k pi^(2k+1) / (2k+1)! and (-1)^k pi^(2k) / (2k)!,
  // rounded to double
  double ps = 7.952054001475513e-07;
  ps = ps * z - 2.1915353447830217e-05;
  ps = ps * z + 0.00046630280576761255;
  ps = ps * z - 0.0073704309457143504;
  ps = ps * z + 0.08214588661112823;
  ps = ps * z - 0.5992645293207921;
  ps = ps * z + 2.5501640398773455;
  ps = ps * z - 5.16771278004997;
  ps = ps * z + 3.141592653589793;
  const double sr = r * ps;
  double pc = -1.3878952462213771e-07;
  pc = pc * z + 4.303069587032947e-06;
  pc = pc * z - 0.0001046381049248457;
  pc = pc * z + 0.0019295743094039231;
  pc = pc * z - 0.02580689139001406;
  pc = pc * z + 0.2353306303588932;
  pc = pc * z - 1.3352627688545895;
  pc = pc * z + 4.0587121264167685;
  pc = pc * z - 4.934802200544679;
  const double cr = 1.0 + z * pc;
  // pi x = q pi/2 + pi r
  const int k = (int)q & 3;
  const double s = (k & 1) ? cr : sr;
  const double c = (k & 1) ? sr : cr;
  *sp = (k & 2) ? -s : s;
  *cp = ((k + 1) & 2) ? -c : c;
}

}  // namespace mlmc
