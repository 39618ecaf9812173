// Special functions of the Green's function generation, written for the device and
// compiled for the host as well (FM_HD), so that the CPU tests can check these exact
// routines against library implementations.
#pragma once
#include <cmath>

#if defined(__HIPCC__)
#define FM_HD __host__ __device__
#else
#define FM_HD
#endif

namespace fm {

// K_nu(x) for nu = 0, 1 from K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt: the
// trapezoidal rule on this doubly-exponentially decaying analytic integrand converges
// geometrically (step 0.1 gives full double precision for the x used here); for large
// x the asymptotic expansion sqrt(pi/2x) e^-x sum_k a_k(nu) / x^k is used instead.
FM_HD inline double bessel_k(int nu, double x) {
  if (x >= 25.0) {
    const double mu = 4.0 * nu * nu;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k <= 30; ++k) {
      term *= (mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (k * 8.0 * x);
      sum += term;
      if (std::fabs(term) < 1e-17 * std::fabs(sum)) break;
    }
    return std::sqrt(3.14159265358979323846 / (2.0 * x)) * std::exp(-x) * sum;
  }
  const double h = 0.1;
  // terms scaled by exp(x) to avoid underflow for larger x
  double sum = 0.5;  // t = 0: exp(-x (cosh 0 - 1)) cosh(0) = 1, half weight
  for (int j = 1; j < 2000; ++j) {
    const double tj = j * h;
    const double ch = std::cosh(tj);
    const double ex = x * (ch - 1.0);
    if (ex > 45.0 + tj) break;
    sum += std::exp(-ex) * (nu ? ch : 1.0);
  }
  return h * sum * std::exp(-x);
}

// Si(x) = int_0^x sin(t) / t dt for x >= 0.  Below 4 the Taylor series
// sum_n (-1)^n x^(2n+1) / ((2n+1) (2n+1)!) (terms stay below 2, so no digits are lost to
// cancellation); from 4 on Si(x) = pi/2 + Im E1(i x), with E1(z) = e^{-z} / (z + 1 -
// 1/(z + 3 - 4/(z + 5 - ...))) evaluated by the modified Lentz method (the continued
// fraction converges quickly for |z| >= 4).
FM_HD inline double sine_integral(double x) {
  const double pi = 3.14159265358979323846;
  if (x < 4.0) {
    const double x2 = x * x;
    double term = x, sum = x;  // term = (-1)^n x^(2n+1) / (2n+1)!
    for (int n = 1; n < 40; ++n) {
      term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
      const double add = term / (2.0 * n + 1.0);
      sum += add;
      if (std::fabs(add) < 1e-18 * std::fabs(sum)) break;
    }
    return sum;
  }
  // continued fraction for e^{z} E1(z), z = i x: b_0 = z + 1, a_j = -j^2, b_j = z + 2j + 1
  const double tiny = 1e-300;
  double br = 1.0, bi = x;          // b_0
  double fr = br, fi = bi;          // f = b_0
  double cr = fr, ci = fi, dr = 0.0, di = 0.0;
  for (int j = 1; j < 100000; ++j) {
    const double a = -(double)j * (double)j;
    br += 2.0;                       // b_j = 2j + 1 + i x
    // d = 1 / (b + a d)
    double tr = br + a * dr, ti = bi + a * di;
    if (std::fabs(tr) + std::fabs(ti) < tiny) tr = tiny;
    double den = tr * tr + ti * ti;
    dr = tr / den;
    di = -ti / den;
    // c = b + a / c
    den = cr * cr + ci * ci;
    cr = br + a * cr / den;
    ci = bi - a * ci / den;
    if (std::fabs(cr) + std::fabs(ci) < tiny) cr = tiny;
    const double er = cr * dr - ci * di, ei = cr * di + ci * dr;  // delta = c d
    const double nr = fr * er - fi * ei, ni = fr * ei + fi * er;
    fr = nr;
    fi = ni;
    if (std::fabs(er - 1.0) + std::fabs(ei) < 1e-16) break;
  }
  // E1(i x) = e^{-i x} / f
  const double den = fr * fr + fi * fi;
  const double qr = fr / den, qi = -fi / den;  // 1 / f
  const double sn = std::sin(x), cs = std::cos(x);
  const double im = -sn * qr + cs * qi;        // Im[(cos x - i sin x)(qr + i qi)]
  return 0.5 * pi + im;
}

// exp(-x) I_n(x) for n = 0 .. count - 1 into row: the power series (x < 1), Miller's
// backward recurrence normalised by exp(x) = I_0 + 2 sum_k I_k (moderate x), or the
// large-argument expansion (x >= 40 (n_max^2 + 10)).
FM_HD inline void scaled_bessel_row(double x, int count, double* row) {
  const int nmax = count - 1;
  if (x < 1.0) {
    // e^{-x} (x/2)^n sum_j (x^2/4)^j / (j! (n + j)!)
    const double q = 0.25 * x * x, ex = std::exp(-x);
    double lead = 1.0;  // (x/2)^n / n!
    for (int n = 0; n <= nmax; ++n) {
      if (n > 0) lead *= 0.5 * x / n;
      double term = 1.0, sum = 1.0;
      for (int j = 1; j < 40; ++j) {
        term *= q / (j * (double)(n + j));
        sum += term;
        if (term < 1e-18 * sum) break;
      }
      row[n] = ex * lead * sum;
    }
    return;
  }
  if (x >= 40.0 * ((double)nmax * nmax + 10.0)) {
    const double pre = 1.0 / std::sqrt(2.0 * 3.14159265358979323846 * x);
    for (int n = 0; n <= nmax; ++n) {
      const double mu = 4.0 * (double)n * n;
      double term = 1.0, sum = 1.0;
      for (int k = 1; k < 12; ++k) {
        term *= -(mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (k * 8.0 * x);
        sum += term;
      }
      row[n] = pre * sum;
    }
    return;
  }
  // backward recurrence I_{n-1} = I_{n+1} + (2n / x) I_n from far above n_max
  const int n0 = (int)std::sqrt((double)nmax * nmax + 80.0 * x) + 24;
  double ip1 = 0.0, in = 1e-280, norm = 0.0;
  for (int n = n0; n >= 1; --n) {
    const double im1 = ip1 + (2.0 * n / x) * in;
    // in is I_n, im1 is I_{n-1}
    norm += 2.0 * in;
    if (n <= nmax) row[n] = in;
    ip1 = in;
    in = im1;
    if (std::fabs(in) > 1e250) {  // rescale everything held so far
      const double s = 1e-250;
      in *= s;
      ip1 *= s;
      norm *= s;
      for (int m = n; m <= nmax && m <= n0; ++m) row[m] *= s;
    }
  }
  norm += in;  // I_0
  row[0] = in;
  const double inv = 1.0 / norm;
  for (int n = 0; n <= nmax; ++n) row[n] *= inv;
}

}  // namespace fm
