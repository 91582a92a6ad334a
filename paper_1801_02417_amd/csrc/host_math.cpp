// Host-side tables of the measurement operator and the SARA dictionary, in FP64.
//
// * Daubechies low-pass filters by spectral factorisation (the wavelet bases of the
//   SARA dictionary, Sec. 3.1): P(y) = sum_{k<p} C(p-1+k, k) y^k is factored, each root y
//   gives z with y = (2 - z - 1/z)/4 and the root inside the unit circle is kept
//   (minimum phase); h(z) ~ (1+z)^p prod (z - z_k), normalised to sum h = sqrt(2), and
//   stored with the highest power of z first.
// * Kaiser-Bessel interpolation kernel of the gridding matrix G and the scaling of the
//   zero-padding operator Z (Sec. 4.1, eq. meas_op): psi(t) = I0(beta sqrt(1-(2t/T)^2)) /
//   I0(beta), its Fourier transform psi_hat in closed form, beta from Beatty, Nishimura &
//   Pauly (2005).  I0 is summed from its power series (Abramowitz & Stegun 9.6.10).
// * Per-tap Chebyshev expansions of psi over the unit interval each tap's argument spans,
//   evaluated on the device.
#include <cmath>
#include <complex>
#include <vector>

#include "psara.h"

namespace psara {

using cd = std::complex<double>;

static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Roots of sum_k c[k] x^k (c[deg] != 0) by the Weierstrass (Durand-Kerner) iteration,
// polished with Newton steps on the original polynomial.
static std::vector<cd> poly_roots(const std::vector<double>& c) {
  const int deg = (int)c.size() - 1;
  std::vector<cd> z(deg);
  if (deg < 1) return z;
  auto eval = [&](cd x) {
    cd v = c[deg];
    for (int k = deg - 1; k >= 0; --k) v = v * x + c[k];
    return v;
  };
  auto deval = [&](cd x) {
    cd v = c[deg] * double(deg);
    for (int k = deg - 1; k >= 1; --k) v = v * x + c[k] * double(k);
    return v;
  };
  const cd seed(0.4, 0.9);
  double rad = 1.0;
  for (int k = 0; k <= deg; ++k) rad = std::max(rad, std::abs(c[k] / c[deg]));
  cd p = 1.0;
  for (int i = 0; i < deg; ++i) { z[i] = p * rad; p *= seed; }
  for (int it = 0; it < 2000; ++it) {
    double change = 0.0;
    for (int i = 0; i < deg; ++i) {
      cd den = c[deg];
      for (int j = 0; j < deg; ++j) if (j != i) den *= (z[i] - z[j]);
      cd dz = eval(z[i]) / den;
      z[i] -= dz;
      change = std::max(change, std::abs(dz) / std::max(1.0, std::abs(z[i])));
    }
    if (change < 1e-17) break;
  }
  for (int i = 0; i < deg; ++i)
    for (int it = 0; it < 4; ++it) {
      cd d = deval(z[i]);
      if (std::abs(d) == 0.0) break;
      z[i] -= eval(z[i]) / d;
    }
  return z;
}

std::vector<double> daubechies(int p) {
  std::vector<double> P(p);
  for (int k = 0; k < p; ++k) P[k] = binom(p - 1 + k, k);
  std::vector<cd> yr = poly_roots(P);
  // polynomial in z, ascending powers, start with (1 + z)^p
  std::vector<cd> poly(p + 1);
  for (int k = 0; k <= p; ++k) poly[k] = binom(p, k);
  for (cd y : yr) {
    cd b = 2.0 - 4.0 * y;
    cd s = std::sqrt(b * b - 4.0);
    cd z1 = 0.5 * (b + s), z2 = 0.5 * (b - s);
    cd zk = std::abs(z1) < 1.0 ? z1 : z2;
    std::vector<cd> nxt(poly.size() + 1, cd(0.0));
    for (size_t k = 0; k < poly.size(); ++k) {   // multiply by (z - zk)
      nxt[k + 1] += poly[k];
      nxt[k] -= zk * poly[k];
    }
    poly.swap(nxt);
  }
  const int F = 2 * p;
  std::vector<double> h(F);
  double sum = 0.0;
  for (int j = 0; j < F; ++j) { h[j] = poly[F - 1 - j].real(); sum += h[j]; }
  const double scale = std::sqrt(2.0) / sum;
  for (double& v : h) v *= scale;
  return h;
}

double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / (double(k) * double(k));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

double kb_beta(int taps, double alpha) {
  const double a = taps / alpha * (alpha - 0.5);
  return M_PI * std::sqrt(a * a - 0.8);
}

double kb_value(int taps, double beta, double t) {
  const double u = 1.0 - (2.0 * t / taps) * (2.0 * t / taps);
  if (u < 0.0) return 0.0;
  return bessel_i0(beta * std::sqrt(u)) / bessel_i0(beta);
}

double kb_hat(int taps, double beta, double nu) {
  const double z2 = beta * beta - (M_PI * taps * nu) * (M_PI * taps * nu);
  double r;
  if (z2 > 1e-24) { double z = std::sqrt(z2); r = std::sinh(z) / z; }
  else if (z2 < -1e-24) { double z = std::sqrt(-z2); r = std::sin(z) / z; }
  else r = 1.0;
  return taps / bessel_i0(beta) * r;
}

// Per-tap polynomial of the Kaiser-Bessel kernel: c[i][k] (k = 0..deg, ascending powers) with
// psi(f - i) ~= sum_k c[i][k] u^k, u = 2f - T + 1 in (-1, 1] for f in (T/2 - 1, T/2].  The
// polynomial interpolates at the deg+1 Chebyshev nodes of [-1, 1] (near-minimax on a unit
// interval of the smooth kernel) and is then rewritten in the monomial basis for Horner
// evaluation; on a single unit interval the coefficients stay small, so Horner's rule loses
// nothing measurable against the Chebyshev form (max error about one rounding of the
// evaluation precision for degree 9 in FP32 and 16 in FP64).
std::vector<double> kb_poly(int taps, double beta, int deg) {
  const int nn = deg + 1;
  std::vector<double> c(size_t(taps) * nn, 0.0);
  // monomial coefficients of T_0 .. T_deg by T_{k+1} = 2u T_k - T_{k-1}
  std::vector<std::vector<double>> tp(nn, std::vector<double>(nn, 0.0));
  tp[0][0] = 1.0;
  if (deg >= 1) tp[1][1] = 1.0;
  for (int k = 1; k < deg; ++k)
    for (int p = 0; p <= k + 1; ++p)
      tp[k + 1][p] = (p > 0 ? 2.0 * tp[k][p - 1] : 0.0) - tp[k - 1][p];
  for (int i = 0; i < taps; ++i) {
    std::vector<double> fv(nn);
    for (int j = 0; j < nn; ++j) {
      const double u = std::cos(M_PI * (j + 0.5) / nn);
      const double f = 0.5 * (u + taps - 1);     // u = 2f - T + 1
      fv[j] = kb_value(taps, beta, f - i);
    }
    for (int k = 0; k < nn; ++k) {
      double s = 0.0;
      for (int j = 0; j < nn; ++j) s += fv[j] * std::cos(M_PI * k * (j + 0.5) / nn);
      const double ck = (k == 0 ? 1.0 : 2.0) * s / nn;
      for (int p = 0; p <= k; ++p) c[size_t(i) * nn + p] += ck * tp[k][p];
    }
  }
  return c;
}

}  // namespace psara

extern "C" int psara_wavelet_filter(int p, double* h) {
  if (p < 1 || p > 8 || !h) return 0;
  std::vector<double> v = psara::daubechies(p);
  for (int j = 0; j < 2 * p; ++j) h[j] = v[j];
  return 2 * p;
}

extern "C" double psara_kb_beta(int taps, double alpha) { return psara::kb_beta(taps, alpha); }
extern "C" double psara_kb_value(int taps, double beta, double t) { return psara::kb_value(taps, beta, t); }
extern "C" double psara_kb_deapod(int taps, double beta, double nu) { return 1.0 / psara::kb_hat(taps, beta, nu); }
