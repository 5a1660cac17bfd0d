// Host-side FP64 tables of the estimator: the truncated cubic
// Battle-Lemarie (BL3) tap polynomials, its window and alias sum per axis,
// FFT twiddles and the |n|^2 -> bin lookup table.
//
// BL3 (third-order orthogonalised Battle-Lemarie scaling function, used for
// assignment in Sec. 2.4.1) is read as the cubic-spline member of the family:
// phi(x) = sum_n c_n beta3(x - n), where beta3 is the centred cubic B-spline
// and c_n are the Fourier coefficients of A(w)^(-1/2),
// A(w) = (2416 + 2382 cos w + 240 cos 2w + 2 cos 3w) / 5040, the alias sum of
// |beta3_hat|^2.  phi is a cubic on every unit interval, so each of the six
// taps j = -2..3 of a particle at fraction f carries a cubic weight
// w_j(f) = phi(j - f).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace mps {
namespace {

constexpr int kFilterHalf = 64;       // c_n, |n| <= 64 (|c_64| ~ 1e-19)
constexpr int kTrapezoid = 2048;      // periodic trapezoid rule, exponentially exact

double autocorr7(double w) {
  return (2416.0 + 2382.0 * std::cos(w) + 240.0 * std::cos(2.0 * w) +
          2.0 * std::cos(3.0 * w)) / 5040.0;
}

// c_n = (1/2pi) int_0^{2pi} A(w)^(-1/2) cos(n w) dw by the trapezoid rule.
std::vector<double> filter_coefficients() {
  std::vector<double> c(kFilterHalf + 1, 0.0);
  for (int k = 0; k < kTrapezoid; ++k) {
    const double w = 2.0 * M_PI * k / kTrapezoid;
    const double g = 1.0 / std::sqrt(autocorr7(w));
    for (int n = 0; n <= kFilterHalf; ++n) c[n] += g * std::cos(n * w);
  }
  for (double& v : c) v /= kTrapezoid;
  return c;
}

double cn(const std::vector<double>& c, int n) {
  n = n < 0 ? -n : n;
  return n <= kFilterHalf ? c[n] : 0.0;
}

// Cubic of phi on [m, m+1] in t = x - m: coefficients of 1, t, t^2, t^3.
// On that interval only beta3(x - n) with n = m-1..m+2 are non-zero; their
// pieces are (1-t)^3/6, 2/3 - t^2 + t^3/2, 1/6 + t/2 + t^2/2 - t^3/2, t^3/6.
void piece(const std::vector<double>& c, int m, double out[4]) {
  static const double basis[4][4] = {
      {1.0 / 6, -0.5, 0.5, -1.0 / 6},
      {2.0 / 3, 0.0, -1.0, 0.5},
      {1.0 / 6, 0.5, 0.5, -0.5},
      {0.0, 0.0, 0.0, 1.0 / 6}};
  for (int p = 0; p < 4; ++p) out[p] = 0.0;
  for (int i = 0; i < 4; ++i) {
    const double ci = cn(c, m - 1 + i);
    for (int p = 0; p < 4; ++p) out[p] += ci * basis[i][p];
  }
}

double horner(const double a[4], double t) {
  return ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
}

// 16-point Gauss-Legendre nodes/weights on [0, 1] via Newton on P_16.
void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
  x->resize(n);
  w->resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    (*x)[i] = 0.5 * (1.0 - z);
    (*w)[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 0.5 * 2/((1-z^2) P'^2)
  }
}

struct Pieces {
  double a[6][4];  // intervals m = -3..2
};

Pieces bl3_pieces() {
  const std::vector<double> c = filter_coefficients();
  Pieces p;
  for (int m = -3; m <= 2; ++m) piece(c, m, p.a[m + 3]);
  return p;
}

}  // namespace

TapPoly bl3_tap_polynomials() {
  const Pieces pc = bl3_pieces();
  TapPoly tp{};
  // tap j covers d = j - f in (j-1, j]: interval m = j-1 with t = 1 - f.
  // Substitute t = 1 - f: sum_p a_p (1 - f)^p.
  static const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
  for (int j = 0; j < kTaps; ++j) {
    const double* a = pc.a[j];  // j index 0 <-> tap -2 <-> interval -3
    for (int q = 0; q < 4; ++q) tp.c[j][q] = 0.0;
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q <= p; ++q)
        tp.c[j][q] += a[p] * binom[p][q] * ((q & 1) ? -1.0 : 1.0);
  }
  return tp;
}

TapBound tap_bounds(const TapPoly& tp, int n_taps) {
  TapBound b;
  for (int j = 0; j < kTaps; ++j) b.k[j] = 0.f;
  for (int j = 0; j < n_taps; ++j) {
    const double* c = tp.c[j];
    double m = 0.0;
    if (c[4] == 0.0 && c[5] == 0.0) {
      // a cubic: |w_j| on [0, 1] peaks at an end or where
      // w_j' = c1 + 2 c2 f + 3 c3 f^2 vanishes
      double cand[4] = {0.0, 1.0, -1.0, -1.0};
      const double qa = 3.0 * c[3], qb = 2.0 * c[2], qc = c[1];
      if (qa != 0.0) {
        const double disc = qb * qb - 4.0 * qa * qc;
        if (disc >= 0.0) {
          const double r = std::sqrt(disc);
          cand[2] = (-qb + r) / (2.0 * qa);
          cand[3] = (-qb - r) / (2.0 * qa);
        }
      } else if (qb != 0.0) {
        cand[2] = -qc / qb;
      }
      for (double f : cand) {
        if (f < 0.0 || f > 1.0) continue;
        m = std::max(m, std::fabs(((c[3] * f + c[2]) * f + c[1]) * f + c[0]));
      }
    } else {
      // higher degree: samples every 1/4096 plus the largest possible change
      // between samples, sum_k k |c_k| / 8192
      constexpr int kSamples = 4096;
      for (int i = 0; i <= kSamples; ++i) {
        const double f = static_cast<double>(i) / kSamples;
        double v = 0.0;
        for (int q = kPolyCoef - 1; q >= 0; --q) v = v * f + c[q];
        m = std::max(m, std::fabs(v));
      }
      double slope = 0.0;
      for (int q = 1; q < kPolyCoef; ++q) slope += q * std::fabs(c[q]);
      m += slope * 0.5 / kSamples;
    }
    // margin for the FP32 evaluation of the taps on the device
    b.k[j] = static_cast<float>(m * 1.0001);
  }
  return b;
}

namespace {

// Centred B-spline of degree n by the Cox-de Boor recursion
//   beta_n(x) = ((x + (n+1)/2) beta_{n-1}(x + 1/2) + ((n+1)/2 - x) beta_{n-1}(x - 1/2)) / n,
// beta_0 = 1 on (-1/2, 1/2].
long double bspline(int n, long double x) {
  if (n == 0) return (x > -0.5L && x <= 0.5L) ? 1.0L : 0.0L;
  const long double h = 0.5L * (n + 1);
  return ((x + h) * bspline(n - 1, x + 0.5L) + (h - x) * bspline(n - 1, x - 0.5L)) / n;
}

}  // namespace

TapPoly bspline_tap_polynomials(int order) {
  // tap t = 0..p-1 is node c + j, j = t - (p-1)/2; with the particle at
  // c + f - s (s = 1/2 for odd p) its weight is beta_{p-1}(j - f + s), one
  // polynomial of degree p - 1 in f on (0, 1): fitted through p interior
  // points in long double
  TapPoly tp{};
  const int d = order - 1;
  const int lo = -((order - 1) / 2);
  const long double s = (order & 1) ? 0.5L : 0.0L;
  for (int t = 0; t < order; ++t) {
    long double a[kPolyCoef][kPolyCoef + 1] = {};
    for (int k = 0; k <= d; ++k) {
      const long double f = (k + 0.5L) / (d + 1);
      long double pw = 1.0L;
      for (int q = 0; q <= d; ++q) {
        a[k][q] = pw;
        pw *= f;
      }
      a[k][d + 1] = bspline(d, (lo + t) - f + s);
    }
    // Gauss-Jordan elimination with partial pivoting
    for (int col = 0; col <= d; ++col) {
      int piv = col;
      for (int r = col + 1; r <= d; ++r)
        if (std::fabs(static_cast<double>(a[r][col])) > std::fabs(static_cast<double>(a[piv][col]))) piv = r;
      for (int q = 0; q <= d + 1; ++q) std::swap(a[col][q], a[piv][q]);
      for (int r = 0; r <= d; ++r) {
        if (r == col) continue;
        const long double g = a[r][col] / a[col][col];
        for (int q = col; q <= d + 1; ++q) a[r][q] -= g * a[col][q];
      }
    }
    for (int q = 0; q <= d; ++q) tp.c[t][q] = static_cast<double>(a[q][d + 1] / a[q][q]);
  }
  return tp;
}

void bspline_axis_tables(int n_grid, int order, std::vector<double>* inv_win2, std::vector<double>* alias) {
  const int half = n_grid / 2;
  inv_win2->assign(half + 1, 1.0);
  alias->assign(half + 1, 1.0);
  // sum_J sinc^(2p)((w + 2 pi J)/2) = sum_m beta_{2p-1}(m) cos(m w) (Poisson)
  std::vector<double> bm(order, 0.0);
  for (int m = 0; m < order; ++m) bm[m] = static_cast<double>(bspline(2 * order - 1, m));
  for (int n = 0; n <= half; ++n) {
    const double w = 2.0 * M_PI * n / n_grid;
    const double h = 0.5 * w;
    const double sinc = n == 0 ? 1.0 : std::sin(h) / h;
    double s2p = 1.0;
    for (int k = 0; k < 2 * order; ++k) s2p *= sinc;
    (*inv_win2)[n] = 1.0 / s2p;
    double c = bm[0];
    for (int m = 1; m < order; ++m) c += 2.0 * bm[m] * std::cos(m * w);
    (*alias)[n] = c;
  }
}

void bl3_axis_tables(int n_grid, std::vector<double>* win2, std::vector<double>* alias) {
  const Pieces pc = bl3_pieces();
  std::vector<double> gx, gw;
  gauss_legendre(16, &gx, &gw);
  // truncated autocorrelation a_s = int phi_t(x) phi_t(x + s) dx, s = 0..5
  double a[6];
  for (int s = 0; s < 6; ++s) {
    double acc = 0.0;
    for (int m = -3; m + s <= 2; ++m)
      for (size_t i = 0; i < gx.size(); ++i)
        acc += gw[i] * horner(pc.a[m + 3], gx[i]) * horner(pc.a[m + s + 3], gx[i]);
    a[s] = acc;
  }
  const int half = n_grid / 2;
  win2->assign(half + 1, 0.0);
  alias->assign(half + 1, 0.0);
  for (int n = 0; n <= half; ++n) {
    const double w = 2.0 * M_PI * n / n_grid;
    double wt = 0.0;
    for (int m = -3; m <= 2; ++m)
      for (size_t i = 0; i < gx.size(); ++i)
        wt += gw[i] * horner(pc.a[m + 3], gx[i]) * std::cos(w * (m + gx[i]));
    (*win2)[n] = wt * wt;
    double cs = a[0];
    for (int s = 1; s < 6; ++s) cs += 2.0 * a[s] * std::cos(s * w);
    (*alias)[n] = cs;
  }
}

// ------------------------------------------------ quadratic-spline reading
// phi(x) = sum_n c_n beta2(x - n), c_n the Fourier coefficients of
// A2(w)^(-1/2), A2(w) = (66 + 52 cos w + 2 cos 2w) / 120 (the alias sum of
// |beta2_hat|^2).  With s = x - m in [-1/2, 1/2] only n = m - 1, m, m + 1
// contribute: phi = c_m (3/4 - s^2) + c_{m-1} (1/2 - s)^2 / 2
// + c_{m+1} (1/2 + s)^2 / 2.
namespace {

constexpr int kFilterHalf2 = 48;  // |c_48| ~ 3e-18

std::vector<double> filter_coefficients2() {
  std::vector<double> c(kFilterHalf2 + 1, 0.0);
  for (int k = 0; k < kTrapezoid; ++k) {
    const double w = 2.0 * M_PI * k / kTrapezoid;
    const double g = 1.0 / std::sqrt((66.0 + 52.0 * std::cos(w) + 2.0 * std::cos(2.0 * w)) / 120.0);
    for (int n = 0; n <= kFilterHalf2; ++n) c[n] += g * std::cos(n * w);
  }
  for (double& v : c) v /= kTrapezoid;
  return c;
}

double cn2(const std::vector<double>& c, int n) {
  n = n < 0 ? -n : n;
  return n <= kFilterHalf2 ? c[n] : 0.0;
}

// phi on [m - 1/2, m + 1/2] as a quadratic in s = x - m: coefficients of
// 1, s, s^2.
void piece2(const std::vector<double>& c, int m, double out[3]) {
  const double a = cn2(c, m - 1), b = cn2(c, m), d = cn2(c, m + 1);
  out[0] = 0.75 * b + 0.125 * a + 0.125 * d;
  out[1] = -0.5 * a + 0.5 * d;
  out[2] = -b + 0.5 * a + 0.5 * d;
}

double phi2(const std::vector<double>& c, double x) {
  const int m = static_cast<int>(std::floor(x + 0.5));
  double a[3];
  piece2(c, m, a);
  const double s = x - m;
  return (a[2] * s + a[1]) * s + a[0];
}

}  // namespace

TapPoly bl3q_tap_polynomials() {
  const std::vector<double> c = filter_coefficients2();
  TapPoly tp{};
  for (int t = 0; t < kTaps; ++t) {
    const int j = t + kTapLo;
    double a[3];
    // f < 1/2: x = j - f lies in [j - 1/2, j], s = -f
    piece2(c, j, a);
    tp.c[t][0] = a[0];
    tp.c[t][1] = -a[1];
    tp.c[t][2] = a[2];
    // f >= 1/2: x = j - f lies in (j - 1, j - 1/2], s = 1 - f
    piece2(c, j - 1, a);
    tp.c[t][3] = a[0] + a[1] + a[2];
    tp.c[t][4] = -a[1] - 2.0 * a[2];
    tp.c[t][5] = a[2];
  }
  return tp;
}

TapBound bl3q_tap_bounds(const TapPoly& tp) {
  TapBound b;
  for (int j = 0; j < kTaps; ++j) {
    double m = 0.0;
    for (int h = 0; h < 2; ++h) {
      const double* q = tp.c[j] + 3 * h;
      const double lo = 0.5 * h, hi = 0.5 * h + 0.5;
      double cand[3] = {lo, hi, -1.0};
      if (q[2] != 0.0) cand[2] = -q[1] / (2.0 * q[2]);
      for (double f : cand) {
        if (f < lo || f > hi) continue;
        m = std::max(m, std::fabs((q[2] * f + q[1]) * f + q[0]));
      }
    }
    b.k[j] = static_cast<float>(m * 1.0001);
  }
  return b;
}

void bl3q_axis_tables(int n_grid, std::vector<double>* win2, std::vector<double>* alias) {
  const std::vector<double> c = filter_coefficients2();
  std::vector<double> gx, gw;
  gauss_legendre(16, &gx, &gw);
  // phi_t on (-3, 3] integrated over the half-unit pieces [h/2 - 3, h/2 - 5/2]
  auto integrate = [&](auto&& f, double lo, double hi) {
    double acc = 0.0;
    const int pieces = static_cast<int>(std::lround(2.0 * (hi - lo)));
    for (int i = 0; i < pieces; ++i)
      for (size_t k = 0; k < gx.size(); ++k) acc += 0.5 * gw[k] * f(lo + 0.5 * (i + gx[k]));
    return acc;
  };
  double a[6];
  for (int s = 0; s < 6; ++s)
    a[s] = integrate([&](double x) { return phi2(c, x) * phi2(c, x + s); }, -3.0, 3.0 - s);
  const int half = n_grid / 2;
  win2->assign(half + 1, 0.0);
  alias->assign(half + 1, 0.0);
  for (int n = 0; n <= half; ++n) {
    const double w = 2.0 * M_PI * n / n_grid;
    const double wt = integrate([&](double x) { return phi2(c, x) * std::cos(w * x); }, -3.0, 3.0);
    (*win2)[n] = wt * wt;
    double cs = a[0];
    for (int s = 1; s < 6; ++s) cs += 2.0 * a[s] * std::cos(s * w);
    (*alias)[n] = cs;
  }
}

std::vector<double> twiddles(int n_grid) {
  std::vector<double> t(2 * n_grid);
  for (int m = 0; m < n_grid; ++m) {
    const double ang = 2.0 * M_PI * m / n_grid;
    t[2 * m] = std::cos(ang);
    t[2 * m + 1] = -std::sin(ang);
  }
  return t;
}

bool bin_lut(int n_grid, double box, int n_bins, const double* k_edges,
             std::vector<int32_t>* lut, std::vector<double>* edges_out) {
  const int64_t half = n_grid / 2;
  const int64_t h2 = half * half;
  const double kf = 2.0 * M_PI / box;
  const double k_nyq = kf * static_cast<double>(half);
  lut->assign(static_cast<size_t>(h2), -1);
  edges_out->assign(n_bins + 1, 0.0);
  if (k_edges == nullptr) {
    const int64_t nb2 = static_cast<int64_t>(n_bins) * n_bins;
    for (int64_t n2 = 1; n2 < h2; ++n2) {
      const int64_t scaled = nb2 * n2;
      int64_t b = static_cast<int64_t>(std::floor(std::sqrt(static_cast<double>(scaled)) /
                                                  static_cast<double>(half)));
      while (b > 0 && (b * half) * (b * half) > scaled) --b;
      while (((b + 1) * half) * ((b + 1) * half) <= scaled) ++b;
      (*lut)[n2] = b < n_bins ? static_cast<int32_t>(b) : -1;
    }
    for (int b = 0; b <= n_bins; ++b) (*edges_out)[b] = k_nyq * b / n_bins;
    return true;
  }
  for (int b = 0; b <= n_bins; ++b) {
    if (!std::isfinite(k_edges[b]) || k_edges[b] < 0.0) return false;
    if (b > 0 && !(k_edges[b] > k_edges[b - 1])) return false;
  }
  if (k_edges[n_bins] > k_nyq * (1.0 + 1e-12)) return false;
  std::vector<double> t(n_bins + 1);
  for (int b = 0; b <= n_bins; ++b) {
    const double r = k_edges[b] / kf;
    t[b] = r * r;
    (*edges_out)[b] = k_edges[b];
  }
  for (int64_t n2 = 1; n2 < h2; ++n2) {
    const double x = static_cast<double>(n2);
    int b = -1;
    while (b + 1 <= n_bins && t[b + 1] <= x) ++b;  // count of t_b <= x, minus 1
    (*lut)[n2] = (b >= 0 && b < n_bins) ? b : -1;
  }
  return true;
}

}  // namespace mps
