// tables.cpp -- float64 window tables generated at plan creation (host side).
//
// * Gauss-Legendre nodes by Newton iteration on P_n (three-term recurrence).
// * Spherical Bessel functions j_0..j_L: upward recurrence from j_0, j_1 when
//   x > L (stable there), Miller's downward recurrence normalised to the larger
//   of the closed forms j_0, j_1 when x <= L, exact values at x = 0.
// * Radial window of the secondary vertices (Sec. 2.2 around Eq.
//   3PCF-multipole-window, times the binning window of each vertex), tabulated
//   for every integer |q|^2 of the grid, k = (2 pi / box) sqrt(|q|^2):
//   the bin average
//     jbar_{l,b}(k) = 3 / (r_{b+1}^3 - r_b^3) int_{r_b}^{r_{b+1}} r^2 j_l(k r) dr
//   (64-point Gauss-Legendre per bin) or the thin shell j_l(k r_b) at the
//   bin's mid radius, optionally times the spherical top-hat window
//   3 j_1(kR) / (kR) of the triple-sphere binning (Sec. 3).
// * Phi-hat per axis: the power spectrum of the cubic B-spline scaling
//   function, sinc^8(pi q / N) (Eq. SFC-3PCF-vertex).
// * FFT twiddles exp(-2 pi i t / N).
// * Normalisation of Y_lm: sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace mp3 {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void sph_bessel_all(int L, double x, double* out) {
  if (x == 0.0) {
    out[0] = 1.0;
    for (int l = 1; l <= L; ++l) out[l] = 0.0;
    return;
  }
  const double s = std::sin(x), c = std::cos(x);
  const double j0 = s / x;
  if (L == 0) {
    out[0] = j0;
    return;
  }
  if (x > (double)L) {
    out[0] = j0;
    out[1] = s / (x * x) - c / x;
    for (int l = 1; l < L; ++l) out[l + 1] = (2.0 * l + 1.0) / x * out[l] - out[l - 1];
    return;
  }
  // Miller: start well above max(L, x) with (0, tiny) and recur downward.
  const int lstart = L + 40 + (int)x;
  double jp1 = 0.0, jl = 1e-280;
  std::vector<double> tmp(L + 1);
  double scale_acc = 1.0;
  for (int l = lstart; l >= 1; --l) {
    double jm1 = (2.0 * l + 1.0) / x * jl - jp1;
    jp1 = jl;
    jl = jm1;
    if (l - 1 <= L) tmp[l - 1] = jl;
    if (std::fabs(jl) > 1e250) {  // rescale to stay in range
      jl *= 1e-250;
      jp1 *= 1e-250;
      for (int k = l - 1; k <= L; ++k) tmp[k] *= 1e-250;
    }
  }
  (void)scale_acc;
  // normalise by whichever of the closed forms j_0, j_1 is larger in
  // magnitude: they never vanish together, so the ratio stays accurate near
  // the zeros of j_0 (x close to n pi)
  const double j1 = s / (x * x) - c / x;
  const double norm = std::fabs(j0) >= std::fabs(j1) ? j0 / tmp[0] : j1 / tmp[1];
  for (int l = 0; l <= L; ++l) out[l] = tmp[l] * norm;
}

double tophat_window(double x) {
  // 3 j_1(x) / x = 3 (sin x - x cos x) / x^3; its series below x = 1e-2
  // (the closed form cancels there)
  if (x < 1e-2) {
    const double x2 = x * x;
    return 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 * x2 * x2 / 15120.0;
  }
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

void jbar_table(int n, double box, int lmax, const std::vector<double>& edges, std::vector<double>& out,
                int binning, double smoothing) {
  const int nbins = (int)edges.size() - 1;
  const int nq2 = nq2_count(n);
  out.assign((size_t)(lmax + 1) * nq2 * nbins, 0.0);
  std::vector<double> xg, wg;
  gauss_legendre(64, xg, wg);
  const double kf = 2.0 * M_PI / box;
  unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int tid) {
    std::vector<double> jl(lmax + 1);
    std::vector<double> acc((size_t)(lmax + 1));
    for (int s = tid; s < nq2; s += (int)nthreads) {
      const double k = kf * std::sqrt((double)s);
      const double wth = smoothing > 0.0 ? tophat_window(k * smoothing) : 1.0;
      for (int b = 0; b < nbins; ++b) {
        const double r1 = edges[b], r2 = edges[b + 1];
        const double half = 0.5 * (r2 - r1), mid = 0.5 * (r2 + r1);
        if (binning == 1) {
          // thin shell at the mid radius
          sph_bessel_all(lmax, k * mid, jl.data());
          for (int l = 0; l <= lmax; ++l) out[((size_t)l * nq2 + s) * nbins + b] = jl[l] * wth;
          continue;
        }
        std::fill(acc.begin(), acc.end(), 0.0);
        for (size_t g = 0; g < xg.size(); ++g) {
          const double r = mid + half * xg[g];
          sph_bessel_all(lmax, k * r, jl.data());
          const double wr = half * wg[g] * r * r;
          for (int l = 0; l <= lmax; ++l) acc[l] += wr * jl[l];
        }
        const double vol = 3.0 / (r2 * r2 * r2 - r1 * r1 * r1);
        for (int l = 0; l <= lmax; ++l) out[((size_t)l * nq2 + s) * nbins + b] = acc[l] * vol * wth;
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nthreads; ++t) th.emplace_back(work, (int)t);
  for (auto& t : th) t.join();
}

void twiddles(int n, std::vector<double>& re, std::vector<double>& im) {
  re.resize(n);
  im.resize(n);
  for (int t = 0; t < n; ++t) {
    // exact values at the quarter points keep the table symmetric
    const double a = -2.0 * M_PI * (double)t / (double)n;
    re[t] = std::cos(a);
    im[t] = std::sin(a);
    if (4 * t == n) { re[t] = 0.0; im[t] = -1.0; }
    if (2 * t == n) { re[t] = -1.0; im[t] = 0.0; }
    if (4 * t == 3 * n) { re[t] = 0.0; im[t] = 1.0; }
  }
}

void phi_hat_axis(int n, std::vector<double>& out) {
  // |B3hat|^2 per axis: B3 is the fourfold self-convolution of the unit box,
  // whose transform at theta = 2 pi q / n is sinc(theta / 2)
  out.resize(n);
  for (int i = 0; i < n; ++i) {
    const int q = i < n / 2 ? i : i - n;
    const double h = M_PI * (double)q / (double)n;
    const double sc = q == 0 ? 1.0 : std::sin(h) / h;
    const double s2 = sc * sc, s4 = s2 * s2;
    out[i] = s4 * s4;
  }
}

// Daubechies-4 scaling function: four orthonormal filter taps, support [0, 3]
namespace {
void d4_filter(double h[4]) {
  const double s = std::sqrt(3.0), d = 4.0 * std::sqrt(2.0);
  h[0] = (1.0 + s) / d;
  h[1] = (3.0 + s) / d;
  h[2] = (3.0 - s) / d;
  h[3] = (1.0 - s) / d;
}
}  // namespace

void d4_table(int level, std::vector<double>& out) {
  double h[4];
  d4_filter(h);
  const double r2 = std::sqrt(2.0);
  // at the integers (phi(0) = phi(3) = 0) the two-scale relation
  // phi(x) = sqrt2 sum_j h_j phi(2x - j) reads phi(1) = sqrt2 (h1 phi(1) + h0 phi(2)),
  // which fixes phi(2) / phi(1); partition of unity fixes phi(1) + phi(2) = 1
  const double ratio = (1.0 - r2 * h[1]) / (r2 * h[0]);
  const double p1 = 1.0 / (1.0 + ratio);
  std::vector<double> cur = {0.0, p1, ratio * p1, 0.0};
  // each level doubles the resolution: even points are known, odd points
  // follow from the relation at the previous level
  for (int r = 1; r <= level; ++r) {
    const int half = 1 << (r - 1);
    std::vector<double> nxt(3 * (1 << r) + 1, 0.0);
    for (size_t i = 0; i < cur.size(); ++i) nxt[2 * i] = cur[i];
    for (int i = 1; i < (int)nxt.size(); i += 2) {
      double acc = 0.0;
      for (int j = 0; j < 4; ++j) {
        const int idx = i - j * half;
        if (idx >= 0 && idx < (int)cur.size()) acc += h[j] * cur[idx];
      }
      nxt[i] = r2 * acc;
    }
    cur.swap(nxt);
  }
  out.swap(cur);
}

void d4_autocorr(const std::vector<double>& t, int level, double a[4]) {
  // int phi_R(x) phi_R(x - s) dx of the piecewise-linear interpolant: on each
  // interval of width h both factors are linear, integrated exactly
  const double h = std::ldexp(1.0, -level);
  const int per = 1 << level;
  for (int s = 0; s < 4; ++s) {
    const int sh = s * per;
    double acc = 0.0;
    for (int i = sh; i + 1 < (int)t.size(); ++i) {
      const double a0 = t[i], a1 = t[i + 1], b0 = t[i - sh], b1 = t[i + 1 - sh];
      acc += 2.0 * a0 * b0 + a0 * b1 + a1 * b0 + 2.0 * a1 * b1;
    }
    a[s] = acc * h / 6.0;
  }
}

void d4_phi_hat_axis(int n, std::vector<double>& out) {
  // |phi_hat(w)|^2 = prod_{j >= 1} |m0(w / 2^j)|^2 with m0(w) = 2^-1/2 sum_k h_k e^{-i k w},
  // at w = 2 pi q / n; 64 factors (the last ones are 1 to double precision)
  double h[4];
  d4_filter(h);
  out.resize(n);
  for (int i = 0; i < n; ++i) {
    const int q = i < n / 2 ? i : i - n;
    const double w = 2.0 * M_PI * (double)q / (double)n;
    double prod = 1.0;
    for (int j = 1; j <= 64; ++j) {
      const double xi = std::ldexp(w, -j);
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 4; ++k) {
        re += h[k] * std::cos(k * xi);
        im -= h[k] * std::sin(k * xi);
      }
      prod *= 0.5 * (re * re + im * im);
    }
    out[i] = prod;
  }
}

void d4_gamma(double g[5][5]) {
  // gamma(s, t) = int phi(x) phi(x - s) phi(x - t) dx over the 19 pairs with
  // |s|, |t|, |s - t| <= 2.  Inserting the two-scale relation in all three
  // factors gives gamma(s, t) = sqrt2 sum_{k,l,m} h_k h_l h_m
  // gamma(2s + l - k, 2t + m - k): a homogeneous system, made unique by
  // sum_{s,t} gamma(s, t) = int phi = 1 (partition of unity).  Solved by
  // Gaussian elimination with partial pivoting, the normalisation replacing
  // the first equation.
  double h[4];
  d4_filter(h);
  const double r2 = std::sqrt(2.0);
  int idx[5][5];
  int np = 0;
  for (int s = -2; s <= 2; ++s)
    for (int t = -2; t <= 2; ++t) idx[s + 2][t + 2] = std::abs(s - t) <= 2 ? np++ : -1;
  std::vector<double> A((size_t)np * (np + 1), 0.0);   // augmented [np][np + 1]
  auto at = [&](int r, int c) -> double& { return A[(size_t)r * (np + 1) + c]; };
  for (int s = -2; s <= 2; ++s) {
    for (int t = -2; t <= 2; ++t) {
      const int r = idx[s + 2][t + 2];
      if (r < 0) continue;
      at(r, r) -= 1.0;
      for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
          for (int m = 0; m < 4; ++m) {
            const int u = 2 * s + l - k, v = 2 * t + m - k;
            if (u < -2 || u > 2 || v < -2 || v > 2 || idx[u + 2][v + 2] < 0) continue;
            at(r, idx[u + 2][v + 2]) += r2 * h[k] * h[l] * h[m];
          }
    }
  }
  for (int c = 0; c <= np; ++c) at(0, c) = 1.0;   // sum of all unknowns = 1
  for (int c = 0; c < np; ++c) {
    int piv = c;
    for (int r = c + 1; r < np; ++r)
      if (std::fabs(at(r, c)) > std::fabs(at(piv, c))) piv = r;
    if (piv != c)
      for (int k = 0; k <= np; ++k) std::swap(at(c, k), at(piv, k));
    for (int r = 0; r < np; ++r) {
      if (r == c) continue;
      const double f = at(r, c) / at(c, c);
      if (f != 0.0)
        for (int k = c; k <= np; ++k) at(r, k) -= f * at(c, k);
    }
  }
  for (int s = 0; s < 5; ++s)
    for (int t = 0; t < 5; ++t) g[s][t] = idx[s][t] < 0 ? 0.0 : at(idx[s][t], np) / at(idx[s][t], idx[s][t]);
}

void b3_gamma(double g[7][7]) {
  // gamma(s, t) = int B3(u) B3(u - s) B3(u - t) du: on each unit interval of
  // B3's support the integrand is a polynomial of degree 9, integrated exactly
  // by 5-point Gauss-Legendre
  std::vector<double> x, w;
  gauss_legendre(5, x, w);
  for (int s = -3; s <= 3; ++s) {
    for (int t = -3; t <= 3; ++t) {
      double acc = 0.0;
      for (int j = -2; j < 2; ++j) {
        for (int q = 0; q < 5; ++q) {
          const double u = j + 0.5 * (x[q] + 1.0);
          acc += 0.5 * w[q] * bspline3(u) * bspline3(u - s) * bspline3(u - t);
        }
      }
      g[s + 3][t + 3] = acc;
    }
  }
}

double bspline3(double u) {
  const double a = std::fabs(u);
  if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
  if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
  return 0.0;
}

void gamma_quadrature(double m[5][4], double wq[5]) {
  std::vector<double> x, w;
  gauss_legendre(5, x, w);
  for (int s = 0; s < 5; ++s) {
    const double xi = 0.5 * (x[s] + 1.0);
    wq[s] = 0.5 * w[s];
    for (int t = 0; t < 4; ++t) m[s][t] = bspline3(xi + 1.0 - t);
  }
}

double ylm_norm(int l, int m) {
  // sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) by a running product
  double r = 1.0;
  for (int k = l - m + 1; k <= l + m; ++k) r /= (double)k;
  return std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * r);
}

}  // namespace mp3
