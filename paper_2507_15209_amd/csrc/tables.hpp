// tables.hpp -- host-side float64 table generation (see tables.cpp).
#pragma once
#include <vector>

namespace mp3 {

// number of distinct integer |q|^2 values tabulated: 0 .. 3 (N/2)^2
inline int nq2_count(int n) { return 3 * (n / 2) * (n / 2) + 1; }

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void sph_bessel_all(int L, double x, double* out);
// [lmax+1][nq2][nbins]; binning 0 = shell average, 1 = thin shell at the mid
// radius; smoothing > 0 multiplies by the top-hat window 3 j_1(kR) / (kR)
void jbar_table(int n, double box, int lmax, const std::vector<double>& edges, std::vector<double>& out,
                int binning = 0, double smoothing = 0.0);
// spherical top-hat window 3 j_1(x) / x
double tophat_window(double x);
// sinc^8(pi q / n) at every index of an axis (q = index mod n in [-n/2, n/2))
void phi_hat_axis(int n, std::vector<double>& out);
void twiddles(int n, std::vector<double>& re, std::vector<double>& im);
// Daubechies-4 scaling function phi at x = i / 2^level, i = 0 .. 3 2^level (cascade algorithm)
void d4_table(int level, std::vector<double>& out);
// int phi_R(x) phi_R(x - s) dx, s = 0 .. 3, of the table's linear interpolant
void d4_autocorr(const std::vector<double>& table, int level, double a[4]);
// |phi_hat(2 pi q / n)|^2 of the Daubechies-4 scaling function per axis index (infinite product)
void d4_phi_hat_axis(int n, std::vector<double>& out);
// connection coefficients int phi phi(. - s) phi(. - t) of the Daubechies-4 function, g[s + 2][t + 2]
void d4_gamma(double g[5][5]);
// connection coefficients int B3 B3(. - s) B3(. - t) of the cubic B-spline, g[s + 3][t + 3]
void b3_gamma(double g[7][7]);
double ylm_norm(int l, int m);
// centred cubic B-spline
double bspline3(double u);
// 5-point Gauss-Legendre nodes xi_s on [0, 1]: m[s][t] = B3(xi_s + 1 - t), weights wq[s]
void gamma_quadrature(double m[5][4], double wq[5]);

}  // namespace mp3
