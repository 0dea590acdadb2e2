// Host-side float64 tables and constants of a plan.
#pragma once

#include <stdint.h>

#include <vector>

namespace pin {

// BBKS transfer function T(k/gamma) and k^ns T^2 (unit amplitude); k in h/Mpc.
double bbks_transfer(double k, double gamma);
// Fourier transform of a unit top-hat, 3 (sin x - x cos x)/x^3.
double tophat_window(double x);
// sigma^2(R) = 1/(2 pi^2) Int k^2 P(k) W_TH(kR)^2 dk for P = k^ns T^2 (unit amplitude), by
// composite 16-point Gauss-Legendre quadrature in ln k over [1e-7, 1e3] h/Mpc.
double sigma2_tophat_unit(double radius, double gamma, double ns);
// sigma(R_k) = sqrt(amplitude * sigma2_tophat_unit(R_k)) at R_k = r0 exp(k step) Mpc/h, k < count
// (the same quadrature, with the radius-independent part of the integrand evaluated once and the
// nodes spread over host threads).
std::vector<double> tophat_sigma_nodes(double r0, double step, int count, double amplitude, double gamma, double ns);
// sigma^2(R) with the Gaussian window, 1/(2 pi^2) Int k^2 P(k) exp(-k^2 R^2) dk (unit amplitude).
double sigma2_gaussian_unit(double radius, double gamma, double ns);
// Radii in cells, largest first from r_max, each with sigma^2 10^dex times the previous one's
// (Gaussian window, box/n Mpc/h per cell), while >= r_min.
std::vector<double> radius_ladder(int n, double box, double r_max, double r_min, double dex, double gamma,
                                  double ns);
// Growing mode of flat LambdaCDM (no radiation), normalised to D(a = 1) = 1, tabulated on
// y = ln a at kGrowthNodes nodes from ln 1e-3 to ln 1e6: D and dD/dy at each node, and
// a_per_D = lim_{a->0} a / D (= the unnormalised D at a = 1).  guide[b] is the last node with
// D <= 2^(guide_l0 + b / guide_inv), kGrowthGuide buckets uniform in log2 D over the table: a
// value's bucket brackets its node interval, so the search for it takes a few steps.
constexpr int kGrowthNodes = 8192;
constexpr int kGrowthGuide = 4096;
struct GrowthTable {
  double y0 = 0, h = 0, a_per_D = 0, lambda_over_m = 0;
  std::vector<double> d, dd;
  std::vector<int32_t> guide;
  double guide_l0 = 0, guide_inv = 0;
};
GrowthTable growth_table(double omega_m);
// Amplitude A with sigma^2(8 Mpc/h) = sigma8^2.
double amplitude_for_sigma8(double sigma8, double gamma, double ns);
// Mode amplitudes of an N^3 field in a box of side L: entry f2 = fx^2 + fy^2 + fz^2 (integer
// frequencies, 0 <= f2 <= 3 (N/2)^2) holds sqrt(P(k) norm), k = (2 pi / L) sqrt(f2), P the BBKS
// spectrum of amplitude A, norm = N^6 / (2 L^3); entry 0 is 0.
std::vector<double> mode_amplitudes(int n, double box, double amplitude, double gamma, double ns);
// Root of the 3rd-order EdS sphere series 1 - x/3 - x^2/21 - 23 x^3/1701 (bisection), and the
// EdS linear collapse threshold (3/20)(12 pi)^(2/3).
double eds_sphere_root();
double eds_delta_c();
// exp(2 pi i m/N), m < N, interleaved (re, im)
std::vector<double> twiddles(int n);
// The same table written to out[2n] (no allocation).
void twiddles_into(int n, double* out);
// exp(-(2 pi f(i) R/N)^2 / 2) for i < N, f(i) the integer frequency of index i
std::vector<double> gaussian_window_table(int n, double radius_cells);

}  // namespace pin
