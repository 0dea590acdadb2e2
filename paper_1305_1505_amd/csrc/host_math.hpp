// Host-side float64 tables and constants of a plan.
#pragma once

#include <vector>

namespace pin {

// BBKS transfer function T(k/gamma) and k^ns T^2 (unit amplitude); k in h/Mpc.
double bbks_transfer(double k, double gamma);
// Fourier transform of a unit top-hat, 3 (sin x - x cos x)/x^3.
double tophat_window(double x);
// sigma^2(R) = 1/(2 pi^2) Int k^2 P(k) W_TH(kR)^2 dk for P = k^ns T^2 (unit amplitude), by
// composite 16-point Gauss-Legendre quadrature in ln k over [1e-7, 1e3] h/Mpc.
double sigma2_tophat_unit(double radius, double gamma, double ns);
// Amplitude A with sigma^2(8 Mpc/h) = sigma8^2.
double amplitude_for_sigma8(double sigma8, double gamma, double ns);
// Root of the 3rd-order EdS sphere series 1 - x/3 - x^2/21 - 23 x^3/1701 (bisection), and the
// EdS linear collapse threshold (3/20)(12 pi)^(2/3).
double eds_sphere_root();
double eds_delta_c();
// exp(2 pi i m/N), m < N, interleaved (re, im)
std::vector<double> twiddles(int n);
// exp(-(2 pi f(i) R/N)^2 / 2) for i < N, f(i) the integer frequency of index i
std::vector<double> gaussian_window_table(int n, double radius_cells);

}  // namespace pin
