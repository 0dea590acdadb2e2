// Host-side float64 tables and constants (spectrum normalisation, twiddles, windows).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace pin {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// 16-point Gauss-Legendre nodes and weights on [-1, 1], by Newton iteration on P_16.
struct GaussLegendre {
  double x[16], w[16];
  GaussLegendre() {
    const int n = 16;
    for (int i = 0; i < n; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        const double dp = n * (z * p0 - p1) / (z * z - 1.0);
        const double dz = p0 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) {
          double q0 = 1.0, q1 = 0.0;
          for (int j = 1; j <= n; ++j) {
            const double q2 = q1;
            q1 = q0;
            q0 = ((2.0 * j - 1.0) * z * q1 - (j - 1.0) * q2) / j;
          }
          const double dq = n * (z * q0 - q1) / (z * z - 1.0);
          x[i] = z;
          w[i] = 2.0 / ((1.0 - z * z) * dq * dq);
          break;
        }
      }
    }
  }
};

}  // namespace

double bbks_transfer(double k, double gamma) {
  const double q = k / gamma;
  const double x = 2.34 * q;
  const double lead = x > 1e-8 ? std::log1p(x) / x : 1.0 - 0.5 * x;
  const double poly = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4);
  return lead * std::pow(poly, -0.25);
}

double tophat_window(double x) {
  if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0 + x * x * x * x / 280.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

double sigma2_tophat_unit(double radius, double gamma, double ns) {
  static const GaussLegendre gl;
  const double a = std::log(1e-7), b = std::log(1e3);
  const int panels = 4000;
  const double h = (b - a) / panels;
  double total = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double mid = a + (p + 0.5) * h;
    double s = 0.0;
    for (int i = 0; i < 16; ++i) {
      const double lnk = mid + 0.5 * h * gl.x[i];
      const double k = std::exp(lnk);
      const double t = bbks_transfer(k, gamma);
      const double w = tophat_window(k * radius);
      s += gl.w[i] * k * k * k * std::pow(k, ns) * t * t * w * w;
    }
    total += 0.5 * h * s;
  }
  return total / (2.0 * kPi * kPi);
}

std::vector<double> tophat_sigma_nodes(double r0, double step, int count, double amplitude, double gamma, double ns) {
  static const GaussLegendre gl;
  const double a = std::log(1e-7), b = std::log(1e3);
  const int panels = 4000;
  const double h = (b - a) / panels;
  std::vector<double> kk((size_t)panels * 16), base((size_t)panels * 16);
  for (int p = 0; p < panels; ++p) {
    const double mid = a + (p + 0.5) * h;
    for (int i = 0; i < 16; ++i) {
      const double k = std::exp(mid + 0.5 * h * gl.x[i]);
      const double t = bbks_transfer(k, gamma);
      kk[(size_t)p * 16 + i] = k;
      base[(size_t)p * 16 + i] = 0.5 * h * gl.w[i] * k * k * k * std::pow(k, ns) * t * t;
    }
  }
  std::vector<double> out((size_t)count);
  auto work = [&](int first, int stride) {
    for (int c = first; c < count; c += stride) {
      const double r = r0 * std::exp(c * step);
      double total = 0.0;
      for (int p = 0; p < panels; ++p) {
        double sp = 0.0;
        for (int i = 0; i < 16; ++i) {
          const double w = tophat_window(kk[(size_t)p * 16 + i] * r);
          sp += base[(size_t)p * 16 + i] * w * w;
        }
        total += sp;
      }
      out[(size_t)c] = std::sqrt(amplitude * total / (2.0 * kPi * kPi));
    }
  };
  const int nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> threads;
  for (int t = 1; t < nt; ++t) threads.emplace_back(work, t, nt);
  work(0, nt);
  for (auto& t : threads) t.join();
  return out;
}

double sigma2_gaussian_unit(double radius, double gamma, double ns) {
  static const GaussLegendre gl;
  const double a = std::log(1e-7), b = std::log(40.0 / radius);
  const int panels = 2000;
  const double h = (b - a) / panels;
  double total = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double mid = a + (p + 0.5) * h;
    double s = 0.0;
    for (int i = 0; i < 16; ++i) {
      const double k = std::exp(mid + 0.5 * h * gl.x[i]);
      const double t = bbks_transfer(k, gamma);
      s += gl.w[i] * k * k * k * std::pow(k, ns) * t * t * std::exp(-(k * radius) * (k * radius));
    }
    total += 0.5 * h * s;
  }
  return total / (2.0 * kPi * kPi);
}

std::vector<double> radius_ladder(int n, double box, double r_max, double r_min, double dex, double gamma,
                                  double ns) {
  const double cell = box / n;
  auto lns2 = [&](double lr) { return std::log(sigma2_gaussian_unit(std::exp(lr) * cell, gamma, ns)); };
  std::vector<double> radii{r_max};
  double cur = lns2(std::log(r_max));
  const double step = dex * std::log(10.0);
  while (true) {
    const double target = cur + step;
    // sigma^2 grows as R shrinks: bracket [lo, hi] in ln R with lns2(lo) >= target > lns2(hi)
    double hi = std::log(radii.back()), lo = hi;
    double flo = cur - target;
    while (flo < 0.0) {
      hi = lo;
      lo -= 0.5;
      if (std::exp(lo) < 1e-3 * r_min) return radii;
      flo = lns2(lo) - target;
    }
    double fhi = lns2(hi) - target;
    // Illinois regula falsi on ln R
    double x = lo;
    for (int it = 0; it < 200 && hi - lo > 1e-14; ++it) {
      x = (lo * fhi - hi * flo) / (fhi - flo);
      const double fx = lns2(x) - target;
      if ((fx >= 0.0) == (flo >= 0.0)) {
        lo = x;
        flo = fx;
        fhi *= 0.5;
      } else {
        hi = x;
        fhi = fx;
        flo *= 0.5;
      }
      if (fx == 0.0) break;
    }
    const double r = std::exp(x);
    if (r < r_min) return radii;
    radii.push_back(r);
    cur = target;
  }
}

GrowthTable growth_table(double om) {
  static const GaussLegendre gl;
  const double ol = 1.0 - om;
  GrowthTable g;
  g.y0 = std::log(1e-3);
  g.h = (std::log(1e6) - g.y0) / (kGrowthNodes - 1);
  g.lambda_over_m = ol / om;
  // I(a) = Int_0^a da' / (a' E)^3 = Int x^(3/2) (om + ol x^3)^(-3/2) dx; in y = ln x the
  // integrand is x^(5/2) (om + ol x^3)^(-3/2)
  auto f = [&](double y) {
    const double x = std::exp(y);
    return std::pow(x, 2.5) * std::pow(om + ol * x * x * x, -1.5);
  };
  auto panel = [&](double y_a, double y_b) {
    double s = 0.0;
    const double mid = 0.5 * (y_a + y_b), half = 0.5 * (y_b - y_a);
    for (int i = 0; i < 16; ++i) s += gl.w[i] * f(mid + half * gl.x[i]);
    return half * s;
  };
  const double ys = std::log(1e-8);
  double I = 0.4 * std::pow(1e-8, 2.5) * std::pow(om, -1.5);   // leading term below a = 1e-8
  // up to the first node, then node by node (four panels per interval)
  const int pre = 4000;
  for (int p = 0; p < pre; ++p) I += panel(ys + (g.y0 - ys) * p / pre, ys + (g.y0 - ys) * (p + 1) / pre);
  auto d_unnorm = [&](double a, double Ia) { return 2.5 * om * std::sqrt(om / (a * a * a) + ol) * Ia; };
  auto dd_unnorm = [&](double a, double Ia) {   // a dD/da
    const double e = std::sqrt(om / (a * a * a) + ol);
    return 2.5 * om * (-1.5 * om / (a * a * a) / e * Ia + e * a * std::pow(a, 1.5) * std::pow(om + ol * a * a * a, -1.5));
  };
  std::vector<double> Iy(kGrowthNodes);
  Iy[0] = I;
  for (int i = 1; i < kGrowthNodes; ++i) {
    const double ya = g.y0 + (i - 1) * g.h;
    for (int q = 0; q < 4; ++q) I += panel(ya + g.h * q / 4, ya + g.h * (q + 1) / 4);
    Iy[i] = I;
  }
  // normalisation at a = 1 (y = 0)
  double I1 = Iy[0];
  const int p1 = 4000;
  for (int p = 0; p < p1; ++p) I1 += panel(g.y0 * (1.0 - (double)p / p1), g.y0 * (1.0 - (double)(p + 1) / p1));
  const double norm = d_unnorm(1.0, I1);
  g.a_per_D = norm;
  g.d.resize(kGrowthNodes);
  g.dd.resize(kGrowthNodes);
  for (int i = 0; i < kGrowthNodes; ++i) {
    const double a = std::exp(g.y0 + i * g.h);
    g.d[i] = d_unnorm(a, Iy[i]) / norm;
    g.dd[i] = dd_unnorm(a, Iy[i]) / norm;
  }
  g.guide_l0 = std::log2(g.d[0]);
  const double hl = (std::log2(g.d[kGrowthNodes - 1]) - g.guide_l0) / (kGrowthGuide - 1);
  g.guide_inv = 1.0 / hl;
  g.guide.resize(kGrowthGuide);
  int node = 0;
  for (int b = 0; b < kGrowthGuide; ++b) {
    const double tb = std::exp2(g.guide_l0 + b * hl);
    while (node + 1 < kGrowthNodes && g.d[node + 1] <= tb) ++node;
    g.guide[b] = node;
  }
  return g;
}

std::vector<double> mode_amplitudes(int n, double box, double amplitude, double gamma, double ns) {
  const int h = n / 2;
  std::vector<double> a((size_t)3 * h * h + 1, 0.0);
  const double norm = amplitude * std::pow((double)n, 6) / (2.0 * box * box * box);
  const double kf = 2.0 * 3.14159265358979323846 / box;
  // the BBKS form of bbks_transfer with its powers as products (this runs when a field is first
  // generated for a box, up to 7.9e5 entries at N = 1024), split over a few threads
  auto fill = [&](size_t lo, size_t hi) {
    for (size_t f2 = lo; f2 < hi; ++f2) {
      const double k = kf * std::sqrt((double)f2);
      const double q = k / gamma;
      const double x = 2.34 * q;
      const double lead = x > 1e-8 ? std::log1p(x) / x : 1.0 - 0.5 * x;
      const double b = 16.1 * q, c = 5.46 * q, d = 6.71 * q;
      const double poly = 1.0 + 3.89 * q + b * b + c * c * c + (d * d) * (d * d);
      const double t = lead / std::sqrt(std::sqrt(poly));
      const double kn = ns == 1.0 ? k : std::pow(k, ns);
      a[f2] = std::sqrt(kn * t * t * norm);
    }
  };
  const size_t total = a.size();
  const size_t workers = total < 65536 ? 1 : 8;
  std::vector<std::thread> pool;
  for (size_t w = 1; w < workers; ++w) pool.emplace_back(fill, 1 + (total - 1) * w / workers, 1 + (total - 1) * (w + 1) / workers);
  fill(1, 1 + (total - 1) / workers);
  for (auto& t : pool) t.join();
  return a;
}

double amplitude_for_sigma8(double sigma8, double gamma, double ns) {
  return sigma8 * sigma8 / sigma2_tophat_unit(8.0, gamma, ns);
}

double eds_sphere_root() {
  auto f = [](double x) { return 1.0 - x / 3.0 - x * x / 21.0 - 23.0 * x * x * x / 1701.0; };
  double lo = 1.0, hi = 3.0;   // f(1) > 0 > f(3)
  for (int i = 0; i < 200; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (f(mid) > 0.0) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

double eds_delta_c() { return 0.15 * std::pow(12.0 * kPi, 2.0 / 3.0); }

void twiddles_into(int n, double* out) {
  for (int m = 0; m < n; ++m) {
    // angle in extended precision, then rounded once to float64
    const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
    out[2 * m] = (double)std::cos(ang);
    out[2 * m + 1] = (double)std::sin(ang);
  }
}

std::vector<double> twiddles(int n) {
  std::vector<double> t(2 * (size_t)n);
  twiddles_into(n, t.data());
  return t;
}

std::vector<double> gaussian_window_table(int n, double radius_cells) {
  std::vector<double> w(n);
  for (int i = 0; i < n; ++i) {
    const double f = i < n / 2 ? i : i - n;
    const double kr = 2.0 * kPi * f * radius_cells / n;
    w[i] = std::exp(-0.5 * kr * kr);
  }
  return w;
}

}  // namespace pin
