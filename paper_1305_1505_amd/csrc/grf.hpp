// Gaussian linear density field (eq. deltal): one thread per half-spectrum mode.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) -- ten rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// with the key bumped by the Weyl increments between rounds.  Counter = mode index
// (i*N + j)*(N/2+1) + l as (low, high) words, c2 = c3 = 0; key = seed as (low, high) words.
// Uniforms u = (2*(w >> 12) + 1) * 2^-53 from w = c1:c0 and c3:c2; Box-Muller in float64.
// Spectrum: P(k) = A k^ns T(k/Gamma)^2 with the BBKS transfer function
//   T(q) = ln(1 + 2.34 q)/(2.34 q) [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3 + (6.71 q)^4]^(-1/4),
// and dk = sqrt(P(k) N^6 / (2 L^3)) (g1 + i g2), the amplitude read from the plan's table by
// f^2 (computed on the host in float64 from the formula above).  On the l = 0 plane the member of each
// (f, -f) pair with the larger i*N + j is drawn, its partner is the conjugate; k = 0 and all
// Nyquist modes are zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace pin {

struct PhiloxOut {
  uint32_t c0, c1, c2, c3;
};

__device__ __forceinline__ PhiloxOut philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                   uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return PhiloxOut{c0, c1, c2, c3};
}

__device__ __forceinline__ double uniform_from_words(uint32_t lo, uint32_t hi) {
  const uint64_t w = ((uint64_t)hi << 32) | lo;
  return (2.0 * (double)(w >> 12) + 1.0) * 0x1.0p-53;
}

struct GrfArgs {
  uint64_t seed;
  // sqrt(P(k) A N^6 / (2 L^3)) by f^2 = fx^2 + fy^2 + fz^2 (the spectrum depends on |k| only, and
  // |k|^2 takes the 3 (N/2)^2 + 1 integer values of f^2 times (2 pi / L)^2), computed once per
  // plan in float64 on the host
  const double* amp;
};

template <typename R>
__global__ void k_grf(typename Cplx<R>::type* __restrict__ dk, int n, GrfArgs g) {
  using V = typename Cplx<R>::type;
  const int nh = n / 2 + 1;
  const size_t total = (size_t)n * n * nh;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int l = (int)(idx % nh);
  const size_t ij = idx / nh;
  const int j = (int)(ij % n);
  const int i = (int)(ij / n);
  const int h = n / 2;
  if (l == h || i == h || j == h || idx == 0) {
    dk[idx] = V{R(0), R(0)};
    return;
  }
  int ci = i, cj = j;
  bool cj_conj = false;
  if (l == 0) {
    const int pi = (n - i) % n, pj = (n - j) % n;
    if ((long long)pi * n + pj > (long long)i * n + j) {
      ci = pi;
      cj = pj;
      cj_conj = true;
    }
  }
  const uint64_t counter = ((uint64_t)ci * n + cj) * nh + l;
  const PhiloxOut o = philox4x32_10((uint32_t)counter, (uint32_t)(counter >> 32), 0u, 0u,
                                    (uint32_t)g.seed, (uint32_t)(g.seed >> 32));
  const double u1 = uniform_from_words(o.c0, o.c1);
  const double u2 = uniform_from_words(o.c2, o.c3);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * 3.14159265358979323846 * u2;
  const double g1 = rad * cos(ang), g2 = rad * sin(ang);
  const int fi = i < h ? i : i - n, fj = j < h ? j : j - n;
  const double amp = g.amp[fi * fi + fj * fj + l * l];
  double re = amp * g1, im = amp * g2;
  if (cj_conj) im = -im;
  dk[idx] = V{(R)re, (R)im};
}

}  // namespace pin
