// Per-point ellipsoidal collapse on the device (section "Collapse times", eq. F).
//
// The paper describes but does not print its collapse formula.  This file implements the reading
// used throughout the library (truncated 3rd-order LPT along the first axis with a
// quasi-spherical correction):
//
//   lambda_1 = largest eigenvalue of T, delta = tr T, mu2 = sum_{i<j} lambda_i lambda_j,
//   mu3 = det T.  The first axis crosses orbits at the smallest D > 0 with
//       J1(D) = 1 - lambda_1 D - (mu2/7) D^2 + (mu3/9 - 10 delta mu2/189) D^3 = 0,
//   (2nd- and 3rd-order LPT traces shared equally by the three axes), i.e. at the largest
//   positive root F_E3 of the monic cubic in F = 1/D
//       P(F) = F^3 - lambda_1 F^2 - (mu2/7) F + (mu3/9 - 10 delta mu2/189),
//   F_E3 = 0 if there is none.  Correction for near-spherical peaks:
//       F = F_E3 * (1 + (X3/delta_c - 1) * s),  s = clamp(1 - 3p/delta, 0, 1) (delta > 0; else 0),
//   p = sqrt(tr(B^2)/6), B = T - (delta/3) I, X3 = 2.05008... the root of the 3rd-order EdS
//   sphere series 1 - x/3 - x^2/21 - 23x^3/1701, delta_c = (3/20)(12 pi)^(2/3).  A sphere gets
//   F = delta/delta_c and a plane F = lambda_1.
//
// Arithmetic: float64.  lambda_1 from the trigonometric closed form of a symmetric 3x3
// eigenproblem, lambda_1 = m + 2p cos(acos(r)/3) with r = det(B)/(2p^3), evaluated as a
// polynomial in sqrt(1 + r) and polished by Newton steps on the characteristic polynomial; near
// r = -1 (1 + r <= 1e-5, lambda_1 ~ lambda_2) the two largest roots nearly coincide and the
// polynomial's root is ill-conditioned in its coefficients, so there the eigenvalue comes from
// cyclic Jacobi rotations instead.  The cubic's largest real root comes from
// the closed form (trigonometric for three real roots, Cardano otherwise) polished by Newton
// steps on P.
#pragma once

#include <hip/hip_runtime.h>

#include "trig_poly.hpp"

namespace pin {

struct CollapseConst {
  // X3 / delta_c - 1, with X3 and delta_c as above (both computed on the host in float64 and
  // passed in, so the constants live in one place).
  double sphere_gain;
};

// Full-precision float64 reciprocal and reciprocal square root from the hardware estimates
// (about 2^-23 relative) and two refinement steps, each of which squares the relative error: a
// few ulp, against the library's correctly rounded division and square root sequences.
__device__ __forceinline__ double rcp_full(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsq_full(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
// sign(v) |v|^(1/3): the float32 hardware log2/exp2 estimate, then two Newton steps in float64
// (the library cube root outside the range where the float32 estimate is a normal number)
__device__ __forceinline__ double cbrt_full(double v) {
  const double a = fabs(v);
  if (a == 0.0) return 0.0;
  if (!(a > 1e-30 && a < 1e30)) return cbrt(v);
  double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)a) * (1.f / 3.f));
  y = y - (y * y * y - a) * (1.0 / 3.0) * rcp_full(y * y);
  y = y - (y * y * y - a) * (1.0 / 3.0) * rcp_full(y * y);
  return copysign(y, v);
}

__device__ __forceinline__ double cubic_largest_real_root(double a, double b, double c) {
  // depressed cubic t^3 + p t + q with F = t - a/3
  const double a3 = a * (1.0 / 3.0);
  const double p = b - a * a3;
  const double q = c - a3 * b + 2.0 * a3 * a3 * a3;
  const double hq = 0.5 * q;
  const double p3 = p * (1.0 / 3.0);
  const double disc = hq * hq + p3 * p3 * p3;
  double t;
  if (disc < 0.0) {
    // three real roots (p < 0): t_k = 2 r cos(theta/3 - 2 pi k/3), cos(theta) = -hq / r^3; the
    // largest from the polynomial in sqrt(1 + cos theta) (within 1.1e-8 of it; the Newton steps
    // below polish it) unless the two largest roots nearly coincide
    const double qr = rsq_full(-p3);
    const double r = -p3 * qr;
    double cth = -hq * (qr * qr * qr);
    cth = fmin(1.0, fmax(-1.0, cth));
    if (cth > -1.0 + 1e-8) {
      const double u = (1.0 + cth) * rsq_full(1.0 + cth);
      double cu = (double)kAcos3U[8];
#pragma unroll
      for (int k = 7; k >= 0; --k) cu = fma(cu, u, (double)kAcos3U[k]);
      t = 2.0 * r * cu;
    } else {
      t = 2.0 * r * cos(acos(cth) * (1.0 / 3.0));
    }
  } else {
    const double sd = disc > 0.0 ? disc * rsq_full(disc) : 0.0;
    const double u = cbrt_full(-hq - copysign(sd, hq));
    t = (u != 0.0) ? (u - p3 * rcp_full(u)) : 0.0;
  }
  double x = t - a3;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double f = ((x + a) * x + b) * x + c;
    const double fp = (3.0 * x + 2.0 * a) * x + b;
    if (fp > 0.0) x -= f * __builtin_amdgcn_rcp(fp);   // approximate reciprocal: the step is a correction
  }
  return x;
}

// Largest eigenvalue of a symmetric 3x3 matrix by cyclic Jacobi rotations (each rotation zeroes
// one off-diagonal element; the eigenvalues are the diagonal once all three are negligible).
__device__ __noinline__ double jacobi_largest_eigenvalue(double a00, double a01, double a02, double a11,
                                                         double a12, double a22) {
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a01 * a01 + a02 * a02 + a12 * a12;
    const double diag = a00 * a00 + a11 * a11 + a22 * a22;
    if (off <= 1e-34 * diag || off == 0.0) break;
    // rotation in the (0,1) plane
    if (a01 != 0.0) {
      const double th = (a11 - a00) / (2.0 * a01);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      a00 -= t * a01;
      a11 += t * a01;
      a01 = 0.0;
      const double g = a02, h = a12;
      a02 = c * g - s * h;
      a12 = s * g + c * h;
    }
    // (0,2)
    if (a02 != 0.0) {
      const double th = (a22 - a00) / (2.0 * a02);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      a00 -= t * a02;
      a22 += t * a02;
      a02 = 0.0;
      const double g = a01, h = a12;
      a01 = c * g - s * h;
      a12 = s * g + c * h;
    }
    // (1,2)
    if (a12 != 0.0) {
      const double th = (a22 - a11) / (2.0 * a12);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      a11 -= t * a12;
      a22 += t * a12;
      a12 = 0.0;
      const double g = a01, h = a02;
      a01 = c * g - s * h;
      a02 = s * g + c * h;
    }
  }
  return fmax(a00, fmax(a11, a22));
}

// Inverse collapse time F of one point from its six tensor components (float64).
__device__ __forceinline__ double collapse_point(double xx, double xy, double xz, double yy, double yz,
                                                 double zz, const CollapseConst& cc) {
  const double delta = xx + yy + zz;
  const double m = delta * (1.0 / 3.0);
  const double mu2 = xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz;
  const double mu3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
  const double bxx = xx - m, byy = yy - m, bzz = zz - m;
  const double off = xy * xy + xz * xz + yz * yz;
  const double p2 = (bxx * bxx + byy * byy + bzz * bzz + 2.0 * off) * (1.0 / 6.0);
  const double qp = p2 > 0.0 ? rsq_full(p2) : 0.0;
  const double p = p2 * qp;
  double l1 = m;
  if (p2 > 0.0) {
    const double detb = bxx * (byy * bzz - yz * yz) - xy * (xy * bzz - yz * xz) + xz * (xy * yz - byy * xz);
    double r = 0.5 * detb * (qp * qp * qp);
    r = fmin(1.0, fmax(-1.0, r));
    if (r > -1.0 + 1e-5) {
      // c(r) = cos(arccos(r)/3) from its polynomial in sqrt(1 + r) (within 1.1e-8), then Newton
      // steps on y^3 - 3 p^2 y - det B, whose largest root y = lambda_1 - m is simple here (the
      // two largest roots are at least ~5e-3 p apart): from 2e-8 p two steps reach the root of
      // the computed polynomial, which the rounding of p^2 and det B moves by ~1e-16 p / sqrt(1 + r)
      // (3e-14 p at the switch; closer to r = -1 the rotations below are backward stable)
      const double u = (1.0 + r) * rsq_full(1.0 + r);
      double c = (double)kAcos3U[8];
#pragma unroll
      for (int k = 7; k >= 0; --k) c = fma(c, u, (double)kAcos3U[k]);
      double y = 2.0 * p * c;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const double f = (y * y - 3.0 * p2) * y - detb;
        const double fp = 3.0 * (y * y - p2);
        if (fp > 0.0) y -= f * __builtin_amdgcn_rcp(fp);
      }
      l1 = m + y;
    } else {
      l1 = jacobi_largest_eigenvalue(xx, xy, xz, yy, yz, zz);
    }
  }
  const double ca = -l1;
  const double cb = -mu2 * (1.0 / 7.0);
  const double cc0 = mu3 * (1.0 / 9.0) - 10.0 * delta * mu2 * (1.0 / 189.0);
  const double root = cubic_largest_real_root(ca, cb, cc0);
  const double fe3 = root > 0.0 ? root : 0.0;
  double s = 0.0;
  if (delta > 0.0) s = fmin(1.0, fmax(0.0, 1.0 - 3.0 * p * rcp_full(delta)));
  return fe3 * (1.0 + cc.sphere_gain * s);
}

// ---------------------------------------------------------------------------------------------
// Mixed-precision path of collapse_point for float32 tensor components.
//
// The invariants are formed in float64 from the float32 components (exact products), and so are
// p = sqrt(p^2) and r = det(B)/(2 p^3), from one reciprocal square root: then 1 + r keeps float64
// absolute accuracy as r -> -1 (lambda_1 -> lambda_2), where c(r) = cos(arccos(r)/3) is steepest,
// and the same holds for the collapse cubic's 1 + r_c at a double root.  c is one float32
// polynomial in sqrt(1 + r) over all of [-1, 1] (trig_poly.hpp), so no lane branches on the sign
// of r.  With 1 + r and 1 + r_c accurate, the closed forms give lambda_1 and the collapse root to
// the polynomial's float32 evaluation (~1e-7 of p and of the root) with no polishing.  The
// cubic's coefficients are taken directly in depressed form (F = t + lambda_1/3).

// c(r) = cos(arccos(r)/3) from opr = 1 + r.
__device__ __forceinline__ float acos3_cos(float opr) {
  const float u = __builtin_amdgcn_sqrtf(fmaxf(opr, 0.f));
  float y = kAcos3U[8];
#pragma unroll
  for (int k = 7; k >= 0; --k) y = fmaf(y, u, kAcos3U[k]);
  return y;
}

__device__ __forceinline__ float fast_cbrt(float v) {
  // sign(v) |v|^(1/3) from the hardware log2/exp2: a few float32 ulp, like the rest of the
  // one-real-root branch's float32 arithmetic (no correction step follows)
  const float a = fabsf(v);
  const float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(a) * (1.f / 3.f));
  return a == 0.f ? 0.f : copysignf(y, v);
}

// 1/sqrt(x) for x > 0 in float64: the hardware estimate y and one Newton step y + y e / 2 with
// the residual e = 1 - x y^2, which squares the estimate's relative error.
__device__ __forceinline__ double rsq_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

__device__ __forceinline__ float collapse_point_mixed(float fxx, float fxy, float fxz, float fyy, float fyz,
                                                      float fzz, float sphere_gain) {
  const double xx = fxx, xy = fxy, xz = fxz, yy = fyy, yz = fyz, zz = fzz;
  const double delta = xx + yy + zz;
  const double m = delta * (1.0 / 3.0);
  const double bxx = xx - m, byy = yy - m, bzz = zz - m;
  const double off = xy * xy + xz * xz + yz * yz;
  const double s6 = bxx * bxx + byy * byy + bzz * bzz + 2.0 * off;   // tr(B^2) = 6 p^2
  const double detb = bxx * (byy * bzz - yz * yz) - xy * (xy * bzz - yz * xz) + xz * (xy * yz - byy * xz);
  // invariants of T = B + m I from those of B (tr B = 0, mu2(B) = -3 p^2): mu2 = 3 m^2 - 3 p^2,
  // mu3 = m (m^2 - 3 p^2) + det B
  const double h3 = 0.5 * s6;
  const double mu2 = delta * m - h3;
  const double mu3 = m * (m * m - h3) + detb;
  // lambda_1 = m + y, y = 2 p c(r) the largest root of y^3 - 3 p^2 y - det B, with
  // r = det B / (2 p^3) = det B (6/tr B^2)^(3/2) / 2; tr B^2 = 0 (a sphere, det B = 0 too) gives
  // p = 0 and r = 0 through the floor
  const double qs = rsq_f64(fmax(s6, 1e-200));
  const double r = detb * (qs * qs * qs) * 7.3484692283495345;      // 6^(3/2) / 2
  const double y = s6 * qs * (2.0 / 2.4494897427831781) * (double)acos3_cos((float)(1.0 + r));
  const double l1 = m + y;
  // collapse cubic P(F) = F^3 - l1 F^2 - (mu2/7) F + c0, c0 = mu3/9 - 10 delta mu2/189; with
  // F = t + l1/3 it is t^3 + 3 p3 t + 2 hq, p3 = -(mu2/21 + l1^2/9), hq = c0/2 - l1 (mu2/42 + l1^2/27)
  const double l1s = l1 * l1;
  const double c0 = mu3 * (1.0 / 9.0) - (delta * mu2) * (10.0 / 189.0);
  const double p3 = -(mu2 * (1.0 / 21.0) + l1s * (1.0 / 9.0));
  const double hq = 0.5 * c0 - l1 * (mu2 * (1.0 / 42.0) + l1s * (1.0 / 27.0));
  const double disc = hq * hq + p3 * p3 * p3;
  double t;
  if (disc < 0.0) {
    // three real roots (p3 < 0): t = 2 sqrt(-p3) c(r_c), r_c = -hq / (-p3)^(3/2)
    const double qc = rsq_f64(-p3);
    const double rc = -hq * (qc * qc * qc);
    t = 2.0 * (-p3 * qc) * (double)acos3_cos((float)(1.0 + rc));
  } else {
    const float sd = __builtin_amdgcn_sqrtf((float)disc);
    const float u = fast_cbrt((float)(-hq) - copysignf(sd, (float)hq));
    t = u != 0.f ? (double)(u - (float)p3 * __builtin_amdgcn_rcpf(u)) : 0.0;
  }
  const double x = t + l1 * (1.0 / 3.0);
  const float fe3 = x > 0.0 ? (float)x : 0.f;
  const float dl = (float)delta;
  const float p = (float)(s6 * qs * (1.0 / 2.4494897427831781));
  const float s = dl > 0.f ? fminf(1.f, fmaxf(0.f, 1.f - 3.f * p * __builtin_amdgcn_rcpf(dl))) : 0.f;
  return fe3 * (1.f + sphere_gain * s);
}

}  // namespace pin
