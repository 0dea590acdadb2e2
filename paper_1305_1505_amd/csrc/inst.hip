// Instantiation of the kernels and their launchers for one grid size and precision.
// Compiled once per supported (N, precision) with -DPIN_INST_N=<N> -DPIN_INST_FP64=<0|1>.
#include "grf.hpp"
#include "kernels.hpp"
#include "ops.hpp"

#ifndef PIN_INST_N
#error "PIN_INST_N must be defined"
#endif
#ifndef PIN_INST_FP64
#error "PIN_INST_FP64 must be defined"
#endif

namespace pin {
namespace {

constexpr int NN = PIN_INST_N;
using RR = std::conditional_t<PIN_INST_FP64 != 0, double, float>;
using VV = Cplx<RR>::type;
static_assert(size_ok(NN) && NN % 2 == 0, "grid size");

void prep(const void* dk, void* g0, double scale, hipStream_t s) {
  const size_t total = (size_t)NN * NN * (NN / 2);
  const int block = 256;
  const int grid = (int)((total + block - 1) / block);
  hipLaunchKernelGGL((k_prep<RR, NN>), dim3(grid), dim3(block), 0, s, static_cast<const VV*>(dk),
                     static_cast<VV*>(g0), (RR)scale);
}

void xpass(int mode, const void* dk, void* out, const void* wtab, const void* tw, double scale, hipStream_t s) {
  using S = Strided<RR, NN, +1>;
  if (mode == 0) {
    hipLaunchKernelGGL((k_xpass<RR, NN, 0>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(dk),
                       static_cast<VV*>(out), static_cast<const RR*>(wtab), static_cast<const VV*>(tw), (RR)scale);
  } else {
    hipLaunchKernelGGL((k_xpass<RR, NN, 1>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(dk),
                       static_cast<VV*>(out), static_cast<const RR*>(nullptr), static_cast<const VV*>(tw), (RR)scale);
  }
}

void xpass_fwdinv(bool hess, const void* in, void* out, const void* tw, double scale, hipStream_t s) {
  using S = Strided<RR, NN, +1>;
  if (hess) {
    hipLaunchKernelGGL((k_xpass_fwdinv<RR, NN, true>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw), (RR)scale);
  } else {
    hipLaunchKernelGGL((k_xpass_fwdinv<RR, NN, false>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw), (RR)scale);
  }
}

void xpass_lpt3(const void* in, void* out, const void* tw, double scale, hipStream_t s) {
  using S = Strided<RR, NN, +1>;
  hipLaunchKernelGGL((k_xpass_lpt3<RR, NN>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                     static_cast<VV*>(out), static_cast<const VV*>(tw), (RR)scale);
}

void ypass(int recipe, const void* in, void* out, const void* tw, hipStream_t s) {
  if (recipe == 0) {
    using S = Strided<RR, NN, +1>;
    hipLaunchKernelGGL((k_ypass_packed<RR, NN, 0>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw), static_cast<VV*>(nullptr));
  } else if (recipe == 1) {
    using S = Strided<RR, NN, +1>;
    hipLaunchKernelGGL((k_ypass_packed<RR, NN, 1>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw), static_cast<VV*>(nullptr));
  } else if (recipe == 3) {
    using S = Strided<RR, NN, +1>;
    hipLaunchKernelGGL((k_ypass_packed<RR, NN, 3>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw), static_cast<VV*>(nullptr));
  } else if (recipe == 4) {
    using S = Strided<RR, NN, +1>;
    hipLaunchKernelGGL((k_ypass_packed<RR, NN, 4>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw), static_cast<VV*>(nullptr));
  } else {
    using S = Strided<RR, NN, -1>;
    hipLaunchKernelGGL((k_ypass_fwd<RR, NN>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                       static_cast<VV*>(out), static_cast<const VV*>(tw));
  }
}

// Hessian (3 packed slots to out) and v_max gradient (2 packed slots to gout) in one y pass.
void ypass_hess_grad(const void* in, void* out, void* gout, const void* tw, hipStream_t s) {
  using S = Strided<RR, NN, +1>;
  hipLaunchKernelGGL((k_ypass_packed<RR, NN, 5>), dim3(S::GRID), dim3(S::T), 0, s, static_cast<const VV*>(in),
                     static_cast<VV*>(out), static_cast<const VV*>(tw), static_cast<VV*>(gout));
}

void zpass_collapse(const void* in, const void* tw, void* F, uint8_t* ridx, int r, double sphere_gain, hipStream_t s) {
  using Z = ZPass<RR, NN, 3, EPI_COLLAPSE>;
  ZArgs a{};
  a.F = F;
  a.ridx = ridx;
  a.r = r;
  a.cc.sphere_gain = sphere_gain;
  hipLaunchKernelGGL((k_zpass<RR, NN, 3, EPI_COLLAPSE>), dim3(Z::GRID), dim3(Z::T), 0, s,
                     static_cast<const VV*>(in), static_cast<const VV*>(tw), a);
}

void zpass_collapse_v(const void* in, const void* gin, const void* tw, void* F, uint8_t* ridx, void* vmax, int r,
                      double sphere_gain, double vscale, hipStream_t s) {
  using Z = ZPass<RR, NN, 3, EPI_COLLAPSE_V>;
  ZArgs a{};
  a.F = F;
  a.ridx = ridx;
  a.r = r;
  a.cc.sphere_gain = sphere_gain;
  a.gin = gin;
  a.vout = vmax;
  a.vscale = vscale;
  hipLaunchKernelGGL((k_zpass<RR, NN, 3, EPI_COLLAPSE_V>), dim3(Z::GRID), dim3(Z::T), 0, s,
                     static_cast<const VV*>(in), static_cast<const VV*>(tw), a);
}

void zpass_store(int nc, const void* in, const void* tw, void* out, hipStream_t s) {
  ZArgs a{};
  a.out = out;
  a.nc = nc;
  if (nc == 6) {
    using Z = ZPass<RR, NN, 3, EPI_STORE>;
    hipLaunchKernelGGL((k_zpass<RR, NN, 3, EPI_STORE>), dim3(Z::GRID), dim3(Z::T), 0, s,
                       static_cast<const VV*>(in), static_cast<const VV*>(tw), a);
  } else {
    using Z = ZPass<RR, NN, 2, EPI_STORE>;
    hipLaunchKernelGGL((k_zpass<RR, NN, 2, EPI_STORE>), dim3(Z::GRID), dim3(Z::T), 0, s,
                       static_cast<const VV*>(in), static_cast<const VV*>(tw), a);
  }
}

void zpass_mu2(const void* in, const void* tw, void* out_slot, void* t6, hipStream_t s) {
  using Z = ZPass<RR, NN, 3, EPI_MU2>;
  ZArgs a{};
  a.out = out_slot;
  a.t6 = t6;
  hipLaunchKernelGGL((k_zpass<RR, NN, 3, EPI_MU2>), dim3(Z::GRID), dim3(Z::T), 0, s,
                     static_cast<const VV*>(in), static_cast<const VV*>(tw), a);
}

void zpass_lpt3(const void* in, const void* t1, const void* tw, void* out_slots, hipStream_t s) {
  using Z = ZPass<RR, NN, 3, EPI_LPT3>;
  ZArgs a{};
  a.out = out_slots;
  a.t6 = const_cast<void*>(t1);
  hipLaunchKernelGGL((k_zpass<RR, NN, 3, EPI_LPT3>), dim3(Z::GRID), dim3(Z::T), 0, s,
                     static_cast<const VV*>(in), static_cast<const VV*>(tw), a);
}

void grf(void* dk, uint64_t seed, const double* amp, hipStream_t s) {
  GrfArgs g{seed, amp};
  const size_t total = (size_t)NN * NN * (NN / 2 + 1);
  const int block = 256;
  const int grid = (int)((total + block - 1) / block);
  hipLaunchKernelGGL((k_grf<RR>), dim3(grid), dim3(block), 0, s, static_cast<VV*>(dk), NN, g);
}

void reset(void* F, uint8_t* ridx, hipStream_t s) {
  const size_t total = (size_t)NN * NN * NN;
  const int block = 256;
  const int grid = (int)((total + block - 1) / block);
  hipLaunchKernelGGL((k_reset<RR>), dim3(grid), dim3(block), 0, s, static_cast<RR*>(F), ridx, total);
}

void redshift(const void* F, size_t count, const double* d, const double* dd, int m, double y0, double h,
              double a_per_D, double lambda_over_m, const int32_t* guide, int guide_count, double guide_l0,
              double guide_inv, void* z, hipStream_t s) {
  if (count == 0) return;
  GrowthArgs g{d, dd, m, y0, h, a_per_D, lambda_over_m, guide, guide_count, (float)guide_l0, (float)guide_inv};
  const int block = 256;
  const int grid = (int)((count + block - 1) / block);
  hipLaunchKernelGGL((k_redshift<RR>), dim3(grid), dim3(block), 0, s, static_cast<const RR*>(F), count, g,
                     static_cast<RR*>(z));
}

void zero(void* p, size_t count, hipStream_t s) {
  if (count == 0) return;
  const int block = 256;
  const int grid = (int)((count + block - 1) / block);
  hipLaunchKernelGGL((k_zero<RR>), dim3(grid), dim3(block), 0, s, static_cast<RR*>(p), count);
}

void collapse_points(const void* t6, size_t count, void* F, double sphere_gain, hipStream_t s) {
  if (count == 0) return;
  CollapseConst cc{sphere_gain};
  const int block = 256;
  const int grid = (int)((count + block - 1) / block);
  hipLaunchKernelGGL((k_collapse_points<RR>), dim3(grid), dim3(block), 0, s, static_cast<const RR*>(t6), count,
                     static_cast<RR*>(F), cc);
}

}  // namespace

#define PIN_CAT2(a, b, c) a##b##_##c
#define PIN_CAT(a, b, c) PIN_CAT2(a, b, c)

const SizeOps* PIN_CAT(ops_, PIN_INST_FP64, PIN_INST_N)() {
  static const SizeOps ops = {
      NN, PIN_INST_FP64 != 0, prep, xpass, xpass_fwdinv, xpass_lpt3, ypass, ypass_hess_grad, zpass_collapse, zpass_collapse_v,
      zpass_store, zpass_mu2, zpass_lpt3, grf, reset, redshift, zero, collapse_points,
      LaunchShape{Strided<RR, NN, +1>::GRID, Strided<RR, NN, +1>::T},
      LaunchShape{Strided<RR, NN, +1>::GRID, Strided<RR, NN, +1>::T},
      LaunchShape{ZPass<RR, NN, 3, EPI_COLLAPSE>::GRID, ZPass<RR, NN, 3, EPI_COLLAPSE>::T}};
  return &ops;
}

}  // namespace pin
