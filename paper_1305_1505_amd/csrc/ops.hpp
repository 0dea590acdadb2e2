// Host-side table of the kernel launchers for one (precision, N).  Each supported pair is
// instantiated in its own translation unit (inst.hip compiled with PIN_INST_N / PIN_INST_FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pin {

struct LaunchShape {
  int grid;
  int block;
};

struct SizeOps {
  int n;
  bool fp64;
  // radius-independent Hessian input g0 = M dk scale / f^2 into one aligned slot
  void (*prep)(const void* dk, void* g0, double scale, hipStream_t s);
  // x pass.  mode 0: Hessian from g0 (3 outputs, window table or null); mode 1: gradient from the
  // user half spectrum (2 outputs).  out = first workspace slot of the outputs.
  void (*xpass)(int mode, const void* dk, void* out, const void* wtab, const void* tw, double scale,
                hipStream_t s);
  // fused forward-x / inverse-x of a second-order source: one input slot -> two output slots
  // (gradient, 2LPT) or three (hess: the Hessian x-pass outputs)
  void (*xpass_fwdinv)(bool hess, const void* in, void* out, const void* tw, double scale, hipStream_t s);
  // fused forward-x / inverse-x of the third-order displacement: four source slots -> three
  void (*xpass_lpt3)(const void* in, void* out, const void* tw, double scale, hipStream_t s);
  // y pass: recipe 0 Hessian (3 half slots -> 3 packed slots), 1 gradient (2 half -> 2 packed),
  // 2 forward (1 half -> 1 half), 3 gradient times i from the Hessian x pass (2 half -> 2 packed),
  // 4 three finished components (3 half -> 2 packed)
  void (*ypass)(int recipe, const void* in, void* out, const void* tw, hipStream_t s);
  // Hessian y pass that also writes the v_max gradient (y recipe 3's slots) to gout
  void (*ypass_hess_grad)(const void* in, void* out, void* gout, const void* tw, hipStream_t s);
  // z pass (packed slots in) with the collapse epilogue at radius index r
  void (*zpass_collapse)(const void* in, const void* tw, void* F, uint8_t* ridx, int r, double sphere_gain,
                         hipStream_t s);
  // z pass with the collapse epilogue and v_max: Hessian packed slots `in`, gradient packed
  // slots `gin`; v_max [3][N^3] written where F_max grows, times vscale
  void (*zpass_collapse_v)(const void* in, const void* gin, const void* tw, void* F, uint8_t* ridx, void* vmax,
                           int r, double sphere_gain, double vscale, hipStream_t s);
  // z pass storing nc = 6 (Hessian) or 3 (gradient) real components to out[nc][N^3]
  void (*zpass_store)(int nc, const void* in, const void* tw, void* out, hipStream_t s);
  // z pass computing the 2LPT source and its forward transform along z into one slot; the six
  // tensor components are also stored to t6[6][N^3] when t6 is not null
  void (*zpass_mu2)(const void* in, const void* tw, void* out_slot, void* t6, hipStream_t s);
  // z pass of the second-order tensor with the third-order source epilogue: reads T1 [6][N^3],
  // writes the z-forward transforms of (sl, cx, cy, cz) to four half slots
  void (*zpass_lpt3)(const void* in, const void* t1, const void* tw, void* out_slots, hipStream_t s);
  // the field of `seed`, mode amplitudes from the plan's table (mode_amplitudes)
  void (*grf)(void* dk, uint64_t seed, const double* amp, hipStream_t s);
  void (*reset)(void* F, uint8_t* ridx, hipStream_t s);
  // collapse redshift of count F values (growth table on the device, see k_redshift)
  void (*redshift)(const void* F, size_t count, const double* d, const double* dd, int m, double y0, double h,
                   double a_per_D, double lambda_over_m, const int32_t* guide, int guide_count, double guide_l0,
                   double guide_inv, void* z, hipStream_t s);
  // count reals of the plan's precision set to zero
  void (*zero)(void* p, size_t count, hipStream_t s);
  // per-point collapse model on [6][count] tensors
  void (*collapse_points)(const void* t6, size_t count, void* F, double sphere_gain, hipStream_t s);
  // launch shapes, for reports
  LaunchShape shape_x, shape_y, shape_z;
};

const SizeOps* find_ops(int n, bool fp64);

}  // namespace pin
