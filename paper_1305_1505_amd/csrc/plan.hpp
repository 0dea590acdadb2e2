// Plan internals shared by the C ABI (capi.cpp) and the serving scheduler (serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <string>
#include <utility>
#include <vector>

#include "fragment.hpp"
#include "errors.hpp"
#include "ops.hpp"
#include "pin.h"

namespace pin {

[[noreturn]] void fail(pin_status s, const std::string& m);
void hip_check(hipError_t e, const char* what);
void* device_alloc(size_t bytes, const char* what);
void set_last_error(const std::string& m);
const char* last_error();

// Run f(); map exceptions to a status and the thread-local last-error message.
template <typename F> pin_status guarded(F&& f) {
  try {
    f();
    return PIN_OK;
  } catch (const PinError& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host out of memory");
    return PIN_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return PIN_ERR_DEVICE;
  } catch (...) {
    set_last_error("unknown error");
    return PIN_ERR_DEVICE;
  }
}

enum KernelClass {
  KC_GRF = 0,
  KC_RESET,
  KC_XPASS_HESS,
  KC_YPASS_HESS,
  KC_ZPASS_COLLAPSE,
  KC_ZPASS_STORE,
  KC_XPASS_GRAD,
  KC_YPASS_GRAD,
  KC_ZPASS_MU2,
  KC_YPASS_FWD,
  KC_XPASS_FWDINV,
  KC_COLLAPSE_POINTS,
  KC_PREP,
  KC_YPASS_VEL,
  KC_ZPASS_COLLAPSE_V,
  KC_ZERO,
  KC_REDSHIFT,
  KC_ZPASS_MU2_STORE,
  KC_XPASS_FWDINV_HESS,
  KC_ZPASS_LPT3,
  KC_XPASS_LPT3,
  KC_YPASS_LPT3,
  KC_COUNT
};
extern const char* const kClassNames[KC_COUNT];

bool size_supported(int n);
void validate_desc(const pin_plan_desc* d);
size_t workspace_bytes(int n, int n_radii, bool fp64);
void check_device_range(const void* p, size_t bytes, const char* name);

}  // namespace pin

struct pin_plan_s {
  int n = 0;
  int nr = 0;            // radii in use
  int nr_capacity = 0;   // radii the window table can hold
  double box = 0, sigma8 = 0, gamma = 0, ns = 0;
  bool fp64 = false;
  size_t real_bytes = 4;
  std::vector<double> radii;
  double amplitude = 0;
  double sphere_gain = 0;
  const pin::SizeOps* ops = nullptr;
  int device = 0;
  void* tw = nullptr;
  // mode amplitudes by f^2 (float64, mode_amplitudes) for the field, one table per box the plan
  // has generated fields for (a serving slot changes its box per request), oldest first
  std::vector<std::pair<double, void*>> amp_tables;
  void* wtab = nullptr;   // (nr_capacity + 1) rows of N window values
  void* X = nullptr;      // 4 half slots (= 2 packed slots)
  void* Y = nullptr;      // 6 half slots (= 3 packed slots)
  void* G = nullptr;      // 1 half slot: the radius-independent Hessian input
  void* V = nullptr;      // 4 half slots (= 2 packed slots) for v_max, allocated on first use
  pin::FragWorkspace frag;  // fragmentation workspace, allocated on first use
  void* L = nullptr;      // 10 half slots for the third-order displacement, allocated on first use:
                          // T1 as six real fields, then four source slots
  void* growth = nullptr; // growth table (D, dD/dy: float64; search guide: int32) after pin_plan_set_growth
  double growth_y0 = 0, growth_h = 0, growth_a_per_D = 0, growth_lom = 0, growth_gl0 = 0, growth_ginv = 0;
  size_t slot_bytes = 0;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events[pin::KC_COUNT];
  std::vector<hipEvent_t> pool;

  size_t complex_bytes() const { return 2 * real_bytes; }
  size_t half_spectrum_bytes() const { return (size_t)n * n * (n / 2 + 1) * complex_bytes(); }
  size_t real_field_bytes() const { return (size_t)n * n * n * real_bytes; }
  char* xslot(int i) const { return static_cast<char*>(X) + (size_t)i * slot_bytes; }
  // window table row r (r < nr_capacity: radius r; r = nr_capacity: all ones, no smoothing)
  void* window_row(int r) const { return static_cast<char*>(wtab) + (size_t)r * n * real_bytes; }

  hipEvent_t take_event();
  void recycle_events();
  // Launch with optional event timing on `s`.
  template <typename F> void launch(int cls, hipStream_t s, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timing) {
      a = take_event();
      b = take_event();
      pin::hip_check(hipEventRecord(a, s), "hipEventRecord");
    }
    f();
    pin::hip_check(hipGetLastError(), pin::kClassNames[cls]);
    if (timing) {
      pin::hip_check(hipEventRecord(b, s), "hipEventRecord");
      events[cls].emplace_back(a, b);
    }
  }
};

namespace pin {

// Create a plan for `desc` whose window table can later hold up to `radii_capacity` radii.
pin_plan plan_create(const pin_plan_desc* desc, int radii_capacity);
void plan_free(pin_plan p);
// Replace the radii (strictly decreasing, <= capacity): window tables uploaded on `s`.
void plan_set_radii(pin_plan p, const double* radii, int n_radii, hipStream_t s);

void plan_generate_field(pin_plan p, uint64_t seed, void* dk, hipStream_t s);
void plan_reset(pin_plan p, void* F, uint8_t* ridx, hipStream_t s);
void plan_run_radii(pin_plan p, const void* dk, void* F, uint8_t* ridx, int r0, int r1, hipStream_t s);
void plan_deformation_tensor(pin_plan p, const void* dk, int r, void* T6, hipStream_t s);
// v_max variants: the reset also zeroes v_max [3][N^3]; the radii also record v_max
void plan_reset_v(pin_plan p, void* F, uint8_t* ridx, void* vmax, hipStream_t s);
void plan_run_radii_v(pin_plan p, const void* dk, void* F, uint8_t* ridx, void* vmax, int r0, int r1, hipStream_t s);
size_t velocity_workspace_bytes(int n, bool fp64);
void plan_displacements(pin_plan p, const void* dk, void* psi1, void* psi2, hipStream_t s);
size_t lpt3_workspace_bytes(int n, bool fp64);
void plan_lpt3_displacement(pin_plan p, const void* dk, void* psi3, hipStream_t s);

}  // namespace pin
