// C ABI of libpin: plan management, argument validation and the per-radius launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "pin.h"
#include "host_math.hpp"
#include "ops.hpp"

namespace {

thread_local std::string g_last_error;

struct PinError : std::exception {
  pin_status status;
  std::string msg;
  PinError(pin_status s, std::string m) : status(s), msg(std::move(m)) {}
  const char* what() const noexcept override { return msg.c_str(); }
};

[[noreturn]] void fail(pin_status s, const std::string& m) { throw PinError(s, m); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(PIN_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
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
  KC_COUNT
};

const char* const kClassNames[KC_COUNT] = {
    "grf",         "reset",       "xpass_hessian", "ypass_hessian", "zpass_collapse", "zpass_store",
    "xpass_gradient", "ypass_gradient", "zpass_mu2", "ypass_forward", "xpass_fwdinv",
    "collapse_points", "prep"};

}  // namespace

struct pin_plan_s {
  int n = 0;
  int nr = 0;
  double box = 0, sigma8 = 0, gamma = 0, ns = 0;
  bool fp64 = false;
  size_t real_bytes = 4;
  std::vector<double> radii;
  double amplitude = 0;
  double sphere_gain = 0;
  const pin::SizeOps* ops = nullptr;
  int device = 0;
  void* tw = nullptr;
  void* wtab = nullptr;
  void* X = nullptr;      // 4 half slots (= 2 packed slots)
  void* Y = nullptr;      // 6 half slots (= 3 packed slots)
  void* G = nullptr;      // 1 half slot: the radius-independent Hessian input
  size_t slot_bytes = 0;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events[KC_COUNT];
  std::vector<hipEvent_t> pool;

  size_t complex_bytes() const { return 2 * real_bytes; }
  size_t half_spectrum_bytes() const { return (size_t)n * n * (n / 2 + 1) * complex_bytes(); }
  size_t real_field_bytes() const { return (size_t)n * n * n * real_bytes; }
  char* xslot(int i) const { return static_cast<char*>(X) + (size_t)i * slot_bytes; }
  char* yslot(int i) const { return static_cast<char*>(Y) + (size_t)i * slot_bytes; }

  hipEvent_t take_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
  void recycle_events() {
    for (auto& v : events) {
      for (auto& pr : v) {
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      v.clear();
    }
  }

  // Launch with optional event timing on `s`.
  template <typename F> void launch(int cls, hipStream_t s, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timing) {
      a = take_event();
      b = take_event();
      hip_check(hipEventRecord(a, s), "hipEventRecord");
    }
    f();
    hip_check(hipGetLastError(), kClassNames[cls]);
    if (timing) {
      hip_check(hipEventRecord(b, s), "hipEventRecord");
      events[cls].emplace_back(a, b);
    }
  }
};

namespace {

bool size_supported(int n) { return pin::find_ops(n, false) != nullptr; }

void validate_desc(const pin_plan_desc* d) {
  if (d == nullptr) fail(PIN_ERR_INVALID_ARG, "desc is NULL");
  if (!size_supported(d->n))
    fail(PIN_ERR_UNSUPPORTED_SIZE, "unsupported grid size N=" + std::to_string(d->n));
  if (!(d->box > 0.0) || !std::isfinite(d->box)) fail(PIN_ERR_INVALID_ARG, "box must be positive and finite");
  if (d->n_radii < 1 || d->n_radii > 254) fail(PIN_ERR_INVALID_ARG, "n_radii must be in [1, 254]");
  if (d->radii_cells == nullptr) fail(PIN_ERR_INVALID_ARG, "radii_cells is NULL");
  for (int i = 0; i < d->n_radii; ++i) {
    const double r = d->radii_cells[i];
    if (!(r > 0.0) || !std::isfinite(r)) fail(PIN_ERR_INVALID_ARG, "radii must be positive and finite");
    if (i > 0 && !(r < d->radii_cells[i - 1]))
      fail(PIN_ERR_INVALID_ARG, "radii must be strictly decreasing (largest first)");
  }
  if (!(d->sigma8 > 0.0) || !std::isfinite(d->sigma8)) fail(PIN_ERR_INVALID_ARG, "sigma8 must be positive");
  if (!(d->gamma > 0.0) || !std::isfinite(d->gamma)) fail(PIN_ERR_INVALID_ARG, "gamma must be positive");
  if (!std::isfinite(d->ns)) fail(PIN_ERR_INVALID_ARG, "ns must be finite");
  if (d->prec != PIN_FP32 && d->prec != PIN_FP64) fail(PIN_ERR_INVALID_ARG, "prec must be PIN_FP32 or PIN_FP64");
}

size_t workspace_bytes(const pin_plan_desc* d) {
  const size_t rb = d->prec == PIN_FP64 ? 8 : 4;
  const size_t slot = (size_t)d->n * d->n * (d->n / 2) * 2 * rb;
  return 11 * slot + (size_t)d->n * 2 * rb + (size_t)d->n * d->n_radii * rb;
}

// Check that [p, p + bytes) lies inside one device allocation of the plan's device.
void check_device_range(const void* p, size_t bytes, const char* name) {
  if (p == nullptr) fail(PIN_ERR_INVALID_ARG, std::string(name) + " is NULL");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  const hipError_t e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(PIN_ERR_INVALID_ARG, std::string(name) + " is not a device allocation");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || (size_t)(q - b) + bytes > size)
    fail(PIN_ERR_INVALID_ARG, std::string(name) + " is smaller than required (" + std::to_string(bytes) + " bytes)");
}

void check_plan(pin_plan p) {
  if (p == nullptr) fail(PIN_ERR_INVALID_ARG, "plan is NULL");
}

template <typename F> pin_status guarded(F&& f) {
  try {
    f();
    return PIN_OK;
  } catch (const PinError& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host out of memory";
    return PIN_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PIN_ERR_DEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return PIN_ERR_DEVICE;
  }
}

void* device_alloc(size_t bytes, const char* what) {
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(PIN_ERR_OUT_OF_MEMORY, std::string("hipMalloc(") + what + ", " + std::to_string(bytes) + " bytes) failed");
  }
  return p;
}

void upload(void* dst, const std::vector<double>& src, bool fp64) {
  if (fp64) {
    hip_check(hipMemcpy(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
  } else {
    std::vector<float> f(src.size());
    for (size_t i = 0; i < src.size(); ++i) f[i] = (float)src[i];
    hip_check(hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  }
}

void free_plan(pin_plan p) {
  if (p == nullptr) return;
  for (auto& v : p->events)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  if (p->tw) (void)hipFree(p->tw);
  if (p->wtab) (void)hipFree(p->wtab);
  if (p->X) (void)hipFree(p->X);
  if (p->Y) (void)hipFree(p->Y);
  if (p->G) (void)hipFree(p->G);
  delete p;
}

void prep_hessian_input(pin_plan p, const void* dk, hipStream_t s) {
  const double scale = 1.0 / ((double)p->n * p->n * p->n);
  p->launch(KC_PREP, s, [&] { p->ops->prep(dk, p->G, scale, s); });
}

void run_radii(pin_plan p, const void* dk, void* F, uint8_t* ridx, int r0, int r1, hipStream_t s) {
  prep_hessian_input(p, dk, s);
  for (int r = r0; r < r1; ++r) {
    const char* w = static_cast<const char*>(p->wtab) + (size_t)r * p->n * p->real_bytes;
    p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, w, p->tw, 1.0, s); });
    p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
    p->launch(KC_ZPASS_COLLAPSE, s, [&] { p->ops->zpass_collapse(p->Y, p->tw, F, ridx, r, p->sphere_gain, s); });
  }
}

}  // namespace

extern "C" {

int pin_size_supported(int n) { return size_supported(n) ? 1 : 0; }

pin_status pin_plan_validate(const pin_plan_desc* desc) {
  return guarded([&] { validate_desc(desc); });
}

pin_status pin_plan_workspace_bytes(const pin_plan_desc* desc, size_t* bytes) {
  return guarded([&] {
    validate_desc(desc);
    if (bytes == nullptr) fail(PIN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = workspace_bytes(desc);
  });
}

pin_status pin_plan_create(const pin_plan_desc* desc, pin_plan* out) {
  pin_plan p = nullptr;
  const pin_status st = guarded([&] {
    validate_desc(desc);
    if (out == nullptr) fail(PIN_ERR_INVALID_ARG, "out is NULL");
    p = new pin_plan_s();
    p->n = desc->n;
    p->nr = desc->n_radii;
    p->box = desc->box;
    p->sigma8 = desc->sigma8;
    p->gamma = desc->gamma;
    p->ns = desc->ns;
    p->fp64 = desc->prec == PIN_FP64;
    p->real_bytes = p->fp64 ? 8 : 4;
    p->radii.assign(desc->radii_cells, desc->radii_cells + desc->n_radii);
    p->ops = pin::find_ops(p->n, p->fp64);
    p->amplitude = pin::amplitude_for_sigma8(p->sigma8, p->gamma, p->ns);
    p->sphere_gain = pin::eds_sphere_root() / pin::eds_delta_c() - 1.0;
    hip_check(hipGetDevice(&p->device), "hipGetDevice");
    p->slot_bytes = (size_t)p->n * p->n * (p->n / 2) * p->complex_bytes();
    p->tw = device_alloc((size_t)p->n * p->complex_bytes(), "twiddles");
    p->wtab = device_alloc((size_t)p->n * p->nr * p->real_bytes, "windows");
    p->X = device_alloc(4 * p->slot_bytes, "workspace X");
    p->Y = device_alloc(6 * p->slot_bytes, "workspace Y");
    p->G = device_alloc(p->slot_bytes, "workspace G");
    upload(p->tw, pin::twiddles(p->n), p->fp64);
    std::vector<double> w;
    w.reserve((size_t)p->n * p->nr);
    for (int r = 0; r < p->nr; ++r) {
      const auto wr = pin::gaussian_window_table(p->n, p->radii[r]);
      w.insert(w.end(), wr.begin(), wr.end());
    }
    upload(p->wtab, w, p->fp64);
    *out = p;
  });
  if (st != PIN_OK) free_plan(p);
  return st;
}

pin_status pin_plan_destroy(pin_plan plan) {
  return guarded([&] {
    check_plan(plan);
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    free_plan(plan);
  });
}

pin_status pin_generate_field(pin_plan plan, uint64_t seed, void* dk, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    const double n = plan->n;
    const double norm = plan->amplitude * std::pow(n, 6) / (2.0 * plan->box * plan->box * plan->box);
    const double kf = 2.0 * 3.14159265358979323846 / plan->box;
    plan->launch(KC_GRF, stream, [&] { plan->ops->grf(dk, seed, norm, kf, plan->gamma, plan->ns, stream); });
  });
}

pin_status pin_collapse_reset(pin_plan plan, void* F, uint8_t* ridx, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(F, plan->real_field_bytes(), "F");
    check_device_range(ridx, (size_t)plan->n * plan->n * plan->n, "ridx");
    plan->launch(KC_RESET, stream, [&] { plan->ops->reset(F, ridx, stream); });
  });
}

pin_status pin_collapse_times_range(pin_plan plan, const void* dk, void* F, uint8_t* ridx, int r_begin, int r_end,
                                    hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (r_begin < 0 || r_end > plan->nr || r_begin >= r_end)
      fail(PIN_ERR_INVALID_ARG, "radius range must satisfy 0 <= r_begin < r_end <= n_radii");
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_device_range(F, plan->real_field_bytes(), "F");
    check_device_range(ridx, (size_t)plan->n * plan->n * plan->n, "ridx");
    run_radii(plan, dk, F, ridx, r_begin, r_end, stream);
  });
}

pin_status pin_collapse_times(pin_plan plan, const void* dk, void* F, uint8_t* ridx, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_device_range(F, plan->real_field_bytes(), "F");
    check_device_range(ridx, (size_t)plan->n * plan->n * plan->n, "ridx");
    plan->launch(KC_RESET, stream, [&] { plan->ops->reset(F, ridx, stream); });
    run_radii(plan, dk, F, ridx, 0, plan->nr, stream);
  });
}

pin_status pin_deformation_tensor(pin_plan plan, const void* dk, int r, void* T6, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (r < -1 || r >= plan->nr) fail(PIN_ERR_INVALID_ARG, "radius index must be -1 or in [0, n_radii)");
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_device_range(T6, 6 * plan->real_field_bytes(), "T6");
    const void* w = r < 0 ? nullptr : static_cast<const char*>(plan->wtab) + (size_t)r * plan->n * plan->real_bytes;
    prep_hessian_input(plan, dk, stream);
    plan->launch(KC_XPASS_HESS, stream, [&] { plan->ops->xpass(0, plan->G, plan->X, w, plan->tw, 1.0, stream); });
    plan->launch(KC_YPASS_HESS, stream, [&] { plan->ops->ypass(0, plan->X, plan->Y, plan->tw, stream); });
    plan->launch(KC_ZPASS_STORE, stream, [&] { plan->ops->zpass_store(6, plan->Y, plan->tw, T6, stream); });
  });
}

pin_status pin_displacements(pin_plan plan, const void* dk, void* psi1, void* psi2, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    if (psi1 == nullptr && psi2 == nullptr) fail(PIN_ERR_INVALID_ARG, "psi1 and psi2 are both NULL");
    if (psi1) check_device_range(psi1, 3 * plan->real_field_bytes(), "psi1");
    if (psi2) check_device_range(psi2, 3 * plan->real_field_bytes(), "psi2");
    const double n3 = (double)plan->n * plan->n * plan->n;
    const double lfac = plan->box / (2.0 * 3.14159265358979323846);
    pin_plan p = plan;
    hipStream_t s = stream;
    if (psi1) {
      // psi1(k) = i (L/2pi) f dk / f^2
      p->launch(KC_XPASS_GRAD, s, [&] { p->ops->xpass(1, dk, p->X, nullptr, p->tw, lfac / n3, s); });
      p->launch(KC_YPASS_GRAD, s, [&] { p->ops->ypass(1, p->X, p->Y, p->tw, s); });
      p->launch(KC_ZPASS_STORE, s, [&] { p->ops->zpass_store(3, p->Y, p->tw, psi1, s); });
    }
    if (psi2) {
      // mu2 of the unsmoothed tensor, forward along z (fused), y, x; then (3/7) i (L/2pi) f / f^2
      // and the inverse gradient transforms.
      prep_hessian_input(p, dk, s);
      p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, nullptr, p->tw, 1.0, s); });
      p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
      p->launch(KC_ZPASS_MU2, s, [&] { p->ops->zpass_mu2(p->Y, p->tw, p->xslot(0), s); });
      p->launch(KC_YPASS_FWD, s, [&] { p->ops->ypass(2, p->xslot(0), p->xslot(1), p->tw, s); });
      p->launch(KC_XPASS_FWDINV, s,
                [&] { p->ops->xpass_fwdinv(p->xslot(1), p->Y, p->tw, (3.0 / 7.0) * lfac / n3, s); });
      p->launch(KC_YPASS_GRAD, s, [&] { p->ops->ypass(1, p->Y, p->X, p->tw, s); });
      p->launch(KC_ZPASS_STORE, s, [&] { p->ops->zpass_store(3, p->X, p->tw, psi2, s); });
    }
  });
}

pin_status pin_inverse_collapse_time(pin_plan plan, const void* T6, size_t count, void* F, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (count == 0) return;
    if (count > ((size_t)1 << 40)) fail(PIN_ERR_INVALID_ARG, "count is too large");
    check_device_range(T6, 6 * count * plan->real_bytes, "T6");
    check_device_range(F, count * plan->real_bytes, "F");
    plan->launch(KC_COLLAPSE_POINTS, stream,
                 [&] { plan->ops->collapse_points(T6, count, F, plan->sphere_gain, stream); });
  });
}

int pin_kernel_class_count(void) { return KC_COUNT; }

const char* pin_kernel_class_name(int cls) {
  if (cls < 0 || cls >= KC_COUNT) return "invalid";
  return kClassNames[cls];
}

pin_status pin_plan_set_timing(pin_plan plan, int enable) {
  return guarded([&] {
    check_plan(plan);
    for (auto& v : plan->events)
      for (auto& pr : v) hip_check(hipEventSynchronize(pr.second), "hipEventSynchronize");
    plan->recycle_events();
    plan->timing = enable != 0;
  });
}

pin_status pin_plan_kernel_time(pin_plan plan, int cls, double* total_ms, long long* launches) {
  return guarded([&] {
    check_plan(plan);
    if (cls < 0 || cls >= KC_COUNT) fail(PIN_ERR_INVALID_ARG, "kernel class out of range");
    if (total_ms == nullptr || launches == nullptr) fail(PIN_ERR_INVALID_ARG, "output pointer is NULL");
    double sum = 0.0;
    for (auto& pr : plan->events[cls]) {
      hip_check(hipEventSynchronize(pr.second), "hipEventSynchronize");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
      sum += ms;
    }
    *total_ms = sum;
    *launches = (long long)plan->events[cls].size();
  });
}

const char* pin_status_string(pin_status s) {
  switch (s) {
    case PIN_OK: return "ok";
    case PIN_ERR_INVALID_ARG: return "invalid argument";
    case PIN_ERR_UNSUPPORTED_SIZE: return "unsupported grid size";
    case PIN_ERR_OUT_OF_MEMORY: return "out of memory";
    case PIN_ERR_DEVICE: return "device error";
    case PIN_ERR_NOT_READY: return "not ready";
    case PIN_ERR_BUDGET: return "request exceeds the HBM budget";
    case PIN_ERR_CANCELLED: return "cancelled";
    case PIN_ERR_SHUTDOWN: return "server shutting down";
    case PIN_ERR_TIMEOUT: return "timed out";
  }
  return "unknown status";
}

const char* pin_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
