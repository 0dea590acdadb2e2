// Plan creation, tables and the launch sequences of the path.
#include "plan.hpp"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdio>
#include <new>

#include "host_math.hpp"

namespace pin {

namespace {
thread_local std::string g_last_error;

// A host-side roctx range around the enqueue of one step of the path: rocprofv3 --marker-trace
// shows it beside the kernels it launched.
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  Range(const char* what, int n, int r) {
    char name[64];
    std::snprintf(name, sizeof name, "%s N=%d r=%d", what, n, r);
    roctxRangePushA(name);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Copy a float64 host table to the device in the plan's precision; waits for the copy (the host
// staging buffer is local).
void upload(void* dst, const std::vector<double>& src, bool fp64, hipStream_t s) {
  std::vector<float> f;
  const void* host = src.data();
  size_t bytes = src.size() * sizeof(double);
  if (!fp64) {
    f.assign(src.begin(), src.end());
    host = f.data();
    bytes = f.size() * sizeof(float);
  }
  hip_check(hipMemcpyAsync(dst, host, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

void prep_hessian_input(pin_plan p, const void* dk, hipStream_t s) {
  const double scale = 1.0 / ((double)p->n * p->n * p->n);
  p->launch(KC_PREP, s, [&] { p->ops->prep(dk, p->G, scale, s); });
}
}  // namespace

const char* const kClassNames[KC_COUNT] = {
    "grf",           "reset",          "xpass_hessian", "ypass_hessian", "zpass_collapse",
    "zpass_store",   "xpass_gradient", "ypass_gradient", "zpass_mu2",    "ypass_forward",
    "xpass_fwdinv",  "collapse_points", "prep",          "ypass_velocity", "zpass_collapse_v",
    "zero",          "redshift",       "zpass_mu2_store", "xpass_fwdinv_hessian", "zpass_lpt3",
    "xpass_lpt3",    "ypass_lpt3"};

void fail(pin_status s, const std::string& m) { throw PinError(s, m); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(PIN_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void set_last_error(const std::string& m) { g_last_error = m; }
const char* last_error() { return g_last_error.c_str(); }

void* device_alloc(size_t bytes, const char* what) {
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(PIN_ERR_OUT_OF_MEMORY, std::string("hipMalloc(") + what + ", " + std::to_string(bytes) + " bytes) failed");
  }
  return p;
}

bool size_supported(int n) { return find_ops(n, false) != nullptr; }

void validate_desc(const pin_plan_desc* d) {
  if (d == nullptr) fail(PIN_ERR_INVALID_ARG, "desc is NULL");
  if (!size_supported(d->n)) fail(PIN_ERR_UNSUPPORTED_SIZE, "unsupported grid size N=" + std::to_string(d->n));
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

size_t workspace_bytes(int n, int n_radii, bool fp64) {
  const size_t rb = fp64 ? 8 : 4;
  const size_t slot = (size_t)n * n * (n / 2) * 2 * rb;
  // workspace slots, twiddles, one window row per radius plus a row of ones (no smoothing)
  return 11 * slot + (size_t)n * 2 * rb + (size_t)n * (n_radii + 1) * rb;
}

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

// The mode-amplitude table for the plan's current box: computed on the host (float64) and
// uploaded on first use of that box, kept for later calls; at most kAmpTables boxes are kept,
// the oldest freed first (hipFree waits for any kernel still reading it).
constexpr size_t kAmpTables = 8;
static const double* amp_table(pin_plan p) {
  for (auto& t : p->amp_tables)
    if (t.first == p->box) return static_cast<const double*>(t.second);
  if (p->amp_tables.size() >= kAmpTables) {
    (void)hipFree(p->amp_tables.front().second);
    p->amp_tables.erase(p->amp_tables.begin());
  }
  const std::vector<double> a = mode_amplitudes(p->n, p->box, p->amplitude, p->gamma, p->ns);
  void* d = device_alloc(a.size() * sizeof(double), "mode amplitudes");
  const hipError_t e = hipMemcpy(d, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    hip_check(e, "hipMemcpy");
  }
  p->amp_tables.emplace_back(p->box, d);
  return static_cast<const double*>(d);
}

pin_plan plan_create(const pin_plan_desc* desc, int radii_capacity) {
  validate_desc(desc);
  if (radii_capacity < desc->n_radii) radii_capacity = desc->n_radii;
  pin_plan p = new pin_plan_s();
  try {
    p->n = desc->n;
    p->nr = desc->n_radii;
    p->nr_capacity = radii_capacity;
    p->box = desc->box;
    p->sigma8 = desc->sigma8;
    p->gamma = desc->gamma;
    p->ns = desc->ns;
    p->fp64 = desc->prec == PIN_FP64;
    p->real_bytes = p->fp64 ? 8 : 4;
    p->ops = find_ops(p->n, p->fp64);
    p->amplitude = amplitude_for_sigma8(p->sigma8, p->gamma, p->ns);
    p->sphere_gain = eds_sphere_root() / eds_delta_c() - 1.0;
    hip_check(hipGetDevice(&p->device), "hipGetDevice");
    p->slot_bytes = (size_t)p->n * p->n * (p->n / 2) * p->complex_bytes();
    p->tw = device_alloc((size_t)p->n * p->complex_bytes(), "twiddles");
    p->wtab = device_alloc((size_t)p->n * (p->nr_capacity + 1) * p->real_bytes, "windows");
    p->X = device_alloc(4 * p->slot_bytes, "workspace X");
    p->Y = device_alloc(6 * p->slot_bytes, "workspace Y");
    p->G = device_alloc(p->slot_bytes, "workspace G");
    upload(p->tw, twiddles(p->n), p->fp64, nullptr);
    (void)amp_table(p);
    upload(p->window_row(p->nr_capacity), std::vector<double>((size_t)p->n, 1.0), p->fp64, nullptr);
    plan_set_radii(p, desc->radii_cells, desc->n_radii, nullptr);
  } catch (...) {
    plan_free(p);
    throw;
  }
  return p;
}

void plan_free(pin_plan p) {
  if (p == nullptr) return;
  for (auto& v : p->events)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  if (p->tw) (void)hipFree(p->tw);
  for (auto& t : p->amp_tables) (void)hipFree(t.second);
  if (p->wtab) (void)hipFree(p->wtab);
  if (p->X) (void)hipFree(p->X);
  if (p->Y) (void)hipFree(p->Y);
  if (p->G) (void)hipFree(p->G);
  if (p->V) (void)hipFree(p->V);
  if (p->L) (void)hipFree(p->L);
  fragment_free(p->frag);
  if (p->growth) (void)hipFree(p->growth);
  delete p;
}

void plan_set_radii(pin_plan p, const double* radii, int n_radii, hipStream_t s) {
  if (n_radii < 1 || n_radii > p->nr_capacity) fail(PIN_ERR_INVALID_ARG, "radius count exceeds the plan capacity");
  std::vector<double> w;
  w.reserve((size_t)p->n * n_radii);
  for (int r = 0; r < n_radii; ++r) {
    const auto wr = gaussian_window_table(p->n, radii[r]);
    w.insert(w.end(), wr.begin(), wr.end());
  }
  upload(p->wtab, w, p->fp64, s);
  p->radii.assign(radii, radii + n_radii);
  p->nr = n_radii;
}

void plan_generate_field(pin_plan p, uint64_t seed, void* dk, hipStream_t s) {
  Range range("pin field");
  const double* amp = amp_table(p);
  p->launch(KC_GRF, s, [&] { p->ops->grf(dk, seed, amp, s); });
}

void plan_reset(pin_plan p, void* F, uint8_t* ridx, hipStream_t s) {
  p->launch(KC_RESET, s, [&] { p->ops->reset(F, ridx, s); });
}

void plan_run_radii(pin_plan p, const void* dk, void* F, uint8_t* ridx, int r0, int r1, hipStream_t s) {
  prep_hessian_input(p, dk, s);
  for (int r = r0; r < r1; ++r) {
    Range range("pin radius", p->n, r);
    const void* w = p->window_row(r);
    p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, w, p->tw, 1.0, s); });
    p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
    p->launch(KC_ZPASS_COLLAPSE, s, [&] { p->ops->zpass_collapse(p->Y, p->tw, F, ridx, r, p->sphere_gain, s); });
  }
}

size_t velocity_workspace_bytes(int n, bool fp64) {
  const size_t rb = fp64 ? 8 : 4;
  return 4 * (size_t)n * n * (n / 2) * 2 * rb;
}

void plan_reset_v(pin_plan p, void* F, uint8_t* ridx, void* vmax, hipStream_t s) {
  plan_reset(p, F, ridx, s);
  p->launch(KC_ZERO, s, [&] { p->ops->zero(vmax, 3 * (size_t)p->n * p->n * p->n, s); });
}

void plan_run_radii_v(pin_plan p, const void* dk, void* F, uint8_t* ridx, void* vmax, int r0, int r1, hipStream_t s) {
  if (p->V == nullptr) p->V = device_alloc(velocity_workspace_bytes(p->n, p->fp64), "workspace V");
  const double vscale = p->box / (2.0 * 3.14159265358979323846);
  prep_hessian_input(p, dk, s);
  for (int r = r0; r < r1; ++r) {
    const void* w = p->window_row(r);
    p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, w, p->tw, 1.0, s); });
    p->launch(KC_YPASS_VEL, s, [&] { p->ops->ypass_hess_grad(p->X, p->Y, p->V, p->tw, s); });
    p->launch(KC_ZPASS_COLLAPSE_V, s, [&] {
      p->ops->zpass_collapse_v(p->Y, p->V, p->tw, F, ridx, vmax, r, p->sphere_gain, vscale, s);
    });
  }
}

void plan_deformation_tensor(pin_plan p, const void* dk, int r, void* T6, hipStream_t s) {
  const void* w = p->window_row(r < 0 ? p->nr_capacity : r);
  prep_hessian_input(p, dk, s);
  p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, w, p->tw, 1.0, s); });
  p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
  p->launch(KC_ZPASS_STORE, s, [&] { p->ops->zpass_store(6, p->Y, p->tw, T6, s); });
}

void plan_displacements(pin_plan p, const void* dk, void* psi1, void* psi2, hipStream_t s) {
  Range range("pin displacements");
  const double n3 = (double)p->n * p->n * p->n;
  const double lfac = p->box / (2.0 * 3.14159265358979323846);
  if (psi1) {
    // psi1(k) = i (L/2pi) f dk / f^2
    p->launch(KC_XPASS_GRAD, s, [&] { p->ops->xpass(1, dk, p->X, nullptr, p->tw, lfac / n3, s); });
    p->launch(KC_YPASS_GRAD, s, [&] { p->ops->ypass(1, p->X, p->Y, p->tw, s); });
    p->launch(KC_ZPASS_STORE, s, [&] { p->ops->zpass_store(3, p->Y, p->tw, psi1, s); });
  }
  if (psi2) {
    // mu2 of the unsmoothed tensor, forward along z (fused into the z pass), y, x; then
    // (3/7) i (L/2pi) f / f^2 and the inverse gradient transforms.
    prep_hessian_input(p, dk, s);
    const void* ones = p->window_row(p->nr_capacity);
    p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, ones, p->tw, 1.0, s); });
    p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
    p->launch(KC_ZPASS_MU2, s, [&] { p->ops->zpass_mu2(p->Y, p->tw, p->xslot(0), nullptr, s); });
    p->launch(KC_YPASS_FWD, s, [&] { p->ops->ypass(2, p->xslot(0), p->xslot(1), p->tw, s); });
    p->launch(KC_XPASS_FWDINV, s,
              [&] { p->ops->xpass_fwdinv(false, p->xslot(1), p->Y, p->tw, (3.0 / 7.0) * lfac / n3, s); });
    p->launch(KC_YPASS_GRAD, s, [&] { p->ops->ypass(1, p->Y, p->X, p->tw, s); });
    p->launch(KC_ZPASS_STORE, s, [&] { p->ops->zpass_store(3, p->X, p->tw, psi2, s); });
  }
}

size_t lpt3_workspace_bytes(int n, bool fp64) {
  const size_t rb = fp64 ? 8 : 4;
  return 10 * (size_t)n * n * (n / 2) * 2 * rb;
}

void plan_lpt3_displacement(pin_plan p, const void* dk, void* psi3, hipStream_t s) {
  Range range("pin 3lpt displacement");
  if (p->L == nullptr) p->L = device_alloc(lpt3_workspace_bytes(p->n, p->fp64), "workspace L");
  const double n3 = (double)p->n * p->n * p->n;
  const double lfac = p->box / (2.0 * 3.14159265358979323846);
  auto lslot = [&](int i) { return static_cast<char*>(p->L) + (size_t)i * p->slot_bytes; };
  // T1 (unsmoothed Hessian of phi1) stored as six real fields in L[0..5], and mu2(T1) forward
  // along z into L[6]; forward y into L[7]
  prep_hessian_input(p, dk, s);
  const void* ones = p->window_row(p->nr_capacity);
  p->launch(KC_XPASS_HESS, s, [&] { p->ops->xpass(0, p->G, p->X, ones, p->tw, 1.0, s); });
  p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
  p->launch(KC_ZPASS_MU2_STORE, s, [&] { p->ops->zpass_mu2(p->Y, p->tw, lslot(6), lslot(0), s); });
  p->launch(KC_YPASS_FWD, s, [&] { p->ops->ypass(2, lslot(6), lslot(7), p->tw, s); });
  // T2 (Hessian of phi2, lap phi2 = mu2): forward x, M / f^2 and the Hessian x outputs, then the
  // Hessian y pass; its z pass forms the third-order sources with T1 and transforms them forward
  // along z into L[6..9]
  p->launch(KC_XPASS_FWDINV_HESS, s, [&] { p->ops->xpass_fwdinv(true, lslot(7), p->X, p->tw, 1.0 / n3, s); });
  p->launch(KC_YPASS_HESS, s, [&] { p->ops->ypass(0, p->X, p->Y, p->tw, s); });
  p->launch(KC_ZPASS_LPT3, s, [&] { p->ops->zpass_lpt3(p->Y, lslot(0), p->tw, lslot(6), s); });
  // sources forward along y into X[0..3], then forward x, the psi3 multipliers and the inverse
  // x transforms into Y[0..2], the inverse y (packed) into X and the inverse z into psi3
  for (int i = 0; i < 4; ++i)
    p->launch(KC_YPASS_FWD, s, [&] { p->ops->ypass(2, lslot(6 + i), p->xslot(i), p->tw, s); });
  p->launch(KC_XPASS_LPT3, s, [&] { p->ops->xpass_lpt3(p->X, p->Y, p->tw, lfac / n3, s); });
  p->launch(KC_YPASS_LPT3, s, [&] { p->ops->ypass(4, p->Y, p->X, p->tw, s); });
  p->launch(KC_ZPASS_STORE, s, [&] { p->ops->zpass_store(3, p->X, p->tw, psi3, s); });
}

}  // namespace pin

hipEvent_t pin_plan_s::take_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  pin::hip_check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void pin_plan_s::recycle_events() {
  for (auto& v : events) {
    for (auto& pr : v) {
      pool.push_back(pr.first);
      pool.push_back(pr.second);
    }
    v.clear();
  }
}
