// C ABI of libpin (include/pin.h): argument validation around the plan operations of plan.cpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <initializer_list>
#include <vector>

#include "pin.h"
#include "host_math.hpp"
#include "plan.hpp"

using namespace pin;

namespace {

void check_plan(pin_plan p) {
  if (p == nullptr) fail(PIN_ERR_INVALID_ARG, "plan is NULL");
}

void check_field_outputs(pin_plan p, const void* F, const void* ridx) {
  check_device_range(F, p->real_field_bytes(), "F");
  check_device_range(ridx, (size_t)p->n * p->n * p->n, "ridx");
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
    *bytes = workspace_bytes(desc->n, desc->n_radii, desc->prec == PIN_FP64);
  });
}

pin_status pin_plan_create(const pin_plan_desc* desc, pin_plan* out) {
  return guarded([&] {
    if (out == nullptr) fail(PIN_ERR_INVALID_ARG, "out is NULL");
    *out = plan_create(desc, desc ? desc->n_radii : 0);
  });
}

pin_status pin_plan_set_radii(pin_plan plan, const double* radii_cells, int n_radii, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    pin_plan_desc d{plan->n, 1.0, n_radii, radii_cells, plan->sigma8, plan->gamma, plan->ns,
                    plan->fp64 ? PIN_FP64 : PIN_FP32};
    validate_desc(&d);
    if (n_radii > plan->nr_capacity) fail(PIN_ERR_INVALID_ARG, "n_radii exceeds the count the plan was created with");
    plan_set_radii(plan, radii_cells, n_radii, stream);
  });
}

pin_status pin_plan_destroy(pin_plan plan) {
  return guarded([&] {
    check_plan(plan);
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    plan_free(plan);
  });
}

pin_status pin_generate_field(pin_plan plan, uint64_t seed, void* dk, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    plan_generate_field(plan, seed, dk, stream);
  });
}

pin_status pin_collapse_reset(pin_plan plan, void* F, uint8_t* ridx, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_field_outputs(plan, F, ridx);
    plan_reset(plan, F, ridx, stream);
  });
}

pin_status pin_collapse_times_range(pin_plan plan, const void* dk, void* F, uint8_t* ridx, int r_begin, int r_end,
                                    hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (r_begin < 0 || r_end > plan->nr || r_begin >= r_end)
      fail(PIN_ERR_INVALID_ARG, "radius range must satisfy 0 <= r_begin < r_end <= n_radii");
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_field_outputs(plan, F, ridx);
    plan_run_radii(plan, dk, F, ridx, r_begin, r_end, stream);
  });
}

pin_status pin_collapse_times(pin_plan plan, const void* dk, void* F, uint8_t* ridx, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_field_outputs(plan, F, ridx);
    plan_reset(plan, F, ridx, stream);
    plan_run_radii(plan, dk, F, ridx, 0, plan->nr, stream);
  });
}

pin_status pin_plan_velocity_workspace_bytes(const pin_plan_desc* desc, size_t* bytes) {
  return guarded([&] {
    validate_desc(desc);
    if (bytes == nullptr) fail(PIN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = velocity_workspace_bytes(desc->n, desc->prec == PIN_FP64);
  });
}

pin_status pin_collapse_reset_v(pin_plan plan, void* F, uint8_t* ridx, void* vmax, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_field_outputs(plan, F, ridx);
    check_device_range(vmax, 3 * plan->real_field_bytes(), "vmax");
    plan_reset_v(plan, F, ridx, vmax, stream);
  });
}

pin_status pin_collapse_times_range_v(pin_plan plan, const void* dk, void* F, uint8_t* ridx, void* vmax, int r_begin,
                                      int r_end, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (r_begin < 0 || r_end > plan->nr || r_begin >= r_end)
      fail(PIN_ERR_INVALID_ARG, "radius range must satisfy 0 <= r_begin < r_end <= n_radii");
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_field_outputs(plan, F, ridx);
    check_device_range(vmax, 3 * plan->real_field_bytes(), "vmax");
    plan_run_radii_v(plan, dk, F, ridx, vmax, r_begin, r_end, stream);
  });
}

pin_status pin_collapse_times_v(pin_plan plan, const void* dk, void* F, uint8_t* ridx, void* vmax, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_field_outputs(plan, F, ridx);
    check_device_range(vmax, 3 * plan->real_field_bytes(), "vmax");
    plan_reset_v(plan, F, ridx, vmax, stream);
    plan_run_radii_v(plan, dk, F, ridx, vmax, 0, plan->nr, stream);
  });
}

pin_status pin_plan_set_growth(pin_plan plan, double omega_m, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (!(omega_m > 0.0 && omega_m <= 1.0)) fail(PIN_ERR_INVALID_ARG, "omega_m must be in (0, 1]");
    const GrowthTable g = growth_table(omega_m);
    std::vector<double> host(g.d);
    host.insert(host.end(), g.dd.begin(), g.dd.end());
    const size_t nd = host.size() * sizeof(double), ng = g.guide.size() * sizeof(int32_t);
    std::vector<unsigned char> bytes(nd + ng);
    std::memcpy(bytes.data(), host.data(), nd);
    std::memcpy(bytes.data() + nd, g.guide.data(), ng);
    if (plan->growth == nullptr) plan->growth = device_alloc(bytes.size(), "growth table");
    hip_check(hipMemcpyAsync(plan->growth, bytes.data(), bytes.size(), hipMemcpyHostToDevice, stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    plan->growth_y0 = g.y0;
    plan->growth_h = g.h;
    plan->growth_a_per_D = g.a_per_D;
    plan->growth_lom = g.lambda_over_m;
    plan->growth_gl0 = g.guide_l0;
    plan->growth_ginv = g.guide_inv;
  });
}

pin_status pin_collapse_redshift(pin_plan plan, const void* F, size_t count, void* zc, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (plan->growth == nullptr) fail(PIN_ERR_INVALID_ARG, "no growth table: call pin_plan_set_growth first");
    if (count == 0) return;
    if (count > ((size_t)1 << 40)) fail(PIN_ERR_INVALID_ARG, "count is too large");
    check_device_range(F, count * plan->real_bytes, "F");
    check_device_range(zc, count * plan->real_bytes, "zc");
    const double* d = static_cast<const double*>(plan->growth);
    plan->launch(KC_REDSHIFT, stream, [&] {
      plan->ops->redshift(F, count, d, d + kGrowthNodes, kGrowthNodes, plan->growth_y0, plan->growth_h,
                          plan->growth_a_per_D, plan->growth_lom,
                          reinterpret_cast<const int32_t*>(d + 2 * kGrowthNodes), kGrowthGuide, plan->growth_gl0,
                          plan->growth_ginv, zc, stream);
    });
  });
}

pin_status pin_radius_ladder(int n, double box, double r_max_cells, double r_min_cells, double dex, double gamma,
                             double ns, double* radii_cells, int capacity, int* count) {
  return guarded([&] {
    if (n < 2 || !(box > 0.0)) fail(PIN_ERR_INVALID_ARG, "n must be >= 2 and box > 0");
    if (!(r_max_cells > r_min_cells && r_min_cells > 0.0)) fail(PIN_ERR_INVALID_ARG, "need r_max > r_min > 0");
    if (!(dex > 0.0)) fail(PIN_ERR_INVALID_ARG, "dex must be > 0");
    if (!(gamma > 0.0)) fail(PIN_ERR_INVALID_ARG, "gamma must be > 0");
    if (count == nullptr) fail(PIN_ERR_INVALID_ARG, "count is NULL");
    const std::vector<double> r = radius_ladder(n, box, r_max_cells, r_min_cells, dex, gamma, ns);
    *count = (int)r.size();
    if (radii_cells != nullptr) {
      if (capacity < (int)r.size()) fail(PIN_ERR_INVALID_ARG, "capacity is smaller than the ladder (see *count)");
      for (size_t i = 0; i < r.size(); ++i) radii_cells[i] = r[i];
    }
  });
}

pin_status pin_deformation_tensor(pin_plan plan, const void* dk, int r, void* T6, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (r < -1 || r >= plan->nr) fail(PIN_ERR_INVALID_ARG, "radius index must be -1 or in [0, n_radii)");
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_device_range(T6, 6 * plan->real_field_bytes(), "T6");
    plan_deformation_tensor(plan, dk, r, T6, stream);
  });
}

pin_status pin_displacements(pin_plan plan, const void* dk, void* psi1, void* psi2, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    if (psi1 == nullptr && psi2 == nullptr) fail(PIN_ERR_INVALID_ARG, "psi1 and psi2 are both NULL");
    if (psi1) check_device_range(psi1, 3 * plan->real_field_bytes(), "psi1");
    if (psi2) check_device_range(psi2, 3 * plan->real_field_bytes(), "psi2");
    plan_displacements(plan, dk, psi1, psi2, stream);
  });
}

void pin_fragment_default_params(pin_fragment_params* out) {
  if (out == nullptr) return;
  out->f_a = 0.285;
  out->f_ra = 0.180;
  out->f_s = 0.060;
  out->f_m = 0.350;
  out->f_rm = 0.700;
}

pin_status pin_plan_fragment_workspace_bytes(const pin_plan_desc* desc, size_t* bytes) {
  return guarded([&] {
    validate_desc(desc);
    if (bytes == nullptr) fail(PIN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = fragment_workspace_bytes(desc->n);
  });
}

pin_status pin_fragment(pin_plan plan, const void* F, const void* vmax, double f_min, const pin_fragment_params* params,
                        int32_t* label, int32_t* halo_size, int* n_halos, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (!(f_min > 0.0) || !std::isfinite(f_min)) fail(PIN_ERR_INVALID_ARG, "f_min must be positive and finite");
    pin_fragment_params prm;
    pin_fragment_default_params(&prm);
    if (params) prm = *params;
    for (double c : {prm.f_a, prm.f_ra, prm.f_s, prm.f_m, prm.f_rm})
      if (!(c >= 0.0) || !std::isfinite(c)) fail(PIN_ERR_INVALID_ARG, "fragmentation constants must be finite and >= 0");
    if (n_halos == nullptr) fail(PIN_ERR_INVALID_ARG, "n_halos is NULL");
    check_device_range(F, plan->real_field_bytes(), "F");
    check_device_range(vmax, 3 * plan->real_field_bytes(), "vmax");
    const size_t vol = (size_t)plan->n * plan->n * plan->n;
    check_device_range(label, vol * sizeof(int32_t), "label");
    if (halo_size) check_device_range(halo_size, vol * sizeof(int32_t), "halo_size");
    fragment_prepare(plan->frag, plan->n, plan->box, plan->amplitude, plan->gamma, plan->ns, stream);
    const FragParams fp{prm.f_a, prm.f_ra, prm.f_s, prm.f_m, prm.f_rm};
    *n_halos = fragment_run(plan->frag, plan->fp64, plan->n, F, vmax, plan->n / plan->box, f_min, fp, label,
                            halo_size, stream);
  });
}

pin_status pin_fragment_catalog(pin_plan plan, int32_t* id, int32_t* n_particles, double* centre, double* displacement,
                                int capacity, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (plan->frag.n_halos < 0) fail(PIN_ERR_INVALID_ARG, "no fragmentation result on this plan");
    if (capacity < plan->frag.n_halos) fail(PIN_ERR_INVALID_ARG, "capacity is smaller than the number of halos");
    const size_t cap = capacity > 0 ? (size_t)capacity : 1;
    check_device_range(id, cap * sizeof(int32_t), "id");
    check_device_range(n_particles, cap * sizeof(int32_t), "n_particles");
    check_device_range(centre, 3 * cap * sizeof(double), "centre");
    check_device_range(displacement, 3 * cap * sizeof(double), "displacement");
    fragment_catalog(plan->frag, plan->box / plan->n, id, n_particles, centre, displacement, capacity, stream);
  });
}

pin_status pin_fragment_mergers(pin_plan plan, double* f, int32_t* keep, int32_t* gone, int32_t* n_keep,
                                int32_t* n_gone, int capacity, int* count, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    if (count == nullptr) fail(PIN_ERR_INVALID_ARG, "count is NULL");
    if (plan->frag.n_halos < 0) fail(PIN_ERR_INVALID_ARG, "no fragmentation result on this plan");
    const int m = plan->frag.n_mergers;
    if (capacity == 0 && f == nullptr && keep == nullptr && gone == nullptr && n_keep == nullptr && n_gone == nullptr) {
      *count = m;   // query
      return;
    }
    if (capacity < m) fail(PIN_ERR_INVALID_ARG, "capacity is smaller than the number of mergers");
    if (m > 0) {
      check_device_range(f, (size_t)m * sizeof(double), "f");
      check_device_range(keep, (size_t)m * sizeof(int32_t), "keep");
      check_device_range(gone, (size_t)m * sizeof(int32_t), "gone");
      check_device_range(n_keep, (size_t)m * sizeof(int32_t), "n_keep");
      check_device_range(n_gone, (size_t)m * sizeof(int32_t), "n_gone");
    }
    *count = fragment_mergers(plan->frag, f, keep, gone, n_keep, n_gone, capacity, stream);
  });
}

pin_status pin_plan_lpt3_workspace_bytes(const pin_plan_desc* desc, size_t* bytes) {
  return guarded([&] {
    validate_desc(desc);
    if (bytes == nullptr) fail(PIN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = lpt3_workspace_bytes(desc->n, desc->prec == PIN_FP64);
  });
}

pin_status pin_lpt3_displacement(pin_plan plan, const void* dk, void* psi3, hipStream_t stream) {
  return guarded([&] {
    check_plan(plan);
    check_device_range(dk, plan->half_spectrum_bytes(), "dk");
    check_device_range(psi3, 3 * plan->real_field_bytes(), "psi3");
    plan_lpt3_displacement(plan, dk, psi3, stream);
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

const char* pin_last_error(void) { return last_error(); }

}  // extern "C"
