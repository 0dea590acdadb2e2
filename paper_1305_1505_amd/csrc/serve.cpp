// HIP executor of the serving scheduler: slots are plans plus per-request buffers and a stream;
// a request is the field kernel followed by one captured hipGraph of the rest of its path.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>
#include <map>
#include <tuple>

#include "plan.hpp"
#include "serve_core.hpp"

namespace pin {
namespace serve {

struct HipSlot {
  int n = 0;
  pin_plan plan = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* dk = nullptr;
  void* F = nullptr;
  uint8_t* ridx = nullptr;
  void* psi1 = nullptr;
  void* psi2 = nullptr;
  // captured graphs by (n_radii, box, want_disp), with the launch count of their last use; at
  // most kMaxGraphs, the least recently used dropped first
  std::map<std::tuple<int, double, int>, std::pair<hipGraphExec_t, uint64_t>> graphs;
  uint64_t launches = 0;
  // roctx range from the request's launch to the poll that sees it done (0: none open)
  roctx_range_id_t range = 0;
};

class HipExec {
 public:
  using Slot = HipSlot;
  static constexpr int kMaxRadii = 254;
  static constexpr size_t kMaxGraphs = 16;

  explicit HipExec(const pin_serve_config& c) : cfg_(c) {}

  pin_status validate(int n, double box, int n_radii, const double* radii, std::string& why) {
    pin_plan_desc d{n, box, n_radii, radii, cfg_.sigma8, cfg_.gamma, cfg_.ns, cfg_.prec};
    try {
      validate_desc(&d);
    } catch (const PinError& e) {
      why = e.msg;
      return e.status;
    }
    return PIN_OK;
  }

  size_t slot_bytes(int n) const {
    const size_t rb = cfg_.prec == PIN_FP64 ? 8 : 4;
    const size_t vol = (size_t)n * n * n;
    return workspace_bytes(n, kMaxRadii, cfg_.prec == PIN_FP64) + (size_t)n * n * (n / 2 + 1) * 2 * rb +
           vol * (rb + 1) + 6 * vol * rb;
  }

  Slot* create_slot(int n) {
    hip_check(hipSetDevice(cfg_.device), "hipSetDevice");
    const double r0 = 1.0;
    pin_plan_desc d{n, 1.0, 1, &r0, cfg_.sigma8, cfg_.gamma, cfg_.ns, cfg_.prec};
    auto* s = new HipSlot();
    try {
      s->n = n;
      s->plan = plan_create(&d, kMaxRadii);
      const size_t rb = s->plan->real_bytes;
      const size_t vol = (size_t)n * n * n;
      hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreateWithFlags");
      hip_check(hipEventCreateWithFlags(&s->done, hipEventDisableTiming), "hipEventCreateWithFlags");
      s->dk = device_alloc(s->plan->half_spectrum_bytes(), "slot field");
      s->F = device_alloc(vol * rb, "slot F");
      s->ridx = static_cast<uint8_t*>(device_alloc(vol, "slot ridx"));
      s->psi1 = device_alloc(3 * vol * rb, "slot psi1");
      s->psi2 = device_alloc(3 * vol * rb, "slot psi2");
    } catch (...) {
      destroy_slot(s);
      throw;
    }
    return s;
  }

  void destroy_slot(Slot* s) {
    if (s == nullptr) return;
    (void)hipSetDevice(cfg_.device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second.first);
    for (void* p : {s->dk, s->F, (void*)s->ridx, s->psi1, s->psi2})
      if (p) (void)hipFree(p);
    if (s->done) (void)hipEventDestroy(s->done);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    plan_free(s->plan);
    delete s;
  }

  void launch(Slot* s, uint64_t seed, double box, const std::vector<double>& radii, int want_disp) {
    hip_check(hipSetDevice(cfg_.device), "hipSetDevice");
    char name[96];
    std::snprintf(name, sizeof name, "pin request N=%d radii=%d seed=%llu", s->n, (int)radii.size(),
                  (unsigned long long)seed);
    s->range = roctxRangeStartA(name);
    pin_plan p = s->plan;
    plan_set_radii(p, radii.data(), (int)radii.size(), s->stream);
    p->box = box;
    plan_generate_field(p, seed, s->dk, s->stream);
    const auto key = std::make_tuple((int)radii.size(), box, want_disp);
    auto it = s->graphs.find(key);
    if (it == s->graphs.end()) {
      if (s->graphs.size() >= kMaxGraphs) {
        // the slot is idle (its previous request completed), so no graph of it is in flight
        auto old = s->graphs.begin();
        for (auto g = s->graphs.begin(); g != s->graphs.end(); ++g)
          if (g->second.second < old->second.second) old = g;
        (void)hipGraphExecDestroy(old->second.first);
        s->graphs.erase(old);
      }
      it = s->graphs.emplace(key, std::make_pair(capture(s, want_disp), uint64_t(0))).first;
    }
    it->second.second = ++s->launches;
    hip_check(hipGraphLaunch(it->second.first, s->stream), "hipGraphLaunch");
    hip_check(hipEventRecord(s->done, s->stream), "hipEventRecord");
  }

  int poll(Slot* s, std::string& err) {
    const hipError_t e = hipEventQuery(s->done);
    if (e == hipErrorNotReady) return 0;
    if (s->range != 0) {
      roctxRangeStop(s->range);
      s->range = 0;
    }
    if (e == hipSuccess) return 1;
    (void)hipGetLastError();
    err = std::string("device error: ") + hipGetErrorString(e);
    return -1;
  }

  void results(Slot* s, int want_disp, pin_result* out) {
    out->F = s->F;
    out->ridx = s->ridx;
    out->psi1 = want_disp ? s->psi1 : nullptr;
    out->psi2 = want_disp ? s->psi2 : nullptr;
  }

  void set_error(const std::string& m) { set_last_error(m); }

 private:
  // The seed-independent rest of the path (reset, every radius, displacements) as one graph on
  // the slot's buffers; no memset nodes (the reset is a kernel).
  hipGraphExec_t capture(Slot* s, int want_disp) {
    pin_plan p = s->plan;
    hip_check(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      plan_reset(p, s->F, s->ridx, s->stream);
      plan_run_radii(p, s->dk, s->F, s->ridx, 0, p->nr, s->stream);
      if (want_disp) plan_displacements(p, s->dk, s->psi1, s->psi2, s->stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(s->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipGraph_t g = nullptr;
    hip_check(hipStreamEndCapture(s->stream, &g), "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "hipGraphInstantiate");
    return ge;
  }

  pin_serve_config cfg_;
};

}  // namespace serve
}  // namespace pin

using ServeExec = pin::serve::HipExec;
static ServeExec serve_make_exec(const pin_serve_config& c) { return ServeExec(c); }
static void serve_set_error(const std::string& m) { pin::set_last_error(m); }

#include "serve_api.inc"
