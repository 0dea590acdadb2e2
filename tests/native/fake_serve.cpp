// Host-only test double of the serving executor: the scheduler core of the library (same source,
// serve_core.hpp and serve_api.inc) driven by an executor that "runs" a request for a fixed
// number of scheduler polls, with failures injectable from the test.  Built by the CPU tests
// with g++; never part of libpin.so.
#include <atomic>
#include <cstring>
#include <string>
#include <vector>

#include "serve_core.hpp"

namespace {

thread_local std::string g_err;
std::atomic<int> g_polls{3};
std::atomic<unsigned long long> g_fail_launch_seed{0}, g_fail_poll_seed{0};
std::atomic<int> g_fail_create{0};
std::atomic<long long> g_creates{0}, g_destroys{0};

bool size_ok(int n) {
  if (n < 8 || n > 1024 || n % 2) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  return m == 1;
}

}  // namespace

struct FakeSlot {
  int n = 0;
  int remaining = 0;
  unsigned long long seed = 0;
  std::vector<char> F, ridx, psi;
};

class FakeExec {
 public:
  using Slot = FakeSlot;
  explicit FakeExec(const pin_serve_config&) {}

  pin_status validate(int n, double box, int nr, const double* radii, std::string& why) {
    if (!size_ok(n)) return why = "unsupported grid size", PIN_ERR_UNSUPPORTED_SIZE;
    if (!(box > 0)) return why = "box must be positive", PIN_ERR_INVALID_ARG;
    if (nr < 1 || nr > 254 || radii == nullptr) return why = "bad radii", PIN_ERR_INVALID_ARG;
    for (int i = 0; i < nr; ++i)
      if (!(radii[i] > 0) || (i && !(radii[i] < radii[i - 1]))) return why = "bad radii", PIN_ERR_INVALID_ARG;
    return PIN_OK;
  }
  size_t slot_bytes(int n) const { return (size_t)n * n * n; }
  Slot* create_slot(int n) {
    if (g_fail_create.load()) throw pin::PinError(PIN_ERR_OUT_OF_MEMORY, "injected allocation failure");
    ++g_creates;
    auto* s = new FakeSlot();
    s->n = n;
    s->F.resize(16);
    s->ridx.resize(16);
    s->psi.resize(16);
    return s;
  }
  void destroy_slot(Slot* s) {
    ++g_destroys;
    delete s;
  }
  void launch(Slot* s, uint64_t seed, double, const std::vector<double>&, int) {
    if (g_fail_launch_seed.load() && seed == g_fail_launch_seed.load())
      throw pin::PinError(PIN_ERR_DEVICE, "injected launch failure");
    s->seed = seed;
    s->remaining = g_polls.load();
  }
  int poll(Slot* s, std::string& err) {
    if (g_fail_poll_seed.load() && s->seed == g_fail_poll_seed.load()) {
      err = "injected device error";
      return -1;
    }
    if (s->remaining > 0) {
      --s->remaining;
      return 0;
    }
    return 1;
  }
  void results(Slot* s, int want_disp, pin_result* out) {
    out->F = s->F.data();
    out->ridx = reinterpret_cast<const uint8_t*>(s->ridx.data());
    out->psi1 = want_disp ? s->psi.data() : nullptr;
    out->psi2 = want_disp ? s->psi.data() : nullptr;
  }
  void set_error(const std::string& m) { g_err = m; }
};

using ServeExec = FakeExec;
static ServeExec serve_make_exec(const pin_serve_config& c) { return ServeExec(c); }
static void serve_set_error(const std::string& m) { g_err = m; }

#include "serve_api.inc"

extern "C" {
const char* pin_last_error(void) { return g_err.c_str(); }
void pin_fake_configure(int polls, unsigned long long fail_launch_seed, unsigned long long fail_poll_seed,
                        int fail_create) {
  g_polls = polls;
  g_fail_launch_seed = fail_launch_seed;
  g_fail_poll_seed = fail_poll_seed;
  g_fail_create = fail_create;
}
long long pin_fake_slot_creates(void) { return g_creates.load(); }
long long pin_fake_slot_destroys(void) { return g_destroys.load(); }
}
