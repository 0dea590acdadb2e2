// Collapse times without device allocation (pin_collapse_times_noalloc).
//
// The same launches as pin_collapse_times on a plan (reset, then per radius the Hessian x, y and
// collapse z passes), but everything a plan would allocate -- the 11 half-spectrum workspace
// slots, the twiddle table and the window table -- lives in one file-scope device array.  Host
// code never passes that array's name to a kernel: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.  Tables are written on
// the caller's stream by two small kernels (twiddles computed on the host in extended precision
// and passed by value, windows computed on the device in float64), so the call queues kernels
// only: no allocation, no copy from host memory, no host wait.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "host_math.hpp"
#include "plan.hpp"

namespace {

// Largest scratch the library holds per device: enough for N = 128 in float32 (11 slots of
// 8 MiB plus tables) and N = 96 in float64.
constexpr size_t kScratchBytes = size_t(96) << 20;
// twiddles travel as kernel arguments: at most this many complex values
constexpr int kMaxN = 128;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace pin {
namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked up once.
void* scratch_address(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (p == nullptr) fail(PIN_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

struct TwiddleArgs {
  double v[2 * kMaxN];  // (cos, sin) of 2 pi m / N, m = 0..N-1
  int n;
};

struct WindowArgs {
  double radius[254];  // cells, one row per radius
  int n, nr;
};

template <typename R>
__global__ void k_noalloc_twiddles(R* tw, TwiddleArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * a.n) tw[i] = (R)a.v[i];
}

// W(kR) = exp(-k^2 R^2 / 2) on integer frequencies f = 0..N/2-1, -N/2..-1, row per radius
template <typename R>
__global__ void k_noalloc_windows(R* w, WindowArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n * a.nr) return;
  const int r = i / a.n, j = i - r * a.n;
  const double f = j < a.n / 2 ? j : j - a.n;
  const double kr = 2.0 * 3.14159265358979323846264338327950288 * f * a.radius[r] / a.n;
  w[i] = (R)exp(-0.5 * kr * kr);
}

template <typename R>
void write_tables(void* tw, void* wtab, const pin_plan_desc* d, hipStream_t s) {
  TwiddleArgs ta{};
  twiddles_into(d->n, ta.v);   // n <= kMaxN, checked by the caller
  ta.n = d->n;
  WindowArgs wa{};
  for (int r = 0; r < d->n_radii; ++r) wa.radius[r] = d->radii_cells[r];
  wa.n = d->n;
  wa.nr = d->n_radii;
  const int block = 256;
  hipLaunchKernelGGL(k_noalloc_twiddles<R>, dim3((2 * d->n + block - 1) / block), dim3(block), 0, s,
                     static_cast<R*>(tw), ta);
  hip_check(hipGetLastError(), "k_noalloc_twiddles");
  hipLaunchKernelGGL(k_noalloc_windows<R>, dim3((d->n * d->n_radii + block - 1) / block), dim3(block), 0, s,
                     static_cast<R*>(wtab), wa);
  hip_check(hipGetLastError(), "k_noalloc_windows");
}

}  // namespace
}  // namespace pin

using namespace pin;

extern "C" pin_status pin_collapse_times_noalloc(const pin_plan_desc* desc, const void* dk, void* F, uint8_t* ridx,
                                                 hipStream_t stream) {
  return guarded([&] {
    validate_desc(desc);
    const bool fp64 = desc->prec == PIN_FP64;
    const size_t need = workspace_bytes(desc->n, desc->n_radii, fp64);
    if (desc->n > kMaxN || need > kScratchBytes)
      fail(PIN_ERR_UNSUPPORTED_SIZE, "pin_collapse_times_noalloc: N=" + std::to_string(desc->n) + " with " +
                                         std::to_string(desc->n_radii) + " radii needs " + std::to_string(need) +
                                         " bytes of scratch, more than its " + std::to_string(kScratchBytes) +
                                         " (float32 N <= 128, float64 N <= 96)");
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) fail(PIN_ERR_DEVICE, "device ordinal beyond the library's table");

    // a plan view over the scratch array: nothing in it owns memory
    pin_plan_s p;
    p.n = desc->n;
    p.nr = p.nr_capacity = desc->n_radii;
    p.fp64 = fp64;
    p.real_bytes = fp64 ? 8 : 4;
    p.ops = find_ops(p.n, fp64);
    p.sphere_gain = eds_sphere_root() / eds_delta_c() - 1.0;
    p.device = dev;
    p.slot_bytes = (size_t)p.n * p.n * (p.n / 2) * p.complex_bytes();
    check_device_range(dk, p.half_spectrum_bytes(), "dk");
    check_device_range(F, p.real_field_bytes(), "F");
    check_device_range(ridx, (size_t)p.n * p.n * p.n, "ridx");

    char* base = static_cast<char*>(scratch_address(dev));
    p.G = base;
    p.X = base + p.slot_bytes;
    p.Y = base + 5 * p.slot_bytes;
    p.tw = base + 11 * p.slot_bytes;
    p.wtab = static_cast<char*>(p.tw) + (size_t)p.n * p.complex_bytes();
    if (fp64)
      write_tables<double>(p.tw, p.wtab, desc, stream);
    else
      write_tables<float>(p.tw, p.wtab, desc, stream);
    plan_reset(&p, F, ridx, stream);
    plan_run_radii(&p, dk, F, ridx, 0, p.nr, stream);
  });
}
