// Thread-sanitizer stress driver for the serving scheduler core (host only): several client
// threads submit, wait, cancel and release against the host executor double while the scheduler
// thread admits and polls.  Exit status 0 and "stress ok" when every request ends consistently.
#include <cstdio>
#include <thread>
#include <vector>

#include "fake_serve.cpp"

int main() {
  pin_fake_configure(2, 0, 0, 0);
  pin_serve_config cfg{3.0 * 64 * 64 * 64, 2, 0, PIN_FP32, 0.8, 0.21, 1.0};
  pin_server srv = nullptr;
  if (pin_serve_create(&cfg, &srv) != PIN_OK) return 1;
  const double radii[3] = {4.0, 2.0, 1.0};
  std::vector<std::thread> th;
  std::vector<int> bad(8, 0);
  for (int k = 0; k < 8; ++k) {
    th.emplace_back([&, k] {
      for (int i = 0; i < 40; ++i) {
        pin_request r{(uint64_t)(1000 * k + i + 1), (k + i) % 2 ? 32 : 64, 10.0, 3, radii, i % 2};
        uint64_t t = 0;
        if (pin_serve_submit(srv, &r, &t) != PIN_OK) { ++bad[k]; continue; }
        if (i % 7 == 3) pin_serve_cancel(srv, t);
        pin_result res;
        const pin_status s = pin_serve_wait(srv, t, 30.0, &res);
        if (s != PIN_OK && s != PIN_ERR_CANCELLED) ++bad[k];
        if (pin_serve_release(srv, t) != PIN_OK) ++bad[k];
        pin_serve_stats_t st;
        pin_serve_stats(srv, &st);
      }
    });
  }
  for (auto& t : th) t.join();
  pin_serve_stats_t st;
  pin_serve_stats(srv, &st);
  pin_serve_destroy(srv);
  int nbad = 0;
  for (int b : bad) nbad += b;
  std::printf("completed %lld cancelled %lld bad %d\n", st.completed, st.cancelled, nbad);
  if (nbad || st.completed + st.cancelled != 8 * 40) return 2;
  std::printf("stress ok\n");
  return 0;
}
