// Serving scheduler: continuous batching of realization requests at request granularity over
// per-size-class slots, admitted against a device-memory budget.
//
// A slot owns everything one request of grid size N needs on the device (a plan's workspace,
// the field and the outputs) and its own stream.  A request is admitted into an idle slot of its
// size class, or into a new slot when the budget allows one more (idle slots of other classes
// are evicted, least recently used first, to make room); its whole path is then queued on the
// slot's stream, so admitted requests of any sizes run concurrently on the device.  Results stay
// in the slot until the client releases them.  Within a size class requests are admitted in
// arrival order; a class that cannot admit its head request does not block other classes.
//
// The scheduler is independent of the device: `Exec` supplies slot creation, launch and
// completion polling (the HIP executor in serve.cpp; a host-only double in the tests).
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "errors.hpp"
#include "pin.h"

namespace pin {
namespace serve {

struct Request {
  uint64_t ticket = 0;
  uint64_t seed = 0;
  int n = 0;
  double box = 0;
  std::vector<double> radii;
  int want_disp = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  enum State { QUEUED, RUNNING, DONE, FAILED, CANCELLED } state = QUEUED;
  pin_status status = PIN_ERR_NOT_READY;
  std::string error;
  bool cancel_requested = false;
  int slot = -1;
};

struct Config {
  double budget_bytes = 0;
  int max_slots_per_class = 4;
};

struct Stats {
  double p50 = 0, p99 = 0, mean = 0;    // latency submit -> done, seconds
  double updates_per_s = 0;             // sum N^3 n_radii of completed / (last done - first submit)
  double hbm_in_use = 0;                // bytes held by slots
  long long completed = 0, failed = 0, cancelled = 0, queued = 0, running = 0, slots = 0;
};

template <class Exec>
class Core {
 public:
  using Slot = typename Exec::Slot;

  Core(Exec& exec, const Config& cfg) : exec_(exec), cfg_(cfg), t0_(clock::now()) {
    thread_ = std::thread([this] { loop(); });
  }
  ~Core() { shutdown(); }

  double now() const { return std::chrono::duration<double>(clock::now() - t0_).count(); }

  // Validates, copies and queues; non-blocking.
  pin_status submit(const pin_request* r, uint64_t* ticket) {
    if (r == nullptr || ticket == nullptr) return fail_status(PIN_ERR_INVALID_ARG, "request or ticket is NULL");
    std::string why;
    const pin_status v = exec_.validate(r->n, r->box, r->n_radii, r->radii_cells, why);
    if (v != PIN_OK) return fail_status(v, why);
    if (r->want_disp != 0 && r->want_disp != 1) return fail_status(PIN_ERR_INVALID_ARG, "want_disp must be 0 or 1");
    if ((double)exec_.slot_bytes(r->n) > cfg_.budget_bytes)
      return fail_status(PIN_ERR_BUDGET, "a slot of this grid size exceeds the HBM budget");
    std::lock_guard<std::mutex> lk(m_);
    if (stopping_) return fail_status(PIN_ERR_SHUTDOWN, "server is shutting down");
    Request q;
    q.ticket = next_ticket_++;
    q.seed = r->seed;
    q.n = r->n;
    q.box = r->box;
    q.radii.assign(r->radii_cells, r->radii_cells + r->n_radii);
    q.want_disp = r->want_disp;
    q.t_submit = now();
    if (first_submit_ < 0) first_submit_ = q.t_submit;
    queue_.push_back(q.ticket);
    *ticket = q.ticket;
    reqs_.emplace(q.ticket, std::move(q));
    cv_work_.notify_all();
    return PIN_OK;
  }

  pin_status poll(uint64_t ticket, pin_result* out) {
    std::lock_guard<std::mutex> lk(m_);
    return poll_locked(ticket, out);
  }

  pin_status wait(uint64_t ticket, double timeout_s, pin_result* out) {
    std::unique_lock<std::mutex> lk(m_);
    const auto deadline = clock::now() + std::chrono::duration_cast<clock::duration>(
                                             std::chrono::duration<double>(timeout_s < 0 ? 0 : timeout_s));
    for (;;) {
      const pin_status s = poll_locked(ticket, out);
      if (s != PIN_ERR_NOT_READY) return s;
      const clock::duration left = deadline - clock::now();
      if (left <= clock::duration::zero()) return fail_status(PIN_ERR_TIMEOUT, "wait timed out");
      sleep_on(cv_done_, lk, std::min<clock::duration>(left, std::chrono::milliseconds(50)));
    }
  }

  pin_status cancel(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(m_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail_status(PIN_ERR_INVALID_ARG, "unknown ticket");
    Request& q = it->second;
    if (q.state == Request::QUEUED) {
      queue_.erase(std::find(queue_.begin(), queue_.end(), ticket));
      finish_locked(q, Request::CANCELLED, PIN_ERR_CANCELLED, "cancelled before admission");
    } else if (q.state == Request::RUNNING) {
      q.cancel_requested = true;   // the device work cannot be recalled; discarded when done
    }
    return PIN_OK;
  }

  pin_status release(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(m_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail_status(PIN_ERR_INVALID_ARG, "unknown ticket");
    Request& q = it->second;
    if (q.state == Request::QUEUED || q.state == Request::RUNNING)
      return fail_status(PIN_ERR_INVALID_ARG, "request not finished (cancel it first)");
    if (q.state == Request::DONE && q.slot >= 0) free_slot_locked(q.slot);
    reqs_.erase(it);
    cv_work_.notify_all();
    return PIN_OK;
  }

  Stats stats() {
    std::lock_guard<std::mutex> lk(m_);
    Stats s;
    std::vector<double> lat = latencies_;
    if (!lat.empty()) {
      std::sort(lat.begin(), lat.end());
      auto pct = [&](double p) {
        const double pos = p * (lat.size() - 1);
        const size_t i = (size_t)pos;
        const double f = pos - i;
        return i + 1 < lat.size() ? lat[i] * (1 - f) + lat[i + 1] * f : lat[i];
      };
      s.p50 = pct(0.50);
      s.p99 = pct(0.99);
      double sum = 0;
      for (double v : lat) sum += v;
      s.mean = sum / lat.size();
    }
    if (last_done_ > first_submit_ && first_submit_ >= 0) s.updates_per_s = updates_ / (last_done_ - first_submit_);
    s.hbm_in_use = (double)in_use_;
    s.completed = completed_;
    s.failed = failed_;
    s.cancelled = cancelled_;
    for (auto& kv : reqs_) {
      if (kv.second.state == Request::QUEUED) ++s.queued;
      if (kv.second.state == Request::RUNNING) ++s.running;
    }
    for (auto& sl : slots_) s.slots += sl.h != nullptr;
    return s;
  }

  void reset_stats() {
    std::lock_guard<std::mutex> lk(m_);
    latencies_.clear();
    updates_ = 0;
    first_submit_ = -1;
    last_done_ = 0;
    completed_ = failed_ = cancelled_ = 0;
  }

  // Stop admitting, cancel queued requests, let running ones finish, free every slot.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(m_);
      if (stopping_) {
        if (!thread_.joinable()) return;
      }
      stopping_ = true;
      for (uint64_t t : queue_) finish_locked(reqs_[t], Request::CANCELLED, PIN_ERR_SHUTDOWN, "server shut down");
      queue_.clear();
      cv_work_.notify_all();
    }
    if (thread_.joinable()) thread_.join();
    std::lock_guard<std::mutex> lk(m_);
    for (size_t i = 0; i < slots_.size(); ++i)
      if (slots_[i].h) destroy_slot_locked((int)i);
    cv_done_.notify_all();
  }

 private:
  using clock = std::chrono::steady_clock;

  // Bounded condition-variable wait.  The deadline is taken on the system clock, whose waits map
  // to pthread_cond_timedwait (visible to thread sanitizers); callers loop on their own steady-
  // clock deadlines, so a wall-clock step only shortens or lengthens one slice.
  static void sleep_on(std::condition_variable& cv, std::unique_lock<std::mutex>& lk, clock::duration d) {
    cv.wait_until(lk, std::chrono::system_clock::now() +
                          std::chrono::duration_cast<std::chrono::system_clock::duration>(d));
  }

  struct SlotInfo {
    Slot* h = nullptr;
    int n = 0;
    size_t bytes = 0;
    bool busy = false;
    uint64_t ticket = 0;
    double last_used = 0;
  };

  pin_status fail_status(pin_status s, const std::string& why) {
    last_error_ = why;
    exec_.set_error(why);
    return s;
  }

  pin_status poll_locked(uint64_t ticket, pin_result* out) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail_status(PIN_ERR_INVALID_ARG, "unknown ticket");
    const Request& q = it->second;
    if (out) {
      *out = pin_result{};
      out->n = q.n;
      out->n_radii = (int)q.radii.size();
      out->t_submit = q.t_submit;
      out->t_admit = q.t_admit;
      out->t_done = q.t_done;
      out->status = q.status;
    }
    if (q.state == Request::QUEUED || q.state == Request::RUNNING) return PIN_ERR_NOT_READY;
    if (q.state == Request::DONE) {
      if (out) exec_.results(slots_[q.slot].h, q.want_disp, out);
      return PIN_OK;
    }
    exec_.set_error(q.error);
    return q.status;
  }

  void finish_locked(Request& q, Request::State st, pin_status status, const std::string& err) {
    q.state = st;
    q.status = status;
    q.error = err;
    q.t_done = now();
    if (st == Request::DONE) {
      ++completed_;
      latencies_.push_back(q.t_done - q.t_submit);
      updates_ += (double)q.n * q.n * q.n * (double)q.radii.size();
      last_done_ = std::max(last_done_, q.t_done);
    } else if (st == Request::FAILED) {
      ++failed_;
    } else {
      ++cancelled_;
    }
    cv_done_.notify_all();
  }

  void free_slot_locked(int i) {
    slots_[i].busy = false;
    slots_[i].ticket = 0;
    slots_[i].last_used = now();
  }

  void destroy_slot_locked(int i) {
    exec_.destroy_slot(slots_[i].h);
    in_use_ -= slots_[i].bytes;
    slots_[i] = SlotInfo{};
  }

  // Slot index for a request of size n, creating or evicting as the budget allows; -1 if none.
  int acquire_slot_locked(int n) {
    int count = 0;
    for (size_t i = 0; i < slots_.size(); ++i) {
      if (!slots_[i].h || slots_[i].n != n) continue;
      ++count;
      if (!slots_[i].busy) return (int)i;
    }
    if (count >= cfg_.max_slots_per_class) return -1;
    const size_t need = exec_.slot_bytes(n);
    while ((double)(in_use_ + need) > cfg_.budget_bytes) {
      int victim = -1;
      for (size_t i = 0; i < slots_.size(); ++i)
        if (slots_[i].h && !slots_[i].busy && (victim < 0 || slots_[i].last_used < slots_[victim].last_used))
          victim = (int)i;
      if (victim < 0) return -1;
      destroy_slot_locked(victim);
    }
    Slot* h = exec_.create_slot(n);   // may throw
    int idx = -1;
    for (size_t i = 0; i < slots_.size(); ++i)
      if (!slots_[i].h) { idx = (int)i; break; }
    if (idx < 0) {
      slots_.push_back(SlotInfo{});
      idx = (int)slots_.size() - 1;
    }
    slots_[idx].h = h;
    slots_[idx].n = n;
    slots_[idx].bytes = need;
    in_use_ += need;
    return idx;
  }

  struct Launch {
    int slot;
    uint64_t ticket;
    Slot* h;
    uint64_t seed;
    double box;
    std::vector<double> radii;
    int want_disp;
  };

  // Admission: requests are matched to slots under the lock; their launches (radius tables,
  // field, graph capture on a slot's first request of a shape, graph replay) run after it is
  // released, so client calls never wait behind them.  Only this thread creates, launches and
  // destroys slots, and a slot being launched is busy with a RUNNING request, so nothing else
  // touches it meanwhile.
  bool admit(std::unique_lock<std::mutex>& lk) {
    std::vector<Launch> todo;
    const bool progressed = admit_locked(todo);
    if (todo.empty()) return progressed;
    lk.unlock();
    std::vector<std::pair<size_t, PinError>> failed;
    for (size_t i = 0; i < todo.size(); ++i) {
      const Launch& l = todo[i];
      try {
        exec_.launch(l.h, l.seed, l.box, l.radii, l.want_disp);
      } catch (const PinError& e) {
        failed.emplace_back(i, e);
      }
    }
    lk.lock();
    for (auto& f : failed) {
      const Launch& l = todo[f.first];
      Request& q = reqs_[l.ticket];
      finish_locked(q, Request::FAILED, f.second.status, f.second.msg);
      destroy_slot_locked(l.slot);
      q.slot = -1;
    }
    return true;
  }

  bool admit_locked(std::vector<Launch>& todo) {
    bool progressed = false;
    std::vector<int> blocked;   // size classes whose head request could not be admitted
    for (auto it = queue_.begin(); it != queue_.end();) {
      Request& q = reqs_[*it];
      if (std::find(blocked.begin(), blocked.end(), q.n) != blocked.end()) {
        ++it;
        continue;
      }
      int s = -1;
      try {
        s = acquire_slot_locked(q.n);
      } catch (const PinError& e) {
        // could not create a slot now: keep the request queued unless nothing else holds memory
        bool others = false;
        for (auto& sl : slots_) others |= sl.h != nullptr;
        if (!others) {
          finish_locked(q, Request::FAILED, e.status, e.msg);
          it = queue_.erase(it);
          progressed = true;
          continue;
        }
        s = -1;
      }
      if (s < 0) {
        blocked.push_back(q.n);
        ++it;
        continue;
      }
      slots_[s].busy = true;
      slots_[s].ticket = q.ticket;
      q.slot = s;
      q.t_admit = now();
      q.state = Request::RUNNING;
      todo.push_back(Launch{s, q.ticket, slots_[s].h, q.seed, q.box, q.radii, q.want_disp});
      it = queue_.erase(it);
      progressed = true;
    }
    return progressed;
  }

  bool poll_running_locked() {
    bool progressed = false;
    for (size_t i = 0; i < slots_.size(); ++i) {
      SlotInfo& sl = slots_[i];
      if (!sl.h || !sl.busy) continue;
      auto it = reqs_.find(sl.ticket);
      if (it == reqs_.end() || it->second.state != Request::RUNNING) continue;
      Request& q = it->second;
      std::string err;
      const int st = exec_.poll(sl.h, err);
      if (st == 0) continue;
      progressed = true;
      if (st < 0) {
        finish_locked(q, Request::FAILED, PIN_ERR_DEVICE, err);
        destroy_slot_locked((int)i);
        q.slot = -1;
      } else if (q.cancel_requested) {
        finish_locked(q, Request::CANCELLED, PIN_ERR_CANCELLED, "cancelled while running");
        free_slot_locked((int)i);
        q.slot = -1;
      } else {
        finish_locked(q, Request::DONE, PIN_OK, "");
      }
    }
    return progressed;
  }

  bool any_running_locked() const {
    for (auto& sl : slots_)
      if (sl.h && sl.busy) return true;
    return false;
  }

  void loop() {
    std::unique_lock<std::mutex> lk(m_);
    for (;;) {
      poll_running_locked();
      if (!stopping_) admit(lk);
      const bool running = std::any_of(reqs_.begin(), reqs_.end(),
                                       [](const auto& kv) { return kv.second.state == Request::RUNNING; });
      if (stopping_ && !running) break;
      // poll the device often while work is in flight; otherwise sleep until woken
      sleep_on(cv_work_, lk, running ? clock::duration(std::chrono::microseconds(50))
                                     : clock::duration(std::chrono::milliseconds(20)));
    }
  }

  Exec& exec_;
  Config cfg_;
  clock::time_point t0_;
  std::mutex m_;
  std::condition_variable cv_work_, cv_done_;
  std::thread thread_;
  std::map<uint64_t, Request> reqs_;
  std::deque<uint64_t> queue_;
  std::vector<SlotInfo> slots_;
  size_t in_use_ = 0;
  uint64_t next_ticket_ = 1;
  bool stopping_ = false;
  std::string last_error_;
  std::vector<double> latencies_;
  double updates_ = 0, first_submit_ = -1, last_done_ = 0;
  long long completed_ = 0, failed_ = 0, cancelled_ = 0;
};

}  // namespace serve
}  // namespace pin
