// The serving loop's scheduler (csrc/sched.hpp) driven by a fake device on
// the CPU: admission under the right-hand-side and memory limits, first-in
// first-out order, cancellation of queued and running requests, failures of
// start and of a round, and destruction with requests in flight.  Built with
// AddressSanitizer + UndefinedBehaviorSanitizer (and ThreadSanitizer) by
// test_sched_host.py; each case prints "ok <name>" or aborts with the failed
// condition.
//
// Usage: sched_fake [case]   (no argument: every case)
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "sched.hpp"

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::abort();                                                       \
    }                                                                     \
  } while (0)

namespace {

struct Req {
  uint64_t id = 0;
  int R = 1;
  int64_t bytes = 0;
  lm_state state = LM_QUEUED;
  lm_status status = LM_OK, fail_status = LM_OK;
  std::string err;
  bool cancel = false;
  double t_submit = 0.0, t_done = 0.0;
  // fake work: rounds until done, whether it converges, whether start fails
  int rounds = 1;
  bool conv = true;
  bool fail_start = false;
  int done_rounds = 0;  // worker-owned
  int tag = 0;
};

double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

// Records what the scheduler asks of the device and checks the limits at every round.
struct FakeDev {
  lmsched::Book<Req>* B = nullptr;
  std::mutex m;  // guards the records below (read by the test thread)
  std::vector<int> start_order;
  std::set<Req*> live;
  int starts = 0, releases = 0, rounds = 0, trims = 0, settles_idle = 0, idle_releases = 0;
  int max_active = 0;
  int64_t max_used = 0;
  int fail_round_at = -1;  // this round fails (once)
  std::atomic<int> round_sleep_us{0};
  std::string err;

  lm_status start(Req* q) {
    std::lock_guard<std::mutex> lk(m);
    CHECK(q->state == LM_RUNNING);
    CHECK(live.insert(q).second);  // started once
    start_order.push_back(q->tag);
    ++starts;
    q->done_rounds = 0;
    if (q->fail_start) {
      err = "fake start failure";
      return LM_ENOMEM;
    }
    return LM_OK;
  }
  void release(Req* q) {
    std::lock_guard<std::mutex> lk(m);
    CHECK(live.erase(q) == 1);  // released once, and only if started
    ++releases;
  }
  bool has_work() {
    std::lock_guard<std::mutex> lk(m);
    return !live.empty();
  }
  lm_status round() {
    {
      std::lock_guard<std::mutex> lb(B->mu);
      CHECK(B->active >= 0 && B->used >= 0);
      CHECK(B->active <= B->max_rhs && B->used <= B->budget);
      max_active = std::max(max_active, B->active);
      max_used = std::max(max_used, B->used);
    }
    if (int us = round_sleep_us.load()) std::this_thread::sleep_for(std::chrono::microseconds(us));
    std::lock_guard<std::mutex> lk(m);
    const int r = rounds++;
    if (r == fail_round_at) {
      err = "fake round failure";
      return LM_EHIP;
    }
    for (Req* q : live) ++q->done_rounds;
    return LM_OK;
  }
  bool finished(Req* q, bool* conv) {
    std::lock_guard<std::mutex> lk(m);
    CHECK(live.count(q) == 1);
    *conv = q->conv;
    return q->done_rounds >= q->rounds;
  }
  void trim(int64_t allow, const std::vector<Req*>& admit) {
    CHECK(allow >= 0 && !admit.empty());
    std::lock_guard<std::mutex> lk(m);
    ++trims;
  }
  void settle(bool idle) {
    std::lock_guard<std::mutex> lk(m);
    if (idle) {
      CHECK(live.empty());
      ++settles_idle;
    }
  }
  void release_idle() {
    std::lock_guard<std::mutex> lk(m);
    CHECK(live.empty());
    ++idle_releases;
  }
  double now() const { return ::now(); }
  std::string last_error() {
    std::lock_guard<std::mutex> lk(m);
    return err;
  }
};

// A scheduler with its worker thread, as the server holds them.
struct Sched {
  lmsched::Book<Req> B;
  FakeDev D;
  std::thread th;
  Sched(int max_rhs, int64_t budget) {
    B.max_rhs = max_rhs;
    B.budget = budget;
    D.B = &B;
    th = std::thread([this] { lmsched::run_worker(B, D); });
  }
  ~Sched() { destroy(); }
  void destroy() {
    if (!th.joinable()) return;
    B.request_stop();
    th.join();
    B.clear();
  }
  uint64_t submit(int R, int64_t bytes, int rounds, int tag, bool conv = true, bool fail_start = false) {
    Req* q = new Req();
    q->R = R;
    q->bytes = bytes;
    q->rounds = rounds;
    q->tag = tag;
    q->conv = conv;
    q->fail_start = fail_start;
    uint64_t id = 0;
    const lm_status st = B.submit(q, now(), &id);
    return st == LM_OK ? id : 0;
  }
  lm_state state(uint64_t id, lm_status* st = nullptr) {
    std::lock_guard<std::mutex> lk(B.mu);
    Req* q = B.find(id);
    CHECK(q);
    if (st) *st = q->status;
    return q->state;
  }
  bool terminal(uint64_t id) {
    const lm_state s = state(id);
    return s == LM_DONE || s == LM_FAILED || s == LM_CANCELLED;
  }
  void wait_all(const std::vector<uint64_t>& ids, double timeout_s = 30.0) {
    const double t0 = now();
    for (uint64_t id : ids)
      while (!terminal(id)) {
        CHECK(now() - t0 < timeout_s);
        std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
  }
  void wait_state(uint64_t id, lm_state s, double timeout_s = 30.0) {
    const double t0 = now();
    while (state(id) != s) {
      CHECK(now() - t0 < timeout_s);
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
  }
  void check_idle() {
    std::lock_guard<std::mutex> lk(B.mu);
    CHECK(B.used == 0 && B.active == 0 && B.queue.empty());
  }
};

// Requests run in submission order; the limits are never exceeded and fill up.
void case_admission_fifo() {
  Sched s(4, 1000);
  s.D.round_sleep_us = 200;
  std::vector<uint64_t> ids;
  const int R[] = {2, 1, 3, 1, 2, 2, 4, 1};
  const int64_t by[] = {300, 500, 200, 400, 600, 100, 300, 900};
  for (int i = 0; i < 8; ++i) ids.push_back(s.submit(R[i], by[i], 3 + i % 3, i));
  for (uint64_t id : ids) CHECK(id != 0);
  s.wait_all(ids);
  for (uint64_t id : ids) {
    lm_status st;
    CHECK(s.state(id, &st) == LM_DONE && st == LM_OK);
  }
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK(s.D.start_order.size() == 8);
  for (int i = 0; i < 8; ++i) CHECK(s.D.start_order[i] == i);
  CHECK(s.D.starts == 8 && s.D.releases == 8 && s.D.live.empty());
  CHECK(s.D.max_active <= 4 && s.D.max_used <= 1000 && s.D.max_active >= 3);
  s.check_idle();
}

// A request that does not fit yet blocks those behind it (no overtaking):
// the small request submitted after the large one starts after it.
void case_head_of_line() {
  Sched s(8, 1000);
  s.D.round_sleep_us = 100;
  const uint64_t a = s.submit(1, 600, 40, 0);  // long-running, holds 600
  s.wait_state(a, LM_RUNNING);
  const uint64_t b = s.submit(1, 700, 2, 1);   // cannot fit while a runs
  const uint64_t c = s.submit(1, 100, 2, 2);   // would fit, but is behind b
  std::this_thread::sleep_for(std::chrono::milliseconds(5));
  CHECK(s.state(b) == LM_QUEUED && s.state(c) == LM_QUEUED);
  s.wait_all({a, b, c});
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK((s.D.start_order == std::vector<int>{0, 1, 2}));
  s.check_idle();
}

// Requests beyond the limits are rejected at submission and never registered.
void case_reject() {
  Sched s(4, 1000);
  CHECK(s.submit(5, 10, 1, 0) == 0);
  CHECK(s.submit(1, 1001, 1, 1) == 0);
  const uint64_t ok = s.submit(4, 1000, 1, 2);  // exactly at both limits
  CHECK(ok != 0);
  s.wait_all({ok});
  std::lock_guard<std::mutex> lk(s.B.mu);
  CHECK(s.B.reqs.size() == 1);
}

// Cancelling a queued request ends it at once; it never starts.
void case_cancel_queued() {
  Sched s(1, 1000);
  s.D.round_sleep_us = 100;
  const uint64_t a = s.submit(1, 10, 50, 0);
  s.wait_state(a, LM_RUNNING);
  const uint64_t b = s.submit(1, 10, 1, 1);
  CHECK(s.B.cancel(b, now()) == LM_OK);
  lm_status st;
  CHECK(s.state(b, &st) == LM_CANCELLED && st == LM_ECANCELLED);
  CHECK(s.B.cancel(b, now()) == LM_OK);  // again: no change
  CHECK(s.state(b) == LM_CANCELLED);
  s.wait_all({a});
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK((s.D.start_order == std::vector<int>{0}));
  s.check_idle();
}

// Cancelling a running request ends it at the next round and gives its slots back.
void case_cancel_running() {
  Sched s(2, 1000);
  s.D.round_sleep_us = 200;
  const uint64_t a = s.submit(2, 500, 1000000, 0);  // would run "forever"
  const uint64_t b = s.submit(2, 500, 2, 1);        // waits for a's slots
  s.wait_state(a, LM_RUNNING);
  CHECK(s.state(b) == LM_QUEUED);
  CHECK(s.B.cancel(a, now()) == LM_OK);
  s.wait_all({a, b});
  lm_status st;
  CHECK(s.state(a, &st) == LM_CANCELLED && st == LM_ECANCELLED);
  CHECK(s.state(b, &st) == LM_DONE && st == LM_OK);
  CHECK(s.B.cancel(a, now()) == LM_OK);  // cancelling a finished request changes nothing
  CHECK(s.state(a) == LM_CANCELLED);
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK(s.D.releases == 2 && s.D.live.empty());
  s.check_idle();
}

// Release only in a terminal state; unknown ids are reported.
void case_release() {
  Sched s(1, 1000);
  s.D.round_sleep_us = 100;
  const uint64_t a = s.submit(1, 10, 30, 0);
  const uint64_t b = s.submit(1, 10, 1, 1);
  s.wait_state(a, LM_RUNNING);
  CHECK(s.B.release(a) == LM_EINVAL);  // running
  CHECK(s.B.release(b) == LM_EINVAL);  // queued
  s.wait_all({a, b});
  CHECK(s.B.release(a) == LM_OK);
  CHECK(s.B.release(a) == LM_ENOTFOUND);
  CHECK(s.B.cancel(a, now()) == LM_ENOTFOUND);
  CHECK(s.B.release(12345) == LM_ENOTFOUND);
  CHECK(s.B.release(b) == LM_OK);
  std::lock_guard<std::mutex> lk(s.B.mu);
  CHECK(s.B.reqs.empty());
}

// GMRES that stops at max_iter: done, with LM_NOT_CONVERGED.
void case_not_converged() {
  Sched s(4, 1000);
  const uint64_t a = s.submit(1, 10, 3, 0, false);
  const uint64_t b = s.submit(1, 10, 2, 1, true);
  s.wait_all({a, b});
  lm_status st;
  CHECK(s.state(a, &st) == LM_DONE && st == LM_NOT_CONVERGED);
  CHECK(s.state(b, &st) == LM_DONE && st == LM_OK);
}

// A failed start fails that request only; it is released once and the others run.
void case_start_failure() {
  Sched s(4, 1000);
  const uint64_t a = s.submit(1, 10, 3, 0);
  const uint64_t b = s.submit(1, 10, 3, 1, true, true);
  const uint64_t c = s.submit(1, 10, 3, 2);
  s.wait_all({a, b, c});
  lm_status st;
  CHECK(s.state(a, &st) == LM_DONE && st == LM_OK);
  CHECK(s.state(b, &st) == LM_FAILED && st == LM_ENOMEM);
  {
    std::lock_guard<std::mutex> lk(s.B.mu);
    CHECK(s.B.find(b)->err == "fake start failure");
  }
  CHECK(s.state(c, &st) == LM_DONE && st == LM_OK);
  // the failed request's slots come back at the next round
  const uint64_t d = s.submit(4, 1000, 1, 3);
  s.wait_all({d});
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK(s.D.starts == 4 && s.D.releases == 4 && s.D.live.empty());
  s.check_idle();
}

// A failed round fails every running request; later requests still run.
void case_round_failure() {
  Sched s(4, 1000);
  s.D.fail_round_at = 1;
  s.D.round_sleep_us = 100;
  const uint64_t a = s.submit(2, 10, 5, 0);
  const uint64_t b = s.submit(2, 10, 5, 1);
  s.wait_all({a, b});
  lm_status st;
  CHECK(s.state(a, &st) == LM_FAILED && st == LM_EHIP);
  CHECK(s.state(b, &st) == LM_FAILED && st == LM_EHIP);
  const uint64_t c = s.submit(4, 10, 2, 2);
  s.wait_all({c});
  CHECK(s.state(c, &st) == LM_DONE && st == LM_OK);
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK(s.D.releases == 3 && s.D.live.empty());
  s.check_idle();
}

// Destroying with requests queued and running: the worker stops after its
// round, every started request is released once and every request is freed.
void case_destroy_in_flight() {
  for (int rep = 0; rep < 20; ++rep) {
    auto* s = new Sched(3, 1000);
    s->D.round_sleep_us = rep % 4 * 50;
    for (int i = 0; i < 12; ++i) s->submit(1 + i % 3, 100 + 50 * (i % 5), 1 + (i * 7) % 11, i);
    std::this_thread::sleep_for(std::chrono::microseconds(rep * 150));
    s->destroy();
    {
      std::lock_guard<std::mutex> lk(s->D.m);
      CHECK(s->D.live.empty() && s->D.starts == s->D.releases);
    }
    CHECK(s->B.reqs.empty());
    delete s;
  }
  // an idle scheduler (worker waiting for work) stops too
  Sched idle(2, 100);
  idle.destroy();
}

// Several client threads submit, poll, cancel and release at random while
// the worker runs; the limits hold and everything is given back.
void case_concurrent_clients() {
  Sched s(6, 2000);
  s.D.round_sleep_us = 20;
  s.D.fail_round_at = 37;  // clients release the failed requests while the worker lets them go
  std::atomic<int> submitted{0};
  auto client = [&](int seed) {
    std::mt19937 rng(seed);
    std::vector<uint64_t> mine;
    for (int i = 0; i < 60; ++i) {
      const int R = 1 + rng() % 3;
      const int64_t by = 50 + rng() % 600;
      const uint64_t id = s.submit(R, by, 1 + rng() % 8, seed * 1000 + i, rng() % 5 != 0, rng() % 17 == 0);
      CHECK(id != 0);
      ++submitted;
      mine.push_back(id);
      if (rng() % 4 == 0) CHECK(s.B.cancel(mine[rng() % mine.size()], now()) == LM_OK);
      if (rng() % 3 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
      for (auto it = mine.begin(); it != mine.end();) {  // release what has ended
        if (s.terminal(*it)) {
          CHECK(s.B.release(*it) == LM_OK);
          it = mine.erase(it);
        } else {
          ++it;
        }
      }
    }
    s.wait_all(mine, 60.0);
    for (uint64_t id : mine) CHECK(s.B.release(id) == LM_OK);
  };
  std::vector<std::thread> ths;
  for (int t = 0; t < 4; ++t) ths.emplace_back(client, 11 + t);
  for (auto& t : ths) t.join();
  CHECK(submitted == 240);
  {
    std::lock_guard<std::mutex> lk(s.B.mu);
    CHECK(s.B.reqs.empty());
  }
  // the worker gives back the last request's slots before it goes idle
  const double t0 = now();
  while (true) {
    {
      std::lock_guard<std::mutex> lk(s.B.mu);
      if (s.B.used == 0 && s.B.active == 0) break;
    }
    CHECK(now() - t0 < 10.0);
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  s.check_idle();
  std::lock_guard<std::mutex> lk(s.D.m);
  CHECK(s.D.max_active <= 6 && s.D.max_used <= 2000);
}

// Kept memory is given back only after the worker has stayed idle for
// idle_release; a request arriving sooner finds it still there.
void case_idle_release() {
  Sched s(4, 1000);
  {
    std::lock_guard<std::mutex> lk(s.B.mu);
    s.B.idle_release = std::chrono::microseconds(1000000);  // long against scheduling delays under the sanitizers
  }
  uint64_t a = s.submit(2, 100, 3, 0);
  s.wait_all({a});
  uint64_t b = s.submit(2, 100, 3, 1);  // at once: before the idle release
  s.wait_all({b});
  {
    std::lock_guard<std::mutex> lk(s.D.m);
    CHECK(s.D.idle_releases == 0 && s.D.settles_idle >= 1);
  }
  const double t0 = now();
  while (true) {
    {
      std::lock_guard<std::mutex> lk(s.D.m);
      if (s.D.idle_releases == 1) break;
    }
    CHECK(now() - t0 < 5.0);
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
  }
  CHECK(now() - t0 > 0.5);  // not before the idle time has passed
  std::this_thread::sleep_for(std::chrono::milliseconds(300));
  {
    std::lock_guard<std::mutex> lk(s.D.m);
    CHECK(s.D.idle_releases == 1);  // once per idle period
  }
  uint64_t c = s.submit(1, 100, 2, 2);
  s.wait_all({c});
  for (uint64_t id : {a, b, c}) CHECK(s.B.release(id) == LM_OK);
  s.check_idle();
}

const std::pair<const char*, void (*)()> kCases[] = {
    {"admission_fifo", case_admission_fifo},     {"head_of_line", case_head_of_line},
    {"reject", case_reject},                     {"cancel_queued", case_cancel_queued},
    {"cancel_running", case_cancel_running},     {"release", case_release},
    {"not_converged", case_not_converged},       {"start_failure", case_start_failure},
    {"round_failure", case_round_failure},       {"destroy_in_flight", case_destroy_in_flight},
    {"concurrent_clients", case_concurrent_clients}, {"idle_release", case_idle_release},
};

}  // namespace

int main(int argc, char** argv) {
  int ran = 0;
  for (const auto& c : kCases) {
    if (argc > 1 && std::strcmp(argv[1], c.first) != 0) continue;
    c.second();
    std::printf("ok %s\n", c.first);
    std::fflush(stdout);
    ++ran;
  }
  if (ran == 0) {
    std::fprintf(stderr, "no case named %s\n", argc > 1 ? argv[1] : "");
    return 2;
  }
  return 0;
}
