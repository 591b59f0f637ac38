// Request bookkeeping and the worker loop of the serving loop, independent of
// the device work (host C++ only, no HIP), so that the scheduling policy runs
// and is tested on the CPU with a fake device.
//
// Policy: requests are admitted first-in first-out while the admitted
// right-hand sides stay <= max_rhs and the admitted footprint stays <= budget
// (a request that does not fit blocks the ones behind it, so none is passed
// over indefinitely); every admitted request advances one step per round;
// a cancelled running request leaves at the start of the next round, a
// queued one at once; destroying the scheduler stops the worker after its
// current round and frees every request.  Device memory kept for reuse when
// the last request leaves (fused-launch and round buffers) is given back
// only when no request arrives within idle_release: a request that follows
// at once does not wait for that memory to be freed and allocated again.
//
// Ownership: a request stays LM_QUEUED or LM_RUNNING, so that no client can
// release (free) it, until the worker has given back its device work and its
// slots; only then does it become LM_DONE, LM_FAILED or LM_CANCELLED, and the
// worker touches it no more.  A failure during a round is therefore recorded
// as pending (fail_status) and made final when the request leaves.
//
// Req needs: uint64_t id; int R; int64_t bytes; lm_state state;
// lm_status status, fail_status; std::string err; bool cancel;
// double t_submit, t_done.
// Dev needs (called by the worker thread only, without the lock held):
//   lm_status start(Req*)            allocate and start an admitted request
//   void release(Req*)               give back what start allocated
//   bool has_work()                  anything to advance this round
//   lm_status round()                advance every started request one step
//   bool finished(Req*, bool* conv)  the request is complete (conv: converged)
//   void trim(int64_t allow, const std::vector<Req*>& admitted)
//   void settle(bool idle)           after the round (idle: nothing admitted)
//   void release_idle()              give back what was kept for reuse, once
//                                    the worker has stayed idle for idle_release
//   double now()
//   std::string last_error()         message of the last failed call
#pragma once
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lmfmm.h"

namespace lmsched {

template <class Req>
struct Book {
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<Req*> queue;
  std::map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  int64_t used = 0;  // footprint of the admitted requests
  int active = 0;    // admitted right-hand sides
  int max_rhs = 64;
  int64_t budget = (int64_t)64 << 30;
  std::chrono::microseconds idle_release{20000};

  // --- called by clients (each takes the lock) ---------------------------------
  // Queues q (already validated); LM_ENOMEM if it can never be admitted, in
  // which case q is deleted.
  lm_status submit(Req* q, double now, uint64_t* id) {
    if (q->R > max_rhs || q->bytes > budget) {
      delete q;
      return LM_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(mu);
    q->id = next_id++;
    q->t_submit = now;
    reqs[q->id] = q;
    queue.push_back(q);
    *id = q->id;
    cv.notify_all();
    return LM_OK;
  }
  // The request or nullptr (lock held by the caller).
  Req* find(uint64_t id) {
    auto it = reqs.find(id);
    return it == reqs.end() ? nullptr : it->second;
  }
  lm_status cancel(uint64_t id, double now) {
    std::lock_guard<std::mutex> lk(mu);
    Req* q = find(id);
    if (!q) return LM_ENOTFOUND;
    if (q->state == LM_QUEUED) {
      queue.erase(std::remove(queue.begin(), queue.end(), q), queue.end());
      q->state = LM_CANCELLED;
      q->status = LM_ECANCELLED;
      q->t_done = now;
    } else if (q->state == LM_RUNNING) {
      q->cancel = true;
    }
    return LM_OK;
  }
  // Frees a finished, failed or cancelled request; LM_EINVAL while it is
  // queued or running.
  lm_status release(uint64_t id) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = reqs.find(id);
    if (it == reqs.end()) return LM_ENOTFOUND;
    Req* q = it->second;
    if (q->state != LM_DONE && q->state != LM_FAILED && q->state != LM_CANCELLED) return LM_EINVAL;
    delete q;
    reqs.erase(it);
    return LM_OK;
  }
  // Records a failure of a running request (worker thread); the request
  // fails when the worker lets it go at the start of the next round.
  void mark_failed(Req* q, lm_status st, const std::string& msg) {
    std::lock_guard<std::mutex> lk(mu);
    if (q->state == LM_RUNNING && q->fail_status == LM_OK) {
      q->fail_status = st;
      q->err = msg;
    }
  }
  // Asks the worker to stop (it finishes its round) and marks running requests cancelled.
  void request_stop() {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
    for (auto& kv : reqs)
      if (kv.second->state == LM_RUNNING) kv.second->cancel = true;
    cv.notify_all();
  }
  // Frees every request (after the worker has been joined).
  void clear() {
    for (auto& kv : reqs) delete kv.second;
    reqs.clear();
    queue.clear();
  }
};

// The worker loop: admission, one round of every admitted request, completion.
template <class Req, class Dev>
void run_worker(Book<Req>& B, Dev& D) {
  std::vector<Req*> running;
  bool kept = false;  // the device keeps memory for reuse since the last request left
  // Gives back q's slots and ends it (lock held); q may be freed by a client after this.
  auto finish = [&](Req* q, lm_state state, lm_status status) {
    B.used -= q->bytes;
    B.active -= q->R;
    q->state = state;
    q->status = status;
    q->t_done = D.now();
  };
  while (true) {
    std::vector<Req*> admit;
    int64_t allow = 0;
    {
      std::unique_lock<std::mutex> lk(B.mu);
      // cancelled and failed running requests leave before the next round
      for (auto it = running.begin(); it != running.end();) {
        Req* q = *it;
        if (q->cancel || q->fail_status < 0) {
          lk.unlock();
          D.release(q);
          lk.lock();
          if (q->fail_status < 0)
            finish(q, LM_FAILED, q->fail_status);
          else
            finish(q, LM_CANCELLED, LM_ECANCELLED);
          it = running.erase(it);
        } else {
          ++it;
        }
      }
      if (B.stop) break;
      // admission: first in, first out, while the slots and the budget allow
      while (!B.queue.empty()) {
        Req* q = B.queue.front();
        if (B.active + q->R > B.max_rhs || B.used + q->bytes > B.budget) break;
        B.queue.pop_front();
        q->state = LM_RUNNING;
        B.used += q->bytes;
        B.active += q->R;
        admit.push_back(q);
      }
      allow = B.budget - B.used;
      if (running.empty() && admit.empty()) {
        auto work = [&] { return B.stop || !B.queue.empty(); };
        if (kept) {
          // system_clock: its timed wait is pthread_cond_timedwait, which
          // the thread sanitizer understands (steady_clock's is not)
          if (!B.cv.wait_until(lk, std::chrono::system_clock::now() + B.idle_release, work)) {
            lk.unlock();
            D.release_idle();
            lk.lock();
            kept = false;
          }
          continue;
        }
        B.cv.wait(lk, work);
        continue;
      }
    }
    if (!admit.empty()) D.trim(allow, admit);
    for (Req* q : admit) {
      const lm_status st = D.start(q);
      if (st >= 0) {
        running.push_back(q);
        continue;
      }
      const std::string msg = D.last_error();
      D.release(q);  // a failed start leaves at once
      std::lock_guard<std::mutex> lk(B.mu);
      q->err = msg;
      finish(q, LM_FAILED, st);
    }
    const lm_status st = D.has_work() ? D.round() : LM_OK;
    if (st < 0) {
      const std::string msg = D.last_error();
      for (Req* q : running) B.mark_failed(q, st, msg);
    }
    for (auto it = running.begin(); it != running.end();) {
      Req* q = *it;
      bool conv = true;
      bool failed;
      {
        std::lock_guard<std::mutex> lk(B.mu);
        failed = q->fail_status < 0;
      }
      if (!failed && D.finished(q, &conv)) {
        D.release(q);
        std::lock_guard<std::mutex> lk(B.mu);
        finish(q, LM_DONE, conv ? LM_OK : LM_NOT_CONVERGED);
        it = running.erase(it);
      } else {
        ++it;
      }
    }
    D.settle(running.empty());
    if (running.empty()) kept = true;
  }
  // stopped: what still runs is released; the requests are freed with the book
  for (Req* q : running) D.release(q);
}

}  // namespace lmsched
