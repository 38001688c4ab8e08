// Scheduling policy of the solve queue, independent of the device.
//
// The "parallel processing" step of DQAOA (arXiv 2506.10531, Sec. V) hands
// many sub-QUBO solves to QAOA solvers and collects their sub-solutions as
// they finish.  This header holds the decisions of the queue that serves that
// stream on one GPU:
//
//  * admission: pending requests are admitted in FIFO order while a slot is
//    free and the request's device bytes fit in the byte budget; a request
//    that can never fit, or a full pending list, is refused at submission;
//  * steps: every step advances all admitted requests together by K
//    evaluations, K the fewest any of them has left (at most
//    MAX_EVALS_PER_STEP), grouped by qubit count (one batch per n);
//    requests whose last evaluation falls in the step are sampled at its end;
//  * early end: rounds are enqueued with at most two in flight; before round
//    k >= 2 the step waits for round k - 2 and ends there if a waiting
//    request could now be admitted or a running one was cancelled, so an
//    arrival waits at most about two evaluations while the device stays busy;
//  * results: a step that samples hands its finished requests' results to
//    the backend, which copies them back while later steps run; those
//    requests keep their slots ("sampled") until the results are collected,
//    at the start of a later step, before the next sampling step, or when
//    nothing else runs;
//  * cancellation: a pending request completes as cancelled at once, a
//    running one at the next step boundary, a sampled one when its results
//    arrive;
//  * bookkeeping: evaluation counts, completion, slot and byte release,
//    timestamps and counters.
//
// The caller supplies the backend that runs a step's work (the device queue
// launches kernels; a host backend on a virtual clock exercises the same
// policy in tests).  A backend provides
//   int  begin(Step&)          upload newly admitted requests, lay out the step;
//   int  round(int k)          enqueue evaluation round k of every group;
//   int  wait_round(int k)     block until round k has finished;
//   int  end(bool sampled)     enqueue sampling of the groups' finished
//                              requests and the copy of their results if
//                              `sampled` (into a result buffer that holds no
//                              uncollected results);
//   void defer(const Done&)    remember that request i of group g's sampled
//                              list has its results in that buffer (lock held);
//   int  collect(bool wait, std::vector<Done>*)  the deferred requests whose
//                              results have arrived (all of them, waiting,
//                              if `wait`);
//   void fetch(const Done&)    copy a collected request's results into it
//                              (lock held);
//   int64_t now()              the clock timestamps are taken from.
#ifndef DQ_SCHED_H
#define DQ_SCHED_H

#include "../../include/dqaoa.h"

#include <algorithm>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace dq {
namespace sched {

constexpr int MAX_EVALS_PER_STEP = 16;

struct Req {
  uint64_t id = 0;
  int n = 0;
  size_t bytes = 0;  // device bytes charged while admitted
  int state = 0;     // 0 pending, 1 admitted, 2 done, 3 sampled (results on their way)
  bool cancel = false;
  bool uploaded = false;
  int slot = -1;
  int evals_done = 0;
  qaoa_solve_result res{};
  std::vector<uint64_t> samples;
  virtual ~Req() = default;
};

// The requests of one qubit count in a step.
struct Group {
  int n = 0;
  std::vector<Req*> ev;  // evaluated in every round of the step
  std::vector<Req*> sm;  // sampled and completed if the step runs all K rounds
};

// A sampled request whose results the backend copies back: request i of
// group gi's sampled list in step-local numbering; the backend records where
// the results go (buffer, offset, size of the group's list).
struct Done {
  Req* r = nullptr;
  int gi = 0, i = 0;
  int buf = 0, ns = 0;
  size_t off = 0;
};

struct Step {
  std::vector<Req*> act;    // admitted, not cancelled
  std::vector<Req*> fresh;  // of those, not uploaded yet
  int K = 0;                // evaluation rounds planned
  std::map<int, Group> groups;  // by n, ascending
};

// Queue state.  Every member function expects `mu` held by the caller.
struct Core {
  int evals = 0;
  size_t budget = 0;
  int max_pending = 1;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<Req*> slots;  // by slot index
  std::vector<int> free_slots;
  size_t in_use = 0;
  uint64_t next_id = 1;
  bool stop = false;
  qaoa_queue_stats st{};

  void init(int nslots, int max_pending_, size_t budget_, int evals_) {
    max_pending = max_pending_;
    budget = budget_;
    evals = evals_;
    slots.assign(nslots, nullptr);
    free_slots.clear();
    for (int i = nslots - 1; i >= 0; --i) free_slots.push_back(i);
  }

  // QAOA_ERR_OUT_OF_MEMORY if the request can never fit the budget,
  // QAOA_ERR_QUEUE_FULL if max_pending requests wait already.
  int submit(std::unique_ptr<Req> r, int64_t now, uint64_t* ticket) {
    if (r->bytes > budget) {
      st.rejected++;
      return QAOA_ERR_OUT_OF_MEMORY;
    }
    if ((int)pending.size() >= max_pending) {
      st.rejected++;
      return QAOA_ERR_QUEUE_FULL;
    }
    r->id = next_id++;
    r->state = 0;
    r->res.t_submit_ns = now;
    r->res.status = QAOA_PENDING;
    *ticket = r->id;
    pending.push_back(r->id);
    reqs[r->id] = std::move(r);
    st.submitted++;
    cv_sched.notify_all();
    return QAOA_OK;
  }

  void complete(Req* r, int status, int64_t now) {
    r->res.status = status;
    r->res.n = r->n;
    r->res.t_done_ns = now;
    if (r->state == 1 || r->state == 3) {
      in_use -= r->bytes;
      slots[r->slot] = nullptr;
      free_slots.push_back(r->slot);
      r->slot = -1;
    }
    r->state = 2;
    if (status == QAOA_OK) st.completed++;
    else if (status == QAOA_ERR_CANCELLED) st.cancelled++;
    cv_done.notify_all();
  }

  // Between steps: cancelled running requests complete, then FIFO admission
  // against free slots and the budget.  Returns the requests resident after
  // (running or sampled).
  int admit(int64_t now) {
    for (Req* r : slots)
      if (r && r->cancel && r->state == 1) complete(r, QAOA_ERR_CANCELLED, now);
    while (!pending.empty() && !free_slots.empty()) {
      Req* r = reqs.at(pending.front()).get();
      if (in_use + r->bytes > budget) break;
      pending.pop_front();
      r->slot = free_slots.back();
      free_slots.pop_back();
      slots[r->slot] = r;
      in_use += r->bytes;
      r->state = 1;
      r->res.t_admit_ns = now;
      st.admitted++;
    }
    int resident = 0;
    for (Req* r : slots) resident += r != nullptr;
    st.peak_active = std::max(st.peak_active, resident);
    st.peak_bytes = std::max(st.peak_bytes, in_use);
    return resident;
  }

  // Resident requests in `state` (1 running, 3 sampled).
  int count(int state) const {
    int c = 0;
    for (Req* r : slots) c += r && r->state == state;
    return c;
  }

  // The next step over the running requests; false if there are none.
  bool plan(Step* s) {
    for (Req* r : slots)
      if (r && !r->cancel && r->state == 1) {
        s->act.push_back(r);
        if (!r->uploaded) s->fresh.push_back(r);
      }
    if (s->act.empty()) return false;
    int K = MAX_EVALS_PER_STEP;
    bool evaluating = false;
    for (Req* r : s->act)
      if (r->evals_done < evals) {
        K = std::min(K, evals - r->evals_done);
        evaluating = true;
      }
    s->K = evaluating ? K : 1;
    for (Req* r : s->act) {
      Group& g = s->groups[r->n];
      g.n = r->n;
      if (r->evals_done < evals) {
        g.ev.push_back(r);
        if (r->evals_done + s->K == evals) g.sm.push_back(r);
      } else {
        g.sm.push_back(r);
      }
    }
    return true;
  }

  // A waiting request that could be admitted right now, or a cancelled one
  // among those running, ends the step early.
  bool should_yield(const std::vector<Req*>& act) const {
    for (Req* r : act)
      if (r->cancel) return true;
    if (pending.empty() || free_slots.empty()) return false;
    return in_use + reqs.at(pending.front())->bytes <= budget;
  }

  // After a failed step: every resident request (running or sampled)
  // completes with `status`.
  void fail_active(int status, int64_t now) {
    for (Req* r : slots)
      if (r) complete(r, status, now);
  }

  // QAOA_ERR_NOT_FOUND if the ticket is unknown or finished.
  int cancel(uint64_t ticket, int64_t now) {
    auto it = reqs.find(ticket);
    if (it == reqs.end() || it->second->state == 2) return QAOA_ERR_NOT_FOUND;
    Req* r = it->second.get();
    if (r->state == 0) {
      pending.erase(std::find(pending.begin(), pending.end(), ticket));
      complete(r, QAOA_ERR_CANCELLED, now);
    } else {
      r->cancel = true;
      cv_sched.notify_all();
    }
    return QAOA_OK;
  }

  bool finished(uint64_t ticket) const {
    auto it = reqs.find(ticket);
    return it == reqs.end() || it->second->state == 2;
  }

  // QAOA_PENDING while queued or running; QAOA_OK once done (result and
  // samples copied out, ticket released); QAOA_ERR_NOT_FOUND if unknown.
  int take(uint64_t ticket, qaoa_solve_result* out, uint64_t* samples) {
    auto it = reqs.find(ticket);
    if (it == reqs.end()) return QAOA_ERR_NOT_FOUND;
    Req* r = it->second.get();
    if (r->state != 2) return QAOA_PENDING;
    if (out) *out = r->res;
    if (samples && !r->samples.empty())
      std::copy(r->samples.begin(), r->samples.end(), samples);
    reqs.erase(it);
    return QAOA_OK;
  }

  qaoa_queue_stats stats() const {
    qaoa_queue_stats out = st;
    out.pending = (int)pending.size();
    int act = 0;
    for (Req* r : slots) act += r != nullptr;
    out.active = act;
    out.bytes_in_use = in_use;
    return out;
  }
};

// Collects the sampled requests whose results have arrived (all of them,
// waiting, if `wait`) and completes them.  Called without the lock.
template <class Backend>
int finish_sampled(Core& c, Backend& b, bool wait) {
  std::vector<Done> done;
  int rc = b.collect(wait, &done);
  if (rc) return rc;
  if (done.empty()) return QAOA_OK;
  std::lock_guard<std::mutex> lk(c.mu);
  for (const Done& d : done) {
    if (d.r->state != 3) continue;  // completed otherwise meanwhile
    b.fetch(d);
    c.complete(d.r, d.r->cancel ? QAOA_ERR_CANCELLED : QAOA_OK, b.now());
  }
  return QAOA_OK;
}

// One step over the running requests (see the header comment).  Called
// without the lock; takes it for planning and bookkeeping only.
template <class Backend>
int run_step(Core& c, Backend& b) {
  int rc = finish_sampled(c, b, false);
  if (rc) return rc;
  Step s;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.plan(&s)) return QAOA_OK;
  }
  rc = b.begin(s);
  if (rc) return rc;
  for (Req* r : s.fresh) r->uploaded = true;
  int Kdone = s.K;
  for (int k = 0; k < s.K; ++k) {
    if (k >= 2) {
      rc = b.wait_round(k - 2);
      if (rc) return rc;
      std::lock_guard<std::mutex> lk(c.mu);
      if (c.should_yield(s.act)) {
        Kdone = k;
        break;
      }
    }
    rc = b.round(k);
    if (rc) return rc;
  }
  // requests reach their last evaluation only when the step ran all K rounds
  // (K is the fewest evaluations any request has left)
  bool sampled = false;
  if (Kdone == s.K)
    for (auto& kv : s.groups) sampled = sampled || !kv.second.sm.empty();
  if (sampled) {
    rc = finish_sampled(c, b, true);  // frees a result buffer
    if (rc) return rc;
  }
  rc = b.end(sampled);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c.mu);
  int gi = 0;
  for (auto& kv : s.groups) {
    Group& g = kv.second;
    for (Req* r : g.ev) r->evals_done += Kdone;
    if (sampled)
      for (size_t i = 0; i < g.sm.size(); ++i) {
        g.sm[i]->state = 3;
        b.defer(Done{g.sm[i], gi, (int)i});
      }
    ++gi;
  }
  c.st.steps++;
  return QAOA_OK;
}

}  // namespace sched
}  // namespace dq

#endif  // DQ_SCHED_H
