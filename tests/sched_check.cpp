// The solve queue's scheduling policy (paper_2506_10531_amd/csrc/sched.h)
// driven on the CPU by a host backend with a virtual clock, in place of the
// GPU.  The backend keeps per-slot "device" state like the real queue (the
// parameters and evaluation count of the request that owns the slot) and
// applies a deterministic stand-in for one evaluation (an Adam-like update
// of one parameter from the request's own data), so every result depends
// only on its request; a round costs virtual time by the 2^n sizes of its
// groups on four streams.  The scheduler's own loop (admit, step) runs as in
// the device queue.  Checked:
//   * FIFO admission, never past the slots or the byte budget, and no
//     overtaking of a waiting head request by a smaller one;
//   * every completed request ran exactly `evals` evaluations on the slot it
//     owned, and its result is bitwise what it gets alone in the queue;
//   * back-pressure (QUEUE_FULL at max_pending, OUT_OF_MEMORY for a request
//     that can never fit), cancellation of pending and running requests,
//     failure of a step, evals = 0, and the ticket life cycle;
//   * latency: with room to admit, an arrival waits at most about three
//     rounds plus a sampling phase (the early end of a step);
//   * timestamps t_submit <= t_admit <= t_done, and the counters.
// Prints "ok <checks>" and exits 0, or lists the failures and exits 1.
#include "../paper_2506_10531_amd/csrc/sched.h"

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <vector>

using namespace dq::sched;

static long checks = 0, fails = 0;
#define CHECK(c, ...)                                       \
  do {                                                      \
    ++checks;                                               \
    if (!(c)) {                                             \
      if (++fails <= 30) {                                  \
        std::printf("FAIL line %d: ", __LINE__);            \
        std::printf(__VA_ARGS__);                           \
        std::printf("\n");                                  \
      }                                                     \
    }                                                       \
  } while (0)

namespace {

constexpr int NSTREAMS = 4;
constexpr int SHOTS = 4;
constexpr int64_t HOST_STEP_NS = 2000, HOST_GROUP_NS = 500;

uint64_t mix64(uint64_t x) {  // SplitMix64 finaliser (seeded test data only)
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

struct TReq : Req {
  double a = 0, b = 0, x0 = 0;
  uint64_t seed = 0;
};

struct Spec {
  int64_t t;  // arrival time
  int n;
  size_t bytes;
  double a, b, x0;
  uint64_t seed;
};

std::vector<Spec> make_trace(int count, uint64_t seed, int nlo, int nhi, int64_t gap) {
  std::vector<Spec> v;
  int64_t t = 0;
  for (int i = 0; i < count; ++i) {
    const uint64_t h = mix64(seed * 1000003 + i);
    Spec s;
    t += (int64_t)(h % (uint64_t)(2 * gap + 1));
    s.t = t;
    s.n = nlo + (int)((h >> 20) % (uint64_t)(nhi - nlo + 1));
    s.bytes = ((size_t)64 << s.n) + 4096;
    s.a = 0.5 + (double)((h >> 30) & 1023) / 1024.0;
    s.b = 0.1 + (double)((h >> 40) & 255) / 512.0;
    s.x0 = -1.0 + (double)((h >> 48) & 4095) / 2048.0;
    s.seed = h;
    v.push_back(s);
  }
  return v;
}

struct Result {
  int status = 1;
  qaoa_solve_result res{};
  std::vector<uint64_t> samples;
  int64_t t_arrive = 0;
};

// The host backend.  Scripted actions (arrivals, cancellations) fire when
// the host clock passes their time, as if another thread called the queue.
struct Fake {
  Core& c;
  int evals;
  int64_t t = 0, dev_free = 0;
  int64_t done_at[2] = {0, 0};  // completion of the last two rounds
  int64_t max_round = 0, sample_cost = 0;
  std::vector<double> x;        // per slot: the parameter
  std::vector<int> count;       // per slot: evaluations applied
  std::vector<uint64_t> owner;  // per slot: request id
  Step* step = nullptr;
  std::vector<std::pair<int64_t, std::function<void()>>> actions;
  size_t next_action = 0;
  int fail_round = -1;  // fail round k of the next step that reaches it
  long rounds = 0, steps = 0;
  std::vector<Done> deferred;  // sampled, results not collected yet
  int64_t res_at = 0;          // when they arrive

  Fake(Core& core, int nslots, int ev) : c(core), evals(ev), x(nslots), count(nslots),
                                         owner(nslots) {}

  void fire() {
    while (next_action < actions.size() && actions[next_action].first <= t)
      actions[next_action++].second();
  }

  int begin(Step& s) {
    step = &s;
    ++steps;
    t += HOST_STEP_NS;
    {
      std::lock_guard<std::mutex> lk(c.mu);
      size_t bytes = 0;
      int resident = 0;
      for (Req* r : c.slots)
        if (r) {
          bytes += r->bytes;
          ++resident;
          CHECK((r->state == 1 || r->state == 3) && c.slots[r->slot] == r, "slot table");
        }
      CHECK(bytes == c.in_use && c.in_use <= c.budget, "bytes %zu in_use %zu budget %zu", bytes,
            c.in_use, c.budget);
      CHECK(resident + (int)c.free_slots.size() == (int)c.slots.size(), "slot count");
    }
    CHECK(s.K >= 1 && s.K <= MAX_EVALS_PER_STEP, "K = %d", s.K);
    int prev_n = -1;
    for (auto& kv : s.groups) {
      CHECK(kv.first > prev_n && kv.second.n == kv.first, "group order");
      prev_n = kv.first;
      for (Req* r : kv.second.ev) {
        CHECK(r->n == kv.first, "group n");
        CHECK(r->evals_done + s.K <= evals, "K past the evaluations left");
      }
      for (Req* r : kv.second.sm)
        CHECK(r->evals_done + (r->evals_done < evals ? s.K : 0) == evals, "sampled early");
    }
    for (Req* r : s.fresh) {  // upload
      const TReq* q = static_cast<const TReq*>(r);
      CHECK(!r->uploaded && r->slot >= 0, "fresh request");
      x[r->slot] = q->x0;
      count[r->slot] = 0;
      owner[r->slot] = r->id;
    }
    fire();
    return QAOA_OK;
  }

  int round(int k) {
    if (k == fail_round) {
      fail_round = -1;
      return QAOA_ERR_HIP;
    }
    ++rounds;
    int64_t stream[NSTREAMS] = {};
    int gi = 0;
    for (auto& kv : step->groups) {
      const Group& g = kv.second;
      t += HOST_GROUP_NS;
      if (g.ev.empty()) {
        ++gi;
        continue;
      }
      for (Req* r : g.ev) {
        const TReq* q = static_cast<const TReq*>(r);
        const int sl = r->slot;
        CHECK(owner[sl] == r->id, "slot %d evaluated for a request it does not hold", sl);
        const double d = q->a * std::cos(x[sl]) + 2.0 * q->b * x[sl];
        x[sl] -= 0.05 * d;
        count[sl]++;
      }
      stream[gi % NSTREAMS] += 5000 + (int64_t)g.ev.size() * ((int64_t)1 << g.n);
      ++gi;
    }
    int64_t cost = 0;
    for (int64_t s : stream) cost = std::max(cost, s);
    max_round = std::max(max_round, cost);
    dev_free = std::max(dev_free, t) + cost;
    done_at[k % 2] = dev_free;
    fire();
    return QAOA_OK;
  }

  int wait_round(int k) {
    t = std::max(t, done_at[k % 2]);
    fire();
    return QAOA_OK;
  }

  // No step is waited for (the device queue orders the next step's work
  // after it); a sampling step's results arrive when its sampling is done.
  int end(bool sampled) {
    if (sampled) {
      CHECK(deferred.empty(), "a sampling step with results still uncollected");
      int64_t cost = 0;
      for (auto& kv : step->groups) cost += 3000 + (int64_t)kv.second.sm.size() * 200;
      sample_cost = std::max(sample_cost, cost);
      dev_free = std::max(dev_free, t) + cost;
      res_at = dev_free;
    }
    fire();
    return QAOA_OK;
  }

  void defer(const Done& d) {
    CHECK(d.r->state == 3, "deferred request not sampled");
    deferred.push_back(d);
  }

  int collect(bool wait, std::vector<Done>* out) {
    if (deferred.empty()) return QAOA_OK;
    if (wait) t = std::max(t, res_at);
    if (t < res_at) return QAOA_OK;
    out->swap(deferred);
    deferred.clear();
    fire();
    return QAOA_OK;
  }

  void fetch(const Done& d) {
    Req* r = d.r;
    const TReq* q = static_cast<const TReq*>(r);
    const int sl = r->slot;
    CHECK(owner[sl] == r->id, "fetch from a slot the request does not hold");
    r->res.gamma[0] = x[sl];
    r->res.beta[0] = (double)count[sl];
    r->res.expect = q->a * std::sin(x[sl]) + q->b * x[sl] * x[sl];
    uint64_t bits;
    std::memcpy(&bits, &x[sl], 8);
    r->res.best_z = q->seed ^ bits;
    r->res.best_c = r->res.expect - 1.0;
    r->samples.clear();
    for (int s = 0; s < SHOTS; ++s) r->samples.push_back(mix64(q->seed + bits + s));
  }

  int64_t now() const { return t; }
};

struct Run {
  std::vector<Result> out;  // by trace index
  qaoa_queue_stats st{};
  int64_t max_round = 0, sample_cost = 0;
  long steps = 0;
};

struct Opts {
  int slots = 16, max_pending = 1 << 20, evals = 37;
  size_t budget = (size_t)1 << 40;
  std::vector<std::pair<int64_t, int>> cancels;  // (time, trace index)
  int fail_round = -1;
  int64_t fail_after = -1;  // arm fail_round once the clock passes this
};

// Serves a trace as the device queue's scheduler thread does: admit, step,
// repeat; when nothing is resident, the clock jumps to the next action.
Run serve(const std::vector<Spec>& trace, const Opts& o) {
  Core c;
  c.init(o.slots, o.max_pending, o.budget, o.evals);
  Fake f(c, o.slots, o.evals);
  Run run;
  run.out.resize(trace.size());
  std::vector<uint64_t> ticket(trace.size(), 0);
  std::vector<std::pair<int64_t, std::function<void()>>> acts;
  for (size_t i = 0; i < trace.size(); ++i)
    acts.push_back({trace[i].t, [&, i] {
                      std::unique_ptr<TReq> r(new TReq());
                      r->n = trace[i].n;
                      r->bytes = trace[i].bytes;
                      r->a = trace[i].a;
                      r->b = trace[i].b;
                      r->x0 = trace[i].x0;
                      r->seed = trace[i].seed;
                      std::lock_guard<std::mutex> lk(c.mu);
                      const int rc = c.submit(std::move(r), f.t, &ticket[i]);
                      run.out[i].t_arrive = f.t;
                      if (rc) run.out[i].status = rc;
                    }});
  for (auto& cn : o.cancels)
    acts.push_back({cn.first, [&, cn] {
                      std::lock_guard<std::mutex> lk(c.mu);
                      if (ticket[cn.second]) (void)c.cancel(ticket[cn.second], f.t);
                    }});
  if (o.fail_after >= 0)
    acts.push_back({o.fail_after, [&] { f.fail_round = o.fail_round; }});
  std::stable_sort(acts.begin(), acts.end(),
                   [](const auto& a, const auto& b) { return a.first < b.first; });
  f.actions = std::move(acts);
  int64_t last_t = -1;
  long idle = 0;  // loop passes without the clock moving
  for (;;) {
    idle = f.t == last_t ? idle + 1 : 0;
    last_t = f.t;
    if (idle > 1000) {
      CHECK(false, "the scheduler stopped making progress at t = %" PRId64, f.t);
      break;
    }
    f.fire();
    int running, sampled;
    {
      std::lock_guard<std::mutex> lk(c.mu);
      c.admit(f.t);
      running = c.count(1);
      sampled = c.count(3);
    }
    if (running || sampled) {
      const int rc = running ? run_step(c, f) : finish_sampled(c, f, true);
      if (rc != QAOA_OK) {
        std::lock_guard<std::mutex> lk(c.mu);
        c.fail_active(QAOA_ERR_HIP, f.t);
        f.deferred.clear();
      }
      continue;
    }
    if (f.next_action < f.actions.size()) {
      f.t = std::max(f.t, f.actions[f.next_action].first);
      continue;
    }
    break;
  }
  std::lock_guard<std::mutex> lk(c.mu);
  for (size_t i = 0; i < trace.size(); ++i) {
    if (!ticket[i]) continue;
    Result& r = run.out[i];
    std::vector<uint64_t> smp(SHOTS, 0);
    const int rc = c.take(ticket[i], &r.res, smp.data());
    CHECK(rc == QAOA_OK, "request %zu not finished (%d)", i, rc);
    r.status = r.res.status;
    if (r.status == QAOA_OK) r.samples = smp;
    CHECK(c.take(ticket[i], nullptr, nullptr) == QAOA_ERR_NOT_FOUND, "ticket released");
  }
  run.st = c.stats();
  run.max_round = f.max_round;
  run.sample_cost = f.sample_cost;
  run.steps = f.steps;
  CHECK(idle > 1000 || (c.in_use == 0 && c.pending.empty() && c.reqs.empty()), "queue drained");
  return run;
}

// The request of trace entry `sp` served by itself in a one-slot queue.
Result alone(const Spec& sp, const Opts& o) {
  Opts a;
  a.slots = 1;
  a.evals = o.evals;
  a.budget = o.budget;
  std::vector<Spec> one{sp};
  one[0].t = 0;
  return serve(one, a).out[0];
}

bool same(const Result& a, const Result& b) {
  return a.status == b.status && std::memcmp(&a.res.gamma[0], &b.res.gamma[0], 8) == 0 &&
         a.res.beta[0] == b.res.beta[0] && std::memcmp(&a.res.expect, &b.res.expect, 8) == 0 &&
         a.res.best_z == b.res.best_z && a.samples == b.samples;
}

void check_fifo(const std::vector<Spec>& trace, const Run& r) {
  int64_t last = -1;
  for (size_t i = 0; i < trace.size(); ++i) {
    const Result& x = r.out[i];
    if (x.status == QAOA_ERR_CANCELLED && x.res.t_admit_ns == 0) continue;  // cancelled pending
    if (x.status != QAOA_OK && x.status != QAOA_ERR_CANCELLED && x.status != QAOA_ERR_HIP)
      continue;  // refused at submission
    CHECK(x.res.t_admit_ns >= last, "request %zu admitted before an earlier one", i);
    last = x.res.t_admit_ns;
    CHECK(x.res.t_submit_ns <= x.res.t_admit_ns && x.res.t_admit_ns <= x.res.t_done_ns,
          "timestamps of %zu", i);
  }
}

// A mixed trace under a tight budget against each request served alone.
void test_mix_equals_alone() {
  const auto trace = make_trace(240, 7, 3, 12, 4000);
  Opts o;
  o.slots = 16;
  o.budget = ((size_t)64 << 12) * 3 + ((size_t)64 << 10) * 4;  // a few requests at a time
  const Run mix = serve(trace, o);
  check_fifo(trace, mix);
  CHECK(mix.st.submitted == 240 && mix.st.admitted == 240 && mix.st.completed == 240 &&
            mix.st.rejected == 0 && mix.st.cancelled == 0,
        "counters %lld %lld %lld", mix.st.submitted, mix.st.admitted, mix.st.completed);
  CHECK(mix.st.peak_bytes <= o.budget && mix.st.peak_active <= o.slots, "peaks");
  CHECK(mix.st.peak_active > 1, "requests shared steps (peak %d)", mix.st.peak_active);
  for (size_t i = 0; i < trace.size(); ++i) {
    CHECK(mix.out[i].status == QAOA_OK, "request %zu status %d", i, mix.out[i].status);
    CHECK(mix.out[i].res.beta[0] == o.evals, "request %zu ran %g evaluations", i,
          mix.out[i].res.beta[0]);
    CHECK(mix.out[i].res.n == trace[i].n, "n");
    CHECK(same(mix.out[i], alone(trace[i], o)), "request %zu differs from its run alone", i);
  }
  // one slot: the same trace served one request at a time, in order
  Opts s1 = o;
  s1.slots = 1;
  const Run seq = serve(trace, s1);
  check_fifo(trace, seq);
  for (size_t i = 0; i < trace.size(); ++i)
    CHECK(same(mix.out[i], seq.out[i]), "request %zu differs one at a time", i);
  CHECK(seq.st.peak_active == 1, "one slot");
}

// With room to admit, an arrival waits at most about three rounds plus a
// sampling phase, however many evaluations the running requests have left.
void test_arrival_latency() {
  std::vector<Spec> trace = make_trace(60, 11, 4, 12, 30000);
  Opts o;
  o.evals = 400;
  o.slots = 64;
  const Run r = serve(trace, o);
  int64_t worst = 0;
  for (size_t i = 0; i < trace.size(); ++i) {
    CHECK(r.out[i].status == QAOA_OK && r.out[i].res.beta[0] == o.evals, "request %zu", i);
    worst = std::max(worst, r.out[i].res.t_admit_ns - r.out[i].t_arrive);
  }
  const int64_t bound = 3 * r.max_round + r.sample_cost + 64 * HOST_GROUP_NS + 2 * HOST_STEP_NS;
  CHECK(worst <= bound, "an arrival waited %" PRId64 " ns (bound %" PRId64 ")", worst, bound);
  CHECK(r.steps > (long)trace.size(), "steps ended early for arrivals (%ld steps)", r.steps);
  // the early ends do not change any result
  for (size_t i = 0; i < trace.size(); i += 7) {
    CHECK(same(r.out[i], alone(trace[i], o)), "request %zu differs from its run alone", i);
  }
}

void test_backpressure_and_budget() {
  Core c;
  c.init(4, 3, 10000, 5);
  auto mk = [](int n, size_t bytes) {
    std::unique_ptr<TReq> r(new TReq());
    r->n = n;
    r->bytes = bytes;
    return r;
  };
  std::lock_guard<std::mutex> lk(c.mu);
  uint64_t t[6] = {};
  CHECK(c.submit(mk(5, 6000), 1, &t[0]) == QAOA_OK, "submit");
  CHECK(c.submit(mk(6, 8000), 2, &t[1]) == QAOA_OK, "submit");
  CHECK(c.submit(mk(3, 1000), 3, &t[2]) == QAOA_OK, "submit");
  CHECK(c.submit(mk(3, 1000), 4, &t[3]) == QAOA_ERR_QUEUE_FULL, "max_pending");
  CHECK(c.submit(mk(9, 10001), 5, &t[4]) == QAOA_ERR_OUT_OF_MEMORY, "never fits");
  CHECK(c.stats().rejected == 2 && c.stats().pending == 3, "counters");
  // the 8000-byte head cannot join the 6000 in use; the 1000-byte request
  // behind it must not overtake it
  CHECK(c.admit(10) == 1, "admitted one");
  CHECK(c.in_use == 6000 && c.pending.size() == 2 && c.pending.front() == t[1], "FIFO head");
  Step s;
  CHECK(c.plan(&s) && s.act.size() == 1 && s.K == 5, "plan");
  CHECK(c.should_yield(s.act) == false, "nothing admissible");
  c.reqs.at(t[0])->cancel = true;
  CHECK(c.should_yield(s.act), "a cancellation ends the step");
  CHECK(c.admit(20) == 2, "the cancelled one leaves; the head and the one behind it enter");
  CHECK(c.take(t[0], nullptr, nullptr) == QAOA_OK, "cancelled result");
  CHECK(c.in_use == 9000 && c.pending.empty(), "head in");
  CHECK(c.submit(mk(3, 1000), 21, &t[5]) == QAOA_OK, "room again");
  CHECK(c.take(t[5], nullptr, nullptr) == QAOA_PENDING, "pending");
  CHECK(c.cancel(t[5], 22) == QAOA_OK, "cancel pending");
  qaoa_solve_result res{};
  CHECK(c.take(t[5], &res, nullptr) == QAOA_OK && res.status == QAOA_ERR_CANCELLED &&
            res.t_admit_ns == 0 && res.t_done_ns == 22,
        "pending cancelled at once");
  CHECK(c.cancel(t[5], 23) == QAOA_ERR_NOT_FOUND && c.cancel(999, 23) == QAOA_ERR_NOT_FOUND,
        "unknown tickets");
  CHECK(c.submit(mk(4, 2000), 24, &t[4]) == QAOA_OK, "submit");
  CHECK(c.admit(30) == 2 && c.in_use == 9000 && c.pending.size() == 1, "over the budget waits");
  const qaoa_queue_stats st = c.stats();
  CHECK(st.cancelled == 2 && st.admitted == 3 && st.active == 2 && st.peak_bytes == 9000,
        "stats %lld %lld %d %zu", st.cancelled, st.admitted, st.active, st.peak_bytes);
}

// Running requests cancelled mid-step end the step early and leave at the
// boundary; the others finish as if alone.
void test_cancel_running() {
  const auto trace = make_trace(20, 5, 5, 10, 1000);
  Opts o;
  o.evals = 200;
  o.slots = 8;
  // request 2 runs by then (a running cancel), 9 and 15 wait (pending cancels)
  o.cancels = {{60000, 2}, {61000, 9}, {trace[15].t + 1, 15}};
  const Run r = serve(trace, o);
  CHECK(r.out[2].res.t_admit_ns > 0 && r.out[2].res.t_admit_ns < 60000, "2 was running");
  CHECK(r.out[2].res.t_done_ns - 60000 <= 3 * r.max_round + r.sample_cost + 20 * HOST_GROUP_NS +
                                               2 * HOST_STEP_NS,
        "the running cancel ended its step early (done at %" PRId64 ")", r.out[2].res.t_done_ns);
  CHECK(r.out[9].res.t_admit_ns == 0 && r.out[15].res.t_admit_ns == 0, "9 and 15 waited");
  for (size_t i = 0; i < trace.size(); ++i) {
    const bool cancelled = i == 2 || i == 9 || i == 15;
    if (cancelled) {
      CHECK(r.out[i].status == QAOA_ERR_CANCELLED, "request %zu status %d", i, r.out[i].status);
      continue;
    }
    CHECK(r.out[i].status == QAOA_OK && r.out[i].res.beta[0] == o.evals, "request %zu", i);
    CHECK(same(r.out[i], alone(trace[i], o)), "request %zu differs from its run alone", i);
  }
  CHECK(r.st.cancelled == 3 && r.st.completed == 17, "counters");
  check_fifo(trace, r);
}

// A failed step completes its admitted requests with QAOA_ERR_HIP; the queue
// serves the rest.
void test_failed_step() {
  const auto trace = make_trace(30, 9, 4, 9, 3000);
  Opts o;
  o.slots = 4;
  o.evals = 40;
  o.fail_round = 3;
  o.fail_after = 20000;
  const Run r = serve(trace, o);
  int failed = 0, ok = 0;
  for (size_t i = 0; i < trace.size(); ++i) {
    if (r.out[i].status == QAOA_ERR_HIP) {
      ++failed;
    } else {
      CHECK(r.out[i].status == QAOA_OK && r.out[i].res.beta[0] == o.evals, "request %zu", i);
      CHECK(same(r.out[i], alone(trace[i], o)), "request %zu differs from its run alone", i);
      ++ok;
    }
  }
  CHECK(failed >= 1 && failed <= o.slots && ok == 30 - failed, "failed %d ok %d", failed, ok);
}

// A request whose results are on their way keeps its slot, is not planned
// again, reads as pending, and completes as cancelled if cancelled then.
void test_results_in_flight() {
  Core c;
  c.init(2, 8, 1 << 20, 2);
  Fake f(c, 2, 2);
  auto mk = [](uint64_t seed) {
    std::unique_ptr<TReq> r(new TReq());
    r->n = 6;
    r->bytes = 1000;
    r->a = 0.7;
    r->b = 0.2;
    r->x0 = 0.3;
    r->seed = seed;
    return r;
  };
  uint64_t ta = 0, tb = 0;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    CHECK(c.submit(mk(1), 0, &ta) == QAOA_OK && c.submit(mk(2), 0, &tb) == QAOA_OK, "submit");
    CHECK(c.admit(0) == 2, "both admitted");
  }
  CHECK(run_step(c, f) == QAOA_OK, "step");  // two rounds, then both sampled
  {
    std::lock_guard<std::mutex> lk(c.mu);
    CHECK(c.count(3) == 2 && c.count(1) == 0 && c.in_use == 2000, "sampled, slots held");
    CHECK(c.take(ta, nullptr, nullptr) == QAOA_PENDING, "results not collected yet");
    Step s;
    CHECK(!c.plan(&s), "sampled requests are not planned");
    CHECK(c.cancel(ta, f.t) == QAOA_OK, "cancel while results are on their way");
    CHECK(c.admit(f.t) == 2 && c.count(3) == 2, "a sampled request leaves only when collected");
  }
  CHECK(finish_sampled(c, f, true) == QAOA_OK, "collect");
  std::lock_guard<std::mutex> lk(c.mu);
  qaoa_solve_result ra{}, rb{};
  CHECK(c.take(ta, &ra, nullptr) == QAOA_OK && ra.status == QAOA_ERR_CANCELLED, "cancelled");
  CHECK(c.take(tb, &rb, nullptr) == QAOA_OK && rb.status == QAOA_OK && rb.beta[0] == 2.0,
        "completed after two evaluations");
  CHECK(c.in_use == 0 && c.count(3) == 0, "slots released");
}

// evals = 0: one step samples every request at its initial parameters.
void test_no_evaluations() {
  const auto trace = make_trace(12, 3, 3, 8, 500);
  Opts o;
  o.evals = 0;
  o.slots = 5;
  const Run r = serve(trace, o);
  for (size_t i = 0; i < trace.size(); ++i) {
    CHECK(r.out[i].status == QAOA_OK && r.out[i].res.beta[0] == 0.0 &&
              r.out[i].res.gamma[0] == trace[i].x0,
          "request %zu", i);
  }
}

}  // namespace

int main() {
  test_backpressure_and_budget();
  test_no_evaluations();
  test_results_in_flight();
  test_cancel_running();
  test_failed_step();
  test_arrival_latency();
  test_mix_equals_alone();
  if (fails) {
    std::printf("%ld of %ld checks failed\n", fails, checks);
    return 1;
  }
  std::printf("ok %ld checks\n", checks);
  return 0;
}
