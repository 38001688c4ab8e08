// Solve queue: continuous batching of sub-QUBO solves on one GPU.
//
// The "parallel processing" step of the DQAOA workflow (arXiv 2506.10531,
// Sec. V) hands many small sub-QUBOs to QAOA solvers and collects their
// sub-solutions asynchronously; the paper's QFw integration submits ansatz
// evaluations to an executor and feeds the results back to the optimiser
// (Sec. VI).  Here one GPU serves that stream of solves:
//
//  * qaoa_submit copies a request (n, Q, initial gamma/beta, seed) into a
//    FIFO.  A scheduler thread admits requests in FIFO order while a slot is
//    free and the request's device bytes fit in the queue's HBM budget.
//  * An admitted request keeps its Q, parameters and Adam moments in a
//    device slot.  Every scheduler step advances all admitted requests by
//    the same number of evaluations: the requests are grouped by qubit
//    count, each group is gathered into a contiguous batch, and one batched
//    adjoint pipeline (forward passes, lambda = C psi, backward passes,
//    fixed-order reductions) plus one Adam update runs per group and
//    evaluation, groups on separate streams.  Requests that finish their
//    evaluations are sampled in the same step and completed.  Requests that
//    arrive meanwhile join at the next step, so their work overlaps with the
//    requests already running.  A step makes up to MAX_EVALS_PER_STEP
//    evaluations, no more than any of its requests has left, enqueued round
//    by round with at most two rounds in flight; before each further round
//    the scheduler looks for a waiting request that a free slot and the
//    byte budget could now take (or a cancellation), and if there is one it
//    ends the step after the rounds already enqueued, so an arrival waits
//    at most about two evaluations while the GPU stays busy.
//  * The big buffers (checkpoints, adjoint state, probabilities) exist only
//    within a step; a request's byte charge is what its group needs for it
//    during a step, so the sum over admitted requests bounds the arena.
//
// Every kernel works per state with a tile structure that depends only on
// (n, p, precision), and every reduction sums in a fixed order, so a
// request's result does not depend on which requests share its batch.
#include "internal.h"
#include "../../include/dqaoa.h"

#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace dq {
int ctx_device(qaoa_ctx* c);
size_t ctx_budget(qaoa_ctx* c);
}  // namespace dq

using namespace dq;

namespace {

constexpr int QN_MAX = 26;      // largest sub-QUBO a request may carry
constexpr int NSTREAMS = 4;
constexpr int MAX_EVALS_PER_STEP = 16;

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

struct Request {
  uint64_t id = 0;
  int n = 0;
  std::vector<double> Q, g0, b0;
  uint64_t seed = 0;
  size_t bytes = 0;
  int state = 0;  // 0 pending, 1 active, 2 done
  bool cancel = false;
  bool uploaded = false;
  int slot = -1;
  int evals_done = 0;
  qaoa_solve_result res{};
  std::vector<uint64_t> samples;
};

// Per-group scratch of one step: contiguous batch arrays plus the pipelines'
// layouts.
struct GroupPlan {
  int n = 0;
  std::vector<Request*> ev, sm;  // evaluating, sampling this step
  Layout lg, ls;
  Carve cv;
  size_t iQe = 0, iGe = 0, iBe = 0, iE = 0, iDg = 0, iDb = 0, iGrad = 0;
  size_t iQs = 0, iGs = 0, iBs = 0, iZ = 0, iBz = 0, iBc = 0, iEs = 0, iSd = 0,
         iSamp = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct qaoa_queue {
  qaoa_ctx* ctx = nullptr;
  qaoa_queue_opts o{};
  int device = 0;
  size_t budget = 0;

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<Request*> slots;  // by slot index
  std::vector<int> free_slots;
  size_t in_use = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread th;
  qaoa_queue_stats st{};

  // device state
  hipStream_t streams[NSTREAMS] = {};
  hipEvent_t ev_up = nullptr;
  hipEvent_t ev_round[2][NSTREAMS] = {};  // the last two evaluation rounds per stream
  char* arena = nullptr;
  double *dQ = nullptr, *dG = nullptr, *dB = nullptr, *dM = nullptr, *dV = nullptr;
  uint64_t* dSeed = nullptr;
  int* dT = nullptr;
  int* dIdx = nullptr;
  // pinned host staging
  double* hUp = nullptr;     // uploads [slots][QN_MAX^2 + 2p]
  int* hIdx = nullptr;       // [2 * slots]
  char* hRes = nullptr;      // results of one step
  size_t hRes_bytes = 0;

  // Captured evaluation steps: the gather, adjoint pipeline and Adam update
  // of one n-group, replayed while the group's size and its places in the
  // arena and index buffer recur (the index contents are uploaded before
  // each replay).  Bounded; the least recently used graph goes first.
  struct GraphKey {
    int n, nb;
    const char* base;
    const int* ie;
    bool operator<(const GraphKey& o) const {
      if (n != o.n) return n < o.n;
      if (nb != o.nb) return nb < o.nb;
      if (base != o.base) return base < o.base;
      return ie < o.ie;
    }
  };
  struct GraphEntry {
    hipGraphExec_t exec;
    uint64_t last;
  };
  std::map<GraphKey, GraphEntry> graphs;
  bool use_graphs = true;
  uint64_t step_no = 0;
  long long graph_launches = 0, graph_captures = 0;

  size_t request_bytes(int n) const;
  void run();
  int step();
  int eval_group(const GroupPlan& g, const int* ie, char* base, hipStream_t s);
  int enqueue_eval(const GroupPlan& g, const int* ie, char* base, hipStream_t s);
  void complete(Request* r, int status);
  bool should_yield(const std::vector<Request*>& act);
};

// Called with the lock held: a waiting request that could be admitted right
// now, or a cancelled request among those running, ends the step early.
bool qaoa_queue::should_yield(const std::vector<Request*>& act) {
  for (Request* r : act)
    if (r->cancel) return true;
  if (pending.empty() || free_slots.empty()) return false;
  return in_use + reqs[pending.front()]->bytes <= budget;
}

// One evaluation of an n-group: gather its requests' Q and parameters,
// the adjoint pipeline, the Adam update.  Kernels only (capturable).
int qaoa_queue::enqueue_eval(const GroupPlan& g, const int* ie, char* base, hipStream_t s) {
  const int n = g.n, nb = (int)g.ev.size(), p = o.p;
  auto A = [&](size_t i) { return base + g.cv.off[i]; };
  double *Q = (double*)A(g.iQe), *gg = (double*)A(g.iGe), *bb = (double*)A(g.iBe);
  double *E = (double*)A(g.iE), *dg = (double*)A(g.iDg), *db = (double*)A(g.iDb);
  hipError_t e = launch_gather(nb, n, p, ie, dQ, QN_MAX * QN_MAX, dG, dB, nullptr, Q, gg, bb,
                               nullptr, s);
  if (e != hipSuccess) return hip_error(e, "gather");
  int rc = enqueue_grad(g.lg, A(g.iGrad), Q, gg, bb, E, dg, db, s, nullptr);
  if (rc) return rc;
  e = launch_adam(nb, p, ie, dG, dB, dM, dV, dg, db, dT, o.lr, o.beta1, o.beta2, o.eps, s);
  if (e != hipSuccess) return hip_error(e, "adam");
  return QAOA_OK;
}

// The group's evaluation as a graph replay when its shape recurs, captured
// on first use; eager when graphs are off.
int qaoa_queue::eval_group(const GroupPlan& g, const int* ie, char* base, hipStream_t s) {
  if (!use_graphs) return enqueue_eval(g, ie, base, s);
  const GraphKey key{g.n, (int)g.ev.size(), base, ie};
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    if (graphs.size() >= 256) {  // evict the least recently used (not in flight:
      auto lru = graphs.begin();  // every step ends with its streams drained)
      for (auto j = graphs.begin(); j != graphs.end(); ++j)
        if (j->second.last < lru->second.last) lru = j;
      (void)hipGraphExecDestroy(lru->second.exec);
      graphs.erase(lru);
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    int rc = enqueue_eval(g, ie, base, s);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (rc || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc ? rc : hip_error(e2, "hipStreamEndCapture");
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
    it = graphs.emplace(key, GraphEntry{ex, step_no}).first;
    ++graph_captures;
  }
  it->second.last = step_no;
  hipError_t e = hipGraphLaunch(it->second.exec, s);
  if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
  ++graph_launches;
  return QAOA_OK;
}

size_t qaoa_queue::request_bytes(int n) const {
  Layout lg, ls;
  if (make_layout(OP_GRAD, o.prec, 1, n, o.p, 1, 0, &lg)) return SIZE_MAX;
  if (make_layout(OP_SAMPLE, o.prec, 1, n, o.p, 1, o.shots, &ls)) return SIZE_MAX;
  const size_t arrays = 2 * align256(n * n * 8 + 256) + 4 * align256(o.p * 8 + 256) +
                        3 * align256(8 + 256) + align256(8 * o.shots + 256) +
                        4 * align256(8 + 256);
  return lg.cv.total + ls.cv.total + arrays + 4096;
}

void qaoa_queue::complete(Request* r, int status) {
  r->res.status = status;
  r->res.n = r->n;
  r->res.t_done_ns = now_ns();
  if (r->state == 1) {
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

// One scheduler step over all admitted requests.  Called without the lock
// held; takes it for bookkeeping only.
int qaoa_queue::step() {
  ++step_no;
  std::vector<Request*> act, fresh;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : slots)
      if (r) {
        if (r->cancel) continue;
        act.push_back(r);
        if (!r->uploaded) fresh.push_back(r);
      }
  }
  if (act.empty()) return QAOA_OK;
  // evaluations per request this step (fewer if an arrival ends it early)
  int K = MAX_EVALS_PER_STEP;
  bool evaluating = false;
  for (Request* r : act)
    if (r->evals_done < o.evals) {
      K = std::min(K, o.evals - r->evals_done);
      evaluating = true;
    }
  if (!evaluating) K = 1;
  const int p = o.p;
  hipStream_t s0 = streams[0];
  // upload newly admitted requests: Q, gamma0, beta0; zero Adam state
  for (size_t i = 0; i < fresh.size(); ++i) {
    Request* r = fresh[i];
    double* h = hUp + i * (QN_MAX * QN_MAX + 2 * p + 1);
    std::memcpy(h, r->Q.data(), sizeof(double) * r->n * r->n);
    std::memcpy(h + QN_MAX * QN_MAX, r->g0.data(), sizeof(double) * p);
    std::memcpy(h + QN_MAX * QN_MAX + p, r->b0.data(), sizeof(double) * p);
    std::memcpy(h + QN_MAX * QN_MAX + 2 * p, &r->seed, sizeof(uint64_t));
    const int sl = r->slot;
    hipError_t e = hipMemcpyAsync(dQ + (size_t)sl * QN_MAX * QN_MAX, h,
                                  sizeof(double) * r->n * r->n, hipMemcpyHostToDevice, s0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dG + (size_t)sl * p, h + QN_MAX * QN_MAX, sizeof(double) * p,
                         hipMemcpyHostToDevice, s0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dB + (size_t)sl * p, h + QN_MAX * QN_MAX + p, sizeof(double) * p,
                         hipMemcpyHostToDevice, s0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dSeed + sl, h + QN_MAX * QN_MAX + 2 * p, sizeof(uint64_t),
                         hipMemcpyHostToDevice, s0);
    if (e == hipSuccess) e = hipMemsetAsync(dM + (size_t)sl * 2 * p, 0, sizeof(double) * 2 * p, s0);
    if (e == hipSuccess) e = hipMemsetAsync(dV + (size_t)sl * 2 * p, 0, sizeof(double) * 2 * p, s0);
    if (e == hipSuccess) e = hipMemsetAsync(dT + sl, 0, sizeof(int), s0);
    if (e != hipSuccess) return hip_error(e, "queue upload");
    r->uploaded = true;
  }
  // groups by n
  std::map<int, GroupPlan> groups;
  for (Request* r : act) {
    GroupPlan& g = groups[r->n];
    g.n = r->n;
    if (r->evals_done < o.evals) {
      g.ev.push_back(r);
      if (r->evals_done + K == o.evals) g.sm.push_back(r);
    } else {
      g.sm.push_back(r);
    }
  }
  // index lists
  int nidx = 0;
  std::vector<std::pair<int, int>> idx_off;  // per group: ev offset, sm offset
  for (auto& kv : groups) {
    GroupPlan& g = kv.second;
    const int a = nidx;
    for (Request* r : g.ev) hIdx[nidx++] = r->slot;
    const int b = nidx;
    for (Request* r : g.sm) hIdx[nidx++] = r->slot;
    idx_off.push_back({a, b});
  }
  hipError_t e = hipMemcpyAsync(dIdx, hIdx, sizeof(int) * nidx, hipMemcpyHostToDevice, s0);
  if (e != hipSuccess) return hip_error(e, "queue index upload");
  e = hipEventRecord(ev_up, s0);
  if (e != hipSuccess) return hip_error(e, "hipEventRecord");
  // plan and carve every group
  size_t off = 0, res_off = 0;
  int gi = 0;
  std::vector<size_t> g_base, g_res;
  for (auto& kv : groups) {
    GroupPlan& g = kv.second;
    const int n = g.n, nb = (int)g.ev.size(), ns = (int)g.sm.size();
    if (nb) {
      int rc = make_layout(OP_GRAD, o.prec, nb, n, p, 1, 0, &g.lg);
      if (rc) return rc;
      g.iQe = g.cv.add((size_t)nb * n * n * 8);
      g.iGe = g.cv.add((size_t)nb * p * 8);
      g.iBe = g.cv.add((size_t)nb * p * 8);
      g.iE = g.cv.add((size_t)nb * 8);
      g.iDg = g.cv.add((size_t)nb * p * 8);
      g.iDb = g.cv.add((size_t)nb * p * 8);
      g.iGrad = g.cv.add(g.lg.cv.total);
    }
    if (ns) {
      int rc = make_layout(OP_SAMPLE, o.prec, ns, n, p, 1, o.shots, &g.ls);
      if (rc) return rc;
      g.iQs = g.cv.add((size_t)ns * n * n * 8);
      g.iGs = g.cv.add((size_t)ns * p * 8);
      g.iBs = g.cv.add((size_t)ns * p * 8);
      g.iZ = g.cv.add((size_t)ns * o.shots * 8);
      g.iBz = g.cv.add((size_t)ns * 8);
      g.iBc = g.cv.add((size_t)ns * 8);
      g.iEs = g.cv.add((size_t)ns * 8);
      g.iSd = g.cv.add((size_t)ns * 8);
      g.iSamp = g.cv.add(g.ls.cv.total);
    }
    g_base.push_back(off);
    off += align256(g.cv.total);
    g_res.push_back(res_off);
    res_off += (size_t)ns * (o.shots + 2 * p + 3) * 8;
    ++gi;
  }
  if (off > budget)
    return set_error(QAOA_ERR_OUT_OF_MEMORY, "step needs %zu arena bytes of %zu", off, budget);
  if (res_off > hRes_bytes)
    return set_error(QAOA_ERR_OUT_OF_MEMORY, "step results exceed the staging buffer");
  // evaluation rounds: round k enqueues one evaluation of every group on the
  // group's stream; from the third round (k = 2) on, the host first waits
  // for round k - 2 and ends the step there if a waiting request could now
  // be admitted
  gi = 0;
  for (auto& kv : groups) {
    hipStream_t s = streams[gi % NSTREAMS];
    (void)kv;
    if (s != s0) {
      e = hipStreamWaitEvent(s, ev_up, 0);
      if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
    }
    ++gi;
  }
  const int nused = std::min<int>((int)groups.size(), NSTREAMS);
  int Kdone = K;
  for (int k = 0; k < K; ++k) {
    if (k >= 2) {
      for (int i = 0; i < nused; ++i) {
        e = hipEventSynchronize(ev_round[k % 2][i]);
        if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
      }
      std::lock_guard<std::mutex> lk(mu);
      if (should_yield(act)) {
        Kdone = k;
        break;
      }
    }
    gi = 0;
    for (auto& kv : groups) {
      GroupPlan& g = kv.second;
      if (!g.ev.empty()) {
        int rc = eval_group(g, dIdx + idx_off[gi].first, arena + g_base[gi],
                            streams[gi % NSTREAMS]);
        if (rc) return rc;
      }
      ++gi;
    }
    for (int i = 0; i < nused; ++i) {
      e = hipEventRecord(ev_round[k % 2][i], streams[i]);
      if (e != hipSuccess) return hip_error(e, "hipEventRecord");
    }
  }
  // requests reach their last evaluation only when the step ran all K rounds
  // (K is the fewest evaluations any request has left)
  const bool sampled = Kdone == K;
  gi = 0;
  for (auto& kv : groups) {
    GroupPlan& g = kv.second;
    hipStream_t s = streams[gi % NSTREAMS];
    char* base = arena + g_base[gi];
    const int n = g.n, ns = sampled ? (int)g.sm.size() : 0;
    const int* is = dIdx + idx_off[gi].second;
    auto A = [&](size_t i) { return base + g.cv.off[i]; };
    if (ns) {
      double *Q = (double*)A(g.iQs), *gg = (double*)A(g.iGs), *bb = (double*)A(g.iBs);
      uint64_t* z = (uint64_t*)A(g.iZ);
      uint64_t* bz = (uint64_t*)A(g.iBz);
      double *bc = (double*)A(g.iBc), *es = (double*)A(g.iEs);
      uint64_t* sd = (uint64_t*)A(g.iSd);
      e = launch_gather(ns, n, p, is, dQ, QN_MAX * QN_MAX, dG, dB, dSeed, Q, gg, bb, sd, s);
      if (e != hipSuccess) return hip_error(e, "gather");
      int rc = enqueue_sample(g.ls, A(g.iSamp), Q, gg, bb, o.shots, 0, sd, z, nullptr, bz,
                              bc, es, s, nullptr);
      if (rc) return rc;
      char* hr = hRes + g_res[gi];
      e = hipMemcpyAsync(hr, z, (size_t)ns * o.shots * 8, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hr + (size_t)ns * o.shots * 8, gg, (size_t)ns * p * 8,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hr + (size_t)ns * (o.shots + p) * 8, bb, (size_t)ns * p * 8,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hr + (size_t)ns * (o.shots + 2 * p) * 8, bz, (size_t)ns * 8,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hr + (size_t)ns * (o.shots + 2 * p + 1) * 8, bc, (size_t)ns * 8,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hr + (size_t)ns * (o.shots + 2 * p + 2) * 8, es, (size_t)ns * 8,
                           hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return hip_error(e, "result copy");
    }
    ++gi;
  }
  for (int i = 0; i < NSTREAMS; ++i) {
    e = hipStreamSynchronize(streams[i]);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  }
  // bookkeeping
  std::lock_guard<std::mutex> lk(mu);
  gi = 0;
  for (auto& kv : groups) {
    GroupPlan& g = kv.second;
    for (Request* r : g.ev) r->evals_done += Kdone;
    const int ns = sampled ? (int)g.sm.size() : 0;
    const char* hr = hRes + g_res[gi];
    for (int i = 0; i < ns; ++i) {
      Request* r = g.sm[i];
      const uint64_t* z = (const uint64_t*)hr;
      const double* gg = (const double*)(hr + (size_t)ns * o.shots * 8);
      const double* bb = (const double*)(hr + (size_t)ns * (o.shots + p) * 8);
      const uint64_t* bz = (const uint64_t*)(hr + (size_t)ns * (o.shots + 2 * p) * 8);
      const double* bc = (const double*)(hr + (size_t)ns * (o.shots + 2 * p + 1) * 8);
      const double* es = (const double*)(hr + (size_t)ns * (o.shots + 2 * p + 2) * 8);
      r->samples.assign(z + (size_t)i * o.shots, z + (size_t)(i + 1) * o.shots);
      for (int j = 0; j < p; ++j) {
        r->res.gamma[j] = gg[i * p + j];
        r->res.beta[j] = bb[i * p + j];
      }
      r->res.best_z = bz[i];
      r->res.best_c = bc[i];
      r->res.expect = es[i];
      complete(r, QAOA_OK);
    }
    ++gi;
  }
  st.steps++;
  return QAOA_OK;
}

void qaoa_queue::run() {
  (void)hipSetDevice(device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        // cancellations of admitted requests take effect between steps
        for (Request* r : slots)
          if (r && r->cancel) complete(r, QAOA_ERR_CANCELLED);
        // FIFO admission against free slots and the byte budget
        while (!pending.empty() && !free_slots.empty()) {
          Request* r = reqs[pending.front()].get();
          if (in_use + r->bytes > budget) break;
          pending.pop_front();
          r->slot = free_slots.back();
          free_slots.pop_back();
          slots[r->slot] = r;
          in_use += r->bytes;
          r->state = 1;
          r->res.t_admit_ns = now_ns();
          st.admitted++;
        }
        int resident = 0;
        for (Request* r : slots) resident += r != nullptr;
        st.peak_active = std::max(st.peak_active, resident);
        st.peak_bytes = std::max(st.peak_bytes, in_use);
        const bool any = resident > 0;
        if (stop) return;
        if (any) break;
        cv_sched.wait(lk);
      }
    }
    int rc = step();
    if (rc != QAOA_OK) {
      // fail every admitted request of this step; keep serving the rest
      std::lock_guard<std::mutex> lk(mu);
      for (Request* r : slots)
        if (r) complete(r, QAOA_ERR_HIP);
      for (int i = 0; i < NSTREAMS; ++i) (void)hipStreamSynchronize(streams[i]);
      (void)hipGetLastError();
    }
  }
}

extern "C" {

int qaoa_queue_create(qaoa_ctx* ctx, const qaoa_queue_opts* opts, qaoa_queue** out) {
  if (!out) return set_error(QAOA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx || !opts) return set_error(QAOA_ERR_INVALID_ARG, "ctx/opts is NULL");
  const qaoa_queue_opts& o = *opts;
  if (o.max_slots < 1 || o.max_slots > 4096)
    return set_error(QAOA_ERR_INVALID_ARG, "max_slots %d outside [1, 4096]", o.max_slots);
  if (o.max_pending < 1)
    return set_error(QAOA_ERR_INVALID_ARG, "max_pending %d < 1", o.max_pending);
  if (o.prec != QAOA_C64 && o.prec != QAOA_C128)
    return set_error(QAOA_ERR_INVALID_ARG, "prec %d", o.prec);
  if (o.p < 1 || o.p > QAOA_MAX_P) return set_error(QAOA_ERR_INVALID_ARG, "p = %d", o.p);
  if (o.evals < 0) return set_error(QAOA_ERR_INVALID_ARG, "evals = %d < 0", o.evals);
  if (o.shots < 1) return set_error(QAOA_ERR_INVALID_ARG, "shots = %d < 1", o.shots);
  if (!(o.lr > 0.0) || !(o.beta1 >= 0.0 && o.beta1 < 1.0) ||
      !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps > 0.0))
    return set_error(QAOA_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
  const int dev = ctx_device(ctx);
  if (dev < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
  std::unique_ptr<qaoa_queue> q(new qaoa_queue());
  q->ctx = ctx;
  q->o = o;
  if (!o.batched) q->o.max_slots = 1;
  q->device = dev;
  {  // DQAOA_QUEUE_GRAPHS=0 runs every evaluation step eagerly
    const char* v = getenv("DQAOA_QUEUE_GRAPHS");
    q->use_graphs = !(v && strcmp(v, "0") == 0);
  }
  const int S = q->o.max_slots, p = o.p;
  if (hipSetDevice(dev) != hipSuccess) return set_error(QAOA_ERR_HIP, "hipSetDevice");
  q->budget = o.hbm_budget;
  if (!q->budget) {  // half the context's budget, within what is free right now
    size_t fr = 0, tot = 0;
    q->budget = ctx_budget(ctx) / 2;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) q->budget = std::min(q->budget, fr / 10 * 8);
  }
  hipError_t e = hipSuccess;
  for (int i = 0; i < NSTREAMS && e == hipSuccess; ++i)
    e = hipStreamCreateWithFlags(&q->streams[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_up, hipEventDisableTiming);
  for (int r = 0; r < 2; ++r)
    for (int i = 0; i < NSTREAMS && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&q->ev_round[r][i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&q->arena, q->budget);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dQ, sizeof(double) * S * QN_MAX * QN_MAX);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dG, sizeof(double) * S * p);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dB, sizeof(double) * S * p);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dM, sizeof(double) * S * 2 * p);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dV, sizeof(double) * S * 2 * p);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dT, sizeof(int) * S);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dSeed, sizeof(uint64_t) * S);
  if (e == hipSuccess) e = hipMalloc((void**)&q->dIdx, sizeof(int) * 2 * S);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&q->hUp, sizeof(double) * S * (QN_MAX * QN_MAX + 2 * p + 1), 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&q->hIdx, sizeof(int) * 2 * S, 0);
  q->hRes_bytes = (size_t)S * (o.shots + 2 * p + 3) * 8;
  if (e == hipSuccess) e = hipHostMalloc((void**)&q->hRes, q->hRes_bytes, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    qaoa_queue* qq = q.release();
    qaoa_queue_destroy(qq);
    return set_error(e == hipErrorOutOfMemory ? QAOA_ERR_OUT_OF_MEMORY : QAOA_ERR_HIP,
                     "queue allocation: %s", hipGetErrorString(e));
  }
  q->slots.assign(S, nullptr);
  for (int i = S - 1; i >= 0; --i) q->free_slots.push_back(i);
  qaoa_queue* qq = q.release();
  qq->th = std::thread([qq] { qq->run(); });
  *out = qq;
  return QAOA_OK;
}

int qaoa_queue_destroy(qaoa_queue* q) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop = true;
  }
  q->cv_sched.notify_all();
  if (q->th.joinable()) q->th.join();
  (void)hipSetDevice(q->device);
  for (int i = 0; i < NSTREAMS; ++i)
    if (q->streams[i]) (void)hipStreamSynchronize(q->streams[i]);
  for (auto& kv : q->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  q->graphs.clear();
  for (int i = 0; i < NSTREAMS; ++i)
    if (q->streams[i]) (void)hipStreamDestroy(q->streams[i]);
  if (q->ev_up) (void)hipEventDestroy(q->ev_up);
  for (int r = 0; r < 2; ++r)
    for (int i = 0; i < NSTREAMS; ++i)
      if (q->ev_round[r][i]) (void)hipEventDestroy(q->ev_round[r][i]);
  void* dev[] = {q->arena, q->dQ, q->dG, q->dB, q->dM, q->dV, q->dT, q->dSeed, q->dIdx};
  for (void* ptr : dev)
    if (ptr) (void)hipFree(ptr);
  void* host[] = {q->hUp, q->hIdx, q->hRes};
  for (void* ptr : host)
    if (ptr) (void)hipHostFree(ptr);
  delete q;
  return QAOA_OK;
}

int qaoa_submit(qaoa_queue* q, const qaoa_solve_req* req, uint64_t* ticket) {
  if (!q || !req || !ticket) return set_error(QAOA_ERR_INVALID_ARG, "NULL argument");
  if (req->n < 1 || req->n > QN_MAX)
    return set_error(QAOA_ERR_INVALID_ARG, "n = %d outside [1, %d]", req->n, QN_MAX);
  if (!req->Q || !req->gamma0 || !req->beta0)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, gamma0 and beta0 must be non-NULL");
  const size_t bytes = q->request_bytes(req->n);
  std::unique_ptr<Request> r(new Request());
  r->n = req->n;
  r->Q.assign(req->Q, req->Q + (size_t)req->n * req->n);
  r->g0.assign(req->gamma0, req->gamma0 + q->o.p);
  r->b0.assign(req->beta0, req->beta0 + q->o.p);
  r->seed = req->seed;
  r->bytes = bytes;
  std::lock_guard<std::mutex> lk(q->mu);
  if (bytes > q->budget) {
    q->st.rejected++;
    return set_error(QAOA_ERR_OUT_OF_MEMORY,
                     "a %d-qubit request needs %zu bytes; the queue budget is %zu", req->n,
                     bytes, q->budget);
  }
  if ((int)q->pending.size() >= q->o.max_pending) {
    q->st.rejected++;
    return set_error(QAOA_ERR_QUEUE_FULL, "%zu requests pending", q->pending.size());
  }
  r->id = q->next_id++;
  r->res.t_submit_ns = now_ns();
  r->res.status = QAOA_PENDING;
  *ticket = r->id;
  q->pending.push_back(r->id);
  q->reqs[r->id] = std::move(r);
  q->st.submitted++;
  q->cv_sched.notify_all();
  return QAOA_OK;
}

static int take_result(qaoa_queue* q, uint64_t ticket, qaoa_solve_result* out,
                       uint64_t* samples) {
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return set_error(QAOA_ERR_NOT_FOUND, "unknown ticket %llu",
                                            (unsigned long long)ticket);
  Request* r = it->second.get();
  if (r->state != 2) return QAOA_PENDING;
  if (out) *out = r->res;
  if (samples && !r->samples.empty())
    std::memcpy(samples, r->samples.data(), r->samples.size() * sizeof(uint64_t));
  q->reqs.erase(it);
  return QAOA_OK;
}

int qaoa_poll(qaoa_queue* q, uint64_t ticket, qaoa_solve_result* out, uint64_t* samples) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  std::lock_guard<std::mutex> lk(q->mu);
  return take_result(q, ticket, out, samples);
}

int qaoa_wait(qaoa_queue* q, uint64_t ticket, int64_t timeout_ns, qaoa_solve_result* out,
              uint64_t* samples) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  std::unique_lock<std::mutex> lk(q->mu);
  auto ready = [&] {
    auto it = q->reqs.find(ticket);
    return it == q->reqs.end() || it->second->state == 2;
  };
  if (timeout_ns < 0) {
    q->cv_done.wait(lk, ready);
  } else if (!q->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
    return set_error(QAOA_ERR_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
  }
  return take_result(q, ticket, out, samples);
}

int qaoa_cancel(qaoa_queue* q, uint64_t ticket) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end() || it->second->state == 2)
    return set_error(QAOA_ERR_NOT_FOUND, "ticket %llu unknown or finished",
                     (unsigned long long)ticket);
  Request* r = it->second.get();
  if (r->state == 0) {
    q->pending.erase(std::find(q->pending.begin(), q->pending.end(), ticket));
    q->complete(r, QAOA_ERR_CANCELLED);
  } else {
    r->cancel = true;
    q->cv_sched.notify_all();
  }
  return QAOA_OK;
}

int qaoa_queue_get_stats(qaoa_queue* q, qaoa_queue_stats* out) {
  if (!q || !out) return set_error(QAOA_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(q->mu);
  *out = q->st;
  out->pending = (int)q->pending.size();
  int act = 0;
  for (Request* r : q->slots) act += r != nullptr;
  out->active = act;
  out->bytes_in_use = q->in_use;
  return QAOA_OK;
}

}  // extern "C"
