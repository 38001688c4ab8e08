// Solve queue: continuous batching of sub-QUBO solves on one GPU.
//
// The "parallel processing" step of the DQAOA workflow (arXiv 2506.10531,
// Sec. V) hands many small sub-QUBOs to QAOA solvers and collects their
// sub-solutions asynchronously; the paper's QFw integration submits ansatz
// evaluations to an executor and feeds the results back to the optimiser
// (Sec. VI).  Here one GPU serves that stream of solves.  The scheduling
// policy (FIFO admission against slots and the byte budget, steps of up to
// MAX_EVALS_PER_STEP evaluations with two rounds in flight, the early end of
// a step for an arrival or a cancellation, bookkeeping) is sched.h; this file
// is its device backend and the C entry points:
//
//  * qaoa_submit copies a request (n, Q, initial gamma/beta, seed) into the
//    FIFO; a scheduler thread admits and steps.
//  * An admitted request keeps its Q, parameters and Adam moments in a
//    device slot.  In every round of a step the requests are grouped by
//    qubit count, each group is gathered into a contiguous batch, and one
//    batched adjoint pipeline (forward passes, lambda = C psi, backward
//    passes, fixed-order reductions) plus one Adam update runs per group,
//    groups on separate streams (a HIP graph per recurring group shape).
//    Requests that finish their evaluations are sampled at the end of the
//    step and completed.
//  * A step that ends early samples nothing, so the host does not wait for
//    its last rounds: the next step's work is ordered after them on the
//    device (its uploads wait for their events; every stream waits for the
//    uploads), and the host plans and enqueues it meanwhile.
//  * The big buffers (checkpoints, adjoint state, probabilities) exist only
//    within a step; a request's byte charge is what its group needs for it
//    during a step, so the sum over admitted requests bounds the arena.
//
// Every kernel works per state with a tile structure that depends only on
// (n, p, precision), and every reduction sums in a fixed order, so a
// request's result does not depend on which requests share its batch.
#include "internal.h"
#include "sched.h"
#include "../../include/dqaoa.h"

#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace dq {
int ctx_device(qaoa_ctx* c);
size_t ctx_budget(qaoa_ctx* c);
}  // namespace dq

using namespace dq;

namespace {

constexpr int QN_MAX = 26;      // largest sub-QUBO a request may carry
constexpr int NSTREAMS = 4;

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

struct Request : sched::Req {
  std::vector<double> Q, g0, b0;
  uint64_t seed = 0;
};

// Per-group scratch of one step: contiguous batch arrays plus the pipelines'
// layouts.
struct GroupPlan {
  const sched::Group* g = nullptr;
  Layout lg, ls;
  Carve cv;
  size_t iQe = 0, iGe = 0, iBe = 0, iE = 0, iDg = 0, iDb = 0, iGrad = 0;
  size_t iQs = 0, iGs = 0, iBs = 0, iZ = 0, iBz = 0, iBc = 0, iEs = 0, iSd = 0,
         iSamp = 0;
  size_t base = 0, res = 0;  // arena and host-result offsets
  int ie = 0, is = 0;        // offsets of its slot lists in the index buffer
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct qaoa_queue {
  qaoa_ctx* ctx = nullptr;
  qaoa_queue_opts o{};
  int device = 0;
  sched::Core core;
  std::thread th;

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
  char* hRes[2] = {};        // results of a sampling step, two buffers in turn
  size_t hRes_bytes = 0;
  hipEvent_t ev_res[2][NSTREAMS] = {};  // a buffer's copies done, per stream
  int res_nused[2] = {};
  int res_next = 0;          // the buffer the next sampling step writes
  std::vector<sched::Done> deferred;  // sampled requests whose results are in flight
  // the step in progress
  std::vector<GroupPlan> gp;
  int nused = 0;
  int last_round = -1;
  int cur_res = -1;          // its result buffer (sampling steps)
  // The host waits for no step: the next step's uploads (stream 0, which every
  // other stream then waits for) wait on the previous step's last work on
  // each stream: its last round's events, or its result copies' events.
  const hipEvent_t* pend_ev = nullptr;
  int pend_nused = 0;

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
  int eval_group(const GroupPlan& g, hipStream_t s);
  int enqueue_eval(const GroupPlan& g, hipStream_t s);

  // backend of sched::run_step
  int begin(sched::Step& s);
  int round(int k);
  int wait_round(int k);
  int end(bool sampled);
  void defer(const sched::Done& d);
  int collect(bool wait, std::vector<sched::Done>* out);
  void fetch(const sched::Done& d);
  int64_t now() const { return now_ns(); }
};

// One evaluation of an n-group: gather its requests' Q and parameters,
// the adjoint pipeline, the Adam update.  Kernels only (capturable).
int qaoa_queue::enqueue_eval(const GroupPlan& g, hipStream_t s) {
  const int n = g.g->n, nb = (int)g.g->ev.size(), p = o.p;
  char* base = arena + g.base;
  const int* ie = dIdx + g.ie;
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
int qaoa_queue::eval_group(const GroupPlan& g, hipStream_t s) {
  if (!use_graphs) return enqueue_eval(g, s);
  const GraphKey key{g.g->n, (int)g.g->ev.size(), arena + g.base, dIdx + g.ie};
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    if (graphs.size() >= 256) {  // evict the least recently used
      auto lru = graphs.begin();
      for (auto j = graphs.begin(); j != graphs.end(); ++j)
        if (j->second.last < lru->second.last) lru = j;
      if (lru->second.last + 1 >= step_no) {
        // used by this step or by the previous one, which may still run
        for (int i = 0; i < NSTREAMS; ++i) {
          hipError_t e = hipStreamSynchronize(streams[i]);
          if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
        }
      }
      (void)hipGraphExecDestroy(lru->second.exec);
      graphs.erase(lru);
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    int rc = enqueue_eval(g, s);
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

// Start of a step: upload the newly admitted requests (Q, gamma0, beta0,
// seed; zero Adam state), the groups' slot lists, and carve every group's
// batch arrays and pipeline scratch out of the arena.
int qaoa_queue::begin(sched::Step& s) {
  ++step_no;
  const int p = o.p;
  hipStream_t s0 = streams[0];
  last_round = -1;
  if (pend_ev) {
    // the previous step's last work on every stream precedes this step's
    // uploads and, through ev_up, all its rounds: slot state, the index
    // buffer and the arena are reused only after it
    for (int i = 0; i < pend_nused; ++i) {
      hipError_t e = hipStreamWaitEvent(s0, pend_ev[i], 0);
      if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
    }
    pend_ev = nullptr;
  }
  for (size_t i = 0; i < s.fresh.size(); ++i) {
    const Request* r = static_cast<const Request*>(s.fresh[i]);
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
  }
  // slot lists: per group, the evaluated then the sampled requests
  gp.assign(s.groups.size(), GroupPlan());
  int nidx = 0, gi = 0;
  for (auto& kv : s.groups) {
    GroupPlan& g = gp[gi++];
    g.g = &kv.second;
    g.ie = nidx;
    for (const sched::Req* r : g.g->ev) hIdx[nidx++] = r->slot;
    g.is = nidx;
    for (const sched::Req* r : g.g->sm) hIdx[nidx++] = r->slot;
  }
  hipError_t e = hipMemcpyAsync(dIdx, hIdx, sizeof(int) * nidx, hipMemcpyHostToDevice, s0);
  if (e != hipSuccess) return hip_error(e, "queue index upload");
  e = hipEventRecord(ev_up, s0);
  if (e != hipSuccess) return hip_error(e, "hipEventRecord");
  // plan and carve every group
  size_t off = 0, res_off = 0;
  for (GroupPlan& g : gp) {
    const int n = g.g->n, nb = (int)g.g->ev.size(), ns = (int)g.g->sm.size();
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
    g.base = off;
    off += align256(g.cv.total);
    g.res = res_off;
    res_off += (size_t)ns * (o.shots + 2 * p + 3) * 8;
  }
  if (off > core.budget)
    return set_error(QAOA_ERR_OUT_OF_MEMORY, "step needs %zu arena bytes of %zu", off,
                     core.budget);
  if (res_off > hRes_bytes)
    return set_error(QAOA_ERR_OUT_OF_MEMORY, "step results exceed the staging buffer");
  // every group's stream starts after the uploads
  for (size_t i = 0; i < gp.size(); ++i) {
    hipStream_t st = streams[i % NSTREAMS];
    if (st != s0) {
      e = hipStreamWaitEvent(st, ev_up, 0);
      if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
    }
  }
  nused = std::min<int>((int)gp.size(), NSTREAMS);
  return QAOA_OK;
}

// Round k: one evaluation of every group on the group's stream; the round's
// end is recorded per stream (two rounds' events are kept).
int qaoa_queue::round(int k) {
  for (size_t gi = 0; gi < gp.size(); ++gi) {
    if (gp[gi].g->ev.empty()) continue;
    int rc = eval_group(gp[gi], streams[gi % NSTREAMS]);
    if (rc) return rc;
  }
  for (int i = 0; i < nused; ++i) {
    hipError_t e = hipEventRecord(ev_round[k % 2][i], streams[i]);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord");
  }
  last_round = k;
  return QAOA_OK;
}

int qaoa_queue::wait_round(int k) {
  for (int i = 0; i < nused; ++i) {
    hipError_t e = hipEventSynchronize(ev_round[k % 2][i]);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
  }
  return QAOA_OK;
}

// End of a step.  A step that samples enqueues, per group, the sampling of
// its finished requests at their final parameters and the copy of their
// results into a host buffer that holds no uncollected results, and records
// when the copies are done; no step is waited for here.
int qaoa_queue::end(bool sampled) {
  const int p = o.p;
  if (!sampled) {
    if (last_round >= 0) {
      pend_ev = ev_round[last_round % 2];
      pend_nused = nused;
    }
    return QAOA_OK;
  }
  const int rb = res_next;
  res_next ^= 1;
  cur_res = rb;
  for (size_t gi = 0; gi < gp.size(); ++gi) {
    const GroupPlan& g = gp[gi];
    const int n = g.g->n, ns = (int)g.g->sm.size();
    if (!ns) continue;
    hipStream_t s = streams[gi % NSTREAMS];
    char* base = arena + g.base;
    auto A = [&](size_t i) { return base + g.cv.off[i]; };
    double *Q = (double*)A(g.iQs), *gg = (double*)A(g.iGs), *bb = (double*)A(g.iBs);
    uint64_t* z = (uint64_t*)A(g.iZ);
    uint64_t* bz = (uint64_t*)A(g.iBz);
    double *bc = (double*)A(g.iBc), *es = (double*)A(g.iEs);
    uint64_t* sd = (uint64_t*)A(g.iSd);
    hipError_t e = launch_gather(ns, n, p, dIdx + g.is, dQ, QN_MAX * QN_MAX, dG, dB, dSeed, Q,
                                 gg, bb, sd, s);
    if (e != hipSuccess) return hip_error(e, "gather");
    int rc = enqueue_sample(g.ls, A(g.iSamp), Q, gg, bb, o.shots, 0, sd, z, nullptr, bz, bc, es,
                            s, nullptr);
    if (rc) return rc;
    char* hr = hRes[rb] + g.res;
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
  for (int i = 0; i < nused; ++i) {
    hipError_t e = hipEventRecord(ev_res[rb][i], streams[i]);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord");
  }
  res_nused[rb] = nused;
  pend_ev = ev_res[rb];
  pend_nused = nused;
  return QAOA_OK;
}

void qaoa_queue::defer(const sched::Done& d) {
  sched::Done x = d;
  x.buf = cur_res;
  x.off = gp[d.gi].res;
  x.ns = (int)gp[d.gi].g->sm.size();
  deferred.push_back(x);
}

// The deferred requests, once every copy into their buffer is done (they
// all share one buffer: a sampling step collects the previous one's first).
int qaoa_queue::collect(bool wait, std::vector<sched::Done>* out) {
  if (deferred.empty()) return QAOA_OK;
  const int rb = deferred.front().buf;
  for (int i = 0; i < res_nused[rb]; ++i) {
    hipError_t e = wait ? hipEventSynchronize(ev_res[rb][i]) : hipEventQuery(ev_res[rb][i]);
    if (e == hipErrorNotReady) {
      (void)hipGetLastError();  // not an error: leave no trace for later launch checks
      return QAOA_OK;
    }
    if (e != hipSuccess) return hip_error(e, "result event");
  }
  out->swap(deferred);
  deferred.clear();
  return QAOA_OK;
}

void qaoa_queue::fetch(const sched::Done& d) {
  const int p = o.p, ns = d.ns, i = d.i;
  sched::Req* r = d.r;
  const char* hr = hRes[d.buf] + d.off;
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
}

void qaoa_queue::run() {
  (void)hipSetDevice(device);
  for (;;) {
    int running = 0;
    {
      std::unique_lock<std::mutex> lk(core.mu);
      for (;;) {
        core.admit(now_ns());
        if (core.stop) return;
        running = core.count(1);
        if (running || core.count(3)) break;
        core.cv_sched.wait(lk);
      }
    }
    // with nothing to run, wait for the results still on their way
    const int rc = running ? sched::run_step(core, *this) : sched::finish_sampled(core, *this, true);
    if (rc != QAOA_OK) {
      // fail every resident request; keep serving the rest
      std::lock_guard<std::mutex> lk(core.mu);
      core.fail_active(QAOA_ERR_HIP, now_ns());
      for (int i = 0; i < NSTREAMS; ++i) (void)hipStreamSynchronize(streams[i]);
      (void)hipGetLastError();
      pend_ev = nullptr;
      deferred.clear();
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
  size_t budget = o.hbm_budget;
  if (!budget) {  // half the context's budget, within what is free right now
    size_t fr = 0, tot = 0;
    budget = ctx_budget(ctx) / 2;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) budget = std::min(budget, fr / 10 * 8);
  }
  q->core.init(S, o.max_pending, budget, o.evals);
  hipError_t e = hipSuccess;
  for (int i = 0; i < NSTREAMS && e == hipSuccess; ++i)
    e = hipStreamCreateWithFlags(&q->streams[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_up, hipEventDisableTiming);
  for (int r = 0; r < 2; ++r)
    for (int i = 0; i < NSTREAMS && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&q->ev_round[r][i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&q->arena, budget);
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
  for (int r = 0; r < 2; ++r) {
    if (e == hipSuccess) e = hipHostMalloc((void**)&q->hRes[r], q->hRes_bytes, 0);
    for (int i = 0; i < NSTREAMS && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&q->ev_res[r][i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    qaoa_queue* qq = q.release();
    qaoa_queue_destroy(qq);
    return set_error(e == hipErrorOutOfMemory ? QAOA_ERR_OUT_OF_MEMORY : QAOA_ERR_HIP,
                     "queue allocation: %s", hipGetErrorString(e));
  }
  qaoa_queue* qq = q.release();
  qq->th = std::thread([qq] { qq->run(); });
  *out = qq;
  return QAOA_OK;
}

int qaoa_queue_destroy(qaoa_queue* q) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  {
    std::lock_guard<std::mutex> lk(q->core.mu);
    q->core.stop = true;
  }
  q->core.cv_sched.notify_all();
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
  for (int r = 0; r < 2; ++r)
    for (int i = 0; i < NSTREAMS; ++i)
      if (q->ev_res[r][i]) (void)hipEventDestroy(q->ev_res[r][i]);
  void* dev[] = {q->arena, q->dQ, q->dG, q->dB, q->dM, q->dV, q->dT, q->dSeed, q->dIdx};
  for (void* ptr : dev)
    if (ptr) (void)hipFree(ptr);
  void* host[] = {q->hUp, q->hIdx, q->hRes[0], q->hRes[1]};
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
  std::lock_guard<std::mutex> lk(q->core.mu);
  const int rc = q->core.submit(std::move(r), now_ns(), ticket);
  if (rc == QAOA_ERR_OUT_OF_MEMORY)
    return set_error(rc, "a %d-qubit request needs %zu bytes; the queue budget is %zu", req->n,
                     bytes, q->core.budget);
  if (rc == QAOA_ERR_QUEUE_FULL)
    return set_error(rc, "%zu requests pending", q->core.pending.size());
  return rc;
}

static int take_result(qaoa_queue* q, uint64_t ticket, qaoa_solve_result* out,
                       uint64_t* samples) {
  const int rc = q->core.take(ticket, out, samples);
  if (rc == QAOA_ERR_NOT_FOUND)
    return set_error(rc, "unknown ticket %llu", (unsigned long long)ticket);
  return rc;
}

int qaoa_poll(qaoa_queue* q, uint64_t ticket, qaoa_solve_result* out, uint64_t* samples) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  std::lock_guard<std::mutex> lk(q->core.mu);
  return take_result(q, ticket, out, samples);
}

int qaoa_wait(qaoa_queue* q, uint64_t ticket, int64_t timeout_ns, qaoa_solve_result* out,
              uint64_t* samples) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  std::unique_lock<std::mutex> lk(q->core.mu);
  auto ready = [&] { return q->core.finished(ticket); };
  if (timeout_ns < 0) {
    q->core.cv_done.wait(lk, ready);
  } else if (!q->core.cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
    return set_error(QAOA_ERR_TIMEOUT, "ticket %llu not done", (unsigned long long)ticket);
  }
  return take_result(q, ticket, out, samples);
}

int qaoa_cancel(qaoa_queue* q, uint64_t ticket) {
  if (!q) return set_error(QAOA_ERR_INVALID_ARG, "queue is NULL");
  std::lock_guard<std::mutex> lk(q->core.mu);
  const int rc = q->core.cancel(ticket, now_ns());
  if (rc == QAOA_ERR_NOT_FOUND)
    return set_error(rc, "ticket %llu unknown or finished", (unsigned long long)ticket);
  return rc;
}

int qaoa_queue_get_stats(qaoa_queue* q, qaoa_queue_stats* out) {
  if (!q || !out) return set_error(QAOA_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(q->core.mu);
  *out = q->core.stats();
  return QAOA_OK;
}

}  // extern "C"
