// Host runtime and C ABI of the QAOA state-vector library (include/dqaoa.h).
//
// A call validates its arguments on the host, plans the state passes
// (make_plan), carves the context's scratch (make_layout), and queues on the
// caller's stream: the fold/coefficient kernel, the tile passes and the
// fixed-order reductions.  Nothing is computed on the host.
#include "internal.h"
#include "../../include/dqaoa.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

namespace dq {

static_assert(MAX_TAB_JOBS >= 3 * QAOA_MAX_P + 1,
              "a four-set forward plan at QAOA_MAX_P layers fits the table jobs");

// ---- errors -------------------------------------------------------------------

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(QAOA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- planning -------------------------------------------------------------------

// Qubit sets: set 0 = bits [0, k0) (contiguous tile, all mixed); set i >= 1 =
// the c low bits (carried for coalescing, not mixed) plus a run of high bits.
// A layer's mixer is the product of the sets' mixers (they commute); layer
// j visits the sets in order 0..m-1 for even j and m-1..0 for odd j, so the
// last set of layer j is the first of layer j+1 and one pass applies the end
// of layer j, the phase of layer j+1 and the start of layer j+1.
bool make_plan(int n, int p, int kmax, int cpref, Plan* P) {
  *P = Plan();
  P->K = kmax;
  if (n < 1 || p < 1 || p > 64 || kmax < 2) return false;
  if (n <= kmax) {
    P->sets = 1;
    P->c = n;
    P->k[0] = n;
    PassDesc d{};
    d.n = n;
    d.k = n;
    d.c = n;
    d.a = n;
    d.mixlo = 0;
    d.lead = -1;
    d.ja = 0;
    d.jb = p - 1;
    d.flags = F_INIT | F_REDUCE;
    d.set = 0;
    P->pass[0] = d;
    P->npass = 1;
    return true;
  }
  int m = 0, c = 0;
  for (int mm = 2; mm <= 4 && !m; ++mm)
    for (int cc = cpref; cc >= 2; --cc)
      if (kmax + (mm - 1) * (kmax - cc) >= n) {
        m = mm;
        c = cc;
        break;
      }
  if (!m) return false;
  const int q = m - 1;
  // balance: tile sizes as equal as possible, set 0 at most kmax
  int k0 = (n + q * c + m - 1) / m;
  if (k0 > kmax) k0 = kmax;
  if (k0 < c) k0 = c;
  int rest = n - k0;
  while ((rest + q - 1) / q > kmax - c) {
    ++k0;
    rest = n - k0;
    if (k0 > kmax) return false;
  }
  P->sets = m;
  P->c = c;
  P->k[0] = k0;
  P->a[0] = 0;
  int a = k0;
  for (int i = 1; i < m; ++i) {
    const int run = rest / q + (i - 1 < rest % q ? 1 : 0);
    P->k[i] = c + run;
    P->a[i] = a;
    a += run;
  }
  auto desc = [&](int set, int lead, int ja, int jb) {
    PassDesc d{};
    d.n = n;
    d.set = set;
    d.lead = lead;
    d.ja = ja;
    d.jb = jb;
    if (set == 0) {
      d.k = P->k[0];
      d.c = d.k;
      d.a = d.k;
      d.mixlo = 0;
    } else {
      d.k = P->k[set];
      d.c = c;
      d.a = P->a[set];
      d.mixlo = c;
    }
    return d;
  };
  auto order = [&](int j, int i) { return (j % 2 == 0) ? i : m - 1 - i; };
  int np = 0;
  P->pass[np++] = desc(order(0, 0), -1, 0, 0);
  for (int j = 0; j < p; ++j) {
    for (int i = 1; i <= m - 2; ++i) P->pass[np++] = desc(order(j, i), j, 1, 0);
    if (j < p - 1) P->pass[np++] = desc(order(j, m - 1), j, j + 1, j + 1);
    else P->pass[np++] = desc(order(j, m - 1), j, 1, 0);
  }
  for (int i = 0; i < np; ++i) {
    int f = 0;
    if (i == 0) f |= F_INIT;
    if (i < np - 1) f |= F_WRITE;
    else f |= F_REDUCE;
    P->pass[i].flags = f;
  }
  P->npass = np;
  return true;
}

// Register-tile plan: the same pass sequence as make_plan, with every tile
// holding K qubits.  Set 0 mixes [0, K); the remaining qubits [K, n) are split
// into runs of at most K - C, and set i's tile is the C low bits plus the
// (K - C)-bit run [a, a + K - C) that ends at its mixed run (or at n), so it
// carries (does not mix) any of those bits below its own run.
bool make_plan_regtile(int n, int p, int K, int C, Plan* P, int cmax, bool rev) {
  *P = Plan();
  P->K = K;
  const int span = K - C;
  if (n <= K || n > 34 || p < 1 || p > 64 || span < 1 || cmax < C || cmax >= K) return false;
  const int m = 1 + (n - K + span - 1) / span;
  if (m > 4) return false;
  const int rest = n - K, q = m - 1;
  int lo[4] = {0}, hi[4] = {0}, a[4] = {0}, cs[4] = {K, C, C, C};
  lo[0] = 0;
  hi[0] = K;
  int cur = K;
  for (int i = 1; i < m; ++i) {
    const int run = rest / q + (i - 1 < rest % q ? 1 : 0);
    lo[i] = cur;
    hi[i] = cur + run;
    cur += run;
    // as many contiguous low bits as the set's run leaves room for (up to
    // cmax): longer HBM runs, and fewer high bits (pages) per tile
    cs[i] = K - run < cmax ? K - run : cmax;
    const int sp = K - cs[i];
    a[i] = hi[i] - sp < cs[i] ? cs[i] : hi[i] - sp;
    if (a[i] + sp > n) a[i] = n - sp;
  }
  P->sets = m;
  P->c = C;
  for (int i = 0; i < m; ++i) {
    P->k[i] = K;
    P->a[i] = a[i];
  }
  auto desc = [&](int set, int lead, int ja, int jb) {
    PassDesc d{};
    d.n = n;
    d.set = set;
    d.lead = lead;
    d.ja = ja;
    d.jb = jb;
    d.k = K;
    if (set == 0) {
      d.c = K;
      d.a = K;
      d.mixlo = 0;
      d.kind = 1;
    } else {
      d.c = cs[set];
      d.a = a[set];
      d.mixlo = cs[set] + (lo[set] - a[set]);
      d.kind = 2;
    }
    return d;
  };
  // the set that finishes layer j's mixer starts layer j + 1; rev starts the
  // first layer on the last set instead of set 0
  auto order = [&](int j, int i) { return ((j % 2 == 0) != rev) ? i : m - 1 - i; };
  int np = 0;
  P->pass[np++] = desc(order(0, 0), -1, 0, 0);
  for (int j = 0; j < p; ++j) {
    for (int i = 1; i <= m - 2; ++i) P->pass[np++] = desc(order(j, i), j, 1, 0);
    if (j < p - 1) P->pass[np++] = desc(order(j, m - 1), j, j + 1, j + 1);
    else P->pass[np++] = desc(order(j, m - 1), j, 1, 0);
  }
  // pending mixer scales at the start of every pass
  int pn = 0, pl[3] = {0}, pm[3] = {0};
  for (int i = 0; i < np; ++i) {
    PassDesc& d = P->pass[i];
    d.flags = (i == 0 ? F_INIT : 0) | (i < np - 1 ? F_WRITE : F_REDUCE);
    if (pn > 2) return false;
    d.pend_n = pn;
    for (int t = 0; t < pn; ++t) {
      d.pend_layer[t] = pl[t];
      d.pend_m[t] = pm[t];
    }
    const int mset = hi[d.set] - lo[d.set];
    if (d.ja <= d.jb) {  // the phase applies every pending factor
      pn = 1;
      pl[0] = d.jb;
      pm[0] = mset;
    } else {
      pl[pn] = d.lead;
      pm[pn] = mset;
      ++pn;
    }
  }
  P->npass = np;
  return true;
}

// Starts on the last set: the set-0 passes (14 qubits mixed per half-mixer,
// contiguous tiles) then take the middle of the plan, where they run faster
// than the kind-2 ones at n = 24 and 32, and a kind-2 set takes the first
// (write-only) and last (read-only) passes.
bool make_plan_reg14(int n, int p, Plan* P) {
  return n >= 15 && make_plan_regtile(n, p, 14, 4, P, 8, true);
}

bool make_plan_reg2set(int n, int p, int K, int C, Plan* P, int cmax) {
  *P = Plan();
  const int span = K - C;
  if (n <= K || n > K + span || p < 1 || p > 64 || cmax < C || cmax >= K) return false;
  // the second set keeps min(cmax, K - (n - K)) contiguous low tile bits: its
  // run of high tile bits is exactly qubits [K, n) unless capped
  const int C1 = 2 * K - n < cmax ? 2 * K - n : cmax;
  const int a = n - (K - C1);
  P->K = K;
  P->sets = 2;
  P->c = C;
  P->k[0] = P->k[1] = K;
  P->a[0] = K;
  P->a[1] = a;
  auto desc = [&](int set, int lead, int ja, int jb) {
    PassDesc d{};
    d.n = n;
    d.set = set;
    d.lead = lead;
    d.ja = ja;
    d.jb = jb;
    d.k = K;
    if (set == 0) {
      d.c = K;
      d.a = K;
      d.mixlo = 0;
      d.kind = 1;
    } else {
      d.c = C1;
      d.a = a;
      d.mixlo = C1 + (K - a);
      d.kind = 2;
    }
    return d;
  };
  int np = 0;
  P->pass[np++] = desc(0, -1, 0, 0);
  for (int j = 0; j < p; ++j) {
    const int set = (j % 2 == 0) ? 1 : 0;
    if (j < p - 1) P->pass[np++] = desc(set, j, j + 1, j + 1);
    else P->pass[np++] = desc(set, j, 1, 0);
  }
  for (int i = 0; i < np; ++i)
    P->pass[i].flags = (i == 0 ? F_INIT : 0) | (i < np - 1 ? F_WRITE : F_REDUCE);
  P->npass = np;
  return true;
}

bool make_plan_reg13(int n, int p, Plan* P) {
  return n >= 14 && n <= 22 && make_plan_reg2set(n, p, 13, 4, P, 8);
}

static bool grad_reg_off() {
  static const bool off = [] {
    const char* v = getenv("DQAOA_GRAD_KERNEL");
    return v && strcmp(v, "lds") == 0;
  }();
  return off;
}

// Register-tile gradients: complex64 on 13-qubit tiles (14 <= n <= 22),
// complex128 on 12-qubit tiles (13 <= n <= 22); DQAOA_GRAD_KERNEL=lds
// selects the LDS-tile adjoint instead.
// Whole-state adjoint (small.hip) for n up to this size; DQAOA_GRAD_KERNEL=lds
// selects the LDS-tile adjoint instead.
static int small_grad_limit(int prec) { return grad_reg_off() ? 0 : small_grad_nmax(prec); }

static bool use_reg13(int op, int prec, int n) {
  return !grad_reg_off() && op == OP_GRAD && prec == QAOA_C64 && n >= 14 && n <= 22;
}
static bool use_reg12(int op, int prec, int n) {
  return !grad_reg_off() && op == OP_GRAD && prec == QAOA_C128 && n >= 13 && n <= 22;
}

// The register-tile kernels serve forward evaluations with n >= 15
// (complex64, 14-qubit tiles) or n >= 14 (complex128, 13-qubit tiles);
// DQAOA_FWD_KERNEL=lds selects the LDS-tile kernel for every pass instead.
static bool fwd_reg_off() {
  static const bool off = [] {
    const char* v = getenv("DQAOA_FWD_KERNEL");
    return v && strcmp(v, "lds") == 0;
  }();
  return off;
}

static bool use_reg14(int op, int prec, int n) {
  return !fwd_reg_off() && op != OP_GRAD && prec == QAOA_C64 && n >= 15 && n <= 34;
}

static bool use_reg13d(int op, int prec, int n) {
  return !fwd_reg_off() && op != OP_GRAD && prec == QAOA_C128 && n >= 14 && n <= 34;
}

bool choose_plan(int op, int prec, int n, int p, Plan* P) {
  if (use_reg14(op, prec, n)) return make_plan_reg14(n, p, P);
  // complex128 forward: 13-qubit tiles, 2 contiguous low qubits in the other
  // sets, first layer on the last set (as the complex64 plan)
  if (use_reg13d(op, prec, n)) return make_plan_regtile(n, p, 13, 2, P, 2, true);
  if (use_reg13(op, prec, n)) return make_plan_reg13(n, p, P);
  if (use_reg12(op, prec, n)) return make_plan_reg2set(n, p, 12, 2, P);
  return make_plan(n, p, kmax_for(prec, op == OP_GRAD), cpref_for(prec), P);
}

int kmax_for(int prec, bool two_tiles) {
  const int k = prec == QAOA_C128 ? 13 : 14;
  return two_tiles ? k - 1 : k;
}
int cpref_for(int prec) { return prec == QAOA_C128 ? 3 : 4; }
static size_t amp_bytes(int prec) { return prec == QAOA_C128 ? 16 : 8; }
static uint64_t ntiles(const PassDesc& d) { return 1ull << (d.n - d.k); }

static bool mul_ok(size_t a, size_t b, size_t* out) {
  if (a && b > SIZE_MAX / a) return false;
  *out = a * b;
  return true;
}

int make_layout(int op, int prec, int B, int n, int p, int S, int shots,
                Layout* L) {
  const bool grad = op == OP_GRAD;
  *L = Layout();
  L->prec = prec;
  L->B = B;
  L->n = n;
  L->p = p;
  L->S = S;
  if (!choose_plan(op, prec, n, p, &L->plan))
    return set_error(QAOA_ERR_UNSUPPORTED, "no pass plan for n = %d", n);
  L->nstates = (size_t)B * S;
  size_t amps;
  if (!mul_ok(((size_t)1) << n, amp_bytes(prec), &L->state_bytes) ||
      !mul_ok(L->state_bytes, L->nstates, &amps))
    return set_error(QAOA_ERR_INVALID_ARG, "state bytes overflow");
  const Plan& P = L->plan;
  L->iW = L->cv.add((size_t)B * n * n * sizeof(double));
  L->iC = L->cv.add(L->nstates * p * sizeof(LayerCoef));
  // per-state tables of every register-tile pass (one record per pass and
  // state; the gradient's checkpoint and adjoint passes have their own)
  const size_t ntab = P.pass[0].kind == 0 ? 1 : (grad ? 2 * (size_t)P.npass - 1 : P.npass);
  L->iTab = L->cv.add(L->nstates * TAB_BYTES * ntab);
  if (!grad) {
    const PassDesc& last = P.pass[P.npass - 1];
    L->iPart = L->cv.add(L->nstates * ntiles(last) * 2 * sizeof(double));
    if (P.npass > 1) L->iState = L->cv.add(amps);
    if (op == OP_SAMPLE) {
      L->iProbs = L->cv.add(amps / 2);  // |psi|^2 in the state precision
      const size_t sd = sample_scratch_doubles(n, (int)L->nstates) / 2;
      L->iBsum = L->cv.add(sd * sizeof(double));
      L->iBcdf = L->cv.add(sd * sizeof(double));
      L->iCz = L->cv.add(L->nstates * (size_t)(shots > 0 ? shots : 1) * sizeof(double));
    }
  } else {
    int nrec = 0;
    for (int i = 0; i < P.npass; ++i) {
      L->rec_base.push_back(nrec);
      nrec += (int)ntiles(P.pass[i]);
    }
    L->nrec = nrec;
    L->iPart = L->cv.add(L->nstates * (size_t)nrec * (2 * p + 2) * sizeof(double));
    for (int i = 0; i + 1 < P.npass; ++i) L->iCk.push_back(L->cv.add(amps));
    if (P.npass > 1) L->iLam = L->cv.add(amps);
  }
  return QAOA_OK;
}

namespace {

struct TimerScope {
  PassTimer* t;
  hipStream_t s;
  TimerScope(PassTimer* tm, hipStream_t st, double bytes) : t(tm), s(st) {
    if (t) t->begin(s, bytes);
  }
  ~TimerScope() {
    if (t) t->end(s);
  }
};

// The forward passes; the last one reduces into `part` and optionally writes
// probabilities (`probs`) or the final state (`psi`).
int run_forward(const Layout& L, char* base, const double* Q,
                const double* gammas, const double* betas, void* probs,
                void* psi, hipStream_t s, PassTimer* tm) {
  double* W = (double*)L.at(base, L.iW);
  LayerCoef* coef = (LayerCoef*)L.at(base, L.iC);
  double* part = (double*)L.at(base, L.iPart);
  void* state = L.plan.npass > 1 ? (void*)L.at(base, L.iState) : nullptr;
  hipError_t e = launch_prep(L.B, L.n, Q, W, (int)L.nstates, L.p, gammas, betas, coef, s);
  if (e != hipSuccess) return hip_error(e, "prep");
  const uint64_t stride = 1ull << L.n;
  const double sb = (double)L.state_bytes * L.nstates;
  char* const tabs = L.at(base, L.iTab);
  const size_t tstride = L.nstates * TAB_BYTES;
  const bool reg = L.plan.pass[0].kind != 0;
  for (int i = 0; i < L.plan.npass; ++i) {
    PassDesc d = L.plan.pass[i];
    const bool last = i == L.plan.npass - 1;
    if (last && probs) d.flags |= F_PROBS;
    if (last && psi) d.flags |= F_WRITE;
    double bytes = 0.0;
    if (!(d.flags & F_INIT)) bytes += sb;
    if (d.flags & F_WRITE) bytes += sb;
    if (d.flags & F_PROBS) bytes += sb / 2;
    TimerScope ts(tm, s, bytes);
    if (reg && i == 0) {
      // every pass's tables in one launch, inside the first pass's bracket
      TabJobs J{};
      if (L.plan.npass > MAX_TAB_JOBS)
        return set_error(QAOA_ERR_INVALID_ARG, "%d passes exceed the %d table jobs of a call",
                         L.plan.npass, MAX_TAB_JOBS);
      J.njobs = L.plan.npass;
      for (int k = 0; k < L.plan.npass; ++k) {
        const PassDesc& dk = L.plan.pass[k];
        J.job[k] = tab_job(dk, fwd_tab_spec(dk), dk.ja <= dk.jb || (dk.flags & F_REDUCE));
      }
      e = L.prec == QAOA_C64
              ? launch_fwd14_tables(J, L.n, (int)L.nstates, L.S, L.p, W, coef, tabs, s)
              : launch_fwd13d_tables(J, L.n, (int)L.nstates, L.S, L.p, W, coef, tabs, s);
      if (e != hipSuccess) return hip_error(e, "pass tables");
    }
    if (d.kind && L.prec == QAOA_C64)
      e = launch_fwd14_pass(d, (int)L.nstates, L.S, L.p, state,
                            (last && psi) ? psi : state, stride, W, coef, part, probs,
                            tabs + i * tstride, s);
    else if (d.kind)
      e = launch_fwd13d_pass(d, (int)L.nstates, L.S, L.p, state,
                             (last && psi) ? psi : state, stride, W, coef, part, probs,
                             tabs + i * tstride, s);
    else
      e = launch_fwd_pass(L.prec, d, (int)L.nstates, L.S, L.p, state,
                          (last && psi) ? psi : state, stride, W, coef, part, probs, s);
    if (e != hipSuccess) return hip_error(e, "forward pass");
  }
  return QAOA_OK;
}

}  // namespace

int enqueue_expect(const Layout& L, char* base, const double* Q,
                   const double* gammas, const double* betas, double* expect,
                   double* norm, void* probs, void* psi, hipStream_t s,
                   PassTimer* tm) {
  if (L.plan.npass == 1 && L.n <= small_fwd_nmax(L.prec) && !fwd_reg_off()) {
    // the whole state in one work-group's registers: one launch, no scratch
    const double out = (double)L.state_bytes * L.nstates * ((probs ? 0.5 : 0.0) + (psi ? 1.0 : 0.0));
    TimerScope ts(tm, s, out);
    hipError_t e = launch_small_expect(L.prec, L.n, L.p, L.S, (int)L.nstates, Q, gammas, betas,
                                       expect, norm, probs, psi, s);
    if (e != hipSuccess) return hip_error(e, "whole-state evaluation");
    return QAOA_OK;
  }
  int rc = run_forward(L, base, Q, gammas, betas, probs, psi, s, tm);
  if (rc) return rc;
  const PassDesc& last = L.plan.pass[L.plan.npass - 1];
  double* outs[2] = {expect, norm};
  int q0[2] = {0, 1}, cnt[2] = {1, 1};
  hipError_t e = launch_reduce_parts((int)L.nstates, (int)ntiles(last), 2,
                                     (double*)L.at(base, L.iPart), outs, q0, cnt, 2, s);
  if (e != hipSuccess) return hip_error(e, "reduce");
  return QAOA_OK;
}

int enqueue_sample(const Layout& L, char* base, const double* Q,
                   const double* gammas, const double* betas, int shots,
                   uint64_t seed, const uint64_t* seeds, uint64_t* z, double* cz, uint64_t* best_z,
                   double* best_c, double* expect, hipStream_t s,
                   PassTimer* tm) {
  void* P = L.at(base, L.iProbs);
  hipError_t e;
  if (L.plan.npass == 1 && L.n <= small_fwd_nmax(L.prec) && !fwd_reg_off()) {
    // probabilities and <C> from the whole-state launch; the folded
    // couplings the shots price their samples with come from prep
    e = launch_prep(L.B, L.n, Q, (double*)L.at(base, L.iW), (int)L.nstates, L.p, gammas, betas,
                    (LayerCoef*)L.at(base, L.iC), s);
    if (e != hipSuccess) return hip_error(e, "prep");
    TimerScope ts(tm, s, 0.5 * (double)L.state_bytes * L.nstates);
    e = launch_small_expect(L.prec, L.n, L.p, L.S, (int)L.nstates, Q, gammas, betas,
                            expect ? expect : (double*)L.at(base, L.iPart), nullptr, P, nullptr,
                            s);
    if (e != hipSuccess) return hip_error(e, "whole-state evaluation");
  } else {
    int rc = run_forward(L, base, Q, gammas, betas, P, nullptr, s, tm);
    if (rc) return rc;
    const PassDesc& last = L.plan.pass[L.plan.npass - 1];
    double* outs[1] = {expect};
    int q0[1] = {0}, cnt[1] = {1};
    e = launch_reduce_parts((int)L.nstates, (int)ntiles(last), 2,
                            (double*)L.at(base, L.iPart), outs, q0, cnt, 1, s);
    if (e != hipSuccess) return hip_error(e, "reduce");
  }
  double* czbuf = cz ? cz : (double*)L.at(base, L.iCz);
  e = launch_sample(L.prec, L.n, (int)L.nstates, P, (double*)L.at(base, L.iBsum),
                    (double*)L.at(base, L.iBcdf), shots, seed, seeds,
                    (double*)L.at(base, L.iW), L.S, z, czbuf, best_z, best_c, s);
  if (e != hipSuccess) return hip_error(e, "sample");
  return QAOA_OK;
}

int enqueue_grad(const Layout& L, char* base, const double* Q,
                 const double* gammas, const double* betas, double* expect,
                 double* dgamma, double* dbeta, hipStream_t s, PassTimer* tm) {
  if (L.n <= small_grad_limit(L.prec)) {
    // psi and lambda of the whole state in one work-group's registers
    TimerScope ts(tm, s, 0.0);
    hipError_t e = launch_small_grad(L.prec, L.n, L.p, L.S, (int)L.nstates, Q, gammas, betas,
                                     expect, dgamma, dbeta, s);
    return e == hipSuccess ? QAOA_OK : hip_error(e, "whole-state gradient");
  }
  double* W = (double*)L.at(base, L.iW);
  LayerCoef* coef = (LayerCoef*)L.at(base, L.iC);
  double* part = (double*)L.at(base, L.iPart);
  const int p = L.p, S = L.S, ns = (int)L.nstates;
  hipError_t e = launch_prep(L.B, L.n, Q, W, ns, p, gammas, betas, coef, s);
  if (e != hipSuccess) return hip_error(e, "prep");
  const Plan& P = L.plan;
  const int np = P.npass;
  const uint64_t stride = 1ull << L.n;
  const double sb = (double)L.state_bytes * L.nstates;
  auto ck = [&](int i) { return (void*)L.at(base, L.iCk[i]); };
  char* const tabs = L.at(base, L.iTab);
  const size_t tstride = (size_t)ns * TAB_BYTES;
  void* lam = np > 1 ? (void*)L.at(base, L.iLam) : nullptr;
  if ((P.K == 13 || P.K == 12) && P.pass[0].kind != 0) {
    const bool c128 = P.K == 12;
    // register-tile gradient: checkpoint passes, the seed pass, middle
    // adjoint passes, and the first pass's adjoint
    // every pass's tables in one launch: checkpoint pass i at job i, the
    // adjoint of pass i at job np - 1 + i (its undone half-mixer flips bit 0
    // and the middle shape undoes a phase)
    auto shape_of = [&](int i) { return i == np - 1 ? 0 : (i == 0 ? 2 : 1); };
    {
      TabJobs J{};
      if (2 * np - 1 > MAX_TAB_JOBS)
        return set_error(QAOA_ERR_INVALID_ARG, "%d passes exceed the %d table jobs of a call",
                         np, MAX_TAB_JOBS);
      J.njobs = 2 * np - 1;
      for (int i = 0; i + 1 < np; ++i) J.job[i] = tab_job(P.pass[i], fwd_tab_spec(P.pass[i]), true);
      for (int i = 0; i < np; ++i) {
        const PassDesc& d = P.pass[i];
        const int sh = shape_of(i);
        const TabSpec t{d.kind == 1 ? (sh == 0 ? d.lead : d.jb) : -1, sh == 1 ? d.jb : -1, -1.0};
        J.job[np - 1 + i] = tab_job(d, t, true);
      }
      TimerScope ts(tm, s, 0.0);
      e = c128 ? launch_grad12_tables(J, L.n, ns, S, p, W, coef, tabs, s)
               : launch_grad13_tables(J, L.n, ns, S, p, W, coef, tabs, s);
      if (e != hipSuccess) return hip_error(e, "pass tables");
    }
    for (int i = 0; i + 1 < np; ++i) {
      PassDesc d = P.pass[i];
      TimerScope ts(tm, s, (i == 0 ? 0.0 : sb) + sb);
      e = c128 ? launch_fwd12_ckpt_pass(d, ns, S, p, i ? ck(i - 1) : nullptr, ck(i), stride, W,
                                        coef, tabs + i * tstride, s)
               : launch_fwd13_ckpt_pass(d, ns, S, p, i ? ck(i - 1) : nullptr, ck(i), stride, W,
                                        coef, tabs + i * tstride, s);
      if (e != hipSuccess) return hip_error(e, "checkpoint pass");
    }
    for (int i = np - 1; i >= 0; --i) {
      const int shape = shape_of(i);
      TimerScope ts(tm, s, (shape == 1 ? 3 : 2) * sb);
      e = (c128 ? launch_bwd12_pass : launch_bwd13_pass)(
          P.pass[i], shape, ns, S, p, ck(i == np - 1 ? i - 1 : i), lam, stride, W, coef, part,
          L.rec_base[i], L.nrec, tabs + (np - 1 + i) * tstride, s);
      if (e != hipSuccess) return hip_error(e, "adjoint pass");
    }
    double* outs[3] = {dgamma, dbeta, expect};
    int q0[3] = {0, p, 2 * p}, cnt[3] = {p, p, 1};
    e = launch_reduce_parts(ns, L.nrec, 2 * p + 2, part, outs, q0, cnt, 3, s);
    if (e != hipSuccess) return hip_error(e, "reduce");
    return QAOA_OK;
  }
  // forward sweep, writing a checkpoint per pass
  for (int i = 0; i + 1 < np; ++i) {
    PassDesc d = P.pass[i];
    d.flags = (i == 0 ? F_INIT : 0) | F_WRITE;
    TimerScope ts(tm, s, (i == 0 ? 0.0 : sb) + sb);
    e = launch_fwd_pass(L.prec, d, ns, S, p, i ? ck(i - 1) : nullptr, ck(i), stride, W,
                        coef, nullptr, nullptr, s);
    if (e != hipSuccess) return hip_error(e, "forward pass");
  }
  // last pass: forward, <C>, lambda = C psi, and its adjoint sweep
  {
    PassDesc d = P.pass[np - 1];
    d.flags = F_LAMBDA | (np == 1 ? F_INIT : F_WRITE);
    TimerScope ts(tm, s, np == 1 ? 0.0 : 2 * sb);
    e = launch_bwd_pass(L.prec, d, ns, S, p, np > 1 ? ck(np - 2) : nullptr, lam, stride,
                        W, coef, part, L.rec_base[np - 1], L.nrec, s);
    if (e != hipSuccess) return hip_error(e, "adjoint pass");
  }
  for (int i = np - 2; i >= 0; --i) {
    PassDesc d = P.pass[i];
    d.flags = i >= 1 ? F_WRITE : 0;
    TimerScope ts(tm, s, (i >= 1 ? 3 : 2) * sb);
    e = launch_bwd_pass(L.prec, d, ns, S, p, ck(i), lam, stride, W, coef, part,
                        L.rec_base[i], L.nrec, s);
    if (e != hipSuccess) return hip_error(e, "adjoint pass");
  }
  double* outs[3] = {dgamma, dbeta, expect};
  int q0[3] = {0, p, 2 * p}, cnt[3] = {p, p, 1};
  e = launch_reduce_parts(ns, L.nrec, 2 * p + 2, part, outs, q0, cnt, 3, s);
  if (e != hipSuccess) return hip_error(e, "reduce");
  return QAOA_OK;
}

}  // namespace dq

using namespace dq;

// ---- context --------------------------------------------------------------------

struct qaoa_ctx : public PassTimer {
  int device = -1;
  size_t budget = 0;
  void* scratch = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  hipStream_t last = nullptr;
  bool any = false;
  bool prof = false;
  struct Rec {
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> recs;
  Rec cur{};
  long long prof_launches = 0;
  double prof_ms = 0.0, prof_bytes = 0.0;

  void begin(hipStream_t s, double bytes) override {
    cur = Rec{};
    cur.bytes = bytes;
    (void)hipEventCreate(&cur.a);
    (void)hipEventCreate(&cur.b);
    (void)hipEventRecord(cur.a, s);
  }
  void end(hipStream_t s) override {
    (void)hipEventRecord(cur.b, s);
    recs.push_back(cur);
  }
  PassTimer* timer() { return prof ? this : nullptr; }
};

namespace {

// Device scratch of qaoa_expect_noalloc: a file-scope array each GPU holds
// from the library's first use on it until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); qaoa_create takes its device address once per
// device and the entry point uses that address.
constexpr size_t NOALLOC_BYTES = QAOA_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_DEVICES = 64;
__device__ __align__(256) char scratch[NOALLOC_BYTES];
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[NOALLOC_DEVICES] = {};

// With `device` current: the device address of `scratch` on it.
int noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_DEVICES)
    return set_error(QAOA_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", device,
                     NOALLOC_DEVICES);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return QAOA_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
  g_noalloc_ptr[device] = static_cast<char*>(ptr);
  return QAOA_OK;
}

struct DeviceGuard {
  int prev = -1;  // the device to restore, -1 if none
  bool ok = true;
  explicit DeviceGuard(int dev) {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur == dev) return;  // already current
    prev = cur;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int acquire(qaoa_ctx* ctx, size_t bytes, hipStream_t stream, char** base) {
  if (bytes > ctx->budget)
    return set_error(QAOA_ERR_OUT_OF_MEMORY,
                     "scratch of %zu bytes exceeds the context budget of %zu",
                     bytes, ctx->budget);
  if (bytes > ctx->cap) {
    if (ctx->scratch) {
      if (ctx->any) {
        hipError_t e = hipEventSynchronize(ctx->done);
        if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
      }
      (void)hipFree(ctx->scratch);
      ctx->scratch = nullptr;
      ctx->cap = 0;
    }
    hipError_t e = hipMalloc(&ctx->scratch, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ctx->scratch = nullptr;
      return set_error(QAOA_ERR_OUT_OF_MEMORY, "hipMalloc(%zu): %s", bytes,
                       hipGetErrorString(e));
    }
    ctx->cap = bytes;
  }
  if (ctx->any && ctx->last != stream) {
    hipError_t e = hipStreamWaitEvent(stream, ctx->done, 0);
    if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
  }
  *base = static_cast<char*>(ctx->scratch);
  return QAOA_OK;
}

int finish(qaoa_ctx* ctx, hipStream_t stream) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "kernel launch");
  e = hipEventRecord(ctx->done, stream);
  if (e != hipSuccess) return hip_error(e, "hipEventRecord");
  ctx->last = stream;
  ctx->any = true;
  return QAOA_OK;
}

int check_common(qaoa_ctx* ctx, int prec, int B, int n, int p, int S) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  if (prec != QAOA_C128 && prec != QAOA_C64)
    return set_error(QAOA_ERR_INVALID_ARG, "prec %d is not QAOA_C128 or QAOA_C64", prec);
  if (B < 1) return set_error(QAOA_ERR_INVALID_ARG, "B = %d < 1", B);
  if (S < 1) return set_error(QAOA_ERR_INVALID_ARG, "S = %d < 1", S);
  if (n < 1 || n > QAOA_MAX_N)
    return set_error(QAOA_ERR_INVALID_ARG, "n = %d outside [1, %d]", n, QAOA_MAX_N);
  if (p < 1 || p > QAOA_MAX_P)
    return set_error(QAOA_ERR_INVALID_ARG, "p = %d outside [1, %d]", p, QAOA_MAX_P);
  if ((long long)B * S > 65535)
    return set_error(QAOA_ERR_INVALID_ARG, "B * S = %lld exceeds 65535 states per call",
                     (long long)B * S);
  return QAOA_OK;
}

// Layout + budget + device checks shared by the compute calls.
int prepare_call(qaoa_ctx* ctx, int op, int prec, int B, int n, int p, int S,
                 int shots, Layout* L) {
  int rc = make_layout(op, prec, B, n, p, S, shots, L);
  if (rc) return rc;
  if (L->cv.total > ctx->budget)
    return set_error(QAOA_ERR_OUT_OF_MEMORY,
                     "scratch of %zu bytes exceeds the budget of %zu", L->cv.total,
                     ctx->budget);
  if (ctx->device < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
  return QAOA_OK;
}

}  // namespace

extern "C" {

const char* qaoa_last_error(void) { return g_err.c_str(); }
const char* qaoa_version(void) { return "dqaoa-gfx950 0.1"; }

int qaoa_create(qaoa_ctx** out, int device, size_t hbm_budget) {
  if (!out) return set_error(QAOA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (device == QAOA_DEVICE_NONE) {
    qaoa_ctx* c = new qaoa_ctx();
    c->device = -1;
    c->budget = hbm_budget ? hbm_budget : SIZE_MAX;
    *out = c;
    return QAOA_OK;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return set_error(QAOA_ERR_NO_DEVICE, "no HIP device available");
  }
  if (device < 0 || device >= count)
    return set_error(QAOA_ERR_NO_DEVICE, "device %d not in [0, %d)", device, count);
  DeviceGuard g(device);
  if (!g.ok) return set_error(QAOA_ERR_HIP, "hipSetDevice(%d) failed", device);
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) return hip_error(e, "hipMemGetInfo");
    hbm_budget = (size_t)(0.9 * (double)fr);
  }
  qaoa_ctx* c = new qaoa_ctx();
  c->device = device;
  c->budget = hbm_budget;
  hipError_t e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete c;
    return hip_error(e, "hipEventCreate");
  }
  int rc = noalloc_setup(device);
  if (rc) {
    (void)hipEventDestroy(c->done);
    delete c;
    return rc;
  }
  *out = c;
  return QAOA_OK;
}

int qaoa_destroy(qaoa_ctx* ctx) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  if (ctx->device >= 0) {
    DeviceGuard g(ctx->device);
    if (ctx->any) (void)hipEventSynchronize(ctx->done);
    for (auto& r : ctx->recs) {
      (void)hipEventSynchronize(r.b);
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
  }
  delete ctx;
  return QAOA_OK;
}

int qaoa_plan(qaoa_ctx* ctx, int prec, int B, int n, int p, int S, int grad,
              qaoa_plan_info* out) {
  int rc = check_common(ctx, prec, B, n, p, S);
  if (rc) return rc;
  if (!out) return set_error(QAOA_ERR_INVALID_ARG, "out is NULL");
  Layout L;
  rc = make_layout(grad ? OP_GRAD : OP_EXPECT, prec, B, n, p, S, 0, &L);
  if (rc) return rc;
  const Plan& P = L.plan;
  const int np = P.npass;
  out->sets = P.sets;
  if (grad) {
    // forward passes 0..np-2 write checkpoints (all but the first read one);
    // the fused last pass reads one checkpoint and writes lambda; backward
    // passes np-2..0 read a checkpoint and lambda, and write lambda (k >= 1).
    out->passes = 2 * np - 1;
    out->state_reads = np > 1 ? (np - 2) + 1 + 2 * (np - 1) : 0;
    out->state_writes = np > 1 ? (np - 1) + 1 + (np - 2) : 0;
  } else {
    out->passes = np;
    out->state_reads = np - 1;
    out->state_writes = np - 1;
  }
  out->tile_qubits = P.k[0];
  out->chunk_qubits = P.c;
  out->scratch_bytes = L.cv.total;
  return QAOA_OK;
}

int qaoa_plan_passes(qaoa_ctx* ctx, int prec, int n, int p, int grad, int* out,
                     int max_passes, int* npass) {
  int rc = check_common(ctx, prec, 1, n, p, 1);
  if (rc) return rc;
  if (!npass || (!out && max_passes > 0))
    return set_error(QAOA_ERR_INVALID_ARG, "out/npass is NULL");
  Plan P;
  if (!choose_plan(grad ? OP_GRAD : OP_EXPECT, prec, n, p, &P))
    return set_error(QAOA_ERR_UNSUPPORTED, "no pass plan for n = %d", n);
  *npass = P.npass;
  for (int i = 0; i < P.npass && i < max_passes; ++i) {
    const PassDesc& d = P.pass[i];
    const int rec[10] = {d.set, d.k, d.c, d.a, d.mixlo, d.lead, d.ja, d.jb, d.flags, d.kind};
    for (int f = 0; f < 10; ++f) out[10 * i + f] = rec[f];
  }
  return QAOA_OK;
}

int qaoa_profile_enable(qaoa_ctx* ctx, int enable) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  ctx->prof = enable != 0;
  return QAOA_OK;
}

int qaoa_profile_read(qaoa_ctx* ctx, int reset, long long* launches,
                      double* total_ms, double* state_bytes) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  if (ctx->device >= 0) {
    DeviceGuard g(ctx->device);
    for (auto& r : ctx->recs) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) return hip_error(e, "hipEventElapsedTime");
      ctx->prof_ms += ms;
      ctx->prof_bytes += r.bytes;
      ctx->prof_launches += 1;
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    ctx->recs.clear();
  }
  if (launches) *launches = ctx->prof_launches;
  if (total_ms) *total_ms = ctx->prof_ms;
  if (state_bytes) *state_bytes = ctx->prof_bytes;
  if (reset) {
    ctx->prof_launches = 0;
    ctx->prof_ms = 0.0;
    ctx->prof_bytes = 0.0;
  }
  return QAOA_OK;
}

int qaoa_expect(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
                const double* Q, const double* gammas, const double* betas,
                double* expect, double* norm, void* probs, qaoa_stream_t stream) {
  int rc = check_common(ctx, prec, B, n, p, S);
  if (rc) return rc;
  if (!Q || !gammas || !betas || !expect)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, gammas, betas and expect must be non-NULL");
  if (n <= small_fwd_nmax(prec) && !fwd_reg_off()) {
    // the whole state in one work-group's registers: no plan and no scratch
    if (ctx->device < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    {
      const size_t amp = prec == QAOA_C64 ? 8 : 16;
      TimerScope ts(ctx->timer(), s, probs ? 0.5 * amp * ((double)B * S) * (double)(1ull << n) : 0.0);
      e = launch_small_expect(prec, n, p, S, B * S, Q, gammas, betas, expect, norm, probs,
                              nullptr, s);
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? QAOA_OK : hip_error(e, "whole-state evaluation");
  }
  Layout L;
  rc = prepare_call(ctx, OP_EXPECT, prec, B, n, p, S, 0, &L);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  char* base = nullptr;
  rc = acquire(ctx, L.cv.total, s, &base);
  if (rc) return rc;
  rc = enqueue_expect(L, base, Q, gammas, betas, expect, norm, probs, nullptr, s,
                      ctx->timer());
  if (rc) return rc;
  return finish(ctx, s);
}

int qaoa_expect_noalloc(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
                        const double* Q, const double* gammas, const double* betas,
                        double* expect, double* norm, void* probs, qaoa_stream_t stream) {
  int rc = check_common(ctx, prec, B, n, p, S);
  if (rc) return rc;
  if (!Q || !gammas || !betas || !expect)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, gammas, betas and expect must be non-NULL");
  Layout L;
  rc = make_layout(OP_EXPECT, prec, B, n, p, S, 0, &L);
  if (rc) return rc;
  if (L.cv.total > NOALLOC_BYTES)
    return set_error(QAOA_ERR_OUT_OF_MEMORY,
                     "qaoa_expect_noalloc: %d state(s) of %d qubits need %zu bytes of scratch; "
                     "its fixed scratch holds %zu",
                     B * S, n, L.cv.total, NOALLOC_BYTES);
  if (ctx->device < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
  char* base = g_noalloc_ptr[ctx->device];  // set by qaoa_create on this device
  if (!base) return set_error(QAOA_ERR_HIP, "no scratch address for device %d", ctx->device);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  rc = enqueue_expect(L, base, Q, gammas, betas, expect, norm, probs, nullptr, s, nullptr);
  if (rc) return rc;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QAOA_OK : hip_error(e, "kernel launch");
}

int qaoa_state(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
               const double* Q, const double* gammas, const double* betas,
               void* psi, double* expect, double* norm, qaoa_stream_t stream) {
  int rc = check_common(ctx, prec, B, n, p, S);
  if (rc) return rc;
  if (!Q || !gammas || !betas || !psi)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, gammas, betas and psi must be non-NULL");
  Layout L;
  rc = prepare_call(ctx, OP_EXPECT, prec, B, n, p, S, 0, &L);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  char* base = nullptr;
  rc = acquire(ctx, L.cv.total, s, &base);
  if (rc) return rc;
  rc = enqueue_expect(L, base, Q, gammas, betas, expect, norm, nullptr, psi, s,
                      ctx->timer());
  if (rc) return rc;
  return finish(ctx, s);
}

int qaoa_sample(qaoa_ctx* ctx, int prec, int B, int n, int p, const double* Q,
                const double* gammas, const double* betas, int shots,
                uint64_t seed, uint64_t* z, double* cz, uint64_t* best_z,
                double* best_c, double* expect, qaoa_stream_t stream) {
  int rc = check_common(ctx, prec, B, n, p, 1);
  if (rc) return rc;
  if (!Q || !gammas || !betas || !z || !best_z || !best_c)
    return set_error(QAOA_ERR_INVALID_ARG,
                     "Q, gammas, betas, z, best_z and best_c must be non-NULL");
  if (shots < 1) return set_error(QAOA_ERR_INVALID_ARG, "shots = %d < 1", shots);
  Layout L;
  rc = prepare_call(ctx, OP_SAMPLE, prec, B, n, p, 1, shots, &L);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  char* base = nullptr;
  rc = acquire(ctx, L.cv.total, s, &base);
  if (rc) return rc;
  rc = enqueue_sample(L, base, Q, gammas, betas, shots, seed, nullptr, z, cz, best_z,
                      best_c, expect, s, ctx->timer());
  if (rc) return rc;
  return finish(ctx, s);
}

int qaoa_grad(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
              const double* Q, const double* gammas, const double* betas,
              double* expect, double* dgamma, double* dbeta, qaoa_stream_t stream) {
  int rc = check_common(ctx, prec, B, n, p, S);
  if (rc) return rc;
  if (!Q || !gammas || !betas || !dgamma || !dbeta)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, gammas, betas, dgamma and dbeta must be non-NULL");
  if (n <= small_grad_limit(prec)) {
    // the whole state in one work-group's registers: no plan and no scratch
    if (ctx->device < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    {
      TimerScope ts(ctx->timer(), s, 0.0);
      e = launch_small_grad(prec, n, p, S, B * S, Q, gammas, betas, expect, dgamma, dbeta, s);
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? QAOA_OK : hip_error(e, "whole-state gradient");
  }
  Layout L;
  rc = prepare_call(ctx, OP_GRAD, prec, B, n, p, S, 0, &L);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  char* base = nullptr;
  rc = acquire(ctx, L.cv.total, s, &base);
  if (rc) return rc;
  rc = enqueue_grad(L, base, Q, gammas, betas, expect, dgamma, dbeta, s, ctx->timer());
  if (rc) return rc;
  return finish(ctx, s);
}

}  // extern "C"

// Used by the solve queue.
namespace dq {
int ctx_device(qaoa_ctx* c) { return c ? c->device : -1; }
size_t ctx_budget(qaoa_ctx* c) { return c ? c->budget : 0; }
}  // namespace dq
