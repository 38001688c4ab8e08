// Batched COBYLA-type optimisation of QAOA parameters (Sec. IV: the paper
// optimises each sub-QUBO's (gamma, beta) from random values with COBYLA).
//
// COBYLA (Powell, 1994) keeps a simplex of n + 1 points, steps to the
// minimiser of the linear interpolant of the objective inside a ball of
// radius rho, keeps the simplex well shaped with geometry steps, and shrinks
// rho from rhobeg to rhoend.  The QAOA parameters are unconstrained, so the
// method reduces to:
//   * start at x_0 and x_0 + rho e_i; the best point is the optimal vertex,
//     the others displacements d_i from it (D = [d_1 .. d_n], A = D^{-1});
//   * model gradient g = A^T (f_i - f_0);
//   * a vertex farther than 2.1 rho from x_0, or nearer than rho / 4 to its
//     opposite face (distance 1 / |row i of A|), is replaced by a geometry
//     step x_0 + rho / 2 * v, v the unit face normal signed so that g.v <= 0
//     (the farthest vertex first, else the flattest);
//   * else the trust step d = -rho g / |g| replaces the vertex j maximising
//     |(A d)_j| (the largest simplex; ties to the smaller j), and a ratio of
//     actual to predicted (rho |g|) reduction below 0.1 halves rho (rho =
//     rhoend once rho <= 1.5 rhoend); when rho cannot shrink further the
//     optimiser stops; g = 0 also shrinks rho;
//   * a point better than x_0 becomes the optimal vertex;
//   * at most maxfun evaluations.
// Each optimiser is a state machine that asks for one point at a time, so
// many run side by side: every round, the points of all running optimisers
// are evaluated by one qaoa_expect call (one problem per optimiser), i.e.
// the GPU sees batches, not single evaluations.
#include "internal.h"
#include "../../include/dqaoa.h"

#include <cmath>
#include <vector>

namespace dq {
int ctx_device(qaoa_ctx* c);
namespace {

constexpr double C_ALPHA = 0.25, C_BETA = 2.1, C_GAMMA = 0.5, C_ETA = 0.1;

// Inverse of the n x n matrix M (column j = M[j*n .. j*n + n)) by
// Gauss-Jordan elimination with partial pivoting; false if singular.
bool invert(int n, const std::vector<double>& M, std::vector<double>& inv) {
  // work on row-major R = M as a matrix (R[r][c] = M[c*n + r]) augmented with I
  std::vector<double> a((size_t)n * 2 * n, 0.0);
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) a[(size_t)r * 2 * n + c] = M[(size_t)c * n + r];
    a[(size_t)r * 2 * n + n + r] = 1.0;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * 2 * n + c]) > std::fabs(a[(size_t)piv * 2 * n + c])) piv = r;
    const double pv = a[(size_t)piv * 2 * n + c];
    if (pv == 0.0 || !std::isfinite(pv)) return false;
    if (piv != c)
      for (int k = 0; k < 2 * n; ++k) std::swap(a[(size_t)piv * 2 * n + k], a[(size_t)c * 2 * n + k]);
    for (int k = 0; k < 2 * n; ++k) a[(size_t)c * 2 * n + k] /= pv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double m = a[(size_t)r * 2 * n + c];
      if (m == 0.0) continue;
      for (int k = 0; k < 2 * n; ++k) a[(size_t)r * 2 * n + k] -= m * a[(size_t)c * 2 * n + k];
    }
  }
  inv.assign((size_t)n * n, 0.0);  // row-major: inv[r*n + c] = (M^{-1})_{rc}
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) inv[(size_t)r * n + c] = a[(size_t)r * 2 * n + n + c];
  return true;
}

struct Cobyla {
  enum { ASK_F0, ASK_INIT, ASK_GEOM, ASK_TRUST, DONE };
  int n = 0, maxfun = 0, nfev = 0, stage = DONE, init_i = 0, pj = 0;
  double rho = 0.0, rhoend = 0.0, f0 = 0.0, pred = 0.0;
  std::vector<double> x0, D, fv, pd;  // D: column j = displacement j

  void start(const double* x, int nv, double rb, double re, int mf) {
    n = nv;
    rho = rb;
    rhoend = re;
    maxfun = mf;
    nfev = 0;
    x0.assign(x, x + n);
    D.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) D[(size_t)j * n + j] = rho;
    fv.assign(n, 0.0);
    pd.assign(n, 0.0);
    stage = ASK_F0;
  }
  // the point to evaluate next
  void point(double* x) const {
    for (int k = 0; k < n; ++k) x[k] = x0[k];
    if (stage == ASK_INIT)
      for (int k = 0; k < n; ++k) x[k] += D[(size_t)init_i * n + k];
    else if (stage == ASK_GEOM || stage == ASK_TRUST)
      for (int k = 0; k < n; ++k) x[k] += pd[k];
  }
  void rebase(int j) {
    std::vector<double> dj(D.begin() + (size_t)j * n, D.begin() + (size_t)(j + 1) * n);
    for (int k = 0; k < n; ++k) x0[k] += dj[k];
    for (int c = 0; c < n; ++c)
      for (int k = 0; k < n; ++k) D[(size_t)c * n + k] -= dj[k];
    for (int k = 0; k < n; ++k) D[(size_t)j * n + k] = -dj[k];
    std::swap(f0, fv[j]);
  }
  void shrink_or_stop() {
    if (rho <= rhoend) {
      stage = DONE;
      return;
    }
    rho *= 0.5;
    if (rho <= 1.5 * rhoend) rho = rhoend;
  }
  // choose the next evaluation (or stop)
  void plan() {
    std::vector<double> A, g(n), dist(n), sig(n);
    for (;;) {
      if (nfev >= maxfun) {
        stage = DONE;
        return;
      }
      if (!invert(n, D, A)) {  // cannot happen for a simplex built by these steps
        stage = DONE;
        return;
      }
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += A[(size_t)r * n + i] * (fv[r] - f0);
        g[i] = s;
        double dn = 0.0, an = 0.0;
        for (int k = 0; k < n; ++k) {
          dn += D[(size_t)i * n + k] * D[(size_t)i * n + k];
          an += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        }
        dist[i] = std::sqrt(dn);
        sig[i] = 1.0 / std::sqrt(an);
      }
      int far = 0, flat = 0;
      for (int i = 1; i < n; ++i) {
        if (dist[i] > dist[far]) far = i;
        if (sig[i] < sig[flat]) flat = i;
      }
      if (dist[far] > C_BETA * rho || sig[flat] < C_ALPHA * rho) {
        const int j = dist[far] > C_BETA * rho ? far : flat;
        double an = 0.0, gv = 0.0;
        for (int k = 0; k < n; ++k) an += A[(size_t)j * n + k] * A[(size_t)j * n + k];
        an = std::sqrt(an);
        for (int k = 0; k < n; ++k) gv += g[k] * A[(size_t)j * n + k] / an;
        const double sgn = gv > 0.0 ? -1.0 : 1.0;
        for (int k = 0; k < n; ++k) pd[k] = C_GAMMA * rho * sgn * A[(size_t)j * n + k] / an;
        pj = j;
        stage = ASK_GEOM;
        return;
      }
      double gn = 0.0;
      for (int k = 0; k < n; ++k) gn += g[k] * g[k];
      gn = std::sqrt(gn);
      if (gn == 0.0) {
        shrink_or_stop();
        if (stage == DONE) return;
        continue;
      }
      for (int k = 0; k < n; ++k) pd[k] = -rho * g[k] / gn;
      pred = rho * gn;
      int j = 0;
      double best = -1.0;
      for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[(size_t)r * n + k] * pd[k];
        if (std::fabs(s) > best) {
          best = std::fabs(s);
          j = r;
        }
      }
      pj = j;
      stage = ASK_TRUST;
      return;
    }
  }
  void tell(double f) {
    ++nfev;
    switch (stage) {
      case ASK_F0:
        f0 = f;
        init_i = 0;
        stage = ASK_INIT;
        if (nfev >= maxfun) stage = DONE;
        return;
      case ASK_INIT: {
        fv[init_i++] = f;
        if (init_i < n) {
          if (nfev >= maxfun) stage = DONE;
          return;
        }
        int b = 0;
        for (int i = 1; i < n; ++i)
          if (fv[i] < fv[b]) b = i;
        if (fv[b] < f0) rebase(b);
        stage = ASK_TRUST;  // placeholder until plan() decides
        plan();
        return;
      }
      case ASK_GEOM:
        for (int k = 0; k < n; ++k) D[(size_t)pj * n + k] = pd[k];
        fv[pj] = f;
        if (f < f0) rebase(pj);
        plan();
        return;
      case ASK_TRUST: {
        const double ratio = (f0 - f) / pred;
        for (int k = 0; k < n; ++k) D[(size_t)pj * n + k] = pd[k];
        fv[pj] = f;
        if (f < f0) rebase(pj);
        if (ratio < C_ETA) {
          shrink_or_stop();
          if (stage == DONE) return;
        }
        plan();
        return;
      }
      default:
        return;
    }
  }
};

}  // namespace
}  // namespace dq

using namespace dq;

extern "C" int qaoa_cobyla(qaoa_ctx* ctx, int prec, int B, int n, int p, const double* Q,
                           const double* theta0, double rhobeg, double rhoend, int maxfun,
                           double* theta, double* expect, int* nfev, int* rounds,
                           double* trace, qaoa_stream_t stream) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  if (prec != QAOA_C128 && prec != QAOA_C64)
    return set_error(QAOA_ERR_INVALID_ARG, "prec %d is not QAOA_C128 or QAOA_C64", prec);
  if (B < 1 || B > 65535) return set_error(QAOA_ERR_INVALID_ARG, "B = %d outside [1, 65535]", B);
  if (n < 1 || n > QAOA_MAX_N)
    return set_error(QAOA_ERR_INVALID_ARG, "n = %d outside [1, %d]", n, QAOA_MAX_N);
  if (p < 1 || p > QAOA_MAX_P)
    return set_error(QAOA_ERR_INVALID_ARG, "p = %d outside [1, %d]", p, QAOA_MAX_P);
  if (!(rhoend > 0.0) || !(rhobeg >= rhoend) || !std::isfinite(rhobeg))
    return set_error(QAOA_ERR_INVALID_ARG, "need rhobeg >= rhoend > 0 (got %g, %g)", rhobeg,
                     rhoend);
  if (maxfun < 1) return set_error(QAOA_ERR_INVALID_ARG, "maxfun = %d < 1", maxfun);
  if (!Q || !theta0 || !theta || !expect)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, theta0, theta and expect must be non-NULL");
  if (ctx_device(ctx) < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
  const int m = 2 * p;
  std::vector<Cobyla> opt(B);
  for (int b = 0; b < B; ++b) opt[b].start(theta0 + (size_t)b * m, m, rhobeg, rhoend, maxfun);
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  (void)hipSetDevice(ctx_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  const size_t nn = (size_t)n * n;
  double *Qc = nullptr, *gd = nullptr, *bd = nullptr, *ed = nullptr;
  int rc = QAOA_OK;
  hipError_t e = hipMalloc(&Qc, (size_t)B * nn * 8);
  if (e == hipSuccess) e = hipMalloc(&gd, (size_t)B * p * 8);
  if (e == hipSuccess) e = hipMalloc(&bd, (size_t)B * p * 8);
  if (e == hipSuccess) e = hipMalloc(&ed, (size_t)B * 8);
  std::vector<int> act, prev_act;
  std::vector<double> hg((size_t)B * p), hb((size_t)B * p), he(B), x(m);
  int nr = 0;
  while (e == hipSuccess && rc == QAOA_OK) {
    act.clear();
    for (int b = 0; b < B; ++b)
      if (opt[b].stage != Cobyla::DONE) act.push_back(b);
    if (act.empty()) break;
    if (act != prev_act) {  // gather the running problems' Q (from the caller's Q)
      for (size_t k = 0; k < act.size() && e == hipSuccess; ++k)
        e = hipMemcpyAsync(Qc + k * nn, Q + (size_t)act[k] * nn, nn * 8, hipMemcpyDeviceToDevice, s);
      prev_act = act;
    }
    for (size_t k = 0; k < act.size(); ++k) {
      opt[act[k]].point(x.data());
      for (int j = 0; j < p; ++j) {
        hg[k * p + j] = x[j];
        hb[k * p + j] = x[p + j];
      }
      if (trace) {  // the point of this problem's next evaluation
        double* t = trace + ((size_t)act[k] * maxfun + opt[act[k]].nfev) * (m + 1);
        for (int j = 0; j < m; ++j) t[j] = x[j];
      }
    }
    const int Ba = (int)act.size();
    if (e == hipSuccess) e = hipMemcpyAsync(gd, hg.data(), (size_t)Ba * p * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(bd, hb.data(), (size_t)Ba * p * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) break;
    rc = qaoa_expect(ctx, prec, Ba, n, p, 1, Qc, gd, bd, ed, nullptr, nullptr, stream);
    if (rc != QAOA_OK) break;
    e = hipMemcpyAsync(he.data(), ed, (size_t)Ba * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    for (size_t k = 0; k < act.size(); ++k) {
      if (trace) trace[((size_t)act[k] * maxfun + opt[act[k]].nfev) * (m + 1) + m] = he[k];
      opt[act[k]].tell(he[k]);
    }
    ++nr;
  }
  if (e != hipSuccess && rc == QAOA_OK) rc = hip_error(e, "cobyla rounds");
  (void)hipStreamSynchronize(s);
  (void)hipFree(Qc);
  (void)hipFree(gd);
  (void)hipFree(bd);
  (void)hipFree(ed);
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc != QAOA_OK) return rc;
  for (int b = 0; b < B; ++b) {
    for (int k = 0; k < m; ++k) theta[(size_t)b * m + k] = opt[b].x0[k];
    expect[b] = opt[b].f0;
    if (nfev) nfev[b] = opt[b].nfev;
  }
  if (rounds) *rounds = nr;
  return QAOA_OK;
}
