// QAOA state-vector oracle: TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct CPU (complex128, FP64) implementation of
// what the GPU path computes.  It exists so that tests, the smoke check and
// the benchmark's CPU-baseline leg can compare the HIP kernels against the
// mathematics of the paper.  It shares no code, header, table or constant
// with the HIP library, and the product path never calls it.
//
// Paper: "GPU-Accelerated Distributed QAOA on Large-scale HPC Ecosystems"
// (arXiv 2506.10531).
//   * Sec. IV, Eq. (1): the objective is minimised over the parameters; for a
//     QUBO the objective is the energy C(z) = z^T Q z of bit string z.
//   * Sec. IV, Eq. (2): |psi(theta)> = prod_{j=1..p} e^{-i H_X beta_j}
//     e^{-i H gamma_j} |+>, with mixing Hamiltonian H_X = -sum_i X_i and the
//     problem Hamiltonian H diagonal with entries C(z).
//   * Sec. IV (after Eq. (2)): the measured bit string is the candidate
//     solution.
//
// Readings of the paper taken here (each one is listed in the design notes):
//   * bit i of the basis index z is variable i / qubit i (little endian);
//   * layer j = 1 acts first on |+>;
//   * e^{-i H_X beta} = e^{+i beta sum_q X_q} = prod_q (cos b I + i sin b X_q)
//     (the paper's sign of H_X taken literally);
//   * the phase uses C(z) itself (no Ising offset dropped);
//   * sampling draws u_s from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
//     and returns the smallest z whose running probability sum exceeds
//     u_s * total;
//   * the optimiser used by the solve loop is Adam (Kingma & Ba 2015) on the
//     exact gradient, in place of the paper's COBYLA.
//
// Parity pins (tests/test_oracle_pins.py): dense matrix exponentials for
// n <= 8, the closed-form p = 1 expectation for quadratic costs, beta = 0 /
// gamma = 0 uniformity and the mean of C, the diagonal-Q product formula,
// conjugation and beta + pi symmetries, exhaustive argmin against itertools,
// the adjoint gradient against central finite differences, and sampling
// frequencies against a chi-square test; the solve loop's Adam trajectory
// against torch.optim.Adam, an independent implementation of the method.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

typedef std::complex<double> cplx;

namespace {

// Sum of x[0..m) by pairwise (cascade) summation: deterministic, error
// O(log m * eps) instead of O(m * eps).
double pairwise_sum(const double* x, size_t m) {
  if (m <= 32) {
    double s = 0.0;
    for (size_t i = 0; i < m; ++i) s += x[i];
    return s;
  }
  size_t h = m / 2;
  return pairwise_sum(x, h) + pairwise_sum(x + h, m - h);
}

// Deterministic parallel pairwise sum: fixed 4096-element blocks summed
// pairwise, then the block sums summed pairwise.  The tree does not depend on
// the number of threads.
double det_sum(const std::vector<double>& x) {
  const size_t B = 4096;
  size_t nb = (x.size() + B - 1) / B;
  std::vector<double> part(nb);
#pragma omp parallel for schedule(static)
  for (long long b = 0; b < (long long)nb; ++b) {
    size_t lo = (size_t)b * B, hi = std::min(x.size(), lo + B);
    part[b] = pairwise_sum(x.data() + lo, hi - lo);
  }
  return pairwise_sum(part.data(), nb);
}

// C(z) = sum_i sum_j Q_ij z_i z_j, summed directly over the set bits of z.
double energy(int n, const double* Q, uint64_t z) {
  double c = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!((z >> i) & 1ull)) continue;
    for (int j = 0; j < n; ++j)
      if ((z >> j) & 1ull) c += Q[(size_t)i * n + j];
  }
  return c;
}

void cost_table(int n, const double* Q, std::vector<double>& C) {
  size_t N = (size_t)1 << n;
  C.resize(N);
#pragma omp parallel for schedule(static)
  for (long long z = 0; z < (long long)N; ++z) C[z] = energy(n, Q, (uint64_t)z);
}

// psi(z) <- e^{-i g C(z)} psi(z): the problem-Hamiltonian factor of Eq. (2).
void apply_phase(std::vector<cplx>& psi, const std::vector<double>& C, double g) {
  size_t N = psi.size();
#pragma omp parallel for schedule(static)
  for (long long z = 0; z < (long long)N; ++z) {
    double a = g * C[z];
    psi[z] *= cplx(std::cos(a), -std::sin(a));
  }
}

// psi <- e^{+i b X_q} psi for every qubit q: the mixer factor of Eq. (2)
// with H_X = -sum_q X_q.  Per pair (z, z | 2^q) with bit q of z clear:
//   a0' = cos b a0 + i sin b a1,  a1' = i sin b a0 + cos b a1.
void apply_mixer(std::vector<cplx>& psi, int n, double b) {
  size_t N = psi.size();
  const cplx c(std::cos(b), 0.0), is(0.0, std::sin(b));
  for (int q = 0; q < n; ++q) {
    size_t m = (size_t)1 << q;
#pragma omp parallel for schedule(static)
    for (long long k = 0; k < (long long)(N / 2); ++k) {
      size_t lo = (size_t)k & (m - 1);
      size_t z0 = (((size_t)k - lo) << 1) | lo;  // insert a 0 at bit q
      size_t z1 = z0 | m;
      cplx a0 = psi[z0], a1 = psi[z1];
      psi[z0] = c * a0 + is * a1;
      psi[z1] = is * a0 + c * a1;
    }
  }
}

// |psi(theta)> of Eq. (2): start from |+> (amplitude 2^{-n/2}), then layer
// j = 1..p applies the phase with gamma_j followed by the mixer with beta_j.
void prepare(int n, int p, const std::vector<double>& C, const double* g,
             const double* b, std::vector<cplx>& psi) {
  size_t N = (size_t)1 << n;
  psi.assign(N, cplx(1.0 / std::sqrt((double)N), 0.0));
  for (int j = 0; j < p; ++j) {
    apply_phase(psi, C, g[j]);
    apply_mixer(psi, n, b[j]);
  }
}

// <C> = sum_z |psi(z)|^2 C(z) and sum_z |psi(z)|^2 (Eq. (1) objective).
void expectation(const std::vector<cplx>& psi, const std::vector<double>& C,
                 double* e, double* nrm) {
  size_t N = psi.size();
  std::vector<double> t(N), u(N);
#pragma omp parallel for schedule(static)
  for (long long z = 0; z < (long long)N; ++z) {
    double pz = std::norm(psi[z]);
    t[z] = pz * C[z];
    u[z] = pz;
  }
  *e = det_sum(t);
  if (nrm) *nrm = det_sum(u);
}

// d<C>/dgamma_j and d<C>/dbeta_j by the adjoint (reverse) method.
// With lambda = C psi_p propagated backwards through the inverse layers:
//   d<C>/dbeta_j  = 2 Re <lambda| i sum_q X_q |psi>  (before undoing M_j)
//                 = -2 Im sum_q <lambda|X_q|psi>,
//   d<C>/dgamma_j = 2 Re <lambda| -i C |psi>        (after undoing M_j)
//                 =  2 Im <lambda|C|psi>,
// because dM/dbeta = i (sum_q X_q) M and dP/dgamma = -i C P.
void adjoint(int n, int p, const std::vector<double>& C, const double* g,
             const double* b, double* e, double* dg, double* db) {
  std::vector<cplx> psi;
  prepare(n, p, C, g, b, psi);
  expectation(psi, C, e, nullptr);
  size_t N = psi.size();
  std::vector<cplx> lam(N);
#pragma omp parallel for schedule(static)
  for (long long z = 0; z < (long long)N; ++z) lam[z] = C[z] * psi[z];
  std::vector<double> t(N);
  for (int j = p - 1; j >= 0; --j) {
    // beta_j: -2 Im sum_q <lambda|X_q|psi>
    double acc = 0.0;
    for (int q = 0; q < n; ++q) {
      size_t m = (size_t)1 << q;
#pragma omp parallel for schedule(static)
      for (long long z = 0; z < (long long)N; ++z)
        t[z] = std::imag(std::conj(lam[z]) * psi[(size_t)z ^ m]);
      acc += det_sum(t);
    }
    db[j] = -2.0 * acc;
    // undo the mixer: M(beta)^dagger = M(-beta)
    apply_mixer(psi, n, -b[j]);
    apply_mixer(lam, n, -b[j]);
    // gamma_j: 2 Im <lambda|C|psi>
#pragma omp parallel for schedule(static)
    for (long long z = 0; z < (long long)N; ++z)
      t[z] = std::imag(std::conj(lam[z]) * psi[z]) * C[z];
    dg[j] = 2.0 * det_sum(t);
    // undo the phase: P(gamma)^dagger = P(-gamma)
    apply_phase(psi, C, -g[j]);
    apply_phase(lam, C, -g[j]);
  }
}

// SplitMix64 output function (Steele, Lea, Flood 2014) evaluated at the
// counter value seed + (s + 1) * golden gamma; the top 53 bits scaled by
// 2^-53 give u_s in [0, 1).
double splitmix_uniform(uint64_t seed, uint64_t s) {
  uint64_t x = seed + (s + 1ull) * 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x = x ^ (x >> 31);
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

extern "C" {

int oracle_num_threads(void) { return omp_get_max_threads(); }

double oracle_energy(int n, const double* Q, uint64_t z) { return energy(n, Q, z); }

// C[z] for all 2^n bit strings.
void oracle_cost_table(int n, const double* Q, double* C_out) {
  std::vector<double> C;
  cost_table(n, Q, C);
  std::memcpy(C_out, C.data(), C.size() * sizeof(double));
}

// The final state |psi(theta)> of Eq. (2) as interleaved (re, im) pairs.
void oracle_state(int n, int p, const double* Q, const double* gammas,
                  const double* betas, double* psi_out) {
  std::vector<double> C;
  cost_table(n, Q, C);
  std::vector<cplx> psi;
  prepare(n, p, C, gammas, betas, psi);
  std::memcpy(psi_out, psi.data(), psi.size() * sizeof(cplx));
}

// For S parameter sets (gammas/betas laid out [S][p]): <C>, the squared norm
// and optionally the probability vector [S][2^n].
void oracle_expect(int n, int p, int S, const double* Q, const double* gammas,
                   const double* betas, double* expect, double* norm,
                   double* probs) {
  std::vector<double> C;
  cost_table(n, Q, C);
  size_t N = (size_t)1 << n;
  std::vector<cplx> psi;
  for (int s = 0; s < S; ++s) {
    prepare(n, p, C, gammas + (size_t)s * p, betas + (size_t)s * p, psi);
    expectation(psi, C, expect + s, norm ? norm + s : nullptr);
    if (probs) {
      double* P = probs + (size_t)s * N;
#pragma omp parallel for schedule(static)
      for (long long z = 0; z < (long long)N; ++z) P[z] = std::norm(psi[z]);
    }
  }
}

// Adjoint gradient for S parameter sets: expect[S], dgamma[S][p], dbeta[S][p].
void oracle_grad(int n, int p, int S, const double* Q, const double* gammas,
                 const double* betas, double* expect, double* dgamma,
                 double* dbeta) {
  std::vector<double> C;
  cost_table(n, Q, C);
  for (int s = 0; s < S; ++s)
    adjoint(n, p, C, gammas + (size_t)s * p, betas + (size_t)s * p, expect + s,
            dgamma + (size_t)s * p, dbeta + (size_t)s * p);
}

double oracle_uniform(uint64_t seed, uint64_t s) { return splitmix_uniform(seed, s); }

// Bit-string sampling from |psi(theta)|^2: shot s draws u_s and returns the
// smallest z with CDF(z) > u_s * CDF(2^n - 1), where CDF is the running FP64
// sum of the probabilities in increasing z.  Also returns C(z_s), the best
// sample (lowest C, ties to the smallest z) and the CDF gap at the chosen z
// (the distance of u_s * total to the nearer boundary of its interval, used by
// tests to discount draws that sit within rounding of a boundary).
void oracle_sample(int n, int p, const double* Q, const double* gammas,
                   const double* betas, int shots, uint64_t seed, uint64_t* z_out,
                   double* cz_out, uint64_t* best_z, double* best_c,
                   double* gap_out) {
  std::vector<double> C;
  cost_table(n, Q, C);
  std::vector<cplx> psi;
  prepare(n, p, C, gammas, betas, psi);
  size_t N = psi.size();
  std::vector<double> cdf(N);
  double run = 0.0;
  for (size_t z = 0; z < N; ++z) {
    run += std::norm(psi[z]);
    cdf[z] = run;
  }
  double total = cdf[N - 1];
  uint64_t bz = 0;
  double bc = 0.0;
  for (int s = 0; s < shots; ++s) {
    double target = splitmix_uniform(seed, (uint64_t)s) * total;
    size_t z = (size_t)(std::upper_bound(cdf.begin(), cdf.end(), target) - cdf.begin());
    if (z >= N) z = N - 1;
    z_out[s] = z;
    double c = C[z];
    if (cz_out) cz_out[s] = c;
    if (gap_out) {
      double lo = z ? cdf[z - 1] : 0.0;
      gap_out[s] = std::min(target - lo, cdf[z] - target);
    }
    if (s == 0 || c < bc || (c == bc && z < bz)) {
      bc = c;
      bz = z;
    }
  }
  if (best_z) *best_z = bz;
  if (best_c) *best_c = bc;
}

// One solve of the serving loop: `evals` iterations of (exact <C> and adjoint
// gradient at theta, then an Adam step), starting from theta0 = (gamma0,
// beta0); then <C> at the final theta and `shots` samples from it.
// Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
//       theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
void oracle_adam_solve(int n, int p, const double* Q, const double* gamma0,
                       const double* beta0, int evals, double lr, double b1,
                       double b2, double eps, int shots, uint64_t seed,
                       double* gamma_out, double* beta_out, double* expect_out,
                       uint64_t* z_out, double* cz_out, uint64_t* best_z,
                       double* best_c) {
  std::vector<double> C;
  cost_table(n, Q, C);
  std::vector<double> th(2 * p), m(2 * p, 0.0), v(2 * p, 0.0), gr(2 * p);
  for (int j = 0; j < p; ++j) {
    th[j] = gamma0[j];
    th[p + j] = beta0[j];
  }
  double e;
  for (int t = 1; t <= evals; ++t) {
    adjoint(n, p, C, th.data(), th.data() + p, &e, gr.data(), gr.data() + p);
    double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    for (int k = 0; k < 2 * p; ++k) {
      m[k] = b1 * m[k] + (1.0 - b1) * gr[k];
      v[k] = b2 * v[k] + (1.0 - b2) * gr[k] * gr[k];
      th[k] -= lr * (m[k] / c1) / (std::sqrt(v[k] / c2) + eps);
    }
  }
  for (int j = 0; j < p; ++j) {
    gamma_out[j] = th[j];
    beta_out[j] = th[p + j];
  }
  std::vector<cplx> psi;
  prepare(n, p, C, th.data(), th.data() + p, psi);
  expectation(psi, C, expect_out, nullptr);
  oracle_sample(n, p, Q, th.data(), th.data() + p, shots, seed, z_out, cz_out,
                best_z, best_c, nullptr);
}

// Exhaustive minimum of C(z); ties go to the smallest z.
void oracle_argmin(int n, const double* Q, uint64_t* z_out, double* c_out) {
  std::vector<double> C;
  cost_table(n, Q, C);
  size_t best = 0;
  for (size_t z = 1; z < C.size(); ++z)
    if (C[z] < C[best]) best = z;
  *z_out = best;
  *c_out = C[best];
}

}  // extern "C"
