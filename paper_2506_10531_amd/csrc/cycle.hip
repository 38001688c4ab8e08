// The DQAOA outer cycle on the device (Sec. V): impact factors of the
// current global solution, impact-factor directed (IFD) windows, the
// sub-QUBO gather, and the aggregation of sub-solutions, plus a host driver
// that runs one cycle through a solve queue.
//
// x is the global 0/1 solution (one byte per variable, non-zero = 1) and
// E(x) = x^T Q x (Eq. (1)).  Flipping x_i changes the energy by
//   d_i (Q_ii + g_i - 2 Q_ii x_i),  d_i = 1 - 2 x_i,  g = (Q + Q^T) x,
// so every impact factor comes from one pass over Q (rows for Q x, columns
// for Q^T x), instead of N full energy evaluations.  Aggregation keeps g
// current: a change d on window S costs dE = d_S^T g_S + d_S^T Q_SS d_S and,
// when accepted, g += (Q + Q^T) d.  All sums are FP64 in a fixed order.
#include "internal.h"
#include "../../include/dqaoa.h"

#include <chrono>
#include <cmath>
#include <vector>

namespace dq {
int ctx_device(qaoa_ctx* c);
namespace {

constexpr int MAX_K = 64;
constexpr int MAX_NV = 65536;

// u = Q x: one wave per row, coalesced along the row.
__global__ void __launch_bounds__(256) rows_kernel(int N, const double* __restrict__ Q,
                                                   const uint8_t* __restrict__ x,
                                                   double* __restrict__ u) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  const double* q = Q + (size_t)i * N;
  double s = 0.0;
  for (int j = lane; j < N; j += 64) s += x[j] ? q[j] : 0.0;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) u[i] = s;
}

// v = Q^T x (a thread per column, rows with x_i = 1 streamed in order),
// then field = u + v (in place: field holds u on entry) and the impact
// factors.
__global__ void __launch_bounds__(256) cols_kernel(int N, const double* __restrict__ Q,
                                                   const uint8_t* __restrict__ x,
                                                   double* field, double* __restrict__ imp) {
  __shared__ uint8_t xs[1024];
  const int j = blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  for (int i0 = 0; i0 < N; i0 += 1024) {
    const int cnt = min(1024, N - i0);
    for (int t = threadIdx.x; t < cnt; t += 256) xs[t] = x[i0 + t] ? 1 : 0;
    __syncthreads();
    if (j < N)
      for (int t = 0; t < cnt; ++t)
        if (xs[t]) v += Q[(size_t)(i0 + t) * N + j];
    __syncthreads();
  }
  if (j >= N) return;
  const double g = field[j] + v;
  const double qjj = Q[(size_t)j * N + j];
  const bool xj = x[j] != 0;
  field[j] = g;
  const double a = qjj + g - (xj ? 2.0 * qjj : 0.0);
  imp[j] = xj ? -a : a;
}

// Fixed-order sum over a block of NTH threads (power of two, <= 1024).
template <int NTH>
__device__ double block_total(double s, double* red) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NTH / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// E(x) = sum_i x_i u_i, one block.
__global__ void __launch_bounds__(1024) energy_kernel(int N, const uint8_t* __restrict__ x,
                                                      const double* __restrict__ u,
                                                      double* __restrict__ e) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += 1024) s += x[i] ? u[i] : 0.0;
  const double t = block_total<1024>(s, red);
  if (threadIdx.x == 0) *e = t;
}

// Rank of |impact| (largest first, ties to the smaller index, NaN last) by
// counting: order[rank_i] = i.  The comparison is a strict total order, so
// the ranks form a permutation whatever the values.
__device__ __forceinline__ double rank_key(double v) { return isnan(v) ? -1.0 : fabs(v); }
__global__ void __launch_bounds__(256) rank_kernel(int N, const double* __restrict__ imp,
                                                   int32_t* __restrict__ order) {
  __shared__ double ks[1024];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double ki = i < N ? rank_key(imp[i]) : 0.0;
  int cnt = 0;
  for (int j0 = 0; j0 < N; j0 += 1024) {
    const int c = min(1024, N - j0);
    for (int t = threadIdx.x; t < c; t += 256) ks[t] = rank_key(imp[j0 + t]);
    __syncthreads();
    for (int t = 0; t < c; ++t) {
      const double kj = ks[t];
      cnt += (kj > ki) || (kj == ki && j0 + t < i);
    }
    __syncthreads();
  }
  if (i < N) order[cnt] = i;
}

// IFD window t: ranked positions t*stride + r (r < k, cyclic), sorted
// ascending (each lane's position = the number of smaller values).
__global__ void __launch_bounds__(64) windows_kernel(int N, const int32_t* __restrict__ order,
                                                     int k, long long stride,
                                                     int32_t* __restrict__ choices) {
  const int t = blockIdx.x, r = threadIdx.x;
  const int v = r < k ? order[(int)(((long long)t * stride + r) % N)] : 0;
  int pos = 0;
  for (int s = 0; s < k; ++s) {
    const int w = __shfl(v, s, 64);
    pos += w < v;
  }
  if (r < k) choices[(size_t)t * k + pos] = v;
}

// ---- BFS / PFS windows (Sec. V-A-3) -----------------------------------------
// Variables i and j interact when W_ij = Q_ij + Q_ji != 0; window t starts at
// order[t mod N].  BFS expands the window's variables first-in first-out and
// takes each one's unselected neighbours by |W| (largest first, ties to the
// smaller index); PFS takes the unselected variable of largest |impact| that
// interacts with the window.  With no such variable both restart from the
// unselected variable of largest |impact|.  Ties go to the smaller index
// everywhere.  One 256-thread work-group per window; the picks are block
// arg-max reductions over N, so a window costs O(k N).
constexpr int TRAV_MAX_N = 16384;

// (key, index) pairs: larger key first, then smaller index; key < 0 = none.
struct Pick {
  double key;
  int idx;
};
__device__ __forceinline__ bool better(const Pick& a, const Pick& b) {
  return a.key > b.key || (a.key == b.key && a.idx < b.idx);
}
__device__ Pick block_pick(Pick p, Pick* red) {
  for (int off = 32; off > 0; off >>= 1) {
    Pick o{__shfl_xor(p.key, off, 64), __shfl_xor(p.idx, off, 64)};
    if (better(o, p)) p = o;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = p;
  __syncthreads();
  Pick b = red[0];
  for (int w = 1; w < 4; ++w)
    if (better(red[w], b)) b = red[w];
  __syncthreads();
  return b;
}

template <bool PFS>
__global__ void __launch_bounds__(256) traverse_kernel(int N, const double* __restrict__ Q,
                                                       const double* __restrict__ imp,
                                                       const int32_t* __restrict__ order, int k,
                                                       int32_t* __restrict__ choices) {
  __shared__ uint8_t sel[TRAV_MAX_N];
  __shared__ uint8_t front[TRAV_MAX_N];
  __shared__ int win[MAX_K];
  __shared__ Pick red[4];
  const int t = blockIdx.x, tid = threadIdx.x;
  for (int i = tid; i < N; i += 256) sel[i] = front[i] = 0;
  if (tid < MAX_K) win[tid] = -1;  // an unfilled place stays out of range
  __syncthreads();
  int seed = order[t % N];
  seed = seed < 0 || seed >= N ? 0 : seed;
  int cnt = 0, head = 0;
  // adds v to the window (and, for PFS, its interacting variables to the frontier)
  auto add = [&](int v) {
    if (tid == 0) {
      sel[v] = 1;
      win[cnt] = v;
    }
    if (PFS)
      for (int i = tid; i < N; i += 256)
        if (i != v && Q[(size_t)v * N + i] + Q[(size_t)i * N + v] != 0.0) front[i] = 1;
    __syncthreads();
    ++cnt;
  };
  add(seed);
  while (cnt < k) {
    Pick p{-1.0, 0x7fffffff};
    if (PFS) {
      for (int i = tid; i < N; i += 256)
        if (front[i] && !sel[i]) {
          const Pick c{fabs(imp[i]), i};
          if (better(c, p)) p = c;
        }
      p = block_pick(p, red);
    } else if (head < cnt) {
      const int u = win[head];
      for (int i = tid; i < N; i += 256) {
        if (sel[i] || i == u) continue;
        const double w = Q[(size_t)u * N + i] + Q[(size_t)i * N + u];
        if (w != 0.0) {
          const Pick c{fabs(w), i};
          if (better(c, p)) p = c;
        }
      }
      p = block_pick(p, red);
      if (p.key < 0.0) {  // u has no unselected neighbour left
        ++head;
        continue;
      }
    }
    if (p.key < 0.0) {  // restart: the unselected variable of largest |impact|
      Pick r{-1.0, 0x7fffffff};
      for (int i = tid; i < N; i += 256)
        if (!sel[i]) {
          const Pick c{fabs(imp[i]), i};
          if (better(c, r)) r = c;
        }
      p = block_pick(r, red);
      if (p.key < 0.0) break;  // every variable selected (k <= N makes this unreachable)
    }
    add(p.idx);
  }
  // the window sorted ascending
  if (tid < k) {
    const int v = win[tid];
    int pos = 0;
    for (int j = 0; j < k; ++j) pos += win[j] < v;
    choices[(size_t)t * k + pos] = v;
  }
}

// subq[t] = Q[S_t, S_t]; an index outside [0, N) makes its row and column NaN.
__global__ void __launch_bounds__(256) gather_kernel(int N, const double* __restrict__ Q, int k,
                                                     const int32_t* __restrict__ choices,
                                                     double* __restrict__ subq) {
  __shared__ int c[MAX_K];
  const int t = blockIdx.x;
  if (threadIdx.x < k) c[threadIdx.x] = choices[(size_t)t * k + threadIdx.x];
  __syncthreads();
  double* out = subq + (size_t)t * k * k;
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int a = c[e / k], b = c[e % k];
    const bool ok = a >= 0 && a < N && b >= 0 && b < N;
    out[e] = ok ? Q[(size_t)a * N + b] : __builtin_nan("");
  }
}

// Aggregation, one block, windows in order.  field and *energy hold (Q+Q^T)x
// and E(x) on entry and are kept current.
__global__ void __launch_bounds__(1024) aggregate_kernel(int N, const double* __restrict__ Q,
                                                         uint8_t* __restrict__ x,
                                                         double* __restrict__ field,
                                                         double* __restrict__ energy, int m,
                                                         int k, const int32_t* __restrict__ choices,
                                                         const uint64_t* __restrict__ subsol,
                                                         int32_t* __restrict__ accepted) {
  __shared__ int c[MAX_K];
  __shared__ double dl[MAX_K];
  __shared__ double red[16];
  __shared__ int bad;
  const int tid = threadIdx.x;
  double e = *energy;
  for (int t = 0; t < m; ++t) {
    if (tid == 0) bad = 0;
    __syncthreads();
    int bit = 0;
    if (tid < k) {
      const int ci = choices[(size_t)t * k + tid];
      c[tid] = ci;
      if (ci < 0 || ci >= N) bad = 1;
      bit = (int)((subsol[t] >> tid) & 1ull);
    }
    __syncthreads();
    if (bad) {
      if (tid == 0 && accepted) accepted[t] = -1;
      __syncthreads();
      continue;
    }
    if (tid < k) dl[tid] = (double)(bit - (x[c[tid]] ? 1 : 0));
    __syncthreads();
    // dE = d^T g + d^T Q_SS d over the window
    double s = 0.0;
    for (int q = tid; q < k * k; q += 1024) {
      const double da = dl[q / k], db = dl[q % k];
      if (da != 0.0 && db != 0.0) s += da * db * Q[(size_t)c[q / k] * N + c[q % k]];
    }
    if (tid < k && dl[tid] != 0.0) s += dl[tid] * field[c[tid]];
    const double de = block_total<1024>(s, red);
    if (de < 0.0) {
      for (int i = tid; i < N; i += 1024) {
        double f = 0.0;
        for (int a = 0; a < k; ++a)
          if (dl[a] != 0.0) f += dl[a] * (Q[(size_t)i * N + c[a]] + Q[(size_t)c[a] * N + i]);
        field[i] += f;
      }
      if (tid < k) x[c[tid]] = (uint8_t)bit;
      e += de;
    }
    if (tid == 0 && accepted) accepted[t] = de < 0.0 ? 1 : 0;
    __syncthreads();
  }
  if (tid == 0) *energy = e;
}

// Argument checks come first (they run on any context); then the device.
int check_ctx(qaoa_ctx* ctx) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  return QAOA_OK;
}
int check_dev(qaoa_ctx* ctx) {
  if (ctx_device(ctx) < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
  return QAOA_OK;
}

int check_nk(int N, int m, int k) {
  if (N < 1 || N > MAX_NV)
    return set_error(QAOA_ERR_INVALID_ARG, "N = %d outside [1, %d]", N, MAX_NV);
  if (m < 1) return set_error(QAOA_ERR_INVALID_ARG, "m = %d < 1", m);
  if (k < 1 || k > MAX_K || k > N)
    return set_error(QAOA_ERR_INVALID_ARG, "k = %d outside [1, min(N, %d)]", k, MAX_K);
  return QAOA_OK;
}

struct Dev {
  int prev = -1;
  explicit Dev(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(d);
  }
  ~Dev() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Q x goes into field first (E(x) is read from it), then field becomes
// (Q + Q^T) x.
hipError_t enqueue_impact(int N, const double* Q, const uint8_t* x, double* imp, double* field,
                          int32_t* order, double* energy, hipStream_t s) {
  hipLaunchKernelGGL(rows_kernel, dim3((N + 3) / 4), dim3(256), 0, s, N, Q, x, field);
  if (energy) hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(1024), 0, s, N, x, field, energy);
  hipLaunchKernelGGL(cols_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, Q, x, field, imp);
  if (order) hipLaunchKernelGGL(rank_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, imp, order);
  return hipGetLastError();
}

}  // namespace
}  // namespace dq

using namespace dq;

extern "C" {

size_t qaoa_cycle_workspace(int N, int m, int k) {
  if (N < 1 || N > MAX_NV || m < 1 || k < 1 || k > MAX_K) return 0;
  // impact [N] doubles; order [N], choices [m*k], accepted [m] int32;
  // subq [m*k*k] doubles; subsol [m] uint64 (each region 256-byte aligned)
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return al((size_t)N * 8) + al((size_t)N * 4) + al((size_t)m * k * 4) + al((size_t)m * 4) +
         al((size_t)m * k * k * 8) + al((size_t)m * 8);
}

int qaoa_impact(qaoa_ctx* ctx, int N, const double* Q, const uint8_t* x, double* impact,
                double* field, int32_t* order, double* energy, qaoa_stream_t stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (N < 1 || N > MAX_NV)
    return set_error(QAOA_ERR_INVALID_ARG, "N = %d outside [1, %d]", N, MAX_NV);
  if (!Q || !x || !impact || !field)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, x, impact and field must be non-NULL");
  rc = check_dev(ctx);
  if (rc) return rc;
  Dev g(ctx_device(ctx));
  hipError_t e = enqueue_impact(N, Q, x, impact, field, order, energy, (hipStream_t)stream);
  return e == hipSuccess ? QAOA_OK : hip_error(e, "impact kernels");
}

int qaoa_ifd_choices(qaoa_ctx* ctx, int N, const int32_t* order, int m, int k, int stride,
                     int32_t* choices, qaoa_stream_t stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = check_nk(N, m, k);
  if (rc) return rc;
  if (stride < 1) return set_error(QAOA_ERR_INVALID_ARG, "stride = %d < 1", stride);
  if (!order || !choices) return set_error(QAOA_ERR_INVALID_ARG, "order and choices must be non-NULL");
  rc = check_dev(ctx);
  if (rc) return rc;
  Dev g(ctx_device(ctx));
  hipLaunchKernelGGL(windows_kernel, dim3(m), dim3(64), 0, (hipStream_t)stream, N, order, k,
                     (long long)stride, choices);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QAOA_OK : hip_error(e, "windows kernel");
}

int qaoa_traversal_choices(qaoa_ctx* ctx, int N, const double* Q, const double* impact,
                           const int32_t* order, int mode, int m, int k, int32_t* choices,
                           qaoa_stream_t stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = check_nk(N, m, k);
  if (rc) return rc;
  if (N > TRAV_MAX_N)
    return set_error(QAOA_ERR_INVALID_ARG, "N = %d exceeds %d for BFS/PFS windows", N, TRAV_MAX_N);
  if (mode != QAOA_DECOMP_BFS && mode != QAOA_DECOMP_PFS)
    return set_error(QAOA_ERR_INVALID_ARG, "mode %d is not QAOA_DECOMP_BFS or _PFS", mode);
  if (!Q || !impact || !order || !choices)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, impact, order and choices must be non-NULL");
  rc = check_dev(ctx);
  if (rc) return rc;
  Dev g(ctx_device(ctx));
  if (mode == QAOA_DECOMP_PFS)
    hipLaunchKernelGGL(traverse_kernel<true>, dim3(m), dim3(256), 0, (hipStream_t)stream, N, Q,
                       impact, order, k, choices);
  else
    hipLaunchKernelGGL(traverse_kernel<false>, dim3(m), dim3(256), 0, (hipStream_t)stream, N, Q,
                       impact, order, k, choices);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QAOA_OK : hip_error(e, "traversal kernel");
}

int qaoa_decompose(qaoa_ctx* ctx, int N, const double* Q, int m, int k, const int32_t* choices,
                   double* subq, qaoa_stream_t stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = check_nk(N, m, k);
  if (rc) return rc;
  if (!Q || !choices || !subq)
    return set_error(QAOA_ERR_INVALID_ARG, "Q, choices and subq must be non-NULL");
  rc = check_dev(ctx);
  if (rc) return rc;
  Dev g(ctx_device(ctx));
  hipLaunchKernelGGL(gather_kernel, dim3(m), dim3(256), 0, (hipStream_t)stream, N, Q, k, choices,
                     subq);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QAOA_OK : hip_error(e, "gather kernel");
}

int qaoa_aggregate(qaoa_ctx* ctx, int N, const double* Q, uint8_t* x, double* field,
                   double* energy, int m, int k, const int32_t* choices, const uint64_t* subsol,
                   int32_t* accepted, qaoa_stream_t stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = check_nk(N, m, k);
  if (rc) return rc;
  if (!Q || !x || !field || !energy || !choices || !subsol)
    return set_error(QAOA_ERR_INVALID_ARG,
                     "Q, x, field, energy, choices and subsol must be non-NULL");
  rc = check_dev(ctx);
  if (rc) return rc;
  Dev g(ctx_device(ctx));
  hipLaunchKernelGGL(aggregate_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, N, Q, x,
                     field, energy, m, k, choices, subsol, accepted);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QAOA_OK : hip_error(e, "aggregate kernel");
}

int qaoa_dqaoa_cycle(qaoa_ctx* ctx, qaoa_queue* q, int N, const double* Q, uint8_t* x,
                     double* field, double* energy, int mode, int m, int k, int stride,
                     const int32_t* choices_in, const double* gamma0, const double* beta0,
                     uint64_t seed, void* work, qaoa_cycle_stats* stats, qaoa_stream_t stream) {
  using clk = std::chrono::steady_clock;
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = check_nk(N, m, k);
  if (rc) return rc;
  if (!q || !Q || !x || !field || !energy || !gamma0 || !beta0 || !work)
    return set_error(QAOA_ERR_INVALID_ARG,
                     "q, Q, x, field, energy, gamma0, beta0 and work must be non-NULL");
  if (mode != QAOA_DECOMP_IFD && mode != QAOA_DECOMP_GIVEN && mode != QAOA_DECOMP_BFS &&
      mode != QAOA_DECOMP_PFS)
    return set_error(QAOA_ERR_INVALID_ARG, "mode %d is not a QAOA_DECOMP_* mode", mode);
  if ((mode == QAOA_DECOMP_BFS || mode == QAOA_DECOMP_PFS) && N > TRAV_MAX_N)
    return set_error(QAOA_ERR_INVALID_ARG, "N = %d exceeds %d for BFS/PFS windows", N, TRAV_MAX_N);
  if (mode == QAOA_DECOMP_IFD && stride < 1)
    return set_error(QAOA_ERR_INVALID_ARG, "stride = %d < 1", stride);
  if (mode == QAOA_DECOMP_GIVEN && !choices_in)
    return set_error(QAOA_ERR_INVALID_ARG, "choices must be given with QAOA_DECOMP_GIVEN");
  if (k > 22) return set_error(QAOA_ERR_INVALID_ARG, "k = %d exceeds the solve queue's 22", k);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* w = (char*)work;
  double* imp = (double*)w;
  w += al((size_t)N * 8);
  int32_t* order = (int32_t*)w;
  w += al((size_t)N * 4);
  int32_t* choices = (int32_t*)w;
  w += al((size_t)m * k * 4);
  int32_t* acc = (int32_t*)w;
  w += al((size_t)m * 4);
  double* subq = (double*)w;
  w += al((size_t)m * k * k * 8);
  uint64_t* subsol = (uint64_t*)w;

  rc = check_dev(ctx);
  if (rc) return rc;
  Dev g(ctx_device(ctx));
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = clk::now();
  hipError_t e = enqueue_impact(N, Q, x, imp, field, mode == QAOA_DECOMP_GIVEN ? nullptr : order,
                                energy, s);
  if (e != hipSuccess) return hip_error(e, "impact kernels");
  if (mode == QAOA_DECOMP_IFD) {
    hipLaunchKernelGGL(windows_kernel, dim3(m), dim3(64), 0, s, N, order, k, (long long)stride,
                       choices);
  } else if (mode == QAOA_DECOMP_BFS) {
    hipLaunchKernelGGL(traverse_kernel<false>, dim3(m), dim3(256), 0, s, N, Q, imp, order, k,
                       choices);
  } else if (mode == QAOA_DECOMP_PFS) {
    hipLaunchKernelGGL(traverse_kernel<true>, dim3(m), dim3(256), 0, s, N, Q, imp, order, k,
                       choices);
  } else {
    e = hipMemcpyAsync(choices, choices_in, (size_t)m * k * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_error(e, "choices copy");
  }
  hipLaunchKernelGGL(gather_kernel, dim3(m), dim3(256), 0, s, N, Q, k, choices, subq);
  std::vector<double> hq((size_t)m * k * k);
  e = hipMemcpyAsync(hq.data(), subq, hq.size() * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "decomposition");
  const auto t1 = clk::now();

  // the sub-QUBO solves: every window through the queue, best samples back
  std::vector<uint64_t> tickets;
  std::vector<uint64_t> best(m, 0);
  tickets.reserve(m);
  size_t next_wait = 0;
  auto wait_one = [&](size_t i) -> int {
    qaoa_solve_result r;
    int wr = qaoa_wait(q, tickets[i], -1, &r, nullptr);
    if (wr != QAOA_OK) return wr;
    if (r.status != QAOA_OK) return set_error(r.status, "sub-QUBO solve %zu failed", i);
    best[i] = r.best_z;
    return QAOA_OK;
  };
  for (int t = 0; t < m; ++t) {
    qaoa_solve_req req;
    req.n = k;
    req.Q = hq.data() + (size_t)t * k * k;
    req.gamma0 = gamma0;
    req.beta0 = beta0;
    req.seed = seed + (uint64_t)t;
    uint64_t tk = 0;
    for (;;) {
      int sr = qaoa_submit(q, &req, &tk);
      if (sr == QAOA_OK) break;
      if (sr != QAOA_ERR_QUEUE_FULL || next_wait >= tickets.size()) {
        for (size_t i = next_wait; i < tickets.size(); ++i) (void)qaoa_cancel(q, tickets[i]);
        return sr;
      }
      int wr = wait_one(next_wait++);
      if (wr != QAOA_OK) return wr;
    }
    tickets.push_back(tk);
  }
  for (; next_wait < tickets.size(); ++next_wait) {
    int wr = wait_one(next_wait);
    if (wr != QAOA_OK) {
      for (size_t i = next_wait + 1; i < tickets.size(); ++i) (void)qaoa_cancel(q, tickets[i]);
      return wr;
    }
  }
  const auto t2 = clk::now();

  e = hipMemcpyAsync(subsol, best.data(), (size_t)m * 8, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_error(e, "sub-solution copy");
  hipLaunchKernelGGL(aggregate_kernel, dim3(1), dim3(1024), 0, s, N, Q, x, field, energy, m, k,
                     choices, subsol, acc);
  std::vector<int32_t> hacc(m);
  double he = 0.0;
  e = hipMemcpyAsync(hacc.data(), acc, (size_t)m * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&he, energy, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "aggregation");
  const auto t3 = clk::now();
  if (stats) {
    auto ms = [](clk::duration d) { return std::chrono::duration<double, std::milli>(d).count(); };
    stats->decompose_ms = ms(t1 - t0);
    stats->solve_ms = ms(t2 - t1);
    stats->aggregate_ms = ms(t3 - t2);
    int na = 0;
    for (int v : hacc) na += v == 1;
    stats->accepted = na;
    stats->energy = he;
  }
  return QAOA_OK;
}

}  // extern "C"
