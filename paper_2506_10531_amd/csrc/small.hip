// Whole-state evaluation of small states (n <= 12) in one launch (gfx950).
//
// A state of 2^n amplitudes fits the registers of one work-group: thread t of
// T = 2^min(n, 8) threads holds amplitudes z = t + 256 r, r < 2^(n - 8), so
// qubits 0..5 are lane bits, 6..7 wave bits and 8.. register bits.  One
// launch folds Q, forms each amplitude's C(z) once in FP64, applies the p
// layers of Eq. (2) of the paper (phase e^{-i gamma C(z)}, then the mixer
// e^{+i beta X} on every qubit) and reduces <C> and the norm (Eq. (1)) in
// FP64, writing the outputs directly: there are no tables, no separate fold
// or reduction launch and no scratch.
//
// The mixer acts per qubit as (a, b) -> (c a + i s b, i s a + c b), c = cos
// beta, s = sin beta: a lane qubit takes its partner amplitude by a lane
// shuffle, the two wave qubits are mixed together through LDS (one exchange
// per layer: the amplitude becomes c^2 a + i c s (a6 + a7) - s^2 a67 from its
// three partners), and the register qubits are butterflies inside a thread.
#include "regtile.h"
#include "../../include/dqaoa.h"

#include <type_traits>

namespace dq {
namespace {

using namespace rt;

struct SmallArgs {
  int n, p, S;
  const double* Q;       // [B][n][n]
  const double* gammas;  // [B*S][p]
  const double* betas;
  double* expect;  // [B*S]
  double* norm;    // nullable
  void* probs;     // nullable [B*S][2^n], state precision
  void* psi;       // nullable [B*S][2^n]
};

template <class V>
__device__ __forceinline__ V shfl_xor_v(V x, int m) {
  V r;
  r.x = __shfl_xor(x.x, m, 64);
  r.y = __shfl_xor(x.y, m, 64);
  return r;
}

// c a + i s b
template <class V, class S>
__device__ __forceinline__ V mix1(V a, V b, S c, S s) {
  V r;
  r.x = fma(c, a.x, -s * b.y);
  r.y = fma(c, a.y, s * b.x);
  return r;
}

// LDS bytes: folded Q, per-layer (gamma / 2 pi, cos beta, sin beta), the
// reduction slots, and the amplitudes when there are wave qubits.
template <class V>
size_t small_lds(int n, int p) {
  const size_t head = ((size_t)n * n + 3 * (size_t)p + 8) * sizeof(double);
  const size_t h16 = (head + 15) & ~(size_t)15;
  return h16 + (n > 6 ? ((size_t)1 << n) * sizeof(V) : 0);
}

template <class V, int NR>
__global__ void __launch_bounds__(256) small_kernel(SmallArgs A) {
  using S = typename std::conditional<sizeof(V) == 8, float, double>::type;
  constexpr int NAMP = 1 << NR;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = A.n, p = A.p;
  const int T = blockDim.x, tid = threadIdx.x;
  const uint64_t st = blockIdx.x;
  double* const Wsh = reinterpret_cast<double*>(smem);
  double* const cs = Wsh + n * n;
  double* const red = cs + 3 * p;
  const size_t head = ((size_t)n * n + 3 * (size_t)p + 8) * sizeof(double);
  V* const buf = reinterpret_cast<V*>(smem + ((head + 15) & ~(size_t)15));

  // W_ii = Q_ii, W_ij = Q_ij + Q_ji: C(z) = sum_i W_ii z_i + sum_{i<j} W_ij z_i z_j
  const double* Q = A.Q + (st / A.S) * n * n;
  for (int e = tid; e < n * n; e += T) {
    const int i = e / n, j = e - i * n;
    Wsh[e] = i == j ? Q[i * n + i] : Q[i * n + j] + Q[j * n + i];
  }
  for (int j = tid; j < p; j += T) {
    double s, c;
    sincos(A.betas[st * p + j], &s, &c);
    cs[3 * j] = A.gammas[st * p + j] * 0.15915494309189533577;
    cs[3 * j + 1] = c;
    cs[3 * j + 2] = s;
  }
  __syncthreads();

  // C(z) of this thread's amplitudes: the low bits (the thread index), the
  // register bits' fields from them, and the couplings among register bits
  // (unrolled over the 8 low bits, so that the LDS reads issue together)
  const int nb = n < 8 ? n : 8;
  double cbase = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < nb && ((tid >> i) & 1)) {
      cbase += Wsh[i * n + i];
#pragma unroll
      for (int j = 0; j < i; ++j)
        if ((tid >> j) & 1) cbase += Wsh[i * n + j];
    }
  double C[NAMP];
  {
    double f[NR > 0 ? NR : 1];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int i = 8 + k;
      double x = Wsh[i * n + i];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if ((tid >> j) & 1) x += Wsh[i * n + j];
      f[k] = x;
    }
#pragma unroll
    for (int r = 0; r < NAMP; ++r) {
      double c = cbase;
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if ((r >> k) & 1) {
          c += f[k];
#pragma unroll
          for (int k2 = 0; k2 < k; ++k2)
            if ((r >> k2) & 1) c += Wsh[(8 + k) * n + 8 + k2];
        }
      C[r] = c;
    }
  }

  V v[NAMP];
  const double a0 = exp2(-0.5 * (double)n);
#pragma unroll
  for (int r = 0; r < NAMP; ++r) v[r] = mkv<V>(a0, 0.0);
  const int nl = n < 6 ? n : 6, nw = n <= 6 ? 0 : (n == 7 ? 1 : 2);
  for (int j = 0; j < p; ++j) {
    const double gp = cs[3 * j];
    const S c = (S)cs[3 * j + 1], s = (S)cs[3 * j + 2];
#pragma unroll
    for (int r = 0; r < NAMP; ++r) v[r] = cmul(v[r], unitv<V>(gp * C[r]));
    for (int q = 0; q < nl; ++q) {
#pragma unroll
      for (int r = 0; r < NAMP; ++r) v[r] = mix1(v[r], shfl_xor_v(v[r], 1 << q), c, s);
    }
    if (nw) {
#pragma unroll
      for (int r = 0; r < NAMP; ++r) buf[(r << 8) | tid] = v[r];
      __syncthreads();
      if (nw == 1) {
#pragma unroll
        for (int r = 0; r < NAMP; ++r) v[r] = mix1(v[r], buf[((r << 8) | tid) ^ 64], c, s);
      } else {
        const S cc = c * c, ss = s * s, sc = s * c;
#pragma unroll
        for (int r = 0; r < NAMP; ++r) {
          const int z = (r << 8) | tid;
          const V b6 = buf[z ^ 64], b7 = buf[z ^ 128], b67 = buf[z ^ 192];
          const S ux = b6.x + b7.x, uy = b6.y + b7.y;
          V o;
          o.x = fma(cc, v[r].x, fma(-sc, uy, -ss * b67.x));
          o.y = fma(cc, v[r].y, fma(sc, ux, -ss * b67.y));
          v[r] = o;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
      for (int r = 0; r < NAMP; ++r)
        if (!((r >> k) & 1)) {
          const V x0 = v[r], x1 = v[r | (1 << k)];
          v[r] = mix1(x0, x1, c, s);
          v[r | (1 << k)] = mix1(x1, x0, c, s);
        }
  }

  // outputs: probabilities and state in the state precision, <C> and the
  // norm in FP64
  double ae = 0.0, an = 0.0;
  const uint64_t o = st << n;
#pragma unroll
  for (int r = 0; r < NAMP; ++r) {
    const double pz = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
    ae = fma(pz, C[r], ae);
    an += pz;
    const uint64_t z = o | (uint64_t)((r << 8) | tid);
    if (A.probs) static_cast<S*>(A.probs)[z] = (S)pz;
    if (A.psi) static_cast<V*>(A.psi)[z] = v[r];
  }
  const int wl = T < 64 ? T : 64;
  for (int off = wl >> 1; off > 0; off >>= 1) {
    ae += __shfl_xor(ae, off, 64);
    an += __shfl_xor(an, off, 64);
  }
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6)] = ae;
    red[2 * (tid >> 6) + 1] = an;
  }
  __syncthreads();
  if (tid == 0) {
    double se = 0.0, sn = 0.0;
    for (int w = 0; w < (T + 63) / 64; ++w) {
      se += red[2 * w];
      sn += red[2 * w + 1];
    }
    A.expect[st] = se;
    if (A.norm) A.norm[st] = sn;
  }
}

template <class V>
hipError_t launch_small_t(const SmallArgs& A, int nstates, hipStream_t stream) {
  const int n = A.n;
  const dim3 grid((unsigned)nstates), blk(1u << (n < 8 ? n : 8));
  const size_t lds = small_lds<V>(n, A.p);
#define DQ_S(NR)                                                                        \
  do {                                                                                  \
    if (lds > 65536) {                                                                  \
      hipError_t e = hipFuncSetAttribute((const void*)small_kernel<V, NR>,              \
                                         hipFuncAttributeMaxDynamicSharedMemorySize,    \
                                         (int)lds);                                     \
      if (e != hipSuccess) return e;                                                    \
    }                                                                                   \
    hipLaunchKernelGGL((small_kernel<V, NR>), grid, blk, lds, stream, A);               \
  } while (0)
  switch (n <= 8 ? 0 : n - 8) {
    case 0: DQ_S(0); break;
    case 1: DQ_S(1); break;
    case 2: DQ_S(2); break;
    case 3: DQ_S(3); break;
    default: DQ_S(4); break;
  }
#undef DQ_S
  return hipGetLastError();
}

}  // namespace

hipError_t launch_small_expect(int prec, int n, int p, int S, int nstates, const double* Q,
                               const double* gammas, const double* betas, double* expect,
                               double* norm, void* probs, void* psi, hipStream_t stream) {
  if (n < 1 || n > SMALL_NMAX || p < 1 || p > 64 || S < 1 || nstates < 1 || !Q || !gammas ||
      !betas || !expect)
    return hipErrorInvalidValue;
  SmallArgs A{n, p, S, Q, gammas, betas, expect, norm, probs, psi};
  return prec == QAOA_C64 ? launch_small_t<float2>(A, nstates, stream)
                          : launch_small_t<double2>(A, nstates, stream);
}

}  // namespace dq
