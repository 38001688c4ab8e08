// Whole-state evaluation and adjoint gradient of small states in one launch
// (gfx950): evaluation up to n = 14 (complex64) or 13 (complex128), the
// gradient up to n = 13 (complex64) or 12 (complex128).
//
// A state of 2^n amplitudes fits the registers of one work-group: thread t of
// T = 2^min(n, 8) threads holds amplitudes z = t + 256 r, r < 2^(n - 8), so
// qubits 0..5 are lane bits, 6..7 wave bits and 8.. register bits.  One
// launch folds Q, forms C(z) in FP64, applies the p layers of Eq. (2) of the
// paper (phase e^{-i gamma C(z)}, then the mixer e^{+i beta X} on every
// qubit) and reduces <C> and the norm (Eq. (1)) in FP64, writing the outputs
// directly: there is no separate fold or reduction launch and no scratch.
// Up to 16 amplitudes per thread keep C(z) per amplitude in registers; with
// 32 or 64 a thread keeps its base value and register-bit fields and forms
// C(z) at each use, with the couplings among register bits from a table in
// LDS shared by all threads.
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

// With 32 or 64 amplitudes per thread, loops over them issue at most `every`
// amplitudes' loads, shuffles or phase factors ahead of their use (otherwise
// the scheduler front-loads all of them and the registers overflow).
template <int NR, int every>
__device__ __forceinline__ void small_fence(int r) {
  if constexpr (NR >= 5)
    if ((r & (every - 1)) == every - 1) __builtin_amdgcn_sched_barrier(0);
}

// c a + i s b
template <class V, class S>
__device__ __forceinline__ V mix1(V a, V b, S c, S s) {
  V r;
  r.x = fma(c, a.x, -s * b.y);
  r.y = fma(c, a.y, s * b.x);
  return r;
}

// LDS: the folded Q, per-layer (gamma / 2 pi, cos beta, sin beta), the
// reduction slots (and, for the gradient, per-layer per-wave sums), the
// register-bit coupling table for more than 4 register bits, then the
// amplitudes (psi, and lambda for the gradient) when there are wave qubits.
__host__ __device__ inline size_t small_ktab(int n) { return n > 12 ? (size_t)1 << (n - 8) : 0; }
__host__ __device__ inline size_t small_head(int n, int p, int grad) {
  const size_t head =
      ((size_t)n * n + 3 * (size_t)p + 8 + (grad ? 8 * (size_t)p : 0) + small_ktab(n)) * 8;
  return (head + 15) & ~(size_t)15;
}
__device__ inline double* small_kptr(double* Wsh, int n, int p, int grad) {
  return Wsh + n * n + 3 * p + 8 + (grad ? 8 * p : 0);
}

// C(z) of a thread's amplitudes z = t + 256 r, by r.
template <int NR, bool STORED = (NR <= 4)>
struct SmallCost {
  double c[1 << NR];
  __device__ __forceinline__ double operator[](int r) const { return c[r]; }
  __device__ __forceinline__ void refresh() {}
};
template <int NR>
struct SmallCost<NR, false> {
  double base;       // the thread's low bits alone
  double f[NR];      // register bit k's field: W_kk plus its couplings to the low bits
  const double* K;   // LDS [2^NR]: couplings among the register bits set in r
  // Called once per layer: the parts pass through an empty asm statement so
  // that the compiler cannot hoist the 2^NR values out of the layer loop
  // (which would hold them all in registers again).
  __device__ __forceinline__ void refresh() {
    asm volatile("" : "+v"(base));
#pragma unroll
    for (int k = 0; k < NR; ++k) asm volatile("" : "+v"(f[k]));
  }
  __device__ __forceinline__ double operator[](int r) const {
    double x = base + K[r];
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if ((r >> k) & 1) x += f[k];
    return x;
  }
};
template <class V>
size_t small_lds(int n, int p, int grad) {
  return small_head(n, p, grad) + (n > 6 ? ((size_t)1 << n) * sizeof(V) * (grad ? 2 : 1) : 0);
}

// Folds Q into LDS (W_ii = Q_ii, W_ij = Q_ij + Q_ji, so that C(z) =
// sum_i W_ii z_i + sum_{i<j} W_ij z_i z_j), stages (gamma / 2 pi, cos beta,
// sin beta) per layer and forms C(z) of the thread's amplitudes (FP64), or
// its parts and the register-bit table Ksh.
template <int NR>
__device__ __forceinline__ void small_setup(const SmallArgs& A, double* Wsh, double* cs,
                                            double* Ksh, SmallCost<NR>& C) {
  constexpr int NAMP = 1 << NR;
  const int n = A.n, p = A.p, T = blockDim.x, tid = threadIdx.x;
  const uint64_t st = blockIdx.x;
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
  // the low bits (the thread index; unrolled over 8 so that the LDS reads
  // issue together), the register bits' fields from them, and the couplings
  // among register bits
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
  if constexpr (NR <= 4) {
    (void)Ksh;
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
      C.c[r] = c;
    }
  } else {
    if (tid < NAMP) {
      double x = 0.0;
      for (int k = 1; k < NR; ++k)
        if ((tid >> k) & 1)
          for (int k2 = 0; k2 < k; ++k2)
            if ((tid >> k2) & 1) x += Wsh[(8 + k) * n + 8 + k2];
      Ksh[tid] = x;
    }
    C.base = cbase;
#pragma unroll
    for (int k = 0; k < NR; ++k) C.f[k] = f[k];
    C.K = Ksh;
    __syncthreads();
  }
}

// The p layers from |+>: phase e^{-i gamma C(z)}, then the mixer on every
// qubit.
template <class V, int NR>
__device__ __forceinline__ void small_layers(V (&v)[1 << NR], SmallCost<NR>& C,
                                             const double* cs, V* buf, int n, int p) {
  using S = typename std::conditional<sizeof(V) == 8, float, double>::type;
  constexpr int NAMP = 1 << NR;
  const int tid = threadIdx.x;
  const double a0 = exp2(-0.5 * (double)n);
#pragma unroll
  for (int r = 0; r < NAMP; ++r) v[r] = mkv<V>(a0, 0.0);
  const int nl = n < 6 ? n : 6, nw = n <= 6 ? 0 : (n == 7 ? 1 : 2);
  for (int j = 0; j < p; ++j) {
    const double gp = cs[3 * j];
    const S c = (S)cs[3 * j + 1], s = (S)cs[3 * j + 2];
    C.refresh();
#pragma unroll
    for (int r = 0; r < NAMP; ++r) {
      v[r] = cmul(v[r], unitv<V>(gp * C[r]));
      small_fence<NR, 4>(r);
    }
    for (int q = 0; q < nl; ++q) {
#pragma unroll
      for (int r = 0; r < NAMP; ++r) {
        v[r] = mix1(v[r], shfl_xor_v(v[r], 1 << q), c, s);
        small_fence<NR, 8>(r);
      }
    }
    if (nw) {
      // amplitude z = t + 256 r of thread t at buf[z]; a partner across the
      // wave bits is the same r of thread t ^ 64, t ^ 128 or t ^ 192, read
      // from a per-partner base at the immediate offset 256 r
      const V* const p6 = buf + (tid ^ 64);
      const V* const p7 = buf + (tid ^ 128);
      const V* const p67 = buf + (tid ^ 192);
#pragma unroll
      for (int r = 0; r < NAMP; ++r) buf[tid + (r << 8)] = v[r];
      __syncthreads();
      if (nw == 1) {
#pragma unroll
        for (int r = 0; r < NAMP; ++r) {
          v[r] = mix1(v[r], p6[r << 8], c, s);
          small_fence<NR, 8>(r);
        }
      } else {
        const S cc = c * c, ss = s * s, sc = s * c;
#pragma unroll
        for (int r = 0; r < NAMP; ++r) {
          const V b6 = p6[r << 8], b7 = p7[r << 8], b67 = p67[r << 8];
          const S ux = b6.x + b7.x, uy = b6.y + b7.y;
          V o;
          o.x = fma(cc, v[r].x, fma(-sc, uy, -ss * b67.x));
          o.y = fma(cc, v[r].y, fma(sc, ux, -ss * b67.y));
          v[r] = o;
          small_fence<NR, 4>(r);
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
}

// Sum of x over the work-group's threads into red[] (one slot per wave),
// returned on thread 0.
__device__ __forceinline__ double small_sum(double x, double* red) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int wl = T < 64 ? T : 64;
  for (int off = wl >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = x;
  __syncthreads();
  double sum = 0.0;
  if (tid == 0)
    for (int w = 0; w < (T + 63) / 64; ++w) sum += red[w];
  __syncthreads();
  return sum;
}

template <class V, int NR>
__global__ void __launch_bounds__(256) small_kernel(SmallArgs A) {
  using S = typename std::conditional<sizeof(V) == 8, float, double>::type;
  constexpr int NAMP = 1 << NR;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = A.n, p = A.p, tid = threadIdx.x;
  const uint64_t st = blockIdx.x;
  double* const Wsh = reinterpret_cast<double*>(smem);
  double* const cs = Wsh + n * n;
  double* const red = cs + 3 * p;
  V* const buf = reinterpret_cast<V*>(smem + small_head(n, p, 0));
  SmallCost<NR> C;
  small_setup<NR>(A, Wsh, cs, small_kptr(Wsh, n, p, 0), C);
  V v[NAMP];
  small_layers<V, NR>(v, C, cs, buf, n, p);

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
  const double se = small_sum(ae, red), sn = small_sum(an, red + 4);
  if (tid == 0) {
    A.expect[st] = se;
    if (A.norm) A.norm[st] = sn;
  }
}

// The adjoint gradient of <C> (Eq. (1)) with respect to every gamma_j and
// beta_j of Eq. (2): the forward layers, lambda = C psi, then for j = p..1
// the mixer undone on psi and lambda with d<C>/dbeta_j = -2 sum_q Im
// <lambda| X_q |psi> taken from the partner amplitudes each qubit's undo
// fetches (X_q commutes with the layer's mixer, so any point of its undo
// gives the same value), d<C>/dgamma_j = 2 Im <lambda| C |psi> where the
// phase was applied, and the phase undone.  FP64 sums; the per-layer sums
// of each wave go to LDS and are added at the end.
template <class V, int NR>
__global__ void __launch_bounds__(256) small_grad_kernel(SmallArgs A, double* dgamma,
                                                        double* dbeta) {
  using S = typename std::conditional<sizeof(V) == 8, float, double>::type;
  constexpr int NAMP = 1 << NR;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = A.n, p = A.p, T = blockDim.x, tid = threadIdx.x;
  const int wave = tid >> 6, nwaves = (T + 63) / 64;
  const uint64_t st = blockIdx.x;
  double* const Wsh = reinterpret_cast<double*>(smem);
  double* const cs = Wsh + n * n;
  double* const red = cs + 3 * p;
  double* const acc = red + 8;  // [2p][4]: per layer and wave, dgamma then dbeta sums
  V* const buf = reinterpret_cast<V*>(smem + small_head(n, p, 1));
  V* const bufl = buf + (n > 6 ? (1 << n) : 0);
  SmallCost<NR> C;
  small_setup<NR>(A, Wsh, cs, small_kptr(Wsh, n, p, 1), C);
  V v[NAMP], l[NAMP];
  small_layers<V, NR>(v, C, cs, buf, n, p);
  double ae = 0.0;
#pragma unroll
  for (int r = 0; r < NAMP; ++r) {
    ae = fma((double)v[r].x * v[r].x + (double)v[r].y * v[r].y, C[r], ae);
    const S cz = (S)C[r];
    l[r] = mkv<V>(cz * v[r].x, cz * v[r].y);
  }
  // Im(conj(a) b)
  auto imc = [](V a, V b) { return (double)a.x * b.y - (double)a.y * b.x; };
  const int nl = n < 6 ? n : 6, nw = n <= 6 ? 0 : (n == 7 ? 1 : 2);
  for (int j = p - 1; j >= 0; --j) {
    const double gp = cs[3 * j];
    const S c = (S)cs[3 * j + 1], s = (S)cs[3 * j + 2];
    C.refresh();
    double xb = 0.0;  // sum_q Im <lambda| X_q |psi>
    // the mixer undone: e^{-i beta X} = c - i s X per qubit
    for (int q = 0; q < nl; ++q) {
#pragma unroll
      for (int r = 0; r < NAMP; ++r) {
        const V vp = shfl_xor_v(v[r], 1 << q), lp = shfl_xor_v(l[r], 1 << q);
        xb += imc(l[r], vp);
        v[r] = mix1(v[r], vp, c, (S)-s);
        l[r] = mix1(l[r], lp, c, (S)-s);
        // bound the shuffles in flight (each holds two partner amplitudes)
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (nw) {
      // partners across the wave bits as in small_layers, for psi and lambda
      const V* const p6 = buf + (tid ^ 64);
      const V* const p7 = buf + (tid ^ 128);
      const V* const p67 = buf + (tid ^ 192);
      const V* const q6 = bufl + (tid ^ 64);
      const V* const q7 = bufl + (tid ^ 128);
      const V* const q67 = bufl + (tid ^ 192);
#pragma unroll
      for (int r = 0; r < NAMP; ++r) {
        buf[tid + (r << 8)] = v[r];
        bufl[tid + (r << 8)] = l[r];
      }
      __syncthreads();
      if (nw == 1) {
#pragma unroll
        for (int r = 0; r < NAMP; ++r) {
          const V vp = p6[r << 8], lp = q6[r << 8];
          xb += imc(l[r], vp);
          v[r] = mix1(v[r], vp, c, (S)-s);
          l[r] = mix1(l[r], lp, c, (S)-s);
        }
      } else {
        // (c - i s X) (x) (c - i s X): c^2 a - i c s (a6 + a7) - s^2 a67
        const S cc = c * c, ss = s * s, sc = s * c;
        auto undo2 = [&](V a, V b6, V b7, V b67) {
          const S ux = b6.x + b7.x, uy = b6.y + b7.y;
          V o;
          o.x = fma(cc, a.x, fma(sc, uy, -ss * b67.x));
          o.y = fma(cc, a.y, fma(-sc, ux, -ss * b67.y));
          return o;
        };
#pragma unroll
        for (int r = 0; r < NAMP; ++r) {
          const V v6 = p6[r << 8], v7 = p7[r << 8], v67 = p67[r << 8];
          const V l6 = q6[r << 8], l7 = q7[r << 8], l67 = q67[r << 8];
          xb += imc(l[r], v6) + imc(l[r], v7);
          v[r] = undo2(v[r], v6, v7, v67);
          l[r] = undo2(l[r], l6, l7, l67);
          if ((r & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
      for (int r = 0; r < NAMP; ++r)
        if (!((r >> k) & 1)) {
          const int r1 = r | (1 << k);
          xb += imc(l[r], v[r1]) + imc(l[r1], v[r]);
          const V v0 = v[r], v1 = v[r1], l0 = l[r], l1 = l[r1];
          v[r] = mix1(v0, v1, c, (S)-s);
          v[r1] = mix1(v1, v0, c, (S)-s);
          l[r] = mix1(l0, l1, c, (S)-s);
          l[r1] = mix1(l1, l0, c, (S)-s);
        }
    // 2 Im <lambda| C |psi> where the phase was applied, then the phase undone
    double xg = 0.0;
#pragma unroll
    for (int r = 0; r < NAMP; ++r) {
      xg = fma(imc(l[r], v[r]), C[r], xg);
      const V u = unitv<V>(-gp * C[r]);
      v[r] = cmul(v[r], u);
      l[r] = cmul(l[r], u);
      small_fence<NR, 4>(r);
    }
    const int wl = T < 64 ? T : 64;
    for (int off = wl >> 1; off > 0; off >>= 1) {
      xg += __shfl_xor(xg, off, 64);
      xb += __shfl_xor(xb, off, 64);
    }
    if ((tid & 63) == 0) {
      acc[(2 * j) * 4 + wave] = xg;
      acc[(2 * j + 1) * 4 + wave] = xb;
    }
  }
  const double se = small_sum(ae, red);
  if (tid == 0 && A.expect) A.expect[st] = se;
  for (int j = tid; j < p; j += T) {
    double g = 0.0, b = 0.0;
    for (int w = 0; w < nwaves; ++w) {
      g += acc[(2 * j) * 4 + w];
      b += acc[(2 * j + 1) * 4 + w];
    }
    dgamma[st * p + j] = 2.0 * g;
    dbeta[st * p + j] = -2.0 * b;
  }
}

template <class V>
hipError_t launch_small_t(const SmallArgs& A, int nstates, double* dgamma, double* dbeta,
                          hipStream_t stream) {
  const int n = A.n;
  const bool grad = dgamma != nullptr;
  const dim3 grid((unsigned)nstates), blk(1u << (n < 8 ? n : 8));
  const size_t lds = small_lds<V>(n, A.p, grad ? 1 : 0);
  auto go = [&](auto kern, auto... args) -> hipError_t {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, blk, lds, stream, A, args...);
    return hipGetLastError();
  };
  constexpr bool c64 = sizeof(V) == 8;
#define DQ_S(NR)                                                              \
  return grad ? go(small_grad_kernel<V, NR>, dgamma, dbeta) : go(small_kernel<V, NR>)
  switch (n <= 8 ? 0 : n - 8) {
    case 0: DQ_S(0);
    case 1: DQ_S(1);
    case 2: DQ_S(2);
    case 3: DQ_S(3);
    case 4: DQ_S(4);
    case 5:
      // psi and lambda of a complex128 state would need 256 KiB of LDS
      if constexpr (c64) {
        DQ_S(5);
      } else {
        if (grad) return hipErrorInvalidValue;
        return go(small_kernel<V, 5>);
      }
    case 6:
      if constexpr (c64) {
        if (grad) return hipErrorInvalidValue;
        return go(small_kernel<V, 6>);
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
#undef DQ_S
}

bool small_args_ok(int n, int nmax, int p, int S, int nstates, const double* Q,
                   const double* gammas, const double* betas) {
  return n >= 1 && n <= nmax && p >= 1 && p <= 64 && S >= 1 && nstates >= 1 && Q && gammas &&
         betas;
}

}  // namespace

hipError_t launch_small_expect(int prec, int n, int p, int S, int nstates, const double* Q,
                               const double* gammas, const double* betas, double* expect,
                               double* norm, void* probs, void* psi, hipStream_t stream) {
  if (!small_args_ok(n, small_fwd_nmax(prec), p, S, nstates, Q, gammas, betas) || !expect)
    return hipErrorInvalidValue;
  SmallArgs A{n, p, S, Q, gammas, betas, expect, norm, probs, psi};
  return prec == QAOA_C64 ? launch_small_t<float2>(A, nstates, nullptr, nullptr, stream)
                          : launch_small_t<double2>(A, nstates, nullptr, nullptr, stream);
}

hipError_t launch_small_grad(int prec, int n, int p, int S, int nstates, const double* Q,
                             const double* gammas, const double* betas, double* expect,
                             double* dgamma, double* dbeta, hipStream_t stream) {
  if (!small_args_ok(n, small_grad_nmax(prec), p, S, nstates, Q, gammas, betas) || !dgamma ||
      !dbeta)
    return hipErrorInvalidValue;
  SmallArgs A{n, p, S, Q, gammas, betas, expect, nullptr, nullptr, nullptr};
  return prec == QAOA_C64 ? launch_small_t<float2>(A, nstates, dgamma, dbeta, stream)
                          : launch_small_t<double2>(A, nstates, dgamma, dbeta, stream);
}

}  // namespace dq
