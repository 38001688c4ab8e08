// gfx950 kernels for the QAOA state-vector path (arXiv 2506.10531, Sec. IV,
// Eq. (2)): per-layer cost phase e^{-i gamma C(z)} and mixer e^{+i beta X} on
// every qubit, <C> and norm reductions, the adjoint gradient, CDF sampling and
// the Adam update.
//
// Execution model.  A state of 2^n amplitudes is processed in tiles of 2^k
// amplitudes held in LDS (k <= 14 for complex64, <= 13 for complex128: 128 KiB
// of the 160 KiB per CU).  A tile is a set of k qubits; the butterflies of all
// of them run inside the tile, so one read + one write of the state per pass
// covers a whole set of qubits.  Because the mixer factors of one layer
// commute, a layer's mixer is split into qubit sets, and the pass that
// finishes layer j on a set also applies the (diagonal) phase of layer j+1 and
// starts layer j+1 on the same set: p layers over two sets take p+1 passes, a
// read and a write of the state per layer.  Inside a tile, each "round"
// gathers 2^R amplitudes that differ in R adjacent tile qubits into registers
// (R = 4 for complex64, 3 for complex128), applies the fused phase / the R
// butterflies / reductions, and scatters them back; the LDS layout is XOR
// swizzled so that every round's gather is bank-conflict free.
//
// The cost C(z) of an amplitude is never stored: per tile the field of the
// block (non-tile) bits on every tile qubit and the block's own energy are
// formed once in LDS; per round each thread forms the energy of its fixed
// tile bits and the field on its R round qubits; the 2^R energies follow by
// adding the in-group couplings.  All of it is FP64.  The phase angle
// gamma*C/(2 pi) is range-reduced in FP64 to [-1/2, 1/2] revolutions before a
// sincospi in the state precision.
#include "internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace dq {
namespace {

template <typename T>
struct Cx;
template <>
struct Cx<float> {
  using V = float2;
  static constexpr int RB = 4;  // round qubits; also the swizzle width
};
template <>
struct Cx<double> {
  using V = double2;
  static constexpr int RB = 3;
};

constexpr int KMAX = 14;
constexpr int NT_MAX = 512;

// XOR swizzle of the LDS slot of local index l: the low RB bits are XORed
// with the next RB bits.  A bijection on [0, 2^k) for any k.
template <typename T>
__device__ __forceinline__ uint32_t swz(uint32_t l) {
  constexpr int s = Cx<T>::RB;
  return l ^ ((l >> s) & ((1u << s) - 1u));
}

// ---- tile geometry ----------------------------------------------------------

__device__ __forceinline__ uint64_t dep_local(uint32_t l, const PassDesc& d) {
  if (d.c >= d.k) return l;
  return (uint64_t)(l & ((1u << d.c) - 1u)) | ((uint64_t)(l >> d.c) << d.a);
}

__device__ __forceinline__ uint64_t dep_block(uint64_t b, const PassDesc& d) {
  if (d.c >= d.k) return b << d.k;
  const int gap = d.a - d.c;  // block bits [c, a)
  const uint64_t lo = b & ((1ull << gap) - 1ull);
  const uint64_t hi = b >> gap;  // block bits [a + k - c, n)
  return (lo << d.c) | (hi << (d.a + d.k - d.c));
}

__device__ __forceinline__ int lpos(int i, const PassDesc& d) {
  return (d.c >= d.k || i < d.c) ? i : d.a + (i - d.c);
}

// Per-tile cost context in LDS.  fl[i] = h_i + sum_{j in block} W_ij z_j for
// tile qubit i; Wl = couplings among tile qubits (zero diagonal); cblk = the
// energy of the block bits alone.
struct TileCtx {
  double cblk;
  double fl[KMAX];
  double Wl[KMAX * KMAX];
};

__device__ void tile_setup(TileCtx* tc, double* tmp, const double* W,
                           const PassDesc& d, uint64_t zb) {
  const int tid = threadIdx.x, n = d.n, k = d.k;
  if (tid < k) {
    const int pi = lpos(tid, d);
    double f = W[pi * n + pi];
    for (int j = 0; j < n; ++j)
      if ((zb >> j) & 1ull) f += W[pi * n + j];
    tc->fl[tid] = f;
  }
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e - i * k;
    tc->Wl[e] = (i == j) ? 0.0 : W[lpos(i, d) * n + lpos(j, d)];
  }
  if (tid < n) {
    double t = 0.0;
    if ((zb >> tid) & 1ull) {
      t = W[tid * n + tid];
      for (int j = 0; j < tid; ++j)
        if ((zb >> j) & 1ull) t += W[tid * n + j];
    }
    tmp[tid] = t;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += tmp[i];
    tc->cblk = s;
  }
  __syncthreads();
}

// Energies C of the 2^R amplitudes l0 | (v << g0), v < 2^R (l0 has the R
// group bits clear), relative to the tile context.
template <int R>
__device__ __forceinline__ void group_cost(uint32_t l0, int k, int g0,
                                           const TileCtx* tc, double* Cv) {
  double cf = tc->cblk;
  for (int i = 0; i < k; ++i) {
    if ((l0 >> i) & 1u) {
      double r = tc->fl[i];
      for (int j = 0; j < i; ++j)
        if ((l0 >> j) & 1u) r += tc->Wl[i * k + j];
      cf += r;
    }
  }
  double g[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = g0 + q;
    double r = tc->fl[i];
    for (int j = 0; j < k; ++j)
      if ((l0 >> j) & 1u) r += tc->Wl[i * k + j];
    g[q] = r;
  }
  double w[R][R];
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int q2 = 0; q2 < q; ++q2) w[q][q2] = tc->Wl[(g0 + q) * k + g0 + q2];
#pragma unroll
  for (int v = 0; v < (1 << R); ++v) {
    double s = cf;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if ((v >> q) & 1) {
        s += g[q];
#pragma unroll
        for (int q2 = 0; q2 < q; ++q2)
          if ((v >> q2) & 1) s += w[q][q2];
      }
    }
    Cv[v] = s;
  }
}

// a <- a * e^{-i 2 pi rev}, rev already reduced to [-1/2, 1/2].
__device__ __forceinline__ void rot(float2& a, double rev) {
  float s, c;
  sincospif(2.0f * (float)rev, &s, &c);
  const float x = a.x, y = a.y;
  a.x = fmaf(x, c, y * s);
  a.y = fmaf(y, c, -x * s);
}
__device__ __forceinline__ void rot(double2& a, double rev) {
  double s, c;
  sincospi(2.0 * rev, &s, &c);
  const double x = a.x, y = a.y;
  a.x = fma(x, c, y * s);
  a.y = fma(y, c, -x * s);
}

// a <- a * e^{-i 2 pi rev} and b <- b * e^{-i 2 pi rev} with one sincos.
__device__ __forceinline__ void rot2(float2& a, float2& b, double rev) {
  float s, c;
  sincospif(2.0f * (float)rev, &s, &c);
  const float x = a.x, y = a.y, u = b.x, w = b.y;
  a.x = fmaf(x, c, y * s);
  a.y = fmaf(y, c, -x * s);
  b.x = fmaf(u, c, w * s);
  b.y = fmaf(w, c, -u * s);
}
__device__ __forceinline__ void rot2(double2& a, double2& b, double rev) {
  double s, c;
  sincospi(2.0 * rev, &s, &c);
  const double x = a.x, y = a.y, u = b.x, w = b.y;
  a.x = fma(x, c, y * s);
  a.y = fma(y, c, -x * s);
  b.x = fma(u, c, w * s);
  b.y = fma(w, c, -u * s);
}

// Phase in revolutions for energy C, reduced in FP64.
__device__ __forceinline__ double phase_rev(double gp, double C) {
  const double t = gp * C;
  return t - rint(t);
}

// One butterfly of the mixer on the pair (a0, a1) (see LayerCoef).
template <int MODE, typename V, typename T>
__device__ __forceinline__ void bfly(V& a0, V& a1, T t) {
  const T x0 = a0.x, y0 = a0.y, x1 = a1.x, y1 = a1.y;
  if (MODE == 0) {
    a0.x = fma(-t, y1, x0);
    a0.y = fma(t, x1, y0);
    a1.x = fma(-t, y0, x1);
    a1.y = fma(t, x0, y1);
  } else {
    a0.x = fma(t, y0, x1);
    a0.y = fma(-t, x0, y1);
    a1.x = fma(t, y1, x0);
    a1.y = fma(-t, x1, y0);
  }
}

template <typename V, typename T>
__device__ __forceinline__ void cscale(V& a, T sr, T si) {
  const T x = a.x, y = a.y;
  a.x = x * sr - y * si;
  a.y = x * si + y * sr;
}

// Deterministic block sum (all threads receive the same value).
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Mixer scale sigma^m for m mixed qubits: c^m (mode 0) or (i s)^m (mode 1);
// `inv` gives the scale of the inverse mixer M(-beta).
__device__ __forceinline__ void mix_scale(const LayerCoef& L, int m, bool inv,
                                          double& sr, double& si) {
  double r = 1.0, i = 0.0;
  if (L.mode == 0) {
    for (int q = 0; q < m; ++q) r *= L.cb;
  } else {
    const double s = inv ? -L.sb : L.sb;
    for (int q = 0; q < m; ++q) {  // multiply by (i s)
      const double nr = -i * s, ni = r * s;
      r = nr;
      i = ni;
    }
  }
  sr = r;
  si = i;
}

// ---- forward round ------------------------------------------------------------

struct RoundOps {
  bool phase;    // apply the phase before the butterflies
  double gp;     // gamma / 2 pi
  bool scale;    // multiply by (sr, si) after the butterflies
  double sr, si;
  bool reduce;   // accumulate |a|^2 C and |a|^2 after the scale
  bool lambda;   // write C * a into the second tile after the scale
};

template <typename T, int R, int MODE>
__device__ void fwd_round(typename Cx<T>::V* tile, typename Cx<T>::V* lam,
                          int k, int g0, const TileCtx* tc, T t,
                          const RoundOps& o, double& ae, double& an) {
  using V = typename Cx<T>::V;
  const int nb = 1 << (k - R);
  const T sr = (T)o.sr, si = (T)o.si;
  for (int ob = threadIdx.x; ob < nb; ob += blockDim.x) {
    const uint32_t l0 =
        ((uint32_t)ob & ((1u << g0) - 1u)) | (((uint32_t)ob >> g0) << (g0 + R));
    V a[1 << R];
#pragma unroll
    for (int v = 0; v < (1 << R); ++v) a[v] = tile[swz<T>(l0 | ((uint32_t)v << g0))];
    double Cv[1 << R];
    if (o.phase || o.reduce || o.lambda) group_cost<R>(l0, k, g0, tc, Cv);
    if (o.phase) {
#pragma unroll
      for (int v = 0; v < (1 << R); ++v) rot(a[v], phase_rev(o.gp, Cv[v]));
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int v = 0; v < (1 << R); ++v)
        if (!((v >> q) & 1)) bfly<MODE>(a[v], a[v | (1 << q)], t);
    if (o.scale) {
#pragma unroll
      for (int v = 0; v < (1 << R); ++v) cscale(a[v], sr, si);
    }
    if (o.reduce) {
#pragma unroll
      for (int v = 0; v < (1 << R); ++v) {
        const double pz = (double)a[v].x * a[v].x + (double)a[v].y * a[v].y;
        ae = fma(pz, Cv[v], ae);
        an += pz;
      }
    }
#pragma unroll
    for (int v = 0; v < (1 << R); ++v) tile[swz<T>(l0 | ((uint32_t)v << g0))] = a[v];
    if (o.lambda) {
#pragma unroll
      for (int v = 0; v < (1 << R); ++v) {
        V b;
        b.x = (T)(Cv[v] * (double)a[v].x);
        b.y = (T)(Cv[v] * (double)a[v].y);
        lam[swz<T>(l0 | ((uint32_t)v << g0))] = b;
      }
    }
  }
}

template <typename T, int MODE>
__device__ void fwd_round_r(int r, typename Cx<T>::V* tile,
                            typename Cx<T>::V* lam, int k, int g0,
                            const TileCtx* tc, T t, const RoundOps& o,
                            double& ae, double& an) {
  if constexpr (Cx<T>::RB >= 4) {
    if (r == 4) return fwd_round<T, 4, MODE>(tile, lam, k, g0, tc, t, o, ae, an);
  }
  if (r == 3) fwd_round<T, 3, MODE>(tile, lam, k, g0, tc, t, o, ae, an);
  else if (r == 2) fwd_round<T, 2, MODE>(tile, lam, k, g0, tc, t, o, ae, an);
  else fwd_round<T, 1, MODE>(tile, lam, k, g0, tc, t, o, ae, an);
}

// One layer's mixer on the pass's qubit set [mixlo, k), optionally preceded
// by that layer's phase, optionally ending with the <C> reduction and the
// adjoint seed lambda = C psi.
template <typename T>
__device__ void fwd_mix(typename Cx<T>::V* tile, typename Cx<T>::V* lam,
                        const PassDesc& d, const TileCtx* tc,
                        const LayerCoef& L, bool phase, bool reduce,
                        bool lambda, double& ae, double& an) {
  constexpr int RB = Cx<T>::RB;
  double sr, si;
  mix_scale(L, d.k - d.mixlo, false, sr, si);
  const T t = (T)L.tb;
  for (int g0 = d.mixlo; g0 < d.k; g0 += RB) {
    const int r = min(RB, d.k - g0);
    const bool last = g0 + r >= d.k;
    RoundOps o;
    o.phase = phase && g0 == d.mixlo;
    o.gp = L.gp;
    o.scale = last;
    o.sr = sr;
    o.si = si;
    o.reduce = reduce && last;
    o.lambda = lambda && last;
    if (L.mode == 0) fwd_round_r<T, 0>(r, tile, lam, d.k, g0, tc, t, o, ae, an);
    else fwd_round_r<T, 1>(r, tile, lam, d.k, g0, tc, t, o, ae, an);
    __syncthreads();
  }
}

// The forward ops of a pass on one tile.
template <typename T>
__device__ void fwd_ops(typename Cx<T>::V* tile, typename Cx<T>::V* lam,
                        const PassDesc& d, const TileCtx* tc,
                        const LayerCoef* cf, bool reduce, bool lambda,
                        double& ae, double& an) {
  const bool has_ph = d.ja <= d.jb;
  if (d.lead >= 0)
    fwd_mix<T>(tile, lam, d, tc, cf[d.lead], false, reduce && !has_ph,
               lambda && !has_ph, ae, an);
  if (has_ph)
    for (int j = d.ja; j <= d.jb; ++j)
      fwd_mix<T>(tile, lam, d, tc, cf[j], true, reduce && j == d.jb,
                 lambda && j == d.jb, ae, an);
}

struct FwdArgs {
  PassDesc d;
  int S, p;
  const void* in;
  void* out;
  uint64_t stride;  // amplitudes between consecutive states
  const double* W;
  const LayerCoef* coef;
  double* part;  // [state][tile][2]
  void* probs;   // [state][2^n]
};

template <typename T>
__global__ void __launch_bounds__(NT_MAX) fwd_pass_kernel(FwdArgs A) {
  using V = typename Cx<T>::V;
  extern __shared__ __align__(16) unsigned char smem[];
  const PassDesc& d = A.d;
  V* tile = reinterpret_cast<V*>(smem);
  TileCtx* tc = reinterpret_cast<TileCtx*>(smem + (sizeof(V) << d.k));
  double* tmp = reinterpret_cast<double*>(tc + 1);  // [64]
  const int st = blockIdx.y;
  const uint64_t ti = blockIdx.x;
  const double* W = A.W + (size_t)(st / A.S) * d.n * d.n;
  const LayerCoef* cf = A.coef + (size_t)st * A.p;
  const uint64_t zb = dep_block(ti, d);
  tile_setup(tc, tmp, W, d, zb);

  const uint32_t nt = 1u << d.k;
  if (d.flags & F_INIT) {
    const T amp = (T)exp2(-0.5 * (double)d.n);
    V v0;
    v0.x = amp;
    v0.y = (T)0;
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x) tile[swz<T>(l)] = v0;
  } else {
    const V* gin = reinterpret_cast<const V*>(A.in) + (uint64_t)st * A.stride;
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x)
      tile[swz<T>(l)] = gin[zb | dep_local(l, d)];
  }
  __syncthreads();

  double ae = 0.0, an = 0.0;
  fwd_ops<T>(tile, nullptr, d, tc, cf, (d.flags & F_REDUCE) != 0, false, ae, an);

  if (d.flags & F_WRITE) {
    V* gout = reinterpret_cast<V*>(A.out) + (uint64_t)st * A.stride;
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x)
      gout[zb | dep_local(l, d)] = tile[swz<T>(l)];
  }
  if (d.flags & F_PROBS) {
    T* P = reinterpret_cast<T*>(A.probs) + ((uint64_t)st << d.n);
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x) {
      const V a = tile[swz<T>(l)];
      P[zb | dep_local(l, d)] = a.x * a.x + a.y * a.y;
    }
  }
  if (d.flags & F_REDUCE) {
    const double se = block_sum(ae, tmp);
    const double sn = block_sum(an, tmp);
    if (threadIdx.x == 0) {
      double* o = A.part + ((uint64_t)st * gridDim.x + ti) * 2;
      o[0] = se;
      o[1] = sn;
    }
  }
}

// ---- adjoint (backward) round ---------------------------------------------------

struct BwdRoundOps {
  bool xq;       // accumulate sum_q Im <lam|X_q|psi> over the round's qubits
  double xq_w;   // weight of this round's sum: the butterflies of earlier
                 // rounds left both tiles without their per-qubit scale
                 // (|c| or |s| per qubit), so the product lacks its square
  bool scale;    // multiply both tiles by (sr, si) after the butterflies
  double sr, si;
  bool phase;    // then accumulate Im <lam|C|psi> and undo the phase
  double gp;     // gamma / 2 pi of the phase being undone
};

template <typename T, int R, int MODE>
__device__ void bwd_round(typename Cx<T>::V* tp, typename Cx<T>::V* tl, int k,
                          int g0, const TileCtx* tc, T t,
                          const BwdRoundOps& o, double& ab, double& ag) {
  using V = typename Cx<T>::V;
  const int nb = 1 << (k - R);
  const T sr = (T)o.sr, si = (T)o.si;
  for (int ob = threadIdx.x; ob < nb; ob += blockDim.x) {
    const uint32_t l0 =
        ((uint32_t)ob & ((1u << g0) - 1u)) | (((uint32_t)ob >> g0) << (g0 + R));
    V a[1 << R], b[1 << R];
#pragma unroll
    for (int v = 0; v < (1 << R); ++v) {
      const uint32_t s = swz<T>(l0 | ((uint32_t)v << g0));
      a[v] = tp[s];
      b[v] = tl[s];
    }
    if (o.xq) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int v = 0; v < (1 << R); ++v) {
          const int u = v ^ (1 << q);
          // Im(conj(lam_v) psi_u) = lx*py - ly*px
          acc += (double)b[v].x * a[u].y - (double)b[v].y * a[u].x;
        }
      ab = fma(o.xq_w, acc, ab);
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int v = 0; v < (1 << R); ++v)
        if (!((v >> q) & 1)) {
          bfly<MODE>(a[v], a[v | (1 << q)], t);
          bfly<MODE>(b[v], b[v | (1 << q)], t);
        }
    if (o.scale) {
#pragma unroll
      for (int v = 0; v < (1 << R); ++v) {
        cscale(a[v], sr, si);
        cscale(b[v], sr, si);
      }
    }
    if (o.phase) {
      double Cv[1 << R];
      group_cost<R>(l0, k, g0, tc, Cv);
#pragma unroll
      for (int v = 0; v < (1 << R); ++v) {
        const double im = (double)b[v].x * a[v].y - (double)b[v].y * a[v].x;
        ag = fma(im, Cv[v], ag);
        rot2(a[v], b[v], phase_rev(-o.gp, Cv[v]));
      }
    }
#pragma unroll
    for (int v = 0; v < (1 << R); ++v) {
      const uint32_t s = swz<T>(l0 | ((uint32_t)v << g0));
      tp[s] = a[v];
      tl[s] = b[v];
    }
  }
}

template <typename T, int MODE>
__device__ void bwd_round_r(int r, typename Cx<T>::V* tp, typename Cx<T>::V* tl,
                            int k, int g0, const TileCtx* tc, T t,
                            const BwdRoundOps& o, double& ab, double& ag) {
  if constexpr (Cx<T>::RB >= 4) {
    if (r == 4) return bwd_round<T, 4, MODE>(tp, tl, k, g0, tc, t, o, ab, ag);
  }
  if (r == 3) bwd_round<T, 3, MODE>(tp, tl, k, g0, tc, t, o, ab, ag);
  else if (r == 2) bwd_round<T, 2, MODE>(tp, tl, k, g0, tc, t, o, ab, ag);
  else bwd_round<T, 1, MODE>(tp, tl, k, g0, tc, t, o, ab, ag);
}

// Undo layer j's mixer on the pass's qubit set (accumulating the set's part
// of d<C>/dbeta_j), then, if `phase`, accumulate d<C>/dgamma_j and undo the
// phase of layer j.  Results go to wsum[p + j] and wsum[j].
template <typename T>
__device__ void bwd_mix(typename Cx<T>::V* tp, typename Cx<T>::V* tl,
                        const PassDesc& d, const TileCtx* tc, const LayerCoef& L,
                        int j, int p, bool phase, double* wsum, double* red) {
  constexpr int RB = Cx<T>::RB;
  double sr, si;
  mix_scale(L, d.k - d.mixlo, true, sr, si);
  const T t = (T)(-L.tb);
  double ab = 0.0, ag = 0.0;
  const double q2 = L.mode == 0 ? L.cb * L.cb : L.sb * L.sb;
  double w = 1.0;
  for (int g0 = d.mixlo; g0 < d.k; g0 += RB) {
    const int r = min(RB, d.k - g0);
    const bool last = g0 + r >= d.k;
    BwdRoundOps o;
    o.xq = true;
    o.xq_w = w;
    for (int q = 0; q < r; ++q) w *= q2;
    o.scale = last;
    o.sr = sr;
    o.si = si;
    o.phase = phase && last;
    o.gp = L.gp;
    if (L.mode == 0) bwd_round_r<T, 0>(r, tp, tl, d.k, g0, tc, t, o, ab, ag);
    else bwd_round_r<T, 1>(r, tp, tl, d.k, g0, tc, t, o, ab, ag);
    __syncthreads();
  }
  const double sb = block_sum(ab, red);
  const double sg = phase ? block_sum(ag, red) : 0.0;
  if (threadIdx.x == 0) {
    wsum[p + j] += -2.0 * sb;
    if (phase) wsum[j] += 2.0 * sg;
  }
  __syncthreads();
}

struct BwdArgs {
  PassDesc d;
  int S, p;
  const void* psi;   // checkpoint read by this pass (unused with F_INIT)
  void* lam;         // adjoint state, read (unless F_LAMBDA) and written (F_WRITE)
  uint64_t stride;
  const double* W;
  const LayerCoef* coef;
  double* part;      // [state][rec][2p + 2]
  int rec_base;      // record of tile 0 of this pass
  int nrec;          // records per state
};

template <typename T>
__global__ void __launch_bounds__(NT_MAX) bwd_pass_kernel(BwdArgs A) {
  using V = typename Cx<T>::V;
  extern __shared__ __align__(16) unsigned char smem[];
  const PassDesc& d = A.d;
  const int p = A.p;
  V* tp = reinterpret_cast<V*>(smem);
  V* tl = tp + (1u << d.k);
  TileCtx* tc = reinterpret_cast<TileCtx*>(smem + 2 * (sizeof(V) << d.k));
  double* tmp = reinterpret_cast<double*>(tc + 1);  // [64]
  double* wsum = tmp + 64;                          // [2p + 2]
  const int st = blockIdx.y;
  const uint64_t ti = blockIdx.x;
  const double* W = A.W + (size_t)(st / A.S) * d.n * d.n;
  const LayerCoef* cf = A.coef + (size_t)st * p;
  const uint64_t zb = dep_block(ti, d);
  for (int q = threadIdx.x; q < 2 * p + 2; q += blockDim.x) wsum[q] = 0.0;
  tile_setup(tc, tmp, W, d, zb);

  const uint32_t nt = 1u << d.k;
  const V* gp_in = reinterpret_cast<const V*>(A.psi) + (uint64_t)st * A.stride;
  V* gl = reinterpret_cast<V*>(A.lam) + (uint64_t)st * A.stride;
  if (d.flags & F_INIT) {
    const T amp = (T)exp2(-0.5 * (double)d.n);
    V v0;
    v0.x = amp;
    v0.y = (T)0;
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x) tp[swz<T>(l)] = v0;
  } else {
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x)
      tp[swz<T>(l)] = gp_in[zb | dep_local(l, d)];
  }
  if (!(d.flags & F_LAMBDA)) {
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x)
      tl[swz<T>(l)] = gl[zb | dep_local(l, d)];
  }
  __syncthreads();

  if (d.flags & F_LAMBDA) {
    // Forward ops of this pass, <C> and norm, and lambda = C psi.
    double ae = 0.0, an = 0.0;
    fwd_ops<T>(tp, tl, d, tc, cf, true, true, ae, an);
    const double se = block_sum(ae, tmp);
    const double sn = block_sum(an, tmp);
    if (threadIdx.x == 0) {
      wsum[2 * p] = se;
      wsum[2 * p + 1] = sn;
    }
    __syncthreads();
  }

  // Reverse ops: layers jb..ja with their phases, then the lead mixer.
  if (d.ja <= d.jb)
    for (int j = d.jb; j >= d.ja; --j)
      bwd_mix<T>(tp, tl, d, tc, cf[j], j, p, true, wsum, tmp);
  if (d.lead >= 0) bwd_mix<T>(tp, tl, d, tc, cf[d.lead], d.lead, p, false, wsum, tmp);

  if (d.flags & F_WRITE) {
    for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x)
      gl[zb | dep_local(l, d)] = tl[swz<T>(l)];
  }
  double* o = A.part + ((uint64_t)st * A.nrec + A.rec_base + ti) * (2 * p + 2);
  for (int q = threadIdx.x; q < 2 * p + 2; q += blockDim.x) o[q] = wsum[q];
}

// ---- preparation, reductions ----------------------------------------------------

__global__ void prep_kernel(int nprob, int n, const double* Q, double* W,
                            int nstates, int p, const double* gammas,
                            const double* betas, LayerCoef* coef) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nw = (uint64_t)nprob * n * n;
  if (i < nw) {
    const uint64_t b = i / ((uint64_t)n * n);
    const int r = (int)((i / n) % n), c = (int)(i % n);
    const double* Qb = Q + b * n * n;
    W[i] = (r == c) ? Qb[r * n + r] : Qb[r * n + c] + Qb[c * n + r];
  }
  const uint64_t nc = (uint64_t)nstates * p;
  if (i < nc) {
    const double g = gammas[i], be = betas[i];
    LayerCoef L;
    L.gp = g * 0.15915494309189533577;
    double s, c;
    sincos(be, &s, &c);
    L.cb = c;
    L.sb = s;
    if (fabs(s) <= fabs(c)) {
      L.mode = 0;
      L.tb = s / c;
    } else {
      L.mode = 1;
      L.tb = c / s;
    }
    L.pad = 0;
    coef[i] = L;
  }
}

struct OutMap {
  double* ptr[4];
  int q0[4];
  int cnt[4];
};

__global__ void reduce_parts_kernel(int nrec, int nq, const double* part,
                                    OutMap om) {
  __shared__ double red[16];
  const int st = blockIdx.x, q = blockIdx.y;
  double s = 0.0;
  for (int r = threadIdx.x; r < nrec; r += blockDim.x)
    s += part[((uint64_t)st * nrec + r) * nq + q];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    for (int m = 0; m < 4; ++m) {
      if (om.ptr[m] && q >= om.q0[m] && q < om.q0[m] + om.cnt[m]) {
        om.ptr[m][(uint64_t)st * om.cnt[m] + (q - om.q0[m])] = s;
      }
    }
  }
}

// ---- sampling ------------------------------------------------------------------

constexpr int SBLK = 12;  // log2 of the probability block used by the CDF

// bsum[st][b] = sum of the block's probabilities, fixed-order tree.
template <typename T>
__global__ void block_sums_kernel(int n, const T* P, double* bsum) {
  __shared__ double red[16];
  const int bl = min(n, SBLK);
  const uint64_t nblk = 1ull << (n - bl);
  const int st = blockIdx.y;
  const uint64_t b = blockIdx.x;
  const T* src = P + ((uint64_t)st << n) + (b << bl);
  double s = 0.0;
  for (int i = threadIdx.x; i < (1 << bl); i += blockDim.x) s += (double)src[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) bsum[(uint64_t)st * nblk + b] = s;
}

// Inclusive prefix of the block sums per state: chunked, fixed order.
__global__ void block_scan_kernel(int n, const double* bsum, double* bcdf) {
  __shared__ double tot[1024];
  const int bl = min(n, SBLK);
  const uint64_t nblk = 1ull << (n - bl);
  const int st = blockIdx.x;
  const double* src = bsum + (uint64_t)st * nblk;
  double* dst = bcdf + (uint64_t)st * nblk;
  const uint64_t nt = blockDim.x;
  const uint64_t per = (nblk + nt - 1) / nt;
  const uint64_t lo = threadIdx.x * per, hi = min(nblk, lo + per);
  double run = 0.0;
  for (uint64_t i = lo; i < hi; ++i) {
    run += src[i];
    dst[i] = run;
  }
  tot[threadIdx.x] = run;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (uint64_t i = 0; i < nt; ++i) {
      const double t = tot[i];
      tot[i] = acc;
      acc += t;
    }
  }
  __syncthreads();
  const double off = tot[threadIdx.x];
  for (uint64_t i = lo; i < hi; ++i) dst[i] += off;
}

__device__ __forceinline__ double splitmix_u(uint64_t seed, uint64_t s) {
  uint64_t x = seed + (s + 1ull) * 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * 0x1.0p-53;
}

// One wave per (state, shot): locate u * total in the block CDF, then walk
// the block in increasing z, 64 amplitudes per round (one coalesced load per
// lane, an FP64 inclusive prefix over the wave on top of the running sum);
// the first lane whose running sum exceeds the target gives z.  C(z) from W
// in FP64, one row per lane.  Four shots per 256-thread work-group.
template <typename T>
__global__ void __launch_bounds__(256) shots_kernel(int n, int shots, uint64_t seed,
                                                    const uint64_t* seeds, const T* P,
                                                    const double* bcdf, const double* W,
                                                    int S, uint64_t* zout, double* czout) {
  const int st = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= shots) return;  // the whole wave
  const int bl = min(n, SBLK);
  const uint64_t nblk = 1ull << (n - bl);
  const double* cdf = bcdf + (uint64_t)st * nblk;
  const double total = cdf[nblk - 1];
  // one seed for the launch: state st draws counters st*shots + s; per-state
  // seeds: every state draws counters 0..shots-1 of its own seed
  const double u = seeds ? splitmix_u(seeds[st], (uint64_t)s)
                         : splitmix_u(seed, (uint64_t)st * shots + s);
  const double target = u * total;
  uint64_t lo = 0, hi = nblk - 1;  // first block with cdf > target
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (cdf[mid] > target) hi = mid;
    else lo = mid + 1;
  }
  double run = lo ? cdf[lo - 1] : 0.0;
  const T* src = P + ((uint64_t)st << n) + (lo << bl);
  const int len = 1 << bl;
  uint64_t z = (lo << bl) + (uint64_t)(len - 1);  // rounding fallback: last of the block
  for (int r = 0; r < len; r += 64) {
    const int cnt = len - r < 64 ? len - r : 64;
    double x = lane < cnt ? (double)src[r + lane] : 0.0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    const uint64_t hit = __ballot(lane < cnt && run + x > target);
    if (hit) {
      z = (lo << bl) + (uint64_t)(r + __ffsll((unsigned long long)hit) - 1);
      break;
    }
    run += __shfl(x, 63);
  }
  const double* Wb = W + (size_t)(st / S) * n * n;
  double c = 0.0;
  if (lane < n && ((z >> lane) & 1ull)) {
    c = Wb[lane * n + lane];
    for (int j = 0; j < lane; ++j)
      if ((z >> j) & 1ull) c += Wb[lane * n + j];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
  if (lane == 0) {
    zout[(uint64_t)st * shots + s] = z;
    czout[(uint64_t)st * shots + s] = c;
  }
}

__global__ void best_kernel(int shots, const uint64_t* z, const double* cz,
                            uint64_t* best_z, double* best_c) {
  __shared__ double sc[256];
  __shared__ uint64_t sz[256];
  const int st = blockIdx.x;
  double bc = 0.0;
  uint64_t bz = ~0ull;
  bool have = false;
  for (int s = threadIdx.x; s < shots; s += blockDim.x) {
    const double c = cz[(uint64_t)st * shots + s];
    const uint64_t zz = z[(uint64_t)st * shots + s];
    if (!have || c < bc || (c == bc && zz < bz)) {
      bc = c;
      bz = zz;
      have = true;
    }
  }
  sc[threadIdx.x] = have ? bc : INFINITY;
  sz[threadIdx.x] = bz;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)blockDim.x; ++i) {
      if (sc[i] < sc[0] || (sc[i] == sc[0] && sz[i] < sz[0])) {
        sc[0] = sc[i];
        sz[0] = sz[i];
      }
    }
    best_z[st] = sz[0];
    best_c[st] = sc[0];
  }
}

// ---- Adam and slot gathers ---------------------------------------------------------

// Adam on (gamma, beta) of batch entry i, stored at slot idx[i] (or i when
// idx is NULL): theta/m/v [slot][2p]; gradients dg/db [i][p]; t[slot] counts
// the steps taken.
__global__ void adam_kernel(int nb, int p, const int* idx, double* gammas,
                            double* betas, double* m, double* v, const double* dg,
                            const double* db, const int* t, double lr, double b1,
                            double b2, double eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * 2 * p) return;
  const int e = i / (2 * p), k = i % (2 * p);
  const int slot = idx ? idx[e] : e;
  const int step = t[slot] + 1;
  const double g = (k < p) ? dg[e * p + k] : db[e * p + k - p];
  double* th = (k < p) ? &gammas[slot * p + k] : &betas[slot * p + k - p];
  const int mi = slot * 2 * p + k;
  const double mm = b1 * m[mi] + (1.0 - b1) * g;
  const double vv = b2 * v[mi] + (1.0 - b2) * g * g;
  m[mi] = mm;
  v[mi] = vv;
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  *th -= lr * (mm / c1) / (sqrt(vv / c2) + eps);
}

__global__ void adam_step_count_kernel(int nb, const int* idx, int* t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) t[idx ? idx[i] : i] += 1;
}

// Batch entry i <- slot idx[i]: Q [n][n] (slot stride qstride doubles) and
// (gamma, beta) [p].
__global__ void gather_kernel(int nb, int n, int p, const int* idx,
                              const double* sQ, int qstride, const double* sG,
                              const double* sB, const uint64_t* sSeed, double* Q,
                              double* g, double* b, uint64_t* seeds) {
  const int e = blockIdx.y;
  if (e >= nb) return;
  const int slot = idx[e];
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n * n; i += blockDim.x * gridDim.x)
    Q[(size_t)e * n * n + i] = sQ[(size_t)slot * qstride + i];
  if (blockIdx.x == 0) {
    for (int j = threadIdx.x; j < p; j += blockDim.x) {
      g[e * p + j] = sG[slot * p + j];
      b[e * p + j] = sB[slot * p + j];
    }
    if (seeds && threadIdx.x == 0) seeds[e] = sSeed[slot];
  }
}

int threads_for(int k, int rb) {
  int nb = 1 << (k > rb ? k - rb : 0);
  int nt = nb < 64 ? 64 : (nb > NT_MAX ? NT_MAX : nb);
  return nt;
}

template <typename KernelT>
hipError_t allow_lds(KernelT* kern, size_t bytes) {
  if (bytes > 65536)
    return hipFuncSetAttribute((const void*)kern,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
  return hipSuccess;
}

}  // namespace

size_t lds_bytes_fwd(int prec, int k) {
  const size_t el = prec == 0 ? 16 : 8;
  return (el << k) + sizeof(TileCtx) + 64 * sizeof(double);
}
size_t lds_bytes_bwd(int prec, int k) {
  const size_t el = prec == 0 ? 16 : 8;
  return 2 * (el << k) + sizeof(TileCtx) + (64 + 2 * 64 + 2) * sizeof(double);
}

hipError_t launch_prep(int nprob, int n, const double* Q, double* W,
                       int nstates, int p, const double* gammas,
                       const double* betas, LayerCoef* coef,
                       hipStream_t stream) {
  const uint64_t nw = (uint64_t)nprob * n * n, nc = (uint64_t)nstates * p;
  const uint64_t work = nw > nc ? nw : nc;
  const int nt = 256;
  const uint64_t nb = (work + nt - 1) / nt;
  hipLaunchKernelGGL(prep_kernel, dim3((unsigned)nb), dim3(nt), 0, stream,
                     nprob, n, Q, W, nstates, p, gammas, betas, coef);
  return hipGetLastError();
}

hipError_t launch_fwd_pass(int prec, const PassDesc& d, int nstates, int S,
                           int p, const void* in, void* out,
                           uint64_t state_stride, const double* W,
                           const LayerCoef* coef, double* part, void* probs,
                           hipStream_t stream) {
  FwdArgs A;
  A.d = d;
  A.S = S;
  A.p = p;
  A.in = in;
  A.out = out;
  A.stride = state_stride;
  A.W = W;
  A.coef = coef;
  A.part = part;
  A.probs = probs;
  const uint64_t ntiles = 1ull << (d.n - d.k);
  const size_t lds = lds_bytes_fwd(prec, d.k);
  dim3 grid((unsigned)ntiles, (unsigned)nstates);
  if (prec == 0) {
    hipError_t e = allow_lds(fwd_pass_kernel<double>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fwd_pass_kernel<double>, grid,
                       dim3(threads_for(d.k, Cx<double>::RB)), lds, stream, A);
  } else {
    hipError_t e = allow_lds(fwd_pass_kernel<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fwd_pass_kernel<float>, grid,
                       dim3(threads_for(d.k, Cx<float>::RB)), lds, stream, A);
  }
  return hipGetLastError();
}

hipError_t launch_bwd_pass(int prec, const PassDesc& d, int nstates, int S,
                           int p, const void* psi_in, void* lam,
                           uint64_t state_stride, const double* W,
                           const LayerCoef* coef, double* part, int rec_base,
                           int nrec, hipStream_t stream) {
  BwdArgs A;
  A.d = d;
  A.S = S;
  A.p = p;
  A.psi = psi_in;
  A.lam = lam;
  A.stride = state_stride;
  A.W = W;
  A.coef = coef;
  A.part = part;
  A.rec_base = rec_base;
  A.nrec = nrec;
  const uint64_t ntiles = 1ull << (d.n - d.k);
  const size_t lds = lds_bytes_bwd(prec, d.k);
  dim3 grid((unsigned)ntiles, (unsigned)nstates);
  if (prec == 0) {
    hipError_t e = allow_lds(bwd_pass_kernel<double>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bwd_pass_kernel<double>, grid,
                       dim3(threads_for(d.k, Cx<double>::RB)), lds, stream, A);
  } else {
    hipError_t e = allow_lds(bwd_pass_kernel<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bwd_pass_kernel<float>, grid,
                       dim3(threads_for(d.k, Cx<float>::RB)), lds, stream, A);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_parts(int nstates, int nrec, int nq,
                               const double* part, double* const* out,
                               const int* q0, const int* cnt, int nmap,
                               hipStream_t stream) {
  OutMap om;
  for (int m = 0; m < 4; ++m) {
    om.ptr[m] = m < nmap ? out[m] : nullptr;
    om.q0[m] = m < nmap ? q0[m] : 0;
    om.cnt[m] = m < nmap ? cnt[m] : 0;
  }
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(nstates, nq), dim3(256), 0,
                     stream, nrec, nq, part, om);
  return hipGetLastError();
}

size_t sample_scratch_doubles(int n, int nstates) {
  const int bl = n < SBLK ? n : SBLK;
  return 2 * ((size_t)nstates << (n - bl));
}

hipError_t launch_sample(int prec, int n, int nstates, const void* probs,
                         double* bsum, double* bcdf, int shots, uint64_t seed,
                         const uint64_t* seeds, const double* W, int S, uint64_t* z,
                         double* cz,
                         uint64_t* best_z, double* best_c,
                         hipStream_t stream) {
  const int bl = n < SBLK ? n : SBLK;
  const uint64_t nblk = 1ull << (n - bl);
  const int nt = 256;
  if (prec == 0)
    hipLaunchKernelGGL(block_sums_kernel<double>, dim3((unsigned)nblk, nstates),
                       dim3(nt), 0, stream, n, (const double*)probs, bsum);
  else
    hipLaunchKernelGGL(block_sums_kernel<float>, dim3((unsigned)nblk, nstates),
                       dim3(nt), 0, stream, n, (const float*)probs, bsum);
  hipLaunchKernelGGL(block_scan_kernel, dim3(nstates), dim3(1024), 0, stream, n,
                     bsum, bcdf);
  const int sb = (shots + 3) / 4;
  if (prec == 0)
    hipLaunchKernelGGL(shots_kernel<double>, dim3(sb, nstates), dim3(256), 0,
                       stream, n, shots, seed, seeds, (const double*)probs, bcdf, W,
                       S, z, cz);
  else
    hipLaunchKernelGGL(shots_kernel<float>, dim3(sb, nstates), dim3(256), 0,
                       stream, n, shots, seed, seeds, (const float*)probs, bcdf, W,
                       S, z, cz);
  hipLaunchKernelGGL(best_kernel, dim3(nstates), dim3(256), 0, stream, shots, z,
                     cz, best_z, best_c);
  return hipGetLastError();
}

hipError_t launch_adam(int nb, int p, const int* idx, double* gammas,
                       double* betas, double* m, double* v, const double* dgamma,
                       const double* dbeta, int* t, double lr, double b1,
                       double b2, double eps, hipStream_t stream) {
  const int work = nb * 2 * p;
  hipLaunchKernelGGL(adam_kernel, dim3((work + 255) / 256), dim3(256), 0,
                     stream, nb, p, idx, gammas, betas, m, v, dgamma, dbeta, t,
                     lr, b1, b2, eps);
  hipLaunchKernelGGL(adam_step_count_kernel, dim3((nb + 255) / 256), dim3(256),
                     0, stream, nb, idx, t);
  return hipGetLastError();
}

hipError_t launch_gather(int nb, int n, int p, const int* idx, const double* sQ,
                         int qstride, const double* sG, const double* sB,
                         const uint64_t* sSeed, double* Q, double* g, double* b,
                         uint64_t* seeds, hipStream_t stream) {
  hipLaunchKernelGGL(gather_kernel, dim3(1, nb), dim3(256), 0, stream, nb, n, p,
                     idx, sQ, qstride, sG, sB, sSeed, Q, g, b, seeds);
  return hipGetLastError();
}

}  // namespace dq
