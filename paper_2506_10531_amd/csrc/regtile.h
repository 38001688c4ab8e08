// Register-tile machinery for complex64 state passes (gfx950), shared by the
// forward pass on 14-qubit tiles and the adjoint passes on 13-qubit tiles.
//
// A tile of 2^K amplitudes (K = R + 8) is held by one work-group of 256
// threads (4 waves) in registers: R "register" tile bits per thread, 6 lane
// bits and 2 wave bits.  A layout names which tile bit each register, lane
// and wave slot holds; register slot 0 is tile bit 0 in every layout (the
// pivot: LDS transposes move one half of the tile, split on bit 0, at a
// time).  Butterflies run on register bits only; lane bits 4 and 5 are
// brought into registers by the gfx950 lane-swap instructions
// (v_permlane16_swap / v_permlane32_swap exchange a register-pair bit with
// lane bit 4 / 5), and other bits through an LDS transpose.
//
// A geometry G provides:
//   using V, S;                                  amplitude type (float2 or
//                                                double2) and its scalar
//   static constexpr int C;                      contiguous low tile bits of
//                                                the sets other than set 0
//   static constexpr int R;                      register bits
//   static constexpr int reg_bit(int L, int s);  tile bit of register slot s
//   static constexpr int lane_bit(int L, int s); tile bit of lane slot s
//   static constexpr int wave_bit(int L, int s); tile bit of wave slot s
#pragma once

#include "internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace dq {
namespace rt {

constexpr int NT = 256;

template <class G>
struct Dim {
  using V = typename G::V;
  using S = typename G::S;
  static constexpr int R = G::R;
  static constexpr int K = R + 8;              // tile bits
  static constexpr int NA = 1 << R;            // amplitudes per thread
  static constexpr int NP = NA / 2;            // register pairs (bit 0)
  static constexpr int HALF = 1 << (K - 1);    // amplitudes per LDS half
  static constexpr int PHYS = HALF + (HALF >> 4);
};

// Padded LDS slot of a half index h (tile index without bit 0): one pad slot
// per 16.  Additive over disjoint bit sets (a register's slot is the thread's
// base plus an immediate offset), and half-index bit j moves the slot by 2^j
// (j < 4) or 2^(j-4) (4 <= j < 8) modulo 16: lane slots 0..3 of every LDS
// layout take one bit from each class, so a 16-lane group of an access hits
// 16 distinct 8-byte banks.
__host__ __device__ constexpr uint32_t phys(uint32_t h) { return h + (h >> 4); }

// Half index of register index q (register slots 1..R-1).
template <class G, int L>
__host__ __device__ constexpr uint32_t reg_off(int q) {
  uint32_t l = 0;
  for (int s = 1; s < G::R; ++s)
    if ((q >> (s - 1)) & 1) l |= 1u << G::reg_bit(L, s);
  return l >> 1;
}

template <class G, int L>
__host__ __device__ __forceinline__ uint32_t thread_bits(int lane, int wave) {
  uint32_t l = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s) l |= (uint32_t)((lane >> s) & 1) << G::lane_bit(L, s);
#pragma unroll
  for (int s = 0; s < 2; ++s) l |= (uint32_t)((wave >> s) & 1) << G::wave_bit(L, s);
  return l;
}

// Tile bits of layout L held by lanes and waves; by registers.
template <class G, int L>
__host__ __device__ constexpr uint32_t thread_mask() {
  uint32_t m = 0;
  for (int s = 0; s < 6; ++s) m |= 1u << G::lane_bit(L, s);
  for (int s = 0; s < 2; ++s) m |= 1u << G::wave_bit(L, s);
  return m;
}
template <class G, int L>
__host__ __device__ constexpr uint32_t reg_bits_of() {
  uint32_t m = 0;
  for (int s = 0; s < G::R; ++s) m |= 1u << G::reg_bit(L, s);
  return m;
}

// Register slots (bit s = slot s) that a round in layout L mixes: its tile
// bits not mixed earlier in the same half-mixer (DONE) and at or above the
// pass's first mixed bit.  Compile-time, so a round has no data-dependent
// control flow.
template <class G, int L, uint32_t DONE, int MIXLO>
__host__ __device__ constexpr unsigned reg_mask() {
  unsigned m = 0;
  for (int s = 0; s < G::R; ++s) {
    const int b = G::reg_bit(L, s);
    if (!((DONE >> b) & 1u) && b >= MIXLO) m |= 1u << s;
  }
  return m;
}
__host__ __device__ constexpr int popc(unsigned m) {
  int c = 0;
  for (; m; m &= m - 1) ++c;
  return c;
}

// Global offset of tile index l: set 0 tiles are bits [0, K); the others are
// bits [0, C) plus [a, a + K - C).
template <int C>
__host__ __device__ __forceinline__ uint64_t dep(uint32_t l, int kind, int a) {
  if (kind == 1) return l;
  return (uint64_t)(l & ((1u << C) - 1u)) | ((uint64_t)(l >> C) << a);
}

// Amplitude and scalar helpers for float2 / double2.
template <class V>
__device__ __forceinline__ V mkv(double x, double y) {
  V r;
  r.x = (decltype(r.x))x;
  r.y = (decltype(r.y))y;
  return r;
}
template <class V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = fma(a.x, b.x, -a.y * b.y);
  r.y = fma(a.x, b.y, a.y * b.x);
  return r;
}

// Barrier for LDS hand-offs only: the fence is restricted to the local
// address space, so it waits for this wave's LDS accesses but not for global
// loads still in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS slot bases of a transpose X -> Y for one thread: the write base (its
// layout-X lane and wave bits, relabelled by the mixed bits they hold when
// flip) and the read base (likewise in layout Y).  A register pair q is then
// written at wb + phys(reg_off<G, X>(q)) and read at rb + phys(reg_off<G, Y>(q)).
template <class G, int X, int Y, int MIXLO>
__host__ __device__ __forceinline__ void transpose_bases(int lane, int wave, bool flip,
                                                         uint32_t& wb, uint32_t& rb) {
  constexpr int K = Dim<G>::K;
  constexpr uint32_t M = ((((1u << K) - 1u) >> MIXLO) << MIXLO) & ~1u;
  constexpr uint32_t M1 = M & thread_mask<G, X>(), M2 = M & ~M1;
  static_assert((M2 & ~thread_mask<G, Y>()) == 0, "a mixed bit is a register bit of both layouts");
  static_assert((reg_bits_of<G, X>() & reg_bits_of<G, Y>()) == 1u, "layouts share only the pivot");
  wb = phys((thread_bits<G, X>(lane, wave) ^ (flip ? M1 : 0u)) >> 1);
  rb = phys((thread_bits<G, Y>(lane, wave) ^ (flip ? M2 : 0u)) >> 1);
}

// Move the tile from layout X to layout Y through LDS, one half at a time.
// With flip, the tile is relabelled on the way: the amplitude at tile index l
// moves to l ^ M, M = the mixed tile bits [MIXLO, K) without bit 0.  X and Y
// share only tile bit 0 among their register bits, so every bit of M is a
// lane or wave bit of X (flipped in the write base) or of Y (flipped in the
// read base): the relabelling costs nothing per access.
template <class G, int X, int Y, int MIXLO>
__device__ __forceinline__ void transpose(typename G::V (&v)[Dim<G>::NA], typename G::V* buf,
                                          int lane, int wave, bool flip) {
  constexpr int NP = Dim<G>::NP;
  uint32_t wb, rb;
  transpose_bases<G, X, Y, MIXLO>(lane, wave, flip, wb, rb);
  typename G::V* const bx = buf + wb;
  typename G::V* const by = buf + rb;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < NP; ++q) bx[phys(reg_off<G, X>(q))] = v[(q << 1) | h];
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NP; ++q) v[(q << 1) | h] = by[phys(reg_off<G, Y>(q))];
    lds_barrier();
  }
}

// (a0, a1) -> (a0 + i t a1, a1 + i t a0) on every register slot in RM.
template <class G, unsigned RM>
__device__ __forceinline__ void mix_round(typename G::V (&v)[Dim<G>::NA], typename G::S t) {
  using S = typename G::S;
  constexpr int NP = Dim<G>::NP;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    if (!((RM >> s) & 1u)) continue;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      // j-th register index with bit s clear
      const int r = ((j >> s) << (s + 1)) | (j & ((1 << s) - 1));
      typename G::V& a0 = v[r];
      typename G::V& a1 = v[r | (1 << s)];
      const S x0 = a0.x, y0 = a0.y, x1 = a1.x, y1 = a1.y;
      a0.x = fma(-t, y1, x0);
      a0.y = fma(t, x1, y0);
      a1.x = fma(-t, y0, x1);
      a1.y = fma(t, x0, y1);
      // bound the butterflies in flight (each needs fresh registers until
      // both of its inputs are dead)
      if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Exchange register slot SR with lane slot SL (4 or 5) for the whole tile
// (every 32-bit word of the register pair is swapped).
template <class G, int SR, int SL>
__device__ __forceinline__ void swap_slot(typename G::V (&v)[Dim<G>::NA]) {
  static_assert(SL == 3 || SL == 4 || SL == 5, "lane slots 3, 4 and 5 only");
  using V = typename G::V;
  constexpr int NA = Dim<G>::NA, NW = sizeof(V) / 4;
  struct Words {
    unsigned w[NW];
  };
  // lane slot 3 (lane bit 3): no swap instruction; each lane sends the word
  // its xor-8 partner needs (DPP row rotation by 8 within a 16-lane row is
  // that exchange) and keeps the other
  const bool c3 = SL == 3 && ((threadIdx.x >> 3) & 1);
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    if ((r >> SR) & 1) continue;
    Words w0 = __builtin_bit_cast(Words, v[r]);
    Words w1 = __builtin_bit_cast(Words, v[r | (1 << SR)]);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      if (SL == 3) {
        const unsigned send = c3 ? w0.w[k] : w1.w[k];
        const unsigned recv = (unsigned)__builtin_amdgcn_mov_dpp((int)send, 0x128, 0xF, 0xF, false);
        if (c3) w0.w[k] = recv;
        else w1.w[k] = recv;
      } else if (SL == 5) {
        const auto px = __builtin_amdgcn_permlane32_swap(w0.w[k], w1.w[k], false, false);
        w0.w[k] = px[0];
        w1.w[k] = px[1];
      } else {
        const auto px = __builtin_amdgcn_permlane16_swap(w0.w[k], w1.w[k], false, false);
        w0.w[k] = px[0];
        w1.w[k] = px[1];
      }
    }
    v[r] = __builtin_bit_cast(V, w0);
    v[r | (1 << SR)] = __builtin_bit_cast(V, w1);
  }
}

// e^{-i 2 pi rev}.  The angle is reduced in FP64 to t in [-1/2, 1/2], then to
// an eighth of a turn: q = rint(4 t), theta = 2 pi (t - q / 4) in
// [-pi/4, pi/4]; sin and cos of theta from their Taylor series through
// theta^9 and theta^10 (truncation below 2e-9 there), rotated by q quarter
// turns.
__device__ __forceinline__ float2 unit(double rev) {
  const float t = (float)(rev - rint(rev));
  const float q = rintf(4.0f * t);
  const float th = 6.28318530717958647692f * fmaf(-0.25f, q, t);
  const float x = th * th;
  const float sn =
      th * fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f),
                        -1.0f / 6.0f),
                1.0f);
  const float cs = fmaf(
      x,
      fmaf(x, fmaf(x, fmaf(x, fmaf(x, -1.0f / 3628800.0f, 1.0f / 40320.0f), -1.0f / 720.0f),
                   1.0f / 24.0f),
           -0.5f),
      1.0f);
  // (cos, sin) of theta + q pi / 2
  const int k = (int)q & 3;
  const float c = (k & 1) ? ((k & 2) ? sn : -sn) : ((k & 2) ? -cs : cs);
  const float s = (k & 1) ? ((k & 2) ? -cs : cs) : ((k & 2) ? -sn : sn);
  return make_float2(c, -s);
}
// e^{-i 2 pi rev} in double precision (complex128 states).
__device__ __forceinline__ double2 unit_d(double rev) {
  double s, c;
  sincospi(2.0 * (rev - rint(rev)), &s, &c);
  return make_double2(c, -s);
}
template <class V>
__device__ __forceinline__ V unitv(double rev) {
  if constexpr (sizeof(V) == 8) return unit(rev);
  else return unit_d(rev);
}

// Mixer scalar of one half-mixer on m qubits, multiplied into (re, im): the
// forward mixer e^{i beta X} is c (I + i tan X) per qubit (mode 0) or
// i s X (I - i cot X) (mode 1); its inverse e^{-i beta X} is c (I - i tan X)
// or -i s X (I + i cot X).
__device__ __forceinline__ void half_scale(const LayerCoef& L, int m, bool inv, double& re,
                                           double& im) {
  double r = 1.0, i = 0.0;
  if (L.mode == 0) {
    for (int q = 0; q < m; ++q) r *= L.cb;
  } else {
    const double sb = inv ? -L.sb : L.sb;
    for (int q = 0; q < m; ++q) {
      const double nr = -i * sb, ni = r * sb;
      r = nr;
      i = ni;
    }
  }
  const double nr = re * r - im * i, ni = re * i + im * r;
  re = nr;
  im = ni;
}
// Arithmetic parameter t of a half-mixer, (a0, a1) -> (a0 + i t a1, ...):
// tan b (mode 0) or -cot b (mode 1) forward, negated for the inverse.
__device__ __forceinline__ double mix_t(const LayerCoef& L, bool inv) {
  const double t = L.mode == 0 ? L.tb : -L.tb;
  return inv ? -t : t;
}

// Per-tile tables for the phase layout PL (FP64):
//   Ll[64]    energy of the lane bits alone (with their block fields)
//   Lw[4]     energy of the wave bits alone (with their block fields)
//   Gl[R][64] field of the lane bits on register slot s
//   Fw[6][4]  coupling of lane slot i to the wave bits
//   Gw[R][4]  field of the wave bits on register slot s
//   Kr[2^R]   couplings among the register bits
// Only the first NF entries depend on the tile's block bits; the others, and
// the factors e^{-i gamma K(r)}, are the same for every tile of a pass and
// state (they depend on the couplings among the tile's qubits only).
template <int R>
struct Tables {
  double Ll[64], Lw[4], Gl[R][64], Fw[6][4], Gw[R][4], Kr[1 << R];
  static constexpr int NF = 64 + 4;
  static constexpr int N = NF + R * 64 + 6 * 4 + R * 4 + (1 << R);
};

// 0.0 or 1.0: bit i of x.  Table sums multiply by it instead of branching,
// so every LDS read of a sum is independent and issued back to back.
__device__ __forceinline__ double bitd(uint64_t x, int i) { return (double)((x >> i) & 1ull); }

// Entry e of the tables, from the tile-local fields fl[K] and couplings
// Wl[K][K].
template <class G, int PL>
__device__ __forceinline__ void table_entry(Tables<G::R>* T, const double* fl, const double* Wl,
                                            int e) {
  constexpr int R = G::R, K = Dim<G>::K;
  if (e < 64) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const int bi = G::lane_bit(PL, i);
      double t = fl[bi];
#pragma unroll
      for (int j = 0; j < i; ++j) t = fma(bitd(e, j), Wl[bi * K + G::lane_bit(PL, j)], t);
      s = fma(bitd(e, i), t, s);
      __builtin_amdgcn_sched_barrier(0);  // at most 6 reads in flight
    }
    T->Ll[e] = s;
    return;
  }
  e -= 64;
  if (e < 4) {
    const int b0 = G::wave_bit(PL, 0), b1 = G::wave_bit(PL, 1);
    const double t1 = fl[b1] + bitd(e, 0) * Wl[b1 * K + b0];
    T->Lw[e] = fma(bitd(e, 0), fl[b0], bitd(e, 1) * t1);
    return;
  }
  e -= 4;
  if (e < R * 64) {
    const int sl = e >> 6, x = e & 63, br = G::reg_bit(PL, sl);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) s = fma(bitd(x, i), Wl[br * K + G::lane_bit(PL, i)], s);
    T->Gl[sl][x] = s;
    return;
  }
  e -= R * 64;
  if (e < 6 * 4) {
    const int li = e >> 2, y = e & 3, bl = G::lane_bit(PL, li);
    T->Fw[li][y] = fma(bitd(y, 0), Wl[bl * K + G::wave_bit(PL, 0)],
                       bitd(y, 1) * Wl[bl * K + G::wave_bit(PL, 1)]);
    return;
  }
  e -= 6 * 4;
  if (e < R * 4) {
    const int sl = e >> 2, y = e & 3, br = G::reg_bit(PL, sl);
    T->Gw[sl][y] = fma(bitd(y, 0), Wl[br * K + G::wave_bit(PL, 0)],
                       bitd(y, 1) * Wl[br * K + G::wave_bit(PL, 1)]);
    return;
  }
  e -= R * 4;
  if (e < (1 << R)) {
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < R; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < i; ++j) t = fma(bitd(e, j), Wl[G::reg_bit(PL, i) * K + G::reg_bit(PL, j)], t);
      s = fma(bitd(e, i), t, s);
      __builtin_amdgcn_sched_barrier(0);
    }
    T->Kr[e] = s;
  }
}

// The thread's cfix and fields g_s in the phase layout (FP64).  Branch-free,
// so that it does not split the straight-line code around it.
template <class G, int PL>
__device__ __forceinline__ void thread_energy(const Tables<G::R>* T, const double* fl,
                                              double cblk, int lane, int wave, double& cfix,
                                              double (&g)[G::R]) {
  double c = cblk + T->Lw[wave] + T->Ll[lane];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double f = T->Fw[i][wave];
    c += ((lane >> i) & 1) ? f : 0.0;
  }
  cfix = c;
#pragma unroll
  for (int s = 0; s < G::R; ++s) g[s] = fl[G::reg_bit(PL, s)] + T->Gl[s][lane] + T->Gw[s][wave];
}

// Per-thread phase factors of one layer: f0 = e^{-i gamma cfix} times a
// scalar (sr, si), fs[s] = e^{-i gamma g_s}; gp = gamma / 2 pi (negated to
// undo the phase).
template <int R, class V>
struct PhaseF {
  V f0, fs[R];
};
template <class G, int PL>
__device__ __forceinline__ PhaseF<G::R, typename G::V> phase_factors(const Tables<G::R>* T,
                                                                     const double* fl, double cblk,
                                                                     int lane, int wave, double gp,
                                                                     double sr, double si) {
  using V = typename G::V;
  double cfix, g[G::R];
  thread_energy<G, PL>(T, fl, cblk, lane, wave, cfix, g);
  PhaseF<G::R, V> P;
  P.f0 = cmul(unitv<V>(gp * cfix), mkv<V>(sr, si));
#pragma unroll
  for (int s = 0; s < G::R; ++s) P.fs[s] = unitv<V>(gp * g[s]);
  return P;
}

// The factor of every register amplitude r: f0 * prod_{s in r} fs[s] *
// KF[r], built as a product tree and handed to fn(r, factor).
template <int R, int S, class V, class F>
__device__ __forceinline__ void phase_tree(const PhaseF<R, V>& P, const V* KF, V p, int r,
                                           F&& fn) {
  if constexpr (S < 0) {
    fn(r, cmul(p, KF[r]));
  } else {
    phase_tree<R, S - 1>(P, KF, p, r, fn);
    phase_tree<R, S - 1>(P, KF, cmul(p, P.fs[S]), r | (1 << S), fn);
    if constexpr (S == 0) __builtin_amdgcn_sched_barrier(0);
  }
}

// Phase of one layer on the register amplitudes.
template <class G>
__device__ __forceinline__ void apply_phase(typename G::V (&v)[Dim<G>::NA],
                                            const typename G::V* KF,
                                            const PhaseF<G::R, typename G::V>& P) {
  phase_tree<G::R, G::R - 1>(P, KF, P.f0, 0,
                             [&](int r, typename G::V f) { v[r] = cmul(v[r], f); });
}

// The register amplitudes set to their phase factors (the state before the
// first phase is uniform and its amplitude is folded into P.f0).
template <class G>
__device__ __forceinline__ void init_phase(typename G::V (&v)[Dim<G>::NA],
                                           const typename G::V* KF,
                                           const PhaseF<G::R, typename G::V>& P) {
  phase_tree<G::R, G::R - 1>(P, KF, P.f0, 0, [&](int r, typename G::V f) { v[r] = f; });
}

// <C> and norm partial sums of the register amplitudes, FP64, from the
// thread's cfix and fields g (thread_energy).
template <class G>
__device__ __forceinline__ void reduce_regs(const typename G::V (&v)[Dim<G>::NA],
                                            const Tables<G::R>* T,
                                            double cfix, const double (&g)[G::R], double& ae,
                                            double& an) {
  constexpr int R = G::R, LO = 3;
#pragma unroll
  for (int hi = 0; hi < (1 << (R - LO)); ++hi) {
    double ch = cfix;
#pragma unroll
    for (int s = LO; s < R; ++s)
      if ((hi >> (s - LO)) & 1) ch += g[s];
#pragma unroll
    for (int lo = 0; lo < (1 << LO); ++lo) {
      const int r = (hi << LO) | lo;
      double c = ch + T->Kr[r];
#pragma unroll
      for (int s = 0; s < LO; ++s)
        if ((lo >> s) & 1) c += g[s];
      const double pz = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
      ae = fma(pz, c, ae);
      an += pz;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Global offset, from the tile's block base, of register pair q of a thread
// in layout L: its lane and wave part (pair_base) plus its register part
// (pair_rel).  The two amplitudes of a pair are at that offset and the next.
template <class G, int L>
__host__ __device__ __forceinline__ uint64_t pair_base(int lane, int wave, int kind, int a) {
  return dep<G::C>(thread_bits<G, L>(lane, wave), kind, a);
}
template <class G, int L>
__host__ __device__ __forceinline__ uint64_t pair_rel(int q, int kind, int a) {
  return dep<G::C>(reg_off<G, L>(q) << 1, kind, a);
}

// Global load/store of the register tile in layout L.  The two amplitudes of
// a register pair differ in tile bit 0 and are adjacent in memory: one
// 16-byte access for complex64, two for complex128.
template <class G, int L>
__device__ __forceinline__ void load_tile(typename G::V (&v)[Dim<G>::NA], const typename G::V* base,
                                          int lane, int wave, int kind, int a) {
  using V = typename G::V;
  const uint64_t tb = pair_base<G, L>(lane, wave, kind, a);
#pragma unroll
  for (int q = 0; q < Dim<G>::NP; ++q) {
    const uint64_t o = tb + pair_rel<G, L>(q, kind, a);
    if constexpr (sizeof(V) == 8) {
      const float4 w = *reinterpret_cast<const float4*>(base + o);
      v[q << 1] = make_float2(w.x, w.y);
      v[(q << 1) | 1] = make_float2(w.z, w.w);
    } else {
      v[q << 1] = base[o];
      v[(q << 1) | 1] = base[o + 1];
    }
  }
}

// sw: tile bit 0 is flipped (each register pair is stored in swapped
// order).  The two orders are separate loops, not per-element selects.
template <class G, int L, bool SW>
__device__ __forceinline__ void store_rows(const typename G::V (&v)[Dim<G>::NA],
                                           typename G::V* base, uint64_t tb, int kind, int a) {
  using V = typename G::V;
#pragma unroll
  for (int q = 0; q < Dim<G>::NP; ++q) {
    const uint64_t o = tb + pair_rel<G, L>(q, kind, a);
    const V u = v[(q << 1) | SW], w = v[(q << 1) | !SW];
    if constexpr (sizeof(V) == 8) {
      *reinterpret_cast<float4*>(base + o) = make_float4(u.x, u.y, w.x, w.y);
    } else {
      base[o] = u;
      base[o + 1] = w;
    }
  }
}
template <class G, int L>
__device__ __forceinline__ void store_tile(const typename G::V (&v)[Dim<G>::NA],
                                           typename G::V* base, int lane, int wave, int kind,
                                           int a, bool sw) {
  const uint64_t tb = pair_base<G, L>(lane, wave, kind, a);
  if constexpr (sizeof(typename G::V) == 16) {
    // complex128: an amplitude per 16-byte store, so the flipped order is an
    // address offset (kept out of a branch, whose two store sequences the
    // compiler may merge through private memory)
    const uint64_t s0 = sw ? 1u : 0u;
#pragma unroll
    for (int q = 0; q < Dim<G>::NP; ++q) {
      const uint64_t o = tb + pair_rel<G, L>(q, kind, a);
      base[o + s0] = v[q << 1];
      base[o + (s0 ^ 1u)] = v[(q << 1) | 1];
    }
  } else {
    if (sw) store_rows<G, L, true>(v, base, tb, kind, a);
    else store_rows<G, L, false>(v, base, tb, kind, a);
  }
}

// |psi|^2 * scale in the state precision (float for complex64, double for
// complex128), a register pair per 8- or 16-byte store.
template <class G, int L, bool SW>
__device__ __forceinline__ void store_prob_rows(const typename G::V (&v)[Dim<G>::NA],
                                                typename G::S* base, uint64_t tb, int kind, int a,
                                                typename G::S scale) {
  using V = typename G::V;
  using S = typename G::S;
#pragma unroll
  for (int q = 0; q < Dim<G>::NP; ++q) {
    const uint64_t o = tb + pair_rel<G, L>(q, kind, a);
    const V u = v[(q << 1) | SW], w = v[(q << 1) | !SW];
    const S pu = scale * (u.x * u.x + u.y * u.y), pw = scale * (w.x * w.x + w.y * w.y);
    *reinterpret_cast<V*>(base + o) = mkv<V>(pu, pw);
  }
}
template <class G, int L>
__device__ __forceinline__ void store_probs(const typename G::V (&v)[Dim<G>::NA],
                                            typename G::S* base, int lane, int wave, int kind,
                                            int a, typename G::S scale, bool sw) {
  const uint64_t tb = pair_base<G, L>(lane, wave, kind, a);
  if (sw) store_prob_rows<G, L, true>(v, base, tb, kind, a, scale);
  else store_prob_rows<G, L, false>(v, base, tb, kind, a, scale);
}

// Sum of x over the work-group (red: NT / 64 doubles of LDS).
__device__ __forceinline__ double block_sum(double x, double* red) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  lds_barrier();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  lds_barrier();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  lds_barrier();
  return s;
}

// Block bits of tile ti (set kind 1: bits [K, n); kind 2: bits [C, a) and
// [a + K - C, n)).
template <int K, int C>
__host__ __device__ __forceinline__ uint64_t tile_base(uint64_t ti, int kind, int a) {
  if (kind == 1) return ti << K;
  const int gap = a - C;
  return ((ti & ((1ull << gap) - 1ull)) << C) | ((ti >> gap) << (a + K - C));
}

// Couplings Wl[K][K] among the tile bits (the same for every tile of a set),
// with the signs of tile bit 0's couplings flipped when f0.
template <int K, int C, int KIND>
__device__ __forceinline__ void tile_couplings(const double* Wsh, int n, int a, bool f0,
                                               double* Wl, int tid) {
  for (int e = tid; e < K * K; e += NT) {
    const int i = e / K, j = e - K * i;
    const int pi = (KIND == 1 || i < C) ? i : a + i - C;
    const int pj = (KIND == 1 || j < C) ? j : a + j - C;
    const double w = (i == j) ? 0.0 : Wsh[pi * n + pj];
    Wl[e] = (f0 && (i == 0) != (j == 0)) ? -w : w;
  }
}

// LDS context of one tile: the folded Q staged in LDS (Wsh, n x n), the
// tile-local fields fl[K] (block fields on the tile bits), couplings Wl[K][K]
// among tile bits and the energy of the block bits (returned).  With f0, the
// tile-local energy is that of z ^ 1 (tile bit 0 flipped, kind 1 only): the
// field and couplings of bit 0 change sign, the other fields gain their
// coupling to bit 0, and the constant gains the old field of bit 0.
// tmp: n + 1 doubles.  Ends with a barrier.
template <int K, int C, int KIND>
__device__ __forceinline__ double tile_context(const double* Wsh, int n, int a, uint64_t zb,
                                               bool f0, double* fl, double* Wl, double* tmp,
                                               int tid) {
  if (tid < K) {
    const int pi = (KIND == 1 || tid < C) ? tid : a + tid - C;
    double f = Wsh[pi * n + pi];
#pragma unroll 8
    for (int j = 0; j < n; ++j) f = fma(bitd(zb, j), Wsh[pi * n + j], f);
    if (f0) f = tid == 0 ? -f : f + Wsh[pi * n];
    fl[tid] = f;
  } else if (tid >= 64 && tid <= 64 + n) {
    // block energy: row i of the block bits (i < n), or the old field of
    // tile bit 0 when it is flipped (i = n; kind 1: tile bit 0 is qubit 0)
    const int i = tid - 64;
    const bool fr = i == n;
    const int row = fr ? 0 : i, cnt = fr ? n : i;
    double t = Wsh[row * n + row];
#pragma unroll 8
    for (int j = 0; j < cnt; ++j) t = fma(bitd(zb, j), Wsh[row * n + j], t);
    tmp[i] = fr ? (f0 ? t : 0.0) : bitd(zb, i) * t;
  }
  tile_couplings<K, C, KIND>(Wsh, n, a, f0, Wl, tid);
  lds_barrier();
  double cblk = 0.0;
  for (int i = 0; i <= n; ++i) cblk += tmp[i];
  return cblk;
}

// e^{-i 2 pi gp K(r)} for the couplings K(r) among the register bits r.
template <class G, int PL>
__device__ __forceinline__ typename G::V reg_factor(const double* Wl, double gp, int r) {
  constexpr int R = G::R, K = Dim<G>::K;
  double k = 0.0;
#pragma unroll
  for (int i = 1; i < R; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < i; ++j) t = fma(bitd(r, j), Wl[G::reg_bit(PL, i) * K + G::reg_bit(PL, j)], t);
    k = fma(bitd(r, i), t, k);
    __builtin_amdgcn_sched_barrier(0);
  }
  return unitv<typename G::V>(gp * k);
}


// Stage the folded Q (n x n) and the state's layer coefficients in LDS while
// the tile's loads are in flight: the Q reads are issued first, then issue(),
// the tile loads, then the LDS writes wait for the Q reads only.  Ends with a
// barrier.
struct NoCopy {
  __device__ double operator()(int) const { return 0.0; }
  __device__ void operator()(int, double) const {}
};
template <int NX = 0, class Issue, class Src = NoCopy, class Dst = NoCopy>
__device__ __forceinline__ void stage_context(const double* W, int n, const LayerCoef* coef, int p,
                                              double* Wsh, LayerCoef* cf, int tid, Issue&& issue,
                                              Src&& src = Src(), Dst&& dst = Dst()) {
  constexpr int NW = (34 * 34 + NT - 1) / NT;
  constexpr int NXT = (NX + NT - 1) / NT;  // extra words per thread (NX words in all)
  const int nn = n * n;
  double wr[NW];
  double xr[NXT > 0 ? NXT : 1];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int e = tid + k * NT;
    wr[k] = e < nn ? W[e] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < NXT; ++k) {
    const int e = tid + k * NT;
    xr[k] = e < NX ? src(e) : 0.0;
  }
  static_assert(sizeof(LayerCoef) == 40, "layer coefficients move as five doubles");
  double cv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (tid < p) {
    const double* c = reinterpret_cast<const double*>(coef + tid);
#pragma unroll
    for (int k = 0; k < 5; ++k) cv[k] = c[k];
  }
  __builtin_amdgcn_sched_barrier(0);
  issue();
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int e = tid + k * NT;
    if (e < nn) Wsh[e] = wr[k];
  }
#pragma unroll
  for (int k = 0; k < NXT; ++k) {
    const int e = tid + k * NT;
    if (e < NX) dst(e, xr[k]);
  }
  if (tid < p) {
    double* c = reinterpret_cast<double*>(cf + tid);
#pragma unroll
    for (int k = 0; k < 5; ++k) c[k] = cv[k];
  }
  lds_barrier();
}

// ---- forward pass --------------------------------------------------------------

// Pass shapes (every pass of a register-tile plan is one of these):
//   P_FIRST  initial state, phase, half-mixer PL -> LA, store
//   P_MID    load, lead half-mixer LA -> PL, phase, half-mixer PL -> LA, store
//   P_LEAD   load, lead half-mixer LA -> PL, store (sets between the ends of a
//            layer when there are more than two)
//   P_LAST   load, lead half-mixer LA -> PL, <C>/norm partials and the
//            optional probability and state outputs
enum { P_FIRST = 0, P_MID = 1, P_LEAD = 2, P_LAST = 3 };

struct FwdArgs {
  PassDesc d;
  int S, p;
  const void* in;   // states (float2 or double2 amplitudes)
  void* out;
  uint64_t stride;
  const double* W;
  const LayerCoef* coef;
  double* part;
  void* probs;      // |psi|^2 in the state precision
  const void* tab = nullptr;  // the pass's PassTab records, TAB_BYTES apart (all_tables_kernel)
};

// The tile-independent part of a pass's tables for one state: Tables
// entries [NF, N) and, for passes with a phase, the register factors.
template <class G>
struct PassTab {
  Tables<G::R> T;
  typename G::V KF[1 << G::R];
};


// Couplings among the tile bits for a run-time kind and c (the job's).
template <int K>
__device__ __forceinline__ void tile_couplings_rt(const double* Wsh, int n, int kind, int c,
                                                  int a, bool f0, double* Wl, int tid) {
  for (int e = tid; e < K * K; e += NT) {
    const int i = e / K, j = e - K * i;
    const int pi = (kind == 1 || i < c) ? i : a + i - c;
    const int pj = (kind == 1 || j < c) ? j : a + j - c;
    const double w = (i == j) ? 0.0 : Wsh[pi * n + pj];
    Wl[e] = (f0 && (i == 0) != (j == 0)) ? -w : w;
  }
}

template <class G, int PL>
__device__ __forceinline__ void tab_entries(PassTab<G>* o, const double* Wl, int kfl, double gp,
                                            int tid) {
  constexpr int R = G::R;
  for (int e = Tables<R>::NF + tid; e < Tables<R>::N; e += NT) table_entry<G, PL>(&o->T, nullptr, Wl, e);
  if (kfl >= 0 && tid < (1 << R)) o->KF[tid] = reg_factor<G, PL>(Wl, gp, tid);
}

// All tables of a call in one launch: work-group (state blockIdx.x, job
// blockIdx.y) writes the PassTab of that pass and state at record
// job * nstates + state (TAB_BYTES apart).  G stands for its geometry family:
// the layouts do not depend on the number of contiguous low bits.
template <class G>
__global__ void __launch_bounds__(NT) all_tables_kernel(TabJobs J, int n, int S, int p,
                                                        int nstates, const double* W,
                                                        const LayerCoef* coef, char* out) {
  constexpr int K = Dim<G>::K;
  const TabJob jb = J.job[blockIdx.y];
  if (jb.kind == 0) return;
  __shared__ double Wsh[34 * 34];
  __shared__ double Wl[K * K];
  __shared__ LayerCoef cf[64];
  const int tid = threadIdx.x, st = blockIdx.x;
  const double* Ws = W + (size_t)(st / S) * n * n;
  for (int e = tid; e < n * n; e += NT) Wsh[e] = Ws[e];
  if (tid < p) cf[tid] = coef[(size_t)st * p + tid];
  lds_barrier();
  const bool f0 = jb.kind == 1 && jb.flip >= 0 && cf[jb.flip].mode != 0;
  tile_couplings_rt<K>(Wsh, n, jb.kind, jb.c, jb.a, f0, Wl, tid);
  lds_barrier();
  PassTab<G>* o =
      reinterpret_cast<PassTab<G>*>(out + ((size_t)blockIdx.y * nstates + st) * TAB_BYTES);
  const double gp = jb.kfl >= 0 ? (jb.neg ? -cf[jb.kfl].gp : cf[jb.kfl].gp) : 0.0;
  if (jb.kind == 1) tab_entries<G, G::template PL<1>>(o, Wl, jb.kfl, gp, tid);
  else tab_entries<G, G::template PL<2>>(o, Wl, jb.kfl, gp, tid);
}

template <class G>
inline hipError_t launch_all_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                    const double* W, const LayerCoef* coef, void* tab,
                                    hipStream_t stream) {
  static_assert(sizeof(PassTab<G>) <= TAB_BYTES, "pass tables exceed their scratch");
  if (!tab || nstates < 1 || J.njobs < 1 || J.njobs > MAX_TAB_JOBS)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(all_tables_kernel<G>, dim3(nstates, J.njobs), dim3(NT), 0, stream, J, n, S,
                     p, nstates, W, coef, static_cast<char*>(tab));
  return hipGetLastError();
}


// Pass shape of a descriptor, or -1.
inline int pass_shape(const PassDesc& d, int p) {
  const bool phase = d.ja <= d.jb;
  if (phase && (d.ja != d.jb || d.jb < 0 || d.jb >= p)) return -1;
  if (d.lead >= p) return -1;
  if (d.flags & F_INIT)
    return (d.lead < 0 && phase && (d.flags & F_WRITE) && !(d.flags & F_REDUCE)) ? P_FIRST : -1;
  if (d.lead < 0) return -1;
  if (d.flags & F_REDUCE) return phase ? -1 : P_LAST;
  if (!(d.flags & F_WRITE)) return -1;
  return phase ? P_MID : P_LEAD;
}

// Tile index of this work-group.  Work-groups are dealt to the 8 XCDs (each
// with its own L2) in turn.  GRP > 1 maps GRP consecutive tiles, whose runs
// lie next to each other in memory, to work-groups 8 apart, i.e. to one XCD
// back to back: when a tile's runs are shorter than a 128 B line, tiles t and
// t ^ 1 share every line, and with runs of a line or less one XCD then fetches
// and writes GRP adjacent runs as one stretch.  A bijection of [0, gridDim.x)
// when gridDim.x is a multiple of 8 GRP (otherwise the identity).
template <int GRP>
__host__ __device__ __forceinline__ uint32_t xcd_map(uint32_t b, uint32_t grid) {
  if constexpr (GRP == 1) {
    (void)grid;
    return b;
  } else {
    static_assert(GRP > 1 && GRP <= 64 && (GRP & (GRP - 1)) == 0, "GRP");
    constexpr uint32_t span = 8u * GRP;
    constexpr int lg = GRP == 2 ? 1 : GRP == 4 ? 2 : GRP == 8 ? 3 : GRP == 16 ? 4 : GRP == 32 ? 5 : 6;
    if (grid % span) return b;
    return (b & ~(span - 1u)) | ((b & 7u) << lg) | ((b >> 3) & (GRP - 1u));
  }
}
template <int GRP>
__device__ __forceinline__ uint64_t xcd_tile() {
  return xcd_map<GRP>(blockIdx.x, gridDim.x);
}

// Tiles per XCD group for a pass shape on runs of RUN bytes (kernel traces,
// n = 24, 16 states): complex64 128 B runs, first 0.495 / 0.511 / 0.500 ms
// with groups of 2 / 4 / 8, middle 0.995 / 0.923 / 0.943, last 0.508 / 0.503
// / 0.493 (0.496 with 16); complex128 64 B runs, first 1.484 / 1.387 / 1.456,
// middle 2.676 / 2.573 / 2.334 and then 2.253 / 2.283 with 16 / 32, last
// 1.218 / 1.203 / 1.074 and then 1.030 / 1.030.  Longer runs keep the plain
// order (groups of 2-8 on 256 B runs slowed the n = 32 step by 1-2%).
template <int KIND, int RUN, int PT>
constexpr int tile_group() {
  if (KIND != 2 || RUN > 128) return 1;
  if (RUN == 128) return PT == P_FIRST ? 2 : (PT == P_LAST ? 8 : 4);
  return PT == P_FIRST ? 4 : 16;
}

// One tile of one pass per work-group (tile index = state * 2^(n-K) + tile
// of the state).  G::LA is the load/store layout and G::PL<KIND> the phase
// layout; the pass mixes tile bits [MIXLO, K).  One straight-line body per
// pass shape keeps the tile's registers in place from load to store.  With
// TRUE_OUT a stored state carries its pending mixer scalar (the adjoint
// passes read such states).
template <class G, int KIND, int MIXLO, int PT, bool TRUE_OUT = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
fwd_kernel(FwdArgs A) {
  using D = Dim<G>;
  using V = typename G::V;
  using S = typename G::S;
  constexpr int K = D::K, NA = D::NA;
  constexpr int LA = G::LA, PL = G::template PL<KIND>;
  constexpr bool LEAD = PT != P_FIRST, PHASE = PT == P_FIRST || PT == P_MID;
  __shared__ V buf[D::PHYS];
  __shared__ Tables<G::R> T;
  __shared__ double fl[K];
  __shared__ double Wl[K * K];
  __shared__ double tmp[40];
  __shared__ V KF[NA];
  __shared__ LayerCoef cf[64];
  const PassDesc& d = A.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = d.n, nlog = n - K;
  const uint64_t tile = xcd_tile<tile_group<KIND, (1 << G::C) * (int)sizeof(V), PT>()>();
  const uint64_t st = tile >> nlog, ti = tile & ((1ull << nlog) - 1ull);
  const uint64_t zb = tile_base<K, G::C>(ti, KIND, d.a);
  const V* const gin = reinterpret_cast<const V*>(A.in) + st * A.stride + zb;
  V* const gout = reinterpret_cast<V*>(A.out) + st * A.stride + zb;
  double* const Wsh = reinterpret_cast<double*>(buf);  // idle until the first transpose
  V v[NA];
  // the tile-independent tables come from the state's PassTab (A.tab),
  // copied to LDS with the folded Q while the tile is in flight
  constexpr int NT1 = Tables<G::R>::N - Tables<G::R>::NF;
  constexpr int NT2 = PHASE ? (int)(sizeof(V) << G::R) / 8 : 0;
  const PassTab<G>* tab =
      reinterpret_cast<const PassTab<G>*>(static_cast<const char*>(A.tab) + st * TAB_BYTES);
  // a lead-only pass has no phase and no reduction: it needs neither the
  // folded Q nor the tile's tables
  stage_context<PT != P_LEAD ? NT1 + NT2 : 0>(
      A.W + (size_t)(st / A.S) * n * n, PT == P_LEAD ? 0 : n, A.coef + st * A.p, A.p, Wsh, cf,
      tid,
      [&] {
        if (PT != P_FIRST) load_tile<G, LA>(v, gin, lane, wave, KIND, d.a);
      },
      [&](int w) {
        return w < NT1 ? (&tab->T.Gl[0][0])[w] : reinterpret_cast<const double*>(tab->KF)[w - NT1];
      },
      [&](int w, double x) {
        if (w < NT1) (&T.Gl[0][0])[w] = x;
        else reinterpret_cast<double*>(KF)[w - NT1] = x;
      });
  // tile bit 0 flipped at PL (only when the pass mixes bit 0)
  const bool f0 = MIXLO == 0 && LEAD && cf[d.lead].mode != 0;
  const double cblk =
      PT == P_LEAD ? 0.0 : tile_context<K, G::C, KIND>(Wsh, n, d.a, zb, f0, fl, Wl, tmp, tid);
  if (PT != P_LEAD) {  // the tables' block-field entries
    for (int e = tid; e < Tables<G::R>::NF; e += NT) table_entry<G, PL>(&T, fl, Wl, e);
    lds_barrier();
  }

  // pending mixer scalar (at the phase, or at the outputs of the last pass)
  double sr = 1.0, si = 0.0;
  for (int i = 0; i < d.pend_n; ++i) half_scale(cf[d.pend_layer[i]], d.pend_m[i], false, sr, si);
  if (LEAD) half_scale(cf[d.lead], K - MIXLO, false, sr, si);
  PhaseF<G::R, V> P;
  // the first pass starts from the uniform amplitude 2^{-n/2}: it folds into
  // the thread factor, and the phase factors become the amplitudes
  if (PT == P_FIRST) sr *= exp2(-0.5 * (double)n), si *= exp2(-0.5 * (double)n);
  bool sw = f0;  // tile bit 0 is flipped
  if (LEAD) {
    const LayerCoef& L = cf[d.lead];
    G::template lead<KIND, MIXLO>(v, buf, lane, wave, (S)mix_t(L, false), L.mode != 0);
  }
  // formed after the lead half-mixer: formed before it, the factors would
  // hold registers through its rounds and transposes
  if (PHASE) P = phase_factors<G, PL>(&T, fl, cblk, lane, wave, cf[d.jb].gp, sr, si);
  if (PHASE) {
    const LayerCoef& L = cf[d.jb];
    if (PT == P_FIRST) init_phase<G>(v, KF, P);
    else apply_phase<G>(v, KF, P);
    G::template trail<KIND, MIXLO>(v, buf, lane, wave, (S)mix_t(L, false), L.mode != 0);
    if (MIXLO == 0 && L.mode != 0) sw = !sw;
    if (TRUE_OUT) {
      double tr = 1.0, tq = 0.0;
      half_scale(L, K - MIXLO, false, tr, tq);
      const V sc = mkv<V>(tr, tq);
#pragma unroll
      for (int r = 0; r < NA; ++r) v[r] = cmul(v[r], sc);
    }
    store_tile<G, LA>(v, gout, lane, wave, KIND, d.a, sw);
  } else if (PT == P_LEAD) {
    if (TRUE_OUT) {
      const V sc = mkv<V>(sr, si);
#pragma unroll
      for (int r = 0; r < NA; ++r) v[r] = cmul(v[r], sc);
    }
    store_tile<G, PL>(v, gout, lane, wave, KIND, d.a, sw);
  } else {
    // outputs of the final pass carry the pending scalar
    if (d.flags & F_PROBS) {
      const S s2 = (S)(sr * sr + si * si);
      store_probs<G, PL>(v, reinterpret_cast<S*>(A.probs) + (st << n) + zb, lane, wave, KIND,
                         d.a, s2, sw);
    }
    if (d.flags & F_WRITE) {
      const V sc = mkv<V>(sr, si);
#pragma unroll
      for (int r = 0; r < NA; ++r) v[r] = cmul(v[r], sc);
      store_tile<G, PL>(v, gout, lane, wave, KIND, d.a, sw);
      sr = 1.0;
      si = 0.0;
    }
    double ae = 0.0, an = 0.0, cfix, g[G::R];
    thread_energy<G, PL>(&T, fl, cblk, lane, wave, cfix, g);
    reduce_regs<G>(v, &T, cfix, g, ae, an);
    const double s2 = sr * sr + si * si;
    const double se = block_sum(ae, tmp) * s2;
    const double sn = block_sum(an, tmp) * s2;
    if (tid == 0) {
      double* o = A.part + tile * 2;
      o[0] = se;
      o[1] = sn;
    }
  }
}

}  // namespace rt
}  // namespace dq
