// Register-tile forward pass for complex64 states (gfx950).
//
// Same pass structure as the LDS-tile pass in kernels.hip (a layer's mixer
// split into commuting qubit sets; the pass finishing layer j on a set also
// applies the phase of layer j+1 and starts layer j+1, Eq. (2) of the paper),
// but the 2^14-amplitude tile lives in registers: 256 threads (4 waves) x 64
// amplitudes, i.e. 6 "register" tile bits per thread, 6 lane bits and 2 wave
// bits.  LDS only moves tile bits between registers and lanes/waves
// (transposes), one half at a time (halves split on tile bit 0, a register
// bit in every layout), so a work-group needs about 77 KiB and two share a
// CU: while one waits at a barrier or on memory, the other computes.
//
// A half-mixer (the mixer of one layer on the pass's qubit set) runs its
// butterflies on register bits only: in each of two layouts, the tile's six
// register bits, plus lane bits 4 and 5 brought into registers by the gfx950
// lane-swap instructions (v_permlane16_swap / v_permlane32_swap exchange a
// register-pair bit with lane bit 4 / 5 at one instruction per two
// registers), with one LDS transpose between the layouts.
//
// The butterfly is the tan/cot form (two FMAs per component); the scalar c^m
// or (i s)^m of each half-mixer is left pending and folded into the next
// phase multiply, or into the outputs of the last pass.  Both forms run the
// same arithmetic, (a0, a1) -> (a0 + i t a1, a1 + i t a0): cos b I + i sin b X
// equals i sin b X (I + i t X) with t = -cot b, and the trailing X on every
// mixed qubit commutes with the whole half-mixer, so it becomes a relabelling
// of the tile.  The transpose inside the half-mixer applies it to tile bits
// 1..13 through its write and read base addresses; a flip of tile bit 0 (only
// set 0 mixes it) stays pending: the phase tables are built for the flipped
// bit and the stores swap the two amplitudes of each register pair.
//
// Phase: C(z) = cfix(thread) + sum_s r_s g_s(thread) + K(r) over the thread's
// 6 register bits r.  cfix and g come from per-tile FP64 tables in LDS (lane
// part, wave part, lane-wave cross terms); the angles gamma*cfix/2pi and
// gamma*g_s/2pi are range-reduced in FP64, and the 64 phase factors are the
// products of the 7 resulting unit complex numbers and of the per-tile factors
// e^{-i gamma K(r)}.  The last pass accumulates <C> in FP64 from the same
// decomposition.
#include "internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace dq {
namespace {

constexpr int NT14 = 256;
constexpr int HALF = 1 << 13;  // amplitudes per LDS half

// Layouts: the tile bit held by register slots 0..5, lane slots 0..5 and wave
// slots 0..1.  Register slot 0 is tile bit 0 everywhere (the transpose pivot).
//   L_A   load/store layout: lane slots are tile bits 1..6 (1 KiB runs)
//   L_A1  L_A with register slots 4, 5 swapped with lane slots 4, 5
//   L_B   set 0: the bits L_A1 leaves unmixed (1..4, 12) in registers
//   L_B1  L_B with register slot 5 swapped with lane slot 4 (bit 13 in
//         registers); phase layout of set 0
//   L_B2  other sets: bits 4, 5, 6, 12, 13 in registers; phase layout
// Set 0 mixes in A, A1 | transpose | B, B1 and back in reverse; the other
// sets in A | transpose | B2 and back.  In every layout that meets LDS (A, A1,
// B, B2) lane slots 0..3 are half-index bits whose swizzled low nibbles are
// independent, so a 16-lane group of an LDS access hits 16 distinct banks.
enum { L_A = 0, L_A1 = 1, L_B = 2, L_B1 = 3, L_B2 = 4 };
__host__ __device__ constexpr int reg_bit(int L, int s) {
  constexpr int t[5][6] = {{0, 7, 8, 9, 10, 11},
                           {0, 7, 8, 9, 5, 6},
                           {0, 1, 2, 3, 4, 12},
                           {0, 1, 2, 3, 4, 13},
                           {0, 4, 12, 13, 5, 6}};
  return t[L][s];
}
__host__ __device__ constexpr int lane_bit(int L, int s) {
  constexpr int t[5][6] = {{1, 2, 3, 4, 5, 6},
                           {1, 2, 3, 4, 10, 11},
                           {5, 6, 7, 8, 13, 9},
                           {5, 6, 7, 8, 12, 9},
                           {1, 2, 3, 8, 7, 9}};
  return t[L][s];
}
__host__ __device__ constexpr int wave_bit(int L, int s) {
  constexpr int t[5][2] = {{12, 13}, {12, 13}, {10, 11}, {10, 11}, {10, 11}};
  return t[L][s];
}

// Padded LDS slot of a half index h (tile index without bit 0): one pad slot
// per 16.  Additive over disjoint bit sets (so a register's slot is the
// thread's base plus an immediate offset), and half-index bit j moves the
// slot by 2^j (j < 4) or 2^(j-4) (4 <= j < 8) modulo 16: lane slots 0..3
// of every LDS layout take one bit from each class, so a 16-lane group of an
// access hits 16 distinct 8-byte banks.
__host__ __device__ constexpr uint32_t phys(uint32_t h) { return h + (h >> 4); }
constexpr int PHYS = HALF + (HALF >> 4);

// Half index of register index r' (register slots 1..5).
template <int L>
__host__ __device__ constexpr uint32_t reg_off(int rp) {
  uint32_t l = 0;
  for (int s = 1; s < 6; ++s)
    if ((rp >> (s - 1)) & 1) l |= 1u << reg_bit(L, s);
  return l >> 1;
}

template <int L>
__device__ __forceinline__ uint32_t thread_bits(int lane, int wave) {
  uint32_t l = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s) l |= (uint32_t)((lane >> s) & 1) << lane_bit(L, s);
#pragma unroll
  for (int s = 0; s < 2; ++s) l |= (uint32_t)((wave >> s) & 1) << wave_bit(L, s);
  return l;
}

// Global offset of tile index l: set 0 tiles are bits [0, 14); the others are
// bits [0, 4) plus [a, a + 10).
__device__ __forceinline__ uint64_t dep14(uint32_t l, int kind, int a) {
  if (kind == 1) return l;
  return (uint64_t)(l & 15u) | ((uint64_t)(l >> 4) << a);
}

// Barrier for LDS hand-offs only: the fence is restricted to the local
// address space, so it waits for this wave's LDS accesses but not for global
// loads still in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Tile bits of layout L held by lanes and waves.
template <int L>
__host__ __device__ constexpr uint32_t thread_mask() {
  uint32_t m = 0;
  for (int s = 0; s < 6; ++s) m |= 1u << lane_bit(L, s);
  for (int s = 0; s < 2; ++s) m |= 1u << wave_bit(L, s);
  return m;
}
// Move the tile from layout X to layout Y through LDS, one half at a time.
// With flip, the tile is relabelled on the way: the amplitude at tile index l
// moves to l ^ M, M = the mixed tile bits [MIXLO, 14) without bit 0.  X and Y
// share only tile bit 0 among their register bits, so every bit of M is a
// lane or wave bit of X (flipped in the write base) or of Y (flipped in the
// read base): the relabelling costs nothing per access.
template <int X, int Y, int MIXLO>
__device__ __forceinline__ void transpose(float2 (&v)[64], float2* buf, int lane, int wave,
                                          bool flip) {
  constexpr uint32_t M = ((0x3FFFu >> MIXLO) << MIXLO) & ~1u;
  constexpr uint32_t M1 = M & thread_mask<X>(), M2 = M & ~M1;
  static_assert((M2 & ~thread_mask<Y>()) == 0, "a mixed bit is a register bit of both layouts");
  const uint32_t tx = thread_bits<X>(lane, wave) ^ (flip ? M1 : 0u);
  const uint32_t ty = thread_bits<Y>(lane, wave) ^ (flip ? M2 : 0u);
  float2* const bx = buf + phys(tx >> 1);
  float2* const by = buf + phys(ty >> 1);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < 32; ++q) bx[phys(reg_off<X>(q))] = v[(q << 1) | h];
    lds_barrier();
#pragma unroll
    for (int q = 0; q < 32; ++q) v[(q << 1) | h] = by[phys(reg_off<Y>(q))];
    lds_barrier();
  }
}

// Register slots (bit s = slot s) that a round in layout L mixes: its tile
// bits not mixed earlier in the same half-mixer (DONE) and at or above the
// pass's first mixed bit.  Compile-time, so a round has no data-dependent
// control flow.
template <int L>
__host__ __device__ constexpr uint32_t reg_bits_of() {
  uint32_t m = 0;
  for (int s = 0; s < 6; ++s) m |= 1u << reg_bit(L, s);
  return m;
}
template <int L, uint32_t DONE, int MIXLO>
__host__ __device__ constexpr unsigned reg_mask() {
  unsigned m = 0;
  for (int s = 0; s < 6; ++s) {
    const int b = reg_bit(L, s);
    if (!((DONE >> b) & 1u) && b >= MIXLO) m |= 1u << s;
  }
  return m;
}

// (a0, a1) -> (a0 + i t a1, a1 + i t a0) on every register slot in RM.
template <unsigned RM>
__device__ __forceinline__ void mix_round(float2 (&v)[64], float t) {
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    if (!((RM >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < 64; ++r) {
      if ((r >> s) & 1) continue;
      float2& a0 = v[r];
      float2& a1 = v[r | (1 << s)];
      const float x0 = a0.x, y0 = a0.y, x1 = a1.x, y1 = a1.y;
      a0.x = fmaf(-t, y1, x0);
      a0.y = fmaf(t, x1, y0);
      a1.x = fmaf(-t, y0, x1);
      a1.y = fmaf(t, x0, y1);
      // bound the butterflies in flight (each needs fresh registers until
      // both of its inputs are dead)
      if ((r & 15) == 14 || (r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Exchange register slot SR with lane slot SL (4 or 5) for the whole tile.
template <int SR, int SL>
__device__ __forceinline__ void swap_slot(float2 (&v)[64]) {
  static_assert(SL == 4 || SL == 5, "lane slots 4 and 5 only");
#pragma unroll
  for (int r = 0; r < 64; ++r) {
    if ((r >> SR) & 1) continue;
    float2& a0 = v[r];
    float2& a1 = v[r | (1 << SR)];
    const unsigned x0 = __builtin_bit_cast(unsigned, a0.x);
    const unsigned x1 = __builtin_bit_cast(unsigned, a1.x);
    const unsigned y0 = __builtin_bit_cast(unsigned, a0.y);
    const unsigned y1 = __builtin_bit_cast(unsigned, a1.y);
    unsigned nx0, nx1, ny0, ny1;
    if (SL == 5) {
      const auto px = __builtin_amdgcn_permlane32_swap(x0, x1, false, false);
      const auto py = __builtin_amdgcn_permlane32_swap(y0, y1, false, false);
      nx0 = px[0], nx1 = px[1], ny0 = py[0], ny1 = py[1];
    } else {
      const auto px = __builtin_amdgcn_permlane16_swap(x0, x1, false, false);
      const auto py = __builtin_amdgcn_permlane16_swap(y0, y1, false, false);
      nx0 = px[0], nx1 = px[1], ny0 = py[0], ny1 = py[1];
    }
    a0 = make_float2(__builtin_bit_cast(float, nx0), __builtin_bit_cast(float, ny0));
    a1 = make_float2(__builtin_bit_cast(float, nx1), __builtin_bit_cast(float, ny1));
  }
}

// Lead half-mixer: from the load layout L_A to the phase layout; trail
// half-mixer: back.  flip (cot form) relabels the tile inside the transpose.
template <int KIND, int MIXLO>
__device__ __forceinline__ void lead_mixer(float2 (&v)[64], float2* buf, int lane, int wave,
                                           float t, bool flip) {
  if constexpr (KIND == 1) {
    constexpr uint32_t D1 = reg_bits_of<L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<L_A1>();
    constexpr uint32_t D3 = D2 | reg_bits_of<L_B>();
    mix_round<reg_mask<L_A, 0, MIXLO>()>(v, t);
    swap_slot<4, 4>(v);
    swap_slot<5, 5>(v);
    mix_round<reg_mask<L_A1, D1, MIXLO>()>(v, t);
    transpose<L_A1, L_B, MIXLO>(v, buf, lane, wave, flip);
    mix_round<reg_mask<L_B, D2, MIXLO>()>(v, t);
    swap_slot<5, 4>(v);
    mix_round<reg_mask<L_B1, D3, MIXLO>()>(v, t);
  } else {
    constexpr uint32_t D1 = reg_bits_of<L_A>();
    mix_round<reg_mask<L_A, 0, MIXLO>()>(v, t);
    transpose<L_A, L_B2, MIXLO>(v, buf, lane, wave, flip);
    mix_round<reg_mask<L_B2, D1, MIXLO>()>(v, t);
  }
}
template <int KIND, int MIXLO>
__device__ __forceinline__ void trail_mixer(float2 (&v)[64], float2* buf, int lane, int wave,
                                            float t, bool flip) {
  if constexpr (KIND == 1) {
    constexpr uint32_t D1 = reg_bits_of<L_B1>();
    constexpr uint32_t D2 = D1 | reg_bits_of<L_B>();
    constexpr uint32_t D3 = D2 | reg_bits_of<L_A1>();
    mix_round<reg_mask<L_B1, 0, MIXLO>()>(v, t);
    swap_slot<5, 4>(v);
    mix_round<reg_mask<L_B, D1, MIXLO>()>(v, t);
    transpose<L_B, L_A1, MIXLO>(v, buf, lane, wave, flip);
    mix_round<reg_mask<L_A1, D2, MIXLO>()>(v, t);
    swap_slot<4, 4>(v);
    swap_slot<5, 5>(v);
    mix_round<reg_mask<L_A, D3, MIXLO>()>(v, t);
  } else {
    constexpr uint32_t D1 = reg_bits_of<L_B2>();
    mix_round<reg_mask<L_B2, 0, MIXLO>()>(v, t);
    transpose<L_B2, L_A, MIXLO>(v, buf, lane, wave, flip);
    mix_round<reg_mask<L_A, D1, MIXLO>()>(v, t);
  }
}

// Arithmetic parameter of a half-mixer.
template <int MIXLO>
__device__ __forceinline__ float mix_t(const LayerCoef& L) {
  return L.mode == 0 ? (float)L.tb : -(float)L.tb;
}

// Complex helpers.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
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

// Mixer scalar of one half-mixer: c^m (mode 0) or (i s)^m (mode 1),
// multiplied into (re, im).
__device__ __forceinline__ void half_scale(const LayerCoef& L, int m, double& re, double& im) {
  double r = 1.0, i = 0.0;
  if (L.mode == 0) {
    for (int q = 0; q < m; ++q) r *= L.cb;
  } else {
    for (int q = 0; q < m; ++q) {
      const double nr = -i * L.sb, ni = r * L.sb;
      r = nr;
      i = ni;
    }
  }
  const double nr = re * r - im * i, ni = re * i + im * r;
  re = nr;
  im = ni;
}

struct F14Args {
  PassDesc d;
  int S, p;
  const float2* in;
  float2* out;
  uint64_t stride;
  const double* W;
  const LayerCoef* coef;
  double* part;
  float* probs;
};

// Per-tile tables for the phase layout PL (FP64):
//   Ll[64]    energy of the lane bits alone (with their block fields)
//   Gl[6][64] field of the lane bits on register slot s
//   Lw[4]     energy of the wave bits alone
//   Fw[6][4]  coupling of lane slot i to the wave bits
//   Gw[6][4]  field of the wave bits on register slot s
//   Kr[64]    couplings among the register bits
struct Tables {
  double Ll[64], Gl[6][64], Lw[4], Fw[6][4], Gw[6][4], Kr[64];
};
constexpr int NTAB = 64 + 6 * 64 + 4 + 6 * 4 + 6 * 4 + 64;

template <int PL>
__device__ __forceinline__ void table_entry(Tables* T, const double* fl, const double* Wl,
                                            int e) {
  if (e < 64) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i)
      if ((e >> i) & 1) {
        const int bi = lane_bit(PL, i);
        s += fl[bi];
        for (int j = 0; j < i; ++j)
          if ((e >> j) & 1) s += Wl[bi * 14 + lane_bit(PL, j)];
      }
    T->Ll[e] = s;
    return;
  }
  e -= 64;
  if (e < 6 * 64) {
    const int sl = e >> 6, x = e & 63, br = reg_bit(PL, sl);
    double s = 0.0;
    for (int i = 0; i < 6; ++i)
      if ((x >> i) & 1) s += Wl[br * 14 + lane_bit(PL, i)];
    T->Gl[sl][x] = s;
    return;
  }
  e -= 6 * 64;
  if (e < 4) {
    double s = 0.0;
    for (int i = 0; i < 2; ++i)
      if ((e >> i) & 1) {
        const int bi = wave_bit(PL, i);
        s += fl[bi];
        for (int j = 0; j < i; ++j)
          if ((e >> j) & 1) s += Wl[bi * 14 + wave_bit(PL, j)];
      }
    T->Lw[e] = s;
    return;
  }
  e -= 4;
  if (e < 6 * 4) {
    const int li = e >> 2, y = e & 3, bl = lane_bit(PL, li);
    double s = 0.0;
    for (int j = 0; j < 2; ++j)
      if ((y >> j) & 1) s += Wl[bl * 14 + wave_bit(PL, j)];
    T->Fw[li][y] = s;
    return;
  }
  e -= 6 * 4;
  if (e < 6 * 4) {
    const int sl = e >> 2, y = e & 3, br = reg_bit(PL, sl);
    double s = 0.0;
    for (int j = 0; j < 2; ++j)
      if ((y >> j) & 1) s += Wl[br * 14 + wave_bit(PL, j)];
    T->Gw[sl][y] = s;
    return;
  }
  e -= 6 * 4;
  if (e < 64) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i)
      if ((e >> i) & 1)
        for (int j = 0; j < i; ++j)
          if ((e >> j) & 1) s += Wl[reg_bit(PL, i) * 14 + reg_bit(PL, j)];
    T->Kr[e] = s;
  }
}

// The thread's cfix and fields g_s in the phase layout (FP64).  Branch-free,
// so that it does not split the straight-line code around it.
template <int PL>
__device__ __forceinline__ void thread_energy(const Tables* T, const double* fl, double cblk,
                                              int lane, int wave, double& cfix, double (&g)[6]) {
  double c = cblk + T->Lw[wave] + T->Ll[lane];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double f = T->Fw[i][wave];
    c += ((lane >> i) & 1) ? f : 0.0;
  }
  cfix = c;
#pragma unroll
  for (int s = 0; s < 6; ++s) g[s] = fl[reg_bit(PL, s)] + T->Gl[s][lane] + T->Gw[s][wave];
}

// Per-thread phase factors of one layer: f0 = e^{-i gamma cfix} times the
// pending mixer scalar, fs[s] = e^{-i gamma g_s}.
struct PhaseF {
  float2 f0, fs[6];
};
template <int PL>
__device__ __forceinline__ PhaseF phase_factors(const Tables* T, const double* fl, double cblk,
                                                int lane, int wave, double gp, double sr,
                                                double si) {
  double cfix, g[6];
  thread_energy<PL>(T, fl, cblk, lane, wave, cfix, g);
  PhaseF P;
  P.f0 = cmul(unit(gp * cfix), make_float2((float)sr, (float)si));
#pragma unroll
  for (int s = 0; s < 6; ++s) P.fs[s] = unit(gp * g[s]);
  return P;
}

// Phase of one layer on the 64 register amplitudes: amplitude r is
// multiplied by f0 * prod_{s in r} fs[s] * KF[r].
__device__ __forceinline__ void apply_phase(float2 (&v)[64], const float2* KF, const PhaseF& P) {
#pragma unroll
  for (int r5 = 0; r5 < 2; ++r5) {
    const float2 p5 = r5 ? cmul(P.f0, P.fs[5]) : P.f0;
#pragma unroll
    for (int r4 = 0; r4 < 2; ++r4) {
      const float2 p4 = r4 ? cmul(p5, P.fs[4]) : p5;
#pragma unroll
      for (int r3 = 0; r3 < 2; ++r3) {
        const float2 p3 = r3 ? cmul(p4, P.fs[3]) : p4;
#pragma unroll
        for (int r2 = 0; r2 < 2; ++r2) {
          const float2 p2 = r2 ? cmul(p3, P.fs[2]) : p3;
#pragma unroll
          for (int r1 = 0; r1 < 2; ++r1) {
            const float2 p1 = r1 ? cmul(p2, P.fs[1]) : p2;
#pragma unroll
            for (int r0 = 0; r0 < 2; ++r0) {
              const float2 p0 = r0 ? cmul(p1, P.fs[0]) : p1;
              const int r = r0 | (r1 << 1) | (r2 << 2) | (r3 << 3) | (r4 << 4) | (r5 << 5);
              v[r] = cmul(v[r], cmul(p0, KF[r]));
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
  }
}

// <C> and norm partial sums of the 64 register amplitudes, FP64, from the
// thread's cfix and fields g (thread_energy).
__device__ __forceinline__ void reduce_regs(const float2 (&v)[64], const Tables* T, double cfix,
                                            const double (&g)[6], double& ae, double& an) {
#pragma unroll
  for (int hi = 0; hi < 8; ++hi) {  // register bits 3..5
    double ch = cfix;
#pragma unroll
    for (int s = 3; s < 6; ++s)
      if ((hi >> (s - 3)) & 1) ch += g[s];
#pragma unroll
    for (int lo = 0; lo < 8; ++lo) {  // register bits 0..2
      const int r = (hi << 3) | lo;
      double c = ch + T->Kr[r];
#pragma unroll
      for (int s = 0; s < 3; ++s)
        if ((lo >> s) & 1) c += g[s];
      const double pz = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
      ae = fma(pz, c, ae);
      an += pz;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Global load/store of the register tile in layout L (the two amplitudes of a
// register pair differ in tile bit 0 and move as one 16-byte access).
template <int L>
__device__ __forceinline__ void load_tile(float2 (&v)[64], const float2* base, int lane, int wave,
                                          int kind, int a) {
  const uint64_t tb = dep14(thread_bits<L>(lane, wave), kind, a);
#pragma unroll
  for (int rp = 0; rp < 32; ++rp) {
    const uint64_t o = tb + dep14(reg_off<L>(rp) << 1, kind, a);
    const float4 q = *reinterpret_cast<const float4*>(base + o);
    v[rp << 1] = make_float2(q.x, q.y);
    v[(rp << 1) | 1] = make_float2(q.z, q.w);
  }
}

// sw: tile bit 0 is flipped (the register pair is stored in swapped order).
// sw: tile bit 0 is flipped (each register pair is stored in swapped
// order).  The two orders are separate loops, not per-element selects.
template <int L, bool SW>
__device__ __forceinline__ void store_rows(const float2 (&v)[64], float2* base, uint64_t tb,
                                           int kind, int a) {
#pragma unroll
  for (int rp = 0; rp < 32; ++rp) {
    const uint64_t o = tb + dep14(reg_off<L>(rp) << 1, kind, a);
    const float2 u = v[(rp << 1) | SW], w = v[(rp << 1) | !SW];
    *reinterpret_cast<float4*>(base + o) = make_float4(u.x, u.y, w.x, w.y);
  }
}
template <int L>
__device__ __forceinline__ void store_tile(const float2 (&v)[64], float2* base, int lane, int wave,
                                           int kind, int a, bool sw) {
  const uint64_t tb = dep14(thread_bits<L>(lane, wave), kind, a);
  if (sw) store_rows<L, true>(v, base, tb, kind, a);
  else store_rows<L, false>(v, base, tb, kind, a);
}

template <int L, bool SW>
__device__ __forceinline__ void store_prob_rows(const float2 (&v)[64], float* base, uint64_t tb,
                                                int kind, int a, float scale) {
#pragma unroll
  for (int rp = 0; rp < 32; ++rp) {
    const uint64_t o = tb + dep14(reg_off<L>(rp) << 1, kind, a);
    const float2 u = v[(rp << 1) | SW], w = v[(rp << 1) | !SW];
    *reinterpret_cast<float2*>(base + o) =
        make_float2(scale * (u.x * u.x + u.y * u.y), scale * (w.x * w.x + w.y * w.y));
  }
}
template <int L>
__device__ __forceinline__ void store_probs(const float2 (&v)[64], float* base, int lane,
                                            int wave, int kind, int a, float scale, bool sw) {
  const uint64_t tb = dep14(thread_bits<L>(lane, wave), kind, a);
  if (sw) store_prob_rows<L, true>(v, base, tb, kind, a, scale);
  else store_prob_rows<L, false>(v, base, tb, kind, a, scale);
}

__device__ __forceinline__ double bsum14(double x, double* red) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  lds_barrier();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  lds_barrier();
  double s = 0.0;
  for (int i = 0; i < NT14 / 64; ++i) s += red[i];
  lds_barrier();
  return s;
}

// Pass shapes (every pass of a register-tile plan is one of these):
//   P_FIRST  initial state, phase, half-mixer PL -> LA, store (set 0)
//   P_MID    load, lead half-mixer LA -> PL, phase, half-mixer PL -> LA, store
//   P_LEAD   load, lead half-mixer LA -> PL, store (sets between the ends of a
//            layer when there are more than two)
//   P_LAST   load, lead half-mixer LA -> PL, <C>/norm partials and the
//            optional probability and state outputs
enum { P_FIRST = 0, P_MID = 1, P_LEAD = 2, P_LAST = 3 };

// One tile of one pass per work-group (tile index = state * 2^(n-14) + tile
// of the state).  Layout 0 is the load/store layout and PL the phase layout;
// the pass mixes tile bits [MIXLO, 14).  One straight-line body per pass
// shape keeps the 128 registers of the tile in place from load to store.
template <int KIND, int MIXLO, int PT>
__global__ void __launch_bounds__(NT14) __attribute__((amdgpu_waves_per_eu(2)))
fwd14_kernel(F14Args A) {
  constexpr int LA = L_A, PL = KIND == 1 ? L_B1 : L_B2;
  constexpr bool LEAD = PT != P_FIRST, PHASE = PT == P_FIRST || PT == P_MID;
  __shared__ float2 buf[PHYS];
  __shared__ Tables T;
  __shared__ double fl[14];
  __shared__ double Wl[14 * 14];
  __shared__ double tmp[40];
  __shared__ float2 KF[64];
  __shared__ LayerCoef cf[64];
  const PassDesc& d = A.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = d.n, nlog = n - 14;
  const uint64_t tile = blockIdx.x;
  const uint64_t st = tile >> nlog, ti = tile & ((1ull << nlog) - 1ull);
  uint64_t zb;
  if (KIND == 1) {
    zb = ti << 14;
  } else {
    const int gap = d.a - 4;
    zb = ((ti & ((1ull << gap) - 1ull)) << 4) | ((ti >> gap) << (d.a + 10));
  }
  // The folded Q and the state's layer coefficients are read first, then the
  // tile's own loads are issued, and Q and the coefficients are staged in LDS
  // (the transpose buffer is idle until the first transpose) while the tile
  // is in flight; the tile context is built from LDS meanwhile.
  const double* W = A.W + (size_t)(st / A.S) * n * n;
  const int nn = n * n;
  double wr[(34 * 34 + NT14 - 1) / NT14];
#pragma unroll
  for (int k = 0; k < (34 * 34 + NT14 - 1) / NT14; ++k) {
    const int e = tid + k * NT14;
    wr[k] = e < nn ? W[e] : 0.0;
  }
  static_assert(sizeof(LayerCoef) == 40, "layer coefficients move as five doubles");
  double cv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (tid < A.p) {
    const double* c = reinterpret_cast<const double*>(A.coef + st * A.p + tid);
#pragma unroll
    for (int k = 0; k < 5; ++k) cv[k] = c[k];
  }
  __builtin_amdgcn_sched_barrier(0);
  float2 v[64];
  if (PT == P_FIRST) {
    const float amp = (float)exp2(-0.5 * (double)n);
#pragma unroll
    for (int r = 0; r < 64; ++r) v[r] = make_float2(amp, 0.0f);
  } else {
    load_tile<LA>(v, A.in + st * A.stride + zb, lane, wave, KIND, d.a);
  }
  __builtin_amdgcn_sched_barrier(0);
  double* const Wsh = reinterpret_cast<double*>(buf);
#pragma unroll
  for (int k = 0; k < (34 * 34 + NT14 - 1) / NT14; ++k) {
    const int e = tid + k * NT14;
    if (e < nn) Wsh[e] = wr[k];
  }
  if (tid < A.p) {
    double* c = reinterpret_cast<double*>(cf + tid);
#pragma unroll
    for (int k = 0; k < 5; ++k) c[k] = cv[k];
  }
  lds_barrier();
  // Tile context: block fields on the tile bits, couplings among the tile
  // bits, the energy of the block bits.  With tile bit 0 flipped after the
  // lead half-mixer (cot form on set 0), the tile-local energy is that of
  // z ^ 1: the field and couplings of bit 0 change sign, the other fields
  // gain their coupling to bit 0, and the constant gains the old field of
  // bit 0.
  const bool f0 = KIND == 1 && LEAD && cf[d.lead].mode != 0;
  if (tid < 14) {
    const int pi = (KIND == 1 || tid < 4) ? tid : d.a + tid - 4;
    double f = Wsh[pi * n + pi];
    for (int j = 0; j < n; ++j)
      if ((zb >> j) & 1ull) f += Wsh[pi * n + j];
    if (f0) f = tid == 0 ? -f : f + Wsh[pi * n];
    fl[tid] = f;
  } else if (tid >= 64 && tid <= 64 + n) {
    const int i = tid - 64;
    double t = 0.0;
    if (i == n) {  // old field of bit 0 (kind 1: tile bit 0 is qubit 0)
      if (f0) {
        t = Wsh[0];
        for (int j = 0; j < n; ++j)
          if ((zb >> j) & 1ull) t += Wsh[j];
      }
    } else if ((zb >> i) & 1ull) {
      t = Wsh[i * n + i];
      for (int j = 0; j < i; ++j)
        if ((zb >> j) & 1ull) t += Wsh[i * n + j];
    }
    tmp[i] = t;
  }
  if (tid < 196) {
    const int i = tid / 14, j = tid - 14 * i;
    const int pi = (KIND == 1 || i < 4) ? i : d.a + i - 4;
    const int pj = (KIND == 1 || j < 4) ? j : d.a + j - 4;
    const double w = (i == j) ? 0.0 : Wsh[pi * n + pj];
    Wl[tid] = (f0 && (i == 0) != (j == 0)) ? -w : w;
  }
  lds_barrier();
  double cblk = 0.0;
  for (int i = 0; i <= n; ++i) cblk += tmp[i];
  if (PT != P_LEAD)
    for (int e = tid; e < NTAB; e += NT14) table_entry<PL>(&T, fl, Wl, e);
  if (PHASE && tid < 64) {
    const LayerCoef& L = cf[d.jb];
    // Kr of this thread's entry, computed here rather than read back
    double k = 0.0;
    for (int i = 0; i < 6; ++i)
      if ((tid >> i) & 1)
        for (int j = 0; j < i; ++j)
          if ((tid >> j) & 1) k += Wl[reg_bit(PL, i) * 14 + reg_bit(PL, j)];
    KF[tid] = unit(L.gp * k);
  }
  lds_barrier();

  // pending mixer scalar (at the phase, or at the outputs of the last pass)
  double sr = 1.0, si = 0.0;
  for (int i = 0; i < d.pend_n; ++i) half_scale(cf[d.pend_layer[i]], d.pend_m[i], sr, si);
  if (LEAD) half_scale(cf[d.lead], 14 - MIXLO, sr, si);
  // per-thread phase factors, or energies for <C>, before the tile arrives
  PhaseF P;
  double cfix = 0.0, g[6];
  if (PHASE) P = phase_factors<PL>(&T, fl, cblk, lane, wave, cf[d.jb].gp, sr, si);
  bool sw = f0;  // tile bit 0 is flipped
  if (LEAD) {
    const LayerCoef& L = cf[d.lead];
    lead_mixer<KIND, MIXLO>(v, buf, lane, wave, mix_t<MIXLO>(L), L.mode != 0);
  }
  if (PHASE) {
    const LayerCoef& L = cf[d.jb];
    apply_phase(v, KF, P);
    trail_mixer<KIND, MIXLO>(v, buf, lane, wave, mix_t<MIXLO>(L), L.mode != 0);
    if (KIND == 1 && L.mode != 0) sw = !sw;
    store_tile<LA>(v, A.out + st * A.stride + zb, lane, wave, KIND, d.a, sw);
  } else if (PT == P_LEAD) {
    store_tile<PL>(v, A.out + st * A.stride + zb, lane, wave, KIND, d.a, sw);
  } else {
    // outputs of the final pass carry the pending scalar
    if (d.flags & F_PROBS) {
      const float s2 = (float)(sr * sr + si * si);
      store_probs<PL>(v, A.probs + (st << n) + zb, lane, wave, KIND, d.a, s2, sw);
    }
    if (d.flags & F_WRITE) {
      const float2 sc = make_float2((float)sr, (float)si);
#pragma unroll
      for (int r = 0; r < 64; ++r) v[r] = cmul(v[r], sc);
      store_tile<PL>(v, A.out + st * A.stride + zb, lane, wave, KIND, d.a, sw);
      sr = 1.0;
      si = 0.0;
    }
    double ae = 0.0, an = 0.0;
    thread_energy<PL>(&T, fl, cblk, lane, wave, cfix, g);
    reduce_regs(v, &T, cfix, g, ae, an);
    const double s2 = sr * sr + si * si;
    const double se = bsum14(ae, tmp) * s2;
    const double sn = bsum14(an, tmp) * s2;
    if (tid == 0) {
      double* o = A.part + tile * 2;
      o[0] = se;
      o[1] = sn;
    }
  }
}

}  // namespace

hipError_t launch_fwd14_pass(const PassDesc& d, int nstates, int S, int p,
                             const void* in, void* out, uint64_t state_stride,
                             const double* W, const LayerCoef* coef,
                             double* part, void* probs, hipStream_t stream) {
  if (d.n < 15 || d.n > 34 || p < 1 || p > 64 || nstates < 1 || S < 1)
    return hipErrorInvalidValue;
  const bool phase = d.ja <= d.jb;
  if (phase && (d.ja != d.jb || d.jb < 0 || d.jb >= p)) return hipErrorInvalidValue;
  if (d.lead >= p) return hipErrorInvalidValue;
  int pt;
  if (d.flags & F_INIT) pt = (d.lead < 0 && phase && d.kind == 1 && (d.flags & F_WRITE) &&
                              !(d.flags & F_REDUCE)) ? P_FIRST : -1;
  else if (d.lead < 0) pt = -1;
  else if (d.flags & F_REDUCE) pt = phase ? -1 : P_LAST;
  else if (!(d.flags & F_WRITE)) pt = -1;
  else pt = phase ? P_MID : P_LEAD;
  if (pt < 0 || (d.kind == 1 && pt == P_LEAD)) return hipErrorInvalidValue;
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 4 || d.mixlo > 13)) return hipErrorInvalidValue;
  F14Args A;
  A.d = d;
  A.S = S;
  A.p = p;
  A.in = reinterpret_cast<const float2*>(in);
  A.out = reinterpret_cast<float2*>(out);
  A.stride = state_stride;
  A.W = W;
  A.coef = coef;
  A.part = part;
  A.probs = reinterpret_cast<float*>(probs);
  const uint64_t total = (uint64_t)nstates << (d.n - 14);

  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT14);
#define DQ_K(K, M, T) hipLaunchKernelGGL((fwd14_kernel<K, M, T>), grid, blk, 0, stream, A)
#define DQ_PT(K, M)                         \
  switch (pt) {                             \
    case P_MID: DQ_K(K, M, P_MID); break;   \
    case P_LEAD: DQ_K(K, M, P_LEAD); break; \
    default: DQ_K(K, M, P_LAST); break;     \
  }
  if (d.kind == 1) {
    switch (pt) {
      case P_FIRST: DQ_K(1, 0, P_FIRST); break;
      case P_MID: DQ_K(1, 0, P_MID); break;
      default: DQ_K(1, 0, P_LAST); break;
    }
  } else {
    switch (d.mixlo) {
      case 4: DQ_PT(2, 4); break;
      case 5: DQ_PT(2, 5); break;
      case 6: DQ_PT(2, 6); break;
      case 7: DQ_PT(2, 7); break;
      case 8: DQ_PT(2, 8); break;
      case 9: DQ_PT(2, 9); break;
      case 10: DQ_PT(2, 10); break;
      case 11: DQ_PT(2, 11); break;
      case 12: DQ_PT(2, 12); break;
      default: DQ_PT(2, 13); break;
    }
  }
#undef DQ_PT
#undef DQ_K
  return hipGetLastError();
}

}  // namespace dq
