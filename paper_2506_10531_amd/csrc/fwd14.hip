// Register-tile forward pass for complex64 states (gfx950).
//
// Same pass structure as the LDS-tile pass in kernels.hip (a layer's mixer
// split into commuting qubit sets; the pass finishing layer j on a set also
// applies the phase of layer j+1 and starts layer j+1, Eq. (2) of the paper),
// but the 2^14-amplitude tile lives in registers: 512 threads x 32 amplitudes
// (5 "register" tile bits per thread; 6 lane bits; 3 wave bits).  LDS is only
// used to move tile bits between registers and lanes/waves (transposes), in
// two 64 KiB halves split on tile bit 0 (a register bit in every layout), so
// two work-groups fit in one CU's 160 KiB and overlap each other's memory and
// compute phases.
//
// A half-mixer (the mixer of one layer on one qubit set) visits three layouts;
// in each, the butterflies of its register bits run in registers and those of
// lane bits 0 and 1 run across lanes with DPP quad permutes.  The butterfly is
// the tan/cot form (two FMAs per component); the scalar c^m or (i s)^m of each
// half-mixer is left pending and folded into the next phase multiply, or into
// the outputs of the last pass.
//
// Phase: C(z) = cfix(thread) + sum_s r_s g_s(thread) + K(r) over the thread's
// 5 register bits r.  cfix and g come from per-tile tables (lane part, wave
// part, lane-wave cross terms) built in LDS in FP64; the angles gamma*cfix/2pi
// and gamma*g_s/2pi are range-reduced in FP64, and the 32 phase factors are
// the products of the 6 resulting unit complex numbers and of the per-tile
// factors e^{-i gamma K(r)}.  The last pass accumulates <C> in FP64 from the
// same decomposition.
#include "internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace dq {
namespace {

constexpr int NT14 = 512;
constexpr int HALF = 1 << 13;                // amplitudes per LDS half
constexpr int PHYS = HALF + (HALF >> 4);     // padded slots per half

// Layouts: the tile bit held by register slots 0..4, lane slots 0..5 and wave
// slots 0..2.  Register slot 0 is tile bit 0 everywhere (the transpose pivot).
//   0: A  (load/store)   1: B (set 0)   2: C (set 0, phase)
//   3: B' (other sets)   4: C' (other sets, phase)
__host__ __device__ constexpr int reg_bit(int L, int s) {
  constexpr int t[5][5] = {{0, 7, 8, 9, 10},
                           {0, 3, 4, 5, 6},
                           {0, 11, 12, 13, 5},
                           {0, 4, 5, 6, 11},
                           {0, 12, 13, 5, 6}};
  return t[L][s];
}
__host__ __device__ constexpr int lane_bit(int L, int s) {
  constexpr int t[5][6] = {{1, 2, 3, 4, 5, 6},
                           {1, 2, 7, 8, 9, 10},
                           {1, 2, 3, 4, 6, 7},
                           {1, 2, 7, 8, 3, 9},
                           {1, 2, 3, 4, 7, 8}};
  return t[L][s];
}
__host__ __device__ constexpr int wave_bit(int L, int s) {
  constexpr int t[5][3] = {{11, 12, 13}, {11, 12, 13}, {8, 9, 10},
                           {10, 12, 13}, {9, 10, 11}};
  return t[L][s];
}

// Padded LDS slot of a half index (tile index without bit 0): one pad slot
// per 16.  Additive over disjoint bit sets, and every layout's lane slots 0..3
// land on half-index bits whose padded strides are 1, 2, 4 and 8 slots (mod
// 16), so every 16-lane group of an access hits 16 distinct 8-byte banks.
__host__ __device__ constexpr uint32_t phys(uint32_t h) { return h + (h >> 4); }

// Half-index offset of register index r' (register slots 1..4).
template <int L>
__host__ __device__ constexpr uint32_t reg_off(int rp) {
  uint32_t l = 0;
  for (int s = 1; s < 5; ++s)
    if ((rp >> (s - 1)) & 1) l |= 1u << reg_bit(L, s);
  return l >> 1;
}

template <int L>
__device__ __forceinline__ uint32_t thread_bits(int lane, int wave) {
  uint32_t l = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s) l |= (uint32_t)((lane >> s) & 1) << lane_bit(L, s);
#pragma unroll
  for (int s = 0; s < 3; ++s) l |= (uint32_t)((wave >> s) & 1) << wave_bit(L, s);
  return l;
}

// Global offset of tile index l: set 0 tiles are bits [0, 14); the others are
// bits [0, 4) plus [a, a + 10).
__device__ __forceinline__ uint64_t dep14(uint32_t l, int kind, int a) {
  if (kind == 1) return l;
  return (uint64_t)(l & 15u) | ((uint64_t)(l >> 4) << a);
}

// Barrier for LDS hand-offs only: the fence is restricted to the local
// address space, so it waits for this wave's LDS accesses but not for the
// global loads of the next tile that are still in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Move the tile from layout X to layout Y through LDS, one half at a time.
template <int X, int Y>
__device__ __forceinline__ void transpose(float2 (&v)[32], float2* buf, int lane, int wave) {
  const uint32_t bx = phys(thread_bits<X>(lane, wave) >> 1);
  const uint32_t by = phys(thread_bits<Y>(lane, wave) >> 1);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int rp = 0; rp < 16; ++rp) buf[bx + phys(reg_off<X>(rp))] = v[(rp << 1) | h];
    lds_barrier();
#pragma unroll
    for (int rp = 0; rp < 16; ++rp) v[(rp << 1) | h] = buf[by + phys(reg_off<Y>(rp))];
    lds_barrier();
  }
}

__device__ __forceinline__ float dpp_x1(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x),
                                                            0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_x2(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x),
                                                            0x4E, 0xF, 0xF, true));
}

// Tile bits a layout's register slots and DPP lane slots touch.
template <int L>
__host__ __device__ constexpr uint32_t layout_mixable() {
  uint32_t m = 0;
  for (int s = 0; s < 5; ++s) m |= 1u << reg_bit(L, s);
  m |= 1u << lane_bit(L, 0);
  m |= 1u << lane_bit(L, 1);
  return m;
}

// Register slots (bit s = slot s) and DPP lane slots (bit 0 = lane bit 0,
// bit 1 = lane bit 1) that a round in layout L mixes: its tile bits not mixed
// earlier in the same half-mixer (DONE) and at or above the pass's first
// mixed bit.  All compile-time, so a round has no data-dependent control flow.
template <int L, uint32_t DONE, int MIXLO>
__host__ __device__ constexpr unsigned reg_mask() {
  unsigned m = 0;
  for (int s = 0; s < 5; ++s) {
    const int b = reg_bit(L, s);
    if (!((DONE >> b) & 1u) && b >= MIXLO) m |= 1u << s;
  }
  return m;
}
template <int L, uint32_t DONE, int MIXLO>
__host__ __device__ constexpr unsigned dpp_mask() {
  unsigned m = 0;
  for (int s = 0; s < 2; ++s) {
    const int b = lane_bit(L, s);
    if (!((DONE >> b) & 1u) && b >= MIXLO) m |= 1u << s;
  }
  return m;
}

template <int MODE, unsigned RM, unsigned DM>
__device__ __forceinline__ void mix_round(float2 (&v)[32], float t) {
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    if (!((RM >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      if ((r >> s) & 1) continue;
      float2& a0 = v[r];
      float2& a1 = v[r | (1 << s)];
      const float x0 = a0.x, y0 = a0.y, x1 = a1.x, y1 = a1.y;
      if (MODE == 0) {
        a0.x = fmaf(-t, y1, x0);
        a0.y = fmaf(t, x1, y0);
        a1.x = fmaf(-t, y0, x1);
        a1.y = fmaf(t, x0, y1);
      } else {
        a0.x = fmaf(t, y0, x1);
        a0.y = fmaf(-t, x0, y1);
        a1.x = fmaf(t, y1, x0);
        a1.y = fmaf(-t, x1, y0);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!((DM >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const float x = v[r].x, y = v[r].y;
      const float xp = s == 0 ? dpp_x1(x) : dpp_x2(x);
      const float yp = s == 0 ? dpp_x1(y) : dpp_x2(y);
      if (MODE == 0) {
        v[r].x = fmaf(-t, yp, x);
        v[r].y = fmaf(t, xp, y);
      } else {
        v[r].x = fmaf(t, y, xp);
        v[r].y = fmaf(-t, x, yp);
      }
      // keep the DPP temporaries of only a few amplitudes live at a time
      if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// One half-mixer (the mixer of one layer on the pass's qubit set): rounds in
// layouts X, Y, Z with transposes X -> Y -> Z between them.
template <int MODE, int X, int Y, int Z, int MIXLO>
__device__ __forceinline__ void half_mixer(float2 (&v)[32], float2* buf, int lane, int wave,
                                           float t) {
  constexpr uint32_t D1 = layout_mixable<X>();
  constexpr uint32_t D2 = D1 | layout_mixable<Y>();
  mix_round<MODE, reg_mask<X, 0, MIXLO>(), dpp_mask<X, 0, MIXLO>()>(v, t);
  transpose<X, Y>(v, buf, lane, wave);
  mix_round<MODE, reg_mask<Y, D1, MIXLO>(), dpp_mask<Y, D1, MIXLO>()>(v, t);
  transpose<Y, Z>(v, buf, lane, wave);
  mix_round<MODE, reg_mask<Z, D2, MIXLO>(), dpp_mask<Z, D2, MIXLO>()>(v, t);
}

// Complex helpers.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 unit(double rev) {  // e^{-i 2 pi rev}
  const double t = rev - rint(rev);
  float s, c;
  sincospif(2.0f * (float)t, &s, &c);
  return make_float2(c, -s);
}

// Mixer scalar of one half-mixer: c^m (mode 0) or (i s)^m (mode 1).
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
  int S, p, nstates;
  const float2* in;
  float2* out;
  uint64_t stride;
  const double* W;
  const LayerCoef* coef;
  double* part;
  float* probs;
};

// Per-tile tables for the phase layout PL (FP64), 512 entries:
//   Ll[64]   energy of the lane bits alone (with their block fields)
//   Gl[5][64] field of the lane bits on register slot s
//   Lw[8]    energy of the wave bits alone
//   Fw[6][8] coupling of lane slot i to the wave bits
//   Gw[5][8] field of the wave bits on register slot s
//   Kr[32]   couplings among the register bits
struct Tables {
  double Ll[64], Gl[5][64], Lw[8], Fw[6][8], Gw[5][8], Kr[32];
};

template <int PL>
__device__ __forceinline__ void build_tables(Tables* T, const double* fl, const double* Wl, int tid) {
  // every thread fills at most one entry (512 entries in total)
  int e = tid;
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
  if (e < 320) {
    const int sl = e >> 6, x = e & 63, br = reg_bit(PL, sl);
    double s = 0.0;
    for (int i = 0; i < 6; ++i)
      if ((x >> i) & 1) s += Wl[br * 14 + lane_bit(PL, i)];
    T->Gl[sl][x] = s;
    return;
  }
  e -= 320;
  if (e < 8) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
      if ((e >> i) & 1) {
        const int bi = wave_bit(PL, i);
        s += fl[bi];
        for (int j = 0; j < i; ++j)
          if ((e >> j) & 1) s += Wl[bi * 14 + wave_bit(PL, j)];
      }
    T->Lw[e] = s;
    return;
  }
  e -= 8;
  if (e < 48) {
    const int li = e >> 3, y = e & 7, bl = lane_bit(PL, li);
    double s = 0.0;
    for (int j = 0; j < 3; ++j)
      if ((y >> j) & 1) s += Wl[bl * 14 + wave_bit(PL, j)];
    T->Fw[li][y] = s;
    return;
  }
  e -= 48;
  if (e < 40) {
    const int sl = e >> 3, y = e & 7, br = reg_bit(PL, sl);
    double s = 0.0;
    for (int j = 0; j < 3; ++j)
      if ((y >> j) & 1) s += Wl[br * 14 + wave_bit(PL, j)];
    T->Gw[sl][y] = s;
    return;
  }
  e -= 40;
  if (e < 32) {
    double s = 0.0;
    for (int i = 0; i < 5; ++i)
      if ((e >> i) & 1)
        for (int j = 0; j < i; ++j)
          if ((e >> j) & 1) s += Wl[reg_bit(PL, i) * 14 + reg_bit(PL, j)];
    T->Kr[e] = s;
  }
}

// The thread's cfix and fields g_s in the phase layout (FP64).
template <int PL>
__device__ __forceinline__ void thread_energy(const Tables* T, const double* fl, double cblk,
                                              int lane, int wave, double& cfix, double (&g)[5]) {
  double c = cblk + T->Lw[wave] + T->Ll[lane];
#pragma unroll
  for (int i = 0; i < 6; ++i)
    if ((lane >> i) & 1) c += T->Fw[i][wave];
  cfix = c;
#pragma unroll
  for (int s = 0; s < 5; ++s) g[s] = fl[reg_bit(PL, s)] + T->Gl[s][lane] + T->Gw[s][wave];
}

// Phase of layer `L` on the 32 register amplitudes, times the pending mixer
// scalar (sr, si).
template <int PL>
__device__ __forceinline__ void apply_phase(float2 (&v)[32], const Tables* T, const float2* KF,
                                            const double* fl, double cblk, int lane, int wave,
                                            double gp, double sr, double si) {
  double cfix, g[5];
  thread_energy<PL>(T, fl, cblk, lane, wave, cfix, g);
  float2 f0 = unit(gp * cfix);
  f0 = cmul(f0, make_float2((float)sr, (float)si));
  float2 fs[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) fs[s] = unit(gp * g[s]);
#pragma unroll
  for (int r4 = 0; r4 < 2; ++r4) {
    const float2 p4 = r4 ? cmul(f0, fs[4]) : f0;
#pragma unroll
    for (int r3 = 0; r3 < 2; ++r3) {
      const float2 p3 = r3 ? cmul(p4, fs[3]) : p4;
#pragma unroll
      for (int r2 = 0; r2 < 2; ++r2) {
        const float2 p2 = r2 ? cmul(p3, fs[2]) : p3;
#pragma unroll
        for (int r1 = 0; r1 < 2; ++r1) {
          const float2 p1 = r1 ? cmul(p2, fs[1]) : p2;
#pragma unroll
          for (int r0 = 0; r0 < 2; ++r0) {
            const float2 p0 = r0 ? cmul(p1, fs[0]) : p1;
            const int r = r0 | (r1 << 1) | (r2 << 2) | (r3 << 3) | (r4 << 4);
            v[r] = cmul(v[r], cmul(p0, KF[r]));
          }
        }
      }
    }
  }
}

// <C> and norm partial sums of the 32 register amplitudes, FP64.
template <int PL>
__device__ __forceinline__ void reduce_regs(const float2 (&v)[32], const Tables* T,
                                            const double* fl, double cblk, int lane, int wave,
                                            double& ae, double& an) {
  double cfix, g[5];
  thread_energy<PL>(T, fl, cblk, lane, wave, cfix, g);
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    double c = cfix + T->Kr[r];
#pragma unroll
    for (int s = 0; s < 5; ++s)
      if ((r >> s) & 1) c += g[s];
    const double pz = (double)v[r].x * v[r].x + (double)v[r].y * v[r].y;
    ae = fma(pz, c, ae);
    an += pz;
  }
}

// Global load/store of the register tile in layout L (pairs of amplitudes
// differing in tile bit 0 move as one 16-byte access).
// Rows rp in [RP0, RP0 + NRP) of the tile (register indices 2rp, 2rp + 1)
// into dst[2 * (rp - RP0) + D0 ...].
template <int L, int RP0, int NRP, int D0, int N>
__device__ __forceinline__ void load_rows(float2 (&dst)[N], const float2* base, int lane,
                                          int wave, int kind, int a) {
  const uint64_t tb = dep14(thread_bits<L>(lane, wave), kind, a);
#pragma unroll
  for (int i = 0; i < NRP; ++i) {
    const int rp = RP0 + i;
    const uint64_t o = tb + dep14(reg_off<L>(rp) << 1, kind, a);
    const float4 q = *reinterpret_cast<const float4*>(base + o);
    dst[D0 + 2 * i] = make_float2(q.x, q.y);
    dst[D0 + 2 * i + 1] = make_float2(q.z, q.w);
  }
}

template <int L>
__device__ __forceinline__ void store_tile(const float2 (&v)[32], float2* base, int lane, int wave,
                                           int kind, int a) {
  const uint64_t tb = dep14(thread_bits<L>(lane, wave), kind, a);
#pragma unroll
  for (int rp = 0; rp < 16; ++rp) {
    const uint64_t o = tb + dep14(reg_off<L>(rp) << 1, kind, a);
    const float2 u = v[rp << 1], w = v[(rp << 1) | 1];
    *reinterpret_cast<float4*>(base + o) = make_float4(u.x, u.y, w.x, w.y);
  }
}

template <int L>
__device__ __forceinline__ void store_probs(const float2 (&v)[32], float* base, int lane,
                                            int wave, int kind, int a, float scale) {
  const uint64_t tb = dep14(thread_bits<L>(lane, wave), kind, a);
#pragma unroll
  for (int rp = 0; rp < 16; ++rp) {
    const uint64_t o = tb + dep14(reg_off<L>(rp) << 1, kind, a);
    const float2 u = v[rp << 1], w = v[(rp << 1) | 1];
    *reinterpret_cast<float2*>(base + o) =
        make_float2(scale * (u.x * u.x + u.y * u.y), scale * (w.x * w.x + w.y * w.y));
  }
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

// Block bits of tile ti.
template <int KIND>
__device__ __forceinline__ uint64_t tile_base(uint64_t ti, int a) {
  if (KIND == 1) return ti << 14;
  const int gap = a - 4;
  return ((ti & ((1ull << gap) - 1ull)) << 4) | ((ti >> gap) << (a + 10));
}

// Per-tile context in LDS: fields of the block bits on the tile bits (fl),
// couplings among tile bits (Wl), the energy of the block bits (returned),
// and the phase tables of layout PL.
template <int KIND, int PL>
__device__ __forceinline__ double tile_context(const PassDesc& d, const double* Wsh, uint64_t zb, double* fl,
                               double* Wl, double* tmp, Tables* T, int tid) {
  const int n = d.n;
  if (tid < 14) {
    const int pi = (KIND == 1 || tid < 4) ? tid : d.a + tid - 4;
    double f = Wsh[pi * n + pi];
    for (int j = 0; j < n; ++j)
      if ((zb >> j) & 1ull) f += Wsh[pi * n + j];
    fl[tid] = f;
  }
  if (tid >= 64 && tid < 64 + 196) {
    const int e = tid - 64, i = e / 14, j = e - 14 * i;
    const int pi = (KIND == 1 || i < 4) ? i : d.a + i - 4;
    const int pj = (KIND == 1 || j < 4) ? j : d.a + j - 4;
    Wl[e] = (i == j) ? 0.0 : Wsh[pi * n + pj];
  }
  if (tid >= 320 && tid < 320 + n) {
    const int i = tid - 320;
    double t = 0.0;
    if ((zb >> i) & 1ull) {
      t = Wsh[i * n + i];
      for (int j = 0; j < i; ++j)
        if ((zb >> j) & 1ull) t += Wsh[i * n + j];
    }
    tmp[i] = t;
  }
  lds_barrier();
  double cblk = 0.0;
  for (int i = 0; i < n; ++i) cblk += tmp[i];
  build_tables<PL>(T, fl, Wl, tid);
  lds_barrier();
  return cblk;
}

// One tile of a pass whose input tile `v` is already in registers (layout LA)
// or, for the first pass, is generated here.  Layouts LA (load), LB, LC
// (phase); the pass mixes tile bits [MIXLO, 14).
template <int LA, int LB, int LC, int MIXLO>
__device__ __forceinline__ void tile14(const F14Args& A, float2 (&v)[32], float2* buf,
                                       Tables* T, float2* KF, const double* fl, double cblk,
                                       int lane, int wave, uint64_t st, uint64_t ti, uint64_t zb,
                                       const LayerCoef* cf) {
  const PassDesc& d = A.d;
  const int m = 14 - d.mixlo;
  // pending mixer scalar at the start of the pass
  double sr = 1.0, si = 0.0;
  for (int i = 0; i < d.pend_n; ++i) half_scale(cf[d.pend_layer[i]], d.pend_m[i], sr, si);
  const bool has_phase = d.ja <= d.jb;
  int where = (d.flags & F_INIT) ? 2 : 0;  // 0: layout LA, 2: layout LC
  if (d.lead >= 0) {  // lead half-mixer: LA -> LB -> LC
    const LayerCoef& L = cf[d.lead];
    const float t = (float)L.tb;
    if (L.mode == 0) half_mixer<0, LA, LB, LC, MIXLO>(v, buf, lane, wave, t);
    else half_mixer<1, LA, LB, LC, MIXLO>(v, buf, lane, wave, t);
    half_scale(L, m, sr, si);
    where = 2;
  }
  if (has_phase) {  // phase of layer jb, then its half-mixer LC -> LB -> LA
    const LayerCoef& L = cf[d.jb];
    if (threadIdx.x < 32) KF[threadIdx.x] = unit(L.gp * T->Kr[threadIdx.x]);
    lds_barrier();
    apply_phase<LC>(v, T, KF, fl, cblk, lane, wave, L.gp, sr, si);
    sr = 1.0;
    si = 0.0;
    const float t = (float)L.tb;
    if (L.mode == 0) half_mixer<0, LC, LB, LA, MIXLO>(v, buf, lane, wave, t);
    else half_mixer<1, LC, LB, LA, MIXLO>(v, buf, lane, wave, t);
    where = 0;
  }
  if (d.flags & F_REDUCE) {
    // outputs of the final pass carry the pending scalar; it is in LC here
    const float fr = (float)sr, fi = (float)si;
    if (d.flags & F_PROBS) {
      const float s2 = (float)(sr * sr + si * si);
      store_probs<LC>(v, A.probs + (st << d.n) + zb, lane, wave, d.kind, d.a, s2);
    }
    if (d.flags & F_WRITE) {
#pragma unroll
      for (int r = 0; r < 32; ++r) v[r] = cmul(v[r], make_float2(fr, fi));
      store_tile<LC>(v, A.out + st * A.stride + zb, lane, wave, d.kind, d.a);
    }
    double ae = 0.0, an = 0.0;
    reduce_regs<LC>(v, T, fl, cblk, lane, wave, ae, an);
    double* red = reinterpret_cast<double*>(KF);  // KF is unused in the last pass
    const double s2 = (d.flags & F_WRITE) ? 1.0 : sr * sr + si * si;
    const double se = bsum14(ae, red) * s2;
    const double sn = bsum14(an, red) * s2;
    if (threadIdx.x == 0) {
      double* o = A.part + ((st << (d.n - 14)) + ti) * 2;
      o[0] = se;
      o[1] = sn;
    }
  } else if (d.flags & F_WRITE) {
    float2* g = A.out + st * A.stride + zb;
    if (where == 0) store_tile<LA>(v, g, lane, wave, d.kind, d.a);
    else store_tile<LC>(v, g, lane, wave, d.kind, d.a);
  }
}

// Persistent kernel: work-group w processes tiles w, w + G, w + 2G, ... of
// all states (tile index = state * 2^(n-14) + tile); while it computes one
// tile, the next tile's loads are in flight into a second register buffer.
template <int KIND, int MIXLO>
__global__ void __launch_bounds__(NT14) fwd14_kernel(F14Args A) {
  constexpr int LB = KIND == 1 ? 1 : 3, LC = KIND == 1 ? 2 : 4;
  __shared__ float2 buf[PHYS];
  __shared__ Tables T;
  __shared__ double fl[14];
  __shared__ double Wl[14 * 14];
  __shared__ double tmp[40];
  __shared__ float2 KF[32];
  __shared__ double Wsh[34 * 34];  // the current problem's folded Q
  __shared__ LayerCoef Csh[64];    // the current state's layer coefficients
  const PassDesc& d = A.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nlog = d.n - 14;
  const uint64_t total = (uint64_t)A.nstates << nlog;
  const uint64_t tmask = (1ull << nlog) - 1ull;
  const bool init = (d.flags & F_INIT) != 0;
  // rows 0..7 of the next tile (half of it) are prefetched into registers
  // while the current tile is computed; rows 8..15 are loaded at tile start
  float2 nxt[16];
  uint64_t tile = blockIdx.x;
  int64_t prob = -1, cst = -1;
  auto tile_ptr = [&](uint64_t t) {
    return A.in + (t >> nlog) * A.stride + tile_base<KIND>(t & tmask, d.a);
  };
  if (!init && tile < total) load_rows<0, 0, 8, 0>(nxt, tile_ptr(tile), lane, wave, d.kind, d.a);
  for (; tile < total; tile += gridDim.x) {
    const uint64_t st = tile >> nlog, ti = tile & tmask;
    const uint64_t zb = tile_base<KIND>(ti, d.a);
    const int64_t pr = (int64_t)(st / A.S);
    if (pr != prob) {  // stage W in LDS (rare: once per problem)
      const double* W = A.W + (size_t)pr * d.n * d.n;
      for (int e = tid; e < d.n * d.n; e += NT14) Wsh[e] = W[e];
      prob = pr;
      __syncthreads();
    }
    if ((int64_t)st != cst) {  // stage the state's layer coefficients in LDS
      const LayerCoef* c = A.coef + st * A.p;
      for (int e = tid; e < A.p; e += NT14) Csh[e] = c[e];
      cst = (int64_t)st;
      __syncthreads();
    }
    const double cblk = tile_context<KIND, LC>(d, Wsh, zb, fl, Wl, tmp, &T, tid);
    float2 v[32];
    if (init) {
      const float amp = (float)exp2(-0.5 * (double)d.n);
#pragma unroll
      for (int r = 0; r < 32; ++r) v[r] = make_float2(amp, 0.0f);
    } else {
      load_rows<0, 8, 8, 16>(v, tile_ptr(tile), lane, wave, d.kind, d.a);
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = nxt[r];
      // Rows 0..7 of the next tile (the last tile re-reads itself, so the
      // loads are unconditional and every wait on this tile's loads has a
      // fixed count that leaves the prefetch in flight).
      const uint64_t nx = tile + gridDim.x < total ? tile + gridDim.x : tile;
      __builtin_amdgcn_sched_barrier(0);
      load_rows<0, 0, 8, 0>(nxt, tile_ptr(nx), lane, wave, d.kind, d.a);
      __builtin_amdgcn_sched_barrier(0);
    }
    tile14<0, LB, LC, MIXLO>(A, v, buf, &T, KF, fl, cblk, lane, wave, st, ti, zb, Csh);
    lds_barrier();  // the next tile rewrites the LDS context
  }
}

int cu_count() {
  static int n = [] {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 256;
    return c > 0 ? c : 256;
  }();
  return n;
}

}  // namespace

hipError_t launch_fwd14_pass(const PassDesc& d, int nstates, int S, int p,
                             const void* in, void* out, uint64_t state_stride,
                             const double* W, const LayerCoef* coef,
                             double* part, void* probs, hipStream_t stream) {
  F14Args A;
  A.d = d;
  A.S = S;
  A.p = p;
  A.nstates = nstates;
  A.in = reinterpret_cast<const float2*>(in);
  A.out = reinterpret_cast<float2*>(out);
  A.stride = state_stride;
  A.W = W;
  A.coef = coef;
  A.part = part;
  A.probs = reinterpret_cast<float*>(probs);
  const uint64_t total = (uint64_t)nstates << (d.n - 14);
  const uint64_t g = (uint64_t)cu_count();  // one 512-thread work-group per CU
  const dim3 grid((unsigned)(total < g ? total : g)), blk(NT14);
#define DQ_K(K, M) hipLaunchKernelGGL((fwd14_kernel<K, M>), grid, blk, 0, stream, A)
  if (d.kind == 1) {
    DQ_K(1, 0);
  } else {
    switch (d.mixlo) {
      case 4: DQ_K(2, 4); break;
      case 5: DQ_K(2, 5); break;
      case 6: DQ_K(2, 6); break;
      case 7: DQ_K(2, 7); break;
      case 8: DQ_K(2, 8); break;
      case 9: DQ_K(2, 9); break;
      case 10: DQ_K(2, 10); break;
      case 11: DQ_K(2, 11); break;
      case 12: DQ_K(2, 12); break;
      case 13: DQ_K(2, 13); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef DQ_K
  return hipGetLastError();
}

}  // namespace dq
