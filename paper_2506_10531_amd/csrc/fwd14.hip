// Register-tile forward pass for complex64 states on 14-qubit tiles (gfx950).
//
// Same pass structure as the LDS-tile pass in kernels.hip (a layer's mixer
// split into commuting qubit sets; the pass finishing layer j on a set also
// applies the phase of layer j+1 and starts layer j+1, Eq. (2) of the paper),
// but the 2^14-amplitude tile lives in registers: 256 threads (4 waves) x 64
// amplitudes, i.e. 6 register tile bits per thread, 6 lane bits and 2 wave
// bits (the machinery is in regtile.h).  A work-group needs about 77 KiB of
// LDS, so two share a CU: while one waits at a barrier or on memory, the
// other computes.
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
#include "regtile.h"

namespace dq {
namespace {

using namespace rt;

// Layouts: the tile bit held by register slots 0..5, lane slots 0..5 and wave
// slots 0..1.
//   L_A   load/store layout: lane slots are tile bits 1..6 (1 KiB runs)
//   L_A1  L_A with register slots 4, 5 swapped with lane slots 4, 5
//   L_B   set 0: the bits L_A1 leaves unmixed (1..4, 12) in registers
//   L_B1  L_B with register slot 5 swapped with lane slot 4 (bit 13 in
//         registers); phase layout of set 0
//   L_B2  other sets: bits 4, 5, 6, 12, 13 in registers; phase layout
// Set 0 mixes in A, A1 | transpose | B, B1 and back in reverse; the other
// sets in A | transpose | B2 and back.  C_ is the number of contiguous low
// tile bits of the other sets (4 to 8): they mix tile bits [MIXLO, 14) with
// MIXLO >= C_, so bits 1..3, never held in registers, are never mixed by them.
template <int C_>
struct G14T {
  using V = float2;
  using S = float;
  static constexpr int C = C_;
  static constexpr int R = 6;
  enum { L_A = 0, L_A1 = 1, L_B = 2, L_B1 = 3, L_B2 = 4 };
  static constexpr int LA = L_A;
  template <int KIND>
  static constexpr int PL = KIND == 1 ? L_B1 : L_B2;
  static constexpr int reg_bit(int L, int s) {
    constexpr int t[5][6] = {{0, 7, 8, 9, 10, 11},
                             {0, 7, 8, 9, 5, 6},
                             {0, 1, 2, 3, 4, 12},
                             {0, 1, 2, 3, 4, 13},
                             {0, 4, 12, 13, 5, 6}};
    return t[L][s];
  }
  static constexpr int lane_bit(int L, int s) {
    constexpr int t[5][6] = {{1, 2, 3, 4, 5, 6},
                             {1, 2, 3, 4, 10, 11},
                             {5, 6, 7, 8, 13, 9},
                             {5, 6, 7, 8, 12, 9},
                             {1, 2, 3, 8, 7, 9}};
    return t[L][s];
  }
  static constexpr int wave_bit(int L, int s) {
    constexpr int t[5][2] = {{12, 13}, {12, 13}, {10, 11}, {10, 11}, {10, 11}};
    return t[L][s];
  }

  // Lead half-mixer: from the load layout to the phase layout; trail
  // half-mixer: back.  flip (cot form) relabels the tile in the transpose.
  template <int KIND, int MIXLO>
  static __device__ __forceinline__ void lead(V (&v)[64], V* buf, int lane, int wave, S t,
                                              bool flip) {
    if constexpr (KIND == 1) {
      constexpr uint32_t D1 = reg_bits_of<G14T, L_A>();
      constexpr uint32_t D2 = D1 | reg_bits_of<G14T, L_A1>();
      constexpr uint32_t D3 = D2 | reg_bits_of<G14T, L_B>();
      mix_round<G14T, reg_mask<G14T, L_A, 0, MIXLO>()>(v, t);
      swap_slot<G14T, 4, 4>(v);
      swap_slot<G14T, 5, 5>(v);
      mix_round<G14T, reg_mask<G14T, L_A1, D1, MIXLO>()>(v, t);
      transpose<G14T, L_A1, L_B, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G14T, reg_mask<G14T, L_B, D2, MIXLO>()>(v, t);
      swap_slot<G14T, 5, 4>(v);
      mix_round<G14T, reg_mask<G14T, L_B1, D3, MIXLO>()>(v, t);
    } else {
      constexpr uint32_t D1 = reg_bits_of<G14T, L_A>();
      mix_round<G14T, reg_mask<G14T, L_A, 0, MIXLO>()>(v, t);
      transpose<G14T, L_A, L_B2, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G14T, reg_mask<G14T, L_B2, D1, MIXLO>()>(v, t);
    }
  }
  template <int KIND, int MIXLO>
  static __device__ __forceinline__ void trail(V (&v)[64], V* buf, int lane, int wave, S t,
                                               bool flip) {
    if constexpr (KIND == 1) {
      constexpr uint32_t D1 = reg_bits_of<G14T, L_B1>();
      constexpr uint32_t D2 = D1 | reg_bits_of<G14T, L_B>();
      constexpr uint32_t D3 = D2 | reg_bits_of<G14T, L_A1>();
      mix_round<G14T, reg_mask<G14T, L_B1, 0, MIXLO>()>(v, t);
      swap_slot<G14T, 5, 4>(v);
      mix_round<G14T, reg_mask<G14T, L_B, D1, MIXLO>()>(v, t);
      transpose<G14T, L_B, L_A1, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G14T, reg_mask<G14T, L_A1, D2, MIXLO>()>(v, t);
      swap_slot<G14T, 4, 4>(v);
      swap_slot<G14T, 5, 5>(v);
      mix_round<G14T, reg_mask<G14T, L_A, D3, MIXLO>()>(v, t);
    } else {
      constexpr uint32_t D1 = reg_bits_of<G14T, L_B2>();
      mix_round<G14T, reg_mask<G14T, L_B2, 0, MIXLO>()>(v, t);
      transpose<G14T, L_B2, L_A, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G14T, reg_mask<G14T, L_A, D1, MIXLO>()>(v, t);
    }
  }
};

}  // namespace

hipError_t launch_fwd14_pass(const PassDesc& d, int nstates, int S, int p,
                             const void* in, void* out, uint64_t state_stride,
                             const double* W, const LayerCoef* coef,
                             double* part, void* probs, void* tab, hipStream_t stream) {
  if (d.n < 15 || d.n > 34 || p < 1 || p > 64 || nstates < 1 || S < 1)
    return hipErrorInvalidValue;
  const int pt = pass_shape(d, p);
  if (pt < 0 || (d.kind == 1 && pt == P_LEAD)) return hipErrorInvalidValue;
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 4 || d.mixlo > 13)) return hipErrorInvalidValue;
  if (d.kind == 2 && d.c != (d.mixlo < 8 ? d.mixlo : 8)) return hipErrorInvalidValue;
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
  A.tab = tab;
  const uint64_t total = (uint64_t)nstates << (d.n - 14);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
  if (pt != P_LEAD && !tab) return hipErrorInvalidValue;
#define DQ_K(K, M, T)                                                                        \
  hipLaunchKernelGGL((fwd_kernel<G14T<(K == 1 ? 4 : M < 8 ? M : 8)>, K, M, T>),             \
                     grid, blk, 0, stream, A)
#define DQ_PT(K, M)                           \
  switch (pt) {                               \
    case P_FIRST: DQ_K(K, M, P_FIRST); break; \
    case P_MID: DQ_K(K, M, P_MID); break;     \
    case P_LEAD: DQ_K(K, M, P_LEAD); break;   \
    default: DQ_K(K, M, P_LAST); break;       \
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

hipError_t launch_fwd14_tables(const TabJobs& J, int n, int nstates, int S, int p,
                               const double* W, const LayerCoef* coef, void* tab,
                               hipStream_t stream) {
  return launch_all_tables<G14T<4>>(J, n, nstates, S, p, W, coef, tab, stream);
}

}  // namespace dq
