// 14-qubit register-tile geometry (6 register bits, 6 lane bits, 2 wave
// bits; see regtile.h) of the complex64 forward pass.
#pragma once

#include "regtile.h"

namespace dq {
namespace rt {
namespace {  // internal linkage: one translation unit instantiates the passes

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
}  // namespace rt
}  // namespace dq
