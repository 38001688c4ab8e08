// 13-qubit register-tile geometry (5 register bits, 6 lane bits, 2 wave
// bits; see regtile.h), shared by the complex64 gradient and the complex128
// forward pass.
#pragma once

#include "regtile.h"

namespace dq {
namespace rt {

// Layouts of the 13-qubit tile (register slots 0..4, lane slots 0..5, wave
// slots 0..1):
//   L_A   load/store: lane slots are tile bits 1..6
//   L_A1  L_A with register slots 3, 4 swapped with lane slots 4, 5
//   L_B   set 0: bits 1..4 in registers
//   L_B1  L_B with register slots 3, 4 swapped with lane slots 4, 5 (bits
//         11, 12 in registers); phase layout of set 0
//   L_B2  other sets: bits 4, 5, 6, 11 in registers
//   L_B3  L_B2 with register slot 1 swapped with lane slot 4 (bit 12 in
//         registers); phase layout of the other sets
// Set 0 mixes in A, A1 | transpose | B, B1 and back in reverse.  The other
// sets keep C contiguous low tile bits: with C = 4 they mix bits [4, 13) in
// A | transpose | B2, B3 and back; with C = 2 they mix bits [2, 13) with the
// set-0 sequence (bits below the first mixed bit are masked out).
template <class V_, class S_, int C_>
struct G13T {
  using V = V_;
  using S = S_;
  static constexpr int C = C_;
  static constexpr int R = 5;
  using G13 = G13T;
  enum { L_A = 0, L_A1 = 1, L_B = 2, L_B1 = 3, L_B2 = 4, L_B3 = 5 };
  static constexpr int LA = L_A;
  template <int KIND>
  static constexpr int PL = (KIND == 1 || C == 2) ? L_B1 : L_B3;
  static constexpr int reg_bit(int L, int s) {
    constexpr int t[6][5] = {{0, 7, 8, 9, 10},  {0, 7, 8, 5, 6},  {0, 1, 2, 3, 4},
                             {0, 1, 2, 11, 12}, {0, 4, 5, 6, 11}, {0, 12, 5, 6, 11}};
    return t[L][s];
  }
  static constexpr int lane_bit(int L, int s) {
    constexpr int t[6][6] = {{1, 2, 3, 4, 5, 6},  {1, 2, 3, 4, 9, 10}, {5, 6, 7, 8, 11, 12},
                             {5, 6, 7, 8, 3, 4},  {1, 2, 3, 8, 12, 7}, {1, 2, 3, 8, 4, 7}};
    return t[L][s];
  }
  static constexpr int wave_bit(int L, int s) {
    constexpr int t[6][2] = {{11, 12}, {11, 12}, {9, 10}, {9, 10}, {9, 10}, {9, 10}};
    return t[L][s];
  }

  // Forward half-mixers (used by the checkpoint passes).
  template <int KIND, int MIXLO>
  static __device__ __forceinline__ void lead(V (&v)[32], V* buf, int lane, int wave,
                                              S t, bool flip) {
    if constexpr (KIND == 1 || C == 2) {
      constexpr uint32_t D1 = reg_bits_of<G13, L_A>();
      constexpr uint32_t D2 = D1 | reg_bits_of<G13, L_A1>();
      constexpr uint32_t D3 = D2 | reg_bits_of<G13, L_B>();
      mix_round<G13, reg_mask<G13, L_A, 0, MIXLO>()>(v, t);
      swap_slot<G13, 3, 4>(v);
      swap_slot<G13, 4, 5>(v);
      mix_round<G13, reg_mask<G13, L_A1, D1, MIXLO>()>(v, t);
      transpose<G13, L_A1, L_B, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G13, reg_mask<G13, L_B, D2, MIXLO>()>(v, t);
      swap_slot<G13, 3, 4>(v);
      swap_slot<G13, 4, 5>(v);
      mix_round<G13, reg_mask<G13, L_B1, D3, MIXLO>()>(v, t);
    } else {
      constexpr uint32_t D1 = reg_bits_of<G13, L_A>();
      constexpr uint32_t D2 = D1 | reg_bits_of<G13, L_B2>();
      mix_round<G13, reg_mask<G13, L_A, 0, MIXLO>()>(v, t);
      transpose<G13, L_A, L_B2, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G13, reg_mask<G13, L_B2, D1, MIXLO>()>(v, t);
      swap_slot<G13, 1, 4>(v);
      mix_round<G13, reg_mask<G13, L_B3, D2, MIXLO>()>(v, t);
    }
  }
  template <int KIND, int MIXLO>
  static __device__ __forceinline__ void trail(V (&v)[32], V* buf, int lane, int wave,
                                               S t, bool flip) {
    if constexpr (KIND == 1 || C == 2) {
      constexpr uint32_t D1 = reg_bits_of<G13, L_B1>();
      constexpr uint32_t D2 = D1 | reg_bits_of<G13, L_B>();
      constexpr uint32_t D3 = D2 | reg_bits_of<G13, L_A1>();
      mix_round<G13, reg_mask<G13, L_B1, 0, MIXLO>()>(v, t);
      swap_slot<G13, 3, 4>(v);
      swap_slot<G13, 4, 5>(v);
      mix_round<G13, reg_mask<G13, L_B, D1, MIXLO>()>(v, t);
      transpose<G13, L_B, L_A1, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G13, reg_mask<G13, L_A1, D2, MIXLO>()>(v, t);
      swap_slot<G13, 3, 4>(v);
      swap_slot<G13, 4, 5>(v);
      mix_round<G13, reg_mask<G13, L_A, D3, MIXLO>()>(v, t);
    } else {
      constexpr uint32_t D1 = reg_bits_of<G13, L_B3>();
      constexpr uint32_t D2 = D1 | reg_bits_of<G13, L_B2>();
      mix_round<G13, reg_mask<G13, L_B3, 0, MIXLO>()>(v, t);
      swap_slot<G13, 1, 4>(v);
      mix_round<G13, reg_mask<G13, L_B2, D1, MIXLO>()>(v, t);
      transpose<G13, L_B2, L_A, MIXLO>(v, buf, lane, wave, flip);
      mix_round<G13, reg_mask<G13, L_A, D2, MIXLO>()>(v, t);
    }
  }
};

}  // namespace rt
}  // namespace dq
