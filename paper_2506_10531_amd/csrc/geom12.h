// 12-qubit register-tile geometry (4 register bits, 6 lane bits, 2 wave
// bits; see regtile.h), used by the complex128 gradient: a tile is 256
// threads x 16 double2 amplitudes, so psi and lambda together take 128 VGPRs.
#pragma once

#include "regtile.h"

namespace dq {
namespace rt {

// Layouts of the 12-qubit tile (register slots 0..3, lane slots 0..5, wave
// slots 0..1):
//   L_A   load/store: lane slots are tile bits 1..6, registers 0, 8, 7, 9
//   L_A1  L_A with register slots 1, 2, 3 swapped with lane slots 3, 4, 5
//         (lane slot 3 by a DPP exchange, 4 and 5 by permlane swaps)
//   L_B   bits 1, 2, 3 in registers; lane slots 0..3 are bits 5, 6, 7, 4
//   L_B1  L_B with register slots 2, 3 swapped with lane slots 4, 5 (bits
//         10, 11 in registers); the phase layout
// Every set mixes in A, A1 | transpose | B, B1 and back in reverse (the
// first mixed bit masks the low bits of the other sets).  Lane slots 0..3 of
// A1 and B hit distinct 16-byte LDS bank groups under the padded transpose.
template <class V_, class S_, int C_>
struct G12T {
  using V = V_;
  using S = S_;
  static constexpr int C = C_;
  static constexpr int R = 4;
  using G12 = G12T;
  enum { L_A = 0, L_A1 = 1, L_B = 2, L_B1 = 3 };
  static constexpr int LA = L_A;
  template <int KIND>
  static constexpr int PL = L_B1;
  static constexpr int reg_bit(int L, int s) {
    constexpr int t[4][4] = {{0, 8, 7, 9}, {0, 4, 5, 6}, {0, 1, 2, 3}, {0, 1, 10, 11}};
    return t[L][s];
  }
  static constexpr int lane_bit(int L, int s) {
    constexpr int t[4][6] = {{1, 2, 3, 4, 5, 6}, {1, 2, 3, 8, 7, 9},
                             {5, 6, 7, 4, 10, 11}, {5, 6, 7, 4, 2, 3}};
    return t[L][s];
  }
  static constexpr int wave_bit(int L, int s) {
    constexpr int t[4][2] = {{10, 11}, {10, 11}, {8, 9}, {8, 9}};
    return t[L][s];
  }

  // The register/lane exchanges between L_A and L_A1, and L_B and L_B1.
  template <class T>
  static __device__ __forceinline__ void swap_a(T& v) {
    swap_slot<G12, 1, 3>(v);
    swap_slot<G12, 2, 4>(v);
    swap_slot<G12, 3, 5>(v);
  }
  template <class T>
  static __device__ __forceinline__ void swap_b(T& v) {
    swap_slot<G12, 2, 4>(v);
    swap_slot<G12, 3, 5>(v);
  }

  // Forward half-mixers (used by the checkpoint passes).
  template <int KIND, int MIXLO>
  static __device__ __forceinline__ void lead(V (&v)[16], V* buf, int lane, int wave, S t,
                                              bool flip) {
    constexpr uint32_t D1 = reg_bits_of<G12, L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G12, L_A1>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G12, L_B>();
    mix_round<G12, reg_mask<G12, L_A, 0, MIXLO>()>(v, t);
    swap_a(v);
    mix_round<G12, reg_mask<G12, L_A1, D1, MIXLO>()>(v, t);
    transpose<G12, L_A1, L_B, MIXLO>(v, buf, lane, wave, flip);
    mix_round<G12, reg_mask<G12, L_B, D2, MIXLO>()>(v, t);
    swap_b(v);
    mix_round<G12, reg_mask<G12, L_B1, D3, MIXLO>()>(v, t);
  }
  template <int KIND, int MIXLO>
  static __device__ __forceinline__ void trail(V (&v)[16], V* buf, int lane, int wave, S t,
                                               bool flip) {
    constexpr uint32_t D1 = reg_bits_of<G12, L_B1>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G12, L_B>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G12, L_A1>();
    mix_round<G12, reg_mask<G12, L_B1, 0, MIXLO>()>(v, t);
    swap_b(v);
    mix_round<G12, reg_mask<G12, L_B, D1, MIXLO>()>(v, t);
    transpose<G12, L_B, L_A1, MIXLO>(v, buf, lane, wave, flip);
    mix_round<G12, reg_mask<G12, L_A1, D2, MIXLO>()>(v, t);
    swap_a(v);
    mix_round<G12, reg_mask<G12, L_A, D3, MIXLO>()>(v, t);
  }
};

}  // namespace rt
}  // namespace dq
