// Bounds and coverage check of the register-tile kernels' index maps, run on
// the host (test infrastructure: built and run by tests/test_index_maps_cpu.py;
// it launches nothing).  It calls the same __host__ __device__ helpers the
// kernels use for their addresses (thread_bits, reg_off, pair_base, pair_rel,
// tile_base, transpose_bases, phys, xcd_map) and checks, for every geometry and every
// pass the library plans for n up to 34:
//   * every layout places each tile bit in exactly one register, lane or wave
//     slot, with tile bit 0 in register slot 0;
//   * the global offsets of a tile's register pairs in the load/store layout
//     and in the phase layout are exactly the tile's 2^K amplitudes, each
//     once, all below 2^n, and the tile bases deposit the tile index onto the
//     remaining bits, so the tiles of a pass cover the state exactly once;
//   * every LDS transpose the half-mixers make (with and without the cot-form
//     relabelling) writes each slot of its half once, inside the buffer, and
//     reads back into every register the amplitude that the target layout
//     assigns to it (tile index l ^ M when relabelling);
//   * the rounds of every half-mixer, in its lead and its trail order, mix
//     each tile bit of the pass's range [MIXLO, K) exactly once and no other;
//   * the work-group -> tile order (xcd_map) is a bijection of the grid.
// Prints "ok <checks>" and exits 0, or prints the first failures and exits 1.
#include "../paper_2506_10531_amd/csrc/geom12.h"
#include "../paper_2506_10531_amd/csrc/geom13.h"
#include "../paper_2506_10531_amd/csrc/geom14.h"
#include "../include/dqaoa.h"

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <initializer_list>
#include <utility>
#include <vector>

using namespace dq::rt;

namespace {

long g_checks = 0;
int g_fails = 0;

void check(bool ok, const char* what, const char* where, long a = 0, long b = 0) {
  ++g_checks;
  if (!ok && g_fails++ < 25) std::printf("FAIL %s [%s] %ld %ld\n", what, where, a, b);
}

// Tile index held by register index r of thread (lane, wave) in layout L.
template <class G, int L>
uint32_t tile_index(int lane, int wave, int r) {
  uint32_t l = thread_bits<G, L>(lane, wave);
  for (int s = 0; s < G::R; ++s)
    if ((r >> s) & 1) l |= 1u << G::reg_bit(L, s);
  return l;
}

template <class G, int L>
void check_layout(const char* g) {
  constexpr int K = Dim<G>::K;
  uint32_t m = 0;
  int cnt = 0;
  for (int s = 0; s < 6; ++s, ++cnt) m |= 1u << G::lane_bit(L, s);
  for (int s = 0; s < 2; ++s, ++cnt) m |= 1u << G::wave_bit(L, s);
  for (int s = 0; s < G::R; ++s, ++cnt) m |= 1u << G::reg_bit(L, s);
  check(m == (1u << K) - 1u && cnt == K, "layout covers the tile bits once", g, L, m);
  check(G::reg_bit(L, 0) == 0, "tile bit 0 is register slot 0", g, L);
}

template <class G, int L>
void check_offsets(const char* g, int n, int kind, int a) {
  constexpr int K = Dim<G>::K, NP = Dim<G>::NP;
  std::vector<uint64_t> want(1u << K), got;
  got.reserve(1u << K);
  for (uint32_t l = 0; l < (1u << K); ++l) want[l] = dep<G::C>(l, kind, a);
  for (int wave = 0; wave < 4; ++wave)
    for (int lane = 0; lane < 64; ++lane) {
      const uint64_t tb = pair_base<G, L>(lane, wave, kind, a);
      for (int q = 0; q < NP; ++q) {
        const uint64_t o = tb + pair_rel<G, L>(q, kind, a);
        // the pair is tile indices 2m and 2m + 1 at o and o + 1
        check(o == dep<G::C>(tile_index<G, L>(lane, wave, q << 1), kind, a),
              "pair offset is its tile index's", g, (long)o);
        got.push_back(o);
        got.push_back(o + 1);
      }
    }
  std::sort(want.begin(), want.end());
  std::sort(got.begin(), got.end());
  check(got == want, "tile offsets are the tile's amplitudes once", g, n, L);
  check(got.back() < (1ull << n), "offsets inside the state", g, n, (long)got.back());
}

template <int K, int C>
void check_blocks(const char* g, int n, int kind, int a, uint64_t local_mask) {
  uint64_t bm = 0;
  for (int i = 0; i < n - K; ++i) {
    const uint64_t b = tile_base<K, C>(1ull << i, kind, a);
    check(b != 0 && (b & (b - 1)) == 0, "tile-index bit deposits one state bit", g, n, i);
    check((b & (local_mask | bm)) == 0, "tile-index bits distinct from tile bits", g, n, i);
    bm |= b;
  }
  const uint64_t all = n - K > 0 ? (1ull << (n - K)) - 1 : 0;
  check(tile_base<K, C>(all, kind, a) == bm, "tile base deposits every tile-index bit", g, n);
  check((bm | local_mask) == (n == 64 ? ~0ull : (1ull << n) - 1), "tiles cover the state", g, n);
}

template <class G, int X, int Y, int MIXLO>
void check_transpose(const char* g) {
  constexpr int K = Dim<G>::K, NP = Dim<G>::NP, PHYS = Dim<G>::PHYS;
  constexpr uint32_t M = ((((1u << K) - 1u) >> MIXLO) << MIXLO) & ~1u;
  for (int flip = 0; flip < 2; ++flip)
    for (int h = 0; h < 2; ++h) {
      std::vector<int64_t> lds(PHYS, -1);
      std::vector<int> reads(PHYS, 0);
      for (int wave = 0; wave < 4; ++wave)
        for (int lane = 0; lane < 64; ++lane) {
          uint32_t wb, rb;
          transpose_bases<G, X, Y, MIXLO>(lane, wave, flip != 0, wb, rb);
          for (int q = 0; q < NP; ++q) {
            const uint32_t slot = wb + phys(reg_off<G, X>(q));
            const bool in = slot < (uint32_t)PHYS;
            check(in, "transpose write inside the buffer", g, MIXLO, slot);
            if (!in) continue;
            check(lds[slot] < 0, "transpose slot written once", g, MIXLO, slot);
            lds[slot] = tile_index<G, X>(lane, wave, (q << 1) | h);
          }
        }
      for (int wave = 0; wave < 4; ++wave)
        for (int lane = 0; lane < 64; ++lane) {
          uint32_t wb, rb;
          transpose_bases<G, X, Y, MIXLO>(lane, wave, flip != 0, wb, rb);
          for (int q = 0; q < NP; ++q) {
            const uint32_t slot = rb + phys(reg_off<G, Y>(q));
            const bool in = slot < (uint32_t)PHYS && lds[slot] >= 0;
            check(in, "transpose read of a written slot", g, MIXLO, slot);
            if (!in) continue;
            ++reads[slot];
            const uint32_t lx = (uint32_t)lds[slot];
            const uint32_t ly = tile_index<G, Y>(lane, wave, (q << 1) | h);
            check((lx ^ (flip ? M : 0u)) == ly, "transpose delivers the layout's amplitude", g,
                  lx, ly);
          }
        }
      for (int i = 0; i < PHYS; ++i)
        check((lds[i] >= 0) == (reads[i] == 1), "every written slot read once", g, i);
    }
}

// The in-register exchanges swap_slot<RS, LS> makes (register slot RS with
// lane slot LS), applied in the mixers' order to layout X's slot table, give
// layout Y's.
template <class G>
void check_swaps(const char* g, int X, int Y, std::initializer_list<std::pair<int, int>> sw) {
  int reg[8], lane[6], wave[2];
  for (int s = 0; s < G::R; ++s) reg[s] = G::reg_bit(X, s);
  for (int s = 0; s < 6; ++s) lane[s] = G::lane_bit(X, s);
  for (int s = 0; s < 2; ++s) wave[s] = G::wave_bit(X, s);
  for (auto [rs, ls] : sw) std::swap(reg[rs], lane[ls]);
  bool same = true;
  for (int s = 0; s < G::R; ++s) same &= reg[s] == G::reg_bit(Y, s);
  for (int s = 0; s < 6; ++s) same &= lane[s] == G::lane_bit(Y, s);
  for (int s = 0; s < 2; ++s) same &= wave[s] == G::wave_bit(Y, s);
  check(same, "register/lane exchanges map the layouts", g, X, Y);
}

// The rounds of a half-mixer, in the order the geometry runs them: layout L
// mixes its register bits at or above the pass's first mixed bit that the
// earlier rounds did not (reg_mask with DONE = the earlier layouts' register
// bits).  Over the rounds every tile bit of [MIXLO, K) must be mixed exactly
// once and no other bit.
template <class G, int MIXLO, uint32_t DONE>
void rounds(uint32_t&, bool&) {}
template <class G, int MIXLO, uint32_t DONE, int L, int... Rest>
void rounds(uint32_t& mixed, bool& twice) {
  constexpr unsigned rm = reg_mask<G, L, DONE, MIXLO>();
  for (int s = 0; s < G::R; ++s)
    if ((rm >> s) & 1u) {
      const uint32_t bit = 1u << G::reg_bit(L, s);
      twice |= (mixed & bit) != 0;
      mixed |= bit;
    }
  rounds<G, MIXLO, DONE | reg_bits_of<G, L>(), Rest...>(mixed, twice);
}
template <class G, int MIXLO, int... Ls>
void check_rounds(const char* g) {
  constexpr int K = Dim<G>::K;
  uint32_t want = 0;
  for (int b = MIXLO; b < K; ++b) want |= 1u << b;
  uint32_t mixed = 0;
  bool twice = false;
  rounds<G, MIXLO, 0u, Ls...>(mixed, twice);
  check(!twice, "no tile bit mixed twice in a half-mixer", g, MIXLO);
  check(mixed == want, "a half-mixer mixes exactly its bits", g, MIXLO, mixed);
}

// ---- geometries --------------------------------------------------------------

using G13D = G13T<double2, double, 2>;
template <int C>
using G13C = G13T<float2, float, C>;
using G12D = G12T<double2, double, 2>;

template <class G>
void check_pass(const char* g, int n, int kind, int a) {
  constexpr int K = Dim<G>::K;
  if (kind == 1) {
    check_offsets<G, G::LA>(g, n, 1, a);
    check_offsets<G, G::template PL<1>>(g, n, 1, a);
  } else {
    check_offsets<G, G::LA>(g, n, 2, a);
    check_offsets<G, G::template PL<2>>(g, n, 2, a);
  }
  uint64_t local = 0;
  for (uint32_t l = 0; l < (1u << K); ++l) local |= dep<G::C>(l, kind, a);
  check_blocks<K, G::C>(g, n, kind, a, local);
}

template <int... Cs>
struct C14 {
  static void pass(int c, const char* g, int n, int kind, int a) {
    bool done = false;
    ((c == Cs ? (check_pass<G14T<Cs>>(g, n, kind, a), done = true) : false), ...);
    check(done, "geometry for the pass", g, c);
  }
};
template <int... Cs>
struct C13 {
  static void pass(int c, const char* g, int n, int kind, int a) {
    bool done = false;
    ((c == Cs ? (check_pass<G13C<Cs>>(g, n, kind, a), done = true) : false), ...);
    check(done, "geometry for the pass", g, c);
  }
};

template <class G, int M>
void transposes_set0_seq() {
  check_transpose<G, G::L_A1, G::L_B, M>("A1->B");
  check_transpose<G, G::L_B, G::L_A1, M>("B->A1");
  check_rounds<G, M, G::L_A, G::L_A1, G::L_B, G::L_B1>("set-0 sequence, lead");
  check_rounds<G, M, G::L_B1, G::L_B, G::L_A1, G::L_A>("set-0 sequence, trail");
}
template <class G, int M>
void transposes_b2_seq() {
  check_transpose<G, G::L_A, G::L_B2, M>("A->B2");
  check_transpose<G, G::L_B2, G::L_A, M>("B2->A");
}

template <class G, int M>
void g14_b2(const char* g) {
  transposes_b2_seq<G, M>();
  check_rounds<G, M, G::L_A, G::L_B2>(g);
  check_rounds<G, M, G::L_B2, G::L_A>(g);
}
template <class G, int M>
void g13_b2(const char* g) {
  transposes_b2_seq<G, M>();
  check_rounds<G, M, G::L_A, G::L_B2, G::L_B3>(g);
  check_rounds<G, M, G::L_B3, G::L_B2, G::L_A>(g);
}
template <int... Ms>
void g14_kind2(std::integer_sequence<int, Ms...>) {
  (g14_b2<G14T<(Ms < 8 ? Ms : 8)>, Ms>("G14T kind 2"), ...);
}
template <int... Ms>
void g13c_kind2(std::integer_sequence<int, Ms...>) {
  (g13_b2<G13C<(Ms < 8 ? Ms : 8)>, Ms>("G13T kind 2"), ...);
}
template <int... Ms>
void g13d_kind2(std::integer_sequence<int, Ms...>) {
  (transposes_set0_seq<G13D, Ms + 2>(), ...);
}
template <int... Ms>
void g12d_kind2(std::integer_sequence<int, Ms...>) {
  (transposes_set0_seq<G12D, Ms + 2>(), ...);
}

// The work-group -> tile order of the passes: a bijection of [0, grid) for
// every grid, and on grids that are a multiple of 8 GRP each XCD (work-group
// index mod 8) runs GRP consecutive tiles back to back.
template <int GRP>
void check_xcd_map() {
  for (uint32_t grid : {1u, 7u, 8u, 16u, 24u, 32u, 40u, 64u, 96u, 128u, 200u, 1024u, 4096u, 65536u}) {
    std::vector<int> seen(grid, 0);
    bool inside = true;
    for (uint32_t b = 0; b < grid; ++b) {
      const uint32_t t = xcd_map<GRP>(b, grid);
      if (t >= grid) inside = false;
      else ++seen[t];
    }
    check(inside, "xcd_map stays inside the grid", "xcd", GRP, grid);
    check(std::all_of(seen.begin(), seen.end(), [](int c) { return c == 1; }),
          "xcd_map is a bijection", "xcd", GRP, grid);
    if (grid % (8u * GRP)) {
      bool id = true;
      for (uint32_t b = 0; b < grid; ++b) id = id && xcd_map<GRP>(b, grid) == b;
      check(id, "xcd_map is the identity on other grids", "xcd", GRP, grid);
      continue;
    }
    bool grouped = true;
    for (uint32_t b = 0; b < grid; b += 8u * GRP)
      for (uint32_t x = 0; x < 8; ++x)
        for (uint32_t j = 0; j < (uint32_t)GRP; ++j)
          grouped = grouped && xcd_map<GRP>(b + 8u * j + x, grid) == b + GRP * x + j;
    check(grouped, "xcd_map deals GRP consecutive tiles to one XCD", "xcd", GRP, grid);
  }
}

template <class G, int... Ls>
void layouts(const char* g, std::integer_sequence<int, Ls...>) {
  (check_layout<G, Ls>(g), ...);
}

}  // namespace

int main() {
  // work-group -> tile order
  check_xcd_map<1>();
  check_xcd_map<2>();
  check_xcd_map<4>();
  check_xcd_map<8>();
  check_xcd_map<16>();
  check_xcd_map<32>();
  // layouts
  layouts<G14T<4>>("G14T", std::make_integer_sequence<int, 5>());
  layouts<G13D>("G13T", std::make_integer_sequence<int, 6>());
  layouts<G12D>("G12T", std::make_integer_sequence<int, 4>());
  // register/lane exchanges of every half-mixer, both directions
  for (auto [x, y] : {std::pair{0, 1}, std::pair{1, 0}}) {
    check_swaps<G14T<4>>("G14T", x, y, {{4, 4}, {5, 5}});
    check_swaps<G13D>("G13T", x, y, {{3, 4}, {4, 5}});
    check_swaps<G12D>("G12T", x, y, {{1, 3}, {2, 4}, {3, 5}});
  }
  for (auto [x, y] : {std::pair{2, 3}, std::pair{3, 2}}) {
    check_swaps<G14T<4>>("G14T", x, y, {{5, 4}});
    check_swaps<G13D>("G13T", x, y, {{3, 4}, {4, 5}});
    check_swaps<G12D>("G12T", x, y, {{2, 4}, {3, 5}});
  }
  check_swaps<G13D>("G13T", 4, 5, {{1, 4}});
  check_swaps<G13D>("G13T", 5, 4, {{1, 4}});
  // transposes of every half-mixer sequence the kernels make
  transposes_set0_seq<G14T<4>, 0>();
  g14_kind2(std::integer_sequence<int, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13>());
  transposes_set0_seq<G13D, 0>();
  g13d_kind2(std::make_integer_sequence<int, 11>());  // MIXLO 2..12
  transposes_set0_seq<G13C<4>, 0>();
  g13c_kind2(std::integer_sequence<int, 4, 5, 6, 7, 8, 9, 10, 11, 12>());
  transposes_set0_seq<G12D, 0>();
  g12d_kind2(std::make_integer_sequence<int, 10>());  // MIXLO 2..11

  // global offsets and tile bases of every register-tile pass of the plans
  qaoa_ctx* h = nullptr;
  if (qaoa_create(&h, QAOA_DEVICE_NONE, 0) != QAOA_OK) {
    std::printf("FAIL host context\n");
    return 1;
  }
  std::vector<int> rec(10 * 400);
  long passes = 0;
  for (int prec = 0; prec < 2; ++prec)
    for (int grad = 0; grad < 2; ++grad)
      for (int n = 1; n <= QAOA_MAX_N; ++n) {
        int np = 0;
        if (qaoa_plan_passes(h, prec, n, 3, grad, rec.data(), 400, &np) != QAOA_OK) {
          check(false, "plan", qaoa_last_error(), n);
          continue;
        }
        for (int i = 0; i < np; ++i) {
          const int* d = &rec[10 * i];
          const int k = d[1], c = d[2], a = d[3], mixlo = d[4], kind = d[9];
          if (kind == 0) continue;  // LDS-tile pass
          ++passes;
          // the transposes above cover MIXLO 0 for set 0 and these ranges otherwise
          const int lo = (prec == QAOA_C128) ? 2 : 4;
          const int hi = (prec == QAOA_C64 && !grad) ? 13 : (prec == QAOA_C64 || !grad) ? 12 : 11;
          check(kind == 1 ? mixlo == 0 : (mixlo >= lo && mixlo <= hi), "MIXLO inside the checked range",
                "plans", n, mixlo);
          if (prec == QAOA_C64 && !grad) {
            check(k == 14, "complex64 forward tile", "G14T", n, k);
            C14<4, 5, 6, 7, 8>::pass(kind == 1 ? 4 : c, "G14T", n, kind, a);
            if (kind == 2) check(c == std::min(mixlo, 8), "contiguous bits follow MIXLO", "G14T", n);
          } else if (prec == QAOA_C128 && !grad) {
            check(k == 13 && (kind == 1 || c == 2), "complex128 forward tile", "G13D", n, c);
            check_pass<G13D>("G13D", n, kind, a);
          } else if (prec == QAOA_C64 && grad) {
            check(k == 13, "complex64 gradient tile", "G13C", n, k);
            C13<4, 5, 6, 7, 8>::pass(kind == 1 ? 4 : c, "G13C", n, kind, a);
          } else {
            check(k == 12 && (kind == 1 || c == 2), "complex128 gradient tile", "G12D", n, c);
            check_pass<G12D>("G12D", n, kind, a);
          }
        }
      }
  qaoa_destroy(h);
  check(passes > 200, "register-tile passes were checked", "plans", passes);
  if (g_fails) {
    std::printf("%d of %ld checks failed\n", g_fails, g_checks);
    return 1;
  }
  std::printf("ok %ld checks over %ld register-tile passes\n", g_checks, passes);
  return 0;
}
