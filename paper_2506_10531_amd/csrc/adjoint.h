// Register-tile adjoint gradient (Sec. IV, Eq. (2); the adjoint method of
// the differentiation form), generic over the tile geometry and amplitude
// type: the backward sweep that propagates lambda = C psi and accumulates
// d<C>/dgamma and d<C>/dbeta, on tiles that hold psi and lambda together in
// registers (13-qubit complex64 tiles, 12-qubit complex128 tiles).
//
// Checkpoints and lambda are stored with their true scale (every pending
// mixer scalar applied), so inside a backward pass both tiles start true and
// every intermediate carries the same known real factor: for the tan-form
// butterflies of the inverse mixer e^{-i beta X} = c (I - i tan X) or
// -i s X (I + i cot X), |c|^2 or |s|^2 per qubit undone.  The X_q terms of
// d<C>/dbeta_j = -2 sum_q Im <lambda| X_q |psi> are evaluated for the qubits
// of each round just before their butterflies (X_q commutes with every factor
// of the layer's mixer, so any point of the undo gives the same value once
// the factor is divided out), and 2 Im <lambda| C |psi> for d<C>/dgamma_j at
// the phase layout (the phase leaves it unchanged).
#pragma once

#include "regtile.h"

namespace dq {
namespace rt {

template <class G>
using Tile = typename G::V[Dim<G>::NA];

// sum over the register slots in RM and the register pairs (r, r | 2^s) of
// Im(conj(l_r) p_{r|2^s}) + Im(conj(l_{r|2^s}) p_r), in the state precision.
template <class G, unsigned RM>
__device__ __forceinline__ double xq_round(const Tile<G>& p, const Tile<G>& l) {
  using S = typename G::S;
  constexpr int NA = Dim<G>::NA;
  S acc = 0;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    if (!((RM >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < NA; ++r) {
      if ((r >> s) & 1) continue;
      const int u = r | (1 << s);
      acc = fma(l[r].x, p[u].y, acc);
      acc = fma(-l[r].y, p[u].x, acc);
      acc = fma(l[u].x, p[r].y, acc);
      acc = fma(-l[u].y, p[r].x, acc);
    }
  }
  return (double)acc;
}

// Accumulator of the X_q terms of one half-mixer undo: ab += w * (terms of
// the round); w is the real factor of the tan-form tiles (times |c|^2 or
// |s|^2 per qubit undone).
struct XqAcc {
  double ab, w, q2;
};

// One round of an undo on both tiles: the round's X_q terms, then its
// butterflies.
template <class G, unsigned RM>
__device__ __forceinline__ void undo_round(Tile<G>& p, Tile<G>& l, typename G::S t, XqAcc& x) {
  if constexpr (RM != 0) {
    x.ab = fma(x.w, xq_round<G, RM>(p, l), x.ab);
    mix_round<G, RM>(p, t);
    mix_round<G, RM>(l, t);
#pragma unroll
    for (int i = 0; i < popc(RM); ++i) x.w *= x.q2;
  }
}
template <class G, int X, int Y, int MIXLO>
__device__ __forceinline__ void transpose2(Tile<G>& p, Tile<G>& l, typename G::V* buf, int lane,
                                           int wave, bool flip) {
  transpose<G, X, Y, MIXLO>(p, buf, lane, wave, flip);
  transpose<G, X, Y, MIXLO>(l, buf, lane, wave, flip);
}

// Energies of the register amplitudes, in groups of 8 (register bits 3 and
// up outer): fn(r, C(z_r)) with C in FP64 from the thread's cfix and fields.
template <int R, class F>
__device__ __forceinline__ void for_energies(const Tables<R>* T, double cfix, const double (&g)[R],
                                             F&& fn) {
#pragma unroll
  for (int hi = 0; hi < (1 << (R - 3)); ++hi) {
    double ch = cfix;
#pragma unroll
    for (int s = 3; s < R; ++s)
      if ((hi >> (s - 3)) & 1) ch += g[s];
#pragma unroll
    for (int lo = 0; lo < 8; ++lo) {
      const int r = (hi << 3) | lo;
      double c = ch + T->Kr[r];
#pragma unroll
      for (int s = 0; s < 3; ++s)
        if ((lo >> s) & 1) c += g[s];
      fn(r, c);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Undo of a half-mixer that ran L_A -> phase layout (the lead), or of one that
// ran phase layout -> L_A (the trail): the inverse butterflies commute, so
// each is undone by the sequence of the other direction with -t.  The
// sequences follow the geometry's layouts (13-qubit tiles: 5 register bits;
// 12-qubit tiles: 4).
template <class G, int KIND, int MIXLO>
__device__ __forceinline__ void undo_to_pl(Tile<G>& p, Tile<G>& l, typename G::V* buf, int lane,
                                           int wave, typename G::S t, bool flip, XqAcc& x) {
  if constexpr (G::R == 4) {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_A1>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G, G::L_B>();
    undo_round<G, reg_mask<G, G::L_A, 0, MIXLO>()>(p, l, t, x);
    G::swap_a(p), G::swap_a(l);
    undo_round<G, reg_mask<G, G::L_A1, D1, MIXLO>()>(p, l, t, x);
    transpose2<G, G::L_A1, G::L_B, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<G, reg_mask<G, G::L_B, D2, MIXLO>()>(p, l, t, x);
    G::swap_b(p), G::swap_b(l);
    undo_round<G, reg_mask<G, G::L_B1, D3, MIXLO>()>(p, l, t, x);
  } else if constexpr (KIND == 1) {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_A1>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G, G::L_B>();
    undo_round<G, reg_mask<G, G::L_A, 0, MIXLO>()>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<G, reg_mask<G, G::L_A1, D1, MIXLO>()>(p, l, t, x);
    transpose2<G, G::L_A1, G::L_B, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<G, reg_mask<G, G::L_B, D2, MIXLO>()>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<G, reg_mask<G, G::L_B1, D3, MIXLO>()>(p, l, t, x);
  } else {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B2>();
    undo_round<G, reg_mask<G, G::L_A, 0, MIXLO>()>(p, l, t, x);
    transpose2<G, G::L_A, G::L_B2, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<G, reg_mask<G, G::L_B2, D1, MIXLO>()>(p, l, t, x);
    swap_slot<G, 1, 4>(p), swap_slot<G, 1, 4>(l);
    undo_round<G, reg_mask<G, G::L_B3, D2, MIXLO>()>(p, l, t, x);
  }
}
template <class G, int KIND, int MIXLO>
__device__ __forceinline__ void undo_to_la(Tile<G>& p, Tile<G>& l, typename G::V* buf, int lane,
                                           int wave, typename G::S t, bool flip, XqAcc& x) {
  if constexpr (G::R == 4) {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_B1>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G, G::L_A1>();
    undo_round<G, reg_mask<G, G::L_B1, 0, MIXLO>()>(p, l, t, x);
    G::swap_b(p), G::swap_b(l);
    undo_round<G, reg_mask<G, G::L_B, D1, MIXLO>()>(p, l, t, x);
    transpose2<G, G::L_B, G::L_A1, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<G, reg_mask<G, G::L_A1, D2, MIXLO>()>(p, l, t, x);
    G::swap_a(p), G::swap_a(l);
    undo_round<G, reg_mask<G, G::L_A, D3, MIXLO>()>(p, l, t, x);
  } else if constexpr (KIND == 1) {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_B1>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G, G::L_A1>();
    undo_round<G, reg_mask<G, G::L_B1, 0, MIXLO>()>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<G, reg_mask<G, G::L_B, D1, MIXLO>()>(p, l, t, x);
    transpose2<G, G::L_B, G::L_A1, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<G, reg_mask<G, G::L_A1, D2, MIXLO>()>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<G, reg_mask<G, G::L_A, D3, MIXLO>()>(p, l, t, x);
  } else {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_B3>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B2>();
    undo_round<G, reg_mask<G, G::L_B3, 0, MIXLO>()>(p, l, t, x);
    swap_slot<G, 1, 4>(p), swap_slot<G, 1, 4>(l);
    undo_round<G, reg_mask<G, G::L_B2, D1, MIXLO>()>(p, l, t, x);
    transpose2<G, G::L_B2, G::L_A, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<G, reg_mask<G, G::L_A, D2, MIXLO>()>(p, l, t, x);
  }
}

// Backward pass shapes:
//   B_SEED   the last forward pass fused with its adjoint: load psi, lead
//            half-mixer, <C> and norm, lambda = C psi, undo the lead on both,
//            store lambda
//   B_MID    load psi (checkpoint) and lambda, undo the trail, 2 Im<l|C|p>,
//            undo the phase, undo the lead, store lambda
//   B_FIRST  pass 0: load psi and lambda, undo the trail, 2 Im<l|C|p>
enum { B_SEED = 0, B_MID = 1, B_FIRST = 2 };

struct BwdArgs {
  PassDesc d;
  int S, p;
  const void* psi;  // checkpoint read by this pass
  void* lam;        // lambda, read (B_MID, B_FIRST) and written (B_SEED, B_MID)
  uint64_t stride;
  const double* W;
  const LayerCoef* coef;
  double* part;  // [state][rec][2p + 2]
  int rec_base, nrec;
  const void* tab = nullptr;  // the pass's PassTab records, TAB_BYTES apart (all_tables_kernel)
};

template <class G, int KIND, int MIXLO, int BT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
bwd_kernel(BwdArgs A) {
  using D = Dim<G>;
  using V = typename G::V;
  using S = typename G::S;
  constexpr int K = D::K, NA = D::NA;
  constexpr int LA = G::LA, PL = G::template PL<KIND>;
  __shared__ V buf[D::PHYS];
  __shared__ Tables<G::R> T;
  __shared__ double fl[K];
  __shared__ double Wl[K * K];
  __shared__ double tmp[40];
  __shared__ V KF[NA];
  __shared__ LayerCoef cf[64];
  const PassDesc& d = A.d;
  const int p = A.p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = d.n, nlog = n - K;
  // runs under 128 bytes: the two tiles sharing each line run on one XCD
  const uint64_t tile = xcd_tile<(KIND == 2 && (1u << G::C) * sizeof(V) < 128) ? 2 : 1>();
  const uint64_t st = tile >> nlog, ti = tile & ((1ull << nlog) - 1ull);
  const uint64_t zb = tile_base<K, G::C>(ti, KIND, d.a);
  double* const Wsh = reinterpret_cast<double*>(buf);
  V vp[NA], vl[NA];
  const V* const psi = reinterpret_cast<const V*>(A.psi);
  V* const lam = reinterpret_cast<V*>(A.lam);
  // the tile-independent tables come from the state's PassTab (A.tab)
  constexpr int NT1 = Tables<G::R>::N - Tables<G::R>::NF;
  constexpr int NT2 = BT == B_MID ? (int)(sizeof(V) << G::R) / 8 : 0;
  const PassTab<G>* tab =
      reinterpret_cast<const PassTab<G>*>(static_cast<const char*>(A.tab) + st * TAB_BYTES);
  stage_context<NT1 + NT2>(
      A.W + (size_t)(st / A.S) * n * n, n, A.coef + st * p, p, Wsh, cf, tid,
      [&] {
        load_tile<G, LA>(vp, psi + st * A.stride + zb, lane, wave, KIND, d.a);
        if (BT != B_SEED) load_tile<G, LA>(vl, lam + st * A.stride + zb, lane, wave, KIND, d.a);
      },
      [&](int w) {
        return w < NT1 ? (&tab->T.Gl[0][0])[w] : reinterpret_cast<const double*>(tab->KF)[w - NT1];
      },
      [&](int w, double x) {
        if (w < NT1) (&T.Gl[0][0])[w] = x;
        else reinterpret_cast<double*>(KF)[w - NT1] = x;
      });
  // the half-mixer whose undo reaches the phase layout: the lead (forward,
  // B_SEED) or the trail (B_MID, B_FIRST); its cot form flips tile bit 0
  const LayerCoef& L1 = cf[BT == B_SEED ? d.lead : d.jb];
  const bool f0 = KIND == 1 && L1.mode != 0;
  const double cblk = tile_context<K, G::C, KIND>(Wsh, n, d.a, zb, f0, fl, Wl, tmp, tid);
  const double gp_undo = BT == B_SEED ? 0.0 : -cf[d.jb].gp;
  for (int e = tid; e < Tables<G::R>::NF; e += NT) table_entry<G, PL>(&T, fl, Wl, e);
  lds_barrier();
  const int m = K - MIXLO;
  // Uniform scalars, all formed before the tiles are touched: q2 per qubit of
  // each undone half-mixer, the factor |.|^2 of the tan-form tiles at the
  // start of the first undo (wa1) and at the phase layout (wa2), and the
  // scalar that makes the stored lambda true (sc).
  const LayerCoef& L2 = cf[BT == B_MID ? d.lead : 0];
  const double q2a = L1.mode == 0 ? L1.cb * L1.cb : L1.sb * L1.sb;
  const double q2b = L2.mode == 0 ? L2.cb * L2.cb : L2.sb * L2.sb;
  double wa1 = 1.0, wa2 = 1.0, sr = 1.0, si = 0.0;
  for (int i = 0; i < m; ++i) (BT == B_SEED ? wa1 : wa2) *= q2a;
  if (BT == B_SEED) half_scale(L1, m, false, sr, si);
  half_scale(L1, m, true, sr, si);
  if (BT == B_MID) half_scale(L2, m, true, sr, si);
  const V sc = mkv<V>(sr, si);
  const bool sw = KIND == 1 && BT == B_MID && (L1.mode != 0) != (L2.mode != 0);
  // factors that undo the phase of layer jb (B_MID), computed before the
  // undo so that they do not interleave with it (complex64); the FP64 factors
  // of complex128 tiles are formed where they are used, so that they do not
  // hold 20 VGPRs through the first undo
  constexpr bool EARLY_P = sizeof(V) == 8;
  PhaseF<G::R, V> P;
  if (BT == B_MID && EARLY_P)
    P = phase_factors<G, PL>(&T, fl, cblk, lane, wave, gp_undo, 1.0, 0.0);
  double se = 0.0, sn = 0.0, sg = 0.0, sb1 = 0.0, sb2 = 0.0;
  if (BT == B_SEED) {
    // forward lead half-mixer on psi, then <C>, norm and lambda = C psi
    G::template lead<KIND, MIXLO>(vp, buf, lane, wave, mix_t(L1, false), L1.mode != 0);
    __builtin_amdgcn_sched_barrier(0);
    double cfix, g[G::R];
    thread_energy<G, PL>(&T, fl, cblk, lane, wave, cfix, g);
    double ae = 0.0, an = 0.0;
    for_energies(&T, cfix, g, [&](int r, double c) {
      const double pz = (double)vp[r].x * vp[r].x + (double)vp[r].y * vp[r].y;
      ae = fma(pz, c, ae);
      an += pz;
      const S cf = (S)c;
      vl[r] = mkv<V>(cf * vp[r].x, cf * vp[r].y);
    });
    se = block_sum(ae, tmp) * wa1;
    sn = block_sum(an, tmp) * wa1;
    // undo the lead on both tiles (lambda = C psi shares psi's scalar)
    XqAcc x{0.0, wa1, q2a};
    undo_to_la<G, KIND, MIXLO>(vp, vl, buf, lane, wave, mix_t(L1, true), L1.mode != 0, x);
    sb1 = x.ab;
  } else {
    // undo the trail (layer jb) on both tiles
    XqAcc x{0.0, 1.0, q2a};
    undo_to_pl<G, KIND, MIXLO>(vp, vl, buf, lane, wave, mix_t(L1, true), L1.mode != 0, x);
    sb1 = x.ab;
    // 2 Im <lambda| C |psi> at the phase layout (the table reads stay below
    // the undo: hoisted above it they would hold registers through it)
    __builtin_amdgcn_sched_barrier(0);
    double cfix, g[G::R];
    thread_energy<G, PL>(&T, fl, cblk, lane, wave, cfix, g);
    double ag = 0.0;
    for_energies(&T, cfix, g, [&](int r, double c) {
      const S im = fma(vl[r].x, vp[r].y, -vl[r].y * vp[r].x);
      ag = fma((double)im, c, ag);
    });
    sg = block_sum(ag, tmp) * wa2;
    if (BT == B_MID) {
      // undo the phase of layer jb, then the lead (layer jb - 1)
      if (!EARLY_P) P = phase_factors<G, PL>(&T, fl, cblk, lane, wave, gp_undo, 1.0, 0.0);
      phase_tree<G::R, G::R - 1>(P, KF, P.f0, 0, [&](int r, V f) {
        vp[r] = cmul(vp[r], f);
        vl[r] = cmul(vl[r], f);
      });
      XqAcc y{0.0, wa2, q2b};
      undo_to_la<G, KIND, MIXLO>(vp, vl, buf, lane, wave, mix_t(L2, true), L2.mode != 0, y);
      sb2 = y.ab;
    }
  }
  if (BT != B_FIRST) {
    // lambda with its true scale
#pragma unroll
    for (int r = 0; r < NA; ++r) vl[r] = cmul(vl[r], sc);
    store_tile<G, LA>(vl, lam + st * A.stride + zb, lane, wave, KIND, d.a, sw);
  }
  // the pass's partial record: dgamma [0, p), dbeta [p, 2p), <C>, norm
  const double xb1 = block_sum(sb1, tmp);
  const double xb2 = BT == B_MID ? block_sum(sb2, tmp) : 0.0;
  double* o = A.part + ((uint64_t)st * A.nrec + A.rec_base + ti) * (2 * p + 2);
  for (int q = tid; q < 2 * p + 2; q += NT) {
    double v = 0.0;
    if (BT == B_SEED) {
      if (q == p + d.lead) v = -2.0 * xb1;
      if (q == 2 * p) v = se;
      if (q == 2 * p + 1) v = sn;
    } else {
      if (q == d.jb) v = 2.0 * sg;
      if (q == p + d.jb) v = -2.0 * xb1;
      if (BT == B_MID && q == p + d.lead) v = -2.0 * xb2;
    }
    o[q] = v;
  }
}

}  // namespace rt
}  // namespace dq
