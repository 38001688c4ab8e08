// Register-tile adjoint gradient for complex64 states on 13-qubit tiles
// (gfx950): the forward sweep that writes one checkpoint per pass and the
// backward sweep that propagates lambda = C psi and accumulates d<C>/dgamma
// and d<C>/dbeta (Sec. IV, Eq. (2) of the paper; the adjoint method of the
// differentiation form).
//
// The plan is the two-set pass plan of the forward register-tile pass with
// 13-qubit tiles: set 0 = qubits [0, 13), set 1 = qubits [13, n) (n <= 22),
// whose tiles are bits [0, 4) plus a 9-bit run.  A tile is 256 threads x 32
// amplitudes (5 register bits, 6 lane bits, 2 wave bits), so the backward
// pass holds both psi and lambda in registers (128 VGPRs).
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
#include "geom13.h"

namespace dq {
namespace {

using namespace rt;

using G13 = G13T<float2, float, 4>;

using V32 = float2[32];

// sum over the register slots in RM and the register pairs (r, r | 2^s) of
// Im(conj(l_r) p_{r|2^s}) + Im(conj(l_{r|2^s}) p_r), in FP32.
template <unsigned RM>
__device__ __forceinline__ float xq_round(const V32& p, const V32& l) {
  float acc = 0.0f;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    if (!((RM >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      if ((r >> s) & 1) continue;
      const int u = r | (1 << s);
      acc = fmaf(l[r].x, p[u].y, acc);
      acc = fmaf(-l[r].y, p[u].x, acc);
      acc = fmaf(l[u].x, p[r].y, acc);
      acc = fmaf(-l[u].y, p[r].x, acc);
    }
  }
  return acc;
}

// Accumulator of the X_q terms of one half-mixer undo: ab += w * (terms of
// the round); w is the real factor of the tan-form tiles (times |c|^2 or
// |s|^2 per qubit undone).
struct XqAcc {
  double ab, w, q2;
};

// One round of an undo on both tiles: the round's X_q terms, then its
// butterflies.
template <unsigned RM, int CNT>
__device__ __forceinline__ void undo_round(V32& p, V32& l, float t, XqAcc& x) {
  if constexpr (RM != 0) {
    x.ab = fma(x.w, (double)xq_round<RM>(p, l), x.ab);
    mix_round<G13, RM>(p, t);
    mix_round<G13, RM>(l, t);
#pragma unroll
    for (int i = 0; i < popc(RM); ++i) x.w *= x.q2;
  }
}
template <int X, int Y, int MIXLO>
__device__ __forceinline__ void transpose2(V32& p, V32& l, float2* buf, int lane, int wave,
                                           bool flip) {
  transpose<G13, X, Y, MIXLO>(p, buf, lane, wave, flip);
  transpose<G13, X, Y, MIXLO>(l, buf, lane, wave, flip);
}

// Energies of the 32 register amplitudes, in groups of 8 (register bits 3, 4
// outer): fn(r, C(z_r)) with C in FP64 from the thread's cfix and fields.
template <class F>
__device__ __forceinline__ void for_energies(const Tables<5>* T, double cfix, const double (&g)[5],
                                             F&& fn) {
#pragma unroll
  for (int hi = 0; hi < 4; ++hi) {
    double ch = cfix;
    if (hi & 1) ch += g[3];
    if (hi & 2) ch += g[4];
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
// each is undone by the sequence of the other direction with -t.
template <int KIND, int MIXLO>
__device__ __forceinline__ void undo_to_pl(V32& p, V32& l, float2* buf, int lane, int wave,
                                           float t, bool flip, XqAcc& x) {
  using G = G13;
  if constexpr (KIND == 1) {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_A1>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G, G::L_B>();
    constexpr unsigned M0 = reg_mask<G, G::L_A, 0, MIXLO>();
    constexpr unsigned M1 = reg_mask<G, G::L_A1, D1, MIXLO>();
    constexpr unsigned M2 = reg_mask<G, G::L_B, D2, MIXLO>();
    constexpr unsigned M3 = reg_mask<G, G::L_B1, D3, MIXLO>();
    undo_round<M0, 0>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<M1, popc(M0)>(p, l, t, x);
    transpose2<G::L_A1, G::L_B, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<M2, popc(M0) + popc(M1)>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<M3, popc(M0) + popc(M1) + popc(M2)>(p, l, t, x);
  } else {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_A>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B2>();
    constexpr unsigned M0 = reg_mask<G, G::L_A, 0, MIXLO>();
    constexpr unsigned M1 = reg_mask<G, G::L_B2, D1, MIXLO>();
    constexpr unsigned M2 = reg_mask<G, G::L_B3, D2, MIXLO>();
    undo_round<M0, 0>(p, l, t, x);
    transpose2<G::L_A, G::L_B2, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<M1, popc(M0)>(p, l, t, x);
    swap_slot<G, 1, 4>(p), swap_slot<G, 1, 4>(l);
    undo_round<M2, popc(M0) + popc(M1)>(p, l, t, x);
  }
}
template <int KIND, int MIXLO>
__device__ __forceinline__ void undo_to_la(V32& p, V32& l, float2* buf, int lane, int wave,
                                           float t, bool flip, XqAcc& x) {
  using G = G13;
  if constexpr (KIND == 1) {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_B1>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B>();
    constexpr uint32_t D3 = D2 | reg_bits_of<G, G::L_A1>();
    constexpr unsigned M0 = reg_mask<G, G::L_B1, 0, MIXLO>();
    constexpr unsigned M1 = reg_mask<G, G::L_B, D1, MIXLO>();
    constexpr unsigned M2 = reg_mask<G, G::L_A1, D2, MIXLO>();
    constexpr unsigned M3 = reg_mask<G, G::L_A, D3, MIXLO>();
    undo_round<M0, 0>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<M1, popc(M0)>(p, l, t, x);
    transpose2<G::L_B, G::L_A1, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<M2, popc(M0) + popc(M1)>(p, l, t, x);
    swap_slot<G, 3, 4>(p), swap_slot<G, 4, 5>(p), swap_slot<G, 3, 4>(l), swap_slot<G, 4, 5>(l);
    undo_round<M3, popc(M0) + popc(M1) + popc(M2)>(p, l, t, x);
  } else {
    constexpr uint32_t D1 = reg_bits_of<G, G::L_B3>();
    constexpr uint32_t D2 = D1 | reg_bits_of<G, G::L_B2>();
    constexpr unsigned M0 = reg_mask<G, G::L_B3, 0, MIXLO>();
    constexpr unsigned M1 = reg_mask<G, G::L_B2, D1, MIXLO>();
    constexpr unsigned M2 = reg_mask<G, G::L_A, D2, MIXLO>();
    undo_round<M0, 0>(p, l, t, x);
    swap_slot<G, 1, 4>(p), swap_slot<G, 1, 4>(l);
    undo_round<M1, popc(M0)>(p, l, t, x);
    transpose2<G::L_B2, G::L_A, MIXLO>(p, l, buf, lane, wave, flip);
    undo_round<M2, popc(M0) + popc(M1)>(p, l, t, x);
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

struct BwdArgs13 {
  PassDesc d;
  int S, p;
  const float2* psi;  // checkpoint read by this pass
  float2* lam;        // lambda, read (B_MID, B_FIRST) and written (B_SEED, B_MID)
  uint64_t stride;
  const double* W;
  const LayerCoef* coef;
  double* part;  // [state][rec][2p + 2]
  int rec_base, nrec;
};

template <int KIND, int MIXLO, int BT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
bwd13_kernel(BwdArgs13 A) {
  using G = G13;
  using D = Dim<G>;
  constexpr int K = D::K, NA = D::NA;
  constexpr int LA = G::LA, PL = G::template PL<KIND>;
  __shared__ float2 buf[D::PHYS];
  __shared__ Tables<G::R> T;
  __shared__ double fl[K];
  __shared__ double Wl[K * K];
  __shared__ double tmp[40];
  __shared__ float2 KF[NA];
  __shared__ LayerCoef cf[64];
  const PassDesc& d = A.d;
  const int p = A.p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = d.n, nlog = n - K;
  const uint64_t tile = blockIdx.x;
  const uint64_t st = tile >> nlog, ti = tile & ((1ull << nlog) - 1ull);
  const uint64_t zb = tile_base<K, G::C>(ti, KIND, d.a);
  double* const Wsh = reinterpret_cast<double*>(buf);
  V32 vp, vl;
  stage_context(A.W + (size_t)(st / A.S) * n * n, n, A.coef + st * p, p, Wsh, cf, tid, [&] {
    load_tile<G, LA>(vp, A.psi + st * A.stride + zb, lane, wave, KIND, d.a);
    if (BT != B_SEED) load_tile<G, LA>(vl, A.lam + st * A.stride + zb, lane, wave, KIND, d.a);
  });
  // the half-mixer whose undo reaches the phase layout: the lead (forward,
  // B_SEED) or the trail (B_MID, B_FIRST); its cot form flips tile bit 0
  const LayerCoef& L1 = cf[BT == B_SEED ? d.lead : d.jb];
  const bool f0 = KIND == 1 && L1.mode != 0;
  const double cblk = tile_context<K, G::C, KIND>(Wsh, n, d.a, zb, f0, fl, Wl, tmp, tid);
  const double gp_undo = BT == B_SEED ? 0.0 : -cf[d.jb].gp;
  tile_tables<G, PL>(&T, KF, fl, Wl, BT == B_MID, gp_undo, tid);
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
  const float2 sc = make_float2((float)sr, (float)si);
  const bool sw = KIND == 1 && BT == B_MID && (L1.mode != 0) != (L2.mode != 0);
  // factors that undo the phase of layer jb (B_MID), computed before the
  // undo so that they do not interleave with it
  PhaseF<G::R, float2> P;
  if (BT == B_MID) P = phase_factors<G, PL>(&T, fl, cblk, lane, wave, gp_undo, 1.0, 0.0);
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
      const float cf = (float)c;
      vl[r] = make_float2(cf * vp[r].x, cf * vp[r].y);
    });
    se = block_sum(ae, tmp) * wa1;
    sn = block_sum(an, tmp) * wa1;
    // undo the lead on both tiles (lambda = C psi shares psi's scalar)
    XqAcc x{0.0, wa1, q2a};
    undo_to_la<KIND, MIXLO>(vp, vl, buf, lane, wave, mix_t(L1, true), L1.mode != 0, x);
    sb1 = x.ab;
  } else {
    // undo the trail (layer jb) on both tiles
    XqAcc x{0.0, 1.0, q2a};
    undo_to_pl<KIND, MIXLO>(vp, vl, buf, lane, wave, mix_t(L1, true), L1.mode != 0, x);
    sb1 = x.ab;
    // 2 Im <lambda| C |psi> at the phase layout (the table reads stay below
    // the undo: hoisted above it they would hold registers through it)
    __builtin_amdgcn_sched_barrier(0);
    double cfix, g[G::R];
    thread_energy<G, PL>(&T, fl, cblk, lane, wave, cfix, g);
    double ag = 0.0;
    for_energies(&T, cfix, g, [&](int r, double c) {
      const float im = fmaf(vl[r].x, vp[r].y, -vl[r].y * vp[r].x);
      ag = fma((double)im, c, ag);
    });
    sg = block_sum(ag, tmp) * wa2;
    if (BT == B_MID) {
      // undo the phase of layer jb, then the lead (layer jb - 1)
      phase_tree<G::R, G::R - 1>(P, KF, P.f0, 0, [&](int r, float2 f) {
        vp[r] = cmul(vp[r], f);
        vl[r] = cmul(vl[r], f);
      });
      XqAcc y{0.0, wa2, q2b};
      undo_to_la<KIND, MIXLO>(vp, vl, buf, lane, wave, mix_t(L2, true), L2.mode != 0, y);
      sb2 = y.ab;
    }
  }
  if (BT != B_FIRST) {
    // lambda with its true scale
#pragma unroll
    for (int r = 0; r < NA; ++r) vl[r] = cmul(vl[r], sc);
    store_tile<G, LA>(vl, A.lam + st * A.stride + zb, lane, wave, KIND, d.a, sw);
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

}  // namespace

hipError_t launch_fwd13_ckpt_pass(const PassDesc& d, int nstates, int S, int p, const void* in,
                                  void* out, uint64_t stride, const double* W,
                                  const LayerCoef* coef, hipStream_t stream) {
  if (d.n < 14 || d.n > 22 || p < 1 || p > 64 || nstates < 1 || S < 1) return hipErrorInvalidValue;
  const int pt = pass_shape(d, p);
  if (pt != P_FIRST && pt != P_MID) return hipErrorInvalidValue;
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 4 || d.mixlo > 12)) return hipErrorInvalidValue;
  FwdArgs A{};
  A.d = d;
  A.S = S;
  A.p = p;
  A.in = in;
  A.out = out;
  A.stride = stride;
  A.W = W;
  A.coef = coef;
  const uint64_t total = (uint64_t)nstates << (d.n - 13);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
#define DQ_K(K, M, T) \
  hipLaunchKernelGGL((fwd_kernel<G13, K, M, T, true>), grid, blk, 0, stream, A)
  if (d.kind == 1) {
    if (pt == P_FIRST) DQ_K(1, 0, P_FIRST);
    else DQ_K(1, 0, P_MID);
  } else {
    switch (d.mixlo) {
      case 4: DQ_K(2, 4, P_MID); break;
      case 5: DQ_K(2, 5, P_MID); break;
      case 6: DQ_K(2, 6, P_MID); break;
      case 7: DQ_K(2, 7, P_MID); break;
      case 8: DQ_K(2, 8, P_MID); break;
      case 9: DQ_K(2, 9, P_MID); break;
      case 10: DQ_K(2, 10, P_MID); break;
      case 11: DQ_K(2, 11, P_MID); break;
      default: DQ_K(2, 12, P_MID); break;
    }
  }
#undef DQ_K
  return hipGetLastError();
}

hipError_t launch_bwd13_pass(const PassDesc& d, int shape, int nstates, int S, int p,
                             const void* psi, void* lam, uint64_t stride, const double* W,
                             const LayerCoef* coef, double* part, int rec_base, int nrec,
                             hipStream_t stream) {
  if (d.n < 14 || d.n > 22 || p < 1 || p > 64 || nstates < 1 || S < 1) return hipErrorInvalidValue;
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 4 || d.mixlo > 12)) return hipErrorInvalidValue;
  const bool phase = d.ja <= d.jb;
  switch (shape) {
    case B_SEED:
      if (d.lead < 0 || d.lead >= p || phase) return hipErrorInvalidValue;
      break;
    case B_MID:
      if (d.lead < 0 || !phase || d.ja != d.jb || d.jb != d.lead + 1 || d.jb >= p)
        return hipErrorInvalidValue;
      break;
    case B_FIRST:
      if (d.lead >= 0 || !phase || d.jb != 0 || d.kind != 1) return hipErrorInvalidValue;
      break;
    default:
      return hipErrorInvalidValue;
  }
  BwdArgs13 A{};
  A.d = d;
  A.S = S;
  A.p = p;
  A.psi = reinterpret_cast<const float2*>(psi);
  A.lam = reinterpret_cast<float2*>(lam);
  A.stride = stride;
  A.W = W;
  A.coef = coef;
  A.part = part;
  A.rec_base = rec_base;
  A.nrec = nrec;
  const uint64_t total = (uint64_t)nstates << (d.n - 13);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
#define DQ_B(K, M, T) hipLaunchKernelGGL((bwd13_kernel<K, M, T>), grid, blk, 0, stream, A)
#define DQ_BT(K, M)                   \
  switch (shape) {                    \
    case B_SEED: DQ_B(K, M, B_SEED); break; \
    default: DQ_B(K, M, B_MID); break;      \
  }
  if (d.kind == 1) {
    switch (shape) {
      case B_SEED: DQ_B(1, 0, B_SEED); break;
      case B_MID: DQ_B(1, 0, B_MID); break;
      default: DQ_B(1, 0, B_FIRST); break;
    }
  } else {
    switch (d.mixlo) {
      case 4: DQ_BT(2, 4); break;
      case 5: DQ_BT(2, 5); break;
      case 6: DQ_BT(2, 6); break;
      case 7: DQ_BT(2, 7); break;
      case 8: DQ_BT(2, 8); break;
      case 9: DQ_BT(2, 9); break;
      case 10: DQ_BT(2, 10); break;
      case 11: DQ_BT(2, 11); break;
      default: DQ_BT(2, 12); break;
    }
  }
#undef DQ_BT
#undef DQ_B
  return hipGetLastError();
}

}  // namespace dq
