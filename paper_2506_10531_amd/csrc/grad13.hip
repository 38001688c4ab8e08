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
#include "adjoint.h"
#include "geom13.h"

namespace dq {
namespace {

using namespace rt;

// C: contiguous low tile bits of the second set, min(MIXLO, 8) (its run of
// high tile bits is exactly its qubits)
template <int C>
using G13C = G13T<float2, float, C>;
using G13 = G13C<4>;


}  // namespace

hipError_t launch_fwd13_ckpt_pass(const PassDesc& d, int nstates, int S, int p, const void* in,
                                  void* out, uint64_t stride, const double* W,
                                  const LayerCoef* coef, void* tab, hipStream_t stream) {
  if (d.n < 14 || d.n > 22 || p < 1 || p > 64 || nstates < 1 || S < 1) return hipErrorInvalidValue;
  const int pt = pass_shape(d, p);
  if (pt != P_FIRST && pt != P_MID) return hipErrorInvalidValue;
  if (d.kind == 2 && pt == P_FIRST) return hipErrorInvalidValue;  // set-0 first passes only
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 4 || d.mixlo > 12)) return hipErrorInvalidValue;
  if (d.kind == 2 && d.c != (d.mixlo < 8 ? d.mixlo : 8)) return hipErrorInvalidValue;
  FwdArgs A{};
  A.d = d;
  A.S = S;
  A.p = p;
  A.in = in;
  A.out = out;
  A.stride = stride;
  A.W = W;
  A.coef = coef;
  A.tab = tab;
  const uint64_t total = (uint64_t)nstates << (d.n - 13);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
  if (!tab) return hipErrorInvalidValue;
#define DQ_K(K, M, T)                                                                  \
  hipLaunchKernelGGL((fwd_kernel<G13C<(K == 1 ? 4 : M < 8 ? M : 8)>, K, M, T, true>),       \
                     grid, blk, 0, stream, A)
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
                             void* tab, hipStream_t stream) {
  if (d.n < 14 || d.n > 22 || p < 1 || p > 64 || nstates < 1 || S < 1) return hipErrorInvalidValue;
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 4 || d.mixlo > 12)) return hipErrorInvalidValue;
  if (d.kind == 2 && d.c != (d.mixlo < 8 ? d.mixlo : 8)) return hipErrorInvalidValue;
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
  BwdArgs A{};
  A.d = d;
  A.S = S;
  A.p = p;
  A.psi = psi;
  A.lam = lam;
  A.stride = stride;
  A.W = W;
  A.coef = coef;
  A.part = part;
  A.rec_base = rec_base;
  A.nrec = nrec;
  A.tab = tab;
  const uint64_t total = (uint64_t)nstates << (d.n - 13);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
  if (!tab) return hipErrorInvalidValue;
#define DQ_B(K, M, T)                                                                  \
  hipLaunchKernelGGL((bwd_kernel<G13C<(K == 1 ? 4 : M < 8 ? M : 8)>, K, M, T>), grid,       \
                     blk, 0, stream, A)
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

hipError_t launch_grad13_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                const double* W, const LayerCoef* coef, void* tab,
                                hipStream_t stream) {
  return launch_all_tables<G13C<4>>(J, n, nstates, S, p, W, coef, tab, stream);
}

}  // namespace dq
