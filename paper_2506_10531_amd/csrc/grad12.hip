// Register-tile adjoint gradient for complex128 states on 12-qubit tiles
// (gfx950): the checkpoint passes and backward passes of the adjoint method
// (Sec. IV, Eq. (2); the differentiation form), on the generic machinery of
// adjoint.h.  A tile is 256 threads x 16 double2 amplitudes (4 register bits,
// 6 lane bits, 2 wave bits), so psi and lambda together take 128 VGPRs; all
// arithmetic is FP64.  Plan: set 0 = qubits [0, 12), set 1 = qubits [12, n)
// (13 <= n <= 22) on tiles of bits [0, 2) plus a 10-bit run; p + 1 passes.
#include "adjoint.h"
#include "geom12.h"

namespace dq {
namespace {

using namespace rt;

using G12D = G12T<double2, double, 2>;

}  // namespace

hipError_t launch_fwd12_ckpt_pass(const PassDesc& d, int nstates, int S, int p, const void* in,
                                  void* out, uint64_t stride, const double* W,
                                  const LayerCoef* coef, void* tab, hipStream_t stream) {
  if (d.n < 13 || d.n > 22 || p < 1 || p > 64 || nstates < 1 || S < 1) return hipErrorInvalidValue;
  const int pt = pass_shape(d, p);
  if (pt != P_FIRST && pt != P_MID) return hipErrorInvalidValue;
  if (d.kind == 2 && pt == P_FIRST) return hipErrorInvalidValue;  // set-0 first passes only
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 2 || d.mixlo > 11)) return hipErrorInvalidValue;
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
  const uint64_t total = (uint64_t)nstates << (d.n - 12);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
  if (!tab) return hipErrorInvalidValue;
#define DQ_K(K, M, T) \
  hipLaunchKernelGGL((fwd_kernel<G12D, K, M, T, true>), grid, blk, 0, stream, A)
  if (d.kind == 1) {
    if (pt == P_FIRST) DQ_K(1, 0, P_FIRST);
    else DQ_K(1, 0, P_MID);
  } else {
    switch (d.mixlo) {
      case 2: DQ_K(2, 2, P_MID); break;
      case 3: DQ_K(2, 3, P_MID); break;
      case 4: DQ_K(2, 4, P_MID); break;
      case 5: DQ_K(2, 5, P_MID); break;
      case 6: DQ_K(2, 6, P_MID); break;
      case 7: DQ_K(2, 7, P_MID); break;
      case 8: DQ_K(2, 8, P_MID); break;
      case 9: DQ_K(2, 9, P_MID); break;
      case 10: DQ_K(2, 10, P_MID); break;
      default: DQ_K(2, 11, P_MID); break;
    }
  }
#undef DQ_K
  return hipGetLastError();
}

hipError_t launch_bwd12_pass(const PassDesc& d, int shape, int nstates, int S, int p,
                             const void* psi, void* lam, uint64_t stride, const double* W,
                             const LayerCoef* coef, double* part, int rec_base, int nrec,
                             void* tab, hipStream_t stream) {
  if (d.n < 13 || d.n > 22 || p < 1 || p > 64 || nstates < 1 || S < 1) return hipErrorInvalidValue;
  if (d.kind == 1 ? d.mixlo != 0 : (d.mixlo < 2 || d.mixlo > 11)) return hipErrorInvalidValue;
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
  const uint64_t total = (uint64_t)nstates << (d.n - 12);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
  if (!tab) return hipErrorInvalidValue;
#define DQ_B(K, M, T) \
  hipLaunchKernelGGL((bwd_kernel<G12D, K, M, T>), grid, blk, 0, stream, A)
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
      case 2: DQ_BT(2, 2); break;
      case 3: DQ_BT(2, 3); break;
      case 4: DQ_BT(2, 4); break;
      case 5: DQ_BT(2, 5); break;
      case 6: DQ_BT(2, 6); break;
      case 7: DQ_BT(2, 7); break;
      case 8: DQ_BT(2, 8); break;
      case 9: DQ_BT(2, 9); break;
      case 10: DQ_BT(2, 10); break;
      default: DQ_BT(2, 11); break;
    }
  }
#undef DQ_BT
#undef DQ_B
  return hipGetLastError();
}

hipError_t launch_grad12_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                const double* W, const LayerCoef* coef, void* tab,
                                hipStream_t stream) {
  return launch_all_tables<G12D>(J, n, nstates, S, p, W, coef, tab, stream);
}

}  // namespace dq
