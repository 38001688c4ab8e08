// Register-tile forward pass for complex128 states on 13-qubit tiles (gfx950).
//
// The pass structure, the mode-free tan/cot mixer with its relabelling and
// the phase decomposition are those of the complex64 pass (regtile.h), with
// FP64 arithmetic throughout: 256 threads x 32 double2 amplitudes (5 register
// bits, 6 lane bits, 2 wave bits), the same 128 VGPRs of tile as the
// complex64 pass.  The phase factors come from sincospi in FP64, so no FP32
// rounding enters the state (this library's complex128 accuracy target is
// 1e-10 relative on <C>; the paper states no tolerance).
//
// The other sets keep only 2 contiguous low tile bits (64 B runs of a
// complex128 state), so their tile mixes up to 11 qubits and n <= 24 needs
// two sets, i.e. p + 1 passes over the state for p layers.
#include "geom13.h"

namespace dq {
namespace {

using namespace rt;
using G13D = G13T<double2, double, 2>;

}  // namespace

hipError_t launch_fwd13d_pass(const PassDesc& d, int nstates, int S, int p, const void* in,
                              void* out, uint64_t state_stride, const double* W,
                              const LayerCoef* coef, double* part, void* probs, void* tab,
                              hipStream_t stream) {
  if (d.n < 14 || d.n > 34 || d.k != 13 || p < 1 || p > 64 || nstates < 1 || S < 1)
    return hipErrorInvalidValue;
  const int pt = pass_shape(d, p);
  if (pt < 0 || (d.kind == 1 && pt == P_LEAD)) return hipErrorInvalidValue;
  if (d.kind == 1 ? (d.mixlo != 0 || d.c != 13)
                  : (d.c != G13D::C || d.mixlo < 2 || d.mixlo > 12))
    return hipErrorInvalidValue;
  FwdArgs A{};
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
  const uint64_t total = (uint64_t)nstates << (d.n - 13);
  if (total > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)total), blk(NT);
  if (pt != P_LEAD && !tab) return hipErrorInvalidValue;
#define DQ_K(K, M, T) \
  hipLaunchKernelGGL((fwd_kernel<G13D, K, M, T>), grid, blk, 0, stream, A)
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
      case 2: DQ_PT(2, 2); break;
      case 3: DQ_PT(2, 3); break;
      case 4: DQ_PT(2, 4); break;
      case 5: DQ_PT(2, 5); break;
      case 6: DQ_PT(2, 6); break;
      case 7: DQ_PT(2, 7); break;
      case 8: DQ_PT(2, 8); break;
      case 9: DQ_PT(2, 9); break;
      case 10: DQ_PT(2, 10); break;
      case 11: DQ_PT(2, 11); break;
      default: DQ_PT(2, 12); break;
    }
  }
#undef DQ_PT
#undef DQ_K
  return hipGetLastError();
}

hipError_t launch_fwd13d_tables(const TabJobs& J, int n, int nstates, int S, int p,
                                const double* W, const LayerCoef* coef, void* tab,
                                hipStream_t stream) {
  return launch_all_tables<G13D>(J, n, nstates, S, p, W, coef, tab, stream);
}

}  // namespace dq
