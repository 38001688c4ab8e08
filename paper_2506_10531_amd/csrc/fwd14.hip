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
#include "geom14.h"

namespace dq {

using rt::G14T;
using namespace rt;

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
