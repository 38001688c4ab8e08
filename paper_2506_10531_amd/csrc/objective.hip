// Sampled objective of a sampler-based QAOA: CVaR_alpha of the shot
// energies C(z_s) of each problem (the measurement of Sec. IV), i.e. the
// mean over the lowest alpha fraction of the empirical distribution, the
// boundary shot weighted fractionally; alpha = 1 is the shot mean.
//
// One work-group per problem.  Shots are ranked in the strict total order
// (energy, shot index) by counting against LDS-staged chunks, so the lowest
// m = ceil(alpha K) shots are exactly those of rank < m, ties included; the
// sum is a fixed-order FP64 block reduction.
#include "internal.h"
#include "../../include/dqaoa.h"

#include <cmath>

namespace dq {
int ctx_device(qaoa_ctx* c);
namespace {

constexpr int MAX_SHOTS = 1 << 16;

__global__ void __launch_bounds__(256) cvar_kernel(int K, const double* __restrict__ cz,
                                                   double alpha, double* __restrict__ out) {
  __shared__ double ch[1024];
  __shared__ double red[4];
  const double* e = cz + (size_t)blockIdx.x * K;
  const double aK = alpha * (double)K;
  const int fl = (int)floor(aK);         // shots with full weight
  const double frac = aK - (double)fl;   // weight of the shot of rank fl
  double s = 0.0;
  for (int i0 = 0; i0 < K; i0 += 256) {
    const int i = i0 + threadIdx.x;
    const double ei = i < K ? e[i] : 0.0;
    int rank = 0;
    for (int j0 = 0; j0 < K; j0 += 1024) {
      const int c = min(1024, K - j0);
      __syncthreads();
      for (int t = threadIdx.x; t < c; t += 256) ch[t] = e[j0 + t];
      __syncthreads();
      for (int t = 0; t < c; ++t) {
        const double ej = ch[t];
        rank += (ej < ei) || (ej == ei && j0 + t < i);
      }
    }
    if (i < K) {
      if (rank < fl) s += ei;
      else if (rank == fl && frac > 0.0) s += frac * ei;
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) / aK;
}

}  // namespace
}  // namespace dq

using namespace dq;

extern "C" int qaoa_cvar(qaoa_ctx* ctx, int B, int shots, const double* cz, double alpha,
                         double* out, qaoa_stream_t stream) {
  if (!ctx) return set_error(QAOA_ERR_INVALID_ARG, "ctx is NULL");
  if (B < 1 || B > 65535) return set_error(QAOA_ERR_INVALID_ARG, "B = %d outside [1, 65535]", B);
  if (shots < 1 || shots > MAX_SHOTS)
    return set_error(QAOA_ERR_INVALID_ARG, "shots = %d outside [1, %d]", shots, MAX_SHOTS);
  if (!(alpha > 0.0 && alpha <= 1.0))
    return set_error(QAOA_ERR_INVALID_ARG, "alpha = %g outside (0, 1]", alpha);
  if (!cz || !out) return set_error(QAOA_ERR_INVALID_ARG, "cz and out must be non-NULL");
  if (ctx_device(ctx) < 0) return set_error(QAOA_ERR_NO_DEVICE, "host-only context");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  (void)hipSetDevice(ctx_device(ctx));
  hipLaunchKernelGGL(cvar_kernel, dim3(B), dim3(256), 0, (hipStream_t)stream, shots, cz, alpha,
                     out);
  hipError_t e = hipGetLastError();
  if (prev >= 0) (void)hipSetDevice(prev);
  return e == hipSuccess ? QAOA_OK : hip_error(e, "cvar kernel");
}
