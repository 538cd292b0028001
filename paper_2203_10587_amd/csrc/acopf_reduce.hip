// gfx950 kernel for per-instance dot products over a batch's packed x
// layout: out[k] = sum_j a[xo_k + j] b[xo_k + j] over the n_k entries of
// instance k.  The backward pass of the batched VJP needs it for the weight
// of the objective gradient: d(w_f grad f . v)/d w_f = grad f . v.
//
// One workgroup per instance (a grid-stride loop over instances): thread t
// adds the products j = t, t + 256, ... in order, then a fixed pairwise tree
// over the 256 partial sums, so the result does not depend on the launch.
#include <hip/hip_runtime.h>

#include "acopf_host.h"

namespace acopf {
namespace {

constexpr int kDotThreads = 256;

__global__ __launch_bounds__(kDotThreads) void k_xdot(const InstOff* __restrict__ table, int count,
                                                      const double* __restrict__ a,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ out) {
  __shared__ double part[kDotThreads];
  const int tid = threadIdx.x;
  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    const InstOff I = table[k];
    const NetDev& N = *I.net;
    const int64_t n = 2 * int64_t(N.nb) + 2 * int64_t(N.ng) + int64_t(N.sl.ns) * N.nb;
    const double* pa = a + I.xo;
    const double* pb = b + I.xo;
    double s = 0.0;
    for (int64_t j = tid; j < n; j += kDotThreads) s = fma(pa[j], pb[j], s);
    part[tid] = s;
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h >>= 1) {
      if (tid < h) part[tid] = part[tid] + part[tid + h];
      __syncthreads();
    }
    if (tid == 0) out[k] = part[0];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_xdot(const InstOff* table, int count, const double* a, const double* b,
                       double* out, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int blocks = count < 65535 ? count : 65535;
  k_xdot<<<blocks, kDotThreads, 0, stream>>>(table, count, a, b, out);
  return hipGetLastError();
}

}  // namespace acopf
