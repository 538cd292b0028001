// On-device random iterates for served requests: a counter-based stream
// (element j of a request drawn from its seed and j alone), so a request's
// iterate does not depend on which batch or window it is drawn in.
//
// Generator: the SplitMix64 output function (Steele, Lea and Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014) applied to
// seed + (j + 1) * gamma, gamma = 0x9E3779B97F4A7C15, then the top 53 bits as
// a double in [0, 1).  Normals by the Box-Muller transform.
#include <hip/hip_runtime.h>

#include "acopf_host.h"

namespace acopf {
namespace {

__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return static_cast<double>(z >> 11) * 0x1.0p-53;
}

// Instance k's x and lambda from its seed; the workgroups of grid row y
// stride over the n + m stream elements.
__device__ __forceinline__ void draw_one(const InstOff& I, uint64_t seed, double pmin, double pmax,
                                         double qmin, double qmax, double* x, double* lam) {
  const NetDev& N = *I.net;
  const int nb = N.nb, ng = N.ng;
  const int n = 2 * nb + 2 * ng;
  const int m = 2 * nb + 2 * (N.nl - (I.out_l >= 0 ? 1 : 0));
  double* xk = x + I.xo;
  double* lk = lam + I.co;
  const double two_pi = 6.283185307179586476925286766559;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n + m; j += gridDim.x * blockDim.x) {
    if (j < n) {
      const double u = uniform01(seed, static_cast<uint64_t>(j));
      double v;
      if (j < nb)
        v = -0.2 + 0.4 * u;
      else if (j < 2 * nb)
        v = 0.95 + 0.1 * u;
      else if (j < 2 * nb + ng)
        v = pmin + (pmax - pmin) * u;
      else
        v = qmin + (qmax - qmin) * u;
      xk[j] = v;
    } else {
      const int r = j - n;
      const double u1 = uniform01(seed, static_cast<uint64_t>(n) + 2ull * r);
      const double u2 = uniform01(seed, static_cast<uint64_t>(n) + 2ull * r + 1ull);
      lk[r] = sqrt(-2.0 * log(1.0 - u1)) * cos(two_pi * u2);
    }
  }
}

__global__ __launch_bounds__(256) void k_draw(const InstOff* __restrict__ table, int first,
                                              const uint64_t* __restrict__ seeds, double pmin,
                                              double pmax, double qmin, double qmax, double* x,
                                              double* lam) {
  const int k = first + static_cast<int>(blockIdx.y);
  draw_one(table[k], seeds[k], pmin, pmax, qmin, qmax, x, lam);
}

// A served window: the seeds travel in the launch arguments (no copy to the
// device first), and each instance's sigma is set to 1.
__global__ __launch_bounds__(256) void k_draw_window(const InstOff* __restrict__ table, int first,
                                                     WindowSeeds seeds, double pmin, double pmax,
                                                     double qmin, double qmax, double* x,
                                                     double* lam, double* sigma) {
  const int k = first + static_cast<int>(blockIdx.y);
  draw_one(table[k], seeds.s[blockIdx.y], pmin, pmax, qmin, qmax, x, lam);
  if (blockIdx.x == 0 && threadIdx.x == 0) sigma[k] = 1.0;
}

}  // namespace

hipError_t launch_draw_window(const InstOff* table, int first, int count, int max_len,
                              const uint64_t* host_seeds, double pmin, double pmax, double qmin,
                              double qmax, double* x, double* lam, double* sigma,
                              hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (count > kWindowSeeds) return hipErrorInvalidValue;
  WindowSeeds ws;
  for (int k = 0; k < count; ++k) ws.s[k] = host_seeds[k];
  const int bx = (max_len + 255) / 256 < 64 ? (max_len + 255) / 256 : 64;
  k_draw_window<<<dim3(bx > 0 ? bx : 1, count), 256, 0, stream>>>(table, first, ws, pmin, pmax,
                                                                  qmin, qmax, x, lam, sigma);
  return hipGetLastError();
}

hipError_t launch_draw(const InstOff* table, int first, int count, int max_len,
                       const uint64_t* seeds, double pmin, double pmax, double qmin, double qmax,
                       double* x, double* lam, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int bx = (max_len + 255) / 256 < 64 ? (max_len + 255) / 256 : 64;
  k_draw<<<dim3(bx > 0 ? bx : 1, count), 256, 0, stream>>>(table, first, seeds, pmin, pmax, qmin,
                                                           qmax, x, lam);
  return hipGetLastError();
}

}  // namespace acopf
