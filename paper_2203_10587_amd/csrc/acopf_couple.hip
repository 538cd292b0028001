// gfx950 kernels for the coupling rows between instances of a batch (paper:
// SCOPFLOW, TCOPFLOW and SOPFLOW sections, the contingency, time and scenario
// coupling constraints -delta <= x_a - x_b <= delta).  A row joins one column
// of a child instance to the same column of its parent instance in the
// packed x; the host lists both columns per row and, for the transposed
// product, every coupled column with the rows that touch it.
#include <hip/hip_runtime.h>

#include "acopf_internal.h"

namespace acopf {
namespace {

__device__ __forceinline__ void put(double* p, double v) { __builtin_nontemporal_store(v, p); }

// Lane per row: r = x[child] - x[parent]; the Jacobian row holds +1 at the
// child column and -1 at the parent column, stored in ascending column order.
__global__ __launch_bounds__(256) void k_couple_rows(const int64_t* __restrict__ cols, int64_t rows,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ c,
                                                     double* __restrict__ jac) {
  const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= rows) return;
  const int64_t a = cols[2 * r], b = cols[2 * r + 1];
  if (c) put(&c[r], x[a] - x[b]);
  if (jac) {
    const bool parent_first = b < a;
    put(&jac[2 * r], parent_first ? -1.0 : 1.0);
    put(&jac[2 * r + 1], parent_first ? 1.0 : -1.0);
  }
}

// Lane per coupled column: u[col] += the signed weights of its rows, added in
// row order (entry = row << 1 | 1 for a parent column, whose sign is -1).
// Each column has one owner, so the sum is fixed whatever the launch.
__global__ __launch_bounds__(256) void k_couple_vjp(const int64_t* __restrict__ tcol,
                                                    const int32_t* __restrict__ tptr,
                                                    const int32_t* __restrict__ tent, int32_t ncols,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ u) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  double s = 0.0;
  for (int q = tptr[j]; q < tptr[j + 1]; ++q) {
    const int32_t e = tent[q];
    const double v = w[e >> 1];
    s += (e & 1) ? -v : v;
  }
  const int64_t col = tcol[j];
  u[col] = u[col] + s;
}

}  // namespace

hipError_t launch_couple_rows(const int64_t* cols, int64_t rows, const double* x, double* c,
                              double* jac, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  const int64_t blocks = (rows + 255) / 256;
  k_couple_rows<<<static_cast<unsigned>(blocks), 256, 0, stream>>>(cols, rows, x, c, jac);
  return hipGetLastError();
}

hipError_t launch_couple_vjp(const int64_t* tcol, const int32_t* tptr, const int32_t* tent,
                             int32_t ncols, const double* w, double* u, hipStream_t stream) {
  if (ncols <= 0) return hipSuccess;
  k_couple_vjp<<<(ncols + 255) / 256, 256, 0, stream>>>(tcol, tptr, tent, ncols, w, u);
  return hipGetLastError();
}

}  // namespace acopf
