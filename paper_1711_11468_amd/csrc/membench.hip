// membench.hip - memory micro-benchmarks mirroring the paper's Sect. 4.1 set
// (copy, copy-19, copy-19 with non-temporal stores, update-19).  They give
// the attainable HBM bandwidth for access patterns shaped like the sweeps:
// 19 read streams and 19 write streams (or 19 in-place streams).
#include "internal.hpp"

namespace lbm {

__global__ void __launch_bounds__(1024)
k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = a[k];
}

template <bool NT>
__global__ void __launch_bounds__(1024)
k_copy19(const double* __restrict__ a, double* __restrict__ b, int64_t n, int64_t stride) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double v[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) v[i] = a[i * stride + k];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (NT) __builtin_nontemporal_store(v[i], &b[i * stride + k]);
    else b[i * stride + k] = v[i];
  }
}

__global__ void __launch_bounds__(1024)
k_update19(double* __restrict__ b, int64_t n, int64_t stride, double s) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double v[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) v[i] = b[i * stride + k];
#pragma unroll
  for (int i = 0; i < 19; ++i) b[i * stride + k] = v[i] * s;
}

hipError_t launch_membench(int kind, const double* a, double* b, int64_t n, int64_t stride,
                           int block, hipStream_t stream) {
  const unsigned grid = (unsigned)((n + block - 1) / block);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_copy, dim3(grid), dim3(block), 0, stream, a, b, n); break;
    case 1:
      hipLaunchKernelGGL(k_copy19<false>, dim3(grid), dim3(block), 0, stream, a, b, n, stride);
      break;
    case 2:
      hipLaunchKernelGGL(k_copy19<true>, dim3(grid), dim3(block), 0, stream, a, b, n, stride);
      break;
    default:
      hipLaunchKernelGGL(k_update19, dim3(grid), dim3(block), 0, stream, b, n, stride, 1.0);
      break;
  }
  return hipGetLastError();
}

}  // namespace lbm
