// membench.hip - memory micro-benchmarks mirroring the paper's Sect. 4.1 set
// (copy, copy-19, copy-19 with non-temporal stores, update-19).  They give
// the attainable HBM bandwidth for access patterns shaped like the sweeps:
// 19 read streams and 19 write streams (or 19 in-place streams).
//
// Kinds 0-3 move one 8-byte element per thread, as the sweeps do.  Kinds
// 4-9 are tuned to bound what the memory system attains for the same
// stream counts: 16-byte accesses, several of them in flight per thread,
// non-temporal stores, and optionally a persistent grid (a fixed number of
// workgroups per compute unit striding over the arrays).
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

// S read streams copied to S write streams (or only read, or only
// written), 16 bytes per access, U accesses per stream and thread in
// flight; a grid-stride loop so that a persistent grid covers the arrays.
// n2 and stride2 count double2 elements.  MODE 0 copy, 1 read (the sum is
// stored only if it is not finite, which finite inputs never are), 2 write.
template <int S, int U, int MODE>
__global__ void __launch_bounds__(1024)
k_streams(const double2* __restrict__ a, double2* __restrict__ b, int64_t n2, int64_t stride2) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x * U;
  double acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x * U + threadIdx.x; base < n2; base += step) {
    double2 v[S][U];
    if (MODE != 2) {
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t k = base + (int64_t)u * blockDim.x;
          v[s][u] = k < n2 ? a[s * stride2 + k] : make_double2(0.0, 0.0);
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = base + (int64_t)u * blockDim.x;
        if (k >= n2) continue;
        if (MODE == 0) {
          __builtin_nontemporal_store(v[s][u].x, &b[s * stride2 + k].x);
          __builtin_nontemporal_store(v[s][u].y, &b[s * stride2 + k].y);
        } else if (MODE == 1) {
          acc += v[s][u].x + v[s][u].y;
        } else {
          __builtin_nontemporal_store((double)s, &b[s * stride2 + k].x);
          __builtin_nontemporal_store((double)u, &b[s * stride2 + k].y);
        }
      }
  }
  if (MODE == 1 && !isfinite(acc)) b[threadIdx.x] = make_double2(acc, acc);
}

// Workgroups of a persistent grid: 8 per compute unit of the device.
static unsigned persistent_grid() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;  // MI355X
  return (unsigned)(8 * cus);
}

hipError_t launch_membench(int kind, const double* a, double* b, int64_t n, int64_t stride,
                           int block, hipStream_t stream) {
  const unsigned grid = (unsigned)((n + block - 1) / block);
  if (kind >= 4) {
    const double2* a2 = (const double2*)a;
    double2* b2 = (double2*)b;
    const int64_t n2 = n / 2, s2 = stride / 2;
    auto blocks = [&](int u) { return (unsigned)((n2 + (int64_t)block * u - 1) / ((int64_t)block * u)); };
    switch (kind) {
      case 4: hipLaunchKernelGGL((k_streams<1, 4, 0>), dim3(blocks(4)), dim3(block), 0, stream, a2, b2, n2, s2); break;
      case 5: hipLaunchKernelGGL((k_streams<4, 2, 0>), dim3(blocks(2)), dim3(block), 0, stream, a2, b2, n2, s2); break;
      case 6: hipLaunchKernelGGL((k_streams<19, 1, 0>), dim3(blocks(1)), dim3(block), 0, stream, a2, b2, n2, s2); break;
      case 7: hipLaunchKernelGGL((k_streams<19, 1, 0>), dim3(persistent_grid()), dim3(block), 0, stream, a2, b2, n2, s2); break;
      case 8: hipLaunchKernelGGL((k_streams<19, 1, 1>), dim3(blocks(1)), dim3(block), 0, stream, a2, b2, n2, s2); break;
      default: hipLaunchKernelGGL((k_streams<19, 1, 2>), dim3(blocks(1)), dim3(block), 0, stream, a2, b2, n2, s2); break;
    }
    return hipGetLastError();
  }
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
