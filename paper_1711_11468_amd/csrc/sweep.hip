// sweep.hip - the fused one-step pull update (paper Sect. 3, "One Step
// Kernels", pull flavour, with the non-temporal stores of Sect. 3 "One Step
// Kernels with Non-Temporal Stores").  One launch advances the whole lattice
// by one time step from the source buffer into the destination buffer.
//
// Direct addressing (full array + flag field): one workgroup per (y, z) row,
// threads stride along x, so the +-x neighbour loads of a row stay inside
// one workgroup (shared L1/L2 lines) and every load and store of a wavefront
// is a contiguous run (SoA).  Periodic wrap is index arithmetic
// (Sect. 3.2); full-way bounce-back is the solid-node branch of the same
// launch (solid nodes send back what they received), half-way bounce-back
// replaces a pull from a solid neighbour by the node's own opposite slot.
//
// List addressing (fluid-node vector + adjacency, Sect. 3): one thread per
// fluid node; 18 int32 adjacency entries give the slot to pull for each
// moving direction, with periodicity and half-way bounce-back already
// folded in, so the kernel has no geometry branches.
#include "d3q19.hpp"
#include "internal.hpp"

namespace lbm {

template <int LAYOUT>
__device__ __forceinline__ int64_t slot(int64_t n, int i, int64_t stride) {
  return LAYOUT == LBM_SOA ? (int64_t)i * stride + n : n * Q + i;
}

template <class ST, int LAYOUT, int BB>
__global__ void __launch_bounds__(1024)
k_sweep_direct(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
               const uint8_t* __restrict__ mask, int nx, int ny, int nz, int64_t stride,
               Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int row = blockIdx.x;
  const int y = row % ny;
  const int z = row / ny;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int n = x + nx * row;
    const bool solid = mask[n] != 0;
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // pull source x - c_i
      const int sx = Vel::cx[i] == 1 ? xm : (Vel::cx[i] == -1 ? xp : x);
      const int sy = Vel::cy[i] == 1 ? ym : (Vel::cy[i] == -1 ? yp : y);
      const int sz = Vel::cz[i] == 1 ? zm : (Vel::cz[i] == -1 ? zp : z);
      const int sn = sx + nx * (sy + ny * sz);
      int64_t at = slot<LAYOUT>(sn, i, stride);
      if (BB == LBM_HALFWAY && i != 0) {
        if (!solid && mask[sn] != 0) at = slot<LAYOUT>(n, Vel::opp[i], stride);
      }
      f[i] = ST::load(src[at], k.inv_scale);
    }
    if (solid) {
      if (BB == LBM_FULLWAY) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          __builtin_nontemporal_store(ST::store(f[Vel::opp[i]], k.scale),
                                      &dst[slot<LAYOUT>(n, i, stride)]);
      }
      continue;
    }
    trt_collide<R, ST::kShifted>(f, k);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store(ST::store(f[i], k.scale), &dst[slot<LAYOUT>(n, i, stride)]);
  }
}

template <class ST>
__global__ void __launch_bounds__(1024)
k_sweep_list(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
             const int32_t* __restrict__ adj, int nf, int64_t stride,
             Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  R f[Q];
  f[0] = ST::load(src[n], k.inv_scale);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int a = adj[(int64_t)(i - 1) * stride + n];
    f[i] = ST::load(src[a], k.inv_scale);
  }
  trt_collide<R, ST::kShifted>(f, k);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(ST::store(f[i], k.scale), &dst[(int64_t)i * stride + n]);
}

template <typename R>
static Collide<R> make_collide(const lbm_params& p) {
  const double tm = 0.5 + p.magic_lambda / (p.tau_plus - 0.5);
  Collide<R> k;
  k.lp = (R)(1.0 / p.tau_plus);
  k.lm = (R)(1.0 / tm);
  k.ap = (R)(1.0 - 0.5 / p.tau_plus);
  k.am = (R)(1.0 - 0.5 / tm);
  k.gx = (R)p.g[0];
  k.gy = (R)p.g[1];
  k.gz = (R)p.g[2];
  if (p.storage == LBM_F16_SHIFTED) {
    k.scale = (R)ldexp(1.0, p.f16_scale_log2);
    k.inv_scale = (R)ldexp(1.0, -p.f16_scale_log2);
  } else {
    k.scale = (R)1;
    k.inv_scale = (R)1;
  }
  return k;
}

template <class ST>
static hipError_t sweep_typed(lbm_ctx* c, const void* src, void* dst) {
  using T = typename ST::T;
  const lbm_params& p = c->p;
  const auto k = make_collide<typename ST::R>(p);
  const T* s = (const T*)src;
  T* d = (T*)dst;
  if (p.addressing == LBM_LIST) {
    const int nf = (int)c->s.n_fluid;
    if (nf == 0) return hipSuccess;
    const int blk = c->block;
    hipLaunchKernelGGL(k_sweep_list<ST>, dim3((nf + blk - 1) / blk), dim3(blk), 0, c->stream,
                       s, d, c->b.adj, nf, c->s.stride, k);
    return hipGetLastError();
  }
  int blk = c->block;
  const int nx_r = ((p.nx + 63) / 64) * 64;
  if (blk > nx_r) blk = nx_r;
  const dim3 grid((unsigned)p.ny * (unsigned)p.nz), block(blk);
#define LBM_LAUNCH(LAY, BB)                                                                   \
  hipLaunchKernelGGL((k_sweep_direct<ST, LAY, BB>), grid, block, 0, c->stream, s, d, c->b.mask, \
                     p.nx, p.ny, p.nz, c->s.stride, k)
  if (p.layout == LBM_SOA) {
    if (p.bounce == LBM_FULLWAY) LBM_LAUNCH(LBM_SOA, LBM_FULLWAY);
    else LBM_LAUNCH(LBM_SOA, LBM_HALFWAY);
  } else {
    if (p.bounce == LBM_FULLWAY) LBM_LAUNCH(LBM_AOS, LBM_FULLWAY);
    else LBM_LAUNCH(LBM_AOS, LBM_HALFWAY);
  }
#undef LBM_LAUNCH
  return hipGetLastError();
}

hipError_t launch_sweep(lbm_ctx* c, const void* src, void* dst) {
  switch (c->p.storage) {
    case LBM_F64: return sweep_typed<StoreF64>(c, src, dst);
    case LBM_F32_SHIFTED: return sweep_typed<StoreF32Shifted>(c, src, dst);
    default: return sweep_typed<StoreF16Shifted>(c, src, dst);
  }
}

}  // namespace lbm
