// sweep.hip - the fused one-step pull update (Sect. 3, "One Step Kernels",
// pull flavour, with the non-temporal stores of "One Step Kernels with
// Non-Temporal Stores") for the SoA layout.  One launch advances the whole
// lattice by one time step from the source buffer into the destination
// buffer.
//
// Direct addressing (full array + flag field): one workgroup per (y, z)
// row, threads stride along x, so the +-x neighbour loads of a row stay
// inside one workgroup (shared L1/L2 lines) and every load and store of a
// wavefront is a contiguous run.  Periodic wrap is index arithmetic
// (Sect. 3.2); full-way bounce-back is the solid-node branch of the same
// launch (solid nodes send back what they received); half-way bounce-back
// replaces a pull from a solid neighbour by the node's own opposite slot,
// steered by a per-node 32-bit link word built once at set-up.
//
// List addressing (fluid-node vector + adjacency, Sect. 3): one thread per
// fluid node; 18 int32 adjacency entries give the slot to pull for each
// moving direction, with periodicity and half-way bounce-back already
// folded in, so the kernel has no geometry branches.
#include "diag.hpp"
#include "launch.hpp"

namespace lbm {

template <class ST, int BB>
__global__ void __launch_bounds__(ST::kRowBlockMax)
k_sweep_soa(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
            const uint8_t* __restrict__ mask, const uint32_t* __restrict__ links, int nx,
            int ny, int nz, int64_t stride, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int row = blockIdx.x;
  const int y = row % ny;
  const int z = row / ny;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int n = x + nx * row;
    uint32_t lk = 0;
    bool solid;
    if (BB == LBM_HALFWAY) {
      lk = links[n];
      solid = (lk & 1u) != 0;
      if (solid) continue;  // half-way: solid nodes hold nothing
    } else {
      solid = mask[n] != 0;
    }
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // pull source x - c_i
      const int sx = Vel::cx[i] == 1 ? xm : (Vel::cx[i] == -1 ? xp : x);
      const int sy = Vel::cy[i] == 1 ? ym : (Vel::cy[i] == -1 ? yp : y);
      const int sz = Vel::cz[i] == 1 ? zm : (Vel::cz[i] == -1 ? zp : z);
      int64_t at = (int64_t)i * stride + (sx + nx * (sy + ny * sz));
      if (BB == LBM_HALFWAY && i != 0 && ((lk >> i) & 1u)) at = (int64_t)Vel::opp[i] * stride + n;
      f[i] = ST::load(src[at], k.inv_scale);
    }
    SrStream rs((uint32_t)n, k.step, ST::kStochastic);
    if (BB == LBM_FULLWAY && solid) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        __builtin_nontemporal_store(ST::store(f[Vel::opp[i]], k.scale, rs.next()),
                                    &dst[(int64_t)i * stride + n]);
      continue;
    }
    trt_collide<R, ST::kShifted>(f, k);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &dst[(int64_t)i * stride + n]);
  }
}

// The same sweep with the diagnostics of the state it reads: one partial
// record per row (fixed-order block reduction), combined afterwards.  It
// repeats the sweep's body rather than sharing it, so that the plain sweep's
// code is untouched by the diagnostics.
template <class ST, int BB>
__global__ void __launch_bounds__(512)
k_sweep_soa_diag(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
                 const uint8_t* __restrict__ mask, const uint32_t* __restrict__ links, int nx,
                 int ny, int nz, int64_t stride, Collide<typename ST::R> k, DiagArgs d) {
  using R = typename ST::R;
  double acc[M_COUNT];
#pragma unroll
  for (int s = 0; s < M_COUNT; ++s) acc[s] = 0.0;
  const int64_t N = (int64_t)nx * ny * nz;
  const int row = blockIdx.x;
  const int y = row % ny;
  const int z = row / ny;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int n = x + nx * row;
    uint32_t lk = 0;
    bool solid;
    if (BB == LBM_HALFWAY) {
      lk = links[n];
      solid = (lk & 1u) != 0;
      if (solid) continue;
    } else {
      solid = mask[n] != 0;
    }
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int sx = Vel::cx[i] == 1 ? xm : (Vel::cx[i] == -1 ? xp : x);
      const int sy = Vel::cy[i] == 1 ? ym : (Vel::cy[i] == -1 ? yp : y);
      const int sz = Vel::cz[i] == 1 ? zm : (Vel::cz[i] == -1 ? zp : z);
      int64_t at = (int64_t)i * stride + (sx + nx * (sy + ny * sz));
      if (BB == LBM_HALFWAY && i != 0 && ((lk >> i) & 1u)) at = (int64_t)Vel::opp[i] * stride + n;
      f[i] = ST::load(src[at], k.inv_scale);
    }
    diag_node<ST>(f, !solid, n, N, d, acc);
    SrStream rs((uint32_t)n, k.step, ST::kStochastic);
    if (BB == LBM_FULLWAY && solid) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        __builtin_nontemporal_store(ST::store(f[Vel::opp[i]], k.scale, rs.next()),
                                    &dst[(int64_t)i * stride + n]);
      continue;
    }
    trt_collide<R, ST::kShifted>(f, k);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &dst[(int64_t)i * stride + n]);
  }
  block_reduce<M_COUNT>(acc, 1u << M_UMAX);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < M_COUNT; ++s) d.partials[(int64_t)blockIdx.x * kStatSlots + s] = acc[s];
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
  SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &dst[(int64_t)i * stride + n]);
}

hipError_t launch_pull(lbm_ctx* c, const void* src, void* dst) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const lbm_params& p = c->p;
    const auto k = make_collide<typename ST::R>(p, c->step);
    const T* s = (const T*)src;
    T* d = (T*)dst;
    const size_t lds = sweep_lds(c, 0);
    if (p.addressing == LBM_LIST) {
      const int nf = (int)c->s.n_fluid;
      if (nf == 0) return hipSuccess;
      const int blk = c->block;
      hipLaunchKernelGGL(k_sweep_list<ST>, dim3((nf + blk - 1) / blk), dim3(blk), lds, c->stream,
                         s, d, c->b.adj, nf, c->s.stride, k);
      return hipGetLastError();
    }
    int blk = row_block(c);
    if (blk > ST::kRowBlockMax) blk = ST::kRowBlockMax;
    const dim3 grid((unsigned)p.ny * (unsigned)p.nz), block(blk);
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_sweep_soa<ST, LBM_FULLWAY>), grid, block, lds, c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, c->s.stride, k);
    else
      hipLaunchKernelGGL((k_sweep_soa<ST, LBM_HALFWAY>), grid, block, lds, c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, c->s.stride, k);
    return hipGetLastError();
  });
}

// The one-step pull over SoA direct addressing with fused diagnostics;
// *rows receives the number of partial records written.
hipError_t launch_pull_diag(lbm_ctx* c, const void* src, void* dst, int residual_mode,
                            double* partials, int64_t* rows) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const lbm_params& p = c->p;
    const auto k = make_collide<typename ST::R>(p, c->step);
    DiagArgs d;
    d.gx = p.g[0];
    d.gy = p.g[1];
    d.gz = p.g[2];
    d.u_prev = c->b.u_prev;
    d.residual_mode = residual_mode;
    d.partials = partials;
    *rows = (int64_t)p.ny * p.nz;
    int blk = row_block(c);
    if (blk > 512) blk = 512;
    const dim3 grid((unsigned)p.ny * (unsigned)p.nz), block(blk);
    const size_t lds = sweep_lds(c, 0);
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_sweep_soa_diag<ST, LBM_FULLWAY>), grid, block, lds, c->stream,
                         (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny, p.nz,
                         c->s.stride, k, d);
    else
      hipLaunchKernelGGL((k_sweep_soa_diag<ST, LBM_HALFWAY>), grid, block, lds, c->stream,
                         (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny, p.nz,
                         c->s.stride, k, d);
    return hipGetLastError();
  });
}

}  // namespace lbm
