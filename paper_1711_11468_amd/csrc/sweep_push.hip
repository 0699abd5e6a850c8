// sweep_push.hip - the one-step update, push flavour (Sect. 3, "One Step
// Kernels"); direct addressing in SoA layout and list addressing.  The AoS
// push runs as a z march of columns (sweep_aos.hip).
#include "gather.hpp"
#include "launch.hpp"

namespace lbm {

// Read the node's own 19 (pre-collision) populations from A, collide and
// write f*_i to slot i of x + c_i in B (Sect. 3 "One Step Kernels").  B then
// holds the pre-collision state of the next step in place.  The scattered,
// misaligned row stores go through L2 as plain stores (the streaming
// nontemporal form measured about 6 % slower on MI355X).  Full-way solid
// nodes send their reversed populations on; under half-way bounce-back a
// population aimed at a solid node lands in slot opp(i) of the node itself.
template <class ST, int LAYOUT, int BB>
__global__ void __launch_bounds__(1024)
k_push_direct(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
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
      if (solid) continue;
    } else {
      solid = mask[n] != 0;
    }
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = ST::load(src[vslot<LAYOUT>(n, i, stride)], k.inv_scale);
    if (!solid) {
      trt_collide<R, ST::kShifted>(f, k);
    } else {
      R g[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) g[i] = f[Vel::opp[i]];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = g[i];
    }
    SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int tx = Vel::cx[i] == 1 ? xp : (Vel::cx[i] == -1 ? xm : x);
      const int ty = Vel::cy[i] == 1 ? yp : (Vel::cy[i] == -1 ? ym : y);
      const int tz = Vel::cz[i] == 1 ? zp : (Vel::cz[i] == -1 ? zm : z);
      int64_t at = vslot<LAYOUT>(tx + (int64_t)nx * (ty + (int64_t)ny * tz), i, stride);
      // link bit opp(i): x - c_opp(i) = x + c_i is solid
      if (BB == LBM_HALFWAY && i != 0 && ((lk >> Vel::opp[i]) & 1u)) at = vslot<LAYOUT>(n, Vel::opp[i], stride);
      dst[at] = ST::store(f[i], k.scale, rs.next());
    }
  }
}

// List push: the push target of direction i is the AA-style adjacency entry
// of opp(i) (slot i of the neighbour x + c_i, or slot opp(i) of the node).
template <class ST>
__global__ void __launch_bounds__(1024)
k_push_list(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
            const int32_t* __restrict__ adj, int nf, int64_t stride, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  R f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = ST::load(src[(int64_t)i * stride + m], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
  dst[m] = ST::store(f[0], k.scale, rs.next());
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int a = adj[(int64_t)(Vel::opp[i] - 1) * stride + m];
    dst[a] = ST::store(f[i], k.scale, rs.next());
  }
}

hipError_t launch_push(lbm_ctx* c, const void* src, void* dst) {
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
      hipLaunchKernelGGL(k_push_list<ST>, dim3((nf + blk - 1) / blk), dim3(blk), lds, c->stream, s,
                         d, c->b.adj, nf, c->s.stride, k);
      return hipGetLastError();
    }
    if (p.layout == LBM_AOS) return launch_push_aos(c, src, dst);
    const dim3 g((unsigned)p.ny * (unsigned)p.nz), b(row_block(c));
#define LBM_PUSH_LAUNCH(LAY, BB)                                                                \
  hipLaunchKernelGGL((k_push_direct<ST, LAY, BB>), g, b, lds, c->stream, s, d, c->b.mask,     \
                     c->b.links, p.nx, p.ny, p.nz, c->s.stride, k)
    if (p.bounce == LBM_FULLWAY) LBM_PUSH_LAUNCH(LBM_SOA, LBM_FULLWAY);
    else LBM_PUSH_LAUNCH(LBM_SOA, LBM_HALFWAY);
#undef LBM_PUSH_LAUNCH
    return hipGetLastError();
  });
}

}  // namespace lbm
