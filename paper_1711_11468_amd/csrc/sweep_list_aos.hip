// sweep_list_aos.hip - the fluid list with array-of-structures records
// (Table 1's list AoS forms): the populations of list node m are the 19
// consecutive values of record m, and the adjacency entries name record
// slots (record * 19 + direction).  One thread per fluid node, as for the
// SoA list; the one-step pull, the AA pattern (local and neighbour steps)
// and the one-step push share the adjacency semantics of the SoA list.
// Records are read and written per lane (152-byte lane stride in FP64), so
// all stores are plain: consecutive lanes fill the same L2 lines.
#include "launch.hpp"

namespace lbm {

constexpr int kListAosMaxBlock = 512;

template <class ST>
__global__ void __launch_bounds__(kListAosMaxBlock)
k_list_aos_pull(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
                const int32_t* __restrict__ adj, int nf, int64_t adj_stride,
                Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const int64_t rec = (int64_t)m * Q;
  R f[Q];
  f[0] = ST::load(src[rec], k.inv_scale);
#pragma unroll
  for (int i = 1; i < Q; ++i) f[i] = ST::load(src[adj[(int64_t)(i - 1) * adj_stride + m]], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[rec + i] = ST::store(f[i], k.scale, rs.next());
}

// AA: the local step reads the node's own record and writes direction i into
// slot opp(i); the neighbour step reads through the AA adjacency and writes
// direction i to the read slot of opp(i).
template <class ST, bool ODD>
__global__ void __launch_bounds__(kListAosMaxBlock)
k_list_aos_aa(typename ST::T* __restrict__ A, const int32_t* __restrict__ adj, int nf,
              int64_t adj_stride, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const int64_t rec = (int64_t)m * Q;
  int64_t a[Q];
  a[0] = rec;
#pragma unroll
  for (int i = 1; i < Q; ++i) a[i] = ODD ? (int64_t)adj[(int64_t)(i - 1) * adj_stride + m] : rec + i;
  R f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = ST::load(A[a[i]], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
#pragma unroll
  for (int i = 0; i < Q; ++i) A[a[Vel::opp[i]]] = ST::store(f[i], k.scale, rs.next());
}

// Push: direction i goes to the AA-style entry of opp(i) (slot i of the
// neighbour's record x + c_i, or slot opp(i) of the node's own record).
template <class ST>
__global__ void __launch_bounds__(kListAosMaxBlock)
k_list_aos_push(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
                const int32_t* __restrict__ adj, int nf, int64_t adj_stride,
                Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const int64_t rec = (int64_t)m * Q;
  R f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = ST::load(src[rec + i], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
  dst[rec] = ST::store(f[0], k.scale, rs.next());
#pragma unroll
  for (int i = 1; i < Q; ++i)
    dst[adj[(int64_t)(Vel::opp[i] - 1) * adj_stride + m]] = ST::store(f[i], k.scale, rs.next());
}

// One update; for the AA pattern src is the lattice and c->aa_odd picks the
// step (dst unused).
hipError_t launch_list_aos(lbm_ctx* c, const void* src, void* dst) {
  const int nf = (int)c->s.n_fluid;
  if (nf == 0) return hipSuccess;
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const auto k = make_collide<typename ST::R>(c->p, c->step);
    const int blk = c->block < kListAosMaxBlock ? c->block : kListAosMaxBlock;
    const dim3 g((nf + blk - 1) / blk), b(blk);
    const size_t lds = sweep_lds(c, 0);
    const int32_t* adj = c->b.adj;
    const int64_t as = c->adj_stride;
    switch (c->p.propagation) {
      case LBM_AA:
        if (c->aa_odd)
          hipLaunchKernelGGL((k_list_aos_aa<ST, true>), g, b, lds, c->stream, (T*)src, adj, nf, as, k);
        else
          hipLaunchKernelGGL((k_list_aos_aa<ST, false>), g, b, lds, c->stream, (T*)src, adj, nf, as, k);
        break;
      case LBM_OS_PUSH:
        hipLaunchKernelGGL(k_list_aos_push<ST>, g, b, lds, c->stream, (const T*)src, (T*)dst, adj, nf,
                           as, k);
        break;
      default:
        hipLaunchKernelGGL(k_list_aos_pull<ST>, g, b, lds, c->stream, (const T*)src, (T*)dst, adj, nf,
                           as, k);
        break;
    }
    return hipGetLastError();
  });
}

}  // namespace lbm
