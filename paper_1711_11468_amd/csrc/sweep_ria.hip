// sweep_ria.hip - sweeps over the run-length fluid list (reduced indirect
// addressing, Sect. 3 "Lattice Representation").  Consecutive fluid nodes
// of a run share one table entry per direction: node m of run r reads
// direction i from entry(i, r) + (m - run_start[r]).  A thread finds its
// run from the 64-node chunk table plus a one-byte offset, so the per-node
// addressing traffic is 1 byte instead of 18 int32 entries; lanes of one
// run read the same table words.  The kernels mirror the list kernels:
// one-step pull, AA neighbour step and one-step push (SoA, half-way
// bounce-back folded into the entries as in the adjacency list).
#include "launch.hpp"

namespace lbm {

struct RunTables {
  const int32_t* start;  // first list index of each run
  const int32_t* adj;    // [18][stride] slot of direction i for the run's first node
  const int32_t* chunk;  // run of node 64c
  const uint8_t* delta;  // run of node m minus the run of its chunk
  int64_t stride;
};

__device__ __forceinline__ void run_of(const RunTables& t, int m, int& r, int& off) {
  r = t.chunk[m >> 6] + (int)t.delta[m];
  off = m - t.start[r];
}

__device__ __forceinline__ int run_slot(const RunTables& t, int i, int r, int off) {
  return t.adj[(int64_t)(i - 1) * t.stride + r] + off;
}

// One-step pull (the run-length form of the list sweep).
template <class ST>
__global__ void __launch_bounds__(1024)
k_sweep_ria(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
            RunTables t, int nf, int64_t stride, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  int r, off;
  run_of(t, m, r, off);
  R f[Q];
  f[0] = ST::load(src[m], k.inv_scale);
#pragma unroll
  for (int i = 1; i < Q; ++i) f[i] = ST::load(src[run_slot(t, i, r, off)], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &dst[(int64_t)i * stride + m]);
}

// AA neighbour (odd) step: entries hold the AA read slots (opp(i) of the
// neighbour x - c_i, or i of the node); direction i is written to the read
// slot of opp(i).  Same register budget as the list AA kernels.
template <class ST>
__global__ void __launch_bounds__(512)
k_aa_ria_odd(typename ST::T* __restrict__ A, RunTables t, int nf, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  int r, off;
  run_of(t, m, r, off);
  R f[Q];
  int32_t a[Q];
  a[0] = m;
#pragma unroll
  for (int i = 1; i < Q; ++i) a[i] = run_slot(t, i, r, off);
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = ST::load(A[a[i]], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
#pragma unroll
  for (int i = 0; i < Q; ++i) A[a[Vel::opp[i]]] = ST::store(f[i], k.scale, rs.next());
}

// One-step push: direction i goes to the AA-style entry of opp(i) (slot i
// of the neighbour x + c_i, or slot opp(i) of the node).
template <class ST>
__global__ void __launch_bounds__(1024)
k_push_ria(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst, RunTables t,
           int nf, int64_t stride, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  int r, off;
  run_of(t, m, r, off);
  R f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = ST::load(src[(int64_t)i * stride + m], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
  dst[m] = ST::store(f[0], k.scale, rs.next());
#pragma unroll
  for (int i = 1; i < Q; ++i) dst[run_slot(t, Vel::opp[i], r, off)] = ST::store(f[i], k.scale, rs.next());
}

static RunTables tables_of(const lbm_ctx* c) {
  RunTables t;
  t.start = c->run_start;
  t.adj = c->run_adj;
  t.chunk = c->chunk_run;
  t.delta = c->run_delta;
  t.stride = c->run_stride;
  return t;
}

hipError_t launch_pull_ria(lbm_ctx* c, const void* src, void* dst) {
  const int nf = (int)c->s.n_fluid;
  if (nf == 0) return hipSuccess;
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const auto k = make_collide<typename ST::R>(c->p, c->step);
    const int blk = c->block;
    hipLaunchKernelGGL(k_sweep_ria<ST>, dim3((nf + blk - 1) / blk), dim3(blk), sweep_lds(c, 0),
                       c->stream, (const T*)src, (T*)dst, tables_of(c), nf, c->s.stride, k);
    return hipGetLastError();
  });
}

hipError_t launch_aa_ria_odd(lbm_ctx* c, void* buf) {
  const int nf = (int)c->s.n_fluid;
  if (nf == 0) return hipSuccess;
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const auto k = make_collide<typename ST::R>(c->p, c->step);
    const int blk = c->block < 512 ? c->block : 512;
    hipLaunchKernelGGL(k_aa_ria_odd<ST>, dim3((nf + blk - 1) / blk), dim3(blk), sweep_lds(c, 0),
                       c->stream, (T*)buf, tables_of(c), nf, k);
    return hipGetLastError();
  });
}

hipError_t launch_push_ria(lbm_ctx* c, const void* src, void* dst) {
  const int nf = (int)c->s.n_fluid;
  if (nf == 0) return hipSuccess;
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const auto k = make_collide<typename ST::R>(c->p, c->step);
    const int blk = c->block;
    hipLaunchKernelGGL(k_push_ria<ST>, dim3((nf + blk - 1) / blk), dim3(blk), sweep_lds(c, 0),
                       c->stream, (const T*)src, (T*)dst, tables_of(c), nf, c->s.stride, k);
    return hipGetLastError();
  });
}

}  // namespace lbm
