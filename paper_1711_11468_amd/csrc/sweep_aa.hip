// sweep_aa.hip - the AA pattern (Sect. 3): one lattice updated in place by
// alternating node-local (even) and neighbour (odd) kernels; direct
// addressing in SoA and AoS layout, list addressing.  The AoS neighbour
// step runs as a z march of columns (sweep_aos.hip).
#include "gather.hpp"
#include "launch.hpp"

namespace lbm {

// The neighbour kernel holds 19 populations plus 19 wrapped source and target
// addresses; at 1024 threads per workgroup (128 VGPRs per lane) the FP64
// form spills, so the AA kernels are built for at most 512.  Both kernels
// write back into lines they (or their row neighbours) have just read; plain
// stores, which keep those lines in L2, measured 8-10 % faster on MI355X than the
// streaming non-temporal form.
constexpr int kAaMaxBlock = 512;

// Local (even) kernel: read a node's own 19 slots, collide, write f*_i into
// the node's slot opp(i).  Neighbour (odd) kernel: population i of node x is
// f*_i(x - c_i), which the local kernel left in slot opp(i) of x - c_i (or,
// under half-way bounce-back from a solid x - c_i, in slot i of x itself);
// after collision f*_i goes to slot i of x + c_i (or slot opp(i) of x when
// x + c_i is solid), where the next local kernel reads it.  Every slot is
// read and written by exactly one node, so both kernels are race-free in
// place.  Under full-way bounce-back solid nodes are storage no-ops (their
// reversal maps each slot onto itself) and are skipped.
template <class ST, int LAYOUT, int BB, bool ODD>
__global__ void __launch_bounds__(kAaMaxBlock)
k_aa_direct(typename ST::T* __restrict__ A, const uint8_t* __restrict__ mask,
         const uint32_t* __restrict__ links, int nx, int ny, int nz, int64_t stride,
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
    uint32_t lk = 0;
    bool solid;
    if (BB == LBM_HALFWAY) {
      lk = links[n];
      solid = (lk & 1u) != 0;
    } else {
      solid = mask[n] != 0;
    }
    if (solid) continue;
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      int64_t at;
      if (!ODD) {
        at = vslot<LAYOUT>(n, i, stride);
      } else {
        const int sx = Vel::cx[i] == 1 ? xm : (Vel::cx[i] == -1 ? xp : x);
        const int sy = Vel::cy[i] == 1 ? ym : (Vel::cy[i] == -1 ? yp : y);
        const int sz = Vel::cz[i] == 1 ? zm : (Vel::cz[i] == -1 ? zp : z);
        at = vslot<LAYOUT>(sx + (int64_t)nx * (sy + (int64_t)ny * sz), Vel::opp[i], stride);
        if (BB == LBM_HALFWAY && i != 0 && ((lk >> i) & 1u)) at = vslot<LAYOUT>(n, i, stride);
      }
      f[i] = ST::load(A[at], k.inv_scale);
    }
    trt_collide<R, ST::kShifted>(f, k);
    SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      int64_t at;
      if (!ODD) {
        at = vslot<LAYOUT>(n, Vel::opp[i], stride);
      } else {
        const int tx = Vel::cx[i] == 1 ? xp : (Vel::cx[i] == -1 ? xm : x);
        const int ty = Vel::cy[i] == 1 ? yp : (Vel::cy[i] == -1 ? ym : y);
        const int tz = Vel::cz[i] == 1 ? zp : (Vel::cz[i] == -1 ? zm : z);
        at = vslot<LAYOUT>(tx + (int64_t)nx * (ty + (int64_t)ny * tz), i, stride);
        if (BB == LBM_HALFWAY && i != 0 && ((lk >> Vel::opp[i]) & 1u)) at = vslot<LAYOUT>(n, Vel::opp[i], stride);
      }
      A[at] = ST::store(f[i], k.scale, rs.next());
    }
  }
}

// List AA: the adjacency holds, for direction i, the slot the neighbour
// kernel reads (opp(i) of the neighbour x - c_i, or i of the node itself when
// that neighbour is solid); the slot it writes for direction i is the read
// slot of opp(i).
template <class ST, bool ODD>
__global__ void __launch_bounds__(kAaMaxBlock)
k_aa_list(typename ST::T* __restrict__ A, const int32_t* __restrict__ adj, int nf,
          int64_t stride, Collide<typename ST::R> k) {
  using R = typename ST::R;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  R f[Q];
  int32_t a[Q];
  a[0] = m;
#pragma unroll
  for (int i = 1; i < Q; ++i)
    a[i] = ODD ? adj[(int64_t)(i - 1) * stride + m] : (int32_t)((int64_t)i * stride + m);
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = ST::load(A[a[i]], k.inv_scale);
  trt_collide<R, ST::kShifted>(f, k);
  SrStream rs((uint32_t)m, k.step, ST::kStochastic);
#pragma unroll
  for (int i = 0; i < Q; ++i) A[a[Vel::opp[i]]] = ST::store(f[i], k.scale, rs.next());
}

// One in-place update of buf; c->aa_odd selects the kernel.
hipError_t launch_aa(lbm_ctx* c, void* buf) {
  if (c->p.addressing == LBM_LIST_RIA && c->aa_odd) return launch_aa_ria_odd(c, buf);
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const lbm_params& p = c->p;
    const auto k = make_collide<typename ST::R>(p, c->step);
    T* A = (T*)buf;
    const bool odd = c->aa_odd != 0;
    const size_t lds = sweep_lds(c, 0);
    if (is_list(p)) {  // the local kernel of the run-length list lands here too
      const int nf = (int)c->s.n_fluid;
      if (nf == 0) return hipSuccess;
      const int blk = c->block < kAaMaxBlock ? c->block : kAaMaxBlock;
      const dim3 g((nf + blk - 1) / blk), b(blk);
      if (odd) hipLaunchKernelGGL((k_aa_list<ST, true>), g, b, lds, c->stream, A, c->b.adj, nf, c->s.stride, k);
      else hipLaunchKernelGGL((k_aa_list<ST, false>), g, b, lds, c->stream, A, c->b.adj, nf, c->s.stride, k);
      return hipGetLastError();
    }
    if (odd && p.layout == LBM_AOS) return launch_aa_aos_odd(c, buf);  // z-marching columns
    const int rb = row_block(c);
    const dim3 g((unsigned)p.ny * (unsigned)p.nz), b(rb < kAaMaxBlock ? rb : kAaMaxBlock);
#define LBM_AA_LAUNCH(LAY, BB, ODD)                                                              \
  hipLaunchKernelGGL((k_aa_direct<ST, LAY, BB, ODD>), g, b, lds, c->stream, A, c->b.mask,      \
                     c->b.links, p.nx, p.ny, p.nz, c->s.stride, k)
#define LBM_AA_LAUNCH_L(LAY)                                  \
  if (p.bounce == LBM_FULLWAY) {                              \
    if (odd) LBM_AA_LAUNCH(LAY, LBM_FULLWAY, true);           \
    else LBM_AA_LAUNCH(LAY, LBM_FULLWAY, false);              \
  } else {                                                    \
    if (odd) LBM_AA_LAUNCH(LAY, LBM_HALFWAY, true);           \
    else LBM_AA_LAUNCH(LAY, LBM_HALFWAY, false);              \
  }
    if (p.layout == LBM_SOA) {
      LBM_AA_LAUNCH_L(LBM_SOA)
    } else {
      LBM_AA_LAUNCH_L(LBM_AOS)
    }
#undef LBM_AA_LAUNCH_L
#undef LBM_AA_LAUNCH
    return hipGetLastError();
  });
}

}  // namespace lbm
