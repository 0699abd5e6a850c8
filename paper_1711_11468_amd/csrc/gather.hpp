// gather.hpp - node-wise access to the canonical (pre-collision) state held
// in a pull buffer, shared by the I/O and diagnostics kernels.
//
// A pull buffer holds post-collision populations.  The canonical state of a
// node is what one streaming pass delivers to it: population i comes from
// the neighbour x - c_i (periodic wrap), or, under half-way bounce-back when
// that neighbour is solid or lies beyond a wall face (an axis that does not
// wrap), from the node's own opposite slot.  For the list representation the
// adjacency list already encodes exactly this.
#pragma once

#include "d3q19.hpp"

namespace lbm {

struct View {
  int nx, ny, nz;
  int64_t stride;          // population stride (SOA) or Q (AOS)
  int64_t adj_stride;      // list adjacency: entries between directions
  const uint8_t* mask;
  const int32_t* adj;
  const int32_t* node_map;
  const int32_t* fluid_index;
  float scale, inv_scale;  // half-precision storage scale (else 1)
  int aa;                  // 0: two-lattice pull buffer; 1: AA lattice after an
                           // even number of updates (canonical in place);
                           // 2: AA lattice after an odd number (post-collision,
                           // stored reversed at the node)
  uint32_t periodic;       // bit a set: axis a wraps; else its faces are walls
};

template <int LAYOUT>
__device__ __forceinline__ int64_t vslot(int64_t n, int i, int64_t stride) {
  return LAYOUT == LBM_SOA ? (int64_t)i * stride + n : n * Q + i;
}

__device__ __forceinline__ int64_t wrap_node(const View& v, int x, int y, int z) {
  x = x < 0 ? x + v.nx : (x >= v.nx ? x - v.nx : x);
  y = y < 0 ? y + v.ny : (y >= v.ny ? y - v.ny : y);
  z = z < 0 ? z + v.nz : (z >= v.nz ? z - v.nz : z);
  return (int64_t)x + (int64_t)v.nx * ((int64_t)y + (int64_t)v.ny * z);
}

// True when (x, y, z), each coordinate at most one step outside the box,
// lies beyond a face of an axis that does not wrap (such nodes are solid).
// WALLS = 0 compiles the fully periodic lattice, where no node does.
// Callers combine it with the solid flag of the wrapped node by a
// branch-free select after an unconditional (in-bounds) load: gfx950 code
// for a short-circuit form that loads the flag only inside the branch
// reused the register of the other branch's load address for the flag and
// then loaded through it on lanes with a solid neighbour.
template <int WALLS>
__device__ __forceinline__ bool beyond_wall(const View& v, int x, int y, int z) {
  if (!WALLS) return false;
  const uint32_t p = v.periodic;
  const bool bx = ((p & 1u) == 0) & ((x < 0) | (x >= v.nx));
  const bool by = ((p & 2u) == 0) & ((y < 0) | (y >= v.ny));
  const bool bz = ((p & 4u) == 0) & ((z < 0) | (z >= v.nz));
  return bx | by | bz;
}

__device__ __forceinline__ void node_xyz(const View& v, int64_t n, int& x, int& y, int& z) {
  x = (int)(n % v.nx);
  const int64_t r = n / v.nx;
  y = (int)(r % v.ny);
  z = (int)(r / v.ny);
}

// Slot of direction i (1..18) for list node m, as the adjacency list holds
// it: read from the list, or, for the run-length list (no per-node
// adjacency), derived from the node map.  Pull semantics (slot i of the
// neighbour x - c_i, else slot opp(i) of the node) unless the lattice is an
// AA lattice after an odd number of updates (slot opp(i) of the neighbour,
// else slot i of the node).
template <int LAYOUT, int WALLS>
__device__ __forceinline__ int64_t list_slot(const View& v, int m, int i) {
  if (v.adj) return v.adj[(int64_t)(i - 1) * v.adj_stride + m];
  int x, y, z;
  node_xyz(v, v.fluid_index[m], x, y, z);
  const int sx = x - Vel::cx[i], sy = y - Vel::cy[i], sz = z - Vel::cz[i];
  const int tw = v.node_map[wrap_node(v, sx, sy, sz)];
  const int t = beyond_wall<WALLS>(v, sx, sy, sz) ? -1 : tw;
  const bool aa = v.aa == 2;
  return t >= 0 ? vslot<LAYOUT>(t, aa ? Vel::opp[i] : i, v.stride)
                : vslot<LAYOUT>(m, aa ? i : Vel::opp[i], v.stride);
}

template <class ST>
__device__ __forceinline__ double to_f64(typename ST::T raw, int i, const View& v) {
  if (ST::kShifted) return (double)ST::load(raw, v.inv_scale) + weight(i);
  return (double)raw;
}

template <class ST>
__device__ __forceinline__ typename ST::T from_f64(double f, int i, const View& v) {
  using T = typename ST::T;
  if (ST::kShifted) return (T)((f - weight(i)) * (double)v.scale);
  return (T)f;
}

// The storage value of the rest state f_i = w_i.
template <class ST>
__device__ __forceinline__ typename ST::T rest_value(int i) {
  using T = typename ST::T;
  return ST::kShifted ? (T)0 : (T)weight(i);
}

// Canonical populations of full node index `node`; false if it holds none
// (solid under half-way bounce-back).
template <class ST, int LAYOUT, int ADDR, int BB, int WALLS>
__device__ __forceinline__ bool gather_canonical(const typename ST::T* __restrict__ src,
                                                 const View& v, int64_t node, double (&f)[Q]) {
  if (ADDR == LBM_LIST) {
    const int m = v.node_map[node];
    if (m < 0) return false;
    f[0] = to_f64<ST>(src[vslot<LAYOUT>(m, 0, v.stride)], 0, v);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int64_t at = v.aa == 1 ? vslot<LAYOUT>(m, i, v.stride) : list_slot<LAYOUT, WALLS>(v, m, i);
      f[i] = to_f64<ST>(src[at], i, v);
    }
    return true;
  }
  const bool solid = v.mask[node] != 0;
  if (BB == LBM_HALFWAY && solid) return false;
  if (v.aa == 1) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = to_f64<ST>(src[vslot<LAYOUT>(node, i, v.stride)], i, v);
    return true;
  }
  int x, y, z;
  node_xyz(v, node, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int sx = x - Vel::cx[i], sy = y - Vel::cy[i], sz = z - Vel::cz[i];
    const int64_t sn = wrap_node(v, sx, sy, sz);
    // two-lattice pull buffer: slot i of the neighbour; AA after an odd
    // number of updates: slot opp(i) of the neighbour (stored reversed)
    int64_t at = vslot<LAYOUT>(sn, v.aa == 2 ? Vel::opp[i] : i, v.stride);
    if (BB == LBM_HALFWAY && i != 0) {
      const bool solid = (v.mask[sn] != 0) | beyond_wall<WALLS>(v, sx, sy, sz);
      if (solid) at = vslot<LAYOUT>(node, v.aa == 2 ? i : Vel::opp[i], v.stride);
    }
    f[i] = to_f64<ST>(src[at], i, v);
  }
  return true;
}

// e_i(rho, u) - w_i in double.
__device__ __forceinline__ double eq_shifted(int i, double rho, double ux, double uy, double uz) {
  const double cu = Vel::cx[i] * ux + Vel::cy[i] * uy + Vel::cz[i] * uz;
  const double usq = ux * ux + uy * uy + uz * uz;
  return weight(i) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
}

// Fixed-order block reduction of NV doubles: wavefront shuffles, then the
// per-wave results combined by thread 0 in wave order.  Slots whose bit is
// set in max_mask combine with fmax, the others with +.  Result valid in
// thread 0.  blockDim.x must be a multiple of 64, at most 1024.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&a)[NV], uint32_t max_mask) {
  __shared__ double sm[16][NV];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const double o = __shfl_down(a[s], off, 64);
      a[s] = ((max_mask >> s) & 1u) ? fmax(a[s], o) : a[s] + o;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < NV; ++s) sm[wid][s] = a[s];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 1; w < nw; ++w) {
#pragma unroll
      for (int s = 0; s < NV; ++s)
        a[s] = ((max_mask >> s) & 1u) ? fmax(a[s], sm[w][s]) : a[s] + sm[w][s];
    }
  }
}

}  // namespace lbm

#include <type_traits>

namespace lbm {

template <int V>
using IC = std::integral_constant<int, V>;

// Call f(walls) with walls = IC<0> for a fully periodic lattice and IC<1>
// when some axis has wall faces; the I/O and diagnostics kernels take it as
// their WALLS parameter.
template <class F>
hipError_t with_walls(const lbm_params& p, F&& f) {
  if (p.periodic == 7u) return f(IC<0>{});
  return f(IC<1>{});
}

// Call f(storage_tag, layout, addressing, bounce) with compile-time tags for
// the parameter combination of p (both lists imply half-way and share the
// LIST tag: node-wise access differs only inside list_slot).
template <class F>
hipError_t dispatch(const lbm_params& p, F&& f) {
  auto by_store = [&](auto st) -> hipError_t {
    if (p.addressing != LBM_DIRECT) {
      if (p.layout == LBM_SOA) return f(st, IC<LBM_SOA>{}, IC<LBM_LIST>{}, IC<LBM_HALFWAY>{});
      return f(st, IC<LBM_AOS>{}, IC<LBM_LIST>{}, IC<LBM_HALFWAY>{});
    }
    if (p.layout == LBM_SOA) {
      if (p.bounce == LBM_FULLWAY) return f(st, IC<LBM_SOA>{}, IC<LBM_DIRECT>{}, IC<LBM_FULLWAY>{});
      return f(st, IC<LBM_SOA>{}, IC<LBM_DIRECT>{}, IC<LBM_HALFWAY>{});
    }
    if (p.bounce == LBM_FULLWAY) return f(st, IC<LBM_AOS>{}, IC<LBM_DIRECT>{}, IC<LBM_FULLWAY>{});
    return f(st, IC<LBM_AOS>{}, IC<LBM_DIRECT>{}, IC<LBM_HALFWAY>{});
  };
  switch (p.storage) {
    case LBM_F64: return by_store(StoreF64{});
    case LBM_F32_SHIFTED: return by_store(StoreF32Shifted{});
    case LBM_F16_SHIFTED: return by_store(StoreF16Shifted{});
    default: return by_store(StoreF16ShiftedSR{});
  }
}

}  // namespace lbm
