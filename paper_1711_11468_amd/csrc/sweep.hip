// sweep.hip - the fused one-step pull update (paper Sect. 3, "One Step
// Kernels", pull flavour, with the non-temporal stores of Sect. 3 "One Step
// Kernels with Non-Temporal Stores").  One launch advances the whole lattice
// by one time step from the source buffer into the destination buffer.
//
// Direct addressing, SoA (full array + flag field): one workgroup per (y, z)
// row, threads stride along x, so the +-x neighbour loads of a row stay
// inside one workgroup (shared L1/L2 lines) and every load and store of a
// wavefront is a contiguous run.  Periodic wrap is index arithmetic
// (Sect. 3.2); full-way bounce-back is the solid-node branch of the same
// launch (solid nodes send back what they received); half-way bounce-back
// replaces a pull from a solid neighbour by the node's own opposite slot,
// steered by a per-node 32-bit link word built once at set-up.
//
// Direct addressing, AoS: node records of 19 values are contiguous, so a
// wavefront reading one direction of 64 nodes would touch 64 records.  The
// workgroup instead stages each of the 9 source rows of its row segment
// (the rows y - c_y, z - c_z the pull reads from) into LDS with contiguous
// loads, picks the directions that row supplies, and writes its results
// back through LDS as one contiguous run of records.
//
// List addressing (fluid-node vector + adjacency, Sect. 3): one thread per
// fluid node; 18 int32 adjacency entries give the slot to pull for each
// moving direction, with periodicity and half-way bounce-back already
// folded in, so the kernel has no geometry branches.
#include "d3q19.hpp"
#include "internal.hpp"

namespace lbm {

constexpr int kLdsPerCU = 163840;  // gfx950: 160 KiB of LDS per compute unit

template <class ST, int BB>
__global__ void __launch_bounds__(1024)
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
    if (solid) {
      if (BB == LBM_FULLWAY) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          __builtin_nontemporal_store(ST::store(f[Vel::opp[i]], k.scale, rs.next()),
                                      &dst[(int64_t)i * stride + n]);
      }
      continue;
    }
    trt_collide<R, ST::kShifted>(f, k);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &dst[(int64_t)i * stride + n]);
  }
}

// AoS tile kernel.  A workgroup owns TY consecutive rows (y0 .. y0+TY-1) of
// one z-layer and walks them in x-segments of BX nodes.  The pull sources of
// that tile are the rows y0-1 .. y0+TY of the layers z, z-1 and z+1; each is
// staged once, whole records, into LDS with contiguous loads, and every
// thread takes from it the directions whose source it is for its own row
// (a staged row supplies up to three output rows).  Results leave through
// LDS again, one output row at a time, as contiguous runs of records.
template <class ST, int BB>
__global__ void __launch_bounds__(1024)
k_sweep_aos(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
            const uint8_t* __restrict__ mask, const uint32_t* __restrict__ links, int nx,
            int ny, int nz, int BX, Collide<typename ST::R> k) {
  using T = typename ST::T;
  using R = typename ST::R;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sm = reinterpret_cast<T*>(lds_raw);
  const int TY = blockDim.x / BX;
  const int t = threadIdx.x, tx = t % BX, ty = t / BX;
  const int tiles_y = (ny + TY - 1) / TY;
  const int z = blockIdx.x / tiles_y;
  const int y0 = (blockIdx.x - z * tiles_y) * TY;
  const int y = y0 + ty;
  for (int x0 = 0; x0 < nx; x0 += BX) {
    const int seg = nx - x0 < BX ? nx - x0 : BX;
    const bool active = y < ny && tx < seg;
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = R(0);
#pragma unroll
    for (int zz = 0; zz < 3; ++zz) {
      const int dz = zz == 0 ? 0 : (zz == 1 ? 1 : -1);  // c_z supplied by this layer
      int sz = z - dz;
      sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
      for (int sr = -1; sr <= TY; ++sr) {
        const int sy = ((y0 + sr) % ny + ny) % ny;
        const int64_t rbase = ((int64_t)sy + (int64_t)ny * sz) * nx;
        const int nrec = seg + 2;  // records x0-1 .. x0+seg
        __syncthreads();
        for (int e = t; e < nrec * Q; e += blockDim.x) {
          const int rr = e / Q;
          const int i = e - rr * Q;
          int xs = x0 - 1 + rr;
          xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
          sm[e] = src[(rbase + xs) * Q + i];
        }
        __syncthreads();
        if (active) {
          const int cy_req = ty - sr;  // y - c_y = y0 + sr
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            if (Vel::cz[i] != dz) continue;
            if (Vel::cy[i] == cy_req) f[i] = ST::load(sm[(tx + 1 - Vel::cx[i]) * Q + i], k.inv_scale);
          }
        }
      }
    }
    const int64_t n = ((int64_t)y + (int64_t)ny * z) * nx + x0 + tx;
    if (active) {
      bool solid;
      if (BB == LBM_HALFWAY) {
        const uint32_t lk = links[n];
        solid = (lk & 1u) != 0;
        if (!solid && (lk >> 1)) {
#pragma unroll
          for (int i = 1; i < Q; ++i)
            if ((lk >> i) & 1u) f[i] = ST::load(src[n * Q + Vel::opp[i]], k.inv_scale);
        }
      } else {
        solid = mask[n] != 0;
      }
      if (!solid) {
        trt_collide<R, ST::kShifted>(f, k);
      } else if (BB == LBM_FULLWAY) {
        R g[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] = f[Vel::opp[i]];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = g[i];
      } else {
        // half-way solids hold no state; keep their slots at the rest value
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = ST::kShifted ? R(0) : R(weight(i));
      }
    }
    for (int w = 0; w < TY; ++w) {
      __syncthreads();
      if (active && ty == w) {
        SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
        for (int i = 0; i < Q; ++i) sm[tx * Q + i] = ST::store(f[i], k.scale, rs.next());
      }
      __syncthreads();
      if (y0 + w < ny) {
        T* out = dst + (((int64_t)(y0 + w) + (int64_t)ny * z) * nx + x0) * Q;
        for (int e = t; e < seg * Q; e += blockDim.x) __builtin_nontemporal_store(sm[e], &out[e]);
      }
    }
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

// ---- AA pattern (one lattice, in place) -------------------------------------
// Local (even) kernel: read a node's own 19 slots, collide, write f*_i into
// the node's slot opp(i).  Neighbour (odd) kernel: population i of node x is
// f*_i(x - c_i), which the local kernel left in slot opp(i) of x - c_i (or,
// under half-way bounce-back from a solid x - c_i, in slot i of x itself);
// after collision f*_i goes to slot i of x + c_i (or slot opp(i) of x when
// x + c_i is solid), where the next local kernel reads it.  Every slot is
// read and written by exactly one node, so both kernels are race-free in
// place.  Under full-way bounce-back solid nodes are storage no-ops (their
// reversal maps each slot onto itself) and are skipped.
template <class ST, int BB, bool ODD>
__global__ void __launch_bounds__(1024)
k_aa_soa(typename ST::T* __restrict__ A, const uint8_t* __restrict__ mask,
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
        at = (int64_t)i * stride + n;
      } else {
        const int sx = Vel::cx[i] == 1 ? xm : (Vel::cx[i] == -1 ? xp : x);
        const int sy = Vel::cy[i] == 1 ? ym : (Vel::cy[i] == -1 ? yp : y);
        const int sz = Vel::cz[i] == 1 ? zm : (Vel::cz[i] == -1 ? zp : z);
        at = (int64_t)Vel::opp[i] * stride + (sx + nx * (sy + ny * sz));
        if (BB == LBM_HALFWAY && i != 0 && ((lk >> i) & 1u)) at = (int64_t)i * stride + n;
      }
      f[i] = ST::load(A[at], k.inv_scale);
    }
    trt_collide<R, ST::kShifted>(f, k);
    SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      int64_t at;
      if (!ODD) {
        at = (int64_t)Vel::opp[i] * stride + n;
      } else {
        const int tx = Vel::cx[i] == 1 ? xp : (Vel::cx[i] == -1 ? xm : x);
        const int ty = Vel::cy[i] == 1 ? yp : (Vel::cy[i] == -1 ? ym : y);
        const int tz = Vel::cz[i] == 1 ? zp : (Vel::cz[i] == -1 ? zm : z);
        at = (int64_t)i * stride + (tx + nx * (ty + ny * tz));
        if (BB == LBM_HALFWAY && i != 0 && ((lk >> Vel::opp[i]) & 1u)) at = (int64_t)Vel::opp[i] * stride + n;
      }
      __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &A[at]);
    }
  }
}

// List AA: the adjacency holds, for direction i, the slot the neighbour
// kernel reads (opp(i) of the neighbour x - c_i, or i of the node itself when
// that neighbour is solid); the slot it writes for direction i is the read
// slot of opp(i).
template <class ST, bool ODD>
__global__ void __launch_bounds__(1024)
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
  for (int i = 0; i < Q; ++i)
    __builtin_nontemporal_store(ST::store(f[i], k.scale, rs.next()), &A[a[Vel::opp[i]]]);
}

// ---- one step, push flavour ----------------------------------------------
// Read the node's own 19 (pre-collision) populations from A, collide and
// write f*_i to slot i of x + c_i in B (Sect. 3 "One Step Kernels").  B then
// holds the pre-collision state of the next step in place.  The scattered,
// misaligned row stores go through L2 as plain stores (the streaming
// nontemporal form measured about 6 % slower here).  Full-way solid
// nodes send their reversed populations on; under half-way bounce-back a
// population aimed at a solid node lands in slot opp(i) of the node itself.
template <class ST, int BB>
__global__ void __launch_bounds__(1024)
k_push_soa(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
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
    for (int i = 0; i < Q; ++i) f[i] = ST::load(src[(int64_t)i * stride + n], k.inv_scale);
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
      int64_t at = (int64_t)i * stride + (tx + nx * (ty + ny * tz));
      // link bit opp(i): x - c_opp(i) = x + c_i is solid
      if (BB == LBM_HALFWAY && i != 0 && ((lk >> Vel::opp[i]) & 1u)) at = (int64_t)Vel::opp[i] * stride + n;
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

// Link words for half-way bounce-back on the full array: bit 0 = the node is
// solid, bit i (1..18) = the pull source x - c_i is solid.
__global__ void k_build_links(const uint8_t* __restrict__ mask, uint32_t* __restrict__ links,
                              int nx, int ny, int nz) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (n >= N) return;
  const int x = (int)(n % nx);
  const int64_t r = n / nx;
  const int y = (int)(r % ny), z = (int)(r / ny);
  uint32_t w = mask[n] != 0 ? 1u : 0u;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int sx = wrap_sub(x, Vel::cx[i], nx);
    const int sy = wrap_sub(y, Vel::cy[i], ny);
    const int sz = wrap_sub(z, Vel::cz[i], nz);
    if (mask[sx + (int64_t)nx * (sy + (int64_t)ny * sz)] != 0) w |= 1u << i;
  }
  links[n] = w;
}

hipError_t launch_build_links(lbm_ctx* c) {
  const int64_t N = c->s.n_nodes;
  hipLaunchKernelGGL(k_build_links, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                     c->b.mask, c->b.links, c->p.nx, c->p.ny, c->p.nz);
  return hipGetLastError();
}

template <typename R>
static Collide<R> make_collide(const lbm_params& p, int64_t step) {
  const double tm = 0.5 + p.magic_lambda / (p.tau_plus - 0.5);
  Collide<R> k;
  k.lp = (R)(1.0 / p.tau_plus);
  k.lm = (R)(1.0 / tm);
  k.ap = (R)(1.0 - 0.5 / p.tau_plus);
  k.am = (R)(1.0 - 0.5 / tm);
  k.gx = (R)p.g[0];
  k.gy = (R)p.g[1];
  k.gz = (R)p.g[2];
  k.step = (uint32_t)step;
  if (p.storage == LBM_F16_SHIFTED || p.storage == LBM_F16_SHIFTED_SR) {
    k.scale = (R)ldexp(1.0, p.f16_scale_log2);
    k.inv_scale = (R)ldexp(1.0, -p.f16_scale_log2);
  } else {
    k.scale = (R)1;
    k.inv_scale = (R)1;
  }
  return k;
}

// Dynamic LDS of a sweep launch: what the kernel needs, raised so that at
// most cu_slots workgroups fit on one compute unit when a cap is set.
static size_t sweep_lds(const lbm_ctx* c, size_t need) {
  if (c->p.cu_slots > 0) {
    size_t cap = (size_t)(kLdsPerCU / c->p.cu_slots) & ~(size_t)255;
    if (cap > need) return cap;
  }
  return need;
}

size_t aos_lds_bytes(const lbm_ctx* c, int bx) {
  const int es = c->p.storage == LBM_F64 ? 8 : (c->p.storage == LBM_F32_SHIFTED ? 4 : 2);  // F16: 2
  return (size_t)(bx + 2) * Q * es;
}

template <class ST>
static hipError_t sweep_typed(lbm_ctx* c, const void* src, void* dst) {
  using T = typename ST::T;
  const lbm_params& p = c->p;
  const auto k = make_collide<typename ST::R>(p, c->step);
  const T* s = (const T*)src;
  T* d = (T*)dst;
  if (p.propagation == LBM_AA) {
    // in place on the source buffer; c->aa_odd selects the kernel
    T* A = (T*)src;
    const bool odd = c->aa_odd != 0;
    if (p.addressing == LBM_LIST) {
      const int nf = (int)c->s.n_fluid;
      if (nf == 0) return hipSuccess;
      const int blk = c->block;
      const dim3 g((nf + blk - 1) / blk), b(blk);
      if (odd) hipLaunchKernelGGL((k_aa_list<ST, true>), g, b, sweep_lds(c, 0), c->stream, A, c->b.adj, nf, c->s.stride, k);
      else hipLaunchKernelGGL((k_aa_list<ST, false>), g, b, sweep_lds(c, 0), c->stream, A, c->b.adj, nf, c->s.stride, k);
      return hipGetLastError();
    }
    int blk = c->block;
    const int nx_r = ((p.nx + 63) / 64) * 64;
    if (blk > nx_r) blk = nx_r;
    const dim3 g((unsigned)p.ny * (unsigned)p.nz), b(blk);
    const size_t lds = sweep_lds(c, 0);
#define LBM_AA_LAUNCH(BB, ODD)                                                                   \
  hipLaunchKernelGGL((k_aa_soa<ST, BB, ODD>), g, b, lds, c->stream, A, c->b.mask, c->b.links, p.nx, \
                     p.ny, p.nz, c->s.stride, k)
    if (p.bounce == LBM_FULLWAY) {
      if (odd) LBM_AA_LAUNCH(LBM_FULLWAY, true);
      else LBM_AA_LAUNCH(LBM_FULLWAY, false);
    } else {
      if (odd) LBM_AA_LAUNCH(LBM_HALFWAY, true);
      else LBM_AA_LAUNCH(LBM_HALFWAY, false);
    }
#undef LBM_AA_LAUNCH
    return hipGetLastError();
  }
  if (p.propagation == LBM_OS_PUSH) {
    if (p.addressing == LBM_LIST) {
      const int nf = (int)c->s.n_fluid;
      if (nf == 0) return hipSuccess;
      const int blk = c->block;
      hipLaunchKernelGGL(k_push_list<ST>, dim3((nf + blk - 1) / blk), dim3(blk), sweep_lds(c, 0),
                         c->stream, s, d, c->b.adj, nf, c->s.stride, k);
      return hipGetLastError();
    }
    int blk = c->block;
    const int nx_r = ((p.nx + 63) / 64) * 64;
    if (blk > nx_r) blk = nx_r;
    const dim3 g((unsigned)p.ny * (unsigned)p.nz), b(blk);
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_push_soa<ST, LBM_FULLWAY>), g, b, sweep_lds(c, 0), c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, c->s.stride, k);
    else
      hipLaunchKernelGGL((k_push_soa<ST, LBM_HALFWAY>), g, b, sweep_lds(c, 0), c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, c->s.stride, k);
    return hipGetLastError();
  }
  if (p.addressing == LBM_LIST) {
    const int nf = (int)c->s.n_fluid;
    if (nf == 0) return hipSuccess;
    const int blk = c->block;
    hipLaunchKernelGGL(k_sweep_list<ST>, dim3((nf + blk - 1) / blk), dim3(blk), sweep_lds(c, 0),
                       c->stream, s, d, c->b.adj, nf, c->s.stride, k);
    return hipGetLastError();
  }
  int blk = c->block;
  const int nx_r = ((p.nx + 63) / 64) * 64;
  if (blk > nx_r) blk = nx_r;
  const dim3 grid((unsigned)p.ny * (unsigned)p.nz), block(blk);
  if (p.layout == LBM_SOA) {
    const size_t lds = sweep_lds(c, 0);
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_sweep_soa<ST, LBM_FULLWAY>), grid, block, lds, c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, c->s.stride, k);
    else
      hipLaunchKernelGGL((k_sweep_soa<ST, LBM_HALFWAY>), grid, block, lds, c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, c->s.stride, k);
  } else {
    // tiles of TY rows x BX nodes: BX = min(128, nx rounded to 64), TY =
    // workgroup size / BX
    int bx = nx_r < 128 ? nx_r : 128;
    int wg = c->block < bx ? bx : c->block;
    wg = wg / bx * bx;
    const int ty = wg / bx;
    const dim3 tgrid((unsigned)((p.ny + ty - 1) / ty) * (unsigned)p.nz), tblock(wg);
    const size_t lds = sweep_lds(c, aos_lds_bytes(c, bx));
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_sweep_aos<ST, LBM_FULLWAY>), tgrid, tblock, lds, c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, bx, k);
    else
      hipLaunchKernelGGL((k_sweep_aos<ST, LBM_HALFWAY>), tgrid, tblock, lds, c->stream, s, d,
                         c->b.mask, c->b.links, p.nx, p.ny, p.nz, bx, k);
  }
  return hipGetLastError();
}

hipError_t launch_sweep(lbm_ctx* c, const void* src, void* dst) {
  switch (c->p.storage) {
    case LBM_F64: return sweep_typed<StoreF64>(c, src, dst);
    case LBM_F32_SHIFTED: return sweep_typed<StoreF32Shifted>(c, src, dst);
    case LBM_F16_SHIFTED: return sweep_typed<StoreF16Shifted>(c, src, dst);
    default: return sweep_typed<StoreF16ShiftedSR>(c, src, dst);
  }
}

}  // namespace lbm
