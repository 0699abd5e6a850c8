// sweep_aos.hip - the one-step pull update for the AoS layout (Sect. 3,
// "One Step Kernels"; node records of 19 values, compared with SoA in
// Sect. 4.2).  Records are contiguous, so a wavefront reading one direction
// of 64 nodes would touch 64 records; the kernel moves whole records between
// HBM and LDS with contiguous loads and stores instead.
#include "launch.hpp"

namespace lbm {

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

size_t aos_lds_bytes(const lbm_ctx* c, int bx) {
  const int es = c->p.storage == LBM_F64 ? 8 : (c->p.storage == LBM_F32_SHIFTED ? 4 : 2);  // F16: 2
  return (size_t)(bx + 2) * Q * es;
}

hipError_t launch_pull_aos(lbm_ctx* c, const void* src, void* dst) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    const lbm_params& p = c->p;
    const auto k = make_collide<typename ST::R>(p, c->step);
    const T* s = (const T*)src;
    T* d = (T*)dst;
    // tiles of TY rows x BX nodes: BX = min(128, nx rounded to 64), TY =
    // workgroup size / BX
    const int nx_r = ((p.nx + 63) / 64) * 64;
    const int bx = nx_r < 128 ? nx_r : 128;
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
    return hipGetLastError();
  });
}

}  // namespace lbm
