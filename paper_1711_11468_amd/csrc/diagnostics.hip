// diagnostics.hip - macroscopic fields, conservation diagnostics, the
// steady-state residual and the analytic verification of the force-driven
// channel flows (paper Sect. 2.1).  All reductions are FP64 and follow a
// fixed order: a grid-stride loop with a fixed grid, wavefront shuffles and
// per-wave partials per workgroup, then one workgroup that combines the
// per-workgroup partials in index order.
#include "gather.hpp"
#include "internal.hpp"

namespace lbm {

View view_of(const lbm_ctx* c);

constexpr int kReduceBlock = 256;

static unsigned reduce_grid(int64_t n) {
  int64_t g = (n + kReduceBlock - 1) / kReduceBlock;
  if (g > kMaxReduceRecords) g = kMaxReduceRecords;
  return (unsigned)(g < 1 ? 1 : g);
}


template <class ST, int LAYOUT, int ADDR, int BB, int WALLS>
__global__ void __launch_bounds__(kReduceBlock)
k_moments(const typename ST::T* __restrict__ src, View v, int64_t n_sites, int64_t n_nodes,
          double gx, double gy, double gz, double* __restrict__ rho_out,
          double* __restrict__ u_out, double* __restrict__ u_prev, int residual_mode,
          double* __restrict__ partials) {
  double acc[M_COUNT];
#pragma unroll
  for (int s = 0; s < M_COUNT; ++s) acc[s] = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sites;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = ADDR == LBM_LIST ? (int64_t)v.fluid_index[s] : s;
    double f[Q];
    if (!gather_canonical<ST, LAYOUT, ADDR, BB, WALLS>(src, v, node, f)) continue;
    double rho, ux, uy, uz, jx, jy, jz;
    moments_f64(f, gx, gy, gz, rho, ux, uy, uz, jx, jy, jz);
    acc[M_MASS] += rho;
    acc[M_PX] += jx;
    acc[M_PY] += jy;
    acc[M_PZ] += jz;
    const bool fluid = ADDR == LBM_LIST ? true : v.mask[node] == 0;
    if (!fluid) continue;
    if (!(isfinite(rho) && isfinite(jx) && isfinite(jy) && isfinite(jz))) acc[M_NONFINITE] += 1.0;
    const double u2 = ux * ux + uy * uy + uz * uz;
    acc[M_UMAX] = fmax(acc[M_UMAX], sqrt(u2));
    if (rho_out) rho_out[node] = rho;
    if (u_out) {
      u_out[node] = ux;
      u_out[n_nodes + node] = uy;
      u_out[2 * n_nodes + node] = uz;
    }
    if (residual_mode > 0) {
      if (residual_mode == 2) {
        const double dx = ux - u_prev[s], dy = uy - u_prev[n_sites + s], dz = uz - u_prev[2 * n_sites + s];
        acc[M_DU2] += dx * dx + dy * dy + dz * dz;
        acc[M_U2] += u2;
      }
      u_prev[s] = ux;
      u_prev[n_sites + s] = uy;
      u_prev[2 * n_sites + s] = uz;
    }
  }
  block_reduce<M_COUNT>(acc, 1u << M_UMAX);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < M_COUNT; ++s) partials[(int64_t)blockIdx.x * kStatSlots + s] = acc[s];
  }
}

hipError_t launch_moments(lbm_ctx* c, const void* src, double* rho_out, double* u_out,
                          int residual_mode, double* partials, int64_t* n_blocks_out) {
  const unsigned grid = reduce_grid(c->s.n_sites);
  *n_blocks_out = grid;
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    return dispatch(c->p, [&](auto st, auto lay, auto addr, auto bb) -> hipError_t {
      using ST = decltype(st);
      hipLaunchKernelGGL((k_moments<ST, decltype(lay)::value, decltype(addr)::value,
                                    decltype(bb)::value, decltype(walls)::value>),
                         dim3(grid), dim3(kReduceBlock), 0, c->stream, (const typename ST::T*)src,
                         view_of(c), c->s.n_sites, c->s.n_nodes, c->p.g[0], c->p.g[1], c->p.g[2],
                         rho_out, u_out, c->b.u_prev, residual_mode, partials);
      return hipGetLastError();
    });
  });
}

// ---- verification ---------------------------------------------------------

struct VerifyArgs {
  int kind;
  double gx, nu;
  const double* ref;  // [3][N] for LBM_VERIFY_REFERENCE
  int64_t n_nodes;
};

// Steady u_x of the slab: g/(2 nu) ((H/2)^2 - zeta^2), H = nz - 2.
__device__ double slab_ux(int z, int nz, double gx, double nu) {
  const double h = 0.5 * (nz - 2);
  const double zeta = z - 0.5 * (nz - 1);
  return gx / (2.0 * nu) * (h * h - zeta * zeta);
}

// Steady u_x of the duct: series over odd n of
// 16 a^2 g / (nu pi^3) (-1)^((n-1)/2) n^-3 [1 - cosh(k z)/cosh(k b)] cos(k y),
// k = n pi / (2a), centred coordinates, half-widths a = (ny-2)/2, b = (nz-2)/2.
__device__ double duct_ux(int y, int z, int ny, int nz, double gx, double nu) {
  const double a = 0.5 * (ny - 2), b = 0.5 * (nz - 2);
  const double Y = y - 0.5 * (ny - 1), Z = fabs(z - 0.5 * (nz - 1));
  double sum = 0.0;
  for (int n = 1; n <= 401; n += 2) {
    const double k = n * M_PI / (2.0 * a);
    const double ratio = (exp(k * (Z - b)) + exp(-k * (Z + b))) / (1.0 + exp(-2.0 * k * b));
    const double sign = ((n - 1) / 2) % 2 == 0 ? 1.0 : -1.0;
    sum += sign / ((double)n * n * n) * (1.0 - ratio) * cos(k * Y);
  }
  return 16.0 * a * a * gx / (nu * M_PI * M_PI * M_PI) * sum;
}

template <class ST, int LAYOUT, int ADDR, int BB, int WALLS>
__global__ void __launch_bounds__(kReduceBlock)
k_verify(const typename ST::T* __restrict__ src, View v, int64_t n_sites, double gx, double gy,
         double gz, VerifyArgs a, double* __restrict__ partials) {
  double acc[V_COUNT];
#pragma unroll
  for (int s = 0; s < V_COUNT; ++s) acc[s] = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sites;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = ADDR == LBM_LIST ? (int64_t)v.fluid_index[s] : s;
    if (ADDR == LBM_DIRECT && v.mask[node] != 0) continue;
    double f[Q];
    if (!gather_canonical<ST, LAYOUT, ADDR, BB, WALLS>(src, v, node, f)) continue;
    double rho, ux, uy, uz, jx, jy, jz;
    moments_f64(f, gx, gy, gz, rho, ux, uy, uz, jx, jy, jz);
    int x, y, z;
    node_xyz(v, node, x, y, z);
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (a.kind == LBM_VERIFY_SLAB) {
      rx = slab_ux(z, v.nz, a.gx, a.nu);
    } else if (a.kind == LBM_VERIFY_DUCT) {
      rx = duct_ux(y, z, v.ny, v.nz, a.gx, a.nu);
    } else {
      rx = a.ref[node];
      ry = a.ref[a.n_nodes + node];
      rz = a.ref[2 * a.n_nodes + node];
    }
    const double ex = ux - rx, ey = uy - ry, ez = uz - rz;
    acc[V_MAXABS] = fmax(acc[V_MAXABS], fmax(fabs(ex), fmax(fabs(ey), fabs(ez))));
    acc[V_ERR2] += ex * ex + ey * ey + ez * ez;
    acc[V_REF2] += rx * rx + ry * ry + rz * rz;
    acc[V_REFMAX] = fmax(acc[V_REFMAX], fmax(fabs(rx), fmax(fabs(ry), fabs(rz))));
    acc[V_COUNT_N] += 1.0;
  }
  block_reduce<V_COUNT>(acc, (1u << V_MAXABS) | (1u << V_REFMAX));
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < V_COUNT; ++s) partials[(int64_t)blockIdx.x * kStatSlots + s] = acc[s];
  }
}

hipError_t launch_verify(lbm_ctx* c, const void* src, int kind, const double* ref_dev,
                         double* partials, int64_t* n_blocks_out) {
  const unsigned grid = reduce_grid(c->s.n_sites);
  *n_blocks_out = grid;
  VerifyArgs a;
  a.kind = kind;
  a.gx = c->p.g[0];
  a.nu = (c->p.tau_plus - 0.5) / 3.0;
  a.ref = ref_dev;
  a.n_nodes = c->s.n_nodes;
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    return dispatch(c->p, [&](auto st, auto lay, auto addr, auto bb) -> hipError_t {
      using ST = decltype(st);
      hipLaunchKernelGGL((k_verify<ST, decltype(lay)::value, decltype(addr)::value,
                                   decltype(bb)::value, decltype(walls)::value>),
                         dim3(grid), dim3(kReduceBlock), 0, c->stream, (const typename ST::T*)src,
                         view_of(c), c->s.n_sites, c->p.g[0], c->p.g[1], c->p.g[2], a, partials);
      return hipGetLastError();
    });
  });
}

// ---- final fixed-order reduction -----------------------------------------
// Workgroup b combines records [b*chunk, min(n, (b+1)*chunk)) into record b
// of `out`: strided per-thread sums, then the block reduction.
__global__ void __launch_bounds__(kReduceBlock)
k_reduce_records(const double* __restrict__ partials, int64_t n, int64_t chunk, int n_slots,
                 uint32_t max_mask, double* __restrict__ out) {
  double acc[kStatSlots];
#pragma unroll
  for (int s = 0; s < kStatSlots; ++s) acc[s] = 0.0;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  for (int64_t b = lo + threadIdx.x; b < hi; b += blockDim.x) {
#pragma unroll
    for (int s = 0; s < kStatSlots; ++s) {
      if (s >= n_slots) break;
      const double p = partials[b * kStatSlots + s];
      acc[s] = ((max_mask >> s) & 1u) ? fmax(acc[s], p) : acc[s] + p;
    }
  }
  block_reduce<kStatSlots>(acc, max_mask);
  if (threadIdx.x == 0) {
    for (int s = 0; s < n_slots; ++s) out[(int64_t)blockIdx.x * kStatSlots + s] = acc[s];
  }
}

hipError_t launch_final_reduce(lbm_ctx* c, double* partials, int64_t n_blocks, int n_slots,
                               uint32_t max_mask, double* out_dev) {
  hipLaunchKernelGGL(k_reduce_records, dim3(1), dim3(kReduceBlock), 0, c->stream, partials,
                     n_blocks, n_blocks, n_slots, max_mask, out_dev);
  return hipGetLastError();
}

hipError_t launch_reduce_records(lbm_ctx* c, double* partials, int64_t n, int n_slots,
                                 uint32_t max_mask, double* stage, double* out_dev) {
  if (n <= kMaxReduceRecords) return launch_final_reduce(c, partials, n, n_slots, max_mask, out_dev);
  const int64_t chunk = (n + kMaxReduceRecords - 1) / kMaxReduceRecords;
  const int64_t groups = (n + chunk - 1) / chunk;  // <= kMaxReduceRecords
  hipLaunchKernelGGL(k_reduce_records, dim3((unsigned)groups), dim3(kReduceBlock), 0, c->stream,
                     partials, n, chunk, n_slots, max_mask, stage);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_final_reduce(c, stage, groups, n_slots, max_mask, out_dev);
}

}  // namespace lbm
