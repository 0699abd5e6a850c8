// state_io.hip - set-up and state transfer kernels: rest-state fill,
// adjacency-list construction (paper Sect. 3 "Lattice Representation",
// Sect. 3.2), canonical export/import and equilibrium initialisation.
#include "gather.hpp"
#include "internal.hpp"

namespace lbm {

static View make_view(const lbm_ctx* c) {
  View v;
  v.nx = c->p.nx;
  v.ny = c->p.ny;
  v.nz = c->p.nz;
  v.stride = c->s.stride;
  v.adj_stride = c->adj_stride;
  v.mask = c->b.mask;
  v.adj = c->b.adj;
  v.node_map = c->b.node_map;
  v.fluid_index = c->b.fluid_index;
  v.periodic = c->p.periodic;
  // push buffers hold the canonical state in place, like an AA lattice after
  // an even number of updates
  v.aa = c->p.propagation == LBM_AA ? (c->aa_odd ? 2 : 1) : (c->p.propagation == LBM_OS_PUSH ? 1 : 0);
  if (c->p.storage == LBM_F16_SHIFTED || c->p.storage == LBM_F16_SHIFTED_SR) {
    v.scale = ldexpf(1.0f, c->p.f16_scale_log2);
    v.inv_scale = ldexpf(1.0f, -c->p.f16_scale_log2);
  } else {
    v.scale = v.inv_scale = 1.0f;
  }
  return v;
}

View view_of(const lbm_ctx* c) { return make_view(c); }

static inline unsigned grid_for(int64_t n, int blk) {
  int64_t g = (n + blk - 1) / blk;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---- rest state -----------------------------------------------------------
template <class ST, int LAYOUT>
__global__ void k_fill_rest(typename ST::T* __restrict__ buf, int64_t total, int64_t stride) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int i = LAYOUT == LBM_SOA ? (int)(e / stride) : (int)(e % Q);
  buf[e] = rest_value<ST>(i);
}

hipError_t launch_fill_rest(lbm_ctx* c, void* buf) {
  return dispatch(c->p, [&](auto st, auto lay, auto, auto) -> hipError_t {
    using ST = decltype(st);
    constexpr int L = decltype(lay)::value;
    const int64_t total = c->s.pdf_bytes / (int64_t)sizeof(typename ST::T);
    hipLaunchKernelGGL((k_fill_rest<ST, L>), dim3(grid_for(total, 256)), dim3(256), 0, c->stream,
                       (typename ST::T*)buf, total, c->s.stride);
    return hipGetLastError();
  });
}

// ---- adjacency list -------------------------------------------------------
// adj[(i-1)*stride + m] = slot a pull of direction i reads for list node m:
// the neighbour's slot i*stride + map(x - c_i), or the node's own opposite
// slot opp(i)*stride + m when the neighbour is solid or beyond a wall face
// (half-way bounce-back).
// For the AA pattern the neighbour kernel reads the reversed slots instead:
// opp(i)*stride + map(x - c_i), or i*stride + m at a solid neighbour.
// Slots are layout-dependent: direction-major (SOA) or record-major (AOS).
template <int WALLS>
__device__ __forceinline__ void adjacency_of(const View& v, int m, int aa, bool aos, int32_t* out,
                                             int64_t out_stride) {
  int x, y, z;
  node_xyz(v, v.fluid_index[m], x, y, z);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int sx = x - Vel::cx[i], sy = y - Vel::cy[i], sz = z - Vel::cz[i];
    const int tw = v.node_map[wrap_node(v, sx, sy, sz)];
    const int t = beyond_wall<WALLS>(v, sx, sy, sz) ? -1 : tw;
    const int dn = aa ? Vel::opp[i] : i;     // direction slot at the neighbour
    const int ds = aa ? i : Vel::opp[i];     // direction slot at the node itself
    const int64_t node = t >= 0 ? t : m;
    const int d = t >= 0 ? dn : ds;
    const int64_t s = aos ? node * Q + d : (int64_t)d * v.stride + node;
    out[(int64_t)(i - 1) * out_stride] = (int32_t)s;
  }
}

template <int WALLS>
__global__ void k_build_adjacency(View v, int nf, int aa, int aos, int32_t* __restrict__ adj) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  adjacency_of<WALLS>(v, m, aa, aos != 0, adj + m, v.adj_stride);
}

hipError_t launch_build_adjacency(lbm_ctx* c) {
  const int nf = (int)c->s.n_fluid;
  if (nf == 0) return hipSuccess;
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    hipLaunchKernelGGL(k_build_adjacency<decltype(walls)::value>, dim3(grid_for(nf, 256)), dim3(256), 0,
                       c->stream, make_view(c), nf, c->p.propagation == LBM_OS ? 0 : 1,
                       c->p.layout == LBM_AOS ? 1 : 0, c->b.adj);
    return hipGetLastError();
  });
}

// Run-length list: the same 18 entries, once per run, for the run's first
// node; node m of run r then uses entry + (m - run_start[r]).
template <int WALLS>
__global__ void k_build_run_adj(View v, const int32_t* __restrict__ run_start, int64_t n_runs,
                                int aa, int64_t run_stride, int32_t* __restrict__ run_adj) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_runs) return;
  adjacency_of<WALLS>(v, run_start[r], aa, false, run_adj + r, run_stride);
}

hipError_t launch_build_run_adj(lbm_ctx* c) {
  if (c->n_runs == 0) return hipSuccess;
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    hipLaunchKernelGGL(k_build_run_adj<decltype(walls)::value>, dim3(grid_for(c->n_runs, 256)), dim3(256),
                       0, c->stream, make_view(c), c->run_start, c->n_runs,
                       c->p.propagation == LBM_OS ? 0 : 1, c->run_stride, c->run_adj);
    return hipGetLastError();
  });
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

// The same words when some axis does not wrap: a source beyond a wall face
// also sets its bit.  The sweeps take the node's own slot wherever the bit
// is set, so such a face reflects like a solid neighbour.
__global__ void k_build_links_walls(const uint8_t* __restrict__ mask, uint32_t* __restrict__ links,
                                    int nx, int ny, int nz, uint32_t periodic) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny * nz;
  if (n >= N) return;
  const int x = (int)(n % nx);
  const int64_t r = n / nx;
  const int y = (int)(r % ny), z = (int)(r / ny);
  // faces of the node that are walls: bit 0/1 low/high x, 2/3 y, 4/5 z
  uint32_t face = 0;
  if (!(periodic & 1u)) face |= (x == 0 ? 1u : 0u) | (x == nx - 1 ? 2u : 0u);
  if (!(periodic & 2u)) face |= (y == 0 ? 4u : 0u) | (y == ny - 1 ? 8u : 0u);
  if (!(periodic & 4u)) face |= (z == 0 ? 16u : 0u) | (z == nz - 1 ? 32u : 0u);
  uint32_t w = mask[n] != 0 ? 1u : 0u;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    // x - c_i leaves the box through the low face of an axis where c > 0
    const uint32_t through = (Vel::cx[i] > 0 ? 1u : Vel::cx[i] < 0 ? 2u : 0u) |
                             (Vel::cy[i] > 0 ? 4u : Vel::cy[i] < 0 ? 8u : 0u) |
                             (Vel::cz[i] > 0 ? 16u : Vel::cz[i] < 0 ? 32u : 0u);
    const int sx = wrap_sub(x, Vel::cx[i], nx);
    const int sy = wrap_sub(y, Vel::cy[i], ny);
    const int sz = wrap_sub(z, Vel::cz[i], nz);
    const bool solid = (mask[sx + (int64_t)nx * (sy + (int64_t)ny * sz)] != 0) | ((face & through) != 0);
    if (solid) w |= 1u << i;
  }
  links[n] = w;
}

hipError_t launch_build_links(lbm_ctx* c) {
  const int64_t N = c->s.n_nodes;
  if (c->p.periodic == 7u)
    hipLaunchKernelGGL(k_build_links, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                       c->b.mask, c->b.links, c->p.nx, c->p.ny, c->p.nz);
  else
    hipLaunchKernelGGL(k_build_links_walls, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                       c->b.mask, c->b.links, c->p.nx, c->p.ny, c->p.nz, c->p.periodic);
  return hipGetLastError();
}

// ---- export ---------------------------------------------------------------
template <class ST, int LAYOUT, int ADDR, int BB, int WALLS>
__global__ void k_export(const typename ST::T* __restrict__ src, View v,
                         const int64_t* __restrict__ ids, int64_t count, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t node = ids[k];
  double f[Q];
  const bool has = gather_canonical<ST, LAYOUT, ADDR, BB, WALLS>(src, v, node, f);
#pragma unroll
  for (int i = 0; i < Q; ++i) out[k * Q + i] = has ? f[i] : 0.0;
}

hipError_t launch_export(lbm_ctx* c, const void* src, const int64_t* ids_dev, int64_t count,
                         double* out_dev) {
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    return dispatch(c->p, [&](auto st, auto lay, auto addr, auto bb) -> hipError_t {
      using ST = decltype(st);
      hipLaunchKernelGGL((k_export<ST, decltype(lay)::value, decltype(addr)::value,
                                   decltype(bb)::value, decltype(walls)::value>),
                         dim3(grid_for(count, 256)), dim3(256), 0, c->stream,
                         (const typename ST::T*)src, make_view(c), ids_dev, count, out_dev);
      return hipGetLastError();
    });
  });
}

// ---- import and equilibrium initialisation --------------------------------
// Both write the pull buffer Q whose streaming image is a given canonical
// state P: Q_i(y) = P_i(y + c_i), or, under half-way bounce-back when
// y + c_i is solid or beyond a wall face, Q_i(y) = P_opp(i)(y) (each slot has
// exactly one image).
// Import reads P from a device array; init evaluates P = e(rho, u) (solids
// under full-way bounce-back hold the rest state).
struct CanonFromArray {
  const double* P;
  __device__ double operator()(int64_t node, int i, const View&) const { return P[node * Q + i]; }
};

// The equilibrium is taken at u - g/(2 rho): the macroscopic velocity is
// u = (sum c f + g/2)/rho, so this makes the state report exactly the
// requested velocity (an equilibrium at u itself would carry an extra
// momentum g/2 per node, which decays only slowly).
struct CanonFromFields {
  const double* rho;  // N or null (1)
  const double* u;    // [3][N] or null (0)
  int64_t n_nodes;
  int fullway;
  double gx, gy, gz;
  __device__ double operator()(int64_t node, int i, const View& v) const {
    if (fullway && v.mask[node] != 0) return weight(i);
    const double r = rho ? rho[node] : 1.0;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (u) {
      ux = u[node];
      uy = u[n_nodes + node];
      uz = u[2 * n_nodes + node];
    }
    const double h = 0.5 / r;
    return weight(i) + eq_shifted(i, r, ux - h * gx, uy - h * gy, uz - h * gz);
  }
};

template <class ST, int LAYOUT, int ADDR, int BB, int WALLS, class SRC>
__global__ void k_scatter_canonical(SRC P, View v, int64_t n_sites, typename ST::T* __restrict__ dst) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sites) return;
  const int64_t node = ADDR == LBM_LIST ? (int64_t)v.fluid_index[s] : s;
  const int64_t site = s;  // slot index: node (direct) or list position
  if (ADDR == LBM_DIRECT && BB == LBM_HALFWAY && v.mask[node] != 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[vslot<LAYOUT>(site, i, v.stride)] = rest_value<ST>(i);
    return;
  }
  if (v.aa) {
    // AA lattice: the canonical state is stored in place (even phase)
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[vslot<LAYOUT>(site, i, v.stride)] = from_f64<ST>(P(node, i, v), i, v);
    return;
  }
  int x, y, z;
  node_xyz(v, node, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int tx = x + Vel::cx[i], ty = y + Vel::cy[i], tz = z + Vel::cz[i];
    const int64_t tn = wrap_node(v, tx, ty, tz);
    double val;
    bool solid = false;
    if (BB == LBM_HALFWAY && i != 0) solid = (v.mask[tn] != 0) | beyond_wall<WALLS>(v, tx, ty, tz);
    if (solid) val = P(node, Vel::opp[i], v);
    else val = P(tn, i, v);
    dst[vslot<LAYOUT>(site, i, v.stride)] = from_f64<ST>(val, i, v);
  }
}

hipError_t launch_import(lbm_ctx* c, const double* canon_dev, void* dst) {
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    return dispatch(c->p, [&](auto st, auto lay, auto addr, auto bb) -> hipError_t {
      using ST = decltype(st);
      const int64_t n = c->s.n_sites;
      hipLaunchKernelGGL((k_scatter_canonical<ST, decltype(lay)::value, decltype(addr)::value,
                                              decltype(bb)::value, decltype(walls)::value,
                                              CanonFromArray>),
                         dim3(grid_for(n, 256)), dim3(256), 0, c->stream, CanonFromArray{canon_dev},
                         make_view(c), n, (typename ST::T*)dst);
      return hipGetLastError();
    });
  });
}

hipError_t launch_init_fields(lbm_ctx* c, const double* rho_dev, const double* u_dev, void* dst) {
  return with_walls(c->p, [&](auto walls) -> hipError_t {
    return dispatch(c->p, [&](auto st, auto lay, auto addr, auto bb) -> hipError_t {
      using ST = decltype(st);
      const int64_t n = c->s.n_sites;
      CanonFromFields P{rho_dev, u_dev, c->s.n_nodes, c->p.bounce == LBM_FULLWAY ? 1 : 0,
                        c->p.g[0], c->p.g[1], c->p.g[2]};
      hipLaunchKernelGGL((k_scatter_canonical<ST, decltype(lay)::value, decltype(addr)::value,
                                              decltype(bb)::value, decltype(walls)::value,
                                              CanonFromFields>),
                         dim3(grid_for(n, 256)), dim3(256), 0, c->stream, P, make_view(c), n,
                         (typename ST::T*)dst);
      return hipGetLastError();
    });
  });
}

}  // namespace lbm
