// sweep_aos.hip - sweeps over the AoS layout with direct addressing: the
// one-step pull and push (Sect. 3, "One Step Kernels") and the neighbour
// step of the AA pattern (Sect. 3, "AA Pattern Kernels"); node records of
// 19 values, compared with SoA in Sect. 4.2.  Records are contiguous, so a
// wavefront reading one direction of 64 nodes would touch 64 records; the
// kernels instead read each source layer once, as whole records, and
// redistribute it through LDS.
//
// A workgroup owns a column of TY x BX nodes (rows y0.., nodes x0..) and
// marches it through the layers zb .. ze-1 of its z chunk.  Each source
// layer is read over the column and its one-node halo with contiguous
// loads, and its populations are sorted by the layer they stream to:
//   c_z = -1 (5 directions): needed by the output layer below, right away;
//   c_z =  0 (9 directions): needed by the output layer itself, next step;
//   c_z = +1 (5 directions): needed by the output layer above, in two steps.
// LDS holds one region per class ("down", "level" and two alternating "up"
// regions), each storing its populations position by position over the
// halo'd column.  The next source layer is loaded into registers while the
// current layer is collided and stored.  A thread's staged elements are
// enumerated class by class, element e of a class being direction e % n_c
// at halo position e / n_c, so a register slot's class is known at compile
// time and its LDS slot is the thread index plus a constant.
//
// Results are stored straight from registers: each of the 19 store
// instructions of a wavefront covers one slot of 64 records, and together
// they write 64 whole contiguous records, which L2 assembles into full
// lines (on MI355X this beat staging the records through LDS, and
// non-temporal stores, which bypass that assembly, were 4.6x slower).
// Columns of 32 x 8 nodes: 1.33x the algorithmic reads for the halo, 68 KB
// of LDS in FP64, two workgroups per compute unit.  The push and the AA
// neighbour step (below) run the same march with one thread per halo'd
// position.
#include "diag.hpp"
#include "launch.hpp"

namespace lbm {

// Population classes of the z march (c = c_z + 1) and the column shape.
namespace zmarch {

// Direction d of class c (c = c_z + 1), in velocity order.
__host__ __device__ constexpr int dir_of(int c, int d) {
  for (int i = 0; i < Q; ++i)
    if (Vel::cz[i] + 1 == c && d-- == 0) return i;
  return -1;
}
__host__ __device__ constexpr int count_of(int c) {
  int n = 0;
  for (int i = 0; i < Q; ++i) n += Vel::cz[i] + 1 == c ? 1 : 0;
  return n;
}
// The directions of class c packed 5 bits each (for a runtime d).
__host__ __device__ constexpr uint64_t packed_dirs(int c) {
  uint64_t v = 0;
  for (int d = 0; d < count_of(c); ++d) v |= (uint64_t)dir_of(c, d) << (5 * d);
  return v;
}
__host__ __device__ constexpr int idx_of(int i) {
  int n = 0;
  for (int j = 0; j < i; ++j) n += Vel::cz[j] == Vel::cz[i] ? 1 : 0;
  return n;
}

template <int BX, int TY>
struct Shape {
  static constexpr int NT = BX * TY, HX = BX + 2, HY = TY + 2, P = HX * HY;
  // register slots per class (the last one padded) and LDS regions
  static constexpr int K0 = (count_of(0) * P + NT - 1) / NT;
  static constexpr int K1 = (count_of(1) * P + NT - 1) / NT;
  static constexpr int K2 = (count_of(2) * P + NT - 1) / NT;
  static constexpr int KE = K0 + K1 + K2;
  static constexpr int D0 = 0, D1 = K0 * NT, D2 = (K0 + K1) * NT;  // up set p at D2 + p*K2*NT
  static constexpr int STAGE = (K0 + K1 + 2 * K2) * NT;
};

template <int BX, int TY, class T>
constexpr size_t lds_bytes() {
  return (size_t)Shape<BX, TY>::STAGE * sizeof(T);
}

}  // namespace zmarch

// The pull march; with DIAG the diagnostics of the state it reads (the
// gathered populations, after the half-way substitution) are accumulated
// per thread and reduced into one partial record per column.
template <class ST, int BB, int BX, int TY, bool DIAG>
__device__ __forceinline__ void aos_pull_march(const typename ST::T* __restrict__ src,
                                               typename ST::T* __restrict__ dst,
                                               const uint8_t* __restrict__ mask,
                                               const uint32_t* __restrict__ links, int nx, int ny,
                                               int nz, int zc, int n_tiles,
                                               const Collide<typename ST::R>& k,
                                               const DiagArgs& dg) {
  using T = typename ST::T;
  using R = typename ST::R;
  using S = zmarch::Shape<BX, TY>;
  constexpr int NT = S::NT, HX = S::HX, P = S::P, K0 = S::K0, K1 = S::K1, K2 = S::K2, KE = S::KE;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);

  // workgroup b runs on XCD b % 8: give each XCD a contiguous range of
  // columns so that neighbouring columns share their halo lines in one L2
  const int per = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= n_tiles) return;
  const int tiles_x = (nx + BX - 1) / BX, tiles_y = (ny + TY - 1) / TY;
  const int tx_t = tile % tiles_x;
  const int ty_t = (tile / tiles_x) % tiles_y;
  const int zb = (tile / tiles_x / tiles_y) * zc;
  const int ze = zb + zc < nz ? zb + zc : nz;
  const int x0 = tx_t * BX, y0 = ty_t * TY;
  const int seg = nx - x0 < BX ? nx - x0 : BX;
  const int segy = ny - y0 < TY ? ny - y0 : TY;
  const int t = threadIdx.x, tx = t % BX, ty = t / BX;
  const bool active = tx < seg && ty < segy;
  const int64_t layer = (int64_t)nx * ny * Q;

  // goff: offset inside a layer of staged element j (below 2^31: the plan
  // rejects larger layers for this form).  Positions past the
  // column's real extent repeat the last real one; the padding elements of
  // a class repeat its last element (their LDS slots are never read).
  uint32_t goff[KE];
  auto setup = [&](int j, int c, int e_raw) {
    const int nd = zmarch::count_of(c), n_c = nd * P;
    const int e = e_raw < n_c ? e_raw : n_c - 1;
    const int pp = e / nd, d = e - pp * nd;
    const int hy = pp / HX, hx = pp - hy * HX;
    int xs = x0 - 1 + (hx < seg + 1 ? hx : seg + 1);
    int ys = y0 - 1 + (hy < segy + 1 ? hy : segy + 1);
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
    const int i = (int)((zmarch::packed_dirs(c) >> (5 * d)) & 31);
    goff[j] = (uint32_t)((ys * nx + xs) * Q + i);
  };
#pragma unroll
  for (int j = 0; j < K0; ++j) setup(j, 0, t + j * NT);
#pragma unroll
  for (int j = 0; j < K1; ++j) setup(K0 + j, 1, t + j * NT);
#pragma unroll
  for (int j = 0; j < K2; ++j) setup(K0 + K1 + j, 2, t + j * NT);
  auto wrapz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  T r[KE];
  auto load_layer = [&](int z) {
    const T* base = src + (int64_t)wrapz(z) * layer;
#pragma unroll
    for (int j = 0; j < KE; ++j) r[j] = base[goff[j]];
  };
  T* const Lt = L + t;
  auto put_up = [&](int par) {
#pragma unroll
    for (int j = 0; j < K2; ++j) Lt[S::D2 + par * K2 * NT + j * NT] = r[K0 + K1 + j];
  };
  auto put_level = [&]() {
#pragma unroll
    for (int j = 0; j < K1; ++j) Lt[S::D1 + j * NT] = r[K0 + j];
  };

  double acc[M_COUNT];
#pragma unroll
  for (int q = 0; q < M_COUNT; ++q) acc[q] = 0.0;
  const int64_t n_all = (int64_t)nx * ny * nz;

  // prologue: up populations of layer zb-1 (set 0), level and up of zb (set 1)
  load_layer(zb - 1);
  put_up(0);
  load_layer(zb);
  put_level();
  put_up(1);
  load_layer(zb + 1);
  const int me = (ty + 1) * HX + tx + 1;
  for (int z = zb; z < ze; ++z) {
    const int s = z - zb;
    const int64_t n = ((int64_t)z * ny + y0 + ty) * nx + x0 + tx;
    uint32_t lk = 0;
    bool solid = false;
    if (active) {
      if (BB == LBM_HALFWAY) {
        lk = links[n];
        solid = (lk & 1u) != 0;
      } else {
        solid = mask[n] != 0;
      }
    }
#pragma unroll
    for (int j = 0; j < K0; ++j) Lt[S::D0 + j * NT] = r[j];  // down of layer z+1
    __syncthreads();
    R f[Q];
    if (active) {
      const T* up = L + S::D2 + (s & 1) * K2 * NT;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int c = Vel::cz[i] + 1, nd = zmarch::count_of(c);
        const int pos = me - Vel::cy[i] * HX - Vel::cx[i];
        const T* reg = c == 0 ? L + S::D0 : (c == 1 ? L + S::D1 : up);
        f[i] = ST::load(reg[pos * nd + zmarch::idx_of(i)], k.inv_scale);
      }
    }
    __syncthreads();
    // layer z+1: level (used at step s+1), up into the set that held layer
    // z-1 (used at step s+2); then start loading layer z+2
    put_level();
    put_up(s & 1);
    if (z + 1 < ze) load_layer(z + 2);
    if (active) {
      if (BB == LBM_HALFWAY) {
        if (!solid && (lk >> 1)) {
#pragma unroll
          for (int i = 1; i < Q; ++i)
            if ((lk >> i) & 1u) f[i] = ST::load(src[n * Q + Vel::opp[i]], k.inv_scale);
        }
      }
      // half-way solids hold no state; full-way solids hold populations in transit
      if constexpr (DIAG) {
        if (!(BB == LBM_HALFWAY && solid)) diag_node<ST>(f, !solid, n, n_all, dg, acc);
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
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = ST::kShifted ? R(0) : R(weight(i));
      }
      SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
      for (int i = 0; i < Q; ++i) dst[n * Q + i] = ST::store(f[i], k.scale, rs.next());
    }
  }
  if constexpr (DIAG) {
    block_reduce<M_COUNT>(acc, 1u << M_UMAX);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < M_COUNT; ++q) dg.partials[(int64_t)tile * kStatSlots + q] = acc[q];
    }
  }
}

template <class ST, int BB, int BX, int TY>
__global__ void __launch_bounds__(BX * TY)
k_sweep_aos(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
            const uint8_t* __restrict__ mask, const uint32_t* __restrict__ links, int nx, int ny,
            int nz, int zc, int n_tiles, Collide<typename ST::R> k) {
  aos_pull_march<ST, BB, BX, TY, false>(src, dst, mask, links, nx, ny, nz, zc, n_tiles, k,
                                        DiagArgs{});
}

template <class ST, int BB, int BX, int TY>
__global__ void __launch_bounds__(BX * TY)
k_sweep_aos_diag(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
                 const uint8_t* __restrict__ mask, const uint32_t* __restrict__ links, int nx,
                 int ny, int nz, int zc, int n_tiles, Collide<typename ST::R> k, DiagArgs d) {
  aos_pull_march<ST, BB, BX, TY, true>(src, dst, mask, links, nx, ny, nz, zc, n_tiles, k, d);
}

// ---- one-step push over AoS records ---------------------------------------
// The push writes f*_i(x) into slot i of x + c_i (or, under half-way
// bounce-back towards a solid node, into slot opp(i) of x).  Seen from the
// destination y, slot i holds f*_i(y - c_i), so a column can produce whole
// destination records if it also collides the nodes of its one-node halo:
// the same z march as the pull, with the collision done on the source side
// before the populations are sorted into the class regions.  One thread per
// halo'd position: it loads that node's record (the 19 loads of a wavefront
// cover consecutive whole records), collides it (rounding to the storage
// format at the source, as the scattering kernel does), and the threads of
// interior positions gather and store their destination records.  Under
// half-way bounce-back a destination whose source y - c_i is solid takes
// its own f*_opp(i), kept in registers from the step that collided it.
template <int BX, int TY>
struct PushShape {
  static constexpr int HX = BX + 2, HY = TY + 2, P = HX * HY;
  static constexpr int NT = (P + 63) / 64 * 64;
  static constexpr int R0 = 0, R1 = 5 * P, R2 = 14 * P;  // down, level, up set 0 (set 1 at R2 + 5P)
  static constexpr int STAGE = 24 * P;
};

template <class ST, int BB, int BX, int TY>
__global__ void __launch_bounds__((PushShape<BX, TY>::NT))
k_push_aos(const typename ST::T* __restrict__ src, typename ST::T* __restrict__ dst,
           const uint8_t* __restrict__ mask, const uint32_t* __restrict__ links, int nx, int ny,
           int nz, int zc, int n_tiles, Collide<typename ST::R> k) {
  using T = typename ST::T;
  using R = typename ST::R;
  using S = PushShape<BX, TY>;
  constexpr int HX = S::HX, P = S::P;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);

  const int per = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= n_tiles) return;
  const int tiles_x = (nx + BX - 1) / BX, tiles_y = (ny + TY - 1) / TY;
  const int tx_t = tile % tiles_x;
  const int ty_t = (tile / tiles_x) % tiles_y;
  const int zb = (tile / tiles_x / tiles_y) * zc;
  const int ze = zb + zc < nz ? zb + zc : nz;
  const int x0 = tx_t * BX, y0 = ty_t * TY;
  const int seg = nx - x0 < BX ? nx - x0 : BX;
  const int segy = ny - y0 < TY ? ny - y0 : TY;
  const int t = threadIdx.x;
  const bool live = t < P;
  const int pt = live ? t : P - 1;
  const int hy = pt / HX, hx = pt - hy * HX;
  const bool interior = live && hx >= 1 && hx <= seg && hy >= 1 && hy <= segy;
  int xs = x0 - 1 + (hx < seg + 1 ? hx : seg + 1);
  int ys = y0 - 1 + (hy < segy + 1 ? hy : segy + 1);
  xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
  ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
  const int64_t plane_nodes = (int64_t)nx * ny;
  const int64_t col = (int64_t)ys * nx + xs;
  auto wrapz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };

  T r[Q];
  uint32_t geo_next = 0;  // link word (half-way) or flag byte of the loaded node
  auto load = [&](int z) {
    const int64_t node = wrapz(z) * plane_nodes + col;
#pragma unroll
    for (int i = 0; i < Q; ++i) r[i] = src[node * Q + i];
    geo_next = BB == LBM_HALFWAY ? links[node] : (uint32_t)mask[node];
  };
  T g[Q];
  auto collide_src = [&](int z) {
    const bool solid = BB == LBM_HALFWAY ? (geo_next & 1u) != 0 : geo_next != 0;
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = ST::load(r[i], k.inv_scale);
    if (!solid) {
      trt_collide<R, ST::kShifted>(f, k);
    } else if (BB == LBM_FULLWAY) {
      R h[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) h[i] = f[Vel::opp[i]];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = h[i];
    }
    SrStream rs((uint32_t)(wrapz(z) * plane_nodes + col), k.step, ST::kStochastic);
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = ST::store(f[i], k.scale, rs.next());
  };
  // class c of g into its region (up: set par) at this thread's position
  auto put = [&](int c, int par) {
    if (!live) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (Vel::cz[i] + 1 != c) continue;
      const int nd = zmarch::count_of(c);
      const int base = c == 0 ? S::R0 : (c == 1 ? S::R1 : S::R2 + par * 5 * P);
      L[base + t * nd + zmarch::idx_of(i)] = g[i];
    }
  };

  T gprev[BB == LBM_HALFWAY ? Q : 1];
  uint32_t geo_cur = 0;
  // Step s collides source layer z+1 = zb+s+1; steps -2 and -1 only fill
  // the regions (up of zb-1, level and up of zb), so that every collision
  // runs through the same code.
  load(zb - 1);
  for (int s = -2; s < ze - zb; ++s) {
    const int z = zb + s;
    collide_src(z + 1);
    if (s >= 0) {
      put(0, 0);  // down populations of layer z+1
      __syncthreads();
      const bool store = interior && !(BB == LBM_HALFWAY && (geo_cur & 1u));
      if (store) {
        const int64_t n = (int64_t)z * plane_nodes + col;
        const T* up = L + S::R2 + (s & 1) * 5 * P;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int c = Vel::cz[i] + 1, nd = zmarch::count_of(c);
          const int pos = t - Vel::cy[i] * HX - Vel::cx[i];
          const T* reg = c == 0 ? L + S::R0 : (c == 1 ? L + S::R1 : up);
          T v = reg[pos * nd + zmarch::idx_of(i)];
          if (BB == LBM_HALFWAY && i != 0 && ((geo_cur >> i) & 1u)) v = gprev[Vel::opp[i]];
          dst[n * Q + i] = v;
        }
      }
      __syncthreads();
    }
    // level populations of layer z+1 (used at step s+1), up populations
    // into the set that held layer z-1 (used at step s+2)
    put(1, 0);
    put(2, s & 1);
    if (BB == LBM_HALFWAY) {
#pragma unroll
      for (int i = 0; i < Q; ++i) gprev[i] = g[i];
    }
    geo_cur = geo_next;
    if (s + 1 < ze - zb) load(z + 2);
  }
}

// ---- AA neighbour step over AoS records -------------------------------------
// Node x reads slot opp(i) of x - c_i and, after collision, writes f*_i into
// slot i of x + c_i, in place.  The reads follow the z march of the push
// skeleton without the collision at the source: one thread per halo'd
// position loads that node's record and sorts its slots into the class
// regions (the slot staged for direction i is opp(i)).  Every slot is read
// and then written by the one node that owns it (x reads and writes slot i
// of x + c_i's record... as opp(i) of its source), so staging whole records
// in place is safe: the slots of other nodes that come along are never used.
//
// The writes: a record receives its slots over three steps (from the nodes
// of the layer below, its own layer and the layer above) and, at the column
// edge, from neighbouring columns, so slot-by-slot stores reach HBM as
// partially written lines about three times each.  Records whose 19 writers
// all lie in this column and chunk ("inner" records: 2 .. seg-1 in x and
// y, layers zb+1 .. ze-2) are therefore assembled in LDS instead: seeded
// with the record as loaded (slots whose writer is a solid node keep their
// value), filled by the writers and stored whole one step after their last
// writer.  Only the edge records are written slot by slot.
template <int BX, int TY>
struct AaShape {
  static constexpr int NI = (BX - 2) * (TY - 2);  // inner records per layer
  static constexpr int OB = 3 * NI * Q;           // assembly ring of three layers
};

template <class ST, int BB, int BX, int TY>
__global__ void __launch_bounds__((PushShape<BX, TY>::NT))
k_aa_aos_odd(typename ST::T* A, const uint8_t* __restrict__ mask,
             const uint32_t* __restrict__ links, int nx, int ny, int nz, int zc, int n_tiles,
             Collide<typename ST::R> k) {
  using T = typename ST::T;
  using R = typename ST::R;
  using S = PushShape<BX, TY>;
  constexpr int HX = S::HX, P = S::P, NI = AaShape<BX, TY>::NI, IW = BX - 2;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* L = reinterpret_cast<T*>(lds_raw);
  T* OB = L + S::STAGE;  // [3][NI][Q]

  const int per = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= n_tiles) return;
  const int tiles_x = (nx + BX - 1) / BX, tiles_y = (ny + TY - 1) / TY;
  const int tx_t = tile % tiles_x;
  const int ty_t = (tile / tiles_x) % tiles_y;
  const int zb = (tile / tiles_x / tiles_y) * zc;
  const int ze = zb + zc < nz ? zb + zc : nz;
  const int x0 = tx_t * BX, y0 = ty_t * TY;
  const int seg = nx - x0 < BX ? nx - x0 : BX;
  const int segy = ny - y0 < TY ? ny - y0 : TY;
  const int t = threadIdx.x;
  const bool live = t < P;
  const int pt = live ? t : P - 1;
  const int hy = pt / HX, hx = pt - hy * HX;
  const bool interior = live && hx >= 1 && hx <= seg && hy >= 1 && hy <= segy;
  int xs = x0 - 1 + (hx < seg + 1 ? hx : seg + 1);
  int ys = y0 - 1 + (hy < segy + 1 ? hy : segy + 1);
  xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
  ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
  const int64_t plane_nodes = (int64_t)nx * ny;
  const int64_t col = (int64_t)ys * nx + xs;
  auto wrapz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  // neighbour record offsets of an interior node (x, y), wrapped per axis
  const int64_t ox[3] = {xs == 0 ? nx - 1 : -1, 0, xs == nx - 1 ? 1 - nx : 1};
  const int64_t oy[3] = {(ys == 0 ? ny - 1 : -1) * (int64_t)nx, 0,
                         (ys == ny - 1 ? 1 - ny : 1) * (int64_t)nx};
  // inner records: halo'd position (hx, hy) and logical layer L
  auto inner_xy = [&](int px, int py) { return px >= 2 && px <= seg - 1 && py >= 2 && py <= segy - 1; };
  auto inner_z = [&](int zl) { return zl >= zb + 1 && zl <= ze - 2; };
  auto ring = [&](int zl) { return (zl - zb + 3) % 3; };
  auto ob_at = [&](int zl, int px, int py) {
    return OB + ((int64_t)ring(zl) * NI + (py - 2) * IW + (px - 2)) * Q;
  };

  T r[Q];
  uint32_t geo_next = 0;
  auto load = [&](int z) {
    const int64_t node = wrapz(z) * plane_nodes + col;
#pragma unroll
    for (int i = 0; i < Q; ++i) r[i] = A[node * Q + i];
    geo_next = BB == LBM_HALFWAY ? links[node] : (uint32_t)mask[node];
  };
  // class c slots of r into its region (up: set par): direction i of the
  // class is staged as slot opp(i)
  auto put = [&](int c, int par) {
    if (!live) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (Vel::cz[i] + 1 != c) continue;
      const int nd = zmarch::count_of(c);
      const int base = c == 0 ? S::R0 : (c == 1 ? S::R1 : S::R2 + par * 5 * P);
      L[base + t * nd + zmarch::idx_of(i)] = r[Vel::opp[i]];
    }
  };

  uint32_t geo_cur = 0;
  load(zb - 1);
  for (int s = -2; s < ze - zb; ++s) {
    const int z = zb + s;
    if (s >= 0) {
      put(0, 0);  // down slots of layer z+1
      if (live && inner_xy(hx, hy) && inner_z(z + 1)) {  // seed its assembly
        T* d = ob_at(z + 1, hx, hy);
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = r[i];
      }
      __syncthreads();
      const bool solid = BB == LBM_HALFWAY ? (geo_cur & 1u) != 0 : geo_cur != 0;
      R f[Q];
      if (interior && !solid) {
        const T* up = L + S::R2 + (s & 1) * 5 * P;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int c = Vel::cz[i] + 1, nd = zmarch::count_of(c);
          const int pos = t - Vel::cy[i] * HX - Vel::cx[i];
          const T* reg = c == 0 ? L + S::R0 : (c == 1 ? L + S::R1 : up);
          f[i] = ST::load(reg[pos * nd + zmarch::idx_of(i)], k.inv_scale);
        }
      }
      __syncthreads();
      // level slots of layer z+1 (used at step s+1), up slots into the set
      // that held layer z-1 (used at step s+2); then load layer z+2
      put(1, 0);
      put(2, s & 1);
      const uint32_t lk = geo_cur;
      geo_cur = geo_next;
      if (s + 1 < ze - zb) load(z + 2);
      if (interior && !solid) {
        const int64_t n = (int64_t)z * plane_nodes + col;
        T* const home = A + n * Q;
        if (BB == LBM_HALFWAY && (lk >> 1)) {
#pragma unroll
          for (int i = 1; i < Q; ++i)
            if ((lk >> i) & 1u) f[i] = ST::load(home[i], k.inv_scale);
        }
        trt_collide<R, ST::kShifted>(f, k);
        const int64_t oz[3] = {(z == 0 ? nz - 1 : -1) * plane_nodes, 0,
                               (z == nz - 1 ? 1 - nz : 1) * plane_nodes};
        SrStream rs((uint32_t)n, k.step, ST::kStochastic);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const T v = ST::store(f[i], k.scale, rs.next());
          // link bit opp(i): x + c_i is solid, the population stays home
          if (BB == LBM_HALFWAY && i != 0 && ((lk >> Vel::opp[i]) & 1u)) {
            if (inner_xy(hx, hy) && inner_z(z)) ob_at(z, hx, hy)[Vel::opp[i]] = v;
            else home[Vel::opp[i]] = v;
          } else {
            const int px = hx + Vel::cx[i], py = hy + Vel::cy[i], zl = z + Vel::cz[i];
            if (inner_xy(px, py) && inner_z(zl)) ob_at(zl, px, py)[i] = v;
            else home[(ox[Vel::cx[i] + 1] + oy[Vel::cy[i] + 1] + oz[Vel::cz[i] + 1]) * Q + i] = v;
          }
        }
      }
      // the records of layer z-1 have had their last writers: store them
      __syncthreads();
      if (inner_z(z - 1) && t < NI) {
        const int px = t % IW + 2, py = t / IW + 2;
        if (px <= seg - 1 && py <= segy - 1) {
          const T* src = ob_at(z - 1, px, py);
          T* dst = A + ((wrapz(z - 1) * plane_nodes) + (int64_t)(y0 + py - 1) * nx + (x0 + px - 1)) * Q;
#pragma unroll
          for (int i = 0; i < Q; ++i) dst[i] = src[i];
        }
      }
      __syncthreads();  // the next step seeds this ring slot again
    } else {
      // s = -2: up slots of layer zb-1 (set 0); s = -1: level and up slots
      // of layer zb (set 1)
      if (s == -1) put(1, 0);
      put(2, s & 1);
      geo_cur = geo_next;
      load(z + 2);
    }
  }
}

template <class ST, int BX, int TY>
static hipError_t launch_push_aos_t(lbm_ctx* c, const void* src, void* dst) {
  using T = typename ST::T;
  const lbm_params& p = c->p;
  const auto k = make_collide<typename ST::R>(p, c->step);
  int zc, n_tiles;
  unsigned grid;
  march_grid(p, BX, TY, zc, n_tiles, grid);
  using S = PushShape<BX, TY>;
  const size_t lds = sweep_lds(c, (size_t)S::STAGE * sizeof(T));
  if (p.bounce == LBM_FULLWAY)
    hipLaunchKernelGGL((k_push_aos<ST, LBM_FULLWAY, BX, TY>), dim3(grid), dim3(S::NT), lds,
                       c->stream, (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny, p.nz,
                       zc, n_tiles, k);
  else
    hipLaunchKernelGGL((k_push_aos<ST, LBM_HALFWAY, BX, TY>), dim3(grid), dim3(S::NT), lds,
                       c->stream, (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny, p.nz,
                       zc, n_tiles, k);
  return hipGetLastError();
}

hipError_t launch_push_aos(lbm_ctx* c, const void* src, void* dst) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    return launch_push_aos_t<ST, 32, 8>(c, src, dst);
  });
}


hipError_t launch_pull_aos(lbm_ctx* c, const void* src, void* dst) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    constexpr int BX = kAosBX, TY = kAosTY;
    const lbm_params& p = c->p;
    const auto k = make_collide<typename ST::R>(p, c->step);
    int zc, n_tiles;
    unsigned grid;
    march_grid(p, BX, TY, zc, n_tiles, grid);
    const size_t lds = sweep_lds(c, zmarch::lds_bytes<BX, TY, T>());
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_sweep_aos<ST, LBM_FULLWAY, BX, TY>), dim3(grid), dim3(BX * TY), lds,
                         c->stream, (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny,
                         p.nz, zc, n_tiles, k);
    else
      hipLaunchKernelGGL((k_sweep_aos<ST, LBM_HALFWAY, BX, TY>), dim3(grid), dim3(BX * TY), lds,
                         c->stream, (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny,
                         p.nz, zc, n_tiles, k);
    return hipGetLastError();
  });
}

hipError_t launch_pull_aos_diag(lbm_ctx* c, const void* src, void* dst, int residual_mode,
                                double* partials, int64_t* records) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    using T = typename ST::T;
    constexpr int BX = kAosBX, TY = kAosTY;
    const lbm_params& p = c->p;
    const auto k = make_collide<typename ST::R>(p, c->step);
    int zc, n_tiles;
    unsigned grid;
    march_grid(p, BX, TY, zc, n_tiles, grid);
    *records = n_tiles;
    DiagArgs d;
    d.gx = p.g[0];
    d.gy = p.g[1];
    d.gz = p.g[2];
    d.u_prev = c->b.u_prev;
    d.residual_mode = residual_mode;
    d.partials = partials;
    const size_t lds = sweep_lds(c, zmarch::lds_bytes<BX, TY, T>());
    if (p.bounce == LBM_FULLWAY)
      hipLaunchKernelGGL((k_sweep_aos_diag<ST, LBM_FULLWAY, BX, TY>), dim3(grid), dim3(BX * TY),
                         lds, c->stream, (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny,
                         p.nz, zc, n_tiles, k, d);
    else
      hipLaunchKernelGGL((k_sweep_aos_diag<ST, LBM_HALFWAY, BX, TY>), dim3(grid), dim3(BX * TY),
                         lds, c->stream, (const T*)src, (T*)dst, c->b.mask, c->b.links, p.nx, p.ny,
                         p.nz, zc, n_tiles, k, d);
    return hipGetLastError();
  });
}

template <class ST, int BX, int TY>
static hipError_t launch_aa_aos_odd_t(lbm_ctx* c, void* buf) {
  using T = typename ST::T;
  using S = PushShape<BX, TY>;
  const lbm_params& p = c->p;
  const auto k = make_collide<typename ST::R>(p, c->step);
  int zc, n_tiles;
  unsigned grid;
  march_grid(p, BX, TY, zc, n_tiles, grid);
  const size_t lds = sweep_lds(c, (size_t)(S::STAGE + AaShape<BX, TY>::OB) * sizeof(T));
  if (p.bounce == LBM_FULLWAY)
    hipLaunchKernelGGL((k_aa_aos_odd<ST, LBM_FULLWAY, BX, TY>), dim3(grid), dim3(S::NT), lds,
                       c->stream, (T*)buf, c->b.mask, c->b.links, p.nx, p.ny, p.nz, zc, n_tiles, k);
  else
    hipLaunchKernelGGL((k_aa_aos_odd<ST, LBM_HALFWAY, BX, TY>), dim3(grid), dim3(S::NT), lds,
                       c->stream, (T*)buf, c->b.mask, c->b.links, p.nx, p.ny, p.nz, zc, n_tiles, k);
  return hipGetLastError();
}

// Column shapes as measured at 512^3 (neighbour step, full-way / half-way):
// FP64 64 x 4 (15.5 / 17.4 ms; 32 x 8: 16.2 / 18.0; 16 x 8: 16.7 / 17.3),
// the 4- and 2-byte storages 16 x 8 (FP32 9.4 / 9.5 ms; 32 x 8: 10.1 / 11.3).
hipError_t launch_aa_aos_odd(lbm_ctx* c, void* buf) {
  return with_storage(c->p, [&](auto st) -> hipError_t {
    using ST = decltype(st);
    if (sizeof(typename ST::T) == 8) return launch_aa_aos_odd_t<ST, 64, 4>(c, buf);
    return launch_aa_aos_odd_t<ST, 16, 8>(c, buf);
  });
}

}  // namespace lbm
