// launch.hpp - host helpers shared by the sweep launchers: collision
// constants, LDS sizing, the row-per-workgroup block size and the storage
// type switch.
#pragma once

#include "d3q19.hpp"
#include "internal.hpp"

namespace lbm {

constexpr int kLdsPerCU = 163840;  // gfx950: 160 KiB of LDS per compute unit

template <typename R>
inline Collide<R> make_collide(const lbm_params& p, int64_t step) {
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
inline size_t sweep_lds(const lbm_ctx* c, size_t need) {
  if (c->p.cu_slots > 0) {
    size_t cap = (size_t)(kLdsPerCU / c->p.cu_slots) & ~(size_t)255;
    if (cap > need) return cap;
  }
  return need;
}

// Workgroup size of a row-per-workgroup launch: the configured size, cut to
// the row length rounded up to whole wavefronts.
inline int row_block(const lbm_ctx* c) {
  const int nx_r = ((c->p.nx + 63) / 64) * 64;
  return c->block > nx_r ? nx_r : c->block;
}

// Launch grid of a z march over BX x TY columns: about 8192 workgroups
// (16 rounds of two per compute unit measured better than fewer, longer
// marches), z chunks of at least 32 layers (each chunk reads two extra
// layers) split evenly, the grid padded to whole rounds of the 8 XCDs.
inline void march_grid(const lbm_params& p, int BX, int TY, int& zc, int& n_tiles,
                       unsigned& grid) {
  const int64_t cols = (int64_t)((p.nx + BX - 1) / BX) * ((p.ny + TY - 1) / TY);
  int64_t nzc = (8192 + cols - 1) / cols;
  const int64_t max_chunks = (p.nz + 31) / 32;
  if (nzc > max_chunks) nzc = max_chunks;
  if (nzc < 1) nzc = 1;
  zc = (int)((p.nz + nzc - 1) / nzc);
  nzc = (p.nz + zc - 1) / zc;
  n_tiles = (int)(cols * nzc);
  grid = (unsigned)((n_tiles + 7) / 8 * 8);
}

// Calls fn(storage tag) for the configured storage.
template <class Fn>
inline hipError_t with_storage(const lbm_params& p, Fn&& fn) {
  switch (p.storage) {
    case LBM_F64: return fn(StoreF64{});
    case LBM_F32_SHIFTED: return fn(StoreF32Shifted{});
    case LBM_F16_SHIFTED: return fn(StoreF16Shifted{});
    default: return fn(StoreF16ShiftedSR{});
  }
}

}  // namespace lbm
