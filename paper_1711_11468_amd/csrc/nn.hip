// nn.hip - BF16 MFMA kernels of the learned warm start (ABI: include/lbm_nn.h).
//
// Convolutions are implicit GEMMs.  On grids that their LDS tiles cover
// (16 x 4 x 4 voxels; 16 x 2 x 4 outputs under stride 2) the
// stride-1 and stride-2 3x3x3 forwards, the stride-1 data gradient (the
// forward of dy with mirrored, transposed weights) and the stride-1 weight
// gradient run through LDS on v_mfma_f32_16x16x32_bf16 (k_conv_fwd_lds,
// k_conv_fwd_lds_s2, k_conv_wgrad_brick below); the other forms use
// v_mfma_f32_16x16x16_bf16, where one wavefront
// owns a 16 x 16 tile of the (voxel x channel) output and walks the K
// dimension (taps x input-channel chunks of 16).  Operand layout of the
// instruction (64 lanes, l = lane): A[i][k] lives in lane i + 16*(k/4),
// element k%4; B[k][j] in lane j + 16*(k/4), element k%4; the float32 result
// D[i][j] in lane j + 16*(i/4), element i%4.  Channels-last tensors make the
// 4 consecutive K elements of a lane 8 contiguous bytes.
#include <stdint.h>

#include <cmath>
#include <mutex>

#include "../../include/lbm_nn.h"
#include "internal.hpp"

namespace lbm {
namespace nn {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8).  Renumbering them so that each XCD works through one contiguous
// range of tiles keeps the neighbouring tiles that share input voxels in the
// same L2.  The grid is launched padded to a multiple of 8; indices at or
// beyond n_real mark padding workgroups, which exit.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n_launched) {
  const int64_t per = n_launched / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

struct Geom {
  int B, D, H, W;     // input grid
  int Do, Ho, Wo;     // output grid
  int ci, co, cstore;
  int act;
  float slope;
  int64_t m_out;      // B*Do*Ho*Wo
  int64_t m_in;       // B*D*H*W
};

__device__ __forceinline__ void tap_offsets(int tap, int taps, int& dz, int& dy, int& dx) {
  if (taps == 27) {
    dz = tap / 9 - 1;
    dy = (tap / 3) % 3 - 1;
    dx = tap % 3 - 1;
  } else {
    dz = dy = dx = 0;
  }
}

// ---- forward --------------------------------------------------------------
// A wavefront owns MT consecutive 16-voxel tiles and all NB 16-channel
// output blocks: per tap and 16-channel input chunk it loads MT A fragments
// and NB B fragments and issues MT x NB MFMAs, so each weight fragment
// serves MT tiles and each input fragment NB output blocks.  The periodic
// neighbour of a lane's voxel is found from per-axis offsets computed once
// (the taps are unrolled, so each tap just adds three of them).
struct AxisOff {
  int base;     // input voxel index of the tap (0, 0, 0) source
  int oz[3], oy[3], ox[3];  // voxel-index offsets of the sources at -1, 0, +1
};

// Offsets of the sources s*c + d (d = -1, 0, 1; periodic) on one axis of
// extent n, scaled by that axis' voxel stride.
__device__ __forceinline__ void axis_offsets(int c, int s, int n, int stride, int (&o)[3]) {
  const int c0 = s * c;
#pragma unroll
  for (int d = -1; d <= 1; ++d) o[d + 1] = (wrapi(c0 + d, n) - c0) * stride;
}

// Moves an A fragment one voxel along the 16 voxels (lanes) of each
// 16-lane row of the wavefront: lane r takes lane r - 1 (down) or r + 1
// (up); the edge lane with no neighbour in the row keeps `edge`.
__device__ __forceinline__ s4 frag_shift(s4 edge, s4 v, bool up) {
  union U { s4 f; int i[2]; };
  U e, a, r;
  e.f = edge;
  a.f = v;
#pragma unroll
  for (int h = 0; h < 2; ++h)
    r.i[h] = up ? __builtin_amdgcn_update_dpp(e.i[h], a.i[h], 0x101, 0xF, 0xF, false)   // row_shl:1
                : __builtin_amdgcn_update_dpp(e.i[h], a.i[h], 0x111, 0xF, 0xF, false);  // row_shr:1
  return r.f;
}

template <int STRIDE, int TAPS, int NB, bool OUTF32, int MT, bool XS>
__global__ void __launch_bounds__(256)
k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
           const float* __restrict__ bias, void* __restrict__ y, int nsplit, Geom g) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = xcd_tile(blockIdx.x, gridDim.x);
  // small grids: nsplit wavefronts share a tile, each with NB of the output
  // channel blocks
  const int64_t wv = blk * 4 + (threadIdx.x >> 6);
  const int part = (int)(wv % nsplit);
  const int64_t v0 = (wv / nsplit) * 16 * MT;
  if (v0 >= g.m_out) return;
  const int row = lane & 15, kq = lane >> 4;
  AxisOff ao[MT];
  bool live[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    live[m] = v0 + 16 * m < g.m_out;
    int64_t t = live[m] ? v0 + 16 * m + row : 0;
    const int xo = (int)(t % g.Wo);
    t /= g.Wo;
    const int yo = (int)(t % g.Ho);
    t /= g.Ho;
    const int zo = (int)(t % g.Do);
    const int b = (int)(t / g.Do);
    ao[m].base = ((b * g.D + STRIDE * zo) * g.H + STRIDE * yo) * g.W + STRIDE * xo;
    axis_offsets(zo, STRIDE, g.D, g.H * g.W, ao[m].oz);
    axis_offsets(yo, STRIDE, g.H, g.W, ao[m].oy);
    axis_offsets(xo, STRIDE, g.W, 1, ao[m].ox);
  }
  f4 acc[MT][NB];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* xl = x + 4 * kq;
  if constexpr (XS) {
    // Stride 1 with x-aligned tiles: the three x taps of a (z, y) pair read
    // the same 16 voxels shifted by one, so one fragment is loaded and
    // shifted across lanes; only the voxels just outside the tile come
    // from memory (one lane per row).
#pragma unroll
    for (int zy = 0; zy < 9; ++zy) {
      const int iz = zy / 3, iy = zy % 3;
      const uint16_t *xc[MT], *xm[MT], *xq[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int o = ao[m].base + ao[m].oz[iz] + ao[m].oy[iy];
        xc[m] = xl + (int64_t)(o + ao[m].ox[1]) * g.ci;
        xm[m] = xl + (int64_t)(o + ao[m].ox[0]) * g.ci;
        xq[m] = xl + (int64_t)(o + ao[m].ox[2]) * g.ci;
      }
      const uint16_t* wp = w + ((int64_t)(3 * zy) * g.co + part * NB * 16 + row) * g.ci + 4 * kq;
      const int64_t tap_stride = (int64_t)g.co * g.ci;
      for (int c0 = 0; c0 < g.ci; c0 += 16) {
        s4 a[3][MT], bv[NB];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          a[1][m] = *(const s4*)(xc[m] + c0);
          s4 e0 = a[1][m], e2 = a[1][m];
          if (row == 0) e0 = *(const s4*)(xm[m] + c0);
          if (row == 15) e2 = *(const s4*)(xq[m] + c0);
          a[0][m] = frag_shift(e0, a[1][m], false);
          a[2][m] = frag_shift(e2, a[1][m], true);
        }
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            bv[nb] = *(const s4*)(wp + ix * tap_stride + (int64_t)nb * 16 * g.ci + c0);
#pragma unroll
          for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[ix][m], bv[nb], acc[m][nb], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int tap = 0; tap < (XS ? 0 : TAPS); ++tap) {
    const int iz = TAPS == 27 ? tap / 9 : 1, iy = TAPS == 27 ? (tap / 3) % 3 : 1,
              ix = TAPS == 27 ? tap % 3 : 1;
    const uint16_t* xp[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
      xp[m] = xl + (int64_t)(ao[m].base + ao[m].oz[iz] + ao[m].oy[iy] + ao[m].ox[ix]) * g.ci;
    const uint16_t* wp = w + ((int64_t)tap * g.co + part * NB * 16 + row) * g.ci + 4 * kq;
    for (int c0 = 0; c0 < g.ci; c0 += 16) {
      s4 a[MT], bv[NB];
#pragma unroll
      for (int m = 0; m < MT; ++m) a[m] = *(const s4*)(xp[m] + c0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bv[nb] = *(const s4*)(wp + (int64_t)nb * 16 * g.ci + c0);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[m], bv[nb], acc[m][nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    if (!live[m]) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = (part * NB + nb) * 16 + row;
      if (co >= g.cstore) continue;
      const float bb = bias ? bias[co] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t vox = v0 + 16 * m + 4 * kq + r;
        float v = acc[m][nb][r] + bb;
        if (g.act) v = v > 0.f ? v : v * g.slope;
        if (OUTF32) ((float*)y)[vox * g.cstore + co] = v;
        else ((uint16_t*)y)[vox * g.cstore + co] = f2bf(v);
      }
    }
  }
}

// ---- forward through LDS, gfx950 16x16x32 MFMA ------------------------------
// Stride-1 3x3x3 convolution on grids whose W is a multiple of 16 and whose
// D and H are multiples of 4.  A workgroup computes a 16 x 4 x 4 (x, y, z)
// block of output voxels for every output channel.  Per chunk of 32 input
// channels (16 for a remainder) it stages the 18 x 6 x 6 input voxels of the
// block and its periodic halo in LDS once; the four wavefronts (one z plane
// each, four 16-voxel rows) then run all 27 taps from LDS, 32 channels of K
// per v_mfma_f32_16x16x32_bf16 (a 16-channel chunk puts two taps side by
// side).
// Operand layout of the instruction (l = lane, e = 0..7 / 0..3): A[i][k] in
// lane i + 16*(k/8), element k%8; B[k][j] in lane j + 16*(k/8), element k%8;
// D[i][j] in lane j + 16*(i/4), element i%4.  A holds the weights (i: output
// channel), B the input (j: voxel of the row), so a lane ends with four
// consecutive output channels of one voxel and stores them at once.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int kLdsTX = 16, kLdsTY = 4, kLdsTZ = 4;
constexpr int kLdsHX = kLdsTX + 2, kLdsHY = kLdsTY + 2, kLdsHZ = kLdsTZ + 2;
constexpr int kLdsHalo = kLdsHX * kLdsHY * kLdsHZ;  // 648 voxels
constexpr int kLdsChunk = 32;                       // input channels per stage
constexpr int kLdsPad = 8;                          // bf16 pad per staged voxel
// Workgroups the LDS forward aims for: output-channel blocks are split over
// workgroups until a launch has at least this many (one per compute unit).
constexpr int64_t kLdsMinGroups = 256;

// Moves a 16-byte fragment one voxel along the 16 lanes of each row of the
// wavefront: lane r takes lane r - 1 (up = false) or r + 1 (up = true); the
// lane with no neighbour in its row takes `edge`.
__device__ __forceinline__ bf8 row_shift8(bf8 edge, bf8 v, bool up) {
  union U { bf8 f; int i[4]; };
  U e, a, r;
  e.f = edge;
  a.f = v;
#pragma unroll
  for (int h = 0; h < 4; ++h)
    r.i[h] = up ? __builtin_amdgcn_update_dpp(e.i[h], a.i[h], 0x101, 0xF, 0xF, false)   // row_shl:1
                : __builtin_amdgcn_update_dpp(e.i[h], a.i[h], 0x111, 0xF, 0xF, false);  // row_shr:1
  return r.f;
}

// One staged chunk of CK (16 or 32) input channels, all 27 taps.  The three
// x taps of a (z, y) pair read the same 16 staged voxels shifted by one, so
// per (z, y) pair and row one fragment is read (the voxels x0 .. x0 + 15)
// with the two halo voxels of the row, each read by all 16 lanes of a row
// at one address (an LDS broadcast); the x - 1 and x + 1 operands are lane
// shifts of it.  CK = 32: lanes take channels 8 * (lane / 16) .. + 7 of one
// tap.  CK = 16: lanes 0-31 and 32-63 take two different (z, y) pairs
// (half = lane / 32) with the same x tap; the ninth pair runs with zero
// weights in the upper half.  srow points at the lane's channel group in the
// staged voxel (x = -1, y = -1, z = wave - 1); wbase at the lane's output
// channel and channel group in tap 0.
template <int CK, int NB>
__device__ __forceinline__ void conv_lds_chunk(const uint16_t* __restrict__ srow,
                                               const uint16_t* __restrict__ wbase, int row, int half,
                                               int ci, int64_t tap_stride, f4 (&acc)[kLdsTY][NB]) {
  constexpr int VS = CK + kLdsPad;
  constexpr int NPAIR = CK == 32 ? 9 : 5;  // instructions per x tap
  const bf8 zero8 = {};
#pragma unroll
  for (int p = 0; p < NPAIR; ++p) {
    // the (z, y) pair of this lane's half
    const int ca = CK == 32 ? p : 2 * p;
    const bool pad = CK == 16 && 2 * p + 1 > 8;
    const int cb = CK == 32 ? p : (pad ? ca : 2 * p + 1);
    const int c = half ? cb : ca;
    const int zy = ((c / 3) * kLdsHY + c % 3) * kLdsHX * VS;  // staged offset of the pair
    bf8 wf[3][NB];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        wf[dx][nb] = *(const bf8*)(wbase + (int64_t)(3 * c + dx) * tap_stride + (int64_t)nb * 16 * ci);
        if (pad && half) wf[dx][nb] = zero8;
      }
#pragma unroll
    for (int m = 0; m < kLdsTY; ++m) {
      const uint16_t* rp = srow + zy + m * kLdsHX * VS;
      const bf8 mid = *(const bf8*)(rp + (row + 1) * VS);
      const bf8 lo = *(const bf8*)(rp);                    // staged x = 0, all lanes of the row
      const bf8 hi = *(const bf8*)(rp + (kLdsHX - 1) * VS);  // staged x = 17
      const bf8 bm = row_shift8(lo, mid, false);           // voxels x - 1
      const bf8 bp = row_shift8(hi, mid, true);            // voxels x + 1
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[0][nb], bm, acc[m][nb], 0, 0, 0);
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[1][nb], mid, acc[m][nb], 0, 0, 0);
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[2][nb], bp, acc[m][nb], 0, 0, 0);
      }
    }
  }
}

template <int NB, bool OUTF32, bool ACC = false>
__global__ void __launch_bounds__(256)
k_conv_fwd_lds(const uint16_t* __restrict__ x, const uint16_t* __restrict__ xc, int c1,
               const uint16_t* __restrict__ w, const float* __restrict__ bias, void* __restrict__ y,
               int64_t n_tiles, int parts, Geom g) {
  extern __shared__ __align__(16) uint16_t stage[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4, half = kq >> 1;
  // workgroup -> (block, part): the `parts` workgroups of a block each take
  // NB of its 16-channel output blocks (consecutive, so on the same XCD)
  int64_t t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= n_tiles * parts) return;
  const int co0 = (int)(t % parts) * NB * 16;
  t /= parts;
  const int tx = g.W / kLdsTX, ty = g.H / kLdsTY, tz = g.D / kLdsTZ;
  const int x0 = (int)(t % tx) * kLdsTX;
  t /= tx;
  const int y0 = (int)(t % ty) * kLdsTY;
  t /= ty;
  const int z0 = (int)(t % tz) * kLdsTZ;
  const int b = (int)(t / tz);
  f4 acc[kLdsTY][NB];
#pragma unroll
  for (int m = 0; m < kLdsTY; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t tap_stride = (int64_t)g.co * g.ci;
  const int vz = wave * kLdsHY * kLdsHX;  // staged voxel (x = -1, y = -1) of the wave's z plane
  for (int c0 = 0; c0 < g.ci; c0 += kLdsChunk) {
    const int ck = g.ci - c0 < kLdsChunk ? g.ci - c0 : kLdsChunk;  // 32 or 16
    const int vs = ck + kLdsPad;                                    // staged voxel stride
    const int pieces = ck / 8;                                      // 16-byte pieces per voxel
    __syncthreads();  // the previous chunk has been read
    for (int p = threadIdx.x; p < kLdsHalo * pieces; p += 256) {
      const int v = p / pieces, piece = p - v * pieces;
      const int hx = v % kLdsHX, hy = (v / kLdsHX) % kLdsHY, hz = v / (kLdsHX * kLdsHY);
      const int gx = wrapi(x0 + hx - 1, g.W), gy = wrapi(y0 + hy - 1, g.H), gz = wrapi(z0 + hz - 1, g.D);
      const int64_t gv = (((int64_t)b * g.D + gz) * g.H + gy) * g.W + gx;
      // channels below c1 come from the coarse tensor, up-sampled by taking
      // the coarse voxel (x / 2, y / 2, z / 2); the rest from x, which then
      // holds g.ci - c1 channels (c1 = 0: x is the whole input)
      const int ch = c0 + piece * 8;
      const bool coarse = ch < c1;
      const int64_t cv = (((int64_t)b * (g.D >> 1) + (gz >> 1)) * (g.H >> 1) + (gy >> 1)) * (g.W >> 1) + (gx >> 1);
      const int64_t off = coarse ? cv * c1 + ch : gv * (g.ci - c1) + (ch - c1);
      const uint16_t* base = coarse ? xc : x;
      *(uint4*)(stage + v * vs + piece * 8) = *(const uint4*)(base + off);
    }
    __syncthreads();
    // channel group of the lane: 8 * (lane / 16) of a 32-channel chunk, or
    // 8 * (lane / 16 % 2) of a 16-channel chunk (the halves take two taps)
    const int grp = ck == 32 ? 8 * kq : 8 * (kq & 1);
    const uint16_t* wbase = w + (int64_t)(co0 + row) * g.ci + c0 + grp;
    if (ck == 32)
      conv_lds_chunk<32, NB>(stage + vz * (32 + kLdsPad) + grp, wbase, row, half, g.ci, tap_stride, acc);
    else
      conv_lds_chunk<16, NB>(stage + vz * (16 + kLdsPad) + grp, wbase, row, half, g.ci, tap_stride, acc);
  }
#pragma unroll
  for (int m = 0; m < kLdsTY; ++m) {
    const int64_t vox = (((int64_t)b * g.Do + z0 + wave) * g.Ho + y0 + m) * g.Wo + x0 + row;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int cb = co0 + nb * 16 + 4 * kq;  // first of the lane's four channels
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = acc[m][nb][e] + (bias ? bias[cb + e] : 0.f);
        if (g.act) v[e] = v[e] > 0.f ? v[e] : v[e] * g.slope;
      }
      if ((g.cstore & 3) == 0 && cb + 4 <= g.cstore) {  // aligned four-channel store
        if (OUTF32) {
          f4* o = (f4*)((float*)y + vox * g.cstore + cb);
          if (ACC) {
            const f4 old = *o;
            *o = f4{old[0] + v[0], old[1] + v[1], old[2] + v[2], old[3] + v[3]};
          } else {
            *o = f4{v[0], v[1], v[2], v[3]};
          }
        } else {
          const uint2 pk = {(uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                            (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16)};
          *(uint2*)((uint16_t*)y + vox * g.cstore + cb) = pk;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (cb + e >= g.cstore) continue;
          if (OUTF32) {
            float* o = (float*)y + vox * g.cstore + cb + e;
            *o = ACC ? *o + v[e] : v[e];
          } else {
            ((uint16_t*)y)[vox * g.cstore + cb + e] = f2bf(v[e]);
          }
        }
      }
    }
  }
}

// Stride-2 3x3x3 forward through LDS (the down-sampling layers), on output
// grids whose W is a multiple of 16 and H and D even.  A workgroup computes
// 16 x 2 x 4 (x, y, z) output voxels: it stages the 33 x 5 x 9 input voxels
// they read (periodic halo included), 16 channels at a time, and each
// wavefront takes one output z plane and two rows.  For a row of 16 outputs
// the x taps read input voxels 2j, 2j + 1 and 2j + 2: the first two are
// read from LDS, the third is the first moved one lane up, its last voxel a
// broadcast.  K pairs two (z, y) taps of 16 channels per instruction, as in
// the stride-1 16-channel chunk.
constexpr int kS2TX = 16, kS2TY = 2, kS2TZ = 4;
constexpr int kS2HX = 2 * kS2TX + 1, kS2HY = 2 * kS2TY + 1, kS2HZ = 2 * kS2TZ + 1;
constexpr int kS2Halo = kS2HX * kS2HY * kS2HZ;  // 1485 voxels
constexpr int kS2VS = 16 + kLdsPad;             // staged voxel stride (16 channels)

template <int NB, bool OUTF32>
__global__ void __launch_bounds__(256)
k_conv_fwd_lds_s2(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                  const float* __restrict__ bias, void* __restrict__ y, int64_t n_tiles, int parts,
                  Geom g) {
  extern __shared__ __align__(16) uint16_t stage[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4, half = kq >> 1;
  int64_t t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= n_tiles * parts) return;
  const int co0 = (int)(t % parts) * NB * 16;
  t /= parts;
  const int tx = g.Wo / kS2TX, ty = g.Ho / kS2TY, tz = g.Do / kS2TZ;
  const int x0 = (int)(t % tx) * kS2TX;
  t /= tx;
  const int y0 = (int)(t % ty) * kS2TY;
  t /= ty;
  const int z0 = (int)(t % tz) * kS2TZ;
  const int b = (int)(t / tz);
  f4 acc[kS2TY][NB];
#pragma unroll
  for (int m = 0; m < kS2TY; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t tap_stride = (int64_t)g.co * g.ci;
  const int grp = 8 * (kq & 1);
  const bf8 zero8 = {};
  for (int c0 = 0; c0 < g.ci; c0 += 16) {
    __syncthreads();  // the previous chunk has been read
    for (int p = threadIdx.x; p < kS2Halo * 2; p += 256) {
      const int v = p >> 1, piece = p & 1;
      const int hx = v % kS2HX, hy = (v / kS2HX) % kS2HY, hz = v / (kS2HX * kS2HY);
      const int gx = wrapi(2 * x0 + hx - 1, g.W), gy = wrapi(2 * y0 + hy - 1, g.H),
                gz = wrapi(2 * z0 + hz - 1, g.D);
      const int64_t gv = (((int64_t)b * g.D + gz) * g.H + gy) * g.W + gx;
      *(uint4*)(stage + v * kS2VS + piece * 8) = *(const uint4*)(x + gv * g.ci + c0 + piece * 8);
    }
    __syncthreads();
    const uint16_t* wbase = w + (int64_t)(co0 + row) * g.ci + c0 + grp;
    // staged voxel (x = -1, y = -1) of the wave's output plane, lane's channels
    const uint16_t* srow = stage + (2 * wave) * kS2HY * kS2HX * kS2VS + grp;
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const bool pad = 2 * p + 1 > 8;
      const int ca = 2 * p, cb = pad ? ca : 2 * p + 1;
      const int c = half ? cb : ca;  // (z, y) tap of this lane's half
      const int dz = c / 3, dy = c % 3;
      bf8 wf[3][NB];
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          wf[dx][nb] = *(const bf8*)(wbase + (int64_t)(3 * c + dx) * tap_stride + (int64_t)nb * 16 * g.ci);
          if (pad && half) wf[dx][nb] = zero8;
        }
#pragma unroll
      for (int m = 0; m < kS2TY; ++m) {
        const uint16_t* rp = srow + (dz * kS2HY + 2 * m + dy) * kS2HX * kS2VS;
        const bf8 ev = *(const bf8*)(rp + (2 * row) * kS2VS);          // input 2j - 1 (tap x - 1)
        const bf8 od = *(const bf8*)(rp + (2 * row + 1) * kS2VS);      // input 2j (tap x)
        const bf8 hi = *(const bf8*)(rp + (kS2HX - 1) * kS2VS);        // staged x = 32, broadcast
        const bf8 nx = row_shift8(hi, ev, true);                        // input 2j + 1 (tap x + 1)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[0][nb], ev, acc[m][nb], 0, 0, 0);
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[1][nb], od, acc[m][nb], 0, 0, 0);
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[2][nb], nx, acc[m][nb], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kS2TY; ++m) {
    const int64_t vox = (((int64_t)b * g.Do + z0 + wave) * g.Ho + y0 + m) * g.Wo + x0 + row;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int cb = co0 + nb * 16 + 4 * kq;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = acc[m][nb][e] + (bias ? bias[cb + e] : 0.f);
        if (g.act) v[e] = v[e] > 0.f ? v[e] : v[e] * g.slope;
      }
      if ((g.cstore & 3) == 0 && cb + 4 <= g.cstore) {
        if (OUTF32) {
          *(f4*)((float*)y + vox * g.cstore + cb) = f4{v[0], v[1], v[2], v[3]};
        } else {
          const uint2 pk = {(uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                            (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16)};
          *(uint2*)((uint16_t*)y + vox * g.cstore + cb) = pk;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (cb + e >= g.cstore) continue;
          if (OUTF32) ((float*)y)[vox * g.cstore + cb + e] = v[e];
          else ((uint16_t*)y)[vox * g.cstore + cb + e] = f2bf(v[e]);
        }
      }
    }
  }
}

// 1x1x1 layer with at most four stored float32 outputs (the network's
// head): one thread per voxel holds its CI inputs and forms the stored
// outputs' dot products in float32; the weights and bias are the same for
// every thread.
template <int CI>
__global__ void k_conv1x1_few(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                              const float* __restrict__ bias, float* __restrict__ y, int64_t m,
                              int cstore, int act, float slope) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m) return;
  float xv[CI];
#pragma unroll
  for (int q = 0; q < CI / 8; ++q) {
    const uint4 u = *(const uint4*)(x + v * CI + 8 * q);
    const uint32_t p[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      xv[8 * q + 2 * h] = bf2f((uint16_t)(p[h] & 0xffffu));
      xv[8 * q + 2 * h + 1] = bf2f((uint16_t)(p[h] >> 16));
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= cstore) break;
    float sum = bias ? bias[c] : 0.f;
#pragma unroll
    for (int k = 0; k < CI; ++k) sum += bf2f(w[c * CI + k]) * xv[k];
    if (act) sum = sum > 0.f ? sum : sum * slope;
    y[v * cstore + c] = sum;
  }
}

// ---- data gradient --------------------------------------------------------
// dx[q] = sum over taps and output voxels p with s*p + off = q of W^T dy[p];
// MT input-voxel tiles per wavefront as in the forward kernel.  For tap
// offset d on an axis the source is t = q - d (periodic); under stride 2
// only even t are images of coarse voxels, at t / 2.  PAR (stride 2, W a
// multiple of 32): a tile holds the 16 voxels x = 32 xb + 2 j + px of one
// row, all of one parity on every axis, so whether a tap reaches the tile
// is the same for all its voxels, and the wavefront skips the taps that
// reach none of its tiles (3.4 of the 27 taps reach a tile on average; the
// tiles of a wavefront share a row, so 6.75 taps reach one of them).
template <int STRIDE, int TAPS, int NB, int MT, bool PAR = false>
__global__ void __launch_bounds__(256)
k_conv_dgrad(const uint16_t* __restrict__ dyp, const uint16_t* __restrict__ wt,
             float* __restrict__ dxp, int accumulate, int nsplit, Geom g) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = xcd_tile(blockIdx.x, gridDim.x);
  // small grids split the output blocks over nsplit wavefronts per tile group
  const int64_t wv = blk * 4 + (threadIdx.x >> 6);
  const int cb0 = (int)(wv % nsplit) * NB * 16;  // first output channel of the wavefront
  const int64_t q0 = (wv / nsplit) * 16 * MT;
  if (q0 >= g.m_in) return;
  const int row = lane & 15, kq = lane >> 4;
  // per tile: coarse-grid voxel offsets of the sources at d = -1, 0, +1 on
  // each axis (index d + 1), and their validity (bit d + 1)
  int base[MT], oz[MT][3], oy[MT][3], ox[MT][3];
  uint32_t vz[MT], vy[MT], vx[MT];
  bool live[MT];
  int64_t first[MT];  // PAR: the tile's first voxel; voxel j is first + 2 j
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    live[m] = q0 + 16 * m < g.m_in;
    int xq, yq, zq, b;
    if (PAR) {
      int64_t t = live[m] ? q0 / 16 + m : 0;  // tile index
      const int px = (int)(t & 1);
      t >>= 1;
      const int xbs = g.W / 32;
      const int xb = (int)(t % xbs);
      t /= xbs;
      yq = (int)(t % g.H);
      t /= g.H;
      zq = (int)(t % g.D);
      b = (int)(t / g.D);
      xq = xb * 32 + 2 * row + px;
      first[m] = (((int64_t)b * g.D + zq) * g.H + yq) * g.W + xb * 32 + px;
    } else {
      int64_t t = live[m] ? q0 + 16 * m + row : 0;
      xq = (int)(t % g.W);
      t /= g.W;
      yq = (int)(t % g.H);
      t /= g.H;
      zq = (int)(t % g.D);
      b = (int)(t / g.D);
      first[m] = 0;
    }
    base[m] = b * g.Do * g.Ho * g.Wo;
    vz[m] = vy[m] = vx[m] = 0;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
      const int tz = wrapi(zq - d, g.D), ty = wrapi(yq - d, g.H), tx = wrapi(xq - d, g.W);
      oz[m][d + 1] = (tz / STRIDE) * g.Ho * g.Wo;
      oy[m][d + 1] = (ty / STRIDE) * g.Wo;
      ox[m][d + 1] = tx / STRIDE;
      if (STRIDE == 1 || (tz & 1) == 0) vz[m] |= 1u << (d + 1);
      if (STRIDE == 1 || (ty & 1) == 0) vy[m] |= 1u << (d + 1);
      if (STRIDE == 1 || (tx & 1) == 0) vx[m] |= 1u << (d + 1);
    }
  }
  // PAR: the taps that reach a tile of the wavefront, one bit per tap (the
  // same for every lane, as W is even and wrapping keeps the parity), held
  // in a scalar register so that skipping a tap is a branch of the whole
  // wavefront (a matrix instruction under a lane mask would still run)
  uint32_t taps_run = 0;
  if (PAR) {
#pragma unroll
    for (int tap = 0; tap < 27; ++tap)
#pragma unroll
      for (int m = 0; m < MT; ++m)
        if ((vz[m] >> (tap / 9)) & (vy[m] >> ((tap / 3) % 3)) & (vx[m] >> (tap % 3)) & 1u) taps_run |= 1u << tap;
    taps_run = __builtin_amdgcn_readfirstlane(taps_run);
  }
  f4 acc[MT][NB];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* dl = dyp + 4 * kq;
#pragma unroll
  for (int tap = 0; tap < TAPS; ++tap) {
    const int iz = TAPS == 27 ? tap / 9 : 1, iy = TAPS == 27 ? (tap / 3) % 3 : 1,
              ix = TAPS == 27 ? tap % 3 : 1;
    const uint16_t* ap[MT];
    bool valid[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      valid[m] = ((vz[m] >> iz) & (vy[m] >> iy) & (vx[m] >> ix) & 1u) != 0;
      ap[m] = dl + (int64_t)(base[m] + oz[m][iz] + oy[m][iy] + ox[m][ix]) * g.co;
    }
    if (PAR && !((taps_run >> tap) & 1u)) continue;
    const uint16_t* bp = wt + ((int64_t)tap * g.ci + cb0 + row) * g.co + 4 * kq;
    for (int c0 = 0; c0 < g.co; c0 += 16) {
      s4 a[MT], bv[NB];
#pragma unroll
      for (int m = 0; m < MT; ++m) a[m] = valid[m] ? *(const s4*)(ap[m] + c0) : s4{0, 0, 0, 0};
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bv[nb] = *(const s4*)(bp + (int64_t)nb * 16 * g.co + c0);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[m], bv[nb], acc[m][nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    if (!live[m]) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = cb0 + nb * 16 + row;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t v = PAR ? first[m] + 2 * (4 * kq + r) : q0 + 16 * m + 4 * kq + r;
        float* o = dxp + v * g.ci + c;
        *o = accumulate ? *o + acc[m][nb][r] : acc[m][nb][r];
      }
    }
  }
}

// wt[tap'][ci][co] = w[tap][co][ci], with tap' = tap, or with the tap
// mirrored through the centre (tap' = taps - 1 - tap, the offset negated
// on every axis) when flip is set: the data gradient of a stride-1 layer is
// then the forward convolution of dy with wt.
__global__ void k_transpose_w(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int taps,
                              int co, int ci, int flip) {
  // one thread per element of wt, so the stores are contiguous
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= taps * co * ci) return;
  const int c_out = e % co;
  const int c_in = (e / co) % ci;
  const int tw = e / (co * ci);
  const int tap = flip ? taps - 1 - tw : tw;
  wt[e] = w[(tap * co + c_out) * ci + c_in];
}

// ---- weight gradient ------------------------------------------------------
// dW[tap][co][ci] = sum over output voxels p of dy[p][co] x[in(p, tap)][ci]:
// a GEMM whose K dimension is the voxel.  Grid (chunks, tap groups); a block
// owns a chunk of output voxels and a group of TPB taps.  Per 64-voxel step
// it stages dy once and the tap-shifted input of every tap of its group
// (16-byte loads, channels-last), both transposed to [channel][voxel] in LDS
// so each MFMA operand is one 8-byte LDS read; the TPB x (co/16) x (ci/16)
// output tiles are spread over the four wavefronts (at most TPW each).
constexpr int kWgRow = 68;  // LDS row: 64 voxels + 4 pad (8-byte aligned, fewer bank conflicts)

// Transposed store of four voxels x eight bf16 channels: row j of dst (rows
// kWgRow apart) receives channel j of voxels 0..3 as one 8-byte word.
__device__ __forceinline__ void store_t4(uint16_t* dst, const uint4 (&v)[4]) {
  const uint32_t w[4][4] = {{v[0].x, v[0].y, v[0].z, v[0].w}, {v[1].x, v[1].y, v[1].z, v[1].w},
                            {v[2].x, v[2].y, v[2].z, v[2].w}, {v[3].x, v[3].y, v[3].z, v[3].w}};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int h = j >> 1, sh = (j & 1) * 16;
    uint2 o;
    o.x = ((w[0][h] >> sh) & 0xffffu) | (((w[1][h] >> sh) & 0xffffu) << 16);
    o.y = ((w[2][h] >> sh) & 0xffffu) | (((w[3][h] >> sh) & 0xffffu) << 16);
    *(uint2*)(dst + j * kWgRow) = o;
  }
}
static_assert(kWgRow % 4 == 0, "8-byte aligned operand rows");

template <int STRIDE, int TAPS, int TPW>
__global__ void __launch_bounds__(256)
k_conv_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dyp,
             float* __restrict__ partial, float* __restrict__ bias_partial, int64_t chunk, int tpb,
             Geom g) {
  extern __shared__ __align__(16) uint16_t wg_lds[];
  __shared__ int vb[64][4];
  uint16_t* dyT = wg_lds;                   // [co][kWgRow]
  uint16_t* xT = wg_lds + g.co * kWgRow;    // [tpb][ci][kWgRow]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tap0 = blockIdx.y * tpb;
  const int64_t ck = xcd_tile(blockIdx.x, gridDim.x);  // this block's chunk
  const int64_t start = ck * chunk;
  if (start >= g.m_out) return;  // padding workgroup (before any barrier)
  int64_t end = start + chunk;
  if (end > g.m_out) end = g.m_out;
  const int nbi = g.ci / 16, nt = (g.co / 16) * nbi, ntiles = tpb * nt;
  const int cvo = g.co / 8, cvi = g.ci / 8;
  const int row = lane & 15, kq = lane >> 4;
  // the bias gradient of this chunk (sum of dy over its voxels), by the
  // first tap group's blocks, one thread per output channel
  const bool do_bias = bias_partial != nullptr && blockIdx.y == 0 && tid < g.co;
  float bsum = 0.f;
  f4 acc[TPW];
  int aoff[TPW], boff[TPW];  // LDS element offsets of this lane's operands, per tile
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    const int tile = wave + 4 * j;
    const int tl = tile / nt, t2 = tile - tl * nt;
    const int mo = t2 / nbi, ni = t2 - mo * nbi;
    aoff[j] = (mo * 16 + row) * kWgRow + 4 * kq;
    boff[j] = (tl * g.ci + ni * 16 + row) * kWgRow + 4 * kq;
  }
  for (int64_t p0 = start; p0 < end; p0 += 64) {
    __syncthreads();  // the previous step's operands are consumed
    if (tid < 64) {
      const int64_t vox = p0 + tid;
      if (vox < end) {
        int64_t t = vox;
        vb[tid][3] = (int)(t % g.Wo);
        t /= g.Wo;
        vb[tid][2] = (int)(t % g.Ho);
        t /= g.Ho;
        vb[tid][1] = (int)(t % g.Do);
        vb[tid][0] = (int)(t / g.Do);
      } else {
        vb[tid][0] = -1;
      }
    }
    // dy: items of 4 voxels x 8 channels; four 16-byte loads become eight
    // 8-byte LDS rows (one channel, four voxels each)
    for (int e = tid; e < 16 * cvo; e += 256) {
      const int p4 = e / cvo, cv = e - p4 * cvo;
      const int64_t vox = p0 + 4 * p4;
      uint4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        v[k] = vox < end ? *(const uint4*)(dyp + (vox + k) * g.co + cv * 8) : make_uint4(0u, 0u, 0u, 0u);
      store_t4(dyT + (cv * 8) * kWgRow + 4 * p4, v);
    }
    __syncthreads();  // voxel coordinates ready
    // input of each tap of the group, same items (an item's voxels may lie
    // in different grid rows when rows are short)
    for (int e = tid; e < tpb * 16 * cvi; e += 256) {
      const int tl = e / (16 * cvi);
      const int r = e - tl * 16 * cvi;
      const int p4 = r / cvi, cv = r - p4 * cvi;
      int dz, dy, dx;
      tap_offsets(tap0 + tl, TAPS, dz, dy, dx);
      uint4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int* c = vb[4 * p4 + k];
        v[k] = make_uint4(0u, 0u, 0u, 0u);
        if (c[0] >= 0) {
          const int zi = wrapi(STRIDE * c[1] + dz, g.D), yi = wrapi(STRIDE * c[2] + dy, g.H),
                    xi = wrapi(STRIDE * c[3] + dx, g.W);
          v[k] = *(const uint4*)(x + ((((int64_t)c[0] * g.D + zi) * g.H + yi) * g.W + xi) * g.ci + cv * 8);
        }
      }
      store_t4(xT + (tl * g.ci + cv * 8) * kWgRow + 4 * p4, v);
    }
    __syncthreads();
    if (do_bias) {
      const uint16_t* r = dyT + tid * kWgRow;
      for (int p = 0; p < 64; ++p) bsum += bf2f(r[p]);
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      if (wave + 4 * j < ntiles) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const s4 a = *(const s4*)(&dyT[aoff[j] + kk * 16]);
          const s4 bv = *(const s4*)(&xT[boff[j] + kk * 16]);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[j], 0, 0, 0);
        }
      }
    }
  }
  // one row of partials per chunk: the weights, then the bias
  const int64_t row_len = (int64_t)TAPS * g.co * g.ci + g.co;
  if (do_bias) bias_partial[ck * row_len + tid] = bsum;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int tile = wave + 4 * j;
    if (tile < ntiles) {
      const int tl = tile / nt, t2 = tile - tl * nt;
      const int mo = t2 / nbi, ni = t2 - mo * nbi;
      float* out = partial + ck * row_len + (int64_t)(tap0 + tl) * g.co * g.ci;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(mo * 16 + 4 * kq + r) * g.ci + ni * 16 + row] = acc[j][r];
    }
  }
}

// Weight gradient of stride-1 3x3x3 layers with 16, 32 or 64 output channels on
// grids of 16 x 4 x 4 bricks (the LDS forward's tiles).  A workgroup owns a
// range of bricks and one 16-channel input block (grid y); per brick it
// stages the brick's dy, transposed to [channel][voxel], and its 18 x 6 x 6 input halo,
// transposed to [channel][halo row][x] (rows of 24 elements), once for all
// 27 taps.  Each of the nine wavefronts owns one (dz, dy) tap pair and its
// three x taps.  The K dimension of v_mfma_f32_16x16x32_bf16 is 32 voxels
// of two brick rows and a lane's eight voxels are consecutive in x, so the
// input operands of the three x taps come from one 16-byte and one 4-byte
// LDS read, taken at offsets of 0, 1 and 2 elements.  The bias gradient is
// the product of dy with an all-ones operand, one K block per wavefront.
constexpr int kWbRowX = 24;                          // staged halo row (18 used)
constexpr int kWbRows = kLdsHY * kLdsHZ;             // 36 halo rows
constexpr int kWbChan = kWbRows * kWbRowX;           // elements per staged input channel
constexpr int kWbBrick = kLdsTX * kLdsTY * kLdsTZ;   // 256 voxels
constexpr int kWbThreads = 576;                      // nine wavefronts

// Channel j of voxels a and c (eight channels each) as one 4-byte word in
// row j of dst (rows `stride` elements apart).
__device__ __forceinline__ void store_pairs(uint16_t* dst, int stride, const uint4& a, const uint4& c) {
  const uint32_t u[4] = {a.x, a.y, a.z, a.w}, v[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int h = j >> 1, sh = (j & 1) * 16;
    *(uint32_t*)(dst + j * stride) = ((u[h] >> sh) & 0xffffu) | (((v[h] >> sh) & 0xffffu) << 16);
  }
}

__device__ __forceinline__ bf8 as_bf8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  union U { bf8 f; uint32_t i[4]; } r;
  r.i[0] = a; r.i[1] = b; r.i[2] = c; r.i[3] = d;
  return r.f;
}

template <int NCO>
__global__ void __launch_bounds__(kWbThreads)
k_conv_wgrad_brick(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dyp,
                   float* __restrict__ partial, int64_t chunks, int64_t per_chunk, int with_bias,
                   Geom g) {
  __shared__ __align__(16) uint16_t xs[16 * kWbChan];
  __shared__ __align__(16) uint16_t dys[NCO * 16 * kWbBrick];
  __shared__ float bsum[8][NCO * 16];
  constexpr int co = NCO * 16;
  // the wavefront index as a scalar: the bias product below is taken under
  // a test of it, which must be a branch of the whole wavefront (matrix
  // instructions do not honour the lane mask)
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t ck = xcd_tile(blockIdx.x, gridDim.x);
  if (ck >= chunks) return;  // padding workgroup (before any barrier)
  const int tx = g.W / kLdsTX, ty = g.H / kLdsTY, tz = g.D / kLdsTZ;
  const int64_t n_bricks = (int64_t)g.B * tz * ty * tx;
  const int64_t br0 = ck * per_chunk;
  const int64_t br1 = br0 + per_chunk < n_bricks ? br0 + per_chunk : n_bricks;
  const int row = lane & 15, grp = lane >> 4;
  const int dzw = wave / 3, dyw = wave % 3;  // the wavefront's (dz, dy) tap pair, offsets + 1
  const int xo = 8 * (grp & 1);              // first x of the lane's eight voxels
  float* out = partial + ck * ((int64_t)27 * co * g.ci + co);
  const bf8 ones = as_bf8(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);
  f4 bacc[NCO];
#pragma unroll
  for (int mo = 0; mo < NCO; ++mo) bacc[mo] = f4{0.f, 0.f, 0.f, 0.f};
  const int cb = blockIdx.y;  // the input block
  {
    f4 acc[NCO][3];
#pragma unroll
    for (int mo = 0; mo < NCO; ++mo)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[mo][k] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t br = br0; br < br1; ++br) {
      int64_t t = br;
      const int x0 = (int)(t % tx) * kLdsTX;
      t /= tx;
      const int y0 = (int)(t % ty) * kLdsTY;
      t /= ty;
      const int z0 = (int)(t % tz) * kLdsTZ;
      const int b = (int)(t / tz);
      __syncthreads();  // the previous brick's operands are consumed
      // input halo: items of two x neighbours x eight channels
      for (int it = tid; it < kWbRows * 18; it += kWbThreads) {
        const int q = it % 9, h = (it / 9) & 1, r = it / 18;
        const int hy = r % kLdsHY, hz = r / kLdsHY;
        const int gz = wrapi(z0 + hz - 1, g.D), gy = wrapi(y0 + hy - 1, g.H);
        const int64_t rb = (((int64_t)b * g.D + gz) * g.H + gy) * g.W;
        const int gx0 = wrapi(x0 + 2 * q - 1, g.W), gx1 = wrapi(x0 + 2 * q, g.W);
        const uint4 a = *(const uint4*)(x + (rb + gx0) * g.ci + cb * 16 + h * 8);
        const uint4 c = *(const uint4*)(x + (rb + gx1) * g.ci + cb * 16 + h * 8);
        store_pairs(xs + h * 8 * kWbChan + r * kWbRowX + 2 * q, kWbChan, a, c);
      }
      // dy of the brick: rows of 16 voxels, items of two voxels x eight channels
      for (int it = tid; it < 16 * 8 * 2 * NCO; it += kWbThreads) {
        const int q = it % 8, h = (it / 8) % (2 * NCO), r = it / (16 * NCO);
        const int64_t vox = (((int64_t)b * g.D + z0 + r / kLdsTY) * g.H + y0 + r % kLdsTY) * g.W + x0 + 2 * q;
        const uint4 a = *(const uint4*)(dyp + vox * co + h * 8);
        const uint4 c = *(const uint4*)(dyp + (vox + 1) * co + h * 8);
        store_pairs(dys + h * 8 * kWbBrick + r * 16 + 2 * q, kWbBrick, a, c);
      }
      __syncthreads();
#pragma unroll 2
      for (int kb = 0; kb < 8; ++kb) {
        const int r = 2 * kb + (grp >> 1);  // brick row of the lane's voxels
        bf8 av[NCO];
#pragma unroll
        for (int mo = 0; mo < NCO; ++mo) av[mo] = *(const bf8*)(dys + (mo * 16 + row) * kWbBrick + r * 16 + xo);
        const int hr = (r / kLdsTY + dzw) * kLdsHY + r % kLdsTY + dyw;
        const uint16_t* xp = xs + row * kWbChan + hr * kWbRowX + xo;
        const uint4 lo = *(const uint4*)xp;
        const uint32_t hi = *(const uint32_t*)(xp + 8);
        const bf8 bm = as_bf8(lo.x, lo.y, lo.z, lo.w);  // dx = -1
        const bf8 b0 = as_bf8((lo.x >> 16) | (lo.y << 16), (lo.y >> 16) | (lo.z << 16),
                              (lo.z >> 16) | (lo.w << 16), (lo.w >> 16) | (hi << 16));  // dx = 0
        const bf8 bp = as_bf8(lo.y, lo.z, lo.w, hi);    // dx = +1
#pragma unroll
        for (int mo = 0; mo < NCO; ++mo) {
          acc[mo][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mo], bm, acc[mo][0], 0, 0, 0);
          acc[mo][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mo], b0, acc[mo][1], 0, 0, 0);
          acc[mo][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mo], bp, acc[mo][2], 0, 0, 0);
        }
        if (with_bias && cb == 0 && kb == wave) {
#pragma unroll
          for (int mo = 0; mo < NCO; ++mo)
            bacc[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mo], ones, bacc[mo], 0, 0, 0);
        }
      }
    }
    // this input block's columns of the chunk's partial row
#pragma unroll
    for (int mo = 0; mo < NCO; ++mo)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int tap = dzw * 9 + dyw * 3 + k;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          out[((int64_t)tap * co + mo * 16 + 4 * grp + e) * g.ci + cb * 16 + row] = acc[mo][k][e];
      }
  }
  if (with_bias && cb == 0) {
    // every column of the all-ones product holds the sum; column 0, in a
    // fixed order over the eight K blocks
    if (wave < 8 && row == 0) {
#pragma unroll
      for (int mo = 0; mo < NCO; ++mo)
#pragma unroll
        for (int e = 0; e < 4; ++e) bsum[wave][mo * 16 + 4 * grp + e] = bacc[mo][e];
    }
    __syncthreads();
    if (tid < co) {
      float sum = 0.f;
#pragma unroll
      for (int w = 0; w < 8; ++w) sum += bsum[w][tid];
      out[(int64_t)27 * co * g.ci + tid] = sum;
    }
  }
}

// Sum chunk partials in a fixed order, in two passes: segments of kSegLen
// consecutive chunks (grid y = segment), then the segment sums in order.
constexpr int kSegLen = 16;

// Fixed-order sum of the per-chunk partial rows (row stride `stride`, the
// first n columns) over segments of kSegLen chunks.
__global__ void k_sum_segments(const float* __restrict__ partial, float* __restrict__ seg,
                               int64_t n, int64_t stride, int64_t chunks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c0 = (int64_t)blockIdx.y * kSegLen;
  int64_t c1 = c0 + kSegLen;
  if (c1 > chunks) c1 = chunks;
  float s = 0.f;
  for (int64_t c = c0; c < c1; ++c) s += partial[c * stride + i];
  seg[(int64_t)blockIdx.y * n + i] = s;
}

// Sum of the segment rows in order; columns below na go to out_a, the rest
// to out_b (the weight and bias gradients of one call).
__global__ void k_sum_chunks(const float* __restrict__ seg, float* __restrict__ out_a, int64_t na,
                             float* __restrict__ out_b, int64_t n, int64_t segs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int64_t c = 0; c < segs; ++c) s += seg[c * n + i];
  if (i < na) out_a[i] = s;
  else out_b[i - na] = s;
}

// ---- elementwise ----------------------------------------------------------
__global__ void k_lrelu_bwd(const float* __restrict__ dx, const uint16_t* __restrict__ y,
                            uint16_t* __restrict__ d, int64_t n, float slope) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  d[i] = f2bf(bf2f(y[i]) > 0.f ? dx[i] : dx[i] * slope);
}

// The same for eight consecutive elements per thread (16-byte loads and
// stores; n a multiple of 8, n / 8 below 2^31).
__global__ void k_lrelu_bwd8(const float* __restrict__ dx, const uint16_t* __restrict__ y,
                             uint16_t* __restrict__ d, int n8, float slope) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  const f4 g0 = *(const f4*)(dx + 8 * i), g1 = *(const f4*)(dx + 8 * i + 4);
  const uint4 yv = *(const uint4*)(y + 8 * i);
  const float g[8] = {g0[0], g0[1], g0[2], g0[3], g1[0], g1[1], g1[2], g1[3]};
  const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
  uint32_t o[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const float a = bf2f((uint16_t)(yw[h] & 0xffffu)) > 0.f ? g[2 * h] : g[2 * h] * slope;
    const float c = bf2f((uint16_t)(yw[h] >> 16)) > 0.f ? g[2 * h + 1] : g[2 * h + 1] * slope;
    o[h] = (uint32_t)f2bf(a) | ((uint32_t)f2bf(c) << 16);
  }
  *(uint4*)(d + 8 * i) = make_uint4(o[0], o[1], o[2], o[3]);
}

// Index arithmetic of the element-wise kernels below runs in I: 32-bit when
// the element count allows it (64-bit division is a long instruction
// sequence on the GPU and dominated these memory-bound kernels).
template <typename I>
__global__ void k_up_concat(const uint16_t* __restrict__ coarse, const uint16_t* __restrict__ skip,
                            uint16_t* __restrict__ cat, I nvox, I d, I h, I w, I c1, I c2) {
  const I e = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
  const I ct = c1 + c2;
  if (e >= nvox * ct) return;
  const I v = e / ct;
  const I c = e - v * ct;
  if (c < c1) {
    I t = v;
    const I xx = t % w;
    t /= w;
    const I yy = t % h;
    t /= h;
    const I zz = t % d;
    const I b = t / d;
    const I cv = ((b * (d / 2) + zz / 2) * (h / 2) + yy / 2) * (w / 2) + xx / 2;
    cat[e] = coarse[cv * c1 + c];
  } else {
    cat[e] = skip[v * c2 + (c - c1)];
  }
}

// The same with 8 channels (16 bytes) per thread, for channel counts that
// are multiples of 8.
template <typename I>
__global__ void k_up_concat8(const uint16_t* __restrict__ coarse, const uint16_t* __restrict__ skip,
                             uint16_t* __restrict__ cat, I nvox, I d, I h, I w, I c1, I c2) {
  const I e = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
  const I g1 = c1 / 8, gt = (c1 + c2) / 8;
  if (e >= nvox * gt) return;
  const I v = e / gt;
  const I gi = e - v * gt;
  uint4 val;
  if (gi < g1) {
    I t = v;
    const I xx = t % w;
    t /= w;
    const I yy = t % h;
    t /= h;
    const I zz = t % d;
    const I b = t / d;
    const I cv = ((b * (d / 2) + zz / 2) * (h / 2) + yy / 2) * (w / 2) + xx / 2;
    val = *(const uint4*)(coarse + cv * c1 + gi * 8);
  } else {
    val = *(const uint4*)(skip + v * c2 + (gi - g1) * 8);
  }
  *(uint4*)(cat + v * (c1 + c2) + gi * 8) = val;
}

template <typename I>
__global__ void k_split_down_coarse(const float* __restrict__ dcat, float* __restrict__ dcoarse,
                                    I ncoarse, I d, I h, I w, I c1, I c2) {
  const I e = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
  if (e >= ncoarse * c1) return;
  const I v = e / c1;
  const I c = e - v * c1;
  const I dc = d / 2, hc = h / 2, wc = w / 2;
  I t = v;
  const I xc = t % wc;
  t /= wc;
  const I yc = t % hc;
  t /= hc;
  const I zc = t % dc;
  const I b = t / dc;
  float s = 0.f;
  for (int k = 0; k < 8; ++k) {
    const I zz = 2 * zc + (k >> 2), yy = 2 * yc + ((k >> 1) & 1), xx = 2 * xc + (k & 1);
    const I fv = ((b * d + zz) * h + yy) * w + xx;
    s += dcat[fv * (c1 + c2) + c];
  }
  dcoarse[e] = s;
}

template <typename I>
__global__ void k_split_down_skip(const float* __restrict__ dcat, float* __restrict__ dskip,
                                  I nfine, I c1, I c2) {
  const I e = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
  if (e >= nfine * c2) return;
  const I v = e / c2;
  const I c = e - v * c2;
  dskip[e] = dcat[v * (c1 + c2) + c1 + c];
}

// Masked MSE: partial (sum of squared errors, fluid count) per block, then
// one block combines them in order; the gradient kernel reads the count.
__global__ void __launch_bounds__(256)
k_mse_partial(const float* __restrict__ pred, const float* __restrict__ tgt,
              const uint8_t* __restrict__ mask, int64_t n, float* __restrict__ partial) {
  __shared__ float s_err[256];
  __shared__ float s_cnt[256];
  float e = 0.f, cnt = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (mask[i] == 0) {
      for (int a = 0; a < 3; ++a) {
        const float d = pred[i * 3 + a] - tgt[i * 3 + a];
        e += d * d;
      }
      cnt += 1.f;
    }
  }
  s_err[threadIdx.x] = e;
  s_cnt[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_err[threadIdx.x] += s_err[threadIdx.x + off];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s_err[0];
    partial[2 * blockIdx.x + 1] = s_cnt[0];
  }
}

// One block: strided per-thread sums, then a fixed-order tree in LDS.
__global__ void __launch_bounds__(256)
k_mse_final(const float* __restrict__ partial, int nblocks, float* __restrict__ loss,
            float* __restrict__ count) {
  __shared__ float se[256], sc[256];
  const int t = threadIdx.x;
  float e = 0.f, c = 0.f;
  for (int b = t; b < nblocks; b += 256) {
    e += partial[2 * b];
    c += partial[2 * b + 1];
  }
  se[t] = e;
  sc[t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      se[t] += se[t + w];
      sc[t] += sc[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    *count = sc[0];
    *loss = sc[0] > 0.f ? se[0] / (3.f * sc[0]) : 0.f;
  }
}

__global__ void k_mse_grad(const float* __restrict__ pred, const float* __restrict__ tgt,
                           const uint8_t* __restrict__ mask, int64_t n,
                           const float* __restrict__ count, uint16_t* __restrict__ dy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * 16) return;
  const int64_t i = e >> 4;
  const int c = (int)(e & 15);
  float gval = 0.f;
  if (c < 3 && mask[i] == 0) gval = 2.f * (pred[i * 3 + c] - tgt[i * 3 + c]) / (3.f * *count);
  dy[e] = f2bf(gval);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, int64_t n, float lr,
                       float b1, float a1, float b2, float a2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + a1 * g;
  const float vi = b2 * v[i] + a2 * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

template <typename I>
__global__ void k_prepare_input(const uint8_t* __restrict__ mask, uint16_t* __restrict__ x, I n,
                                I cpad) {
  const I e = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
  if (e >= n * cpad) return;
  const I i = e / cpad;
  const I c = e - i * cpad;
  const bool solid = mask[i] != 0;
  float v = 0.f;
  if (c == 0) v = solid ? 1.f : 0.f;
  if (c == 1) v = solid ? 0.f : 1.f;
  x[e] = f2bf(v);
}

// Distance to the nearest solid voxel: a chamfer distance on the
// 26-neighbourhood (steps of 1, sqrt 2 and sqrt 3), on periodic cubes of
// edge n, relaxed from 0 on solids and dmax on fluid; one sweep moves the
// front by one voxel, so after ceil(dmax) sweeps every distance below dmax
// has its final value.
// One sweep, as a thread per (x, y) column and run of RUN planes in z
// (consecutive lanes take consecutive x, so every load is coalesced): the
// thread keeps the 3 x 3 source values around its column in the planes
// z - 1, z and z + 1 in registers and slides them along z, loading nine new
// values per voxel instead of 26.  Indices are 32-bit (the caller checks
// that the cubes hold fewer than 2^31 voxels).
template <int RUN>
__global__ void k_dist_relax(const uint8_t* __restrict__ mask, const float* __restrict__ src,
                             float* __restrict__ dst, int n, int n_threads, float dmax) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_threads) return;
  const int x = t % n;
  int r = t / n;
  const int y = r % n;
  r /= n;
  const int runs = n / RUN;
  const int z0 = (r % runs) * RUN;
  const int cube = (r / runs) * n * n * n;
  const int n2 = n * n;
  auto wrap = [n](int v) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  // in-plane offsets of the 3 x 3 neighbourhood, j = 3 * (dy + 1) + dx + 1
  int off[9];
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) off[3 * (dy + 1) + dx + 1] = wrap(y + dy) * n + wrap(x + dx);
  // step length to the neighbour at (dx, dy, dz)
  auto step = [](int dx, int dy, int dz) {
    const int k = dx * dx + dy * dy + dz * dz;
    return k == 1 ? 1.f : (k == 2 ? 1.41421356f : 1.73205081f);
  };
  float pm[9], pc[9], pp[9];
  {
    const int bm = cube + wrap(z0 - 1) * n2, bc = cube + z0 * n2, bp = cube + wrap(z0 + 1) * n2;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      pm[j] = src[bm + off[j]];
      pc[j] = src[bc + off[j]];
      pp[j] = src[bp + off[j]];
    }
  }
#pragma unroll
  for (int i = 0; i < RUN; ++i) {
    const int e = cube + (z0 + i) * n2 + off[4];
    float best = pc[4];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int j = 3 * (dy + 1) + dx + 1;
        best = fminf(best, pm[j] + step(dx, dy, -1));
        if (j != 4) best = fminf(best, pc[j] + step(dx, dy, 0));
        best = fminf(best, pp[j] + step(dx, dy, 1));
      }
    dst[e] = mask[e] != 0 ? 0.f : fminf(best, dmax);
    if (i + 1 < RUN) {
      const int bn = cube + wrap(z0 + i + 2) * n2;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        pm[j] = pc[j];
        pc[j] = pp[j];
        pp[j] = src[bn + off[j]];
      }
    }
  }
}

__global__ void k_dist_init(const uint8_t* __restrict__ mask, float* __restrict__ d, int64_t total,
                            float dmax) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) d[e] = mask[e] != 0 ? 0.f : dmax;
}

// Input channels: 0 solid, 1 fluid, 2 d/dmax, 3 (d/dmax)^2, the rest zero.
// One thread per voxel and group of 8 channels (one 16-byte store), for
// channel counts that are multiples of 8.
__global__ void k_features8(const uint8_t* __restrict__ mask, const float* __restrict__ dist,
                            uint16_t* __restrict__ x, int64_t total, int cpad, float dmax) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int groups = cpad / 8;
  if (e >= total * groups) return;
  const int64_t i = e / groups;
  const int g = (int)(e - i * groups);
  uint4 v = {0u, 0u, 0u, 0u};
  if (g == 0) {
    const bool solid = mask[i] != 0;
    const float q = dist[i] / dmax;
    v.x = (uint32_t)f2bf(solid ? 1.f : 0.f) | ((uint32_t)f2bf(solid ? 0.f : 1.f) << 16);
    v.y = (uint32_t)f2bf(q) | ((uint32_t)f2bf(q * q) << 16);
  }
  *(uint4*)(x + i * cpad + 8 * g) = v;
}

__global__ void k_features(const uint8_t* __restrict__ mask, const float* __restrict__ dist,
                           uint16_t* __restrict__ x, int64_t total, int cpad, float dmax) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total * cpad) return;
  const int64_t i = e / cpad;
  const int c = (int)(e - i * cpad);
  const bool solid = mask[i] != 0;
  const float q = dist[i] / dmax;
  float v = 0.f;
  if (c == 0) v = solid ? 1.f : 0.f;
  if (c == 1) v = solid ? 0.f : 1.f;
  if (c == 2) v = q;
  if (c == 3) v = q * q;
  x[e] = f2bf(v);
}

// Network labels from solver velocities: out[i][a] = scale * u[a*n + i] on
// fluid voxels, 0 on solids (the inverse of k_velocity_out).
__global__ void k_velocity_labels(const double* __restrict__ u, const uint8_t* __restrict__ mask,
                                  double scale, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool solid = mask[i] != 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[i * 3 + a] = solid ? 0.f : (float)(scale * u[a * n + i]);
}

__global__ void k_velocity_out(const float* __restrict__ pred, const uint8_t* __restrict__ mask,
                               double scale, double* __restrict__ u, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool solid = mask[i] != 0;
  for (int a = 0; a < 3; ++a) u[a * n + i] = solid ? 0.0 : scale * (double)pred[i * 3 + a];
}

__global__ void k_to_bf16(const float* __restrict__ s, uint16_t* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = f2bf(s[i]);
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline unsigned pad_xcd(unsigned n) { return (n + kXcds - 1) / kXcds * kXcds; }

static int check_desc(const nn_conv_desc* d) {
  if (!d) { set_error("descriptor is NULL"); return -1; }
  if (d->batch < 1 || d->d < 1 || d->h < 1 || d->w < 1) { set_error("bad grid"); return -1; }
  if (d->c_in < 16 || d->c_in % 16 || d->c_in > 128) { set_error("c_in must be a multiple of 16 in [16,128]"); return -1; }
  if (d->c_out < 16 || d->c_out % 16 || d->c_out > 128) { set_error("c_out must be a multiple of 16 in [16,128]"); return -1; }
  if (d->taps != 27 && d->taps != 1) { set_error("taps must be 27 or 1"); return -1; }
  if (d->stride != 1 && d->stride != 2) { set_error("stride must be 1 or 2"); return -1; }
  if (d->stride == 2 && (d->taps != 27 || d->d % 2 || d->h % 2 || d->w % 2)) {
    set_error("stride 2 needs 3x3x3 taps and even grid sizes");
    return -1;
  }
  const int64_t m_in = (int64_t)d->batch * d->d * d->h * d->w;
  if (m_in >= 0x7fffffffLL) { set_error("more than 2^31 voxels"); return -1; }
  if (m_in % (16 * d->stride * d->stride * d->stride)) {
    set_error("voxel counts of the input and output grids must be multiples of 16");
    return -1;
  }
  if (d->c_store < 1 || d->c_store > d->c_out) { set_error("bad c_store"); return -1; }
  if ((d->c_out / 16) * (d->c_in / 16) > 32) { set_error("c_out*c_in exceeds 32 tiles of 16x16"); return -1; }
  return 0;
}

static Geom make_geom(const nn_conv_desc* d) {
  Geom g;
  g.B = d->batch;
  g.D = d->d;
  g.H = d->h;
  g.W = d->w;
  g.Do = d->d / d->stride;
  g.Ho = d->h / d->stride;
  g.Wo = d->w / d->stride;
  g.ci = d->c_in;
  g.co = d->c_out;
  g.cstore = d->c_store;
  g.act = d->act;
  g.slope = d->slope;
  g.m_out = (int64_t)g.B * g.Do * g.Ho * g.Wo;
  g.m_in = (int64_t)g.B * g.D * g.H * g.W;
  return g;
}

// Tap group and tiles per wave of the weight-gradient launch: the largest
// group (27, 9, 3 or 1 taps) whose tiles fit 14 per wave and whose staged
// operands fit 64 KiB of LDS.
static void wgrad_plan(const nn_conv_desc* d, int* tpb, int* tpw, size_t* lds) {
  const int nt = (d->c_out / 16) * (d->c_in / 16);
  const int cands[4] = {27, 9, 3, 1};
  int best = 1;
  for (int k = 0; k < 4; ++k) {
    const int t = cands[k];
    if (d->taps % t) continue;
    const size_t bytes = (size_t)(d->c_out + t * d->c_in) * kWgRow * 2;
    if (t * nt <= 56 && bytes <= 65536) { best = t; break; }
  }
  *tpb = best;
  *tpw = (best * nt + 3) / 4;
  *lds = (size_t)(d->c_out + best * d->c_in) * kWgRow * 2;
}

// Voxel chunks of the weight gradient (a multiple of 64 voxels each): about
// 1024 blocks over chunks and tap groups, with the per-chunk partials
// (taps x co x ci floats each) kept under 32 MiB.
static int64_t wgrad_chunk(const nn_conv_desc* d, const Geom& g, int64_t* chunks) {
  int tpb, tpw;
  size_t lds;
  wgrad_plan(d, &tpb, &tpw, &lds);
  const int groups = d->taps / tpb;
  int64_t c = (1024 + groups - 1) / groups;
  const int64_t per_chunk_bytes = (int64_t)d->taps * d->c_out * d->c_in * 4;
  const int64_t cap = (int64_t)32 * 1024 * 1024 / per_chunk_bytes;
  if (c > cap) c = cap;
  if (c > (g.m_out + 63) / 64) c = (g.m_out + 63) / 64;
  if (c < 1) c = 1;
  int64_t per = (g.m_out + c - 1) / c;
  per = (per + 63) / 64 * 64;
  *chunks = (g.m_out + per - 1) / per;
  return per;
}

// Tiles per wavefront: four while that still leaves about 4096 waves.
static int pick_mt(int64_t m) { return m >= 4 * 16 * 4096 ? 4 : (m >= 2 * 16 * 4096 ? 2 : 1); }

template <int STRIDE, int TAPS, bool F32, int MT>
static void launch_fwd_mt(int nb, const uint16_t* x, const uint16_t* w, const float* bias, void* y,
                          const Geom& g, hipStream_t s) {
  // grids with fewer than 4096 wavefronts split the output channels
  int nsplit = 1;
  while (nsplit < nb && nb % (2 * nsplit) == 0 && (int64_t)nblk(g.m_out / 16, MT) * nsplit < 4096)
    nsplit *= 2;
  const int nbw = nb / nsplit;
  const int64_t tiles = nblk(g.m_out / 16, MT);
  const dim3 grid(pad_xcd(nblk(tiles * nsplit, 4))), block(256);
  // stride 1 with rows of whole tiles: the x taps share one fragment
  const bool xs = STRIDE == 1 && TAPS == 27 && g.Wo % 16 == 0;
  switch (nbw) {
#define CASE(N)                                                                                  \
  case N:                                                                                        \
    if (xs)                                                                                      \
      hipLaunchKernelGGL((k_conv_fwd<STRIDE, TAPS, N, F32, MT, true>), grid, block, 0, s, x, w,  \
                         bias, y, nsplit, g);                                                    \
    else                                                                                         \
      hipLaunchKernelGGL((k_conv_fwd<STRIDE, TAPS, N, F32, MT, false>), grid, block, 0, s, x, w, \
                         bias, y, nsplit, g);                                                    \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
  }
}

template <int STRIDE, int TAPS, bool F32>
static void launch_fwd_nb(int nb, const uint16_t* x, const uint16_t* w, const float* bias, void* y,
                          const Geom& g, hipStream_t s) {
  switch (pick_mt(g.m_out)) {
    case 4: launch_fwd_mt<STRIDE, TAPS, F32, 4>(nb, x, w, bias, y, g, s); break;
    case 2: launch_fwd_mt<STRIDE, TAPS, F32, 2>(nb, x, w, bias, y, g, s); break;
    default: launch_fwd_mt<STRIDE, TAPS, F32, 1>(nb, x, w, bias, y, g, s); break;
  }
}

// The LDS forward for stride-1 3x3x3 layers on grids it tiles; false if
// the layer does not qualify (then the per-wavefront kernel runs).
template <bool F32, bool ACC = false>
static bool launch_fwd_lds(int nb, const uint16_t* x, const uint16_t* xc, int c1, const uint16_t* w,
                           const float* bias, void* y, const Geom& g, hipStream_t s) {
  if (g.W % kLdsTX || g.H % kLdsTY || g.D % kLdsTZ) return false;
  const int64_t n_tiles = (int64_t)g.B * (g.D / kLdsTZ) * (g.H / kLdsTY) * (g.W / kLdsTX);
  // output blocks per workgroup: the most (4, 2 or 1) that divides nb and
  // still gives kLdsMinGroups workgroups, else 1
  int per = 1;
  for (int c = 4; c > 1; c /= 2)
    if (nb % c == 0 && n_tiles * (nb / c) >= kLdsMinGroups) { per = c; break; }
  const int parts = nb / per;
  const dim3 grid(pad_xcd((unsigned)(n_tiles * parts))), block(256);
  // LDS for the widest chunk of this layer (16-channel layers stage 24
  // elements per voxel, which lets more workgroups share a compute unit)
  const size_t lds = (size_t)kLdsHalo * ((g.ci < kLdsChunk ? g.ci : kLdsChunk) + kLdsPad) * 2;
  switch (per) {
    case 1: hipLaunchKernelGGL((k_conv_fwd_lds<1, F32, ACC>), grid, block, lds, s, x, xc, c1, w, bias, y, n_tiles, parts, g); break;
    case 2: hipLaunchKernelGGL((k_conv_fwd_lds<2, F32, ACC>), grid, block, lds, s, x, xc, c1, w, bias, y, n_tiles, parts, g); break;
    default: hipLaunchKernelGGL((k_conv_fwd_lds<4, F32, ACC>), grid, block, lds, s, x, xc, c1, w, bias, y, n_tiles, parts, g); break;
  }
  return true;
}

// The LDS stride-2 forward; false if the layer's output grid does not tile.
template <bool F32>
static bool launch_fwd_lds_s2(int nb, const uint16_t* x, const uint16_t* w, const float* bias, void* y,
                              const Geom& g, hipStream_t s) {
  if (g.Wo % kS2TX || g.Ho % kS2TY || g.Do % kS2TZ) return false;
  const int64_t n_tiles = (int64_t)g.B * (g.Do / kS2TZ) * (g.Ho / kS2TY) * (g.Wo / kS2TX);
  int per = 1;
  for (int c = 4; c > 1; c /= 2)
    if (nb % c == 0 && n_tiles * (nb / c) >= kLdsMinGroups) { per = c; break; }
  const int parts = nb / per;
  const dim3 grid(pad_xcd((unsigned)(n_tiles * parts))), block(256);
  const size_t lds = (size_t)kS2Halo * kS2VS * 2;
  switch (per) {
    case 1: hipLaunchKernelGGL((k_conv_fwd_lds_s2<1, F32>), grid, block, lds, s, x, w, bias, y, n_tiles, parts, g); break;
    case 2: hipLaunchKernelGGL((k_conv_fwd_lds_s2<2, F32>), grid, block, lds, s, x, w, bias, y, n_tiles, parts, g); break;
    default: hipLaunchKernelGGL((k_conv_fwd_lds_s2<4, F32>), grid, block, lds, s, x, w, bias, y, n_tiles, parts, g); break;
  }
  return true;
}

template <int STRIDE, int TAPS, int MT, bool PAR>
static void launch_dgrad_mt(int nb, const uint16_t* dy, const uint16_t* wt, float* dx, int acc,
                            const Geom& g, hipStream_t s) {
  // grids with fewer than 4096 wavefronts split the output blocks
  int nsplit = 1;
  while (nsplit < nb && nb % (2 * nsplit) == 0 && (int64_t)nblk(g.m_in / 16, MT) * nsplit < 4096)
    nsplit *= 2;
  const dim3 grid(pad_xcd(nblk(nblk(g.m_in / 16, MT) * nsplit, 4))), block(256);
  switch (nb / nsplit) {
#define CASE(N)                                                                                   \
  case N:                                                                                         \
    hipLaunchKernelGGL((k_conv_dgrad<STRIDE, TAPS, N, MT, PAR>), grid, block, 0, s, dy, wt, dx, acc, \
                       nsplit, g);                                                                \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
  }
}

template <int STRIDE, int TAPS>
static void launch_dgrad_nb(int nb, const uint16_t* dy, const uint16_t* wt, float* dx, int acc,
                            const Geom& g, hipStream_t s) {
  // stride 2 on rows of whole 32-voxel blocks: tiles of one parity class
  constexpr bool kPar = STRIDE == 2 && TAPS == 27;
  if (kPar && g.W % 32 == 0) {
    switch (pick_mt(g.m_in)) {
      case 4: launch_dgrad_mt<STRIDE, TAPS, 4, kPar>(nb, dy, wt, dx, acc, g, s); break;
      case 2: launch_dgrad_mt<STRIDE, TAPS, 2, kPar>(nb, dy, wt, dx, acc, g, s); break;
      default: launch_dgrad_mt<STRIDE, TAPS, 1, kPar>(nb, dy, wt, dx, acc, g, s); break;
    }
    return;
  }
  switch (pick_mt(g.m_in)) {
    case 4: launch_dgrad_mt<STRIDE, TAPS, 4, false>(nb, dy, wt, dx, acc, g, s); break;
    case 2: launch_dgrad_mt<STRIDE, TAPS, 2, false>(nb, dy, wt, dx, acc, g, s); break;
    default: launch_dgrad_mt<STRIDE, TAPS, 1, false>(nb, dy, wt, dx, acc, g, s); break;
  }
}

template <int STRIDE, int TAPS>
static void launch_wgrad_tpw(int tpw, int tpb, size_t lds, const uint16_t* x, const uint16_t* dy,
                             float* partial, float* bias_partial, int64_t chunk, int64_t chunks,
                             const Geom& g, hipStream_t s) {
  const dim3 grid(pad_xcd((unsigned)chunks), TAPS / tpb), block(256);
  const int t = tpw <= 2 ? 2 : (tpw <= 4 ? 4 : (tpw <= 8 ? 8 : 14));
  switch (t) {
#define CASE(N)                                                                                   \
  case N:                                                                                         \
    hipLaunchKernelGGL((k_conv_wgrad<STRIDE, TAPS, N>), grid, block, lds, s, x, dy, partial,       \
                       bias_partial, chunk, tpb, g);                                              \
    break;
    CASE(2) CASE(4) CASE(8) CASE(14)
#undef CASE
  }
}

}  // namespace nn
}  // namespace lbm

using namespace lbm::nn;
using lbm::set_error;

#define NN_HIP_CHECK(what)                                                    \
  do {                                                                        \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess) {                                                   \
      set_error("%s: %s", what, hipGetErrorString(e_));                       \
      return -4;                                                              \
    }                                                                         \
  } while (0)

extern "C" {

int nn_conv3d_fwd(const nn_conv_desc* d, const uint16_t* x, const uint16_t* w, const float* bias,
                  void* y, void* stream) {
  if (check_desc(d)) return -1;
  if (!x || !w || !y) { set_error("null tensor"); return -1; }
  const Geom g = make_geom(d);
  hipStream_t s = (hipStream_t)stream;
  const int nb = d->c_out / 16;
  if (d->taps == 27 && d->stride == 1 &&
      (d->out_f32 ? launch_fwd_lds<true>(nb, x, nullptr, 0, w, bias, y, g, s)
                  : launch_fwd_lds<false>(nb, x, nullptr, 0, w, bias, y, g, s))) {
    NN_HIP_CHECK("conv fwd");
    return 0;
  }
  if (d->taps == 27 && d->stride == 2 &&
      (d->out_f32 ? launch_fwd_lds_s2<true>(nb, x, w, bias, y, g, s)
                  : launch_fwd_lds_s2<false>(nb, x, w, bias, y, g, s))) {
    NN_HIP_CHECK("conv fwd");
    return 0;
  }
  if (d->taps == 1 && d->stride == 1 && d->out_f32 && d->c_store <= 4 &&
      (d->c_in == 16 || d->c_in == 32) && ((uintptr_t)x & 15) == 0) {
    const dim3 grid(nblk(g.m_out, 256)), block(256);
    if (d->c_in == 16)
      hipLaunchKernelGGL(k_conv1x1_few<16>, grid, block, 0, s, x, w, bias, (float*)y, g.m_out, d->c_store,
                         d->act, d->slope);
    else
      hipLaunchKernelGGL(k_conv1x1_few<32>, grid, block, 0, s, x, w, bias, (float*)y, g.m_out, d->c_store,
                         d->act, d->slope);
    NN_HIP_CHECK("conv fwd 1x1");
    return 0;
  }
  if (d->taps == 1) {
    if (d->stride != 1) { set_error("1x1x1 convolution has stride 1"); return -1; }
    if (d->out_f32) launch_fwd_nb<1, 1, true>(nb, x, w, bias, y, g, s);
    else launch_fwd_nb<1, 1, false>(nb, x, w, bias, y, g, s);
  } else if (d->stride == 1) {
    if (d->out_f32) launch_fwd_nb<1, 27, true>(nb, x, w, bias, y, g, s);
    else launch_fwd_nb<1, 27, false>(nb, x, w, bias, y, g, s);
  } else {
    if (d->out_f32) launch_fwd_nb<2, 27, true>(nb, x, w, bias, y, g, s);
    else launch_fwd_nb<2, 27, false>(nb, x, w, bias, y, g, s);
  }
  NN_HIP_CHECK("conv fwd");
  return 0;
}

int nn_conv3d_fwd_upcat(const nn_conv_desc* d, const uint16_t* coarse, int32_t c_coarse,
                        const uint16_t* skip, const uint16_t* w, const float* bias, void* y, void* stream) {
  if (check_desc(d)) return -1;
  if (!coarse || !skip || !w || !y) { set_error("null tensor"); return -1; }
  if (d->stride != 1 || d->taps != 27) { set_error("the fused up-sample/concat needs a stride-1 3x3x3 layer"); return -1; }
  if (c_coarse < 8 || c_coarse % 8 || c_coarse >= d->c_in) {
    set_error("c_coarse must be a multiple of 8 below c_in");
    return -1;
  }
  if (d->d % 2 || d->h % 2 || d->w % 2) { set_error("the fine grid must have even sizes"); return -1; }
  const Geom g = make_geom(d);
  hipStream_t s = (hipStream_t)stream;
  const int nb = d->c_out / 16;
  const bool ok = d->out_f32 ? launch_fwd_lds<true>(nb, skip, coarse, c_coarse, w, bias, y, g, s)
                             : launch_fwd_lds<false>(nb, skip, coarse, c_coarse, w, bias, y, g, s);
  if (!ok) {
    set_error("the fused up-sample/concat needs w %% 16, h %% 4 and d %% 4 == 0");
    return -1;
  }
  NN_HIP_CHECK("conv fwd upcat");
  return 0;
}

int nn_conv3d_dgrad(const nn_conv_desc* d, const uint16_t* dy, const uint16_t* w, uint16_t* w_t,
                    float* dx, int32_t accumulate, void* stream) {
  if (check_desc(d)) return -1;
  if (!dy || !w || !w_t || !dx) { set_error("null tensor"); return -1; }
  const Geom g = make_geom(d);
  hipStream_t s = (hipStream_t)stream;
  const int64_t nw = (int64_t)d->taps * d->c_out * d->c_in;
  // stride-1 3x3x3 layers on grids the LDS forward tiles: dx is the forward
  // convolution of dy (c_out channels in, c_in out, no bias or activation)
  // with the mirrored, transposed weights, added to dx when accumulating
  const bool lds = d->taps == 27 && d->stride == 1 && g.W % kLdsTX == 0 && g.H % kLdsTY == 0 &&
                   g.D % kLdsTZ == 0 && ((uintptr_t)dy & 15) == 0 && ((uintptr_t)w_t & 15) == 0;
  hipLaunchKernelGGL(k_transpose_w, dim3(nblk(nw, 256)), dim3(256), 0, s, w, w_t, d->taps, d->c_out,
                     d->c_in, lds ? 1 : 0);
  if (lds) {
    Geom gt = g;
    gt.ci = g.co;
    gt.co = g.ci;
    gt.cstore = g.ci;
    gt.act = 0;
    if (accumulate) launch_fwd_lds<true, true>(d->c_in / 16, dy, nullptr, 0, w_t, nullptr, dx, gt, s);
    else launch_fwd_lds<true, false>(d->c_in / 16, dy, nullptr, 0, w_t, nullptr, dx, gt, s);
    NN_HIP_CHECK("conv dgrad");
    return 0;
  }
  const int nb = d->c_in / 16;
  if (d->taps == 1) launch_dgrad_nb<1, 1>(nb, dy, w_t, dx, accumulate, g, s);
  else if (d->stride == 1) launch_dgrad_nb<1, 27>(nb, dy, w_t, dx, accumulate, g, s);
  else launch_dgrad_nb<2, 27>(nb, dy, w_t, dx, accumulate, g, s);
  NN_HIP_CHECK("conv dgrad");
  return 0;
}

int64_t nn_conv3d_wgrad_workspace(const nn_conv_desc* d) {
  if (check_desc(d)) return -1;
  const Geom g = make_geom(d);
  int64_t chunks;
  wgrad_chunk(d, g, &chunks);
  const int64_t segs = (chunks + kSegLen - 1) / kSegLen;
  return ((chunks + segs) * d->taps * d->c_out * d->c_in + (chunks + segs) * d->c_out) *
         (int64_t)sizeof(float);
}

int nn_conv3d_wgrad(const nn_conv_desc* d, const uint16_t* x, const uint16_t* dy, float* dw,
                    float* db, float* workspace, void* stream) {
  if (check_desc(d)) return -1;
  if (!x || !dy || !dw || !workspace) { set_error("null tensor"); return -1; }
  const Geom g = make_geom(d);
  hipStream_t s = (hipStream_t)stream;
  int64_t chunks;
  const int64_t chunk = wgrad_chunk(d, g, &chunks);
  const int64_t nw = (int64_t)d->taps * d->c_out * d->c_in;
  const int64_t segs = (chunks + kSegLen - 1) / kSegLen;
  // workspace: [chunks][nw + c_out] partial rows (weights, then bias), then
  // [segs][n] segment sums of the n columns wanted; one pair of summing
  // launches covers both gradients
  const int64_t row = nw + d->c_out;
  const int64_t n = db ? row : nw;
  float* seg = workspace + chunks * row;
  int tpb, tpw;
  size_t lds;
  wgrad_plan(d, &tpb, &tpw, &lds);
  float* bp = db ? workspace + nw : nullptr;
  const bool brick = d->taps == 27 && d->stride == 1 && (d->c_out == 16 || d->c_out == 32 || d->c_out == 64) &&
                     g.W % kLdsTX == 0 && g.H % kLdsTY == 0 && g.D % kLdsTZ == 0 &&
                     ((uintptr_t)x & 15) == 0 && ((uintptr_t)dy & 15) == 0;
  if (brick) {
    const int64_t n_bricks = g.m_out / kWbBrick;
    const int64_t per = (n_bricks + chunks - 1) / chunks;
    const dim3 grid(pad_xcd((unsigned)chunks), d->c_in / 16), block(kWbThreads);
    if (d->c_out == 16)
      hipLaunchKernelGGL(k_conv_wgrad_brick<1>, grid, block, 0, s, x, dy, workspace, chunks, per, db ? 1 : 0, g);
    else if (d->c_out == 32)
      hipLaunchKernelGGL(k_conv_wgrad_brick<2>, grid, block, 0, s, x, dy, workspace, chunks, per, db ? 1 : 0, g);
    else
      hipLaunchKernelGGL(k_conv_wgrad_brick<4>, grid, block, 0, s, x, dy, workspace, chunks, per, db ? 1 : 0, g);
  } else if (d->taps == 1) launch_wgrad_tpw<1, 1>(tpw, tpb, lds, x, dy, workspace, bp, chunk, chunks, g, s);
  else if (d->stride == 1) launch_wgrad_tpw<1, 27>(tpw, tpb, lds, x, dy, workspace, bp, chunk, chunks, g, s);
  else launch_wgrad_tpw<2, 27>(tpw, tpb, lds, x, dy, workspace, bp, chunk, chunks, g, s);
  hipLaunchKernelGGL(k_sum_segments, dim3(nblk(n, 256), (unsigned)segs), dim3(256), 0, s, workspace,
                     seg, n, row, chunks);
  hipLaunchKernelGGL(k_sum_chunks, dim3(nblk(n, 256)), dim3(256), 0, s, seg, dw, nw, db, n, segs);
  NN_HIP_CHECK("conv wgrad");
  return 0;
}

int nn_lrelu_bwd(const float* dx, const uint16_t* y, uint16_t* dy_pre, int64_t n, float slope,
                 void* stream) {
  if (!dx || !y || !dy_pre || n < 0) { set_error("bad arguments"); return -1; }
  if (n == 0) return 0;
  if (n % 8 == 0 && n / 8 < 0x7fffffffLL && ((uintptr_t)dx & 15) == 0 && ((uintptr_t)y & 15) == 0 &&
      ((uintptr_t)dy_pre & 15) == 0)
    hipLaunchKernelGGL(k_lrelu_bwd8, dim3(nblk(n / 8, 256)), dim3(256), 0, (hipStream_t)stream, dx, y,
                       dy_pre, (int)(n / 8), slope);
  else
    hipLaunchKernelGGL(k_lrelu_bwd, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, dx, y,
                       dy_pre, n, slope);
  NN_HIP_CHECK("lrelu bwd");
  return 0;
}

int nn_up_concat(const uint16_t* coarse, const uint16_t* skip, uint16_t* cat, int32_t batch,
                 int32_t d, int32_t h, int32_t w, int32_t c1, int32_t c2, void* stream) {
  if (!coarse || !skip || !cat || batch < 1 || d % 2 || h % 2 || w % 2 || c1 < 1 || c2 < 1) {
    set_error("bad arguments");
    return -1;
  }
  const int64_t nvox = (int64_t)batch * d * h * w;
  const bool small = nvox * (c1 + c2) < ((int64_t)1 << 31);
  if (c1 % 8 == 0 && c2 % 8 == 0) {
    const dim3 grid(nblk(nvox * ((c1 + c2) / 8), 256));
    if (small)
      hipLaunchKernelGGL(k_up_concat8<uint32_t>, grid, dim3(256), 0, (hipStream_t)stream, coarse,
                         skip, cat, (uint32_t)nvox, d, h, w, c1, c2);
    else
      hipLaunchKernelGGL(k_up_concat8<int64_t>, grid, dim3(256), 0, (hipStream_t)stream, coarse,
                         skip, cat, nvox, d, h, w, c1, c2);
  } else {
    const dim3 grid(nblk(nvox * (c1 + c2), 256));
    if (small)
      hipLaunchKernelGGL(k_up_concat<uint32_t>, grid, dim3(256), 0, (hipStream_t)stream, coarse,
                         skip, cat, (uint32_t)nvox, d, h, w, c1, c2);
    else
      hipLaunchKernelGGL(k_up_concat<int64_t>, grid, dim3(256), 0, (hipStream_t)stream, coarse,
                         skip, cat, nvox, d, h, w, c1, c2);
  }
  NN_HIP_CHECK("up concat");
  return 0;
}

int nn_split_down(const float* dcat, float* dcoarse, float* dskip, int32_t batch, int32_t d,
                  int32_t h, int32_t w, int32_t c1, int32_t c2, void* stream) {
  if (!dcat || !dcoarse || !dskip || batch < 1 || d % 2 || h % 2 || w % 2 || c1 < 1 || c2 < 1) {
    set_error("bad arguments");
    return -1;
  }
  const int64_t nfine = (int64_t)batch * d * h * w;
  const int64_t ncoarse = nfine / 8;
  const dim3 gc(nblk(ncoarse * c1, 256)), gs(nblk(nfine * c2, 256));
  if (nfine * (c1 + c2) < ((int64_t)1 << 31)) {
    hipLaunchKernelGGL(k_split_down_coarse<uint32_t>, gc, dim3(256), 0, (hipStream_t)stream, dcat,
                       dcoarse, (uint32_t)ncoarse, d, h, w, c1, c2);
    hipLaunchKernelGGL(k_split_down_skip<uint32_t>, gs, dim3(256), 0, (hipStream_t)stream, dcat,
                       dskip, (uint32_t)nfine, c1, c2);
  } else {
    hipLaunchKernelGGL(k_split_down_coarse<int64_t>, gc, dim3(256), 0, (hipStream_t)stream, dcat,
                       dcoarse, ncoarse, d, h, w, c1, c2);
    hipLaunchKernelGGL(k_split_down_skip<int64_t>, gs, dim3(256), 0, (hipStream_t)stream, dcat,
                       dskip, nfine, c1, c2);
  }
  NN_HIP_CHECK("split down");
  return 0;
}

// The three masked-MSE launches on a 4096-float workspace: per-block
// partials (two floats for each of at most kMseMaxBlocks blocks), then the
// fluid count at index 2 * kMseMaxBlocks + 1.  Every slot the final kernel
// reads is written by the same call, so the workspace needs no clearing.
constexpr int kMseMaxBlocks = 2046;
constexpr int kMseWorkspace = 4096;
static int masked_mse_launch(const float* pred, const float* target, const uint8_t* mask,
                             int64_t n, uint16_t* dy, float* loss, float* workspace,
                             hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > kMseMaxBlocks) nb = kMseMaxBlocks;
  hipLaunchKernelGGL(k_mse_partial, dim3(nb), dim3(256), 0, s, pred, target, mask, n, workspace);
  float* count = workspace + 2 * kMseMaxBlocks + 1;
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, s, workspace, nb, loss, count);
  hipLaunchKernelGGL(k_mse_grad, dim3(nblk(n * 16, 256)), dim3(256), 0, s, pred, target, mask, n,
                     count, dy);
  NN_HIP_CHECK("masked mse");
  return 0;
}

int nn_masked_mse(const float* pred, const float* target, const uint8_t* mask, int64_t n,
                  uint16_t* dy, float* loss, float* workspace, void* stream) {
  if (!pred || !target || !mask || !dy || !loss || !workspace || n < 1) {
    set_error("bad arguments");
    return -1;
  }
  return masked_mse_launch(pred, target, mask, n, dy, loss, workspace, (hipStream_t)stream);
}

// ---- allocation-free masked MSE ------------------------------------------
// The workspace of nn_masked_mse_noalloc is this file-scope device array
// (16 KiB; every GPU the library runs on holds its own copy until the
// process ends).  Host code never uses the array's name as an address: the
// device address is taken once per device with hipGetSymbolAddress, with
// that device current, and kept in scratch_dev[].
static __device__ __align__(256) float scratch[kMseWorkspace];

constexpr int kMaxDevices = 64;
constexpr int64_t kMseNoallocMaxVoxels = 0x7fffffffLL;
static std::mutex scratch_mu;
static float* scratch_dev[kMaxDevices] = {};

static float* scratch_of_current_device() {
  int dev = -1;
  const hipError_t e0 = hipGetDevice(&dev);
  if (e0 != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("nn_masked_mse_noalloc: no usable current device (%s, id %d)",
              hipGetErrorString(e0), dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("nn_masked_mse_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                hipGetErrorString(e));
      return nullptr;
    }
    scratch_dev[dev] = (float*)p;
  }
  return scratch_dev[dev];
}

int nn_masked_mse_noalloc(const float* pred, const float* target, const uint8_t* mask,
                          int64_t n, uint16_t* dy, float* loss, void* stream) {
  if (!pred || !target || !mask || !dy || !loss || n < 1) {
    set_error("bad arguments");
    return -1;
  }
  if (n > kMseNoallocMaxVoxels) {
    set_error("nn_masked_mse_noalloc: %lld voxels exceed the maximum of %lld", (long long)n,
              (long long)kMseNoallocMaxVoxels);
    return -1;
  }
  float* ws = scratch_of_current_device();
  if (!ws) return -4;
  return masked_mse_launch(pred, target, mask, n, dy, loss, ws, (hipStream_t)stream);
}

int nn_adam_step(float* param, const float* grad, float* m, float* v, uint16_t* param_bf16,
                 int64_t n, double lr, double beta1, double beta2, double eps, int32_t t,
                 void* stream) {
  if (!param || !grad || !m || !v || !param_bf16 || n < 1 || t < 1 || !(beta1 >= 0.0) ||
      !(beta1 < 1.0) || !(beta2 >= 0.0) || !(beta2 < 1.0) || !(eps > 0.0)) {
    set_error("bad arguments");
    return -1;
  }
  // The complements 1 - beta and the bias corrections 1 - beta^t are
  // formed in double: in float, 1 - 0.999f already carries a relative
  // error of 1.3e-5 from the representation of beta2.
  const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, param, grad, m,
                     v, param_bf16, n, (float)lr, (float)beta1, (float)(1.0 - beta1),
                     (float)beta2, (float)(1.0 - beta2), (float)eps, (float)c1, (float)c2);
  NN_HIP_CHECK("adam");
  return 0;
}

int nn_prepare_input(const uint8_t* mask, uint16_t* x, int64_t n, int32_t c_pad, void* stream) {
  if (!mask || !x || n < 1 || c_pad < 2) { set_error("bad arguments"); return -1; }
  if ((int64_t)n * c_pad < ((int64_t)1 << 31))
    hipLaunchKernelGGL(k_prepare_input<uint32_t>, dim3(nblk((int64_t)n * c_pad, 256)), dim3(256), 0,
                       (hipStream_t)stream, mask, x, (uint32_t)n, (uint32_t)c_pad);
  else
    hipLaunchKernelGGL(k_prepare_input<int64_t>, dim3(nblk((int64_t)n * c_pad, 256)), dim3(256), 0,
                       (hipStream_t)stream, mask, x, (int64_t)n, (int64_t)c_pad);
  NN_HIP_CHECK("prepare input");
  return 0;
}

int nn_prepare_input_dist(const uint8_t* mask, uint16_t* x, int32_t batch, int32_t n,
                          int32_t c_pad, float dmax, float* work, void* stream) {
  if (!mask || !x || !work || batch < 1 || n < 1 || c_pad < 4 || !(dmax >= 1.f) ||
      !(dmax <= 64.f)) {
    set_error("bad arguments");
    return -1;
  }
  const int64_t total = (int64_t)batch * n * n * n;
  if (total >= 0x7fffffffLL) {
    set_error("more than 2^31 voxels");
    return -1;
  }
  hipStream_t s = (hipStream_t)stream;
  float* a = work;
  float* b = work + total;
  hipLaunchKernelGGL(k_dist_init, dim3(nblk(total, 256)), dim3(256), 0, s, mask, a, total, dmax);
  const int sweeps = (int)ceilf(dmax);
  constexpr int kRun = 8;  // planes per thread when n allows
  const bool runs = n % kRun == 0;
  const int threads = (int)(runs ? total / kRun : total);
  for (int k = 0; k < sweeps; ++k) {
    if (runs)
      hipLaunchKernelGGL(k_dist_relax<kRun>, dim3(nblk(threads, 256)), dim3(256), 0, s, mask, a, b, n,
                         threads, dmax);
    else
      hipLaunchKernelGGL(k_dist_relax<1>, dim3(nblk(threads, 256)), dim3(256), 0, s, mask, a, b, n,
                         threads, dmax);
    float* t = a;
    a = b;
    b = t;
  }
  if (c_pad % 8 == 0 && ((uintptr_t)x & 15) == 0)
    hipLaunchKernelGGL(k_features8, dim3(nblk(total * (c_pad / 8), 256)), dim3(256), 0, s, mask, a, x,
                       total, c_pad, dmax);
  else
    hipLaunchKernelGGL(k_features, dim3(nblk(total * c_pad, 256)), dim3(256), 0, s, mask, a, x, total,
                       c_pad, dmax);
  NN_HIP_CHECK("prepare input with distance");
  return 0;
}

int nn_velocity_labels(const double* u, const uint8_t* mask, double scale, float* out, int64_t n,
                       void* stream) {
  if (!u || !mask || !out || n < 1) { set_error("bad arguments"); return -1; }
  hipLaunchKernelGGL(k_velocity_labels, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, u,
                     mask, scale, out, n);
  NN_HIP_CHECK("velocity labels");
  return 0;
}

int nn_velocity_out(const float* pred, const uint8_t* mask, double scale, double* u, int64_t n,
                    void* stream) {
  if (!pred || !mask || !u || n < 1) { set_error("bad arguments"); return -1; }
  hipLaunchKernelGGL(k_velocity_out, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, pred,
                     mask, scale, u, n);
  NN_HIP_CHECK("velocity out");
  return 0;
}

int nn_to_bf16(const float* src, uint16_t* dst, int64_t n, void* stream) {
  if (!src || !dst || n < 1) { set_error("bad arguments"); return -1; }
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, src, dst, n);
  NN_HIP_CHECK("to bf16");
  return 0;
}

}  // extern "C"
