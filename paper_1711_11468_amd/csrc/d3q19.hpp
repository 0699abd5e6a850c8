// d3q19.hpp - device-side D3Q19 velocity set, storage formats and the TRT
// collision with split body forcing.
//
// The model (paper Sect. 2: D3Q19, two-relaxation-time collision, bounce-back;
// Sect. 2.1: constant body force) with the standard formulas:
//   rho = sum_i f_i,  u = (sum_i c_i f_i + g/2) / rho
//   e_i = w_i rho [1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u]
//   F_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . g
//   f*_i = f_i - (f+_i - e+_i)/tau+ - (f-_i - e-_i)/tau-
//          + (1 - 1/(2 tau+)) F+_i + (1 - 1/(2 tau-)) F-_i
// where x+_i = (x_i + x_opp(i))/2 and x-_i = (x_i - x_opp(i))/2, and
// tau- = 1/2 + Lambda/(tau+ - 1/2).
//
// Velocity order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 diagonals, each
// opposite pair adjacent (i odd, i+1), so opp(i) = i+1 for odd i >= 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/lbm.h"

namespace lbm {

constexpr int Q = 19;

struct Vel {
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

__host__ __device__ constexpr double weight(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---- storage formats ------------------------------------------------------
// R: arithmetic type of the collision; T: element type in memory.
// Shifted formats store h_i = f_i - w_i (scaled by 2^s for half precision)
// and run the collision on h directly.
// store(v, scale, key): key identifies (node, direction, time step) and is
// used only by the stochastically rounded format.
struct StoreF64 {
  using T = double;
  using R = double;
  static constexpr bool kShifted = false;
  static constexpr bool kStochastic = false;
  static constexpr int kRowBlockMax = 1024;  // largest row workgroup of the SoA pull
  __device__ __forceinline__ static R load(T v, R) { return v; }
  __device__ __forceinline__ static T store(R v, R, uint32_t) { return v; }
};

// double -> float with stochastic rounding: a uniform 29-bit random value
// is added to the magnitude below the last float mantissa bit and the sum
// is truncated, so a value rounds up with probability equal to its fraction
// of a float ulp and the expected stored value equals the input.  The
// truncation is done on the bit fields (a few integer operations; the
// library's round-toward-zero conversion expands to compare-and-select
// sequences that tripled the sweep's instruction count).  Magnitudes below
// the float normal range (2^-126) are flushed to zero and those beyond it
// saturate to infinity; the populations stored here lie far inside it.
__device__ __forceinline__ float sr_f64_to_f32(double v, uint32_t rnd) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t sign = (uint32_t)(b >> 32) & 0x80000000u;
  const unsigned long long mag = (b & 0x7fffffffffffffffull) + (unsigned long long)(rnd >> 3);
  const int e = (int)(mag >> 52) - (1023 - 127);  // float biased exponent
  uint32_t fb;
  if (e <= 0) fb = 0u;
  else if (e >= 255) fb = 0x7f800000u;
  else fb = ((uint32_t)e << 23) | ((uint32_t)(mag >> 29) & 0x7fffffu);
  return __uint_as_float(fb | sign);
}

// Float storage of h = f - w.  The collision runs in double and each stored
// value is rounded stochastically.  With float arithmetic and nearest
// rounding the per-node sums of 19 values of size |h| round at ~1e-10 on
// a 130 x 130 duct, 1e-4 of the force the node gains per step; repeated
// identically over the ~10^4 updates the flow takes to settle, they left
// 2.7e-5 of the steady velocity.  Stochastic rounding keeps every store
// unbiased and uncorrelated from step to step.
struct StoreF32Shifted {
  using T = float;
  using R = double;
  static constexpr bool kShifted = true;
  static constexpr bool kStochastic = true;
  // The double collision needs more than the 128 registers a 1024-thread
  // bound leaves; with 512-thread rows it runs without spilling.
  static constexpr int kRowBlockMax = 512;
  __device__ __forceinline__ static R load(T v, R) { return (R)v; }
  // rnd: a random word whose top 29 bits are uniformly distributed
  __device__ __forceinline__ static T store(R v, R, uint32_t rnd) { return sr_f64_to_f32(v, rnd); }
};

struct StoreF16Shifted {
  using T = _Float16;
  using R = float;
  static constexpr bool kShifted = true;
  static constexpr bool kStochastic = false;
  static constexpr int kRowBlockMax = 1024;  // largest row workgroup of the SoA pull
  // scale = 2^s on store, 2^-s on load: exact (power of two), so the only
  // rounding is the float -> half conversion (round to nearest even).
  __device__ __forceinline__ static R load(T v, R inv_scale) { return (R)v * inv_scale; }
  __device__ __forceinline__ static T store(R v, R scale, uint32_t) { return (T)(v * scale); }
};

// 32-bit finaliser of MurmurHash3 (Appleby): a bijective avalanche mixer.
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// float -> half with stochastic rounding, by the gfx950 conversion
// instruction: it adds the top 13 bits of the random word below the last
// half-precision mantissa bit of the magnitude and truncates, so a value
// rounds up with probability equal to its fraction of an ulp and the
// expected stored value equals the input (small increments are not lost).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

struct StoreF16ShiftedSR {
  using T = _Float16;
  using R = float;
  static constexpr bool kShifted = true;
  static constexpr bool kStochastic = true;
  static constexpr int kRowBlockMax = 1024;  // largest row workgroup of the SoA pull
  __device__ __forceinline__ static R load(T v, R inv_scale) { return (R)v * inv_scale; }
  // rnd: a random word whose top 13 bits are uniformly distributed
  __device__ __forceinline__ static T store(R v, R scale, uint32_t rnd) {
    const half2_t z = {(_Float16)0, (_Float16)0};
    return __builtin_amdgcn_cvt_sr_f16_f32(z, v * scale, rnd, false)[0];
  }
};

// Random bits for stochastic rounding.  One hash per (node, time step):
// mix32 of the node index xor a hash of the step; the 19 values of the node
// then take successive states of a 32-bit linear congruential generator
// (Numerical Recipes constants) seeded with it; the conversion uses the top
// 13 bits of each state (the well-mixed ones).  Deterministic: a function of
// (node, direction, step).
struct SrStream {
  uint32_t s;
  __device__ __forceinline__ SrStream(uint32_t node, uint32_t step, bool on)
      : s(on ? mix32(node * 0x9E3779B1u ^ mix32(step * 0x85ebca77u + 0x165667b1u)) : 0u) {}
  __device__ __forceinline__ uint32_t next() {
    s = s * 1664525u + 1013904223u;
    return s;
  }
};

// Collision constants in the arithmetic type.
template <typename R>
struct Collide {
  R lp, lm;          // 1/tau+, 1/tau-
  R ap, am;          // 1 - 1/(2 tau+), 1 - 1/(2 tau-)
  R gx, gy, gz;      // body-force density
  R scale, inv_scale;  // storage scale (half precision only), else 1
  uint32_t step;       // time step being computed (stochastic rounding key)
};

// The collision in double arithmetic (FP64 storage, and FP32 storage, whose
// collision runs in double): the textbook form, with u = J / rho.  Its
// register footprint keeps the FP64 sweep free of scratch spills.
template <typename R, bool SHIFTED>
__device__ __forceinline__ void trt_collide_double(R (&f)[Q], const Collide<R>& k) {
  R s = f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) s += f[i];
  const R rho = SHIFTED ? R(1) + s : s;
  R jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R d = f[i] - f[i + 1];
    if (Vel::cx[i] != 0) jx += Vel::cx[i] > 0 ? d : -d;
    if (Vel::cy[i] != 0) jy += Vel::cy[i] > 0 ? d : -d;
    if (Vel::cz[i] != 0) jz += Vel::cz[i] > 0 ? d : -d;
  }
  const R inv_rho = R(1) / rho;
  const R ux = (jx + R(0.5) * k.gx) * inv_rho;
  const R uy = (jy + R(0.5) * k.gy) * inv_rho;
  const R uz = (jz + R(0.5) * k.gz) * inv_rho;
  const R usq = ux * ux + uy * uy + uz * uz;
  const R ug = ux * k.gx + uy * k.gy + uz * k.gz;
  // e_i - (SHIFTED ? w_i : 0) = w_i (s + rho (3 cu + 9/2 cu^2 - 3/2 usq))
  {
    const R w = R(weight(0));
    const R e0 = w * (s - R(1.5) * rho * usq);
    const R F0 = w * (R(-3) * ug);
    f[0] = f[0] + k.lp * (e0 - f[0]) + k.ap * F0;
  }
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R w = R(weight(i));
    const R cu = R(Vel::cx[i]) * ux + R(Vel::cy[i]) * uy + R(Vel::cz[i]) * uz;
    const R cg = R(Vel::cx[i]) * k.gx + R(Vel::cy[i]) * k.gy + R(Vel::cz[i]) * k.gz;
    const R ep = w * (s + rho * (R(4.5) * cu * cu - R(1.5) * usq));
    const R em = w * (R(3) * rho * cu);
    const R Fp = w * (R(9) * cu * cg - R(3) * ug);
    const R Fm = w * (R(3) * cg);
    const R fp = R(0.5) * (f[i] + f[i + 1]);
    const R fm = R(0.5) * (f[i] - f[i + 1]);
    const R sym = k.lp * (ep - fp) + k.ap * Fp;
    const R asym = k.lm * (em - fm) + k.am * Fm;
    f[i] = f[i] + sym + asym;
    f[i + 1] = f[i + 1] + sym - asym;
  }
}

// The collision in float arithmetic (FP16 storage): the equilibrium's odd
// part is formed from J = rho u directly and the constant 3 w_i is a float
// pair hi + lo (see below), which removes the systematic momentum gain the
// rounding of the float weights would leave.
template <typename R, bool SHIFTED>
__device__ __forceinline__ void trt_collide_float(R (&f)[Q], const Collide<R>& k) {
  R s = f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) s += f[i];
  const R rho = SHIFTED ? R(1) + s : s;
  R jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R d = f[i] - f[i + 1];
    if (Vel::cx[i] != 0) jx += Vel::cx[i] > 0 ? d : -d;
    if (Vel::cy[i] != 0) jy += Vel::cy[i] > 0 ? d : -d;
    if (Vel::cz[i] != 0) jz += Vel::cz[i] > 0 ? d : -d;
  }
  // J = rho u = j + g/2; the equilibrium's odd part, 3 w rho (c.u), is
  // formed from J directly rather than as rho * ((c.J) / rho).
  const R Jx = jx + R(0.5) * k.gx, Jy = jy + R(0.5) * k.gy, Jz = jz + R(0.5) * k.gz;
  const R inv_rho = R(1) / rho;
  const R ux = Jx * inv_rho;
  const R uy = Jy * inv_rho;
  const R uz = Jz * inv_rho;
  const R Ju = Jx * ux + Jy * uy + Jz * uz;  // rho u^2
  const R ug = ux * k.gx + uy * k.gy + uz * k.gz;
  // e_i - (SHIFTED ? w_i : 0) = w_i (s + 3 c.J + 9/2 (c.J)(c.u) - 3/2 J.u)
  {
    const R w = R(weight(0));
    const R e0 = w * (s - R(1.5) * Ju);
    const R F0 = w * (R(-3) * ug);
    f[0] = f[0] + k.lp * (e0 - f[0]) + k.ap * F0;
  }
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R w = R(weight(i));
    const R cu = R(Vel::cx[i]) * ux + R(Vel::cy[i]) * uy + R(Vel::cz[i]) * uz;
    const R cJ = R(Vel::cx[i]) * Jx + R(Vel::cy[i]) * Jy + R(Vel::cz[i]) * Jz;
    const R cg = R(Vel::cx[i]) * k.gx + R(Vel::cy[i]) * k.gy + R(Vel::cz[i]) * k.gz;
    const R ep = w * (s + (R(4.5) * cJ * cu - R(1.5) * Ju));
    // The odd part returns the momentum sum_i c_i em_i = 3 sum_i w_i c_i c_i . J
    // = J.  In float, 1/18 and 1/36 both round up by 7.45e-9 (relative), so
    // with float weights every collision would keep J (1 + 7.45e-9): a
    // multiplicative gain of ~6.6e-9 per update that, over the ~10^4
    // updates a duct takes to develop, outgrows the storage rounding
    // (1e-4 of the velocity on a 130 x 130 duct).  The constant 3 w_i is
    // therefore split into a float pair hi + lo, exact to ~1e-15.
    const R w3hi = (R)(3.0 * weight(i));
    const R w3lo = (R)(3.0 * weight(i) - (double)w3hi);
    const R em = w3hi * cJ + w3lo * cJ;
    const R Fp = w * (R(9) * cu * cg - R(3) * ug);
    const R Fm = w * (R(3) * cg);
    const R fp = R(0.5) * (f[i] + f[i + 1]);
    const R fm = R(0.5) * (f[i] - f[i + 1]);
    const R sym = k.lp * (ep - fp) + k.ap * Fp;
    const R asym = k.lm * (em - fm) + k.am * Fm;
    f[i] = f[i] + sym + asym;
    f[i + 1] = f[i + 1] + sym - asym;
  }
}

// In-place TRT collision of one fluid node.  SHIFTED: f holds h = f - w.
template <typename R, bool SHIFTED>
__device__ __forceinline__ void trt_collide(R (&f)[Q], const Collide<R>& k) {
  if constexpr (std::is_same<R, float>::value)
    trt_collide_float<R, SHIFTED>(f, k);
  else
    trt_collide_double<R, SHIFTED>(f, k);
}

// Density and velocity of a (pre-collision, unshifted) node in double.
__device__ __forceinline__ void moments_f64(const double (&f)[Q], double gx, double gy,
                                            double gz, double& rho, double& ux,
                                            double& uy, double& uz, double& jx,
                                            double& jy, double& jz) {
  double s = f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) s += f[i];
  jx = jy = jz = 0.0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    jx += Vel::cx[i] * f[i];
    jy += Vel::cy[i] * f[i];
    jz += Vel::cz[i] * f[i];
  }
  rho = s;
  ux = (jx + 0.5 * gx) / rho;
  uy = (jy + 0.5 * gy) / rho;
  uz = (jz + 0.5 * gz) / rho;
}

// Periodic neighbour coordinate v - c for c in {-1, 0, 1}.
__device__ __forceinline__ int wrap_sub(int v, int c, int n) {
  int r = v - c;
  return r < 0 ? r + n : (r >= n ? r - n : r);
}

}  // namespace lbm
