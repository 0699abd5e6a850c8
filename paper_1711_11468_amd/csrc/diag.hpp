// diag.hpp - the diagnostics a sweep can take on the fly: the FP64 moments
// of the populations it has gathered, accumulated per thread and reduced
// per workgroup into one partial record (fixed order), combined afterwards
// by the two-stage reduction of diagnostics.hip.
#pragma once

#include "gather.hpp"
#include "internal.hpp"

namespace lbm {

// Diagnostics fused into a sweep (the state it reads is the canonical state
// before the update): per node the FP64 moments of the gathered populations,
// accumulated as mass and momentum over every state-holding node and, over
// fluid nodes, max |u|, the non-finite count and the residual sums against
// (and then into) the velocity history u_prev [3][N].
struct DiagArgs {
  double gx, gy, gz;
  double* u_prev;
  int residual_mode;  // 0: none, 1: store u only, 2: sums against u_prev, then store
  double* partials;   // [rows][kStatSlots]
};

template <class ST>
__device__ __forceinline__ void diag_node(const typename ST::R (&f)[Q], bool fluid, int64_t n,
                                          int64_t N, const DiagArgs& d, double (&acc)[M_COUNT]) {
  double fd[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) fd[i] = ST::kShifted ? (double)f[i] + weight(i) : (double)f[i];
  double rho, ux, uy, uz, jx, jy, jz;
  moments_f64(fd, d.gx, d.gy, d.gz, rho, ux, uy, uz, jx, jy, jz);
  acc[M_MASS] += rho;
  acc[M_PX] += jx;
  acc[M_PY] += jy;
  acc[M_PZ] += jz;
  if (!fluid) return;
  if (!(isfinite(rho) && isfinite(jx) && isfinite(jy) && isfinite(jz))) acc[M_NONFINITE] += 1.0;
  const double u2 = ux * ux + uy * uy + uz * uz;
  acc[M_UMAX] = fmax(acc[M_UMAX], sqrt(u2));
  if (d.residual_mode > 0) {
    if (d.residual_mode == 2) {
      const double ex = ux - d.u_prev[n], ey = uy - d.u_prev[N + n], ez = uz - d.u_prev[2 * N + n];
      acc[M_DU2] += ex * ex + ey * ey + ez * ez;
      acc[M_U2] += u2;
    }
    d.u_prev[n] = ux;
    d.u_prev[N + n] = uy;
    d.u_prev[2 * N + n] = uz;
  }
}

}  // namespace lbm
