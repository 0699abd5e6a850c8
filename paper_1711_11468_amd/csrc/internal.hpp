// internal.hpp - host-side context record and kernel launcher declarations
// shared by the translation units of the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

struct lbm_ctx {
  lbm_params p;
  lbm_sizes s;
  lbm_buffers b;
  hipStream_t stream;
  int cur;             // index of the buffer holding the current state
  int aa_odd;          // AA: the next launch is the neighbour kernel
  int64_t step;        // updates since init
  int u_prev_valid;    // u_prev holds the velocity of a previous call
  int block;           // threads per workgroup for the sweeps
  int device;
  int64_t adj_stride;  // LIST: entries between adjacency directions
  // LIST_RIA run tables, carved out of b.ria: run_start[n_runs + 1] (first
  // list index of each run, then n_fluid), run_adj[18][run_stride] (the
  // slot of direction i for the run's first node), chunk_run[ceil(Nf/64)]
  // (the run of node 64c) and run_delta[Nf] (run of node m minus the run
  // of its 64-node chunk, < 64).
  int64_t n_runs;
  int64_t run_stride;
  int32_t* run_start;
  int32_t* run_adj;
  int32_t* chunk_run;
  uint8_t* run_delta;
};

namespace lbm {

// True for the two fluid-list addressings.
inline bool is_list(const lbm_params& p) { return p.addressing != LBM_DIRECT; }

void set_error(const char* fmt, ...);

inline void* pdf_buf(lbm_ctx* c, int which) { return which == 0 ? c->b.pdf_a : c->b.pdf_b; }

// Launchers: each enqueues on c->stream and returns a hipError_t.
// One update of the lattice: the one-step pull sweep (SoA direct or list),
// its AoS form, the push form (src -> dst), or the AA pattern (in place on
// buf, the kernel chosen by c->aa_odd).
hipError_t launch_pull(lbm_ctx* c, const void* src, void* dst);
hipError_t launch_pull_aos(lbm_ctx* c, const void* src, void* dst);
// The AoS pull with the diagnostics fused in: one partial record per column
// into `partials`; *records = number written.
hipError_t launch_pull_aos_diag(lbm_ctx* c, const void* src, void* dst, int residual_mode,
                                double* partials, int64_t* records);
// Column shape of the AoS marches (x, y nodes).
constexpr int kAosBX = 32, kAosTY = 8;
hipError_t launch_push_aos(lbm_ctx* c, const void* src, void* dst);
hipError_t launch_aa_aos_odd(lbm_ctx* c, void* buf);
hipError_t launch_push(lbm_ctx* c, const void* src, void* dst);
hipError_t launch_aa(lbm_ctx* c, void* buf);
// Fluid list in AoS records: pull, push and both AA steps.
hipError_t launch_list_aos(lbm_ctx* c, const void* src, void* dst);
// The one-step pull (SoA direct) with the diagnostics of the state it reads
// fused in: per-row partials (kStatSlots doubles each) into `partials`;
// *rows = number of records written.
hipError_t launch_pull_diag(lbm_ctx* c, const void* src, void* dst, int residual_mode,
                            double* partials, int64_t* rows);
// Run-length list (LIST_RIA): the pull and push sweeps and the AA
// neighbour kernel (the AA local kernel needs no addressing).
hipError_t launch_pull_ria(lbm_ctx* c, const void* src, void* dst);
hipError_t launch_push_ria(lbm_ctx* c, const void* src, void* dst);
hipError_t launch_aa_ria_odd(lbm_ctx* c, void* buf);
hipError_t launch_build_run_adj(lbm_ctx* c);
hipError_t launch_fill_rest(lbm_ctx* c, void* buf);
hipError_t launch_build_adjacency(lbm_ctx* c);
hipError_t launch_build_links(lbm_ctx* c);
hipError_t launch_export(lbm_ctx* c, const void* src, const int64_t* ids_dev, int64_t count,
                         double* out_dev);
hipError_t launch_import(lbm_ctx* c, const double* canon_dev, void* dst);
hipError_t launch_init_fields(lbm_ctx* c, const double* rho_dev, const double* u_dev, void* dst);
// Moments + block partials; then a one-block fixed-order final reduction
// into partials[0..kStatSlots).  residual_mode: 0 none, 1 compute.
constexpr int kStatSlots = 12;
hipError_t launch_moments(lbm_ctx* c, const void* src, double* rho_out, double* u_out,
                          int residual_mode, double* partials, int64_t* n_blocks_out);
hipError_t launch_verify(lbm_ctx* c, const void* src, int kind, const double* ref_dev,
                         double* partials, int64_t* n_blocks_out);
hipError_t launch_final_reduce(lbm_ctx* c, double* partials, int64_t n_blocks, int n_slots,
                               uint32_t max_mask, double* out_dev);
// Fixed-order reduction of any number of partial records: contiguous groups
// into at most kMaxReduceRecords records in `stage`, then one workgroup.
hipError_t launch_reduce_records(lbm_ctx* c, double* partials, int64_t n, int n_slots,
                                 uint32_t max_mask, double* stage, double* out_dev);
constexpr int64_t kMaxReduceRecords = 4096;
// Forms whose sweep can carry the diagnostics: the one-step pull with
// direct addressing (SoA: one record per (y, z) row; AoS: one per column of
// the z march).
inline bool fused_diag_form(const lbm_params& p) {
  return p.propagation == LBM_OS && p.addressing == LBM_DIRECT;
}
// Scratch layout: [records][kStatSlots] partials, [kMaxReduceRecords]
// [kStatSlots] second-stage partials, [kStatSlots] result.  The AoS march
// runs at most 8192 + (its columns per layer) workgroups.
inline int64_t stat_records(const lbm_params& p) {
  int64_t rows = 0;
  if (fused_diag_form(p))
    rows = p.layout == LBM_SOA ? (int64_t)p.ny * p.nz
                               : 8192 + (int64_t)((p.nx + kAosBX - 1) / kAosBX) * ((p.ny + kAosTY - 1) / kAosTY);
  return rows > kMaxReduceRecords ? rows : kMaxReduceRecords;
}
// Slot layouts of the two reductions.
enum { M_MASS = 0, M_PX, M_PY, M_PZ, M_DU2, M_U2, M_UMAX, M_NONFINITE, M_COUNT };
enum { V_MAXABS = 0, V_ERR2, V_REF2, V_REFMAX, V_COUNT_N, V_COUNT };
hipError_t launch_membench(int kind, const double* a, double* b, int64_t n, int64_t stride,
                           int block, hipStream_t stream);

}  // namespace lbm
