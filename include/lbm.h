/*
 * lbm.h - C ABI of the MI355X (gfx950) D3Q19 TRT lattice Boltzmann library.
 *
 * The library runs the fused one-step pull update of the paper
 * "Lattice Boltzmann Benchmark Kernels as a Testbed for Performance
 * Analysis" (Wittmann et al.): per node, gather the 19 populations from the
 * neighbours of a source lattice, apply the two-relaxation-time (TRT)
 * collision with a constant body force, and store the 19 results at the
 * node in a destination lattice (Sect. 3, "One Step Kernels", pull
 * variant; the non-temporal-store refinement of Sect. 3 is applied to every
 * store of the one-step pull sweeps).  Beside it stand the AA pattern and
 * the push flavour of Sect. 3.  Lattices are represented as a full array
 * with a flag field ("direct" addressing) or as a fluid-node vector with an
 * adjacency list ("list", indirect addressing, optionally run-length
 * reduced), Sect. 3 "Lattice Representation", in
 * structure-of-arrays or array-of-structures layout (Sect. 3 "Data Layout").
 * Bounce-back is full-way or half-way (Sect. 2, Sect. 3.2); periodicity is
 * part of the index arithmetic or of the adjacency list (Sect. 3.2), per
 * axis (lbm_params.periodic).
 *
 * Conventions shared by every entry point:
 *  - Return value: LBM_OK (0) or a negative LBM_E* code.  No C++ exception
 *    crosses the ABI.  lbm_strerror() names a code; lbm_last_error()
 *    returns a thread-local message describing the most recent failure.
 *  - Device buffers are owned by the caller (allocated with any HIP
 *    allocator) and borrowed by a context until lbm_destroy().  The library
 *    itself allocates only short-lived device scratch inside the set-up and
 *    I/O calls (init, import, export, verify), never inside lbm_step().
 *  - Work is enqueued on the HIP stream given at lbm_init_geometry().
 *    lbm_step() is asynchronous; calls that return host data
 *    (lbm_macroscopic, lbm_step_diag, lbm_verify, lbm_export_pdfs)
 *    synchronise that stream.
 *  - Geometry: nodes (x, y, z), 0 <= x < nx etc., linear node index
 *    n = x + nx*(y + ny*z).  The lattice wraps on every axis (a 3-torus);
 *    walls are solid nodes of the mask, so a channel of nx*ny*nz nodes
 *    includes its wall layers (Sect. 4.4 counts 500*98*98 fluid nodes for
 *    a 500x100x100 channel).  Masks are uint8, 0 = fluid, non-zero = solid.
 *  - Velocity order (canonical, also the export/import layout):
 *      0 rest; 1..6 = +x, -x, +y, -y, +z, -z;
 *      7..18 = (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0),
 *              (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1),
 *              (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 *    Weights 1/3 (rest), 1/18 (axis), 1/36 (diagonal).
 *  - Model (Sect. 2 names D3Q19, TRT and bounce-back; the formulas are
 *    the standard ones): rho = sum f, u = (sum c f + g/2)/rho, second-order
 *    equilibrium, TRT rates 1/tau+ and 1/tau- with
 *    tau- = 1/2 + Lambda/(tau+ - 1/2), split forcing with the
 *    (1 - 1/(2 tau)) prefactor on each half.
 *  - State alignment: for the one-step pull the buffers hold
 *    post-collision populations.  The canonical "pre-collision" state that
 *    export/import use is that buffer after one streaming (gather) pass,
 *    which is what a collide-then-stream implementation holds after the
 *    same number of updates.  The push buffers hold the canonical state
 *    directly; the AA lattice holds it in place after an even number of
 *    updates and as reversed post-collision values after an odd number.
 *    Export and import translate every form, so the canonical state does
 *    not depend on layout, addressing or propagation.
 */
#ifndef LBM_MI355X_H
#define LBM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)      /* bad argument or parameter combination      */
#define LBM_ENOMEM (-2)      /* host or scratch device allocation failed   */
#define LBM_EOVERFLOW (-3)   /* lattice too large for 32-bit indices       */
#define LBM_EDEVICE (-4)     /* a HIP call failed (see lbm_last_error)     */
#define LBM_ENONFINITE (-5)  /* non-finite populations detected            */
#define LBM_ENOTCONV (-6)    /* residual target not reached (reserved: no
                                entry point returns it yet)                */

/* ---- enumerations ---------------------------------------------------- */
#define LBM_SOA 0            /* populations of one direction contiguous    */
#define LBM_AOS 1            /* populations of one node contiguous         */

#define LBM_DIRECT 0         /* full array + flag field (all N nodes)      */
#define LBM_LIST 1           /* fluid-node vector + int32 adjacency        */
#define LBM_LIST_RIA 2       /* fluid-node vector with reduced indirect
                                addressing (Sect. 3): runs of consecutive
                                fluid nodes whose 18 source slots all
                                advance by one with the node share one
                                table entry; no per-node adjacency         */

#define LBM_F64 0            /* double populations (the paper's storage)   */
#define LBM_F32_SHIFTED 1    /* float  h = f - w, double collide, store
                                rounded stochastically (hash of node,
                                direction, step)                           */
#define LBM_F16_SHIFTED 2    /* _Float16 h = (f - w) * 2^s, float collide,
                                round to nearest even on store             */
#define LBM_F16_SHIFTED_SR 3 /* as LBM_F16_SHIFTED, stochastic rounding on
                                store (hash of node, direction, step): the
                                expected stored value is exact, so updates
                                smaller than half an ulp are not lost      */

#define LBM_OS 0             /* one step, two lattices A -> B (Sect. 3)    */
#define LBM_AA 1             /* AA pattern, one lattice updated in place:
                                alternating node-local (even) and
                                neighbour (odd) kernels (Sect. 3)          */
#define LBM_OS_PUSH 2        /* one step, two lattices, push flavour: read
                                the node, collide, scatter to neighbours   */

#define LBM_FULLWAY 0        /* solids store and reverse populations       */
#define LBM_HALFWAY 1        /* mid-link reflection in the same step       */

#define LBM_VERIFY_SLAB 0       /* plates normal to z, flow along x        */
#define LBM_VERIFY_DUCT 1       /* walls normal to y and z, flow along x   */
#define LBM_VERIFY_REFERENCE 2  /* caller's velocity field                 */

/* ---- parameter and buffer records ------------------------------------ */
typedef struct {
  int32_t nx, ny, nz;       /* nodes per axis, walls included; each >= 1   */
  uint32_t periodic;        /* bit 0 x, bit 1 y, bit 2 z: the axis wraps
                               (Sect. 3.2).  On an axis whose bit is clear
                               the box faces are walls: nodes beyond them
                               count as solid.  Half-way bounce-back then
                               reflects at the face, half a link outside
                               the boundary layer.  Full-way bounce-back
                               needs the two boundary layers of such an
                               axis to be solid (else EINVAL); they keep
                               the populations in transit, so the result
                               is the same as with the axis wrapped.
                               Other bits: EINVAL.                         */
  int32_t layout;           /* LBM_SOA | LBM_AOS (LIST_RIA requires SOA)   */
  int32_t addressing;       /* LBM_DIRECT | LBM_LIST | LBM_LIST_RIA        */
  int32_t storage;          /* LBM_F64 | LBM_F32_SHIFTED | LBM_F16_SHIFTED
                               | LBM_F16_SHIFTED_SR                        */
  int32_t bounce;           /* LBM_FULLWAY | LBM_HALFWAY (lists: HALFWAY)  */
  int32_t f16_scale_log2;   /* s for the F16 storages, 0..24; else ignored */
  int32_t block;            /* threads per workgroup, 0 = default; a
                               multiple of 64 up to 1024 (the AA kernels
                               and the FP32-storage SoA pull take at most
                               512 and cut larger values; the
                               AoS column marches - pull, push, AA
                               neighbour step - run their own shapes)      */
  int32_t pad;              /* extra elements between direction arrays
                               (SOA/LIST); -1 = automatic                  */
  int32_t cu_slots;         /* at most this many sweep workgroups per
                               compute unit (reserved LDS caps residency);
                               0 = no cap                                  */
  int32_t propagation;      /* LBM_OS (pull) | LBM_AA | LBM_OS_PUSH (AA
                               uses pdf_a only; pdf_b may be NULL)         */
  double tau_plus;          /* > 1/2; kinematic viscosity (tau+ - 1/2)/3   */
  double magic_lambda;      /* Lambda > 0                                  */
  double g[3];              /* body-force density, lattice units           */
} lbm_params;

typedef struct {
  int64_t n_nodes;          /* nx*ny*nz                                    */
  int64_t n_fluid;          /* nodes with mask == 0                        */
  int64_t n_sites;          /* nodes the sweep updates: N (direct) or Nf   */
  int64_t stride;           /* elements between direction arrays (SOA);
                               19 for AOS (records, also for LIST)         */
  int64_t pdf_bytes;        /* size of EACH of pdf_a and pdf_b             */
  int64_t mask_bytes;       /* device mask: N bytes                        */
  int64_t adj_bytes;        /* LIST: 18 direction arrays of int32 slots
                               (SOA: stride entries apart; AOS: Nf padded
                               to 64); else 0                              */
  int64_t fluid_index_bytes;/* LIST, LIST_RIA: Nf int32 (list -> node)     */
  int64_t node_map_bytes;   /* LIST, LIST_RIA: N int32 (node -> list/-1)   */
  int64_t links_bytes;      /* DIRECT + HALFWAY: N uint32 link words       */
  int64_t u_prev_bytes;     /* 3*n_sites doubles for the residual          */
  int64_t scratch_bytes;    /* reduction partials (for OS + DIRECT one
                               record per workgroup of the fused sweep)    */
  double bytes_per_update;  /* algorithmic HBM bytes per site update       */
  int64_t n_runs;           /* LIST_RIA: number of runs; else 0            */
  int64_t ria_bytes;        /* LIST_RIA: run tables (library-internal
                               layout, filled at init); else 0             */
} lbm_sizes;

typedef struct {            /* device pointers, caller-owned               */
  void* pdf_a;              /* pdf_bytes, 256-byte aligned                 */
  void* pdf_b;              /* pdf_bytes, 256-byte aligned (LBM_OS only)   */
  uint8_t* mask;            /* mask_bytes                                  */
  int32_t* adj;             /* LIST only, else NULL                        */
  int32_t* fluid_index;     /* LIST and LIST_RIA, else NULL                */
  int32_t* node_map;        /* LIST and LIST_RIA, else NULL                */
  uint32_t* links;          /* DIRECT + HALFWAY only (bit 0: node solid,
                               bit i: neighbour x - c_i solid), else NULL  */
  double* u_prev;           /* optional (NULL: no residual)                */
  void* scratch;            /* scratch_bytes                               */
  void* ria;                /* LIST_RIA only (ria_bytes), else NULL        */
} lbm_buffers;

typedef struct {
  double mass;              /* sum of all populations held by the lattice
                               (includes populations in transit inside
                               full-way solid nodes)                       */
  double momentum[3];       /* sum of c_i f_i over the same populations    */
  double u_max;             /* max |u| over fluid nodes                    */
  double residual;          /* ||u - u_prev|| / ||u|| over fluid nodes, or
                               -1 if u_prev is NULL or not yet filled      */
  int64_t nonfinite;        /* fluid nodes with a non-finite population    */
  int64_t step;             /* updates applied since init                  */
} lbm_stats;

typedef struct {
  double max_abs;           /* max |u - u_ref| over compared nodes, all
                               three components                            */
  double rel_l2;            /* ||u - u_ref||_2 / ||u_ref||_2               */
  double ref_max;           /* max |u_ref|                                 */
  int64_t n_compared;       /* fluid nodes compared                        */
} lbm_verify_result;

typedef struct lbm_ctx lbm_ctx;

/* ---- entry points ---------------------------------------------------- */

/* Sizes of every buffer for a parameter set and a host mask (N bytes).
 * Counts fluid nodes (and, for LIST_RIA, the runs); validates parameters
 * (tau+ > 1/2, Lambda > 0, dims >= 1 and <= 65535 on y and z, N < 2^31,
 * the lists need every population slot index below 2^31, the AoS one-step
 * pull needs 19*nx*ny < 2^31).  Allocates nothing.
 * Errors: EINVAL, EOVERFLOW. */
int lbm_plan(const lbm_params* params, const uint8_t* mask_host, lbm_sizes* out);

/* Geometry set-up (Sect. 3 "Lattice Representation"; Sect. 3.2): copies the
 * mask to bufs->mask; for DIRECT + HALFWAY builds the link words; for LIST
 * builds the fluid-node vector (x fastest; for AOS, x fastest within
 * columns of 16 x 16 nodes taken through all layers, column after column,
 * so that nodes sharing source records are listed close together),
 * the node map and the adjacency list (18 int32 per node: the slot a pull
 * reads for direction i, which is the neighbour's slot, wrapped
 * periodically, or the node's own opposite slot when the neighbour is solid
 * - half-way bounce-back); for LIST_RIA builds the fluid-node vector, the
 * node map and the run tables instead of the adjacency list (a run is a
 * maximal set of consecutive fluid nodes of one x-row, away from the x
 * wrap, whose 18 neighbours x - c_i have the same fluid/solid status as
 * those of the previous node; along a run every source slot advances by
 * one, so one table entry per run serves all its nodes, Sect. 3
 * "Lattice Representation"); then fills both PDF buffers with the rest state
 * f_i = w_i.  `stream` is a hipStream_t (NULL = default stream).  On
 * success *out owns host metadata only.  Synchronises the stream.
 * Errors: EINVAL, EOVERFLOW, ENOMEM, EDEVICE. */
int lbm_init_geometry(lbm_ctx** out, const lbm_params* params,
                      const uint8_t* mask_host, const lbm_buffers* bufs,
                      void* stream);

/* Initialise the state to equilibrium node by node so that the state's
 * density and velocity (as lbm_macroscopic reports them) are rho and u:
 * f = e(rho, u - g/(2 rho)) on fluid nodes, since the velocity of a state
 * is (sum c f + g/2)/rho; solids get the rest state.  rho_dev: N doubles or
 * NULL (rho = 1); u_dev: 3*N doubles, component-major [3][N], or NULL
 * (u = 0).  Both are device pointers indexed by full node index.  Resets
 * the step counter and the residual history.  Errors: EINVAL, EDEVICE. */
int lbm_init_fields(lbm_ctx* ctx, const double* rho_dev, const double* u_dev);

/* Enqueue n fused stream-collide updates, one kernel launch each.
 * LBM_OS: source and destination buffers swap after every launch (Sect. 3
 * "One Step Kernels"); each node gathers from its neighbours.  LBM_OS_PUSH:
 * the same buffers, each node scatters its collided populations to its
 * neighbours.  LIST_RIA runs the list kernels with run tables in place of
 * the adjacency.  LBM_AA: one buffer; launches alternate between the
 * node-local kernel (read a node's populations, collide, write them back
 * reversed) and the neighbour kernel (read each population from the slot
 * the previous local step left it in at the neighbour, collide, write it
 * where the next local step expects it), Sect. 3 "AA Pattern Kernels".
 * Asynchronous.  Errors: EINVAL (n < 0), EDEVICE. */
int lbm_step(lbm_ctx* ctx, int32_t n);

/* Macroscopic fields and diagnostics of the current state.  rho_dev (N
 * doubles) and u_dev ([3][N] doubles) are optional device outputs indexed
 * by full node index; solids get 0.  Fills *out (host) with mass, momentum,
 * max |u|, the residual against the velocity stored at the previous call
 * (then stores the current one; needs bufs->u_prev) and the non-finite
 * count.  Reductions are FP64 and run in a fixed order.  Synchronises.
 * Returns ENONFINITE if any fluid population is not finite (the stats are
 * still filled).  Errors: EINVAL, EDEVICE, ENONFINITE. */
int lbm_macroscopic(lbm_ctx* ctx, double* rho_dev, double* u_dev,
                    lbm_stats* out);

/* One update with the diagnostics of the state it starts from: the same
 * *out that lbm_macroscopic(ctx, NULL, NULL, out) returns before the update
 * (out->step is the count before it, and the residual history advances
 * likewise), followed by the same update as lbm_step(ctx, 1).  For
 * LBM_OS + LBM_DIRECT (SoA or AoS) the moments are taken inside the sweep
 * from the populations it gathers (one pass over the lattice instead of
 * two, the diagnostics are part of the fused kernel, Sect. 3 "One Step
 * Kernels"); every other form runs the two calls in turn.  Sums are FP64
 * and combine per-workgroup partials in a fixed order (not the order
 * lbm_macroscopic uses, so sums can differ from it in the last bits).  The update is applied whatever
 * the state holds.  Synchronises.  Returns ENONFINITE if the state it
 * started from had a non-finite fluid population (the stats are filled and
 * the update has run).  Errors: EINVAL, EDEVICE, ENONFINITE. */
int lbm_step_diag(lbm_ctx* ctx, lbm_stats* out);

/* Compare the current velocity with a reference (Sect. 2.1 verification):
 * LBM_VERIFY_SLAB: u_x = g_x/(2 nu) [(H/2)^2 - zeta^2], H = nz - 2, zeta =
 *   z - (nz-1)/2 (plates are the solid layers z = 0, nz-1, walls half a
 *   node outside the outermost fluid layer); u_y = u_z = 0.
 * LBM_VERIFY_DUCT: the Fourier series of steady flow in a rectangular duct
 *   with half-widths a = (ny-2)/2, b = (nz-2)/2, walls placed likewise.
 *   Both forms assume the walls are solid boundary layers of the mask; a
 *   box whose walls are the faces of non-periodic axes compares with
 *   LBM_VERIFY_REFERENCE.
 * LBM_VERIFY_REFERENCE: ref_dev is a device [3][N] double field.
 * Synchronises.  Errors: EINVAL, EDEVICE. */
int lbm_verify(lbm_ctx* ctx, int32_t kind, const double* ref_dev,
               lbm_verify_result* out);

/* Canonical pre-collision populations, as double, of `count` nodes given by
 * full node index in node_ids_host (host int64), written to out_host (host,
 * count*19 doubles, node-major, canonical velocity order).  node_ids_host
 * NULL means all N nodes in order (count must be N).  Nodes that hold no
 * state (solids under half-way bounce-back) read as zeros.  Synchronises.
 * Errors: EINVAL (bad id or count), ENOMEM, EDEVICE. */
int lbm_export_pdfs(lbm_ctx* ctx, const int64_t* node_ids_host, int64_t count,
                    double* out_host);

/* Replace the state with a canonical pre-collision state given for all N
 * nodes (host, N*19 doubles, node-major; entries of nodes that hold no
 * state are ignored).  Inverse of the export mapping; values are rounded
 * to the storage type.  Resets the residual history, keeps the step count.
 * Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
int lbm_import_pdfs(lbm_ctx* ctx, const double* host_in);

/* Query: sizes, step count and which buffer is current (0 = pdf_a). */
int lbm_get_sizes(const lbm_ctx* ctx, lbm_sizes* out);
int64_t lbm_step_count(const lbm_ctx* ctx);
int lbm_current_buffer(const lbm_ctx* ctx);

/* Release host metadata.  Device buffers stay with the caller. */
void lbm_destroy(lbm_ctx* ctx);

const char* lbm_strerror(int code);
const char* lbm_last_error(void);

/* Memory micro-benchmarks that mirror the paper's Sect. 4.1 set, each one
 * kernel launch on `stream` (asynchronous):
 *   kind 0 copy:        b[k] = a[k], one array of n doubles;
 *   kind 1 copy-19:     19 arrays of n doubles, b_i[k] = a_i[k];
 *   kind 2 copy-19-nt:  as kind 1 with non-temporal stores;
 *   kind 3 update-19:   19 arrays of n doubles updated in place,
 *                       a_i[k] = a_i[k] * 1.0.
 * Kinds 0-3 move one 8-byte element per thread.  Kinds 4-9 bound the
 * attainable bandwidth of the same stream counts: 16-byte accesses,
 * several in flight per thread, non-temporal stores:
 *   kind 4 copy-v:      one array of n doubles (as kind 0);
 *   kind 5 copy-4-v:    4 arrays of n doubles;
 *   kind 6 copy-19-v:   19 arrays of n doubles;
 *   kind 7 copy-19-vp:  as kind 6 on a persistent grid (8 workgroups per
 *                       compute unit, grid-stride loop);
 *   kind 8 read-19-v:   19 arrays of n doubles read (b untouched for
 *                       finite data);
 *   kind 9 write-19-v:  19 arrays of n doubles written (a unused).
 * Kinds 4-9 need even n and stride and 16-byte aligned a and b.
 * a and b are device buffers of 19*stride doubles (kinds 1-3, 5-9; kinds
 * 0 and 4 use the first n).  Errors: EINVAL, EDEVICE. */
int lbm_membench(int32_t kind, const double* a, double* b, int64_t n,
                 int64_t stride, int32_t block, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MI355X_H */
