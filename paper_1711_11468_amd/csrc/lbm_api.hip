// lbm_api.hip - host runtime behind the C ABI declared in include/lbm.h:
// parameter validation, sizing, geometry set-up (fluid-node compaction on
// the host, adjacency on the device), the step loop with A/B buffer swap,
// diagnostics, verification and canonical state transfer.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "d3q19.hpp"
#include <cstdlib>

#include "internal.hpp"

namespace lbm {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

static int hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return LBM_EDEVICE;
}

#define LBM_HIP(call, what)                 \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

static int elem_size(int storage) {
  return storage == LBM_F64 ? 8 : (storage == LBM_F32_SHIFTED ? 4 : 2);  // F16 kinds: 2
}

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

constexpr int kListTile = 16;  // AoS list order: columns of 16 x 16 nodes

static int validate(const lbm_params* p) {
  if (!p) { set_error("params is NULL"); return LBM_EINVAL; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { set_error("dimensions must be >= 1"); return LBM_EINVAL; }
  if ((int64_t)p->ny * p->nz > 0x7fffffffLL) { set_error("ny*nz too large"); return LBM_EOVERFLOW; }
  if (p->periodic & ~7u) { set_error("periodic takes bits 0 (x), 1 (y) and 2 (z) only"); return LBM_EINVAL; }
  if (!(p->tau_plus > 0.5)) { set_error("tau_plus must exceed 1/2"); return LBM_EINVAL; }
  if (!(p->magic_lambda > 0.0)) { set_error("magic_lambda must be positive"); return LBM_EINVAL; }
  if (p->layout != LBM_SOA && p->layout != LBM_AOS) { set_error("bad layout"); return LBM_EINVAL; }
  if (p->addressing != LBM_DIRECT && p->addressing != LBM_LIST && p->addressing != LBM_LIST_RIA) {
    set_error("bad addressing");
    return LBM_EINVAL;
  }
  if (p->storage < LBM_F64 || p->storage > LBM_F16_SHIFTED_SR) { set_error("bad storage"); return LBM_EINVAL; }
  if (p->bounce != LBM_FULLWAY && p->bounce != LBM_HALFWAY) { set_error("bad bounce"); return LBM_EINVAL; }
  if (is_list(*p) && p->bounce != LBM_HALFWAY) {
    set_error("list addressing requires half-way bounce-back");
    return LBM_EINVAL;
  }
  if (p->addressing == LBM_LIST_RIA && p->layout != LBM_SOA) {
    set_error("the run-length list requires the SOA layout");
    return LBM_EINVAL;
  }
  if ((p->storage == LBM_F16_SHIFTED || p->storage == LBM_F16_SHIFTED_SR) &&
      (p->f16_scale_log2 < 0 || p->f16_scale_log2 > 24)) {
    set_error("f16_scale_log2 must be in [0, 24]");
    return LBM_EINVAL;
  }
  if (p->block != 0 && (p->block < 64 || p->block > 1024 || p->block % 64 != 0)) {
    set_error("block must be 0 or a multiple of 64 in [64, 1024]");
    return LBM_EINVAL;
  }
  if (p->pad < -1 || p->pad > (1 << 24)) { set_error("pad must be -1 or in [0, 2^24]"); return LBM_EINVAL; }
  if (p->cu_slots < 0 || p->cu_slots > 64) { set_error("cu_slots must be in [0, 64]"); return LBM_EINVAL; }
  if (p->layout == LBM_AOS && p->addressing == LBM_DIRECT && p->propagation == LBM_OS &&
      (int64_t)p->nx * p->ny * Q > 0x7fffffffLL) {
    set_error("the AoS one-step pull needs nx*ny*19 < 2^31 (one layer's populations)");
    return LBM_EOVERFLOW;
  }
  if (p->propagation != LBM_OS && p->propagation != LBM_AA && p->propagation != LBM_OS_PUSH) {
    set_error("bad propagation");
    return LBM_EINVAL;
  }

  for (int a = 0; a < 3; ++a)
    if (!(p->g[a] == p->g[a]) || p->g[a] > 1e30 || p->g[a] < -1e30) { set_error("bad g"); return LBM_EINVAL; }
  return LBM_OK;
}

// Full-way bounce-back stores the populations that enter a solid node, so a
// wall face needs solid nodes to hold them: on every axis that does not wrap,
// both boundary layers must be solid.  The sweeps still wrap such an axis;
// only solid boundary nodes then exchange populations across it, and those
// never reach a fluid node, so the fluid sees walls at the faces.
static int check_faces(const lbm_params* p, const uint8_t* mask) {
  if (p->bounce != LBM_FULLWAY || p->periodic == 7u) return LBM_OK;
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const char* name = "xyz";
  for (int a = 0; a < 3; ++a) {
    if (p->periodic & (1u << a)) continue;
    const int n = a == 0 ? nx : (a == 1 ? ny : nz);
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int c = a == 0 ? x : (a == 1 ? y : z);
          if (c != 0 && c != n - 1) continue;
          if (mask[x + (int64_t)nx * (y + (int64_t)ny * z)] == 0) {
            set_error("full-way bounce-back with %c not periodic needs solid boundary layers %c = 0 "
                      "and %c = %d; node (%d, %d, %d) is fluid",
                      name[a], name[a], name[a], n - 1, x, y, z);
            return LBM_EINVAL;
          }
        }
  }
  return LBM_OK;
}

// Byte offsets of the run tables inside the ria buffer (layout in lbm_ctx).
struct RiaLayout {
  int64_t run_stride, start_off, adj_off, chunk_off, delta_off, bytes;
};

static RiaLayout ria_layout(int64_t n_runs, int64_t n_fluid) {
  RiaLayout L;
  L.run_stride = round_up(n_runs < 1 ? 1 : n_runs, 64);
  L.start_off = 0;
  L.adj_off = round_up((n_runs + 1) * 4, 256);
  L.chunk_off = L.adj_off + round_up((Q - 1) * L.run_stride * 4, 256);
  L.delta_off = L.chunk_off + round_up(((n_fluid + 63) / 64 + 1) * 4, 256);
  L.bytes = L.delta_off + round_up(n_fluid < 1 ? 1 : n_fluid, 256);
  return L;
}

// Runs of the run-length list.  List node m (x-fastest order) continues the
// run of m - 1 iff node m - 1 is its x-neighbour in the same row, neither
// pull source of the pair wraps around in x (2 <= x <= nx - 2), and for
// every direction the sources x - c_i of both nodes are both fluid or both
// solid: then each source slot of m is that of m - 1 plus one.  Fills
// is_start[m] when the pointer is given; returns the number of runs.
static int64_t find_runs(const lbm_params* p, const uint8_t* mask, uint8_t* is_start) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  int64_t runs = 0, m = 0;
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y) {
      const int64_t row = (int64_t)nx * (y + (int64_t)ny * z);
      // the nine source rows (y - c_y, z - c_z) of this row; NULL for a row
      // beyond a wall face (all of it counts as solid)
      const uint8_t* src_row[Q];
      for (int i = 0; i < Q; ++i) {
        const int ty = y - Vel::cy[i], tz = z - Vel::cz[i];
        const bool out = (!(p->periodic & 2u) && (ty < 0 || ty >= ny)) ||
                         (!(p->periodic & 4u) && (tz < 0 || tz >= nz));
        const int sy = (ty + ny) % ny, sz = (tz + nz) % nz;
        src_row[i] = out ? nullptr : mask + (int64_t)nx * (sy + (int64_t)ny * sz);
      }
      for (int x = 0; x < nx; ++x) {
        if (mask[row + x] != 0) continue;
        bool start = x < 2 || x > nx - 2 || mask[row + x - 1] != 0;
        for (int i = 1; i < Q && !start; ++i) {
          if (!src_row[i]) continue;
          const int sx = x - Vel::cx[i];
          start = (src_row[i][sx] != 0) != (src_row[i][sx - 1] != 0);
        }
        if (start) ++runs;
        if (is_start) is_start[m] = start ? 1 : 0;
        ++m;
      }
    }
  }
  return runs;
}

// Entries between the direction arrays of the list adjacency: the population
// stride for SOA, the fluid count padded to 64 for AOS records.
static int64_t list_adj_stride(const lbm_params* p, const lbm_sizes* s) {
  return p->layout == LBM_AOS ? round_up(s->n_sites < 1 ? 1 : s->n_sites, 64) : s->stride;
}

static int plan_sizes(const lbm_params* p, int64_t n_fluid, int64_t n_runs, lbm_sizes* s) {
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  if (N >= 0x7fffffffLL) { set_error("lattice of %lld nodes exceeds 32-bit node indices", (long long)N); return LBM_EOVERFLOW; }
  const int es = elem_size(p->storage);
  memset(s, 0, sizeof *s);
  s->n_nodes = N;
  s->n_fluid = n_fluid;
  s->n_sites = is_list(*p) ? n_fluid : N;
  if (p->layout == LBM_AOS) {
    s->stride = Q;
    s->pdf_bytes = round_up((s->n_sites < 1 ? 1 : s->n_sites) * Q * es, 256);
  } else {
    // Direction arrays start on 256-byte boundaries.  The automatic pad
    // shifts consecutive arrays by 1 KiB when their natural spacing is a
    // multiple of 64 KiB, so the 19 streams do not start on the same HBM
    // channel.
    const int64_t align = 256 / es;
    int64_t st = round_up(s->n_sites < 1 ? 1 : s->n_sites, align);
    if (p->pad >= 0) st += round_up(p->pad, align);
    else if ((st * es) % 65536 == 0) st += 1024 / es;
    s->stride = st;
    s->pdf_bytes = st * Q * es;
  }
  s->mask_bytes = round_up(N, 256);
  if (is_list(*p)) {
    const int64_t slots = p->layout == LBM_AOS ? s->n_sites * Q : s->stride * Q;
    if (slots >= 0x7fffffffLL) {
      set_error("list of %lld fluid nodes overflows int32 adjacency entries", (long long)n_fluid);
      return LBM_EOVERFLOW;
    }
    if (p->addressing == LBM_LIST) s->adj_bytes = round_up(list_adj_stride(p, s) * (Q - 1) * 4, 256);
    s->fluid_index_bytes = round_up((n_fluid < 1 ? 1 : n_fluid) * 4, 256);
    s->node_map_bytes = round_up(N * 4, 256);
  }
  if (p->addressing == LBM_LIST_RIA) {
    s->n_runs = n_runs;
    s->ria_bytes = ria_layout(n_runs, n_fluid).bytes;
  }
  const bool links = p->addressing == LBM_DIRECT && p->bounce == LBM_HALFWAY;
  if (links) s->links_bytes = round_up(N * 4, 256);
  s->u_prev_bytes = round_up(3 * (s->n_sites < 1 ? 1 : s->n_sites) * 8, 256);
  s->scratch_bytes = round_up((stat_records(*p) + kMaxReduceRecords + 1) * kStatSlots * 8, 256);
  // Algorithmic HBM bytes per site update: 19 loads + 19 stores of one
  // element, plus the flag byte (direct, full-way), the link word (direct,
  // half-way), 18 int32 adjacency entries (list) or, for the run-length
  // list, the run offset byte, the chunk word per 64 nodes and the run's
  // start and 18 entries once per run.
  // The AA pattern on the lists reads the addressing in the neighbour kernel
  // only: every other update (Table 1: 340 B/FLUP for the FP64 list).
  // On the full array, solid nodes move populations only where they store
  // them: the full-way pull and push sweeps reverse them; half-way sweeps
  // and the AA kernels read just the solid node's flag or link word.
  double addr = links ? 4.0 : 1.0;
  if (p->addressing == LBM_LIST) addr = 4.0 * (Q - 1);
  if (p->addressing == LBM_LIST_RIA)
    addr = 1.0 + 4.0 / 64 + (n_fluid > 0 ? 4.0 * Q * (double)n_runs / (double)n_fluid : 0.0);
  if (is_list(*p) && p->propagation == LBM_AA) addr *= 0.5;
  double moved = 2.0 * Q * es;
  const bool solids_move = p->bounce == LBM_FULLWAY && p->propagation != LBM_AA;
  if (!is_list(*p) && !solids_move && N > 0) moved *= (double)n_fluid / (double)N;
  s->bytes_per_update = moved + addr;
  return LBM_OK;
}

static int64_t count_fluid(const lbm_params* p, const uint8_t* mask) {
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  int64_t nf = 0;
  for (int64_t n = 0; n < N; ++n) nf += mask[n] == 0;
  return nf;
}

static bool aligned256(const void* ptr) { return ((uintptr_t)ptr & 255u) == 0; }

}  // namespace lbm

using namespace lbm;

extern "C" {

const char* lbm_last_error(void) { return g_err; }

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "success";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EOVERFLOW: return "lattice too large for 32-bit indices";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_ENONFINITE: return "non-finite populations";
    case LBM_ENOTCONV: return "not converged";
    default: return "unknown error";
  }
}

int lbm_plan(const lbm_params* params, const uint8_t* mask_host, lbm_sizes* out) {
  int rc = validate(params);
  if (rc) return rc;
  if (!mask_host || !out) { set_error("mask_host and out must be non-NULL"); return LBM_EINVAL; }
  const int64_t N = (int64_t)params->nx * params->ny * params->nz;
  if (N >= 0x7fffffffLL) { set_error("lattice too large"); return LBM_EOVERFLOW; }
  rc = check_faces(params, mask_host);
  if (rc) return rc;
  const int64_t runs = params->addressing == LBM_LIST_RIA ? find_runs(params, mask_host, nullptr) : 0;
  return plan_sizes(params, count_fluid(params, mask_host), runs, out);
}

int lbm_init_geometry(lbm_ctx** out, const lbm_params* params, const uint8_t* mask_host,
                      const lbm_buffers* bufs, void* stream) {
  if (!out) { set_error("out is NULL"); return LBM_EINVAL; }
  *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  if (!mask_host || !bufs) { set_error("mask_host and bufs must be non-NULL"); return LBM_EINVAL; }
  lbm_sizes s;
  const int64_t N = (int64_t)params->nx * params->ny * params->nz;
  if (N >= 0x7fffffffLL) { set_error("lattice too large"); return LBM_EOVERFLOW; }
  rc = check_faces(params, mask_host);
  if (rc) return rc;
  const bool ria = params->addressing == LBM_LIST_RIA;
  std::vector<uint8_t> run_starts;
  int64_t runs = 0;
  if (ria) {
    const int64_t nf = count_fluid(params, mask_host);
    try {
      run_starts.resize((size_t)(nf > 0 ? nf : 1));
    } catch (...) {
      set_error("host allocation failed");
      return LBM_ENOMEM;
    }
    runs = find_runs(params, mask_host, run_starts.data());
  }
  rc = plan_sizes(params, count_fluid(params, mask_host), runs, &s);
  if (rc) return rc;
  const bool two = params->propagation != LBM_AA;
  if (!bufs->pdf_a || (two && !bufs->pdf_b) || !bufs->mask || !bufs->scratch) {
    set_error("pdf_a, pdf_b (one-step propagation), mask and scratch are required");
    return LBM_EINVAL;
  }
  if (!aligned256(bufs->pdf_a) || (two && !aligned256(bufs->pdf_b))) {
    set_error("pdf buffers must be 256-byte aligned");
    return LBM_EINVAL;
  }
  if (params->addressing == LBM_LIST && (!bufs->adj || !bufs->fluid_index || !bufs->node_map)) {
    set_error("list addressing needs adj, fluid_index and node_map");
    return LBM_EINVAL;
  }
  if (ria && (!bufs->ria || !bufs->fluid_index || !bufs->node_map)) {
    set_error("run-length list addressing needs ria, fluid_index and node_map");
    return LBM_EINVAL;
  }
  if (s.links_bytes > 0 && !bufs->links) {
    set_error("direct addressing with half-way bounce-back needs the links buffer");
    return LBM_EINVAL;
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) { set_error("host allocation failed"); return LBM_ENOMEM; }
  c->p = *params;
  c->s = s;
  c->b = *bufs;
  if (params->addressing != LBM_LIST) c->b.adj = nullptr;
  if (!is_list(*params)) {
    c->b.fluid_index = nullptr;
    c->b.node_map = nullptr;
  }
  if (!ria) c->b.ria = nullptr;
  c->n_runs = runs;
  c->adj_stride = list_adj_stride(params, &s);
  if (ria) {
    const RiaLayout L = ria_layout(runs, s.n_fluid);
    char* base = (char*)c->b.ria;
    c->run_stride = L.run_stride;
    c->run_start = (int32_t*)(base + L.start_off);
    c->run_adj = (int32_t*)(base + L.adj_off);
    c->chunk_run = (int32_t*)(base + L.chunk_off);
    c->run_delta = (uint8_t*)(base + L.delta_off);
  }
  if (s.links_bytes == 0) c->b.links = nullptr;
  c->stream = (hipStream_t)stream;
  c->cur = 0;
  c->aa_odd = 0;
  c->step = 0;
  c->u_prev_valid = 0;
  // default workgroup size as measured: 512 (a row sweep covers a 512-node
  // row in one pass; on the 384^3 sphere pack the list and run-length push
  // ran 6-10% faster at 512 than at 128 or 256)
  c->block = params->block ? params->block : 512;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDevice"); }

  auto fail = [&](hipError_t err, const char* what) {
    delete c;
    return hip_fail(err, what);
  };
  e = hipMemcpyAsync(c->b.mask, mask_host, (size_t)N, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return fail(e, "mask upload");
  if (c->b.links) {
    e = launch_build_links(c);
    if (e != hipSuccess) return fail(e, "link words kernel");
  }
  if (is_list(*params)) {
    // Fluid-node vector and the node -> list map.  x-fastest order, except
    // for the AoS list: there consecutive list nodes share source records
    // (a record holds the populations bound for up to 9 neighbour rows), so
    // the list runs through columns of kListTile x kListTile nodes, each
    // listed x fastest, then y, then z through all layers; the consumers
    // of a record then sit close together in list order and find it in L2
    // (on MI355X, 384^3 sphere pack: pull 3.95 -> 3.36 ms, AA 5.18 -> 3.55,
    // push 7.33 -> 3.89).
    std::vector<int32_t> fidx, nmap;
    try {
      fidx.resize((size_t)(s.n_fluid > 0 ? s.n_fluid : 1));
      nmap.resize((size_t)N);
    } catch (...) {
      delete c;
      set_error("host allocation failed");
      return LBM_ENOMEM;
    }
    int32_t m = 0;
    if (params->addressing == LBM_LIST && params->layout == LBM_AOS) {
      const int nx = params->nx, ny = params->ny, nz = params->nz;
      for (int64_t n = 0; n < N; ++n) nmap[n] = -1;
      for (int y0 = 0; y0 < ny; y0 += kListTile)
        for (int x0 = 0; x0 < nx; x0 += kListTile)
          for (int z = 0; z < nz; ++z)
            for (int y = y0; y < y0 + kListTile && y < ny; ++y)
              for (int x = x0; x < x0 + kListTile && x < nx; ++x) {
                const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (mask_host[n] == 0) {
                  fidx[m] = (int32_t)n;
                  nmap[n] = m++;
                }
              }
    } else {
      for (int64_t n = 0; n < N; ++n) {
        if (mask_host[n] == 0) {
          fidx[m] = (int32_t)n;
          nmap[n] = m++;
        } else {
          nmap[n] = -1;
        }
      }
    }
    e = hipMemcpyAsync(c->b.fluid_index, fidx.data(), (size_t)s.n_fluid * 4, hipMemcpyHostToDevice,
                       c->stream);
    if (e != hipSuccess) return fail(e, "fluid index upload");
    e = hipMemcpyAsync(c->b.node_map, nmap.data(), (size_t)N * 4, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return fail(e, "node map upload");
    std::vector<int32_t> rstart, chunk;
    std::vector<uint8_t> delta;
    if (ria) {
      // run starts, the run of each 64-node chunk's first node and each
      // node's offset from it (a chunk holds at most 64 runs)
      const int64_t nf = s.n_fluid;
      try {
        rstart.resize((size_t)runs + 1);
        chunk.resize((size_t)((nf + 63) / 64 + 1));
        delta.resize((size_t)(nf > 0 ? nf : 1));
      } catch (...) {
        delete c;
        set_error("host allocation failed");
        return LBM_ENOMEM;
      }
      int64_t r = -1;
      for (int64_t k = 0; k < nf; ++k) {
        if (run_starts[k]) rstart[++r] = (int32_t)k;
        if (k % 64 == 0) chunk[k / 64] = (int32_t)r;
        delta[k] = (uint8_t)(r - chunk[k / 64]);
      }
      rstart[runs] = (int32_t)nf;
      e = hipMemcpyAsync(c->run_start, rstart.data(), (size_t)(runs + 1) * 4, hipMemcpyHostToDevice,
                         c->stream);
      if (e == hipSuccess && nf > 0)
        e = hipMemcpyAsync(c->chunk_run, chunk.data(), (size_t)((nf + 63) / 64) * 4,
                           hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess && nf > 0)
        e = hipMemcpyAsync(c->run_delta, delta.data(), (size_t)nf, hipMemcpyHostToDevice, c->stream);
      if (e != hipSuccess) return fail(e, "run table upload");
      e = launch_build_run_adj(c);
      if (e != hipSuccess) return fail(e, "run table kernel");
    } else {
      e = launch_build_adjacency(c);
      if (e != hipSuccess) return fail(e, "adjacency kernel");
    }
    // the host vectors are released below only after the copies completed
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(e, "adjacency sync");
  }
  e = launch_fill_rest(c, c->b.pdf_a);
  if (e != hipSuccess) return fail(e, "rest fill A");
  if (two) {
    e = launch_fill_rest(c, c->b.pdf_b);
    if (e != hipSuccess) return fail(e, "rest fill B");
  } else {
    c->b.pdf_b = nullptr;
  }
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(e, "init sync");
  *out = c;
  return LBM_OK;
}

int lbm_init_fields(lbm_ctx* c, const double* rho_dev, const double* u_dev) {
  if (!c) { set_error("ctx is NULL"); return LBM_EINVAL; }
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  c->aa_odd = 0;  // AA: equilibrium written in place (even phase)
  LBM_HIP(launch_init_fields(c, rho_dev, u_dev, pdf_buf(c, c->cur)), "init fields kernel");
  LBM_HIP(hipStreamSynchronize(c->stream), "init fields sync");
  c->step = 0;
  c->u_prev_valid = 0;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int32_t n) {
  if (!c || n < 0) { set_error("bad ctx or negative step count"); return LBM_EINVAL; }
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  for (int32_t k = 0; k < n; ++k) {
    const bool list_aos = is_list(c->p) && c->p.layout == LBM_AOS;
    if (c->p.propagation == LBM_AA) {
      hipError_t e = list_aos ? launch_list_aos(c, pdf_buf(c, 0), nullptr) : launch_aa(c, pdf_buf(c, 0));
      if (e != hipSuccess) return hip_fail(e, "AA sweep launch");
      c->aa_odd = 1 - c->aa_odd;
    } else {
      const void* src = pdf_buf(c, c->cur);
      void* dst = pdf_buf(c, 1 - c->cur);
      const bool ria = c->p.addressing == LBM_LIST_RIA;
      hipError_t e;
      if (list_aos) e = launch_list_aos(c, src, dst);
      else if (c->p.propagation == LBM_OS_PUSH) e = ria ? launch_push_ria(c, src, dst) : launch_push(c, src, dst);
      else if (ria) e = launch_pull_ria(c, src, dst);
      else if (c->p.layout == LBM_AOS) e = launch_pull_aos(c, src, dst);
      else e = launch_pull(c, src, dst);
      if (e != hipSuccess) return hip_fail(e, "sweep launch");
      c->cur = 1 - c->cur;
    }
    c->step += 1;
  }
  return LBM_OK;
}

static double* stats_stage(const lbm_ctx* c) {
  return (double*)c->b.scratch + stat_records(c->p) * kStatSlots;
}

static double* stats_result(const lbm_ctx* c) {
  return stats_stage(c) + kMaxReduceRecords * kStatSlots;
}

// Downloads the reduced moments, fills *out and advances the residual
// history; `step` is the update count of the state they describe.
static int finish_stats(lbm_ctx* c, int residual_mode, int64_t step, lbm_stats* out) {
  double r[kStatSlots];
  LBM_HIP(hipMemcpyAsync(r, stats_result(c), sizeof(double) * M_COUNT, hipMemcpyDeviceToHost,
                         c->stream),
          "stats download");
  LBM_HIP(hipStreamSynchronize(c->stream), "stats sync");
  out->mass = r[M_MASS];
  out->momentum[0] = r[M_PX];
  out->momentum[1] = r[M_PY];
  out->momentum[2] = r[M_PZ];
  out->u_max = r[M_UMAX];
  out->nonfinite = (int64_t)r[M_NONFINITE];
  out->residual = residual_mode == 2 ? (r[M_U2] > 0 ? sqrt(r[M_DU2] / r[M_U2]) : (r[M_DU2] > 0 ? INFINITY : 0.0)) : -1.0;
  out->step = step;
  if (residual_mode > 0) c->u_prev_valid = 1;
  if (out->nonfinite > 0) {
    set_error("%lld fluid nodes hold non-finite populations", (long long)out->nonfinite);
    return LBM_ENONFINITE;
  }
  return LBM_OK;
}

int lbm_macroscopic(lbm_ctx* c, double* rho_dev, double* u_dev, lbm_stats* out) {
  if (!c || !out) { set_error("ctx and out must be non-NULL"); return LBM_EINVAL; }
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  const int64_t N = c->s.n_nodes;
  if (rho_dev) LBM_HIP(hipMemsetAsync(rho_dev, 0, (size_t)N * 8, c->stream), "rho clear");
  if (u_dev) LBM_HIP(hipMemsetAsync(u_dev, 0, (size_t)N * 24, c->stream), "u clear");
  const int residual_mode = c->b.u_prev ? (c->u_prev_valid ? 2 : 1) : 0;
  double* partials = (double*)c->b.scratch;
  int64_t nb = 0;
  LBM_HIP(launch_moments(c, pdf_buf(c, c->cur), rho_dev, u_dev, residual_mode, partials, &nb),
          "moments kernel");
  LBM_HIP(launch_final_reduce(c, partials, nb, M_COUNT, 1u << M_UMAX, stats_result(c)),
          "reduce kernel");
  return finish_stats(c, residual_mode, c->step, out);
}

int lbm_step_diag(lbm_ctx* c, lbm_stats* out) {
  if (!c || !out) { set_error("ctx and out must be non-NULL"); return LBM_EINVAL; }
  if (!fused_diag_form(c->p)) {
    const int rc = lbm_macroscopic(c, nullptr, nullptr, out);
    if (rc != LBM_OK && rc != LBM_ENONFINITE) return rc;
    const int rs = lbm_step(c, 1);
    return rs != LBM_OK ? rs : rc;
  }
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  const int residual_mode = c->b.u_prev ? (c->u_prev_valid ? 2 : 1) : 0;
  double* partials = (double*)c->b.scratch;
  int64_t rows = 0;
  if (c->p.layout == LBM_SOA)
    LBM_HIP(launch_pull_diag(c, pdf_buf(c, c->cur), pdf_buf(c, 1 - c->cur), residual_mode,
                             partials, &rows),
            "fused sweep launch");
  else
    LBM_HIP(launch_pull_aos_diag(c, pdf_buf(c, c->cur), pdf_buf(c, 1 - c->cur), residual_mode,
                                 partials, &rows),
            "fused sweep launch");
  const int64_t described = c->step;
  c->cur = 1 - c->cur;
  c->step += 1;
  LBM_HIP(launch_reduce_records(c, partials, rows, M_COUNT, 1u << M_UMAX, stats_stage(c),
                                stats_result(c)),
          "reduce kernels");
  return finish_stats(c, residual_mode, described, out);
}

int lbm_verify(lbm_ctx* c, int32_t kind, const double* ref_dev, lbm_verify_result* out) {
  if (!c || !out) { set_error("ctx and out must be non-NULL"); return LBM_EINVAL; }
  if (kind != LBM_VERIFY_SLAB && kind != LBM_VERIFY_DUCT && kind != LBM_VERIFY_REFERENCE) {
    set_error("unknown verification kind %d", kind);
    return LBM_EINVAL;
  }
  if (kind == LBM_VERIFY_REFERENCE && !ref_dev) { set_error("reference field is NULL"); return LBM_EINVAL; }
  if (kind == LBM_VERIFY_SLAB && c->p.nz < 3) { set_error("slab needs nz >= 3"); return LBM_EINVAL; }
  if (kind == LBM_VERIFY_DUCT && (c->p.ny < 3 || c->p.nz < 3)) { set_error("duct needs ny, nz >= 3"); return LBM_EINVAL; }
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  double* partials = (double*)c->b.scratch;
  int64_t nb = 0;
  LBM_HIP(launch_verify(c, pdf_buf(c, c->cur), kind, ref_dev, partials, &nb), "verify kernel");
  double* res_dev = stats_result(c);
  LBM_HIP(launch_final_reduce(c, partials, nb, V_COUNT, (1u << V_MAXABS) | (1u << V_REFMAX), res_dev),
          "reduce kernel");
  double r[kStatSlots];
  LBM_HIP(hipMemcpyAsync(r, res_dev, sizeof(double) * V_COUNT, hipMemcpyDeviceToHost, c->stream),
          "verify download");
  LBM_HIP(hipStreamSynchronize(c->stream), "verify sync");
  out->max_abs = r[V_MAXABS];
  out->rel_l2 = r[V_REF2] > 0 ? sqrt(r[V_ERR2] / r[V_REF2]) : sqrt(r[V_ERR2]);
  out->ref_max = r[V_REFMAX];
  out->n_compared = (int64_t)r[V_COUNT_N];
  return LBM_OK;
}

int lbm_export_pdfs(lbm_ctx* c, const int64_t* node_ids_host, int64_t count, double* out_host) {
  if (!c || !out_host || count < 0) { set_error("bad arguments"); return LBM_EINVAL; }
  const int64_t N = c->s.n_nodes;
  if (!node_ids_host && count != N) { set_error("count must equal N when node_ids is NULL"); return LBM_EINVAL; }
  if (node_ids_host) {
    for (int64_t k = 0; k < count; ++k)
      if (node_ids_host[k] < 0 || node_ids_host[k] >= N) {
        set_error("node id %lld out of range", (long long)node_ids_host[k]);
        return LBM_EINVAL;
      }
  }
  if (count == 0) return LBM_OK;
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  const int64_t chunk = count < (int64_t)(1 << 22) ? count : (int64_t)(1 << 22);
  int64_t* ids_dev = nullptr;
  double* out_dev = nullptr;
  std::vector<int64_t> ids;
  try {
    ids.resize((size_t)chunk);
  } catch (...) {
    set_error("host allocation failed");
    return LBM_ENOMEM;
  }
  if (hipMalloc(&ids_dev, (size_t)chunk * 8) != hipSuccess ||
      hipMalloc(&out_dev, (size_t)chunk * Q * 8) != hipSuccess) {
    if (ids_dev) (void)hipFree(ids_dev);
    set_error("export scratch allocation failed");
    return LBM_ENOMEM;
  }
  int rc = LBM_OK;
  for (int64_t k0 = 0; k0 < count && rc == LBM_OK; k0 += chunk) {
    const int64_t m = (count - k0) < chunk ? (count - k0) : chunk;
    for (int64_t k = 0; k < m; ++k) ids[k] = node_ids_host ? node_ids_host[k0 + k] : k0 + k;
    hipError_t e = hipMemcpyAsync(ids_dev, ids.data(), (size_t)m * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_export(c, pdf_buf(c, c->cur), ids_dev, m, out_dev);
    if (e == hipSuccess)
      e = hipMemcpyAsync(out_host + k0 * Q, out_dev, (size_t)m * Q * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(e, "export");
  }
  (void)hipFree(ids_dev);
  (void)hipFree(out_dev);
  return rc;
}

int lbm_import_pdfs(lbm_ctx* c, const double* host_in) {
  if (!c || !host_in) { set_error("bad arguments"); return LBM_EINVAL; }
  LBM_HIP(hipSetDevice(c->device), "hipSetDevice");
  const size_t bytes = (size_t)c->s.n_nodes * Q * 8;
  double* canon = nullptr;
  if (hipMalloc(&canon, bytes) != hipSuccess) {
    set_error("import scratch allocation of %zu bytes failed", bytes);
    return LBM_ENOMEM;
  }
  hipError_t e = hipMemcpyAsync(canon, host_in, bytes, hipMemcpyHostToDevice, c->stream);
  c->aa_odd = 0;  // AA: the canonical state is written in place (even phase)
  if (e == hipSuccess) e = launch_import(c, canon, pdf_buf(c, c->cur));
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(canon);
  if (e != hipSuccess) return hip_fail(e, "import");
  c->u_prev_valid = 0;
  return LBM_OK;
}

int lbm_get_sizes(const lbm_ctx* c, lbm_sizes* out) {
  if (!c || !out) { set_error("bad arguments"); return LBM_EINVAL; }
  *out = c->s;
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

int lbm_current_buffer(const lbm_ctx* c) { return c ? c->cur : -1; }

void lbm_destroy(lbm_ctx* c) { delete c; }

int lbm_membench(int32_t kind, const double* a, double* b, int64_t n, int64_t stride, int32_t block,
                 void* stream) {
  if (kind < 0 || kind > 9 || !b || (kind != 3 && kind != 9 && !a) || n <= 0) { set_error("bad membench arguments"); return LBM_EINVAL; }
  if (kind != 0 && kind != 4 && stride < n) { set_error("stride must be >= n"); return LBM_EINVAL; }
  if (kind >= 4 && (n % 2 || stride % 2 || ((uintptr_t)a | (uintptr_t)b) % 16)) {
    set_error("membench kinds 4-9 need even n and stride and 16-byte aligned arrays");
    return LBM_EINVAL;
  }
  if (block < 64 || block > 1024 || block % 64) { set_error("bad block"); return LBM_EINVAL; }
  LBM_HIP(launch_membench(kind, a, b, n, stride, block, (hipStream_t)stream), "membench launch");
  return LBM_OK;
}

}  // extern "C"
