// Internal declarations of the gfdm library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/gfdm.h"

struct gf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  std::string err;
  // grow-only scratch arena (device); carved per call, valid until the next
  // call on this context
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  // device address of the library's fixed workspace on this context's device
  // (used by the entry points that allocate nothing); set by gf_create
  void *fixed_scratch = nullptr;
  // orders the context's work across gf_set_stream (the calls share scratch)
  hipEvent_t stream_order = nullptr;
  // small pinned host buffer for read-backs
  void *host_pinned = nullptr;
  size_t host_pinned_bytes = 0;
  // team sizes (lanes per particle) of the batched stencil and application
  // kernels per (model, neighbour-count band); set by gf_autotune
  int wteam[2][4] = {{8, 8, 8, 16}, {8, 8, 8, 16}};
  int fteam[2][4] = {{8, 8, 8, 16}, {8, 8, 8, 16}};  // fused stencil + application kernel
  int ateam[2][4] = {{4, 8, 8, 16}, {4, 8, 8, 16}};
  // LDS staging limit of the tile kernels (gf_set_tile_capacity); 0 = their own
  int tile_cap = 0;
  // optional per-kernel timing with HIP events (gf_profile_enable)
  int profile = 0;
  struct ProfRec {
    const char *name;
    hipEvent_t start, stop;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
};

// Brackets a kernel launch with events on the given stream (default: the
// context stream) when profiling is enabled (names must be string literals).
struct ProfScope {
  gf_ctx *ctx;
  hipStream_t sm;
  int idx = -1;
  ProfScope(gf_ctx *c, const char *name, hipStream_t s = nullptr);
  ~ProfScope();
};


// Row groups of the batched kernels: particles of one model whose neighbour
// count falls in one band, in Morton (cell) order.
enum { GF_NBAND = 4 };
static const int kBandHi[GF_NBAND] = {24, 48, 128, 1 << 30};

struct gf_nbr {
  int device = 0;
  int64_t n = 0;
  int64_t nnz = 0;
  int32_t max_row = 0;
  int cross = 0;
  int64_t *row_ptr = nullptr;  // [n+1]
  int32_t *col = nullptr;      // [nnz]
  int32_t *order = nullptr;    // [n] particles in cell (Morton) order
  int32_t *grouped = nullptr;  // [n] particles grouped by (model, band), Morton order inside
  int64_t group_start[2 * GF_NBAND + 1] = {0};  // host copy of the group offsets
  int32_t *rev = nullptr;      // [nnz] position of (j,i) for entry (i,j); built lazily
  // rows in grouped (Morton) order, built lazily: grow_ptr[t] = entries of the
  // rows grouped[0..t), gpos[i] = position of particle i in grouped
  int64_t *grow_ptr = nullptr; // [n+1]
  int32_t *gpos = nullptr;     // [n]
  // grev[g]: position, in the grouped layout, of the twin (j, i) of the entry
  // (i, j) at grouped position g; -1 for self entries and missing twins
  int32_t *grev = nullptr;     // [nnz]
  // Neighbour tiles: per model, the rows of the bands 0..kTileBand (at most
  // kTileBandRow neighbours; one contiguous range of the grouped order) are
  // cut, in that order, into tiles of kTileRows rows.  tile_u holds, per
  // tile, the sorted distinct neighbour indices of its rows (tile t owns
  // tile_u[tile_off[t] .. tile_off[t+1])); slot[k] is the position of col[k]
  // in its row's tile list.  Kernels stage a tile's list in LDS once and
  // address it through slot[].
  uint16_t *slot = nullptr;    // [nnz]
  int32_t *tile_u = nullptr;   // [tile_off[ntiles]]
  int64_t *tile_off = nullptr; // [ntiles + 1]
  int64_t ntiles = 0;
  int64_t tile_start[3] = {0};  // host: tiles of model m are [tile_start[m], tile_start[m+1])
  int32_t tile_max[2] = {0};    // host: largest tile list of each model
};
constexpr int kTileRows = 32;
constexpr int kTileBand = 2;                   // bands 0..kTileBand are tiled
constexpr int kTileBandRow = 128;              // = kBandHi[kTileBand]
// entries of padding after the slot array (and the solver's matrix values),
// so that the SpMV can read a row's entries in aligned groups of four
constexpr int kQuadPad = 4;

// Launch units of the batched kernels: per model, the tiled rows (bands
// 0..kTileBand) and each untiled band.  Team sizes live in
// ctx->wteam/fteam/ateam[model][band] (band = kTileBand for the tiled unit).
// staging capacity of a tile kernel with its own limit `own`
inline int tile_capacity(const gf_ctx *ctx, int own) { return (ctx && ctx->tile_cap > 0 && ctx->tile_cap < own) ? ctx->tile_cap : own; }

struct LaunchUnit {
  int model, band;
  bool tiled;
  int64_t row0, nrows;    // range of gf_nbr::grouped
  int64_t tile0, ntiles;  // tiled units: their tiles
  int tile_max;
};
inline int launch_units(const gf_nbr *nb, LaunchUnit *out) {
  int k = 0;
  for (int m = 0; m < 2; ++m) {
    const int64_t r0 = nb->group_start[m * GF_NBAND], r1 = nb->group_start[m * GF_NBAND + kTileBand + 1];
    if (r1 > r0) {
      out[k].model = m; out[k].band = kTileBand; out[k].tiled = nb->tile_start[m + 1] > nb->tile_start[m];
      out[k].row0 = r0; out[k].nrows = r1 - r0;
      out[k].tile0 = nb->tile_start[m]; out[k].ntiles = nb->tile_start[m + 1] - nb->tile_start[m];
      out[k].tile_max = nb->tile_max[m];
      ++k;
    }
    for (int band = kTileBand + 1; band < GF_NBAND; ++band) {
      const int g = m * GF_NBAND + band;
      if (nb->group_start[g + 1] <= nb->group_start[g]) continue;
      out[k].model = m; out[k].band = band; out[k].tiled = false;
      out[k].row0 = nb->group_start[g]; out[k].nrows = nb->group_start[g + 1] - nb->group_start[g];
      out[k].tile0 = 0; out[k].ntiles = 0; out[k].tile_max = 0;
      ++k;
    }
  }
  return k;
}

// ------------------------------------------------------------------ new particles
// device view of a gf_new_particles output (entry points that create particles)
struct NewOut {
  double *x, *y, *z, *h;
  int8_t *model, *kind;
  double *nx, *ny, *nz;
  double *mass, *rho, *phi;
  double *height, *diam;
  int32_t *src;
  int64_t cap;
};

inline NewOut new_out(const gf_new_particles *o) {
  NewOut r;
  r.x = o->x; r.y = o->y; r.z = o->z; r.h = o->h;
  r.model = o->model; r.kind = o->kind;
  r.nx = o->nx; r.ny = o->ny; r.nz = o->nz;
  r.mass = o->mass; r.rho = o->rho; r.phi = o->phi;
  r.height = o->height; r.diam = o->diam; r.src = o->src;
  r.cap = o->cap;
  return r;
}
// argument check of a gf_new_particles output with nphi fields and its count
gf_status check_out(gf_ctx *ctx, const gf_new_particles *o, int nphi, int64_t *count);

// ------------------------------------------------------------------ errors
gf_status set_error(gf_ctx *ctx, gf_status st, const char *fmt, ...);

#define GF_HIP(ctx, call)                                                          \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return set_error((ctx), GF_EHIP, "%s failed: %s (%s:%d)", #call,            \
                       hipGetErrorString(e_), __FILE__, __LINE__);                 \
  } while (0)

#define GF_LAUNCH_CHECK(ctx) GF_HIP(ctx, hipGetLastError())

// ------------------------------------------------------------------ scratch
struct Arena {
  char *base = nullptr;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    size_t a = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(base + a);
    off = a + count * sizeof(T);
    return p;
  }
};
size_t arena_bytes(const std::vector<size_t> &sizes);
// looks up (once per device, with the device current) the address of the
// fixed workspace used by gf_gfdm_weights_apply_noalloc and stores it in ctx
gf_status fixed_scratch_init(gf_ctx *ctx);
gf_status ensure_scratch(gf_ctx *ctx, size_t bytes, Arena *arena);
gf_status ensure_host(gf_ctx *ctx, size_t bytes);

// validation of a particle struct against a neighbour handle
gf_status check_particles(gf_ctx *ctx, const gf_particles *p, bool need_kind, bool need_normals);
gf_status check_nbr(gf_ctx *ctx, const gf_nbr *nbr, int64_t n);
gf_status ensure_rev(gf_ctx *ctx, gf_nbr *nbr);
// grouped row offsets, positions and twin map (needs the reverse-edge map)
gf_status ensure_grouped_rows(gf_ctx *ctx, gf_nbr *nbr);
gf_status tune_apply(gf_ctx *ctx, const gf_nbr *nbr, const void *w, gf_dtype wtype);

// device-wide exclusive scans (in place allowed): out[k] = sum_{t<k} in[t],
// out[n] = total.  tmp must hold scan_tmp_elems(n) elements of the output type.
size_t scan_tmp_elems(int64_t n);
gf_status scan_i32_to_i64(gf_ctx *ctx, const int32_t *in, int64_t *out, int64_t n, int64_t *tmp);
gf_status scan_i32_to_i32(gf_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *tmp);

static inline unsigned grid_for(int64_t work_items, int block) {
  int64_t g = (work_items + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (unsigned)g;
}

// support weight parameters shared by the stencil kernels
struct WeightFn {
  double alpha, ea, inv_den;  // e^{-a}, 1/(1 - e^{-a})
  double nl2a;                // -a log2(e)
};
static inline WeightFn make_weight_fn(double alpha) {
  WeightFn f;
  f.alpha = alpha;
  f.ea = std::exp(-alpha);
  f.inv_den = 1.0 / (1.0 - f.ea);
  f.nl2a = -alpha * 1.4426950408889634;
  return f;
}
