// Context, errors, scratch memory and device-wide scans.
#include <cstdarg>
#include <cstring>

#include "internal.h"

gf_status set_error(gf_ctx *ctx, gf_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

extern "C" const char *gf_version(void) { return "gfdm-mi355x 0.1 (gfx950)"; }

extern "C" gf_status gf_create(int device, void *stream, gf_ctx **out) {
  if (!out) return GF_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GF_EINVAL;
  gf_ctx *ctx = new gf_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return GF_EHIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
  const gf_status st = fixed_scratch_init(ctx);
  if (st != GF_OK) { delete ctx; return st; }
  *out = ctx;
  return GF_OK;
}

extern "C" gf_status gf_set_stream(gf_ctx *ctx, void *stream) {
  if (!ctx) return GF_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  if (s == ctx->stream) return GF_OK;
  // Every call of a context uses its scratch arena, so work enqueued on the
  // new stream must not overtake what the context enqueued on the old one:
  // the new stream waits for an event recorded on the old stream.  (Not
  // while the new stream is being captured into a graph: a captured stream
  // cannot wait on work outside the capture; the caller orders it.)
  GF_HIP(ctx, hipSetDevice(ctx->device));
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  GF_HIP(ctx, hipStreamIsCapturing(s, &cap));
  if (cap == hipStreamCaptureStatusNone) {
    if (!ctx->stream_order) GF_HIP(ctx, hipEventCreateWithFlags(&ctx->stream_order, hipEventDisableTiming));
    GF_HIP(ctx, hipEventRecord(ctx->stream_order, ctx->stream));
    GF_HIP(ctx, hipStreamWaitEvent(s, ctx->stream_order, 0));
  }
  ctx->stream = s;
  return GF_OK;
}

extern "C" void gf_destroy(gf_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->scratch) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->scratch);
  }
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  if (ctx->stream_order) (void)hipEventDestroy(ctx->stream_order);
  for (auto &r : ctx->prof_pending) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
  delete ctx;
}

static hipEvent_t prof_event(gf_ctx *ctx) {
  if (!ctx->prof_pool.empty()) {
    hipEvent_t e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(gf_ctx *c, const char *name, hipStream_t s) : ctx(c), sm(s ? s : (c ? c->stream : nullptr)) {
  if (!ctx || !ctx->profile) return;
  gf_ctx::ProfRec r;
  r.name = name;
  r.start = prof_event(ctx);
  r.stop = prof_event(ctx);
  if (!r.start || !r.stop) return;
  (void)hipEventRecord(r.start, sm);
  idx = (int)ctx->prof_pending.size();
  ctx->prof_pending.push_back(r);
}

ProfScope::~ProfScope() {
  if (idx >= 0) (void)hipEventRecord(ctx->prof_pending[idx].stop, sm);
}

extern "C" gf_status gf_set_tile_capacity(gf_ctx *ctx, int entries) {
  if (!ctx) return GF_EINVAL;
  ctx->tile_cap = entries > 0 ? entries : 0;
  return GF_OK;
}

extern "C" gf_status gf_profile_enable(gf_ctx *ctx, int on) {
  if (!ctx) return GF_EINVAL;
  ctx->profile = on ? 1 : 0;
  return GF_OK;
}

extern "C" gf_status gf_profile_read(gf_ctx *ctx, char *buf, size_t len) {
  if (!ctx || !buf || len == 0) return GF_EINVAL;
  std::vector<std::string> names;
  std::vector<double> total;
  std::vector<long> count;
  for (auto &r : ctx->prof_pending) {
    float ms = 0.0f;
    (void)hipEventSynchronize(r.stop);
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) ms = 0.0f;
    size_t k = 0;
    while (k < names.size() && names[k] != r.name) ++k;
    if (k == names.size()) { names.push_back(r.name); total.push_back(0.0); count.push_back(0); }
    total[k] += ms;
    count[k] += 1;
    ctx->prof_pool.push_back(r.start);
    ctx->prof_pool.push_back(r.stop);
  }
  ctx->prof_pending.clear();
  std::string out;
  char line[256];
  for (size_t k = 0; k < names.size(); ++k) {
    snprintf(line, sizeof(line), "%s %ld %.6f\n", names[k].c_str(), count[k], total[k]);
    out += line;
  }
  if (out.size() + 1 > len) return set_error(ctx, GF_ECAPACITY, "profile buffer too small");
  memcpy(buf, out.c_str(), out.size() + 1);
  return GF_OK;
}

extern "C" const char *gf_last_error(const gf_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

size_t arena_bytes(const std::vector<size_t> &sizes) {
  size_t t = 0;
  for (size_t s : sizes) t += ((s + 255) & ~size_t(255)) + 256;
  return t;
}

gf_status ensure_scratch(gf_ctx *ctx, size_t bytes, Arena *arena) {
  if (bytes > ctx->scratch_bytes) {
    if (ctx->scratch) {
      GF_HIP(ctx, hipStreamSynchronize(ctx->stream));
      GF_HIP(ctx, hipFree(ctx->scratch));
      ctx->scratch = nullptr;
      ctx->scratch_bytes = 0;
    }
    size_t want = bytes + bytes / 4 + (1 << 20);
    if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
      ctx->scratch = nullptr;
      return set_error(ctx, GF_ENOMEM, "scratch allocation of %zu bytes failed", want);
    }
    ctx->scratch_bytes = want;
  }
  arena->base = (char *)ctx->scratch;
  arena->off = 0;
  return GF_OK;
}

gf_status ensure_host(gf_ctx *ctx, size_t bytes) {
  if (bytes > ctx->host_pinned_bytes) {
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    ctx->host_pinned = nullptr;
    ctx->host_pinned_bytes = 0;
    if (hipHostMalloc(&ctx->host_pinned, bytes, 0) != hipSuccess) {
      ctx->host_pinned = nullptr;
      return set_error(ctx, GF_ENOMEM, "pinned host allocation failed");
    }
    ctx->host_pinned_bytes = bytes;
  }
  return GF_OK;
}

gf_status check_particles(gf_ctx *ctx, const gf_particles *p, bool need_kind, bool need_normals) {
  if (!ctx) return GF_EINVAL;
  if (!p) return set_error(ctx, GF_EINVAL, "particles is NULL");
  if (p->n <= 0) return set_error(ctx, GF_EINVAL, "particle count must be positive (got %lld)", (long long)p->n);
  if (p->n >= (int64_t)0x7fffffff) return set_error(ctx, GF_ECAPACITY, "at most 2^31-2 particles");
  if (!p->x || !p->y || !p->z || !p->h || !p->model)
    return set_error(ctx, GF_EINVAL, "x, y, z, h and model are required");
  if (need_kind && !p->kind) return set_error(ctx, GF_EINVAL, "kind is required by this call");
  if (need_normals && (!p->nx || !p->ny || !p->nz))
    return set_error(ctx, GF_EINVAL, "normals are required by this call");
  GF_HIP(ctx, hipSetDevice(ctx->device));
  return GF_OK;
}

gf_status check_nbr(gf_ctx *ctx, const gf_nbr *nbr, int64_t n) {
  if (!nbr) return set_error(ctx, GF_EINVAL, "neighbour handle is NULL");
  if (nbr->n != n)
    return set_error(ctx, GF_EINVAL, "neighbour handle built for %lld particles, call has %lld",
                     (long long)nbr->n, (long long)n);
  if (nbr->device != ctx->device) return set_error(ctx, GF_EINVAL, "neighbour handle is on another device");
  return GF_OK;
}

// ------------------------------------------------------------------ scans
// 256 threads per block, 4 consecutive items per thread.
namespace {
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T *total) {
  __shared__ T wsum[kScanBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanBlock) k_scan_partials(const TI *in, int64_t n, TO *bsum) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += (TO)in[base + k];
  TO tot;
  block_exclusive_scan<TO>(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb block sums in place by one block; bsum[nb] = total
template <typename TO>
__global__ void __launch_bounds__(kScanBlock) k_scan_single(TO *bsum, int64_t nb) {
  TO carry = 0;
  for (int64_t c = 0; c < nb; c += kScanTile) {
    int64_t base = c + (int64_t)threadIdx.x * kScanItems;
    TO v[kScanItems];
    TO s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (base + k < nb) ? bsum[base + k] : (TO)0;
      s += v[k];
    }
    TO tot;
    TO off = block_exclusive_scan<TO>(s, &tot);
    TO run = carry + off;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < nb) bsum[base + k] = run;
      run += v[k];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const TI *in, int64_t n, const TO *bsum,
                                                           int64_t nb, TO *out) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO v[kScanItems];
  TO s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? (TO)in[base + k] : (TO)0;
    s += v[k];
  }
  TO tot;
  TO run = bsum[blockIdx.x] + block_exclusive_scan<TO>(s, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

template <typename TI, typename TO>
gf_status scan_impl(gf_ctx *ctx, const TI *in, TO *out, int64_t n, TO *tmp) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_scan_partials<TI, TO>), dim3((unsigned)nb), dim3(kScanBlock), 0, ctx->stream,
                     in, n, tmp);
  GF_LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL((k_scan_single<TO>), dim3(1), dim3(kScanBlock), 0, ctx->stream, tmp, nb);
  GF_LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nb), dim3(kScanBlock), 0, ctx->stream,
                     in, n, tmp, nb, out);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}
}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile + 2); }

gf_status scan_i32_to_i64(gf_ctx *ctx, const int32_t *in, int64_t *out, int64_t n, int64_t *tmp) {
  return scan_impl<int32_t, int64_t>(ctx, in, out, n, tmp);
}
gf_status scan_i32_to_i32(gf_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *tmp) {
  return scan_impl<int32_t, int32_t>(ctx, in, out, n, tmp);
}

extern "C" gf_status gf_set_team_sizes(gf_ctx *ctx, const int *teams, int *previous) {
  if (!ctx) return GF_EINVAL;
  int (*const tab[3])[GF_NBAND] = {ctx->wteam, ctx->ateam, ctx->fteam};
  if (teams) {
    for (int q = 0; q < 3 * 2 * GF_NBAND; ++q) {
      const int t = teams[q];
      const bool apply = q / (2 * GF_NBAND) == 1;
      const bool ok = t == 0 || t == 4 || t == 8 || t == 16 || (apply && (t == 32 || t == 64));
      if (!ok)
        return set_error(ctx, GF_EINVAL, "team size %d at position %d (stencil and fused kernels: 4, 8 or 16; "
                         "application: 4, 8, 16, 32 or 64; 0 keeps the current size)", t, q);
    }
  }
  for (int q = 0; q < 3 * 2 * GF_NBAND; ++q) {
    const int k = q / (2 * GF_NBAND), g = q % (2 * GF_NBAND);
    int &slot = tab[k][g / GF_NBAND][g % GF_NBAND];
    if (previous) previous[q] = slot;
    if (teams && teams[q] > 0) slot = teams[q];
  }
  return GF_OK;
}
