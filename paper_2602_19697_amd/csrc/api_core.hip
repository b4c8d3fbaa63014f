// Context, error plumbing, allocation and object views of the C ABI.
#include "bf_internal.h"

#include <vector>

#include <cstdlib>
#include <cstring>

bf_status bf_fail(bf_ctx* ctx, bf_status st, const char* fmt, ...) {
  if (ctx) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
    va_end(ap);
  }
  return st;
}

int bf_mixed_restart() {
  const char* v = getenv("BF_MIXED_RESTART");
  if (!v) return 0;
  const int x = atoi(v);
  return x < 0 ? 0 : x;
}

bf_status bf_dev_alloc(bf_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return BF_OK;
  hipError_t e = hipMallocFromPoolAsync(p, bytes, ctx->mempool, ctx->stream);
  if (e != hipSuccess) {
    *p = nullptr;
    return bf_fail(ctx, BF_ERR_OOM, "device allocation of %zu bytes failed: %s", bytes,
                   hipGetErrorString(e));
  }
  return BF_OK;
}

static void carve(char* base, std::initializer_list<bf_part> parts) {
  size_t off = 0;
  for (const bf_part& q : parts) {
    *q.p = q.bytes ? base + off : nullptr;
    off += (q.bytes + 255) / 256 * 256;
  }
}

static size_t parts_bytes(std::initializer_list<bf_part> parts) {
  size_t total = 0;
  for (const bf_part& q : parts) total += (q.bytes + 255) / 256 * 256;
  return total;
}

bf_status bf_dev_alloc_parts(bf_ctx* ctx, void** block, std::initializer_list<bf_part> parts) {
  char* base = nullptr;
  BF_TRY(bf_dev_alloc(ctx, (void**)&base, parts_bytes(parts)));
  *block = base;
  carve(base, parts);
  return BF_OK;
}

void bf_dev_free(bf_ctx* ctx, void* p) {
  if (p) (void)hipFreeAsync(p, ctx->stream);
}

bf_status bf_obj_alloc(bf_ctx* ctx, void** p, size_t bytes) {
  if (!ctx->objalloc.alloc) return bf_dev_alloc(ctx, p, bytes);
  *p = nullptr;
  if (bytes == 0) return BF_OK;
  *p = ctx->objalloc.alloc(ctx->objalloc.user, bytes, (void*)ctx->stream);
  if (!*p) return bf_fail(ctx, BF_ERR_OOM, "the caller's allocator returned no memory for %zu bytes", bytes);
  return BF_OK;
}

bf_status bf_obj_alloc_parts(bf_ctx* ctx, void** block, std::initializer_list<bf_part> parts) {
  char* base = nullptr;
  BF_TRY(bf_obj_alloc(ctx, (void**)&base, parts_bytes(parts)));
  *block = base;
  carve(base, parts);
  return BF_OK;
}

void bf_obj_free(bf_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->objalloc.release) ctx->objalloc.release(ctx->objalloc.user, p, (void*)ctx->stream);
  else bf_dev_free(ctx, p);
}

bf_status bf_ws(bf_ctx* ctx, int slot, size_t bytes, void** out) {
  if (ctx->ws_bytes[slot] < bytes) {
    bf_dev_free(ctx, ctx->ws[slot]);
    ctx->ws[slot] = nullptr;
    ctx->ws_bytes[slot] = 0;
    size_t want = bytes + bytes / 8 + 4096;
    BF_TRY(bf_dev_alloc(ctx, &ctx->ws[slot], want));
    ctx->ws_bytes[slot] = want;
  }
  *out = ctx->ws[slot];
  return BF_OK;
}

bf_status bf_pinned(bf_ctx* ctx, size_t bytes, void** out) {
  if (ctx->pinned_bytes < bytes) {
    if (ctx->pinned) {
      BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
      BF_HIP(ctx, hipHostFree(ctx->pinned));
    }
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    size_t want = bytes < 4096 ? 4096 : bytes;
    BF_HIP(ctx, hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_bytes = want;
  }
  *out = ctx->pinned;
  return BF_OK;
}

bf_status bf_launch_check(bf_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bf_fail(ctx, BF_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return BF_OK;
}

hipEvent_t bf_event_get(bf_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void bf_timing_add(bf_ctx* ctx, const char* name, hipEvent_t start, hipEvent_t stop) {
  ctx->recs.push_back({name, start, stop, 0});
}

void bf_timing_mark_idle(bf_ctx* ctx, size_t from, size_t to) {
  for (size_t i = from; i < to && i < ctx->recs.size(); ++i) ctx->recs[i].idle = 1;
}

extern "C" {

bf_status bf_set_timing(bf_ctx* ctx, int32_t enable) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  ctx->timing = enable ? 1 : 0;
  return BF_OK;
}

bf_status bf_get_timings(bf_ctx* ctx, bf_kernel_time* out, int32_t cap, int32_t* n_out) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, n_out && (cap == 0 || out), "bf_get_timings: NULL argument");
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int32_t n = 0;
  for (auto& r : ctx->recs) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    char name[sizeof(out[0].name)];
    snprintf(name, sizeof(name), "%s%s", r.name, r.idle ? "_idle" : "");
    int32_t slot = -1;
    for (int32_t i = 0; i < n && i < cap; ++i)
      if (strncmp(out[i].name, name, sizeof(out[i].name)) == 0) slot = i;
    if (slot < 0 && n < cap) {
      slot = n++;
      memset(&out[slot], 0, sizeof(bf_kernel_time));
      strncpy(out[slot].name, name, sizeof(out[slot].name) - 1);
    }
    if (slot >= 0) {
      out[slot].launches += 1;
      out[slot].total_ms += ms;
    }
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.clear();
  *n_out = n;
  return BF_OK;
}

const char* bf_version(void) { return "bayesfusion-gfx950 0.1"; }

bf_status bf_create(bf_ctx** out, int32_t device, void* hip_stream, const bf_allocator* alloc) {
  if (!out) return BF_ERR_INVALID_ARG;
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->release)) return BF_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return BF_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return BF_ERR_HIP;
  bf_ctx* ctx = new (std::nothrow) bf_ctx();
  if (!ctx) return BF_ERR_OOM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (alloc) ctx->objalloc = *alloc;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->cu_count = prop.multiProcessorCount;
  hipMemPoolProps pp;
  memset(&pp, 0, sizeof(pp));
  pp.allocType = hipMemAllocationTypePinned;
  pp.handleTypes = hipMemHandleTypeNone;
  pp.location.type = hipMemLocationTypeDevice;
  pp.location.id = device;
  uint64_t keep = UINT64_MAX;
  if (hipMemPoolCreate(&ctx->mempool, &pp) != hipSuccess ||
      hipMemPoolSetAttribute(ctx->mempool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
    if (ctx->mempool) (void)hipMemPoolDestroy(ctx->mempool);
    delete ctx;
    return BF_ERR_HIP;
  }
  if (bf_pcg_scratch_init(ctx) != BF_OK) {
    fprintf(stderr, "bf_create: %s\n", ctx->err);
    (void)hipMemPoolDestroy(ctx->mempool);
    delete ctx;
    return BF_ERR_HIP;
  }
  *out = ctx;
  return BF_OK;
}

bf_status bf_destroy(bf_ctx* ctx) {
  if (!ctx) return BF_OK;
  (void)hipSetDevice(ctx->device);
  for (int s = 0; s < bf_ctx::WS_COUNT; ++s) bf_dev_free(ctx, ctx->ws[s]);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  // Allocations still held by bands or systems keep the pool alive until
  // they are freed; everything else returns to the device here.
  (void)hipMemPoolDestroy(ctx->mempool);
  delete ctx;
  return BF_OK;
}

bf_status bf_set_stream(bf_ctx* ctx, void* hip_stream) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return BF_OK;
}

const char* bf_last_error(const bf_ctx* ctx) { return ctx ? ctx->err : "null context"; }

bf_status bf_band_view(const bf_band* band, bf_band_arrays* out) {
  if (!band || !out) return BF_ERR_INVALID_ARG;
  out->n = band->n;
  out->dense_side = band->P;
  out->keys = band->keys;
  out->tsdf = band->tsdf;
  out->w = band->w;
  out->nbr = band->nbr;
  out->deg = band->deg;
  out->dense_tsdf = band->dense_tsdf;
  out->dense_w = band->dense_w;
  out->tsdf_voxel_views = band->tsdf_voxel_views;
  out->tsdf_box_tests = band->tsdf_box_tests;
  out->tsdf_tile_tests = band->tsdf_tile_tests;
  return BF_OK;
}

bf_status bf_band_free(bf_ctx* ctx, bf_band* band) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  if (!band) return BF_OK;
  bf_obj_free(ctx, band->block);
  bf_obj_free(ctx, band->dense_tsdf);
  bf_obj_free(ctx, band->dense_w);
  delete band;
  return BF_OK;
}

bf_status bf_system_view(const bf_system* sys, bf_system_arrays* out) {
  if (!sys || !out) return BF_ERR_INVALID_ARG;
  out->n = sys->n;
  out->Lambda = sys->Lambda;
  out->b = sys->b;
  out->rhs = sys->rhs;
  out->diag = sys->diag;
  out->diag32 = sys->diag32;
  out->acc = sys->acc;
  out->kind = sys->kind;
  out->off = sys->off;
  out->nb26 = sys->nb26;
  out->n_samples = sys->n_samples;
  out->n_cells = sys->n_cells;
  return BF_OK;
}

bf_status bf_system_free(bf_ctx* ctx, bf_system* sys) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  if (!sys) return BF_OK;
  bf_obj_free(ctx, sys->block);
  delete sys;
  return BF_OK;
}

}  // extern "C"
