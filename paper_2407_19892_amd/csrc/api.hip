// Context, errors, workspace and synchronisation of the C ABI.
#include <rocblas/rocblas.h>

#include "gmgm_internal.h"

gmgm_status set_err(gmgm_ctx* c, gmgm_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

gmgm_status hip_err(gmgm_ctx* c, hipError_t e, const char* what) {
  return set_err(c, e == hipErrorOutOfMemory ? GMGM_E_NOMEM : GMGM_E_HIP, "%s: %s", what,
                 hipGetErrorString(e));
}

gmgm_status ws_get(gmgm_ctx* c, int slot, size_t bytes, void** out) {
  if (slot < 0 || slot >= WS_COUNT) return set_err(c, GMGM_E_ARG, "bad workspace slot");
  if (c->arena) {
    // fixed arena: slots are carved from it for the duration of one call and
    // nothing is allocated; a slot asked for again with no more bytes keeps
    // its region (so data left in it by an earlier stage stays valid)
    if (c->arena_slots.size() < WS_COUNT) c->arena_slots.resize(WS_COUNT);
    DevBuf& a = c->arena_slots[slot];
    if (bytes == 0) bytes = 256;
    if (!a.ptr || a.bytes < bytes) {
      const size_t off = (c->arena_top + 255) & ~(size_t)255;
      if (off > c->arena_bytes || bytes > c->arena_bytes - off)
        return set_err(c, GMGM_E_NOMEM, "fixed workspace of %zu bytes exhausted (slot %d wants %zu more)",
                       c->arena_bytes, slot, bytes);
      a.ptr = (char*)c->arena + off;
      a.bytes = bytes;
      c->arena_top = off + bytes;
    }
    *out = a.ptr;
    return GMGM_OK;
  }
  if (c->bufs.size() < WS_COUNT) c->bufs.resize(WS_COUNT);
  DevBuf& b = c->bufs[slot];
  if (bytes == 0) bytes = 256;
  if (b.bytes < bytes) {
    if (b.ptr) {
      // the old buffer may still be read by queued kernels
      GMGM_HIP(c, hipStreamSynchronize(c->stream));
      GMGM_HIP(c, hipFree(b.ptr));
      b.ptr = nullptr;
      b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return set_err(c, GMGM_E_NOMEM, "workspace allocation of %zu bytes failed: %s", want,
                     hipGetErrorString(e));
    }
    b.bytes = want;
  }
  *out = b.ptr;
  return GMGM_OK;
}

void arena_begin(gmgm_ctx* c, void* base, size_t bytes) {
  c->arena = base;
  c->arena_bytes = bytes;
  c->arena_top = 0;
  c->arena_slots.assign(WS_COUNT, DevBuf{});
}

void arena_end(gmgm_ctx* c) {
  c->arena = nullptr;
  c->arena_bytes = 0;
  c->arena_top = 0;
  c->arena_slots.clear();
}

gmgm_status blas_handle(gmgm_ctx* c, void** out) {
  if (!c->rocblas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success)
      return set_err(c, GMGM_E_HIP, "rocblas_create_handle failed");
    c->rocblas = h;
  }
  if (rocblas_set_stream((rocblas_handle)c->rocblas, c->stream) != rocblas_status_success)
    return set_err(c, GMGM_E_HIP, "rocblas_set_stream failed");
  *out = c->rocblas;
  return GMGM_OK;
}

extern "C" int gmgm_version(void) { return 100; }

extern "C" gmgm_status gmgm_create(gmgm_ctx_t* out, int device, void* stream) {
  if (!out) return GMGM_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GMGM_E_ARG;
  gmgm_ctx* c = new gmgm_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipMalloc(&c->dev_status, sizeof(int)) != hipSuccess ||
      hipHostMalloc(&c->host_status, sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipMemset(c->dev_status, 0, sizeof(int)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    if (c->dev_status) (void)hipFree(c->dev_status);
    if (c->host_status) (void)hipHostFree(c->host_status);
    delete c;
    return GMGM_E_HIP;
  }
  c->bufs.resize(WS_COUNT);
  // the device address of the fixed workspace of the allocation-free entry
  // point (looked up once per device, with the device current); a failure is
  // kept and reported by that entry point
  c->scratch_status = noalloc_scratch_address(device, &c->scratch, &c->scratch_bytes);
  *out = c;
  return GMGM_OK;
}


static hipEvent_t pool_event(gmgm_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t timing_start(gmgm_ctx* c) {
  if (!c->timing) return nullptr;
  hipEvent_t e = pool_event(c);
  if (e && hipEventRecord(e, c->stream) != hipSuccess) return nullptr;
  return e;
}

void timing_stop(gmgm_ctx* c, hipEvent_t start) {
  if (!start) return;
  hipEvent_t e = pool_event(c);
  if (!e || hipEventRecord(e, c->stream) != hipSuccess) return;
  c->timed.emplace_back(start, e);
}

extern "C" gmgm_status gmgm_set_timing(gmgm_ctx_t c, int enable) {
  GMGM_CHECK_CTX(c);
  c->timing = enable != 0;
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_kernel_times(gmgm_ctx_t c, double* total_ms, int64_t* count) {
  GMGM_CHECK_CTX(c);
  if (!total_ms || !count) return set_err(c, GMGM_E_ARG, "null output pointer");
  GMGM_HIP(c, hipSetDevice(c->device));
  GMGM_HIP(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (auto& p : c->timed) {
    float ms = 0.0f;
    GMGM_HIP(c, hipEventElapsedTime(&ms, p.first, p.second));
    tot += ms;
    c->ev_pool.push_back(p.first);
    c->ev_pool.push_back(p.second);
  }
  *total_ms = tot;
  *count = (int64_t)c->timed.size();
  c->timed.clear();
  return GMGM_OK;
}

extern "C" void gmgm_destroy(gmgm_ctx_t c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->timed) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->rocblas) (void)rocblas_destroy_handle((rocblas_handle)c->rocblas);
  for (auto& b : c->bufs)
    if (b.ptr) (void)hipFree(b.ptr);
  (void)hipFree(c->dev_status);
  (void)hipHostFree(c->host_status);
  delete c;
}

extern "C" gmgm_status gmgm_set_stream(gmgm_ctx_t c, void* stream) {
  GMGM_CHECK_CTX(c);
  c->stream = (hipStream_t)stream;
  return GMGM_OK;
}

extern "C" const char* gmgm_last_error(gmgm_ctx_t c) { return c ? c->err.c_str() : "null context"; }

extern "C" gmgm_status gmgm_sync(gmgm_ctx_t c) {
  GMGM_CHECK_CTX(c);
  GMGM_HIP(c, hipSetDevice(c->device));
  GMGM_HIP(c, hipMemcpyAsync(c->host_status, c->dev_status, sizeof(int), hipMemcpyDeviceToHost,
                             c->stream));
  GMGM_HIP(c, hipStreamSynchronize(c->stream));
  GMGM_HIP(c, hipGetLastError());
  int s = *c->host_status;
  if (s != DEV_OK) {
    GMGM_HIP(c, hipMemsetAsync(c->dev_status, 0, sizeof(int), c->stream));
    GMGM_HIP(c, hipStreamSynchronize(c->stream));
    if (s == DEV_NONFINITE) return set_err(c, GMGM_E_DOMAIN, "a kernel found a non-finite input");
    if (s == DEV_OVERFLOW) return set_err(c, GMGM_E_OVERFLOW, "a device buffer overflowed");
    if (s == DEV_BADINDEX)
      return set_err(c, GMGM_E_SHAPE, "malformed CSR input (row_ptr not monotone within [0, nnz] or a "
                                      "column index outside [0, p))");
    return set_err(c, GMGM_E_HIP, "device fault code %d", s);
  }
  return GMGM_OK;
}
