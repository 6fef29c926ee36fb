// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gmgm.h"

// Device-side fault codes written into the context's status word.
enum : int { DEV_OK = 0, DEV_NONFINITE = 1, DEV_OVERFLOW = 2, DEV_BADINDEX = 3 };

// A device buffer the context owns and grows on demand.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct gmgm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int* dev_status = nullptr;        // one int, DEV_* code of the first device fault
  int* host_status = nullptr;       // pinned mirror
  std::vector<DevBuf> bufs;         // workspace slots, indexed by purpose
  void* rocblas = nullptr;          // lazily created library handles
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;  // free events
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;   // recorded (start, stop) pairs
  // fixed arena (set for the duration of an allocation-free call): ws_get
  // carves slots from it instead of allocating
  void* arena = nullptr;
  size_t arena_bytes = 0, arena_top = 0;
  std::vector<DevBuf> arena_slots;
  // this device's fixed workspace of the allocation-free entry point
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipError_t scratch_status = hipSuccess;
};

// Record a start event on the context stream when timing is on (returns nullptr otherwise).
hipEvent_t timing_start(gmgm_ctx* c);
// Record the matching stop event.
void timing_stop(gmgm_ctx* c, hipEvent_t start);

// Workspace slots.
enum WsSlot : int {
  WS_VP = 0, WS_WP, WS_NORMS, WS_CAND, WS_MISC, WS_FALLBACK, WS_SCALES, WS_VP2, WS_WP2, WS_CAND2,
  WS_GRAM0, WS_GRAM1, WS_GRAM2, WS_GRAM3, WS_SOLVE0, WS_SOLVE1, WS_SOLVE2, WS_MLP0, WS_MLP1, WS_EIGH0,
  WS_EIGH1, WS_SKETCH, WS_RF0, WS_RF1, WS_RF2, WS_THR0, WS_THR1, WS_THR2, WS_SKEP0, WS_SKEP1, WS_SKEP2, WS_SYM0, WS_SYM1, WS_SYM2,
  WS_COUNT
};

gmgm_status set_err(gmgm_ctx* c, gmgm_status s, const char* fmt, ...);
gmgm_status hip_err(gmgm_ctx* c, hipError_t e, const char* what);
// The context's rocBLAS handle (created on first use, bound to the context stream).
gmgm_status blas_handle(gmgm_ctx* c, void** out);
// Pointer to a workspace slot of at least `bytes` bytes (grown when needed, or
// carved from the fixed arena while one is set).
gmgm_status ws_get(gmgm_ctx* c, int slot, size_t bytes, void** out);
// Carve every workspace slot from [base, base + bytes) until arena_end.
void arena_begin(gmgm_ctx* c, void* base, size_t bytes);
void arena_end(gmgm_ctx* c);
// Device address and size of the fixed workspace of the allocation-free
// recomposition entry point on `device` (the current device).
hipError_t noalloc_scratch_address(int device, void** ptr, size_t* bytes);

#define GMGM_CHECK_CTX(c)                 \
  do {                                    \
    if (!(c)) return GMGM_E_ARG;          \
    (c)->err.clear();                     \
  } while (0)

#define GMGM_HIP(c, expr)                                   \
  do {                                                      \
    hipError_t e__ = (expr);                                \
    if (e__ != hipSuccess) return hip_err((c), e__, #expr); \
  } while (0)

#define GMGM_TRY(expr)                       \
  do {                                       \
    gmgm_status s__ = (expr);                \
    if (s__ != GMGM_OK) return s__;          \
  } while (0)

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
