// Contexts, status strings, error recording and argument checks.

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "bs_internal.h"

namespace bs {
namespace {
thread_local char g_last_error[512] = "";
}

bs_status fail(bs_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return s;
}

void clear_error() { g_last_error[0] = '\0'; }

bs_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return BS_OK;
  return fail(BS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bs_status check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

bs_status check_ctx(const bs_ctx* ctx, const char* op) {
  if (!ctx) return fail(BS_ERR_INVALID_ARG, "%s: ctx is NULL", op);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
    return fail(BS_ERR_INVALID_ARG, "%s: current device %d is not the context's device %d", op, dev, ctx->device);
  return BS_OK;
}

bs_status check_dtype(const char* op, bs_dtype d) {
  if (dtype_size(d) == 0) return fail(BS_ERR_INVALID_ARG, "%s: unknown dtype %d", op, static_cast<int>(d));
  return BS_OK;
}

bs_status check_vec(const char* op, const char* name, const void* p, int64_t n, bs_dtype d) {
  if (n < 0) return fail(BS_ERR_INVALID_ARG, "%s: negative length %lld", op, static_cast<long long>(n));
  if (n > 0 && !p) return fail(BS_ERR_INVALID_ARG, "%s: %s is NULL", op, name);
  if (p && !aligned_to(p, static_cast<uintptr_t>(dtype_size(d))))
    return fail(BS_ERR_INVALID_ARG, "%s: %s is not aligned to its %d-byte element", op, name, dtype_size(d));
  return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" const char* bs_status_string(bs_status s) {
  switch (s) {
    case BS_OK: return "BS_OK";
    case BS_ERR_INVALID_ARG: return "BS_ERR_INVALID_ARG";
    case BS_ERR_UNSUPPORTED: return "BS_ERR_UNSUPPORTED";
    case BS_ERR_ALLOC: return "BS_ERR_ALLOC";
    case BS_ERR_HIP: return "BS_ERR_HIP";
    case BS_ERR_NO_CONVERGENCE: return "BS_ERR_NO_CONVERGENCE";
  }
  return "BS_ERR_UNKNOWN";
}

extern "C" const char* bs_last_error(void) { return g_last_error; }

extern "C" const char* bs_version(void) { return "bs-mi355x 0.1 (gfx950)"; }

extern "C" bs_status bs_ctx_create(int device, bs_ctx** out) {
  if (!out) return fail(BS_ERR_INVALID_ARG, "bs_ctx_create: out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fail(BS_ERR_INVALID_ARG, "bs_ctx_create: device %d not available (%d devices)", device, count);
  int prev = 0;
  bs_status s;
  if ((s = check_hip(hipGetDevice(&prev), "bs_ctx_create"))) return s;
  if ((s = check_hip(hipSetDevice(device), "bs_ctx_create"))) return s;
  bs_ctx* c = new bs_ctx();
  c->device = device;
  void* ws = nullptr;
  const size_t bytes = sizeof(double) * 2 * kMaxReduceBlocks;
  if (hipMalloc(&ws, bytes) != hipSuccess) {
    delete c;
    (void)hipSetDevice(prev);
    return fail(BS_ERR_ALLOC, "bs_ctx_create: cannot allocate %zu bytes of workspace", bytes);
  }
  c->partials = static_cast<double*>(ws);
  s = check_hip(hipMemset(ws, 0, bytes), "bs_ctx_create");
  if (!s) s = check_hip(hipDeviceSynchronize(), "bs_ctx_create");
  if (s) {
    (void)hipFree(ws);
    delete c;
    (void)hipSetDevice(prev);
    return s;
  }
  // Defaults measured on MI355X at n = 7.2e8 binary64 values: element-wise
  // operations run one 16-byte packet per thread in a one-pass grid; the
  // reductions grid-stride with several packets in flight per thread.
  for (int op = 0; op < OP_COUNT; ++op)
    for (int d = 0; d < 3; ++d) c->tune[op][d] = Tune{1, 1 << 30, 0};
  for (int d = 0; d < 3; ++d) {
    c->tune[OP_NORM][d] = Tune{8, 4096, 0};
    c->tune[OP_DOT][d] = Tune{8, 4096, 0};
    c->tune[OP_CG_UPDATE][d] = Tune{4, kMaxReduceBlocks, 0};
    // gather: rows in global order; scatter: tiles read in local order
    c->tune[OP_GATHER][d] = Tune{1, 1 << 30, 1};
    c->tune[OP_SCATTER][d] = Tune{1, 1 << 30, 1};
  }
  (void)hipSetDevice(prev);
  *out = c;
  return BS_OK;
}

extern "C" bs_status bs_ctx_destroy(bs_ctx* ctx) {
  if (!ctx) return BS_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipFree(ctx->partials);
  (void)hipSetDevice(prev);
  delete ctx;
  return check_hip(e, "bs_ctx_destroy");
}

extern "C" bs_status bs_ctx_set_tune(bs_ctx* ctx, int op, bs_dtype dtype, int unroll, int grid_cap, int variant) {
  if (!ctx) return fail(BS_ERR_INVALID_ARG, "bs_ctx_set_tune: ctx is NULL");
  if (op < 0 || op >= OP_COUNT) return fail(BS_ERR_INVALID_ARG, "bs_ctx_set_tune: unknown op %d", op);
  if (dtype_size(dtype) == 0) return fail(BS_ERR_INVALID_ARG, "bs_ctx_set_tune: unknown dtype %d", (int)dtype);
  if (!(unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8))
    return fail(BS_ERR_INVALID_ARG, "bs_ctx_set_tune: unroll must be 1, 2, 4 or 8");
  if (grid_cap < 1) return fail(BS_ERR_INVALID_ARG, "bs_ctx_set_tune: grid_cap must be positive");
  if (variant < 0 || variant > 7 || (variant & kVariantMask) == 3)
    return fail(BS_ERR_INVALID_ARG, "bs_ctx_set_tune: variant must be 0, 1 or 2, optionally plus 4");
  // every dtype currently shares one entry per op
  for (int d = 0; d < 3; ++d) ctx->tune[op][d] = Tune{unroll, grid_cap, variant};
  return BS_OK;
}

extern "C" bs_status bs_ctx_get_tune(const bs_ctx* ctx, int op, bs_dtype dtype, int* unroll, int* grid_cap,
                                     int* variant) {
  if (!ctx || op < 0 || op >= OP_COUNT || dtype_size(dtype) == 0)
    return fail(BS_ERR_INVALID_ARG, "bs_ctx_get_tune: bad argument");
  const Tune& t = ctx->tune[op][static_cast<int>(dtype)];
  if (unroll) *unroll = t.unroll;
  if (grid_cap) *grid_cap = t.grid_cap;
  if (variant) *variant = t.variant;
  return BS_OK;
}
