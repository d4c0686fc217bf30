// Contexts, status strings, error recording and argument checks.

#include <dlfcn.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

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

namespace {

const char* const kOpNames[OP_COUNT] = {"copy", "axpy", "norm", "dot", "cg_update", "gather", "scatter", "batch"};
const char* const kDtypeNames[3] = {"f64", "f32", "bf16"};

void set_one(TuneList& L, Tune t) {
  L.count = 1;
  L.n_min[0] = 0;
  L.t[0] = t;
}

// Defaults measured on MI355X at n = 7.2e8 binary64 values: element-wise
// operations run one 16-byte packet per thread in a one-pass grid; the
// reductions grid-stride with several packets in flight per thread.
void set_defaults(bs_ctx* c) {
  for (int op = 0; op < OP_COUNT; ++op)
    for (int d = 0; d < 3; ++d) set_one(c->tune[op][d], Tune{1, 1 << 30, 0});
  for (int d = 0; d < 3; ++d) {
    set_one(c->tune[OP_NORM][d], Tune{8, 4096, 0});
    set_one(c->tune[OP_DOT][d], Tune{8, 4096, 0});
    set_one(c->tune[OP_CG_UPDATE][d], Tune{4, kMaxReduceBlocks, 0});
    // gather: rows in global order; scatter: tiles read in local order, two
    // tiles per workgroup
    set_one(c->tune[OP_GATHER][d], Tune{1, 1 << 30, 1});
    set_one(c->tune[OP_SCATTER][d], Tune{2, 1 << 30, 1});
    // persistent batch: 8 items per claim, every resident workgroup
    set_one(c->tune[OP_BATCH][d], Tune{8, 1 << 30, 0});
  }
}

bs_status check_tune(const char* op, int unroll, int grid_cap, int variant) {
  if (!(unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8))
    return fail(BS_ERR_INVALID_ARG, "%s: unroll must be 1, 2, 4 or 8", op);
  if (grid_cap < 1) return fail(BS_ERR_INVALID_ARG, "%s: grid_cap must be positive", op);
  if (variant < 0 || variant > 27 || (variant & kVariantMask) == 3 || ((variant & kNoXcdRemap) && (variant & kGroupOrder)))
    return fail(BS_ERR_INVALID_ARG, "%s: variant must be 0, 1 or 2, optionally plus 4 or 8, optionally plus 16", op);
  return BS_OK;
}

// Insert or replace the entry for n_min in a list kept sorted by n_min.
bool put_entry(TuneList& L, int64_t n_min, Tune t) {
  for (int j = 0; j < L.count; ++j)
    if (L.n_min[j] == n_min) {
      L.t[j] = t;
      return true;
    }
  if (L.count == kTuneEntries) return false;
  int j = L.count++;
  while (j > 0 && L.n_min[j - 1] > n_min) {
    L.n_min[j] = L.n_min[j - 1];
    L.t[j] = L.t[j - 1];
    --j;
  }
  L.n_min[j] = n_min;
  L.t[j] = t;
  return true;
}

}  // namespace

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
  const size_t pair_bytes = sizeof(double) * 2 * kPartialPairs;
  const size_t bytes = pair_bytes + 256;  // the pairs, then the counter of single-launch reductions
  if (hipMalloc(&ws, bytes) != hipSuccess) {
    delete c;
    (void)hipSetDevice(prev);
    return fail(BS_ERR_ALLOC, "bs_ctx_create: cannot allocate %zu bytes of workspace", bytes);
  }
  c->partials = static_cast<double*>(ws);
  c->counter = reinterpret_cast<unsigned int*>(static_cast<char*>(ws) + pair_bytes);
  s = check_hip(hipMemset(ws, 0, bytes), "bs_ctx_create");
  if (!s) s = check_hip(hipDeviceSynchronize(), "bs_ctx_create");
  if (s) {
    (void)hipFree(ws);
    delete c;
    (void)hipSetDevice(prev);
    return s;
  }
  if ((s = bs_ctx_reset_tune(c))) {
    (void)hipFree(ws);
    delete c;
    (void)hipSetDevice(prev);
    return s;
  }
  (void)hipSetDevice(prev);
  *out = c;
  return BS_OK;
}

// The built-in defaults, then a tune table next to the library (written by
// the autotuner), or the one BS_TUNE_FILE names ("none": keep the defaults).
extern "C" bs_status bs_ctx_reset_tune(bs_ctx* ctx) {
  bs_status s;
  if ((s = check_ctx(ctx, "bs_ctx_reset_tune"))) return s;
  set_defaults(ctx);
  std::string path;
  if (const char* env = std::getenv("BS_TUNE_FILE")) {
    path = env;
  } else {
    Dl_info info{};
    if (dladdr(reinterpret_cast<void*>(&bs_ctx_create), &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t slash = path.find_last_of('/');
      path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tune_gfx950.txt";
      if (FILE* f = std::fopen(path.c_str(), "r")) {
        std::fclose(f);
      } else {
        path.clear();
      }
    }
  }
  if (path.empty() || path == "none") return BS_OK;
  int entries = 0;
  if ((s = bs_ctx_load_tune(ctx, path.c_str(), &entries))) set_defaults(ctx);
  return s;
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
  if (bs_status s = check_tune("bs_ctx_set_tune", unroll, grid_cap, variant)) return s;
  // one entry for every dtype and length
  for (int d = 0; d < 3; ++d) set_one(ctx->tune[op][d], Tune{unroll, grid_cap, variant});
  return BS_OK;
}

extern "C" bs_status bs_ctx_set_tune_entry(bs_ctx* ctx, int op, bs_dtype dtype, int64_t n_min, int unroll,
                                           int grid_cap, int variant) {
  const char* name = "bs_ctx_set_tune_entry";
  if (!ctx) return fail(BS_ERR_INVALID_ARG, "%s: ctx is NULL", name);
  if (op < 0 || op >= OP_COUNT) return fail(BS_ERR_INVALID_ARG, "%s: unknown op %d", name, op);
  if (dtype_size(dtype) == 0) return fail(BS_ERR_INVALID_ARG, "%s: unknown dtype %d", name, (int)dtype);
  if (n_min < 0) return fail(BS_ERR_INVALID_ARG, "%s: n_min must be >= 0", name);
  if (bs_status s = check_tune(name, unroll, grid_cap, variant)) return s;
  if (!put_entry(ctx->tune[op][static_cast<int>(dtype)], n_min, Tune{unroll, grid_cap, variant}))
    return fail(BS_ERR_INVALID_ARG, "%s: at most %d entries per operation and dtype", name, kTuneEntries);
  return BS_OK;
}

extern "C" bs_status bs_ctx_tune_for(const bs_ctx* ctx, int op, bs_dtype dtype, int64_t n, int* unroll,
                                     int* grid_cap, int* variant) {
  if (!ctx || op < 0 || op >= OP_COUNT || dtype_size(dtype) == 0 || n < 0)
    return fail(BS_ERR_INVALID_ARG, "bs_ctx_tune_for: bad argument");
  const Tune& t = tune_for(ctx, op, static_cast<int>(dtype), n);
  if (unroll) *unroll = t.unroll;
  if (grid_cap) *grid_cap = t.grid_cap;
  if (variant) *variant = t.variant;
  return BS_OK;
}

extern "C" bs_status bs_ctx_load_tune(bs_ctx* ctx, const char* path, int* n_entries) {
  const char* name = "bs_ctx_load_tune";
  if (!ctx || !path) return fail(BS_ERR_INVALID_ARG, "%s: NULL argument", name);
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(BS_ERR_INVALID_ARG, "%s: cannot open %s", name, path);
  TuneList fresh[OP_COUNT][3];
  bool seen[OP_COUNT][3] = {};
  char line[512];
  int lineno = 0, entries = 0;
  bs_status s = BS_OK;
  while (!s && std::fgets(line, sizeof(line), f)) {
    ++lineno;
    char* hash = std::strchr(line, '#');
    if (hash) *hash = '\0';
    char op_name[32], dt_name[16];
    long long n_min = 0;
    int unroll = 0, grid_cap = 0, variant = 0, used = 0;
    const int got = std::sscanf(line, "%31s %15s %lld %d %d %d %n", op_name, dt_name, &n_min, &unroll, &grid_cap,
                                &variant, &used);
    if (got <= 0) continue;  // blank or comment
    if (got != 6 || line[used] != '\0') {
      s = fail(BS_ERR_INVALID_ARG, "%s: %s line %d: expected 'op dtype n_min unroll grid_cap variant'", name, path,
               lineno);
      break;
    }
    const int op = static_cast<int>(std::find_if(kOpNames, kOpNames + OP_COUNT,
                                                 [&](const char* q) { return std::strcmp(q, op_name) == 0; }) -
                                    kOpNames);
    const int d = static_cast<int>(std::find_if(kDtypeNames, kDtypeNames + 3,
                                                [&](const char* q) { return std::strcmp(q, dt_name) == 0; }) -
                                   kDtypeNames);
    if (op == OP_COUNT || d == 3) {
      s = fail(BS_ERR_INVALID_ARG, "%s: %s line %d: unknown operation or dtype", name, path, lineno);
      break;
    }
    if (n_min < 0 || (s = check_tune(name, unroll, grid_cap, variant))) {
      if (!s) s = fail(BS_ERR_INVALID_ARG, "%s: %s line %d: negative n_min", name, path, lineno);
      break;
    }
    if (!seen[op][d]) {
      seen[op][d] = true;
      fresh[op][d].count = 0;
    }
    if (!put_entry(fresh[op][d], n_min, Tune{unroll, grid_cap, variant})) {
      s = fail(BS_ERR_INVALID_ARG, "%s: %s line %d: too many entries for %s %s", name, path, lineno, op_name, dt_name);
      break;
    }
    ++entries;
  }
  std::fclose(f);
  if (s) return s;
  for (int op = 0; op < OP_COUNT; ++op)
    for (int d = 0; d < 3; ++d)
      if (seen[op][d] && fresh[op][d].n_min[0] != 0)
        return fail(BS_ERR_INVALID_ARG, "%s: %s: %s %s has no entry for n_min 0", name, path, kOpNames[op],
                    kDtypeNames[d]);
  for (int op = 0; op < OP_COUNT; ++op)
    for (int d = 0; d < 3; ++d)
      if (seen[op][d]) ctx->tune[op][d] = fresh[op][d];
  if (n_entries) *n_entries = entries;
  return BS_OK;
}

extern "C" bs_status bs_ctx_get_tune(const bs_ctx* ctx, int op, bs_dtype dtype, int* unroll, int* grid_cap,
                                     int* variant) {
  if (!ctx || op < 0 || op >= OP_COUNT || dtype_size(dtype) == 0)
    return fail(BS_ERR_INVALID_ARG, "bs_ctx_get_tune: bad argument");
  const Tune& t = ctx->tune[op][static_cast<int>(dtype)].t[0];
  if (unroll) *unroll = t.unroll;
  if (grid_cap) *grid_cap = t.grid_cap;
  if (variant) *variant = t.variant;
  return BS_OK;
}
