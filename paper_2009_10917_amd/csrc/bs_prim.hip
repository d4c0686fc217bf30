// Set-up primitives of the plan (Section 5's mesh set-up): an exclusive
// prefix sum of int32 counts and a stable least-significant-digit radix sort
// of (uint32 key, int32 value) pairs.  Both are deterministic: integer sums
// are exact, and the sort places equal keys in their input order, so the
// CSR of Z^T lists each row's local indices in ascending order.
//
// Scan: tiles of 2048 values (eight per thread, in order); each tile is
// scanned in registers and across its waves (shuffles, then LDS), its total
// goes to a sums array, the sums are scanned the same way (recursively),
// and every tile adds its offset.
//
// Sort: eight-bit digits, one pass per digit up to the requested key bits.
// A pass counts each tile's digits (tiles of 2048 keys), scans the counts
// in digit-major order (all tiles' counts of digit 0, then digit 1, ...), so
// that entry (d, t) is where tile t's keys of digit d start, and scatters:
// the tile walks its keys in eight rounds of 256 in input order; within a
// wave, the lanes holding the same digit are found with eight ballots (one
// per digit bit), a lane's rank is the number of such lanes below it, and
// the waves of a round and the earlier rounds add their counts of that
// digit in order.  Every key therefore lands after all equal keys that
// precede it in the input: the pass is stable.

#include <hip/hip_runtime.h>

#include "bs_internal.h"
#include "bs_prim.h"

namespace bs {
namespace {

constexpr int kItems = 8;
constexpr int kTileN = kBlock * kItems;  // 2048
constexpr int kWaves = kBlock / 64;
constexpr int kDigits = 256;

inline unsigned int tiles_for(int64_t n) { return static_cast<unsigned int>((n + kTileN - 1) / kTileN); }

// Exclusive scan of one value per thread over the workgroup; *total gets
// the sum.
__device__ __forceinline__ int32_t block_exclusive(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    if (i < w) base += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// out[i] = in[tile start] + ... + in[i - 1] within each tile; sums[tile] = the
// tile's total (when sums is given).  in and out may be the same array.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t* in, int32_t* out, int64_t n,
                                                       int32_t* __restrict__ sums) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTileN + static_cast<int64_t>(threadIdx.x) * kItems;
  int32_t v[kItems];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int32_t total = 0;
  int32_t run = block_exclusive(s, &total);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (sums && threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                     const int32_t* __restrict__ offs) {
  const int32_t o = offs[blockIdx.x];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTileN;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k * kBlock + threadIdx.x;
    if (i < n) out[i] += o;
  }
}

// counts[d * tiles + t] = number of keys of tile t whose digit is d.
__global__ __launch_bounds__(kBlock) void k_digit_counts(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                         int32_t* __restrict__ counts, int64_t tiles) {
  __shared__ int32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTileN;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t p = base + k * kBlock + threadIdx.x;
    if (p < n) atomicAdd(&h[(keys[p] >> shift) & (kDigits - 1)], 1);
  }
  __syncthreads();
  counts[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile by the digit at `shift` (see the top).
__global__ __launch_bounds__(kBlock) void k_digit_scatter(const uint32_t* __restrict__ kin,
                                                          const int32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                          int32_t* __restrict__ vout, int64_t n, int shift,
                                                          const int32_t* __restrict__ offs, int64_t tiles) {
  __shared__ int32_t run[kDigits];
  __shared__ int32_t wcnt[kWaves][kDigits];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  run[threadIdx.x] = offs[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x];
#pragma unroll
  for (int i = 0; i < kWaves; ++i) wcnt[i][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTileN;
  for (int r = 0; r < kItems; ++r) {
    const int64_t p = base + r * kBlock + threadIdx.x;  // input order: round, wave, lane
    const bool valid = p < n;
    const uint32_t key = valid ? kin[p] : 0u;
    const int32_t val = valid ? vin[p] : 0;
    const int d = static_cast<int>((key >> shift) & (kDigits - 1));
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);  // the lowest lane of each digit
    __syncthreads();
    if (valid) {
      int32_t dst = run[d];
      for (int i = 0; i < w; ++i) dst += wcnt[i][d];
      kout[dst + rank] = key;
      vout[dst + rank] = val;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      add += wcnt[i][threadIdx.x];
      wcnt[i][threadIdx.x] = 0;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

struct Tmp {
  void* p = nullptr;
  ~Tmp() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

bs_status scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t st, const char* op) {
  if (n <= 0) return BS_OK;
  const int64_t tiles = tiles_for(n);
  if (tiles == 1) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, st, in, out, n, static_cast<int32_t*>(nullptr));
    return check_launch(op);
  }
  Tmp sums;
  if (hipMalloc(&sums.p, tiles * sizeof(int32_t)) != hipSuccess)
    return fail(BS_ERR_ALLOC, "%s: cannot allocate %lld scan sums", op, static_cast<long long>(tiles));
  int32_t* s = static_cast<int32_t*>(sums.p);
  hipLaunchKernelGGL(k_scan_tiles, dim3(static_cast<unsigned int>(tiles)), dim3(kBlock), 0, st, in, out, n, s);
  bs_status r = check_launch(op);
  if (!r) r = scan_exclusive_i32(s, s, tiles, st, op);
  if (!r) {
    hipLaunchKernelGGL(k_scan_add, dim3(static_cast<unsigned int>(tiles)), dim3(kBlock), 0, st, out, n, s);
    r = check_launch(op);
  }
  if (!r) r = check_hip(hipStreamSynchronize(st), op);  // the sums are freed on return
  return r;
}

bs_status sort_pairs_u32(uint32_t* keys, uint32_t* keys_alt, int32_t* vals, int32_t* vals_alt, int64_t n, int bits,
                         hipStream_t st, const char* op, bool* in_alt) {
  *in_alt = false;
  if (n <= 0 || bits <= 0) return BS_OK;
  const int64_t tiles = tiles_for(n);
  const int64_t nc = tiles * kDigits;
  if (nc >= (int64_t(1) << 31)) return fail(BS_ERR_INVALID_ARG, "%s: too many keys to sort", op);
  Tmp counts;
  if (hipMalloc(&counts.p, nc * sizeof(int32_t)) != hipSuccess)
    return fail(BS_ERR_ALLOC, "%s: cannot allocate %lld digit counts", op, static_cast<long long>(nc));
  int32_t* c = static_cast<int32_t*>(counts.p);
  uint32_t *k0 = keys, *k1 = keys_alt;
  int32_t *v0 = vals, *v1 = vals_alt;
  bs_status r = BS_OK;
  for (int shift = 0; shift < bits && !r; shift += 8) {
    hipLaunchKernelGGL(k_digit_counts, dim3(static_cast<unsigned int>(tiles)), dim3(kBlock), 0, st, k0, n, shift, c,
                       tiles);
    r = check_launch(op);
    if (!r) r = scan_exclusive_i32(c, c, nc, st, op);
    if (!r) {
      hipLaunchKernelGGL(k_digit_scatter, dim3(static_cast<unsigned int>(tiles)), dim3(kBlock), 0, st, k0, v0, k1, v1,
                         n, shift, c, tiles);
      r = check_launch(op);
    }
    std::swap(k0, k1);
    std::swap(v0, v1);
    *in_alt = !*in_alt;
  }
  if (!r) r = check_hip(hipStreamSynchronize(st), op);  // the counts are freed on return
  return r;
}

}  // namespace bs
