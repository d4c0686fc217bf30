// Mesh scatter map, gather/scatter plan, BS6 gather and BS7 scatter
// (Section 2, eq. scatter_def; Section 5; Listings 4 and 5).
//
// Plan: a copy of the scatter ids plus the CSR form of Z^T without values
// (row g = ascending local indices l with map[l] == g).  The CSR is built on
// the device: a degree histogram, an exclusive scan for the row starts and
// a stable radix sort of (map[l], l) pairs for the column ids.
//
// Gather follows the paper's blocking (Section 5): every workgroup takes
// about the same number of nonzeros (a `chunk` of the CSR), the rows whose
// first nonzero falls in its chunk (blockStarts), stages the local values of
// its window in LDS and adds each row from LDS in CSR order.  Unlike the
// paper's listing, the window start is known from the block index alone, so
// the column-id and value loads are issued before the row starts arrive and
// the two dependent chains overlap.
//
// Scatter processes tiles of consecutive local entries in the order of the
// smallest global id each tile references, so that tiles touching
// neighbouring global entries run close together in time and share cache
// lines; each tile still reads its ids and writes its values contiguously.
//
// Workgroups are renumbered per XCD so that neighbouring blocks, which share
// cache lines, run on the same XCD's L2.

#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

using dev::bf16;
using dev::Storage;

// ---------------------------------------------------------------- orientations

// The 24 proper rotations of the hex as (axis permutation, flips), axis
// permutations in lexicographic order, flip masks ascending, improper ones
// (odd permutation parity xor odd number of flips) skipped.
struct OrientTable {
  int8_t pi[24][3];
  int8_t flip[24][3];
};

OrientTable make_orient_table() {
  OrientTable t{};
  int p[3] = {0, 1, 2};
  int n = 0;
  do {
    const int inv = (p[0] > p[1]) + (p[0] > p[2]) + (p[1] > p[2]);
    for (int f = 0; f < 8; ++f) {
      const int f0 = f & 1, f1 = (f >> 1) & 1, f2 = (f >> 2) & 1;
      if (((inv & 1) ^ f0 ^ f1 ^ f2) != 0) continue;
      for (int d = 0; d < 3; ++d) t.pi[n][d] = static_cast<int8_t>(p[d]);
      t.flip[n][0] = static_cast<int8_t>(f0);
      t.flip[n][1] = static_cast<int8_t>(f1);
      t.flip[n][2] = static_cast<int8_t>(f2);
      ++n;
    }
  } while (std::next_permutation(p, p + 3));
  return t;
}

// Global id of local node l, or -1 when the slot's element or orientation
// is out of range.
__host__ __device__ inline int32_t hex_node(int64_t l, int64_t K, int N, const int32_t* perm,
                                            const uint8_t* orient, const OrientTable& T) {
  const int64_t Np = N + 1, Np3 = Np * Np * Np, M = K * N + 1, E = K * K * K;
  const int64_t s = l / Np3, rem = l - s * Np3;
  const int64_t t[3] = {rem % Np, (rem / Np) % Np, rem / (Np * Np)};
  const int64_t e = perm ? perm[s] : s;
  const int o = orient ? orient[s] : 0;
  if (e < 0 || e >= E || o >= 24) return -1;
  int64_t off[3];
  for (int d = 0; d < 3; ++d) {
    const int64_t v = t[T.pi[o][d]];
    off[d] = T.flip[o][d] ? N - v : v;
  }
  const int64_t X = N * (e % K) + off[0], Y = N * ((e / K) % K) + off[1], Z = N * (e / (K * K)) + off[2];
  return static_cast<int32_t>(X + M * (Y + M * Z));
}

__global__ __launch_bounds__(kBlock) void k_hex_map(int64_t K, int N, const int32_t* __restrict__ perm,
                                                    const uint8_t* __restrict__ orient, OrientTable T,
                                                    int32_t* __restrict__ map, int64_t n_local,
                                                    int* __restrict__ bad) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= n_local) return;
  const int32_t g = hex_node(l, K, N, perm, orient, T);
  map[l] = g;
  if (g < 0) atomicOr(bad, 1);
}

bs_status check_mesh(int64_t K, int N, int64_t* n_local) {
  if (K < 1 || N < 1) return fail(BS_ERR_INVALID_ARG, "hex map: K and N must be >= 1");
  const double ng = static_cast<double>(K * N + 1), nl = static_cast<double>(K) * K * K * (N + 1.0) * (N + 1) * (N + 1);
  if (ng * ng * ng >= 2147483648.0 || nl >= 2147483648.0)
    return fail(BS_ERR_INVALID_ARG, "hex map: mesh K=%lld N=%d exceeds 32-bit node ids", (long long)K, N);
  *n_local = K * K * K * (N + 1) * (N + 1) * (N + 1);
  return BS_OK;
}

// ---------------------------------------------------------------- plan set-up kernels

__global__ __launch_bounds__(kBlock) void k_plan_prepare(const int32_t* __restrict__ map, int64_t n_local,
                                                         int32_t n_global, int32_t* __restrict__ map_copy,
                                                         uint32_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                         int32_t* __restrict__ deg, int* __restrict__ bad) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= n_local) return;
  const int32_t m = map[l];
  map_copy[l] = m;
  vals[l] = static_cast<int32_t>(l);
  if (m >= n_global) {
    atomicOr(bad, 1);
    keys[l] = static_cast<uint32_t>(n_global);
  } else if (m < 0) {
    keys[l] = static_cast<uint32_t>(n_global);  // masked: sorts after every row
  } else {
    keys[l] = static_cast<uint32_t>(m);
    atomicAdd(&deg[m], 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_degree(const int32_t* __restrict__ rs, int32_t n_global,
                                                   int32_t* __restrict__ deg) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (g < n_global) deg[g] = rs[g + 1] - rs[g];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_weights(const int32_t* __restrict__ map, const int32_t* __restrict__ rs,
                                                    int64_t n_local, typename Storage<T>::E* __restrict__ w) {
  using S = Storage<T>;
  using C = typename S::C;
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= n_local) return;
  const int32_t m = map[l];
  if (m < 0) {
    w[l] = S::store(C(0));
  } else {
    const double d = static_cast<double>(rs[m + 1] - rs[m]);
    w[l] = S::store(static_cast<C>(1.0 / d));
  }
}

// ---------------------------------------------------------------- BS6 gather

template <class T, int RPT>
__global__ __launch_bounds__(kBlock) void k_gather(const int32_t* __restrict__ rs, const int32_t* __restrict__ ci,
                                                   const typename Storage<T>::E* __restrict__ xL,
                                                   typename Storage<T>::E* __restrict__ xG, int32_t n_global, bool remap) {
  using S = Storage<T>;
  using C = typename S::C;
  constexpr int R = kBlock * RPT;    // rows per workgroup
  constexpr int CAP = 8 * R;         // staged values: up to an average degree of 8
  constexpr int L = CAP / kBlock;    // staged values per thread
  __shared__ C lds[CAP];
  const int32_t b = static_cast<int32_t>(remap ? dev::xcd_block(blockIdx.x, gridDim.x) : blockIdx.x);
  const int32_t row0 = b * R;
  const int32_t row1 = min(row0 + R, n_global);
  const int32_t base = rs[row0];
  const int32_t nnz = rs[row1] - base;
  if (nnz <= CAP) {
    C v[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int32_t i = threadIdx.x + k * kBlock;
      if (i < nnz) v[k] = S::load(xL[ci[base + i]]);
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int32_t i = threadIdx.x + k * kBlock;
      if (i < nnz) lds[i] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int32_t row = row0 + q * kBlock + threadIdx.x;
      if (row < row1) {
        const int32_t a = rs[row] - base, e = rs[row + 1] - base;
        C s = C(0);
        for (int32_t j = a; j < e; ++j) s += lds[j];
        xG[row] = S::store(s);
      }
    }
  } else {
    // rows of unusually high degree: same order of additions, straight from memory
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int32_t row = row0 + q * kBlock + threadIdx.x;
      if (row < row1) {
        C s = C(0);
        for (int32_t j = rs[row]; j < rs[row + 1]; ++j) s += S::load(xL[ci[j]]);
        xG[row] = S::store(s);
      }
    }
  }
}

// ---------------------------------------------------------------- BS7 scatter

template <class E, int U>
__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t* __restrict__ map, const E* __restrict__ xG,
                                                    E* __restrict__ xL, int64_t n_local) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * kBlock * U;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock * U + threadIdx.x; i < n_local; i += step) {
    int32_t id[U];
    E v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t l = i + static_cast<int64_t>(u) * kBlock;
      id[u] = (l < n_local) ? dev::ld_nt(map + l) : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (id[u] >= 0) v[u] = xG[id[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (id[u] >= 0) dev::st_nt(xL + i + static_cast<int64_t>(u) * kBlock, v[u]);
  }
}

// ---------------------------------------------------------------- plan: gather blocks, scatter tiles

// block_starts[b] = first row g with row_starts[g] >= b*chunk (b < n_blocks);
// block_starts[n_blocks] = n_global.
__global__ __launch_bounds__(kBlock) void k_block_starts(const int32_t* __restrict__ rs, int32_t n_global, int64_t chunk,
                                                         int64_t n_blocks, int32_t* __restrict__ bstart) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (b > n_blocks) return;
  if (b == n_blocks) {
    bstart[b] = n_global;
    return;
  }
  const int64_t target = b * chunk;
  int64_t lo = 0, hi = n_global;  // answer in [0, n_global]
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (rs[mid] >= target) hi = mid; else lo = mid + 1;
  }
  bstart[b] = static_cast<int32_t>(lo);
}

// key[t] = smallest unmasked id among the tile's entries (INT32_MAX if none).
__global__ __launch_bounds__(kBlock) void k_tile_keys(const int32_t* __restrict__ map, int64_t n_local,
                                                      uint32_t* __restrict__ key, int32_t* __restrict__ tile) {
  __shared__ int32_t s_min[kBlock / 64];
  const int64_t t = blockIdx.x;
  int32_t m = INT32_MAX;
  for (int k = threadIdx.x; k < kTile; k += kBlock) {
    const int64_t l = t * kTile + k;
    if (l < n_local) {
      const int32_t v = map[l];
      if (v >= 0 && v < m) m = v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
  if (threadIdx.x % 64 == 0) s_min[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / 64; ++i) m = min(m, s_min[i]);
    m = min(m, s_min[0]);
    key[t] = static_cast<uint32_t>(m);
    tile[t] = static_cast<int32_t>(t);
  }
}

// ---------------------------------------------------------------- BS6 gather, nonzero-balanced

template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_nnz(const int32_t* __restrict__ rs, const int32_t* __restrict__ ci,
                                                       const int32_t* __restrict__ bstart,
                                                       const typename Storage<T>::E* __restrict__ xL,
                                                       typename Storage<T>::E* __restrict__ xG, int64_t chunk,
                                                       int64_t nnz, bool remap) {
  using S = Storage<T>;
  using C = typename S::C;
  constexpr int L = kStage / kBlock;
  __shared__ C lds[kStage];            // local values of the CSR window
  __shared__ int32_t srs[kStage + 1];  // row starts of the block's rows
  const int64_t b = remap ? dev::xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t w0 = b * chunk;  // CSR window [w0, w0 + kStage)
  // 1. window values: column ids, then the local values they name
  C v[L];
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int64_t j = w0 + threadIdx.x + k * kBlock;
    if (j < nnz) v[k] = S::load(xL[dev::ld_nt(ci + j)]);
  }
  // 2. meanwhile, the block's rows and their starts
  const int32_t r0 = bstart[b], r1 = bstart[b + 1];
  const int32_t nrows = r1 - r0;
  const bool rows_staged = nrows <= kStage;
  if (rows_staged) {
#pragma unroll
    for (int k = 0; k <= L; ++k) {
      const int32_t q = threadIdx.x + k * kBlock;
      if (q <= nrows) srs[q] = rs[r0 + q];
    }
  }
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int64_t j = w0 + threadIdx.x + k * kBlock;
    if (j < nnz) lds[threadIdx.x + k * kBlock] = v[k];
  }
  __syncthreads();
  const int64_t lo = rows_staged ? srs[0] : rs[r0];
  const int64_t hi = rows_staged ? srs[nrows] : rs[r1];
  // 3. each thread adds whole rows in CSR order; rows longer than the stage
  //    (only with huge degrees) are added from memory in the same order
  const bool staged = lo >= w0 && hi <= w0 + kStage;
  for (int32_t q = threadIdx.x; q < nrows; q += kBlock) {
    const int32_t a = rows_staged ? srs[q] : rs[r0 + q];
    const int32_t e = rows_staged ? srs[q + 1] : rs[r0 + q + 1];
    C s = C(0);
    if (staged) {
      for (int32_t j = a; j < e; ++j) s += lds[j - w0];
    } else {
      for (int32_t j = a; j < e; ++j) s += S::load(xL[ci[j]]);
    }
    dev::st_nt(xG + r0 + q, S::store(s));
  }
}

// ---------------------------------------------------------------- BS7 scatter, tile order

template <class E>
__global__ __launch_bounds__(kBlock) void k_scatter_tiles(const int32_t* __restrict__ map,
                                                          const int32_t* __restrict__ order,
                                                          const E* __restrict__ xG, E* __restrict__ xL,
                                                          int64_t n_local, bool remap) {
  constexpr int P = kTile / kBlock;
  const uint32_t t = remap ? dev::xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t l0 = static_cast<int64_t>(order[t]) * kTile + threadIdx.x;
  int32_t id[P];
  E v[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int64_t l = l0 + k * kBlock;
    id[k] = (l < n_local) ? dev::ld_nt(map + l) : -1;
  }
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (id[k] >= 0) v[k] = xG[id[k]];
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (id[k] >= 0) dev::st_nt(xL + l0 + k * kBlock, v[k]);
}

inline unsigned int blocks_for(int64_t n) { return static_cast<unsigned int>((n + kBlock - 1) / kBlock); }

template <class T>
bs_status run_gather(bs_ctx* ctx, const bs_gs* gs, const void* xL, void* xG, hipStream_t st) {
  using E = typename Storage<T>::E;
  const Tune& tn = ctx->tune[OP_GATHER][0];
  const bool remap = (tn.variant & 2) == 0;
  if ((tn.variant & 1) == 0) {
    hipLaunchKernelGGL((k_gather_nnz<T>), dim3(static_cast<unsigned int>(gs->n_blocks)), dim3(kBlock), 0, st,
                       gs->row_starts, gs->col_ids, gs->block_starts, static_cast<const E*>(xL), static_cast<E*>(xG),
                       gs->chunk, gs->n_unmasked, remap);
  } else {
    const unsigned int g = static_cast<unsigned int>((gs->n_global + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_gather<T, 1>), dim3(g), dim3(kBlock), 0, st, gs->row_starts, gs->col_ids,
                       static_cast<const E*>(xL), static_cast<E*>(xG), static_cast<int32_t>(gs->n_global), remap);
  }
  return check_launch("bs_gather");
}

template <class E, int U>
void launch_scatter_map(const bs_gs* gs, int cap, const void* xG, void* xL, hipStream_t st) {
  const int64_t per = static_cast<int64_t>(kBlock) * U;
  int64_t g = (gs->n_local + per - 1) / per;
  if (g > cap) g = cap;
  hipLaunchKernelGGL((k_scatter<E, U>), dim3(static_cast<unsigned int>(g)), dim3(kBlock), 0, st, gs->map,
                     static_cast<const E*>(xG), static_cast<E*>(xL), gs->n_local);
}

template <class T>
bs_status run_scatter(bs_ctx* ctx, const bs_gs* gs, const void* xG, void* xL, hipStream_t st) {
  using E = typename Storage<T>::E;
  const Tune& tn = ctx->tune[OP_SCATTER][0];
  if ((tn.variant & 1) == 0) {
    hipLaunchKernelGGL((k_scatter_tiles<E>), dim3(static_cast<unsigned int>(gs->n_tiles)), dim3(kBlock), 0, st,
                       gs->map, gs->tile_order, static_cast<const E*>(xG), static_cast<E*>(xL), gs->n_local,
                       (tn.variant & 2) == 0);
  } else if (tn.unroll >= 8) {
    launch_scatter_map<E, 8>(gs, tn.grid_cap, xG, xL, st);
  } else if (tn.unroll >= 4) {
    launch_scatter_map<E, 4>(gs, tn.grid_cap, xG, xL, st);
  } else if (tn.unroll >= 2) {
    launch_scatter_map<E, 2>(gs, tn.grid_cap, xG, xL, st);
  } else {
    launch_scatter_map<E, 1>(gs, tn.grid_cap, xG, xL, st);
  }
  return check_launch("bs_scatter");
}

bs_status check_gs_op(const char* op, bs_ctx* ctx, const bs_gs* gs, bs_dtype dtype, const void* xL,
                      const void* xG) {
  bs_status s;
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype))) return s;
  if (!gs) return fail(BS_ERR_INVALID_ARG, "%s: plan is NULL", op);
  if (gs->device != ctx->device) return fail(BS_ERR_INVALID_ARG, "%s: plan and context are on different devices", op);
  if ((s = check_vec(op, "xL", xL, gs->n_local, dtype)) || (s = check_vec(op, "xG", xG, gs->n_global, dtype)))
    return s;
  const uintptr_t a = reinterpret_cast<uintptr_t>(xL), b = reinterpret_cast<uintptr_t>(xG);
  const uintptr_t na = static_cast<uintptr_t>(gs->n_local) * dtype_size(dtype);
  const uintptr_t nb = static_cast<uintptr_t>(gs->n_global) * dtype_size(dtype);
  if (na && nb && a < b + nb && b < a + na) return fail(BS_ERR_INVALID_ARG, "%s: xL and xG overlap", op);
  return BS_OK;
}

void free_plan(bs_gs* gs) {
  if (!gs) return;
  (void)hipFree(gs->map);
  (void)hipFree(gs->row_starts);
  (void)hipFree(gs->col_ids);
  (void)hipFree(gs->block_starts);
  (void)hipFree(gs->tile_order);
  delete gs;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" bs_status bs_mesh_hex_map_host(int64_t K, int N, const int32_t* perm, const uint8_t* orient,
                                          int32_t* map) {
  int64_t n_local = 0;
  bs_status s;
  if ((s = check_mesh(K, N, &n_local))) return s;
  if (!map) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map_host: map is NULL");
  const OrientTable T = make_orient_table();
  bool bad = false;
  for (int64_t l = 0; l < n_local; ++l) {
    map[l] = hex_node(l, K, N, perm, orient, T);
    bad |= map[l] < 0;
  }
  if (bad) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map_host: perm or orientation entry out of range");
  return BS_OK;
}

extern "C" bs_status bs_mesh_hex_map(int64_t K, int N, const int32_t* d_perm, const uint8_t* d_orient, int32_t* d_map,
                                     void* stream) {
  int64_t n_local = 0;
  bs_status s;
  if ((s = check_mesh(K, N, &n_local))) return s;
  if (!d_map) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map: d_map is NULL");
  if (!aligned_to(d_map, 4) || (d_perm && !aligned_to(d_perm, 4)))
    return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map: misaligned int32 array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* bad = nullptr;
  if (hipMalloc(&bad, sizeof(int)) != hipSuccess) return fail(BS_ERR_ALLOC, "bs_mesh_hex_map: flag allocation");
  int h_bad = 0;
  s = check_hip(hipMemsetAsync(bad, 0, sizeof(int), st), "bs_mesh_hex_map");
  if (!s) {
    hipLaunchKernelGGL(k_hex_map, dim3(blocks_for(n_local)), dim3(kBlock), 0, st, K, N, d_perm, d_orient,
                       make_orient_table(), d_map, n_local, bad);
    s = check_launch("bs_mesh_hex_map");
  }
  if (!s) s = check_hip(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st), "bs_mesh_hex_map");
  if (!s) s = check_hip(hipStreamSynchronize(st), "bs_mesh_hex_map");
  (void)hipFree(bad);
  if (s) return s;
  if (h_bad) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map: perm or orientation entry out of range");
  return BS_OK;
}

extern "C" bs_status bs_gs_create(bs_ctx* ctx, const int32_t* d_map, int64_t n_local, int64_t n_global, void* stream,
                                  bs_gs** out) {
  const char* op = "bs_gs_create";
  bs_status s;
  if (!out) return fail(BS_ERR_INVALID_ARG, "%s: out is NULL", op);
  *out = nullptr;
  if ((s = check_ctx(ctx, op))) return s;
  if (n_local < 0 || n_global < 0 || n_local >= 2147483647LL || n_global >= 2147483647LL)
    return fail(BS_ERR_INVALID_ARG, "%s: sizes must lie in [0, 2^31 - 1)", op);
  if (n_local > 0 && !d_map) return fail(BS_ERR_INVALID_ARG, "%s: d_map is NULL", op);
  if (d_map && !aligned_to(d_map, 4)) return fail(BS_ERR_INVALID_ARG, "%s: d_map is not 4-byte aligned", op);
  hipStream_t st = static_cast<hipStream_t>(stream);

  bs_gs* gs = new bs_gs();
  gs->device = ctx->device;
  gs->n_local = n_local;
  gs->n_global = n_global;
  uint32_t* keys = nullptr;
  uint32_t* keys_out = nullptr;
  int32_t* vals = nullptr;
  int32_t* vals_out = nullptr;
  int32_t* deg = nullptr;
  int* bad = nullptr;
  void* tmp = nullptr;
  const size_t nl = static_cast<size_t>(n_local > 0 ? n_local : 1);
  const size_t ng = static_cast<size_t>(n_global);
  auto cleanup = [&]() {
    (void)hipFree(keys);
    (void)hipFree(keys_out);
    (void)hipFree(vals);
    (void)hipFree(vals_out);
    (void)hipFree(deg);
    (void)hipFree(bad);
    (void)hipFree(tmp);
  };
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
  if (!alloc(reinterpret_cast<void**>(&gs->map), nl * 4) ||
      !alloc(reinterpret_cast<void**>(&gs->row_starts), (ng + 1) * 4) ||
      !alloc(reinterpret_cast<void**>(&keys), nl * 4) || !alloc(reinterpret_cast<void**>(&keys_out), nl * 4) ||
      !alloc(reinterpret_cast<void**>(&vals), nl * 4) || !alloc(reinterpret_cast<void**>(&vals_out), nl * 4) ||
      !alloc(reinterpret_cast<void**>(&deg), (ng + 1) * 4) || !alloc(reinterpret_cast<void**>(&bad), sizeof(int))) {
    cleanup();
    free_plan(gs);
    return fail(BS_ERR_ALLOC, "%s: out of device memory (n_local=%lld, n_global=%lld)", op, (long long)n_local,
                (long long)n_global);
  }
  int h_bad = 0;
  int32_t h_total = 0;
  s = check_hip(hipMemsetAsync(bad, 0, sizeof(int), st), op);
  if (!s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ng + 1)), dim3(kBlock), 0, st, deg, static_cast<int64_t>(ng + 1), 0);
    if (n_local > 0)
      hipLaunchKernelGGL(k_plan_prepare, dim3(blocks_for(n_local)), dim3(kBlock), 0, st, d_map, n_local,
                         static_cast<int32_t>(n_global), gs->map, keys, vals, deg, bad);
    s = check_launch(op);
  }
  if (!s) s = check_hip(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st), op);
  if (!s) s = check_hip(hipStreamSynchronize(st), op);
  if (!s && h_bad) s = fail(BS_ERR_INVALID_ARG, "%s: map entry >= n_global (%lld)", op, (long long)n_global);
  // row starts: exclusive scan of the degrees (n_global + 1 entries, last degree 0)
  size_t tmp_bytes = 0, sort_bytes = 0;
  int end_bit = 1;
  while ((static_cast<uint64_t>(1) << end_bit) <= static_cast<uint64_t>(n_global)) ++end_bit;
  if (!s) {
    s = check_hip(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, deg, gs->row_starts,
                                                   static_cast<int>(ng + 1), st), op);
    if (!s && n_local > 0)
      s = check_hip(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, keys, keys_out, vals, vals_out,
                                                        static_cast<int>(n_local), 0, end_bit, st), op);
    if (sort_bytes > tmp_bytes) tmp_bytes = sort_bytes;
    if (!s && !alloc(&tmp, tmp_bytes ? tmp_bytes : 1)) s = fail(BS_ERR_ALLOC, "%s: scratch allocation", op);
  }
  if (!s)
    s = check_hip(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, deg, gs->row_starts, static_cast<int>(ng + 1), st),
                  op);
  if (!s && n_local > 0) {
    size_t b = tmp_bytes;
    s = check_hip(hipcub::DeviceRadixSort::SortPairs(tmp, b, keys, keys_out, vals, vals_out,
                                                      static_cast<int>(n_local), 0, end_bit, st), op);
  }
  if (!s)
    s = check_hip(hipMemcpyAsync(&h_total, gs->row_starts + ng, sizeof(int32_t), hipMemcpyDeviceToHost, st), op);
  if (!s) s = check_hip(hipStreamSynchronize(st), op);
  if (!s) {
    gs->n_unmasked = h_total;
    if (!alloc(reinterpret_cast<void**>(&gs->col_ids), static_cast<size_t>(h_total > 0 ? h_total : 1) * 4))
      s = fail(BS_ERR_ALLOC, "%s: column-id allocation", op);
  }
  if (!s && h_total > 0)
    s = check_hip(hipMemcpyAsync(gs->col_ids, vals_out, static_cast<size_t>(h_total) * 4, hipMemcpyDeviceToDevice, st),
                  op);
  // largest degree (for plan info and for choosing gather paths)
  int32_t* d_max = reinterpret_cast<int32_t*>(bad);
  int32_t h_max = 0;
  if (!s && ng > 0) {
    size_t b = 0;
    s = check_hip(hipcub::DeviceReduce::Max(nullptr, b, deg, d_max, static_cast<int>(ng), st), op);
    if (!s && b <= tmp_bytes) {
      s = check_hip(hipcub::DeviceReduce::Max(tmp, b, deg, d_max, static_cast<int>(ng), st), op);
    } else if (!s) {
      void* t2 = nullptr;
      if (!alloc(&t2, b)) {
        s = fail(BS_ERR_ALLOC, "%s: scratch allocation", op);
      } else {
        s = check_hip(hipcub::DeviceReduce::Max(t2, b, deg, d_max, static_cast<int>(ng), st), op);
        if (!s) s = check_hip(hipStreamSynchronize(st), op);
        (void)hipFree(t2);
      }
    }
    if (!s) s = check_hip(hipMemcpyAsync(&h_max, d_max, sizeof(int32_t), hipMemcpyDeviceToHost, st), op);
  }
  if (!s) s = check_hip(hipStreamSynchronize(st), op);
  gs->max_degree = h_max;
  // gather blocks: windows of kStage values, consecutive windows `chunk` apart
  if (!s) {
    const int64_t md = h_max;
    gs->chunk = (md <= kStage / 2) ? kStage - md : kStage / 2;
    gs->n_blocks = (gs->n_unmasked + gs->chunk - 1) / gs->chunk;
    if (gs->n_blocks < 1) gs->n_blocks = 1;
    if (!alloc(reinterpret_cast<void**>(&gs->block_starts), static_cast<size_t>(gs->n_blocks + 1) * 4)) {
      s = fail(BS_ERR_ALLOC, "%s: block-start allocation", op);
    } else {
      hipLaunchKernelGGL(k_block_starts, dim3(blocks_for(gs->n_blocks + 1)), dim3(kBlock), 0, st, gs->row_starts,
                         static_cast<int32_t>(n_global), gs->chunk, gs->n_blocks, gs->block_starts);
      s = check_launch(op);
    }
  }
  // scatter tiles, sorted (stably) by the smallest global id they reference
  if (!s) {
    gs->n_tiles = (n_local + kTile - 1) / kTile;
    if (!alloc(reinterpret_cast<void**>(&gs->tile_order), static_cast<size_t>(gs->n_tiles > 0 ? gs->n_tiles : 1) * 4))
      s = fail(BS_ERR_ALLOC, "%s: tile-order allocation", op);
  }
  if (!s && gs->n_tiles > 0) {
    // keys/vals (n_local entries each) are free again and n_tiles < n_local
    const int nt = static_cast<int>(gs->n_tiles);
    hipLaunchKernelGGL(k_tile_keys, dim3(static_cast<unsigned int>(nt)), dim3(kBlock), 0, st, gs->map, n_local, keys,
                       vals);
    s = check_launch(op);
    size_t b = 0;
    if (!s) s = check_hip(hipcub::DeviceRadixSort::SortPairs(nullptr, b, keys, keys_out, vals, gs->tile_order, nt, 0, 32, st), op);
    void* t2 = nullptr;
    if (!s && !alloc(&t2, b ? b : 1)) s = fail(BS_ERR_ALLOC, "%s: scratch allocation", op);
    if (!s) s = check_hip(hipcub::DeviceRadixSort::SortPairs(t2, b, keys, keys_out, vals, gs->tile_order, nt, 0, 32, st), op);
    if (!s) s = check_hip(hipStreamSynchronize(st), op);
    (void)hipFree(t2);
  }
  cleanup();
  if (s) {
    free_plan(gs);
    return s;
  }
  *out = gs;
  return BS_OK;
}

extern "C" bs_status bs_gs_destroy(bs_gs* gs) {
  if (!gs) return BS_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(gs->device);
  free_plan(gs);
  (void)hipSetDevice(prev);
  return BS_OK;
}

extern "C" bs_status bs_gs_info(const bs_gs* gs, int64_t* n_local, int64_t* n_global, int64_t* n_unmasked,
                                int64_t* max_degree) {
  if (!gs) return fail(BS_ERR_INVALID_ARG, "bs_gs_info: plan is NULL");
  if (n_local) *n_local = gs->n_local;
  if (n_global) *n_global = gs->n_global;
  if (n_unmasked) *n_unmasked = gs->n_unmasked;
  if (max_degree) *max_degree = gs->max_degree;
  return BS_OK;
}

extern "C" bs_status bs_gs_csr(const bs_gs* gs, int32_t* d_row_starts, int32_t* d_col_ids, void* stream) {
  if (!gs) return fail(BS_ERR_INVALID_ARG, "bs_gs_csr: plan is NULL");
  if (!d_row_starts || (gs->n_unmasked > 0 && !d_col_ids))
    return fail(BS_ERR_INVALID_ARG, "bs_gs_csr: output is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  bs_status s = check_hip(hipMemcpyAsync(d_row_starts, gs->row_starts, static_cast<size_t>(gs->n_global + 1) * 4,
                                         hipMemcpyDeviceToDevice, st),
                          "bs_gs_csr");
  if (!s && gs->n_unmasked > 0)
    s = check_hip(hipMemcpyAsync(d_col_ids, gs->col_ids, static_cast<size_t>(gs->n_unmasked) * 4,
                                 hipMemcpyDeviceToDevice, st),
                  "bs_gs_csr");
  return s;
}

extern "C" bs_status bs_gs_degree(const bs_gs* gs, int32_t* d_deg, void* stream) {
  if (!gs) return fail(BS_ERR_INVALID_ARG, "bs_gs_degree: plan is NULL");
  if (gs->n_global == 0) return BS_OK;
  if (!d_deg || !aligned_to(d_deg, 4)) return fail(BS_ERR_INVALID_ARG, "bs_gs_degree: d_deg is NULL or misaligned");
  hipLaunchKernelGGL(k_degree, dim3(blocks_for(gs->n_global)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                     gs->row_starts, static_cast<int32_t>(gs->n_global), d_deg);
  return check_launch("bs_gs_degree");
}

extern "C" bs_status bs_gs_weights(const bs_gs* gs, bs_dtype dtype, void* d_wL, void* stream) {
  bs_status s;
  if (!gs) return fail(BS_ERR_INVALID_ARG, "bs_gs_weights: plan is NULL");
  if ((s = check_dtype("bs_gs_weights", dtype)) || (s = check_vec("bs_gs_weights", "d_wL", d_wL, gs->n_local, dtype)))
    return s;
  if (gs->n_local == 0) return BS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 g(blocks_for(gs->n_local));
  switch (dtype) {
    case BS_F64:
      hipLaunchKernelGGL(k_weights<double>, g, dim3(kBlock), 0, st, gs->map, gs->row_starts, gs->n_local,
                         static_cast<double*>(d_wL));
      break;
    case BS_F32:
      hipLaunchKernelGGL(k_weights<float>, g, dim3(kBlock), 0, st, gs->map, gs->row_starts, gs->n_local,
                         static_cast<float*>(d_wL));
      break;
    case BS_BF16:
      hipLaunchKernelGGL(k_weights<bf16>, g, dim3(kBlock), 0, st, gs->map, gs->row_starts, gs->n_local,
                         static_cast<uint16_t*>(d_wL));
      break;
  }
  return check_launch("bs_gs_weights");
}

extern "C" bs_status bs_gather(bs_ctx* ctx, const bs_gs* gs, bs_dtype dtype, const void* xL, void* xG, void* stream) {
  bs_status s;
  if ((s = check_gs_op("bs_gather", ctx, gs, dtype, xL, xG))) return s;
  if (gs->n_global == 0) return BS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case BS_F64: return run_gather<double>(ctx, gs, xL, xG, st);
    case BS_F32: return run_gather<float>(ctx, gs, xL, xG, st);
    case BS_BF16: return run_gather<bf16>(ctx, gs, xL, xG, st);
  }
  return fail(BS_ERR_INVALID_ARG, "bs_gather: unknown dtype");
}

extern "C" bs_status bs_scatter(bs_ctx* ctx, const bs_gs* gs, bs_dtype dtype, const void* xG, void* xL,
                                void* stream) {
  bs_status s;
  if ((s = check_gs_op("bs_scatter", ctx, gs, dtype, xL, xG))) return s;
  if (gs->n_local == 0) return BS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case BS_F64: return run_scatter<double>(ctx, gs, xG, xL, st);
    case BS_F32: return run_scatter<float>(ctx, gs, xG, xL, st);
    case BS_BF16: return run_scatter<bf16>(ctx, gs, xG, xL, st);
  }
  return fail(BS_ERR_INVALID_ARG, "bs_scatter: unknown dtype");
}
