// BS6 gather and BS7 scatter (Table 1; Listings 4 and 5).
//
// Both take a plan (bs_plan.hip).  Each has three kernels, chosen by the
// context's tune variant; all give the same bits.
//
// Gather x_G = Z^T x_L adds the local copies of every global node one at a
// time in ascending local index, starting from +0.0.  Workgroups take about
// the same number of nonzeros of the CSR (the paper's blockStarts blocking,
// Section 5), stage the local values of their CSR window in LDS and then add
// whole rows from LDS.  The window start is known from the block index, so
// the column-id and value loads are issued at once rather than after the
// row starts arrive.
//   0  rows in the plan's permuted order: by default in groups of 9
//      consecutive scatter tiles of the visiting order (each row in the
//      first group holding one of its copies, ascending global id within a
//      group), so that a row's copies lie in tiles whose cache lines are
//      still in L2 and x_G is written in runs (needs every degree to fit in
//      a byte, otherwise kernel 1 runs)
//   1  rows in global order
//   2  fixed blocks of 256 rows in global order
//
// Scatter x_L = Z x_G copies x_G[map[l]] to every unmasked local entry.
//   0  tiles of 512 local entries, visited in order of their smallest global
//      id; each tile reads its x_G values in ascending global id (so that a
//      wave reads runs of neighbouring entries), turns them around in LDS
//      and writes its x_L entries contiguously (the default)
//   1  the same tiles, read in local order
//   2  local order over the whole vector, `unroll` entries per thread
//
// For gather kernel 0 and scatter kernel 0, tune variant + 16 selects cached
// instead of nontemporal accesses (arrays that stay in the last-level cache
// between calls).
//
// Workgroups are renumbered per XCD so that neighbouring blocks, which share
// cache lines, run on the same XCD's L2: by default each XCD takes one
// contiguous range of blocks; the tune variant may instead keep the dispatch
// order (+4) or give each XCD runs of 256 blocks in every group of 2048 (+8).

#include <type_traits>

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

using dev::bf16;
using dev::Storage;

// Accesses of the index words and of the values the kernels stream: by
// default nontemporal; with NT = false (tune variant + 16, for meshes whose
// arrays stay in the 256 MB last-level cache from one call to the next)
// ordinary cached ones.
template <bool NT, class X>
__device__ __forceinline__ X ld_pol(const X* p) {
  if constexpr (NT) return dev::ld_nt(p);
  else return *p;
}
template <bool NT, class X>
__device__ __forceinline__ void st_pol(X* p, const X& v) {
  if constexpr (NT) dev::st_nt(p, v);
  else *p = v;
}

// ---------------------------------------------------------------- BS6 gather, rows in visiting order

// ((+0 + v[a]) + v[a+1]) + ... + v[e-1], with the LDS reads issued four at a time.
template <class C>
__device__ __forceinline__ C row_sum(const C* v, int32_t a, int32_t e) {
  C s = C(0);
  int32_t j = a;
  for (; j + 4 <= e; j += 4) {
    const C t0 = v[j], t1 = v[j + 1], t2 = v[j + 2], t3 = v[j + 3];
    s += t0;
    s += t1;
    s += t2;
    s += t3;
  }
  for (; j < e; ++j) s += v[j];
  return s;
}

// A workgroup owns the rows of one block and the CSR window of their
// nonzeros (at most kStage).  The plan stores the window in ascending local
// index, one word per entry (segment rank, column mod 512, CSR offset,
// row-start bit), so that lanes of one load share cache lines; each value is
// put in LDS at its CSR offset, the rows' starts are recovered from the
// row-start bits, and every row adds its copies from LDS in CSR order, i.e.
// in ascending local index, as the definition of x_G = Z^T x_L does.
// Seven workgroups per CU: 21.5 KB of LDS each, and at most 72 VGPRs.
template <class T, bool NT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_gather_perm(
    const uint32_t* __restrict__ words, const int32_t* __restrict__ segs, const int32_t* __restrict__ segoff,
    const int32_t* __restrict__ prows, const int32_t* __restrict__ runoff, const int32_t* __restrict__ runs,
    const int32_t* __restrict__ pbstart, const int32_t* __restrict__ pbnz0,
    const typename Storage<T>::E* __restrict__ xL, typename Storage<T>::E* __restrict__ xG, int64_t n_pblocks,
    int64_t n_nzrows, int64_t n_rows, int wg_order) {
  using S = Storage<T>;
  using C = typename S::C;
  using E = typename S::E;
  static_assert(2 * kRunCap * sizeof(int32_t) <= kStage * sizeof(C), "the run table fits in the value stage");
  constexpr int L = kStage / kBlock;
  static_assert(L == 8, "a thread scans the row-start bytes of 8 offsets as one word");
  constexpr int kSegCap = 256;
  __shared__ C lds[kStage];                    // the window's local values, CSR order
  __shared__ uint64_t sraw[(kStage + 8) / 4];  // row-start bytes (until step 3), then 16-bit row starts
  __shared__ int32_t lseg[kSegCap];            // the window's segment ids, when they fit (else read in place)
  __shared__ int32_t wsum[kBlock / 64];
  uint64_t* first64 = sraw;
  uint8_t* first = reinterpret_cast<uint8_t*>(sraw);
  uint16_t* sst = reinterpret_cast<uint16_t*>(sraw);
  const int t = threadIdx.x;
  const int64_t b = dev::block_order(blockIdx.x, gridDim.x, wg_order);
  if (b >= n_pblocks) {  // rows without copies: +0.0
    const int64_t q = n_nzrows + (b - n_pblocks) * kBlock + t;
    if (q < n_rows) st_pol<NT>(xG + prows[q], S::store(C(0)));
    return;
  }
  const int64_t w0 = pbnz0[b];
  const int32_t n = static_cast<int32_t>(pbnz0[b + 1] - w0);  // <= kStage
  if (n == 0) return;  // a trailing block whose range holds no row start
  const int32_t s0 = segoff[b], ns = segoff[b + 1] - s0;      // <= n
  const int32_t r0 = pbstart[b], nrows = pbstart[b + 1] - r0;  // in [1, n]
  const int32_t u0 = runoff[b], nr = runoff[b + 1] - u0;        // in [1, nrows]
  const bool by_runs = nr <= kRunCap;
  // the run table (first row, first id) sits in the value stage until step 4
  int32_t* rpos = reinterpret_cast<int32_t*>(lds);
  int32_t* rgid = rpos + kRunCap;
  // 1. the window's words, its segment ids, and the rows' global ids (as
  //    runs, or, for a block with many runs, those of the rows this thread
  //    adds in step 5: q = t + k kBlock); lanes past the end repeat the last
  //    entry, so that no load waits behind a branch
  uint32_t wd[L];
#pragma unroll
  for (int k = 0; k < L; ++k) wd[k] = ld_pol<NT>(words + w0 + min(t + k * kBlock, n - 1));
  int32_t gid[L];
  if (by_runs) {
    for (int i = t; i < nr; i += kBlock) {
      rpos[i] = runs[2 * (u0 + i)];
      rgid[i] = runs[2 * (u0 + i) + 1];
    }
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k) gid[k] = prows[r0 + min(t + k * kBlock, nrows - 1)];
  }
  const bool seg_lds = ns <= kSegCap;
  if (seg_lds)
    for (int i = t; i < ns; i += kBlock) lseg[i] = segs[s0 + i];
#pragma unroll
  for (int k = 0; k < L; ++k)
    if (t + k * kBlock < n) first[(wd[k] >> 1) & 2047u] = static_cast<uint8_t>(wd[k] & 1u);
  __syncthreads();
  // 2. the values, in address order
  E v[L];
  if (seg_lds) {
#pragma unroll
    for (int k = 0; k < L; ++k)
      v[k] = xL[static_cast<int64_t>(lseg[wd[k] >> 21]) * 512 + ((wd[k] >> 12) & 511u)];
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k)
      v[k] = xL[static_cast<int64_t>(segs[s0 + (wd[k] >> 21)]) * 512 + ((wd[k] >> 12) & 511u)];
  }
  // 3. meanwhile the rows' global ids from the runs (the last run that
  //    starts at or before the row) and the row starts: thread t reads the
  //    row-start bytes of offsets t*L .. t*L+L-1 (every offset below n was
  //    written once)
  if (by_runs) {  // the eight searches advance together, one LDS read each per step
    int32_t q[L], lo[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      q[k] = min(t + k * kBlock, nrows - 1);
      lo[k] = 0;
    }
    for (int step = 1 << (31 - __clz(nr)); step > 0; step >>= 1) {
#pragma unroll
      for (int k = 0; k < L; ++k) {
        const int probe = min(lo[k] + step, nr - 1);
        if (rpos[probe] <= q[k]) lo[k] = max(lo[k], probe);
      }
    }
#pragma unroll
    for (int k = 0; k < L; ++k) gid[k] = rgid[lo[k]] + (q[k] - rpos[lo[k]]);
  }
  const uint64_t fl = first64[t];
  int32_t tsum = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) tsum += (t * L + i < n) ? static_cast<int32_t>((fl >> (8 * i)) & 1u) : 0;
  const int lane = t % 64, w = t / 64;
  int32_t incl = tsum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();  // also: every row-start byte has been read
  int32_t before = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) before += (i < w) ? wsum[i] : 0;
  int32_t row = before + incl - tsum;
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (t * L + i < n && ((fl >> (8 * i)) & 1u)) sst[row++] = static_cast<uint16_t>(t * L + i);
  if (t == 0) sst[nrows] = static_cast<uint16_t>(n);
  // 4. the values into LDS at their CSR offsets
#pragma unroll
  for (int k = 0; k < L; ++k)
    if (t + k * kBlock < n) lds[(wd[k] >> 1) & 2047u] = S::load(v[k]);
  __syncthreads();
  // 5. each thread adds whole rows in CSR order
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int32_t q = t + k * kBlock;
    if (q < nrows) st_pol<NT>(xG + gid[k], S::store(row_sum<C>(lds, sst[q], sst[q + 1])));
  }
}

// ---------------------------------------------------------------- BS6 gather, rows in global order

template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_nnz(const int32_t* __restrict__ rs, const int32_t* __restrict__ ci,
                                                       const int32_t* __restrict__ bstart,
                                                       const typename Storage<T>::E* __restrict__ xL,
                                                       typename Storage<T>::E* __restrict__ xG, int64_t chunk,
                                                       int64_t nnz, int wg_order) {
  using S = Storage<T>;
  using C = typename S::C;
  constexpr int L = kStage / kBlock;
  __shared__ C lds[kStage];            // local values of the CSR window
  __shared__ int32_t srs[kStage + 1];  // row starts of the block's rows
  const int64_t b = dev::block_order(blockIdx.x, gridDim.x, wg_order);
  const int64_t w0 = b * chunk;  // CSR window [w0, w0 + kStage)
  // 1. window values: all column ids, then the local values they name
  //    (lanes past the end repeat the last entry, so that no load waits
  //    behind a branch).  The plan has at least one block, so a plan
  //    without nonzeros has a block with an empty window.
  C v[L];
  if (w0 < nnz) {
    int32_t col[L];
#pragma unroll
    for (int k = 0; k < L; ++k) col[k] = dev::ld_nt(ci + min(w0 + threadIdx.x + k * kBlock, nnz - 1));
#pragma unroll
    for (int k = 0; k < L; ++k) v[k] = S::load(xL[col[k]]);
  }
  // 2. meanwhile, the block's rows and their starts
  const int32_t r0 = bstart[b], r1 = bstart[b + 1];
  const int32_t nrows = r1 - r0;
  const bool rows_staged = nrows <= kStage;
  if (rows_staged) {
    int32_t st[L + 1];
#pragma unroll
    for (int k = 0; k <= L; ++k) st[k] = rs[r0 + min(static_cast<int32_t>(threadIdx.x) + k * kBlock, nrows)];
#pragma unroll
    for (int k = 0; k <= L; ++k) {
      const int32_t q = threadIdx.x + k * kBlock;
      if (q <= nrows) srs[q] = st[k];
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
      s = row_sum<C>(lds, static_cast<int32_t>(a - w0), static_cast<int32_t>(e - w0));
    } else {
      for (int32_t j = a; j < e; ++j) s += S::load(xL[ci[j]]);
    }
    dev::st_nt(xG + r0 + q, S::store(s));
  }
}

// ---------------------------------------------------------------- BS6 gather, fixed row blocks

template <class T, int RPT>
__global__ __launch_bounds__(kBlock) void k_gather(const int32_t* __restrict__ rs, const int32_t* __restrict__ ci,
                                                   const typename Storage<T>::E* __restrict__ xL,
                                                   typename Storage<T>::E* __restrict__ xG, int32_t n_global, int wg_order) {
  using S = Storage<T>;
  using C = typename S::C;
  constexpr int R = kBlock * RPT;    // rows per workgroup
  constexpr int CAP = 8 * R;         // staged values: up to an average degree of 8
  constexpr int L = CAP / kBlock;    // staged values per thread
  __shared__ C lds[CAP];
  const int32_t b = static_cast<int32_t>(dev::block_order(blockIdx.x, gridDim.x, wg_order));
  const int32_t row0 = b * R;
  const int32_t row1 = min(row0 + R, n_global);
  const int32_t base = rs[row0];
  const int32_t nnz = rs[row1] - base;
  if (nnz <= CAP) {
    if (nnz > 0) {  // all column ids, then all values (lanes past the end repeat the last entry)
      int32_t col[L];
#pragma unroll
      for (int k = 0; k < L; ++k) col[k] = ci[base + min(static_cast<int32_t>(threadIdx.x) + k * kBlock, nnz - 1)];
      C v[L];
#pragma unroll
      for (int k = 0; k < L; ++k) v[k] = S::load(xL[col[k]]);
#pragma unroll
      for (int k = 0; k < L; ++k) {
        const int32_t i = threadIdx.x + k * kBlock;
        if (i < nnz) lds[i] = v[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int32_t row = row0 + q * kBlock + threadIdx.x;
      if (row < row1) {
        xG[row] = S::store(row_sum<C>(lds, rs[row] - base, rs[row + 1] - base));
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

// ---------------------------------------------------------------- BS7 scatter, sorted tiles

// A workgroup takes TPW consecutive tiles of the visiting order.  Within a
// tile the (global id, local offset) pairs are read in ascending global id
// (PACKED: one word per pair, id - tile minimum above the 9-bit offset), the
// values fetched in that order and put in place through LDS, and the tile's
// entries are written contiguously.  The plan stores the pairs in visiting
// order, so they are loaded alongside the tile's index, not after it.
template <class E, int TPW, bool PACKED, bool NT>
__global__ __launch_bounds__(kBlock) void k_scatter_sorted(const int32_t* __restrict__ order,
                                                           const int32_t* __restrict__ tgid,
                                                           const uint16_t* __restrict__ tloc,
                                                           const uint32_t* __restrict__ tword,
                                                           const int32_t* __restrict__ tmin,
                                                           const int32_t* __restrict__ tcnt, const E* __restrict__ xG,
                                                           E* __restrict__ xL, int64_t n_local, int64_t n_tiles,
                                                           int wg_order) {
  constexpr int P = kTile / kBlock;
  __shared__ E val[TPW][kTile];
  __shared__ uint8_t has[TPW][kTile];
  const int64_t t0 = static_cast<int64_t>(dev::block_order(blockIdx.x, gridDim.x, wg_order)) * TPW;
  int64_t tile[TPW];
  int cnt[TPW];
  int32_t g0[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) tile[i] = order[min(t0 + i, n_tiles - 1)];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int64_t v = min(t0 + i, n_tiles - 1);
    cnt[i] = (t0 + i < n_tiles) ? tcnt[v] : 0;
    if (PACKED) g0[i] = tmin[v];
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k) has[i][threadIdx.x + k * kBlock] = 0;
  int32_t g[TPW][P];
  uint16_t o[TPW][P];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int q = min(static_cast<int>(threadIdx.x) + k * kBlock, kTile - 1);
      const int64_t v = min(t0 + i, n_tiles - 1);
      if (PACKED) {
        const uint32_t w = ld_pol<NT>(tword + v * kTile + q);
        g[i][k] = g0[i] + static_cast<int32_t>(w >> 9);
        o[i][k] = static_cast<uint16_t>(w & 511u);
      } else {
        g[i][k] = ld_pol<NT>(tgid + v * kTile + q);
        o[i][k] = ld_pol<NT>(tloc + v * kTile + q);
      }
    }
  E v[TPW][P];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int q = threadIdx.x + k * kBlock;
      v[i][k] = xG[q < cnt[i] ? g[i][k] : 0];
    }
  __syncthreads();  // has[] cleared
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (static_cast<int>(threadIdx.x) + k * kBlock < cnt[i]) {
        val[i][o[i][k]] = v[i][k];
        has[i][o[i][k]] = 1;
      }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int64_t base = tile[i] * kTile;
    const int64_t rem = n_local - base;
    const int ntile = (t0 + i < n_tiles) ? (rem < kTile ? static_cast<int>(rem) : kTile) : 0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int q = threadIdx.x + k * kBlock;
      if (q < ntile && has[i][q]) st_pol<NT>(xL + base + q, val[i][q]);
    }
  }
}

// ---------------------------------------------------------------- BS7 scatter, tiles in local order

// A workgroup takes TPW consecutive tiles of the visiting order and copies
// xG[map[l]] to xL[l] over each: ids first, then values, then stores.
template <class E, int TPW>
__global__ __launch_bounds__(kBlock) void k_scatter_tiles(const int32_t* __restrict__ map,
                                                          const int32_t* __restrict__ order,
                                                          const E* __restrict__ xG, E* __restrict__ xL,
                                                          int64_t n_local, int64_t n_tiles, int wg_order) {
  constexpr int P = kTile / kBlock;
  const int64_t t0 = static_cast<int64_t>(dev::block_order(blockIdx.x, gridDim.x, wg_order)) * TPW;
  int64_t l0[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) l0[i] = static_cast<int64_t>(order[min(t0 + i, n_tiles - 1)]) * kTile + threadIdx.x;
  int32_t id[TPW][P];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k) id[i][k] = dev::ld_nt(map + min(l0[i] + k * kBlock, n_local - 1));
  E v[TPW][P];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k) v[i][k] = xG[max(id[i][k], 0)];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int64_t l = l0[i] + k * kBlock;
      if (t0 + i < n_tiles && l < n_local && id[i][k] >= 0) dev::st_nt(xL + l, v[i][k]);
    }
}

// ---------------------------------------------------------------- BS7 scatter, local order

template <class E, int U>
__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t* __restrict__ map, const E* __restrict__ xG,
                                                    E* __restrict__ xL, int64_t n_local, int64_t n_global) {
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
      if (id[u] >= 0 && id[u] < n_global) v[u] = xG[id[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (id[u] >= 0 && id[u] < n_global) dev::st_nt(xL + i + static_cast<int64_t>(u) * kBlock, v[u]);
  }
}

inline unsigned int blocks_for(int64_t n) { return static_cast<unsigned int>((n + kBlock - 1) / kBlock); }

template <class T> constexpr int dtype_index() { return std::is_same<T, double>::value ? 0 : std::is_same<T, float>::value ? 1 : 2; }

// Bytes one gather or scatter moves: both value vectors and one 4-byte index
// per local entry (what decides whether cached accesses can pay).
template <class E>
int64_t gs_operand_bytes(const bs_gs* gs) {
  return (gs->n_local + gs->n_global) * static_cast<int64_t>(sizeof(E)) + 4 * gs->n_local;
}

template <class T>
bs_status run_gather(bs_ctx* ctx, const bs_gs* gs, const void* xL, void* xG, hipStream_t st) {
  using E = typename Storage<T>::E;
  const Tune& tn = tune_for(ctx, OP_GATHER, dtype_index<T>(), gs->n_local);
  const int order = gs_order(tn.variant);
  int kind = tn.variant & kVariantMask;
  if (kind == 0 && !gs->has_perm) kind = 1;
  if (kind == 0) {
    const int64_t zero_blocks = (gs->n_global - gs->n_nzrows + kBlock - 1) / kBlock;
    const int64_t grid = gs->n_pblocks + zero_blocks;
    if (grid > 0) {
      if (cached_access(tn.variant, gs_operand_bytes<E>(gs)))
        hipLaunchKernelGGL((k_gather_perm<T, false>), dim3(static_cast<unsigned int>(grid)), dim3(kBlock), 0, st,
                           gs->perm_words, gs->perm_segs, gs->perm_segoff, gs->perm_rows, gs->perm_runoff,
                           gs->perm_runs, gs->perm_bstart, gs->perm_bnz0, static_cast<const E*>(xL),
                           static_cast<E*>(xG), gs->n_pblocks, gs->n_nzrows, gs->n_global, order);
      else
        hipLaunchKernelGGL((k_gather_perm<T, true>), dim3(static_cast<unsigned int>(grid)), dim3(kBlock), 0, st,
                           gs->perm_words, gs->perm_segs, gs->perm_segoff, gs->perm_rows, gs->perm_runoff,
                           gs->perm_runs, gs->perm_bstart, gs->perm_bnz0, static_cast<const E*>(xL),
                           static_cast<E*>(xG), gs->n_pblocks, gs->n_nzrows, gs->n_global, order);
    }
  } else if (kind == 1) {
    hipLaunchKernelGGL((k_gather_nnz<T>), dim3(static_cast<unsigned int>(gs->n_blocks)), dim3(kBlock), 0, st,
                       gs->row_starts, gs->col_ids, gs->block_starts, static_cast<const E*>(xL), static_cast<E*>(xG),
                       gs->chunk, gs->n_unmasked, order);
  } else {
    const unsigned int g = blocks_for(gs->n_global);
    hipLaunchKernelGGL((k_gather<T, 1>), dim3(g), dim3(kBlock), 0, st, gs->row_starts, gs->col_ids,
                       static_cast<const E*>(xL), static_cast<E*>(xG), static_cast<int32_t>(gs->n_global), order);
  }
  return check_launch("bs_gather");
}

template <class E, int U>
void launch_scatter_map(const int32_t* map, int64_t n_local, int64_t n_global, int cap, const void* xG, void* xL,
                        hipStream_t st) {
  const int64_t per = static_cast<int64_t>(kBlock) * U;
  int64_t g = (n_local + per - 1) / per;
  if (g > cap) g = cap;
  hipLaunchKernelGGL((k_scatter<E, U>), dim3(static_cast<unsigned int>(g)), dim3(kBlock), 0, st, map,
                     static_cast<const E*>(xG), static_cast<E*>(xL), n_local, n_global);
}

// Plain scatter from a map (local order, `unroll` entries per thread).
template <class E>
void scatter_by_map(int unroll, const int32_t* map, int64_t n_local, int64_t n_global, int cap, const void* xG,
                    void* xL, hipStream_t st) {
  if (unroll >= 8) launch_scatter_map<E, 8>(map, n_local, n_global, cap, xG, xL, st);
  else if (unroll >= 4) launch_scatter_map<E, 4>(map, n_local, n_global, cap, xG, xL, st);
  else if (unroll >= 2) launch_scatter_map<E, 2>(map, n_local, n_global, cap, xG, xL, st);
  else launch_scatter_map<E, 1>(map, n_local, n_global, cap, xG, xL, st);
}

template <class E, int TPW, bool NT>
void launch_scatter_sorted_nt(const bs_gs* gs, int wg_order, const void* xG, void* xL, hipStream_t st) {
  const unsigned int grid = static_cast<unsigned int>((gs->n_tiles + TPW - 1) / TPW);
  if (gs->tile_packed)
    hipLaunchKernelGGL((k_scatter_sorted<E, TPW, true, NT>), dim3(grid), dim3(kBlock), 0, st, gs->tile_order,
                       static_cast<const int32_t*>(nullptr), static_cast<const uint16_t*>(nullptr), gs->tile_word,
                       gs->tile_min, gs->tile_count, static_cast<const E*>(xG), static_cast<E*>(xL), gs->n_local,
                       gs->n_tiles, wg_order);
  else
    hipLaunchKernelGGL((k_scatter_sorted<E, TPW, false, NT>), dim3(grid), dim3(kBlock), 0, st, gs->tile_order,
                       gs->tile_gid, gs->tile_loc, static_cast<const uint32_t*>(nullptr),
                       static_cast<const int32_t*>(nullptr), gs->tile_count, static_cast<const E*>(xG),
                       static_cast<E*>(xL), gs->n_local, gs->n_tiles, wg_order);
}

template <class E, int TPW>
void launch_scatter_sorted(const bs_gs* gs, int wg_order, bool cached, const void* xG, void* xL, hipStream_t st) {
  if (cached) launch_scatter_sorted_nt<E, TPW, false>(gs, wg_order, xG, xL, st);
  else launch_scatter_sorted_nt<E, TPW, true>(gs, wg_order, xG, xL, st);
}

template <class E, int TPW>
void launch_scatter_tiles(const bs_gs* gs, int wg_order, const void* xG, void* xL, hipStream_t st) {
  const unsigned int grid = static_cast<unsigned int>((gs->n_tiles + TPW - 1) / TPW);
  hipLaunchKernelGGL((k_scatter_tiles<E, TPW>), dim3(grid), dim3(kBlock), 0, st, gs->map, gs->tile_order,
                     static_cast<const E*>(xG), static_cast<E*>(xL), gs->n_local, gs->n_tiles, wg_order);
}

template <class T>
bs_status run_scatter(bs_ctx* ctx, const bs_gs* gs, const void* xG, void* xL, hipStream_t st) {
  using E = typename Storage<T>::E;
  const Tune& tn = tune_for(ctx, OP_SCATTER, dtype_index<T>(), gs->n_local);
  const int order = gs_order(tn.variant);
  const int kind = tn.variant & kVariantMask;
  if (kind <= 1) {
    // tiles per workgroup: the tune entry's unroll, rounded down to 1, 2 or 4
    const int tpw = tn.unroll >= 4 ? 4 : tn.unroll >= 2 ? 2 : 1;
    // (with no global entries every local entry is masked: nothing to write,
    // and the kernels' padding lanes read xG[0])
    if (gs->n_tiles > 0 && gs->n_global > 0) {
      if (kind == 0) {
        const bool cached = cached_access(tn.variant, gs_operand_bytes<E>(gs));
        if (tpw == 4) launch_scatter_sorted<E, 4>(gs, order, cached, xG, xL, st);
        else if (tpw == 2) launch_scatter_sorted<E, 2>(gs, order, cached, xG, xL, st);
        else launch_scatter_sorted<E, 1>(gs, order, cached, xG, xL, st);
      } else {
        if (tpw == 4) launch_scatter_tiles<E, 4>(gs, order, xG, xL, st);
        else if (tpw == 2) launch_scatter_tiles<E, 2>(gs, order, xG, xL, st);
        else launch_scatter_tiles<E, 1>(gs, order, xG, xL, st);
      }
    }
  } else {
    scatter_by_map<E>(tn.unroll, gs->map, gs->n_local, gs->n_global, tn.grid_cap, xG, xL, st);
  }
  return check_launch("bs_gs_scatter");
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

}  // namespace
}  // namespace bs

using namespace bs;

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

extern "C" bs_status bs_gs_scatter(bs_ctx* ctx, const bs_gs* gs, bs_dtype dtype, const void* xG, void* xL,
                                   void* stream) {
  bs_status s;
  if ((s = check_gs_op("bs_gs_scatter", ctx, gs, dtype, xL, xG))) return s;
  if (gs->n_local == 0) return BS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case BS_F64: return run_scatter<double>(ctx, gs, xG, xL, st);
    case BS_F32: return run_scatter<float>(ctx, gs, xG, xL, st);
    case BS_BF16: return run_scatter<bf16>(ctx, gs, xG, xL, st);
  }
  return fail(BS_ERR_INVALID_ARG, "bs_gs_scatter: unknown dtype");
}

extern "C" bs_status bs_scatter(bs_ctx* ctx, bs_dtype dtype, int64_t n_local, const int32_t* d_map,
                                int64_t n_global, const void* xG, void* xL, void* stream) {
  const char* op = "bs_scatter";
  bs_status s;
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype))) return s;
  if (n_local < 0 || n_global < 0) return fail(BS_ERR_INVALID_ARG, "%s: negative length", op);
  if (n_local > 0 && !d_map) return fail(BS_ERR_INVALID_ARG, "%s: d_map is NULL", op);
  if (d_map && !aligned_to(d_map, 4)) return fail(BS_ERR_INVALID_ARG, "%s: d_map is not 4-byte aligned", op);
  if ((s = check_vec(op, "xL", xL, n_local, dtype)) || (s = check_vec(op, "xG", xG, n_global, dtype))) return s;
  const uintptr_t a = reinterpret_cast<uintptr_t>(xL), b = reinterpret_cast<uintptr_t>(xG),
                  c = reinterpret_cast<uintptr_t>(d_map);
  const uintptr_t na = static_cast<uintptr_t>(n_local) * dtype_size(dtype);
  const uintptr_t nb = static_cast<uintptr_t>(n_global) * dtype_size(dtype);
  const uintptr_t nc = static_cast<uintptr_t>(n_local) * 4;
  if (na && nb && a < b + nb && b < a + na) return fail(BS_ERR_INVALID_ARG, "%s: xL and xG overlap", op);
  if (na && a < c + nc && c < a + na) return fail(BS_ERR_INVALID_ARG, "%s: xL overlaps the map", op);
  if (n_local == 0) return BS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the plain kernel in local order; its entries per thread and grid cap
  // come from the scatter's tune entry
  const Tune& tn = tune_for(ctx, OP_SCATTER, static_cast<int>(dtype), n_local);
  switch (dtype) {
    case BS_F64: scatter_by_map<double>(tn.unroll, d_map, n_local, n_global, tn.grid_cap, xG, xL, st); break;
    case BS_F32: scatter_by_map<float>(tn.unroll, d_map, n_local, n_global, tn.grid_cap, xG, xL, st); break;
    case BS_BF16: scatter_by_map<uint16_t>(tn.unroll, d_map, n_local, n_global, tn.grid_cap, xG, xL, st); break;
  }
  return check_launch(op);
}
