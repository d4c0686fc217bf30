// Gather/scatter plan: everything BS6 and BS7 need, built once per map on
// the device (Section 5: the mesh set-up that stores Z as an id array and
// Z^T in CSR form without values, plus the blockStarts offsets).
//
//   CSR of Z^T        degree histogram, exclusive scan (row starts), stable
//                     radix sort of (map[l], l) pairs (column ids)
//   gather blocks     rows in global order, split so that every workgroup
//                     takes about the same number of nonzeros
//   scatter tiles     tiles of kTile local entries, visited in order of the
//                     smallest global id each references; inside a tile the
//                     entries sorted by global id (bitonic sort in LDS)
//   gather order      rows in groups of kRowGroupTiles consecutive visited
//                     tiles (each row in the first group holding one of its
//                     copies, ascending global id within a group), as a
//                     permuted CSR with byte degrees
//
// The last two are orderings of work only: no vector is renumbered, and the
// results of gather and scatter are the same bits whichever order is used.

#include <new>
#include <string>
#include <vector>

#include "bs_device.h"
#include "bs_internal.h"
#include "bs_order.h"
#include "bs_prim.h"

namespace bs {
namespace {

inline unsigned int blocks_for(int64_t n) { return static_cast<unsigned int>((n + kBlock - 1) / kBlock); }

constexpr int64_t kOrderLeaf = 16;  // elements per part where the bisection of the element graph stops
// Default gather order: rows keyed by groups of this many consecutive tiles
// of the scatter's visiting order (tiles sorted by their smallest global id),
// rows of a group in ascending global id.
constexpr int32_t kRowGroupTiles = 9;

// Device memory owned until released.
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool alloc(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, bytes ? bytes : 1) == hipSuccess;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
  template <class T>
  T* release() {
    T* q = static_cast<T*>(p);
    p = nullptr;
    return q;
  }
};

// ---------------------------------------------------------------- kernels

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = static_cast<int32_t>(i);
}

// Copy the map, count ids >= n_global, build sort keys (masked entries get
// key n_global, after every row) and the degree histogram.
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
    keys[l] = static_cast<uint32_t>(n_global);
  } else {
    keys[l] = static_cast<uint32_t>(m);
    atomicAdd(&deg[m], 1);
  }
}

// Largest degree and number of rows without copies.
__global__ __launch_bounds__(kBlock) void k_degree_stats(const int32_t* __restrict__ deg, int64_t n,
                                                         int* __restrict__ max_deg, unsigned long long* __restrict__ zeros) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  int d = (i < n) ? deg[i] : 0;
  int z = (i < n && deg[i] == 0) ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) {
    d = max(d, __shfl_xor(d, off, 64));
    z += __shfl_xor(z, off, 64);
  }
  if (threadIdx.x % 64 == 0) {
    atomicMax(max_deg, d);
    if (z) atomicAdd(zeros, static_cast<unsigned long long>(z));
  }
}

// bstart[b] = first index k in [0, n_rows] with starts[k] >= b*chunk
// (b < n_blocks); bstart[n_blocks] = n_rows; optionally bnz0[b] = starts[bstart[b]]
// for b <= n_blocks.
__global__ __launch_bounds__(kBlock) void k_block_starts(const int32_t* __restrict__ starts, int64_t n_rows,
                                                         int64_t chunk, int64_t n_blocks, int32_t* __restrict__ bstart,
                                                         int32_t* __restrict__ bnz0) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (b > n_blocks) return;
  if (b == n_blocks) {
    bstart[b] = static_cast<int32_t>(n_rows);
    if (bnz0) bnz0[b] = starts[n_rows];
    return;
  }
  const int64_t target = b * chunk;
  int64_t lo = 0, hi = n_rows;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (starts[mid] >= target) hi = mid; else lo = mid + 1;
  }
  bstart[b] = static_cast<int32_t>(lo);
  if (bnz0) bnz0[b] = starts[lo];
}

// Per tile: smallest unmasked id (key for the visiting order) and the tile's
// entries sorted by (id, local offset), masked and padding entries last.
//
// Also the packed form: tword[e] = (id - tmin[tile]) << 9 | offset for the
// tile's valid pairs (tmin: its smallest id), with *wide set when a tile's
// ids span 2^23 or more (the packed form then does not apply).
__global__ __launch_bounds__(kBlock) void k_tile_sort(const int32_t* __restrict__ map, int64_t n_local,
                                                      uint32_t* __restrict__ tkey, int32_t* __restrict__ tidx,
                                                      int32_t* __restrict__ tgid, uint16_t* __restrict__ tloc,
                                                      int32_t* __restrict__ tcnt, uint32_t* __restrict__ tword,
                                                      int32_t* __restrict__ tmin, int* __restrict__ wide) {
  static_assert(kTile == 512, "packed tile words hold a 9-bit offset");
  __shared__ uint64_t key[kTile];
  __shared__ int s_cnt;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  for (int k = threadIdx.x; k < kTile; k += kBlock) {
    const int64_t l = base + k;
    const int32_t g = (l < n_local) ? map[l] : -1;
    const uint64_t hi = (g >= 0) ? static_cast<uint64_t>(static_cast<uint32_t>(g)) : 0xFFFFFFFFull;
    key[k] = (hi << 16) | static_cast<uint64_t>(k);
  }
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  // bitonic sorting network over kTile keys (all distinct: the low bits hold k)
  for (int size = 2; size <= kTile; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < kTile; i += kBlock) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const uint64_t a = key[i], b = key[j];
          if ((a > b) == up) {
            key[i] = b;
            key[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  int mine = 0;
  const uint32_t g0 = static_cast<uint32_t>(key[0] >> 16);  // smallest valid id (if any)
  for (int k = threadIdx.x; k < kTile; k += kBlock) {
    const uint64_t v = key[k];
    const uint32_t g = static_cast<uint32_t>(v >> 16);
    const bool valid = g != 0xFFFFFFFFu;
    tgid[base + k] = valid ? static_cast<int32_t>(g) : -1;
    tloc[base + k] = static_cast<uint16_t>(v & 0xFFFFu);
    tword[base + k] = valid ? ((g - g0) << 9) | static_cast<uint32_t>(v & 0x1FFu) : 0u;
    if (valid && g - g0 >= (1u << 23)) atomicOr(wide, 1);
    mine += valid;
  }
  atomicAdd(&s_cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    tcnt[blockIdx.x] = s_cnt;
    tkey[blockIdx.x] = static_cast<uint32_t>(key[0] >> 16);  // 0xFFFFFFFF when the tile has no valid entry
    tidx[blockIdx.x] = static_cast<int32_t>(blockIdx.x);
    tmin[blockIdx.x] = static_cast<int32_t>(g0);
  }
}

// The sorted pairs of the tiles in visiting order: entry v of the outputs
// holds tile order[v] (so that a scatter workgroup reads them by its own
// position, in parallel with order[v]).
__global__ __launch_bounds__(kBlock) void k_tile_permute(const int32_t* __restrict__ order,
                                                         const int32_t* __restrict__ tcnt,
                                                         const int32_t* __restrict__ tmin,
                                                         const uint32_t* __restrict__ tword,
                                                         const int32_t* __restrict__ tgid,
                                                         const uint16_t* __restrict__ tloc, int32_t* __restrict__ vcnt,
                                                         int32_t* __restrict__ vmin, uint32_t* __restrict__ vword,
                                                         int32_t* __restrict__ vgid, uint16_t* __restrict__ vloc) {
  const int64_t v = blockIdx.x;
  const int64_t tile = order[v];
  if (threadIdx.x == 0) {
    vcnt[v] = tcnt[tile];
    if (vmin) vmin[v] = tmin[tile];
  }
  for (int k = threadIdx.x; k < kTile; k += kBlock) {
    if (vword) vword[v * kTile + k] = tword[tile * kTile + k];
    if (vgid) {
      vgid[v * kTile + k] = tgid[tile * kTile + k];
      vloc[v * kTile + k] = tloc[tile * kTile + k];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_invert(const int32_t* __restrict__ order, int64_t n,
                                                   int32_t* __restrict__ rank) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) rank[order[i]] = static_cast<int32_t>(i);
}

// key[g] = smallest group (visiting rank / group) of a tile holding a copy
// of row g.
__global__ __launch_bounds__(kBlock) void k_row_keys(const int32_t* __restrict__ map, int64_t n_local,
                                                     const int32_t* __restrict__ tile_rank, int32_t group,
                                                     uint32_t* __restrict__ key) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= n_local) return;
  const int32_t g = map[l];
  if (g >= 0) atomicMin(&key[g], static_cast<uint32_t>(tile_rank[l / kTile] / group));
}

// key[t] = smallest group of an element overlapping tile t (local entries
// [t kTile, (t + 1) kTile) of n_local).
__global__ __launch_bounds__(kBlock) void k_tile_elem_keys(int64_t n_tiles, int64_t n_local, int64_t P,
                                                           const int32_t* __restrict__ elem_rank, int64_t group,
                                                           uint32_t* __restrict__ key) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= n_tiles) return;
  const int64_t l0 = t * kTile;
  const int64_t l1 = (l0 + kTile < n_local ? l0 + kTile : n_local) - 1;
  uint32_t k = 0xffffffffu;
  for (int64_t e = l0 / P; e <= l1 / P; ++e) k = min(k, static_cast<uint32_t>(elem_rank[e] / group));
  key[t] = k;
}

// key[g] = smallest group (visiting rank / group) of an element holding a
// copy of row g (elements: runs of P consecutive local entries).
__global__ __launch_bounds__(kBlock) void k_elem_row_keys(const int32_t* __restrict__ map, int64_t n_local, int64_t P,
                                                          const int32_t* __restrict__ elem_rank, int64_t group,
                                                          uint32_t* __restrict__ key) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= n_local) return;
  const int32_t g = map[l];
  if (g >= 0) atomicMin(&key[g], static_cast<uint32_t>(elem_rank[l / P] / group));
}

// The 8 corner ids of each element of degree N: corner c is local node
// N * (c & 1, (c >> 1) & 1, c >> 2) (local index i + (N+1)(j + (N+1) k)).
__global__ __launch_bounds__(kBlock) void k_elem_corners(const int32_t* __restrict__ map, int64_t n_elem, int N,
                                                         int32_t* __restrict__ corners) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= n_elem * 8) return;
  const int64_t e = t >> 3;
  const int c = static_cast<int>(t & 7);
  const int64_t P1 = N + 1;
  const int64_t off = N * ((c & 1) + P1 * (((c >> 1) & 1) + P1 * (c >> 2)));
  corners[t] = map[e * P1 * P1 * P1 + off];
}

// Row keys of a lattice-tiled order: global id g is lattice point
// (g mod mx, (g / mx) mod my, g / (mx my)); its key is the index of its
// tile x tile x tile block in lattice order (blocks along x fastest) and,
// within the block, of its bx x by x bz box (nbx x nby x nbz boxes, in the
// same order); rows without copies get the largest key so that they come
// last.
__global__ __launch_bounds__(kBlock) void k_lattice_keys(const int32_t* __restrict__ rs, int64_t n_global, int64_t mx,
                                                         int64_t my, int64_t tile, int64_t ntx, int64_t nty,
                                                         int64_t bx, int64_t by, int64_t bz, int64_t nbx, int64_t nby,
                                                         int64_t nbz, uint32_t* __restrict__ key) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (g >= n_global) return;
  if (rs[g + 1] == rs[g]) {
    key[g] = 0xffffffffu;
    return;
  }
  const int64_t x = g % mx, y = (g / mx) % my, z = g / (mx * my);
  const int64_t t = x / tile + ntx * (y / tile + nty * (z / tile));
  const int64_t b = (x % tile) / bx + nbx * ((y % tile) / by + nby * ((z % tile) / bz));
  key[g] = static_cast<uint32_t>(t * nbx * nby * nbz + b);
}

// Per gather block: the entries of its window [bnz0[b], bnz0[b+1]) (at most
// kStage) in ascending column id, each packed into one word (the layout the
// gather kernel reads):
//   bits 21..31  rank of the column's 512-entry segment among the window's
//                distinct segments (ascending),
//   bits 12..20  column mod 512,
//   bits  1..11  the entry's offset in the window (its CSR position),
//   bit   0      set when that CSR position starts a row.
// Also the sorted column ids (scols, for the segment list) and the number of
// distinct segments (nseg).  A bitonic sort of (column, offset) keys in LDS.
__global__ __launch_bounds__(kBlock) void k_window_pack(const int32_t* __restrict__ cols,
                                                        const int32_t* __restrict__ prs,
                                                        const int32_t* __restrict__ bstart,
                                                        const int32_t* __restrict__ bnz0, int32_t* __restrict__ scols,
                                                        uint32_t* __restrict__ words, int32_t* __restrict__ nseg) {
  static_assert(kStage == 2048 && kStage == 8 * kBlock, "window offsets and segment ranks take 11 bits");
  constexpr int L = kStage / kBlock;
  __shared__ uint64_t key[kStage];
  __shared__ uint8_t first[kStage];
  __shared__ int32_t wsum[kBlock / 64];
  const int64_t a = bnz0[blockIdx.x];
  const int32_t n = static_cast<int32_t>(bnz0[blockIdx.x + 1] - a);
  for (int t = threadIdx.x; t < kStage; t += kBlock) {
    key[t] = (t < n) ? (static_cast<uint64_t>(static_cast<uint32_t>(cols[a + t])) << 16) | static_cast<uint64_t>(t)
                     : ~0ull;
    first[t] = 0;
  }
  __syncthreads();
  for (int32_t r = bstart[blockIdx.x] + threadIdx.x; r < bstart[blockIdx.x + 1]; r += kBlock)
    first[prs[r] - a] = 1;
  for (int k = 2; k <= kStage; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < kStage; t += kBlock) {
        const int p = t ^ j;
        if (p > t) {
          const uint64_t u = key[t], v = key[p];
          if ((u > v) == ((t & k) == 0)) {
            key[t] = v;
            key[p] = u;
          }
        }
      }
      __syncthreads();
    }
  }
  // segment ranks: thread t owns sorted entries t*L .. t*L+L-1
  const int i0 = threadIdx.x * L;
  int32_t prev = (i0 > 0 && i0 - 1 < n) ? static_cast<int32_t>(key[i0 - 1] >> 16) : -1;
  int32_t c[L];
  bool fresh[L];
  int32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    c[i] = (i0 + i < n) ? static_cast<int32_t>(key[i0 + i] >> 16) : -1;
    fresh[i] = (i0 + i < n) && (prev < 0 || (c[i] >> 9) != (prev >> 9));
    prev = c[i];
    cnt += fresh[i];
  }
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  int32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int32_t before = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    before += (i < w) ? wsum[i] : 0;
    total += wsum[i];
  }
  int32_t seen = before + incl - cnt;  // distinct segments before entry i0
#pragma unroll
  for (int i = 0; i < L; ++i) {
    if (i0 + i >= n) break;
    seen += fresh[i];
    const uint32_t off = static_cast<uint32_t>(key[i0 + i] & 0xffffu);
    words[a + i0 + i] = (static_cast<uint32_t>(seen - 1) << 21) | ((static_cast<uint32_t>(c[i]) & 511u) << 12) |
                        (off << 1) | static_cast<uint32_t>(first[off]);
    scols[a + i0 + i] = c[i];
  }
  if (threadIdx.x == 0) nseg[blockIdx.x] = total;
}

// The segment list of each window: segs[segoff[b] + rank] = segment id.
__global__ __launch_bounds__(kBlock) void k_window_segs(const int32_t* __restrict__ scols,
                                                        const uint32_t* __restrict__ words,
                                                        const int32_t* __restrict__ bnz0,
                                                        const int32_t* __restrict__ segoff, int32_t* __restrict__ segs) {
  const int64_t a = bnz0[blockIdx.x];
  const int32_t n = static_cast<int32_t>(bnz0[blockIdx.x + 1] - a);
  for (int32_t i = threadIdx.x; i < n; i += kBlock) {
    const int32_t c = scols[a + i];
    if (i == 0 || (scols[a + i - 1] >> 9) != (c >> 9)) segs[segoff[blockIdx.x] + (words[a + i] >> 21)] = c >> 9;
  }
}

// Runs of consecutive global ids among the rows of each gather block: a row
// starts a run when it is the block's first or its id is not one more than
// the previous row's.  Counting pass (nruns[b]), then, with the offsets
// runoff, the filling pass: runs[2 i] = the run's first row (offset in the
// block), runs[2 i + 1] = its first global id, for i = runoff[b] + rank.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_row_runs(const int32_t* __restrict__ rows,
                                                     const int32_t* __restrict__ bstart, int32_t* __restrict__ nruns,
                                                     const int32_t* __restrict__ runoff, int32_t* __restrict__ runs) {
  constexpr int L = kStage / kBlock;
  __shared__ int32_t wsum[kBlock / 64];
  const int32_t r0 = bstart[blockIdx.x], nrows = bstart[blockIdx.x + 1] - r0;  // <= kStage
  const int i0 = threadIdx.x * L;
  int32_t prev = (i0 > 0 && i0 - 1 < nrows) ? rows[r0 + i0 - 1] : 0;
  int32_t g[L];
  bool st[L];
  int32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int q = i0 + i;
    g[i] = (q < nrows) ? rows[r0 + q] : 0;
    st[i] = (q < nrows) && (q == 0 || g[i] != prev + 1);
    prev = g[i];
    cnt += st[i];
  }
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  int32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int32_t before = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    before += (i < w) ? wsum[i] : 0;
    total += wsum[i];
  }
  if (!FILL) {
    if (threadIdx.x == 0) nruns[blockIdx.x] = total;
    return;
  }
  int64_t idx = runoff[blockIdx.x] + before + incl - cnt;
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (st[i]) {
      runs[2 * idx] = i0 + i;
      runs[2 * idx + 1] = g[i];
      ++idx;
    }
}

// Degrees of the rows in visiting order.
__global__ __launch_bounds__(kBlock) void k_perm_degrees(const int32_t* __restrict__ rows, int64_t n_nzrows,
                                                         const int32_t* __restrict__ rs, int32_t* __restrict__ d32) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (k > n_nzrows) return;
  if (k == n_nzrows) {
    d32[k] = 0;  // so that the exclusive scan's last entry is the total
    return;
  }
  const int32_t g = rows[k];
  d32[k] = rs[g + 1] - rs[g];
}

// Columns of the rows in visiting order.
__global__ __launch_bounds__(kBlock) void k_perm_cols(const int32_t* __restrict__ rows, int64_t n_nzrows,
                                                      const int32_t* __restrict__ rs, const int32_t* __restrict__ ci,
                                                      const int32_t* __restrict__ prs, int32_t* __restrict__ pcols) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= n_nzrows) return;
  const int32_t g = rows[k];
  const int32_t a = rs[g], e = rs[g + 1], o = prs[k];
  for (int32_t j = a; j < e; ++j) pcols[o + (j - a)] = ci[j];
}

__global__ __launch_bounds__(kBlock) void k_degree(const int32_t* __restrict__ rs, int32_t n_global,
                                                   int32_t* __restrict__ deg) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (g < n_global) deg[g] = rs[g + 1] - rs[g];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_weights(const int32_t* __restrict__ map, const int32_t* __restrict__ rs,
                                                    int64_t n_local, typename dev::Storage<T>::E* __restrict__ w) {
  using S = dev::Storage<T>;
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

// ---------------------------------------------------------------- host helpers

struct Builder {
  const char* op;
  hipStream_t st;
  bs_status s = BS_OK;

  bool ok() const { return s == BS_OK; }
  void hip(hipError_t e) {
    if (s == BS_OK && e != hipSuccess) s = check_hip(e, op);
  }
  void launched() {
    if (s == BS_OK) s = check_launch(op);
  }
  void need(DevBuf& b, size_t bytes, const char* what) {
    if (s == BS_OK && !b.alloc(bytes)) s = fail(BS_ERR_ALLOC, "%s: cannot allocate %zu bytes (%s)", op, bytes, what);
  }
  template <class T>
  T read(const T* d) {
    T h{};
    hip(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, st));
    hip(hipStreamSynchronize(st));
    return h;
  }
  // out[i] = in[0] + ... + in[i-1] (the library's own scan)
  void scan(const int32_t* in, int32_t* out, int64_t n) {
    if (ok()) s = scan_exclusive_i32(in, out, n, st, op);
  }
  // stable sort of (key, value) pairs by the low `bits` key bits into
  // k1/v1 (k0/v0 are clobbered)
  void sort(uint32_t* k0, uint32_t* k1, int32_t* v0, int32_t* v1, int64_t n, int bits) {
    if (!ok()) return;
    bool in_alt = false;
    s = sort_pairs_u32(k0, k1, v0, v1, n, bits, st, op, &in_alt);
    if (ok() && !in_alt && n > 0) {  // an even number of passes ended in k0/v0
      hip(hipMemcpyAsync(k1, k0, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
      hip(hipMemcpyAsync(v1, v0, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      hip(hipStreamSynchronize(st));
    }
  }
};

int sort_bits(uint64_t max_key) {
  int bits = 1;
  while (bits < 32 && (static_cast<uint64_t>(1) << bits) <= max_key) ++bits;
  return bits;
}

// CSR of Z^T, degrees; validates the map.
void build_csr(Builder& B, bs_gs* gs, const int32_t* d_map) {
  const int64_t nl = gs->n_local, ng = gs->n_global;
  DevBuf map, rs, keys, keys_out, vals, vals_out, deg, flags;
  B.need(map, nl * 4, "map");
  B.need(rs, (ng + 1) * 4, "row starts");
  B.need(keys, nl * 4, "keys");
  B.need(keys_out, nl * 4, "keys");
  B.need(vals, nl * 4, "values");
  B.need(vals_out, nl * 4, "values");
  B.need(deg, (ng + 1) * 4, "degrees");
  B.need(flags, 64, "flags");
  if (!B.ok()) return;
  B.hip(hipMemsetAsync(flags.p, 0, 64, B.st));
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ng + 1)), dim3(kBlock), 0, B.st, deg.as<int32_t>(), ng + 1, 0);
  if (nl > 0)
    hipLaunchKernelGGL(k_plan_prepare, dim3(blocks_for(nl)), dim3(kBlock), 0, B.st, d_map, nl,
                       static_cast<int32_t>(ng), map.as<int32_t>(), keys.as<uint32_t>(), vals.as<int32_t>(),
                       deg.as<int32_t>(), flags.as<int>());
  B.launched();
  if (B.ok() && B.read(flags.as<int>())) {
    B.s = fail(BS_ERR_INVALID_ARG, "%s: map entry >= n_global (%lld)", B.op, static_cast<long long>(ng));
    return;
  }
  int32_t* dg = deg.as<int32_t>();
  int32_t* rsp = rs.as<int32_t>();
  B.scan(dg, rsp, ng + 1);
  if (nl > 0) {
    const int bits = sort_bits(static_cast<uint64_t>(ng));
    uint32_t* k0 = keys.as<uint32_t>();
    uint32_t* k1 = keys_out.as<uint32_t>();
    int32_t* v0 = vals.as<int32_t>();
    int32_t* v1 = vals_out.as<int32_t>();
    B.sort(k0, k1, v0, v1, nl, bits);
  }
  if (!B.ok()) return;
  gs->n_unmasked = B.read(rsp + ng);
  // degree statistics
  B.hip(hipMemsetAsync(flags.p, 0, 64, B.st));
  if (ng > 0)
    hipLaunchKernelGGL(k_degree_stats, dim3(blocks_for(ng)), dim3(kBlock), 0, B.st, dg, ng, flags.as<int>(),
                       reinterpret_cast<unsigned long long*>(flags.as<char>() + 8));
  B.launched();
  if (!B.ok()) return;
  gs->max_degree = B.read(flags.as<int>());
  DevBuf ci;
  B.need(ci, gs->n_unmasked * 4, "column ids");
  if (gs->n_unmasked > 0)
    B.hip(hipMemcpyAsync(ci.p, vals_out.p, gs->n_unmasked * 4, hipMemcpyDeviceToDevice, B.st));
  B.hip(hipStreamSynchronize(B.st));
  if (!B.ok()) return;
  gs->map = map.release<int32_t>();
  gs->row_starts = rs.release<int32_t>();
  gs->col_ids = ci.release<int32_t>();
}

// Rows in global order, nonzero-balanced blocks.
void build_gather_blocks(Builder& B, bs_gs* gs) {
  gs->chunk = (gs->max_degree <= kStage / 2) ? kStage - gs->max_degree : kStage / 2;
  gs->n_blocks = (gs->n_unmasked + gs->chunk - 1) / gs->chunk;
  if (gs->n_blocks < 1) gs->n_blocks = 1;
  DevBuf bstart;
  B.need(bstart, (gs->n_blocks + 1) * 4, "block starts");
  if (!B.ok()) return;
  hipLaunchKernelGGL(k_block_starts, dim3(blocks_for(gs->n_blocks + 1)), dim3(kBlock), 0, B.st, gs->row_starts,
                     gs->n_global, gs->chunk, gs->n_blocks, bstart.as<int32_t>(), static_cast<int32_t*>(nullptr));
  B.launched();
  B.hip(hipStreamSynchronize(B.st));
  if (B.ok()) gs->block_starts = bstart.release<int32_t>();
}

// Element visiting ranks for a gather or scatter order (elements: runs of P
// local entries).
struct ElementOrder {
  const int32_t* rank;  // device, [n_local / P]
  int64_t P;
  int64_t group;  // elements of consecutive ranks visited as one group
};

// Sorted tiles and their visiting order: by the smallest global id of each
// tile, or (eo) by the smallest rank of an element the tile overlaps.
void build_scatter_tiles(Builder& B, bs_gs* gs, const ElementOrder* eo = nullptr) {
  const int64_t nt = (gs->n_local + kTile - 1) / kTile;
  gs->n_tiles = nt;
  DevBuf tgid, tloc, tcnt, order, tkey, tkey_out, tidx, tword, tmin, wide, vcnt, vmin, vword, vgid, vloc;
  B.need(tgid, nt * kTile * 4, "tile ids");
  B.need(tloc, nt * kTile * 2, "tile offsets");
  B.need(tword, nt * kTile * 4, "tile words");
  B.need(tmin, nt * 4, "tile minima");
  B.need(wide, 64, "flag");
  B.need(tcnt, nt * 4, "tile counts");
  B.need(order, nt * 4, "tile order");
  B.need(tkey, nt * 4, "tile keys");
  B.need(tkey_out, nt * 4, "tile keys");
  B.need(tidx, nt * 4, "tile indices");
  if (!B.ok()) return;
  B.hip(hipMemsetAsync(wide.p, 0, 64, B.st));
  if (nt > 0) {
    hipLaunchKernelGGL(k_tile_sort, dim3(static_cast<unsigned int>(nt)), dim3(kBlock), 0, B.st, gs->map, gs->n_local,
                       tkey.as<uint32_t>(), tidx.as<int32_t>(), tgid.as<int32_t>(), tloc.as<uint16_t>(),
                       tcnt.as<int32_t>(), tword.as<uint32_t>(), tmin.as<int32_t>(), wide.as<int>());
    if (eo)
      hipLaunchKernelGGL(k_tile_elem_keys, dim3(blocks_for(nt)), dim3(kBlock), 0, B.st, nt, gs->n_local, eo->P,
                         eo->rank, eo->group, tkey.as<uint32_t>());
    B.launched();
    uint32_t* k0 = tkey.as<uint32_t>();
    uint32_t* k1 = tkey_out.as<uint32_t>();
    int32_t* v0 = tidx.as<int32_t>();
    int32_t* v1 = order.as<int32_t>();
    B.sort(k0, k1, v0, v1, nt, 32);
  }
  B.hip(hipStreamSynchronize(B.st));
  if (!B.ok()) return;
  gs->tile_packed = B.read(wide.as<int>()) == 0;
  // the kept form of the pairs, in visiting order
  B.need(vcnt, nt * 4, "tile counts");
  if (gs->tile_packed) {  // one word per pair
    B.need(vmin, nt * 4, "tile minima");
    B.need(vword, nt * kTile * 4, "tile words");
  } else {
    B.need(vgid, nt * kTile * 4, "tile ids");
    B.need(vloc, nt * kTile * 2, "tile offsets");
  }
  if (!B.ok()) return;
  if (nt > 0)
    hipLaunchKernelGGL(k_tile_permute, dim3(static_cast<unsigned int>(nt)), dim3(kBlock), 0, B.st,
                       order.as<int32_t>(), tcnt.as<int32_t>(), tmin.as<int32_t>(), tword.as<uint32_t>(),
                       tgid.as<int32_t>(), tloc.as<uint16_t>(), vcnt.as<int32_t>(), vmin.as<int32_t>(),
                       vword.as<uint32_t>(), vgid.as<int32_t>(), vloc.as<uint16_t>());
  B.launched();
  B.hip(hipStreamSynchronize(B.st));
  if (!B.ok()) return;
  if (gs->tile_packed) {
    gs->tile_word = vword.release<uint32_t>();
    gs->tile_min = vmin.release<int32_t>();
  } else {
    gs->tile_gid = vgid.release<int32_t>();
    gs->tile_loc = vloc.release<uint16_t>();
  }
  gs->tile_count = vcnt.release<int32_t>();
  gs->tile_order = order.release<int32_t>();
}

// Rows in visiting order (needs the tile order and the CSR).
// Lattice description for a tiled gather order (global ids are lattice points).
struct LatticeOrder {
  int64_t mx, my, mz, tile, bx, by, bz;  // box sides inside a tile (tile: none)
};

// Rows with copies in a permuted order and the CSR in that order: by default
// the visiting order of the scatter tiles, or (lat) lattice tiles, or (eo)
// the first visited element holding a copy.
void build_gather_order(Builder& B, bs_gs* gs, int64_t n_zero_rows, const LatticeOrder* lat = nullptr,
                        const ElementOrder* eo = nullptr) {
  gs->has_perm = false;
  // a window (chunk + max_degree - 1 entries) must fit the stage, whose offsets take 11 bits
  if (gs->max_degree > kStage / 2) return;
  const int64_t nl = gs->n_local, ng = gs->n_global, nt = gs->n_tiles;
  const int64_t nz = ng - n_zero_rows;  // rows with copies
  DevBuf rank, rkey, rkey_out, rows0, rows, d32, prs, pcols, scols, words, nseg, segoff, segs, bstart, bnz0;
  DevBuf nruns, runoff, runs;
  B.need(rank, nt * 4, "tile ranks");
  B.need(rkey, ng * 4, "row keys");
  B.need(rkey_out, ng * 4, "row keys");
  B.need(rows0, ng * 4, "rows");
  B.need(rows, ng * 4, "row order");
  B.need(d32, (nz + 1) * 4, "degrees");
  B.need(prs, (nz + 1) * 4, "row starts");
  B.need(pcols, gs->n_unmasked * 4, "columns");
  if (!B.ok()) return;
  if (ng > 0) hipLaunchKernelGGL(k_iota, dim3(blocks_for(ng)), dim3(kBlock), 0, B.st, rows0.as<int32_t>(), ng);
  if (eo) {
    if (ng > 0)
      hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ng)), dim3(kBlock), 0, B.st, rkey.as<int32_t>(), ng, -1);
    if (nl > 0)
      hipLaunchKernelGGL(k_elem_row_keys, dim3(blocks_for(nl)), dim3(kBlock), 0, B.st, gs->map, nl, eo->P, eo->rank,
                         eo->group, rkey.as<uint32_t>());
  } else if (lat) {
    const int64_t ntx = (lat->mx + lat->tile - 1) / lat->tile, nty = (lat->my + lat->tile - 1) / lat->tile;
    const int64_t nbx = (lat->tile + lat->bx - 1) / lat->bx, nby = (lat->tile + lat->by - 1) / lat->by,
                  nbz = (lat->tile + lat->bz - 1) / lat->bz;
    if (ng > 0)
      hipLaunchKernelGGL(k_lattice_keys, dim3(blocks_for(ng)), dim3(kBlock), 0, B.st, gs->row_starts, ng, lat->mx,
                         lat->my, lat->tile, ntx, nty, lat->bx, lat->by, lat->bz, nbx, nby, nbz, rkey.as<uint32_t>());
  } else {
    if (nt > 0)
      hipLaunchKernelGGL(k_invert, dim3(blocks_for(nt)), dim3(kBlock), 0, B.st, gs->tile_order, nt, rank.as<int32_t>());
    if (ng > 0)
      hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ng)), dim3(kBlock), 0, B.st, rkey.as<int32_t>(), ng, -1);
    if (nl > 0)
      hipLaunchKernelGGL(k_row_keys, dim3(blocks_for(nl)), dim3(kBlock), 0, B.st, gs->map, nl, rank.as<int32_t>(),
                         kRowGroupTiles, rkey.as<uint32_t>());
  }
  B.launched();
  if (ng > 0) {
    uint32_t* k0 = rkey.as<uint32_t>();
    uint32_t* k1 = rkey_out.as<uint32_t>();
    int32_t* v0 = rows0.as<int32_t>();
    int32_t* v1 = rows.as<int32_t>();
    B.sort(k0, k1, v0, v1, ng, 32);
  }
  hipLaunchKernelGGL(k_perm_degrees, dim3(blocks_for(nz + 1)), dim3(kBlock), 0, B.st, rows.as<int32_t>(), nz,
                     gs->row_starts, d32.as<int32_t>());
  B.launched();
  int32_t* dp = d32.as<int32_t>();
  int32_t* pp = prs.as<int32_t>();
  B.scan(dp, pp, nz + 1);
  if (nz > 0)
    hipLaunchKernelGGL(k_perm_cols, dim3(blocks_for(nz)), dim3(kBlock), 0, B.st, rows.as<int32_t>(), nz,
                       gs->row_starts, gs->col_ids, prs.as<int32_t>(), pcols.as<int32_t>());
  B.launched();
  const int64_t nb = (gs->n_unmasked + gs->chunk - 1) / gs->chunk;
  B.need(bstart, (nb + 1) * 4, "block starts");
  B.need(bnz0, (nb + 1) * 4, "block offsets");
  B.need(scols, gs->n_unmasked * 4, "sorted columns");
  B.need(words, gs->n_unmasked * 4, "window words");
  B.need(nseg, (nb + 1) * 4, "segment counts");
  B.need(segoff, (nb + 1) * 4, "segment offsets");
  if (!B.ok()) return;
  hipLaunchKernelGGL(k_block_starts, dim3(blocks_for(nb + 1)), dim3(kBlock), 0, B.st, prs.as<int32_t>(), nz, gs->chunk,
                     nb, bstart.as<int32_t>(), bnz0.as<int32_t>());
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nb + 1)), dim3(kBlock), 0, B.st, nseg.as<int32_t>(), nb + 1, 0);
  if (nb > 0)
    hipLaunchKernelGGL(k_window_pack, dim3(static_cast<unsigned int>(nb)), dim3(kBlock), 0, B.st, pcols.as<int32_t>(),
                       prs.as<int32_t>(), bstart.as<int32_t>(), bnz0.as<int32_t>(), scols.as<int32_t>(),
                       words.as<uint32_t>(), nseg.as<int32_t>());
  B.launched();
  int32_t* ns = nseg.as<int32_t>();
  int32_t* so = segoff.as<int32_t>();
  B.scan(ns, so, nb + 1);
  const int64_t total_segs = B.ok() ? static_cast<int64_t>(B.read(so + nb)) : 0;
  B.need(segs, (total_segs > 0 ? total_segs : 1) * 4, "window segments");
  if (!B.ok()) return;
  if (nb > 0)
    hipLaunchKernelGGL(k_window_segs, dim3(static_cast<unsigned int>(nb)), dim3(kBlock), 0, B.st, scols.as<int32_t>(),
                       words.as<uint32_t>(), bnz0.as<int32_t>(), so, segs.as<int32_t>());
  B.launched();
  // runs of consecutive row ids per block
  B.need(nruns, (nb + 1) * 4, "run counts");
  B.need(runoff, (nb + 1) * 4, "run offsets");
  if (!B.ok()) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nb + 1)), dim3(kBlock), 0, B.st, nruns.as<int32_t>(), nb + 1, 0);
  if (nb > 0)
    hipLaunchKernelGGL(k_row_runs<false>, dim3(static_cast<unsigned int>(nb)), dim3(kBlock), 0, B.st,
                       rows.as<int32_t>(), bstart.as<int32_t>(), nruns.as<int32_t>(), static_cast<const int32_t*>(nullptr),
                       static_cast<int32_t*>(nullptr));
  B.launched();
  int32_t* nr = nruns.as<int32_t>();
  int32_t* ro = runoff.as<int32_t>();
  B.scan(nr, ro, nb + 1);
  const int64_t total_runs = B.ok() ? static_cast<int64_t>(B.read(ro + nb)) : 0;
  B.need(runs, (total_runs > 0 ? total_runs : 1) * 8, "row runs");
  if (!B.ok()) return;
  if (nb > 0)
    hipLaunchKernelGGL(k_row_runs<true>, dim3(static_cast<unsigned int>(nb)), dim3(kBlock), 0, B.st, rows.as<int32_t>(),
                       bstart.as<int32_t>(), static_cast<int32_t*>(nullptr), ro, runs.as<int32_t>());
  B.launched();
  B.hip(hipStreamSynchronize(B.st));
  if (!B.ok()) return;
  gs->perm_rows = rows.release<int32_t>();
  gs->perm_runoff = runoff.release<int32_t>();
  gs->perm_runs = runs.release<int32_t>();
  gs->perm_words = words.release<uint32_t>();
  gs->perm_segs = segs.release<int32_t>();
  gs->perm_segoff = segoff.release<int32_t>();
  gs->perm_bstart = bstart.release<int32_t>();
  gs->perm_bnz0 = bnz0.release<int32_t>();
  gs->n_nzrows = nz;
  gs->n_pblocks = nb;
  gs->has_perm = true;
}

}  // namespace

void free_plan(bs_gs* gs) {
  if (!gs) return;
  for (void* p : {static_cast<void*>(gs->map), static_cast<void*>(gs->row_starts), static_cast<void*>(gs->col_ids),
                  static_cast<void*>(gs->block_starts), static_cast<void*>(gs->tile_order),
                  static_cast<void*>(gs->tile_gid), static_cast<void*>(gs->tile_loc),
                  static_cast<void*>(gs->tile_word), static_cast<void*>(gs->tile_min),
                  static_cast<void*>(gs->tile_count), static_cast<void*>(gs->perm_rows),
                  static_cast<void*>(gs->perm_words), static_cast<void*>(gs->perm_segs),
                  static_cast<void*>(gs->perm_segoff), static_cast<void*>(gs->perm_runoff),
                  static_cast<void*>(gs->perm_runs),
                  static_cast<void*>(gs->perm_bstart), static_cast<void*>(gs->perm_bnz0)})
    if (p) (void)hipFree(p);
  delete gs;
}

}  // namespace bs

using namespace bs;

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
  bs_gs* gs = new bs_gs();
  gs->device = ctx->device;
  gs->n_local = n_local;
  gs->n_global = n_global;
  Builder B{op, static_cast<hipStream_t>(stream)};
  build_csr(B, gs, d_map);
  // rows without copies, for the gather order
  int64_t zero_rows = 0;
  if (B.ok()) {
    DevBuf deg, cnt;
    B.need(deg, n_global * 4, "degrees");
    B.need(cnt, 64, "counter");
    if (B.ok()) {
      B.hip(hipMemsetAsync(cnt.p, 0, 64, B.st));
      if (n_global > 0) {
        hipLaunchKernelGGL(k_degree, dim3(blocks_for(n_global)), dim3(kBlock), 0, B.st, gs->row_starts,
                           static_cast<int32_t>(n_global), deg.as<int32_t>());
        hipLaunchKernelGGL(k_degree_stats, dim3(blocks_for(n_global)), dim3(kBlock), 0, B.st, deg.as<int32_t>(),
                           n_global, cnt.as<int>(), reinterpret_cast<unsigned long long*>(cnt.as<char>() + 8));
      }
      B.launched();
      if (B.ok()) zero_rows = static_cast<int64_t>(B.read(reinterpret_cast<unsigned long long*>(cnt.as<char>() + 8)));
    }
  }
  if (B.ok()) build_gather_blocks(B, gs);
  if (B.ok()) build_scatter_tiles(B, gs);
  if (B.ok()) build_gather_order(B, gs, zero_rows);
  if (!B.ok()) {
    free_plan(gs);
    return B.s;
  }
  *out = gs;
  return BS_OK;
}

extern "C" bs_status bs_gs_order_rows(bs_gs* gs, int64_t mx, int64_t my, int64_t mz, int32_t tile, int32_t bx,
                                      int32_t by, int32_t bz, void* stream) {
  const char* op = "bs_gs_order_rows";
  if (!gs) return fail(BS_ERR_INVALID_ARG, "%s: plan is NULL", op);
  if (mx < 1 || my < 1 || mz < 1 || tile < 1 || mx * my * mz != gs->n_global)
    return fail(BS_ERR_INVALID_ARG, "%s: need mx*my*mz == n_global and tile >= 1", op);
  if (bx < 0 || by < 0 || bz < 0) return fail(BS_ERR_INVALID_ARG, "%s: box sides must be >= 0", op);
  if (bx == 0 || bx > tile) bx = tile;
  if (by == 0 || by > tile) by = tile;
  if (bz == 0 || bz > tile) bz = tile;
  // boxes per tile, then tiles, as 32-bit keys (each factor < 2^31; checked before every product)
  const int64_t t64 = tile;
  const int64_t fxy = ((t64 + bx - 1) / bx) * ((t64 + by - 1) / by);
  const int64_t nb = (fxy < 0xffffffffLL) ? fxy * ((t64 + bz - 1) / bz) : 0xffffffffLL;
  const int64_t ntiles = ((mx + tile - 1) / tile) * ((my + tile - 1) / tile) * ((mz + tile - 1) / tile);
  if (nb >= 0xffffffffLL || ntiles >= 0xffffffffLL / nb) return fail(BS_ERR_INVALID_ARG, "%s: too many tiles", op);
  if (!gs->has_perm) return fail(BS_ERR_UNSUPPORTED, "%s: the plan has no permuted order (a degree exceeds 1024)", op);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(gs->device);
  int32_t* old_rows = gs->perm_rows;
  uint32_t* old_words = gs->perm_words;
  int32_t* old_segs = gs->perm_segs;
  int32_t* old_segoff = gs->perm_segoff;
  int32_t* old_runoff = gs->perm_runoff;
  int32_t* old_runs = gs->perm_runs;
  int32_t* old_bstart = gs->perm_bstart;
  int32_t* old_bnz0 = gs->perm_bnz0;
  const int64_t zero_rows = gs->n_global - gs->n_nzrows;
  Builder B{op, static_cast<hipStream_t>(stream)};
  const LatticeOrder lat{mx, my, mz, tile, bx, by, bz};
  build_gather_order(B, gs, zero_rows, &lat);
  if (B.ok()) {
    for (void* q : {static_cast<void*>(old_rows), static_cast<void*>(old_words), static_cast<void*>(old_segs),
                    static_cast<void*>(old_segoff), static_cast<void*>(old_runoff), static_cast<void*>(old_runs),
                    static_cast<void*>(old_bstart), static_cast<void*>(old_bnz0)})
      (void)hipFree(q);
  } else {
    gs->has_perm = true;  // the previous order is still in place
  }
  (void)hipSetDevice(prev);
  return B.s;
}

extern "C" bs_status bs_gs_order_elements(bs_gs* gs, int64_t nodes_per_element, const int32_t* d_elem_rank,
                                          int64_t elements_per_group, void* stream) {
  const char* op = "bs_gs_order_elements";
  if (!gs) return fail(BS_ERR_INVALID_ARG, "%s: plan is NULL", op);
  const int64_t P = nodes_per_element;
  if (P < 1 || gs->n_local % P != 0)
    return fail(BS_ERR_INVALID_ARG, "%s: n_local must be a multiple of nodes_per_element >= 1", op);
  if (elements_per_group < 1 || elements_per_group > 2147483647LL)
    return fail(BS_ERR_INVALID_ARG, "%s: elements_per_group must lie in [1, 2^31)", op);
  if (d_elem_rank && !aligned_to(d_elem_rank, 4))
    return fail(BS_ERR_INVALID_ARG, "%s: d_elem_rank is not 4-byte aligned", op);
  int N = 0;
  if (!d_elem_rank) {
    while (static_cast<int64_t>(N + 1) * (N + 1) * (N + 1) < P) ++N;
    if (static_cast<int64_t>(N + 1) * (N + 1) * (N + 1) != P || N < 1)
      return fail(BS_ERR_INVALID_ARG, "%s: nodes_per_element must be (N+1)^3 with N >= 1 to derive an order", op);
  }
  if (!gs->has_perm) return fail(BS_ERR_UNSUPPORTED, "%s: the plan has no permuted order (a degree exceeds 1024)", op);
  const int64_t n_elem = gs->n_local / P;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(gs->device);
  Builder B{op, static_cast<hipStream_t>(stream)};
  DevBuf rank_buf;
  const int32_t* rank = d_elem_rank;
  if (!d_elem_rank) {
    // corners to the host, the bisection order, ranks back to the device
    DevBuf cbuf;
    B.need(cbuf, static_cast<size_t>(n_elem) * 8 * 4, "element corners");
    B.need(rank_buf, static_cast<size_t>(n_elem) * 4, "element ranks");
    std::vector<int32_t> corners, hrank;
    std::string err;
    if (B.ok() && n_elem > 0) {
      hipLaunchKernelGGL(k_elem_corners, dim3(blocks_for(n_elem * 8)), dim3(kBlock), 0, B.st, gs->map, n_elem, N,
                         cbuf.as<int32_t>());
      B.launched();
      try {
        corners.resize(static_cast<size_t>(n_elem) * 8);
      } catch (const std::bad_alloc&) {
        B.s = fail(BS_ERR_ALLOC, "%s: cannot allocate %lld host corner ids", op, static_cast<long long>(n_elem * 8));
      }
      B.hip(hipMemcpyAsync(corners.data(), cbuf.p, corners.size() * 4, hipMemcpyDeviceToHost, B.st));
      B.hip(hipStreamSynchronize(B.st));
      if (B.ok() && !element_order_bisection(corners.data(), n_elem, kOrderLeaf, hrank, err))
        B.s = fail(BS_ERR_ALLOC, "%s: %s", op, err.c_str());
      B.hip(hipMemcpyAsync(rank_buf.p, hrank.data(), hrank.size() * 4, hipMemcpyHostToDevice, B.st));
      B.hip(hipStreamSynchronize(B.st));
    }
    rank = rank_buf.as<int32_t>();
  }
  if (!B.ok()) {
    (void)hipSetDevice(prev);
    return B.s;
  }
  int32_t* old_rows = gs->perm_rows;
  uint32_t* old_words = gs->perm_words;
  int32_t* old_segs = gs->perm_segs;
  int32_t* old_segoff = gs->perm_segoff;
  int32_t* old_runoff = gs->perm_runoff;
  int32_t* old_runs = gs->perm_runs;
  int32_t* old_bstart = gs->perm_bstart;
  int32_t* old_bnz0 = gs->perm_bnz0;
  const int64_t zero_rows = gs->n_global - gs->n_nzrows;
  const ElementOrder eo{rank, P, elements_per_group};
  build_gather_order(B, gs, zero_rows, nullptr, &eo);
  if (B.ok()) {
    for (void* q : {static_cast<void*>(old_rows), static_cast<void*>(old_words), static_cast<void*>(old_segs),
                    static_cast<void*>(old_segoff), static_cast<void*>(old_runoff), static_cast<void*>(old_runs),
                    static_cast<void*>(old_bstart), static_cast<void*>(old_bnz0)})
      (void)hipFree(q);
  } else {
    gs->has_perm = true;  // the previous order is still in place
    (void)hipSetDevice(prev);
    return B.s;
  }
  // the scatter's tiles in the same element order
  bs_gs old = *gs;
  gs->tile_order = gs->tile_gid = gs->tile_min = gs->tile_count = nullptr;
  gs->tile_loc = nullptr;
  gs->tile_word = nullptr;
  build_scatter_tiles(B, gs, &eo);
  if (B.ok()) {
    for (void* q : {static_cast<void*>(old.tile_order), static_cast<void*>(old.tile_gid),
                    static_cast<void*>(old.tile_loc), static_cast<void*>(old.tile_word),
                    static_cast<void*>(old.tile_min), static_cast<void*>(old.tile_count)})
      (void)hipFree(q);
  } else {
    gs->tile_order = old.tile_order;
    gs->tile_gid = old.tile_gid;
    gs->tile_loc = old.tile_loc;
    gs->tile_word = old.tile_word;
    gs->tile_min = old.tile_min;
    gs->tile_count = old.tile_count;
    gs->tile_packed = old.tile_packed;
  }
  (void)hipSetDevice(prev);
  return B.s;
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
  if (!d_row_starts || (gs->n_unmasked > 0 && !d_col_ids)) return fail(BS_ERR_INVALID_ARG, "bs_gs_csr: output is NULL");
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
      hipLaunchKernelGGL(k_weights<dev::bf16>, g, dim3(kBlock), 0, st, gs->map, gs->row_starts, gs->n_local,
                         static_cast<uint16_t*>(d_wL));
      break;
  }
  return check_launch("bs_gs_weights");
}
