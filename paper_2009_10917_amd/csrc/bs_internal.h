// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bs.h"

namespace bs {

// Record a failure for bs_last_error() and return its status.
bs_status fail(bs_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Turn the pending HIP error (if any) after a launch into BS_ERR_HIP.
bs_status check_launch(const char* what);
bs_status check_hip(hipError_t e, const char* what);

// Element size in bytes of a storage dtype (0 for an unknown dtype).
inline int dtype_size(bs_dtype d) {
  switch (d) {
    case BS_F64: return 8;
    case BS_F32: return 4;
    case BS_BF16: return 2;
  }
  return 0;
}

inline bool aligned_to(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Checks common to every vector operation: known dtype, n >= 0, non-NULL and
// element-aligned pointers when n > 0, and the caller's device matching the
// context.  Returns BS_OK or the failure status (with the message recorded).
bs_status check_ctx(const bs_ctx* ctx, const char* op);
bs_status check_vec(const char* op, const char* name, const void* p, int64_t n, bs_dtype d);
bs_status check_dtype(const char* op, bs_dtype d);

// Launch-shape knobs of one operation.  `unroll` selects the compiled
// variant (16-byte packets per thread per loop trip: 1, 2, 4 or 8),
// `grid_cap` bounds the number of 256-thread workgroups (the kernels
// grid-stride beyond it) and `variant` picks an alternative kernel where an
// operation has one (gather and scatter).
struct Tune {
  int unroll;
  int grid_cap;
  int variant;
};

enum Op { OP_COPY = 0, OP_AXPY, OP_NORM, OP_DOT, OP_CG_UPDATE, OP_GATHER, OP_SCATTER, OP_BATCH, OP_COUNT };

// Tune entries of one operation and dtype, by length: entry k applies to
// lengths n >= n_min[k] up to the next entry's n_min (n_min[0] == 0,
// ascending).  Gather and scatter use the plan's local length.
constexpr int kTuneEntries = 16;
struct TuneList {
  int count;
  int64_t n_min[kTuneEntries];
  Tune t[kTuneEntries];
};

// Largest number of workgroups a reduction may use: the context's partial
// buffer holds one compensated pair per workgroup.  The CG solver, the
// operator and the batch keep to kMaxReduceBlocks; norm, dot and the CG
// update may use up to kMaxStreamBlocks (one-pass grids of long vectors).
constexpr int kMaxReduceBlocks = 65536;
constexpr int kMaxStreamBlocks = 1 << 21;
constexpr int kBlock = 256;
constexpr int kFinishBlock = 1024;  // threads of the second reduction stage
// Above kFinishDirect pairs the second stage runs in two launches: workgroup
// b adds pairs [b*kFinishChunk, (b+1)*kFinishChunk) into pair b of a second
// area (after the first kMaxStreamBlocks pairs), then one workgroup adds
// those in order.
constexpr int kFinishDirect = 16384;
constexpr int kFinishChunk = 4096;
constexpr int kPartialPairs = kMaxStreamBlocks + kMaxStreamBlocks / kFinishChunk;

}  // namespace bs

struct bs_ctx {
  int device;
  double* partials;  // 2 * kPartialPairs doubles: (sum, compensation) per workgroup, then the chunk sums
  unsigned int* counter;  // single-launch reductions: workgroups that have published their pair (0 between launches)
  bs::TuneList tune[bs::OP_COUNT][3];
};

namespace bs {
// The entry that applies to length n.
inline const Tune& tune_for(const bs_ctx* c, int op, int dt, int64_t n) {
  const TuneList& L = c->tune[op][dt];
  int k = 0;
  for (int j = 1; j < L.count; ++j)
    if (L.n_min[j] <= n) k = j;
  return L.t[k];
}
}  // namespace bs

struct bs_gs {
  int device;
  int64_t n_local;
  int64_t n_global;
  int64_t n_unmasked;
  int64_t max_degree;
  int32_t* map;         // [n_local] copy of the scatter ids
  int32_t* row_starts;  // [n_global + 1] CSR of Z^T (rows in global order)
  int32_t* col_ids;     // [n_unmasked]

  // Gather, rows in global order, nonzero-balanced: block b adds rows
  // [block_starts[b], block_starts[b+1]), whose nonzeros lie in the CSR
  // window [b*chunk, b*chunk + kStage).
  int32_t* block_starts;  // [n_blocks + 1]
  int64_t n_blocks;
  int64_t chunk;

  // Scatter: tiles of kTile consecutive local entries, visited in the order
  // of the smallest global id each references (tile_order[v] is the v-th
  // tile visited); for the v-th tile visited, entry k of tile_gid/tile_loc
  // (at v * kTile + k) is its k-th smallest (global id, local offset) pair,
  // masked entries excluded (tile_count[v] valid pairs): the pairs are
  // stored in visiting order.
  // When every tile's ids span less than 2^23 (tile_packed), the pairs are
  // kept as one word each instead: tile_word = (id - tile_min[t]) << 9 |
  // offset, tile_min[v] the tile's smallest id (visiting order again);
  // tile_gid/tile_loc are then not kept.
  int32_t* tile_order;   // [n_tiles]
  int32_t* tile_gid;     // [n_tiles * kTile]
  uint16_t* tile_loc;    // [n_tiles * kTile]
  bool tile_packed;
  uint32_t* tile_word;   // [n_tiles * kTile]
  int32_t* tile_min;     // [n_tiles]
  int32_t* tile_count;   // [n_tiles]
  int64_t n_tiles;

  // Gather, rows in a permuted order: by default in groups of consecutive
  // tiles of tile_order (each row in the first group holding one of its
  // copies), or in lattice blocks (bs_gs_order_rows), or by element groups
  // (bs_gs_order_elements); perm_rows lists rows with copies first, then rows
  // without copies.  Nonzero-balanced blocks as above: block b adds rows
  // [perm_bstart[b], perm_bstart[b+1]), whose nonzeros are the CSR positions
  // [perm_bnz0[b], perm_bnz0[b+1]) (at most kStage of them, since chunk +
  // max_degree <= kStage).  Each window is stored in ascending column id
  // (so that a block reads its local values in address order), one word per
  // entry: the rank of the column's 512-entry segment among the window's
  // segments (bits 21..31; the segment ids are perm_segs[perm_segoff[b] +
  // rank]), the column mod 512 (bits 12..20), the entry's CSR offset in the
  // window (bits 1..11; rows list their copies in ascending local index) and
  // whether that offset starts a row (bit 0).  The rows of block b, as runs
  // of consecutive global ids: perm_runs[2 i] is the run's first row
  // (offset in the block) and perm_runs[2 i + 1] its first global id, for i
  // in [perm_runoff[b], perm_runoff[b+1]).  Built only when every degree is at most
  // kStage / 2 (has_perm).
  bool has_perm;
  int32_t* perm_rows;    // [n_global]
  uint32_t* perm_words;  // [n_unmasked]
  int32_t* perm_segs;    // [perm_segoff[n_pblocks]]
  int32_t* perm_segoff;  // [n_pblocks + 1]
  int32_t* perm_runoff;  // [n_pblocks + 1]
  int32_t* perm_runs;    // [2 perm_runoff[n_pblocks]]
  int32_t* perm_bstart;  // [n_pblocks + 1]
  int32_t* perm_bnz0;    // [n_pblocks + 1]
  int64_t n_nzrows;
  int64_t n_pblocks;
};

struct bs_elem {
  int device;
  int N;
  double gll_x[16], gll_w[16];  // GLL nodes and weights (N+1 used)
  double gauss_x[16], gauss_w[16];
  double* tables;  // device: the MFMA operand matrices of the local operator (N <= 7)
};

namespace bs {
constexpr int kStage = 2048;  // values staged in LDS per gather workgroup
constexpr int kRunCap = 256;  // row-id runs a gather workgroup takes from LDS (more: it reads the row ids)
constexpr int kTile = 512;    // local entries per scatter workgroup
static_assert(kTile == 2 * kBlock, "scatter tiles hold two entries per thread");
static_assert(kStage == 8 * kBlock, "gather stages eight values per thread");

// Kernel choice for gather and scatter (Tune::variant & kVariantMask), and
// the flags that replace the default workgroup order (each XCD one
// contiguous range of blocks): kNoXcdRemap keeps the hardware's dispatch
// order, kGroupOrder gives each XCD runs of 256 blocks in every group of
// 2048.  At most one of the two may be set.
constexpr int kVariantMask = 3;
constexpr int kNoXcdRemap = 4;
constexpr int kGroupOrder = 8;
constexpr int kCachedAccess = 16;  // cached instead of nontemporal accesses (streaming ops; gather and scatter kernel 0)
// Cached accesses pay while one call's operands fit the last-level cache (256 MB
// of MALL plus 8 x 4 MB of L2); past that they evict what the next call reads and
// run slower than nontemporal ones (a weighted norm over 305 MB: 5.1 against
// 6.5 TB/s), so the variant's + 16 is honoured only up to this many bytes.
constexpr int64_t kCachedBytesMax = int64_t{288} << 20;
inline bool cached_access(int variant, int64_t bytes) {
  return (variant & kCachedAccess) != 0 && bytes <= kCachedBytesMax;
}

// Workgroup order (see dev::block_order) a gather or scatter variant selects.
inline int gs_order(int variant) { return (variant & kNoXcdRemap) ? 0 : (variant & kGroupOrder) ? 1 : 2; }

void free_plan(bs_gs* gs);

// The Helmholtz operator in the form CG uses (bs_elem.hip): yL = A_L Z p,
// Ap = Z^T yL, and in partials the compensated pairs of p . Ap, one per
// workgroup of the local operator (helm_dot_blocks of them: the resident
// workgroups, about 512);
// the local operator returns at once when *done is set.  The caller checks
// the arguments.  Asynchronous on st (on the current device).
int helm_dot_blocks(int64_t n_elem);
bs_status helm_apply_dot(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* geo, double lambda,
                         const double* p, double* yL, double* Ap, double* partials, const int32_t* done,
                         hipStream_t st);
}  // namespace bs
