// BS1-BS5: copy, AXPY, norm, inner product and the fused CG update
// (Table 1; Listings 1-3; Algorithm 1 steps 8-10).
//
// All five stream their operands once through 16-byte packets (dwordx4
// loads and stores).  A workgroup of 256 threads handles U packets per
// thread per trip and the grid strides over the vector beyond `grid_cap`
// workgroups, numbered in the dispatch order or grouped per XCD (the tune
// variant).  Scalar elements that precede the first 16-byte boundary or
// follow the last full packet are handled by workgroup 0.  When the operands
// are not mutually 16-byte aligned the same kernels run with one-element
// packets.
//
// The reductions accumulate per thread in compensated form (sum plus
// running error), combine the 64 lanes of a wave by xor-shuffles and the
// waves of a workgroup through LDS, and store one pair per workgroup; a
// second launch of one 1024-thread workgroup adds the pairs in index order,
// as the paper's two-kernel reductions do (Section 5).  Grids of more than
// 16384 workgroups (one-pass grids over long vectors) first add their pairs
// in chunks of 4096, one workgroup per chunk, in one more launch.  Finishing inside the
// first launch would need an agent-scope fence per workgroup, which on this
// 8-XCD part costs more than the second launch.

#include <mutex>
#include <type_traits>

#include "bs_stream_ops.h"

namespace bs {
namespace {

using namespace ops;

template <class T, int V, int U, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_copy(const typename Storage<T>::E* __restrict__ x,
                                                 typename Storage<T>::E* __restrict__ y, Span sp) {
  CopyOp<T, V, NT> op{{}, x, y, sp.head};
  stream_loop<U, NB>(op, sp);
}

// ---------------------------------------------------------------- BS2 AXPY


template <class T, int V, int U, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_axpy(typename Storage<T>::C alpha, const typename Storage<T>::E* __restrict__ x,
                                                 typename Storage<T>::C beta, typename Storage<T>::E* __restrict__ y,
                                                 Span sp) {
  AxpyOp<T, V, NT> op{{}, alpha, beta, x, y, sp.head};
  stream_loop<U, NB>(op, sp);
}

// ---------------------------------------------------------------- BS3 norm


template <class T, int V, int U, bool W, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_norm(const typename Storage<T>::E* __restrict__ x,
                                                 const typename Storage<T>::E* __restrict__ w, Span sp,
                                                 double* partials, double* out, unsigned int* counter) {
  using C = typename Storage<T>::C;
  NormOp<T, V, W, NT> op{{}, x, w, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U, NB>(op, sp);
  dev::block_finish<NB>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, counter, out);
}

// ---------------------------------------------------------------- BS4 inner product


template <class T, int V, int U, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_dot(const typename Storage<T>::E* __restrict__ x,
                                                const typename Storage<T>::E* __restrict__ y, Span sp,
                                                double* partials, double* out, unsigned int* counter) {
  using C = typename Storage<T>::C;
  DotOp<T, V, NT> op{{}, x, y, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U, NB>(op, sp);
  dev::block_finish<NB>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, counter, out);
}

// ---------------------------------------------------------------- BS5 fused CG update


template <class T, int V, int U, bool W, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_cg_update(typename Storage<T>::C alpha, typename Storage<T>::E* __restrict__ x,
                                                      const typename Storage<T>::E* __restrict__ p,
                                                      typename Storage<T>::E* __restrict__ r,
                                                      const typename Storage<T>::E* __restrict__ Ap,
                                                      const typename Storage<T>::E* __restrict__ w, Span sp,
                                                      double* partials, double* out, unsigned int* counter) {
  using C = typename Storage<T>::C;
  CgOp<T, V, W, NT> op{{}, alpha, x, p, r, Ap, w, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U, NB>(op, sp);
  dev::block_finish<NB>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, counter, out);
}

// ---------------------------------------------------------------- device scalars

// Scalar of the device-scalar forms: h * (num / den) in binary64, a NULL
// pointer reading as 1.0 (so with both NULL the host value h alone).  Every
// thread reads the two doubles when the kernel starts; they were written by
// an earlier kernel on the stream.
struct DevScalar {
  double h;
  const double* num;
  const double* den;
};

__device__ __forceinline__ double dev_scalar(const DevScalar& s) {
  double q = s.num ? *s.num : 1.0;
  if (s.den) q = q / *s.den;
  return s.h * q;
}

template <class T, int V, int U, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_axpy_dev(DevScalar a, const typename Storage<T>::E* __restrict__ x,
                                                     DevScalar b, typename Storage<T>::E* __restrict__ y, Span sp) {
  using C = typename Storage<T>::C;
  AxpyOp<T, V, NT> op{{}, static_cast<C>(dev_scalar(a)), static_cast<C>(dev_scalar(b)), x, y, sp.head};
  stream_loop<U, NB>(op, sp);
}

template <class T, int V, int U, bool W, int NB, bool NT>
__global__ __launch_bounds__(NB) void k_cg_update_dev(DevScalar a, typename Storage<T>::E* __restrict__ x,
                                                          const typename Storage<T>::E* __restrict__ p,
                                                          typename Storage<T>::E* __restrict__ r,
                                                          const typename Storage<T>::E* __restrict__ Ap,
                                                          const typename Storage<T>::E* __restrict__ w, Span sp,
                                                          double* partials, double* out, unsigned int* counter) {
  using C = typename Storage<T>::C;
  CgOp<T, V, W, NT> op{{}, static_cast<C>(dev_scalar(a)), x, p, r, Ap, w, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U, NB>(op, sp);
  dev::block_finish<NB>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, counter, out);
}

// ---------------------------------------------------------------- host side


// Second stage of every reduction: one workgroup adds the G per-workgroup
// pairs, thread t taking pairs t, t + 1024, ... in order.
__global__ __launch_bounds__(kFinishBlock) void k_finish(const double* __restrict__ partials, int G,
                                                          double* __restrict__ out) {
  DW<double> r{0.0, 0.0};
  for (int i = threadIdx.x; i < G; i += kFinishBlock) r = dev::dw_add(r, DW<double>{partials[2 * i], partials[2 * i + 1]});
  r = dev::block_reduce<kFinishBlock>(r);
  if (threadIdx.x == 0) *out = r.s + r.c;
}

// First half of a two-launch second stage (more than kFinishDirect pairs):
// workgroup b adds pairs [b*kFinishChunk, min((b+1)*kFinishChunk, G)) the
// same way and stores the compensated pair in sums[b].
__global__ __launch_bounds__(kFinishBlock) void k_finish_chunks(const double* __restrict__ partials, int G,
                                                                double* __restrict__ sums) {
  const int b0 = blockIdx.x * kFinishChunk;
  const int b1 = min(b0 + kFinishChunk, G);
  DW<double> r{0.0, 0.0};
  for (int i = b0 + threadIdx.x; i < b1; i += kFinishBlock)
    r = dev::dw_add(r, DW<double>{partials[2 * i], partials[2 * i + 1]});
  r = dev::block_reduce<kFinishBlock>(r);
  if (threadIdx.x == 0) {
    sums[2 * blockIdx.x] = r.s;
    sums[2 * blockIdx.x + 1] = r.c;
  }
}

// Up to this many workgroups a reduction finishes in its own launch (the
// last workgroup adds the pairs, dev::block_finish).  Each workgroup's
// release is a write-back of its XCD's L2 (gfx950's L2s are not coherent
// with one another), which beyond about a hundred workgroups costs more
// than the second launch it saves (measured: norm at n = 2.8 M, 23 against
// 12 us with 1024); longer grids keep the second stage.
constexpr int kLastBlockMax = 128;

// The counter a reduction launch of `grid` workgroups finishes with (NULL:
// the two-launch form).
inline unsigned int* finish_counter(unsigned int* counter, int grid) {
  return (grid > 1 && grid <= kLastBlockMax) ? counter : nullptr;
}

// Second stage over `grid` pairs in `partials`; `sums` holds the chunk sums
// of the two-launch form (grid / kFinishChunk pairs, rounded up).  Nothing
// to do when the launch finished itself (`counter` non-NULL).
bs_status finish_on(const double* partials, double* sums, int grid, double* out, hipStream_t st, const char* op,
                    const unsigned int* counter = nullptr) {
  bs_status s = check_launch(op);
  if (s || grid == 1 || counter) return s;
  if (grid <= kFinishDirect) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, partials, grid, out);
    return check_launch(op);
  }
  const int chunks = (grid + kFinishChunk - 1) / kFinishChunk;
  hipLaunchKernelGGL(k_finish_chunks, dim3(chunks), dim3(kFinishBlock), 0, st, partials, grid, sums);
  if ((s = check_launch(op))) return s;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, sums, chunks, out);
  return check_launch(op);
}

bs_status finish(bs_ctx* ctx, int grid, double* out, hipStream_t st, const char* op, const unsigned int* counter) {
  // chunks <= kMaxStreamBlocks / kFinishChunk
  return finish_on(ctx->partials, ctx->partials + 2 * static_cast<size_t>(kMaxStreamBlocks), grid, out, st, op,
                   counter);
}

// Tune variant of a streaming operation -> Span::order (1 and 2 select the
// XCD-grouped workgroup orders; anything else keeps the dispatch order).
inline int stream_order(int variant) {
  const int o = variant & 3;
  return (o == 1 || o == 2) ? o : 0;
}

inline int norm_unroll(int u) { return (u >= 8) ? 8 : (u >= 4) ? 4 : (u >= 2) ? 2 : 1; }

// Threads per workgroup of a streaming kernel, from its tune variant: + 4
// selects 128, + 8 selects 512, otherwise 256 (the two low bits keep the
// workgroup order).  Unaligned operands (one element per packet) always run
// 256-thread workgroups.
inline int stream_block(const Span& sp, int variant) {
  if (sp.vwidth == 1) return kBlock;
  const int s = (variant >> 2) & 3;
  return s == 1 ? 128 : s == 2 ? 512 : kBlock;
}

// Cache policy of a streaming launch over `bytes` of operands: nontemporal
// accesses unless the tune variant asks for cached ones (+16, the small-size
// regime) and the operands fit the last-level cache.
inline bool stream_nt(int variant, int64_t bytes) { return !cached_access(variant, bytes); }

// Operand bytes of a call that touches `vectors` vectors of n elements.
template <class T>
int64_t operand_bytes(int64_t n, int vectors) {
  return n * vectors * static_cast<int64_t>(sizeof(typename Storage<T>::E));
}

// Launch `K<T, V, U, NB, NT>` for the runtime unroll, packet width, block
// size and cache policy.
#define BS_DISPATCH_U(KERNEL_ARGS, VN, u, NB, NT, grid, stream, ...)                                      \
  do {                                                                                                     \
    if ((u) == 8) {                                                                                        \
      hipLaunchKernelGGL((KERNEL_ARGS(VN, 8, NB, NT)), dim3(grid), dim3(NB), 0, stream, __VA_ARGS__);      \
    } else if ((u) == 4) {                                                                                 \
      hipLaunchKernelGGL((KERNEL_ARGS(VN, 4, NB, NT)), dim3(grid), dim3(NB), 0, stream, __VA_ARGS__);      \
    } else if ((u) == 2) {                                                                                 \
      hipLaunchKernelGGL((KERNEL_ARGS(VN, 2, NB, NT)), dim3(grid), dim3(NB), 0, stream, __VA_ARGS__);      \
    } else {                                                                                               \
      hipLaunchKernelGGL((KERNEL_ARGS(VN, 1, NB, NT)), dim3(grid), dim3(NB), 0, stream, __VA_ARGS__);      \
    }                                                                                                      \
  } while (0)

#define BS_DISPATCH_NT(KERNEL_ARGS, VN, u, NB, nt, grid, stream, ...)                                     \
  do {                                                                                                     \
    if (nt)                                                                                                \
      BS_DISPATCH_U(KERNEL_ARGS, VN, u, NB, true, grid, stream, __VA_ARGS__);                              \
    else                                                                                                   \
      BS_DISPATCH_U(KERNEL_ARGS, VN, u, NB, false, grid, stream, __VA_ARGS__);                             \
  } while (0)

#define BS_DISPATCH_NB(KERNEL_ARGS, T, sp, u, nb, nt, grid, stream, ...)                                   \
  do {                                                                                                     \
    constexpr int VN = Storage<T>::V;                                                                      \
    if ((sp).vwidth == 1) {                                                                                \
      hipLaunchKernelGGL((KERNEL_ARGS(1, 4, kBlock, true)), dim3(grid), dim3(kBlock), 0, stream,            \
                         __VA_ARGS__);                                                                     \
    } else if ((nb) == 128) {                                                                              \
      BS_DISPATCH_NT(KERNEL_ARGS, VN, u, 128, nt, grid, stream, __VA_ARGS__);                              \
    } else if ((nb) == 512) {                                                                              \
      BS_DISPATCH_NT(KERNEL_ARGS, VN, u, 512, nt, grid, stream, __VA_ARGS__);                              \
    } else {                                                                                               \
      BS_DISPATCH_NT(KERNEL_ARGS, VN, u, 256, nt, grid, stream, __VA_ARGS__);                              \
    }                                                                                                      \
  } while (0)


#define K_COPY(V, U, NB, NT) k_copy<T, V, U, NB, NT>
#define K_AXPY(V, U, NB, NT) k_axpy<T, V, U, NB, NT>
#define K_DOT(V, U, NB, NT) k_dot<T, V, U, NB, NT>
#define K_AXPY_DEV(V, U, NB, NT) k_axpy_dev<T, V, U, NB, NT>
#define K_NORM_W(V, U, NB, NT) k_norm<T, V, U, true, NB, NT>
#define K_NORM(V, U, NB, NT) k_norm<T, V, U, false, NB, NT>
#define K_UPD_W(V, U, NB, NT) k_cg_update<T, V, U, true, NB, NT>
#define K_UPD(V, U, NB, NT) k_cg_update<T, V, U, false, NB, NT>
#define K_UPD_DEV_W(V, U, NB, NT) k_cg_update_dev<T, V, U, true, NB, NT>
#define K_UPD_DEV(V, U, NB, NT) k_cg_update_dev<T, V, U, false, NB, NT>

template <class T> constexpr int dtype_index() { return std::is_same<T, double>::value ? 0 : std::is_same<T, float>::value ? 1 : 2; }

template <class T>
bs_status run_copy(bs_ctx* ctx, int64_t n, const void* x, void* y, hipStream_t st) {
  Span sp = make_span<T>(n, {x, y});
  const Tune& tn = tune_for(ctx, OP_COPY, dtype_index<T>(), n);
  sp.order = stream_order(tn.variant);
  const int u = norm_unroll(tn.unroll);
  const int nb = stream_block(sp, tn.variant);
  const bool nt = stream_nt(tn.variant, operand_bytes<T>(n, 2));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, tn.grid_cap, nb);
  BS_DISPATCH_NB(K_COPY, T, sp, u, nb, nt, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<typename Storage<T>::E*>(y), sp);
  return check_launch("bs_copy");
}

template <class T>
bs_status run_axpy(bs_ctx* ctx, int64_t n, double alpha, const void* x, double beta, void* y, hipStream_t st) {
  using C = typename Storage<T>::C;
  Span sp = make_span<T>(n, {x, y});
  const Tune& tn = tune_for(ctx, OP_AXPY, dtype_index<T>(), n);
  sp.order = stream_order(tn.variant);
  const int u = norm_unroll(tn.unroll);
  const int nb = stream_block(sp, tn.variant);
  const bool nt = stream_nt(tn.variant, operand_bytes<T>(n, 3));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, tn.grid_cap, nb);
  BS_DISPATCH_NB(K_AXPY, T, sp, u, nb, nt, g, st, static_cast<C>(alpha), static_cast<const typename Storage<T>::E*>(x), static_cast<C>(beta),
              static_cast<typename Storage<T>::E*>(y), sp);
  return check_launch("bs_axpy");
}

template <class T>
bs_status run_norm(bs_ctx* ctx, int64_t n, const void* x, const void* w, double* out, hipStream_t st) {
  Span sp = make_span<T>(n, {x, w});
  const Tune& tn = tune_for(ctx, OP_NORM, dtype_index<T>(), n);
  sp.order = stream_order(tn.variant);
  const int u = norm_unroll(tn.unroll);
  const int cap = tn.grid_cap < kMaxStreamBlocks ? tn.grid_cap : kMaxStreamBlocks;
  const int nb = stream_block(sp, tn.variant);
  const bool nt = stream_nt(tn.variant, operand_bytes<T>(n, w ? 2 : 1));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap, nb);
  unsigned int* cnt = finish_counter(ctx->counter, g);
  if (w)
    BS_DISPATCH_NB(K_NORM_W, T, sp, u, nb, nt, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<const typename Storage<T>::E*>(w), sp,
                  ctx->partials, out, cnt);
  else
    BS_DISPATCH_NB(K_NORM, T, sp, u, nb, nt, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<const typename Storage<T>::E*>(x), sp,
                  ctx->partials, out, cnt);
  return finish(ctx, g, out, st, "bs_norm", cnt);
}

template <class T>
bs_status run_dot(bs_ctx* ctx, int64_t n, const void* x, const void* y, double* out, hipStream_t st) {
  Span sp = make_span<T>(n, {x, y});
  const Tune& tn = tune_for(ctx, OP_DOT, dtype_index<T>(), n);
  sp.order = stream_order(tn.variant);
  const int u = norm_unroll(tn.unroll);
  const int cap = tn.grid_cap < kMaxStreamBlocks ? tn.grid_cap : kMaxStreamBlocks;
  const int nb = stream_block(sp, tn.variant);
  const bool nt = stream_nt(tn.variant, operand_bytes<T>(n, 2));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap, nb);
  unsigned int* cnt = finish_counter(ctx->counter, g);
  BS_DISPATCH_NB(K_DOT, T, sp, u, nb, nt, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<const typename Storage<T>::E*>(y), sp, ctx->partials, out, cnt);
  return finish(ctx, g, out, st, "bs_dot", cnt);
}

// BS5 with an explicit launch shape and reduction buffers: `partials` holds
// at least `cap` pairs, `sums` at least cap / kFinishChunk (rounded up).
template <class T>
bs_status launch_cg_update(int64_t n, double alpha, void* x, const void* p, void* r, const void* Ap, const void* w,
                           double* out, int unroll, int cap, int variant, double* partials, double* sums,
                           unsigned int* counter, hipStream_t st, const char* op) {
  using C = typename Storage<T>::C;
  using E = typename Storage<T>::E;
  Span sp = make_span<T>(n, {x, p, r, Ap, w});
  sp.order = stream_order(variant);
  const int u = norm_unroll(unroll);
  const int nb = stream_block(sp, variant);
  const bool nt = stream_nt(variant, operand_bytes<T>(n, w ? 7 : 6));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap, nb);
  if (g > cap)
    return fail(BS_ERR_INVALID_ARG, "%s: %d workgroups need more reduction pairs than the %d the buffer holds", op, g,
                cap);
  unsigned int* cnt = finish_counter(counter, g);
  if (w)
    BS_DISPATCH_NB(K_UPD_W, T, sp, u, nb, nt, g, st, static_cast<C>(alpha), static_cast<E*>(x),
                  static_cast<const E*>(p), static_cast<E*>(r), static_cast<const E*>(Ap), static_cast<const E*>(w),
                  sp, partials, out, cnt);
  else
    BS_DISPATCH_NB(K_UPD, T, sp, u, nb, nt, g, st, static_cast<C>(alpha), static_cast<E*>(x),
                  static_cast<const E*>(p), static_cast<E*>(r), static_cast<const E*>(Ap), static_cast<const E*>(p),
                  sp, partials, out, cnt);
  return finish_on(partials, sums, g, out, st, op, cnt);
}

template <class T>
bs_status run_cg_update(bs_ctx* ctx, int64_t n, double alpha, void* x, const void* p, void* r, const void* Ap,
                        const void* w, double* out, hipStream_t st) {
  const Tune& tn = tune_for(ctx, OP_CG_UPDATE, dtype_index<T>(), n);
  const int cap = tn.grid_cap < kMaxStreamBlocks ? tn.grid_cap : kMaxStreamBlocks;
  return launch_cg_update<T>(n, alpha, x, p, r, Ap, w, out, tn.unroll, cap, tn.variant, ctx->partials,
                             ctx->partials + 2 * static_cast<size_t>(kMaxStreamBlocks), ctx->counter, st,
                             "bs_cg_update");
}

// ---------------------------------------------------------------- allocation-free BS5

// Reduction buffer of bs_cg_update_noalloc: kNoAllocPairs per-workgroup
// pairs, then the chunk sums of the second stage, then (in the last 256
// bytes) the counter of the single-launch finish, which starts at zero (the
// array is zero-initialised when the code object loads) and which every
// launch that uses it leaves at zero.  One copy per device, held until the
// process ends.  Host code never passes `scratch` itself (in host code it
// names a host-side stand-in): it passes the device address that
// hipGetSymbolAddress returns for the current device.
constexpr int kNoAllocPairs = kMaxReduceBlocks;
constexpr int kNoAllocSums = (kNoAllocPairs + kFinishChunk - 1) / kFinishChunk;
constexpr int kNoAllocCounter = 2 * (kNoAllocPairs + kNoAllocSums);  // offset (in doubles) of the counter
constexpr int kNoAllocUnroll = 4;  // the built-in launch shape of the CG update
static __device__ __align__(256) double scratch[kNoAllocCounter + 32];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
bs_status scratch_for_current_device(double** out, const char* op) {
  int device = -1;
  if (bs_status s = check_hip(hipGetDevice(&device), op)) return s;
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(BS_ERR_UNSUPPORTED, "%s: device %d is beyond the %d devices the scratch table holds", op, device,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (bs_status s = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), op)) return s;
    if (!ptr) return fail(BS_ERR_HIP, "%s: no device address for the scratch buffer", op);
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return BS_OK;
}

template <class T>
bs_status run_axpy_dev(bs_ctx* ctx, int64_t n, DevScalar a, const void* x, DevScalar b, void* y, hipStream_t st) {
  using E = typename Storage<T>::E;
  Span sp = make_span<T>(n, {x, y});
  const Tune& tn = tune_for(ctx, OP_AXPY, dtype_index<T>(), n);
  sp.order = stream_order(tn.variant);
  const int u = norm_unroll(tn.unroll);
  const int nb = stream_block(sp, tn.variant);
  const bool nt = stream_nt(tn.variant, operand_bytes<T>(n, 3));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, tn.grid_cap, nb);
  BS_DISPATCH_NB(K_AXPY_DEV, T, sp, u, nb, nt, g, st, a, static_cast<const E*>(x), b, static_cast<E*>(y), sp);
  return check_launch("bs_axpy_dev");
}

template <class T>
bs_status run_cg_update_dev(bs_ctx* ctx, int64_t n, DevScalar a, void* x, const void* p, void* r, const void* Ap,
                            const void* w, double* out, hipStream_t st) {
  using E = typename Storage<T>::E;
  Span sp = make_span<T>(n, {x, p, r, Ap, w});
  const Tune& tn = tune_for(ctx, OP_CG_UPDATE, dtype_index<T>(), n);
  sp.order = stream_order(tn.variant);
  const int u = norm_unroll(tn.unroll);
  const int cap = tn.grid_cap < kMaxStreamBlocks ? tn.grid_cap : kMaxStreamBlocks;
  const int nb = stream_block(sp, tn.variant);
  const bool nt = stream_nt(tn.variant, operand_bytes<T>(n, w ? 7 : 6));
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap, nb);
  unsigned int* cnt = finish_counter(ctx->counter, g);
  if (w)
    BS_DISPATCH_NB(K_UPD_DEV_W, T, sp, u, nb, nt, g, st, a, static_cast<E*>(x), static_cast<const E*>(p),
                  static_cast<E*>(r), static_cast<const E*>(Ap), static_cast<const E*>(w), sp, ctx->partials, out, cnt);
  else
    BS_DISPATCH_NB(K_UPD_DEV, T, sp, u, nb, nt, g, st, a, static_cast<E*>(x), static_cast<const E*>(p),
                  static_cast<E*>(r), static_cast<const E*>(Ap), static_cast<const E*>(p), sp, ctx->partials, out, cnt);
  return finish(ctx, g, out, st, "bs_cg_update_dev", cnt);
}

bs_status check_scalar_ptr(const char* op, const char* name, const double* d) {
  if (d && !aligned_to(d, 8)) return fail(BS_ERR_INVALID_ARG, "%s: %s is not 8-byte aligned", op, name);
  return BS_OK;
}

// Pointer [p, p + n*s) and [q, q + m*s) overlap?
inline bool overlap(const void* p, int64_t nb, const void* q, int64_t mb) {
  if (!p || !q || nb == 0 || mb == 0) return false;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p), b = reinterpret_cast<uintptr_t>(q);
  return a < b + static_cast<uintptr_t>(mb) && b < a + static_cast<uintptr_t>(nb);
}

}  // namespace
}  // namespace bs

using namespace bs;

#define BS_TYPED(dtype, CALL)                                        \
  switch (dtype) {                                                   \
    case BS_F64: { using T = double; return CALL; }                  \
    case BS_F32: { using T = float; return CALL; }                   \
    case BS_BF16: { using T = dev::bf16; return CALL; }              \
  }                                                                  \
  return fail(BS_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype)

extern "C" bs_status bs_copy(bs_ctx* ctx, bs_dtype dtype, int64_t n, const void* x, void* y, void* stream) {
  bs_status s;
  if ((s = check_ctx(ctx, "bs_copy")) || (s = check_dtype("bs_copy", dtype)) ||
      (s = check_vec("bs_copy", "x", x, n, dtype)) || (s = check_vec("bs_copy", "y", y, n, dtype)))
    return s;
  const int64_t nb = n * dtype_size(dtype);
  if (overlap(x, nb, y, nb)) return fail(BS_ERR_INVALID_ARG, "bs_copy: y overlaps x");
  if (n == 0) return BS_OK;
  BS_TYPED(dtype, run_copy<T>(ctx, n, x, y, static_cast<hipStream_t>(stream)));
}

extern "C" bs_status bs_axpy(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, const void* x, double beta,
                             void* y, void* stream) {
  bs_status s;
  if ((s = check_ctx(ctx, "bs_axpy")) || (s = check_dtype("bs_axpy", dtype)) ||
      (s = check_vec("bs_axpy", "x", x, n, dtype)) || (s = check_vec("bs_axpy", "y", y, n, dtype)))
    return s;
  const int64_t nb = n * dtype_size(dtype);
  if (overlap(x, nb, y, nb)) return fail(BS_ERR_INVALID_ARG, "bs_axpy: y overlaps x");
  if (n == 0) return BS_OK;
  BS_TYPED(dtype, run_axpy<T>(ctx, n, alpha, x, beta, y, static_cast<hipStream_t>(stream)));
}

extern "C" bs_status bs_norm(bs_ctx* ctx, bs_dtype dtype, int64_t n, const void* x, const void* w, double* d_out,
                             void* stream) {
  bs_status s;
  if ((s = check_ctx(ctx, "bs_norm")) || (s = check_dtype("bs_norm", dtype)) ||
      (s = check_vec("bs_norm", "x", x, n, dtype)))
    return s;
  if (w && (s = check_vec("bs_norm", "w", w, n, dtype))) return s;
  if (!d_out) return fail(BS_ERR_INVALID_ARG, "bs_norm: d_out is NULL");
  if (!aligned_to(d_out, 8)) return fail(BS_ERR_INVALID_ARG, "bs_norm: d_out is not 8-byte aligned");
  BS_TYPED(dtype, run_norm<T>(ctx, n, x, w, d_out, static_cast<hipStream_t>(stream)));
}

extern "C" bs_status bs_dot(bs_ctx* ctx, bs_dtype dtype, int64_t n, const void* x, const void* y, double* d_out,
                            void* stream) {
  bs_status s;
  if ((s = check_ctx(ctx, "bs_dot")) || (s = check_dtype("bs_dot", dtype)) ||
      (s = check_vec("bs_dot", "x", x, n, dtype)) || (s = check_vec("bs_dot", "y", y, n, dtype)))
    return s;
  if (!d_out) return fail(BS_ERR_INVALID_ARG, "bs_dot: d_out is NULL");
  if (!aligned_to(d_out, 8)) return fail(BS_ERR_INVALID_ARG, "bs_dot: d_out is not 8-byte aligned");
  BS_TYPED(dtype, run_dot<T>(ctx, n, x, y, d_out, static_cast<hipStream_t>(stream)));
}

extern "C" bs_status bs_cg_update(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, void* x, const void* p,
                                  void* r, const void* Ap, const void* w, double* d_rr, void* stream) {
  bs_status s;
  const char* op = "bs_cg_update";
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype)) || (s = check_vec(op, "x", x, n, dtype)) ||
      (s = check_vec(op, "p", p, n, dtype)) || (s = check_vec(op, "r", r, n, dtype)) ||
      (s = check_vec(op, "Ap", Ap, n, dtype)))
    return s;
  if (w && (s = check_vec(op, "w", w, n, dtype))) return s;
  if (!d_rr) return fail(BS_ERR_INVALID_ARG, "bs_cg_update: d_rr is NULL");
  if (!aligned_to(d_rr, 8)) return fail(BS_ERR_INVALID_ARG, "bs_cg_update: d_rr is not 8-byte aligned");
  const int64_t nb = n * dtype_size(dtype);
  if (overlap(x, nb, r, nb) || overlap(x, nb, p, nb) || overlap(x, nb, Ap, nb) || overlap(x, nb, w, nb) ||
      overlap(r, nb, p, nb) || overlap(r, nb, Ap, nb) || overlap(r, nb, w, nb))
    return fail(BS_ERR_INVALID_ARG, "bs_cg_update: x or r overlaps another operand");
  BS_TYPED(dtype, run_cg_update<T>(ctx, n, alpha, x, p, r, Ap, w, d_rr, static_cast<hipStream_t>(stream)));
}

extern "C" bs_status bs_cg_update_noalloc(bs_dtype dtype, int64_t n, double alpha, void* x, const void* p, void* r,
                                          const void* Ap, const void* w, double* d_rr, void* stream) {
  bs_status s;
  const char* op = "bs_cg_update_noalloc";
  if ((s = check_dtype(op, dtype)) || (s = check_vec(op, "x", x, n, dtype)) || (s = check_vec(op, "p", p, n, dtype)) ||
      (s = check_vec(op, "r", r, n, dtype)) || (s = check_vec(op, "Ap", Ap, n, dtype)))
    return s;
  if (w && (s = check_vec(op, "w", w, n, dtype))) return s;
  if (!d_rr) return fail(BS_ERR_INVALID_ARG, "bs_cg_update_noalloc: d_rr is NULL");
  if (!aligned_to(d_rr, 8)) return fail(BS_ERR_INVALID_ARG, "bs_cg_update_noalloc: d_rr is not 8-byte aligned");
  const int64_t nb = n * dtype_size(dtype);
  if (overlap(x, nb, r, nb) || overlap(x, nb, p, nb) || overlap(x, nb, Ap, nb) || overlap(x, nb, w, nb) ||
      overlap(r, nb, p, nb) || overlap(r, nb, Ap, nb) || overlap(r, nb, w, nb))
    return fail(BS_ERR_INVALID_ARG, "bs_cg_update_noalloc: x or r overlaps another operand");
  double* buf = nullptr;
  if ((s = scratch_for_current_device(&buf, op))) return s;
  double* sums = buf + 2 * static_cast<size_t>(kNoAllocPairs);
  unsigned int* counter = reinterpret_cast<unsigned int*>(buf + kNoAllocCounter);
  BS_TYPED(dtype, launch_cg_update<T>(n, alpha, x, p, r, Ap, w, d_rr, kNoAllocUnroll, kNoAllocPairs, 0, buf, sums,
                                      counter, static_cast<hipStream_t>(stream), op));
}

extern "C" bs_status bs_axpy_dev(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha, const double* d_alpha_num,
                                 const double* d_alpha_den, const void* x, double beta, const double* d_beta_num,
                                 const double* d_beta_den, void* y, void* stream) {
  bs_status s;
  const char* op = "bs_axpy_dev";
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype)) || (s = check_vec(op, "x", x, n, dtype)) ||
      (s = check_vec(op, "y", y, n, dtype)) || (s = check_scalar_ptr(op, "d_alpha_num", d_alpha_num)) ||
      (s = check_scalar_ptr(op, "d_alpha_den", d_alpha_den)) || (s = check_scalar_ptr(op, "d_beta_num", d_beta_num)) ||
      (s = check_scalar_ptr(op, "d_beta_den", d_beta_den)))
    return s;
  const int64_t nb = n * dtype_size(dtype);
  if (overlap(x, nb, y, nb)) return fail(BS_ERR_INVALID_ARG, "%s: y overlaps x", op);
  for (const double* q : {d_alpha_num, d_alpha_den, d_beta_num, d_beta_den})
    if (overlap(q, 8, y, nb)) return fail(BS_ERR_INVALID_ARG, "%s: y overlaps a scalar", op);
  if (n == 0) return BS_OK;
  const DevScalar a{alpha, d_alpha_num, d_alpha_den}, b{beta, d_beta_num, d_beta_den};
  BS_TYPED(dtype, run_axpy_dev<T>(ctx, n, a, x, b, y, static_cast<hipStream_t>(stream)));
}

extern "C" bs_status bs_cg_update_dev(bs_ctx* ctx, bs_dtype dtype, int64_t n, double alpha,
                                      const double* d_alpha_num, const double* d_alpha_den, void* x, const void* p,
                                      void* r, const void* Ap, const void* w, double* d_rr, void* stream) {
  bs_status s;
  const char* op = "bs_cg_update_dev";
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype)) || (s = check_vec(op, "x", x, n, dtype)) ||
      (s = check_vec(op, "p", p, n, dtype)) || (s = check_vec(op, "r", r, n, dtype)) ||
      (s = check_vec(op, "Ap", Ap, n, dtype)) || (s = check_scalar_ptr(op, "d_alpha_num", d_alpha_num)) ||
      (s = check_scalar_ptr(op, "d_alpha_den", d_alpha_den)))
    return s;
  if (w && (s = check_vec(op, "w", w, n, dtype))) return s;
  if (!d_rr) return fail(BS_ERR_INVALID_ARG, "%s: d_rr is NULL", op);
  if (!aligned_to(d_rr, 8)) return fail(BS_ERR_INVALID_ARG, "%s: d_rr is not 8-byte aligned", op);
  if (d_rr == d_alpha_num || d_rr == d_alpha_den) return fail(BS_ERR_INVALID_ARG, "%s: d_rr is a scalar input", op);
  const int64_t nb = n * dtype_size(dtype);
  if (overlap(x, nb, r, nb) || overlap(x, nb, p, nb) || overlap(x, nb, Ap, nb) || overlap(x, nb, w, nb) ||
      overlap(r, nb, p, nb) || overlap(r, nb, Ap, nb) || overlap(r, nb, w, nb))
    return fail(BS_ERR_INVALID_ARG, "%s: x or r overlaps another operand", op);
  for (const double* q : {d_alpha_num, d_alpha_den, static_cast<const double*>(d_rr)})
    if (overlap(q, 8, x, nb) || overlap(q, 8, r, nb)) return fail(BS_ERR_INVALID_ARG, "%s: x or r overlaps a scalar", op);
  const DevScalar a{alpha, d_alpha_num, d_alpha_den};
  BS_TYPED(dtype, run_cg_update_dev<T>(ctx, n, a, x, p, r, Ap, w, d_rr, static_cast<hipStream_t>(stream)));
}
