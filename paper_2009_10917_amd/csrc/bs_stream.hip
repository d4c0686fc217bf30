// BS1-BS5: copy, AXPY, norm, inner product and the fused CG update
// (Table 1; Listings 1-3; Algorithm 1 steps 8-10).
//
// All five stream their operands once through 16-byte packets (dwordx4
// loads and stores).  A workgroup of 256 threads handles U packets per
// thread per trip and the grid strides over the vector beyond `grid_cap`
// workgroups.  Scalar elements that precede the first 16-byte boundary or
// follow the last full packet are handled by workgroup 0.  When the operands
// are not mutually 16-byte aligned the same kernels run with one-element
// packets.
//
// The reductions accumulate per thread in compensated form (sum plus
// running error), combine the 64 lanes of a wave by xor-shuffles and the
// waves of a workgroup through LDS, and store one pair per workgroup; a
// second launch of one 1024-thread workgroup adds the pairs in index order,
// as the paper's two-kernel reductions do (Section 5).  Finishing inside the
// first launch would need an agent-scope fence per workgroup, which on this
// 8-XCD part costs more than the second launch.

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

using dev::bf16;
using dev::DW;
using dev::Storage;
using dev::vget;
using dev::vset;

// Layout of one vector operation over n elements: `head` scalar elements,
// then `nvec` packets of `vwidth` elements, then the scalar tail.
struct Span {
  int64_t n;
  int64_t nvec;
  int32_t head;
  int32_t vwidth;
};

// Element handled by thread threadIdx.x of workgroup 0 in the scalar head or
// tail, or -1.  head < V <= 8 and tail < V, so 32 threads cover both.
__device__ __forceinline__ int64_t scalar_index(const Span& sp) {
  const int t = threadIdx.x;
  const int64_t tail_start = sp.head + sp.nvec * sp.vwidth;
  if (t < sp.head) return t;
  if (t >= 16 && t < 32 && tail_start + (t - 16) < sp.n) return tail_start + (t - 16);
  return -1;
}

// The streaming loop shared by BS1-BS5.  Thread t of workgroup b owns
// packets i, i + 256, ..., i + (U-1)*256 with i = b*256*U + t and strides by
// the whole grid.  Each trip first issues all of its loads (op.load), then
// computes and stores (op.apply), so U packets per operand are in flight.
// Trips that are entirely in range run without bounds checks; only the last
// (ragged) trip of a thread checks each packet.
template <int U, class Op>
__device__ __forceinline__ void stream_loop(Op& op, const Span& sp) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * kBlock * U;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock * U + threadIdx.x;
  for (; i + static_cast<int64_t>(U - 1) * kBlock < sp.nvec; i += step) {
    typename Op::Regs r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) op.load(r[u], i + u * kBlock);
#pragma unroll
    for (int u = 0; u < U; ++u) op.apply(r[u], i + u * kBlock);
  }
  if (i < sp.nvec) {
    typename Op::Regs r[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * kBlock < sp.nvec) op.load(r[u], i + u * kBlock);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * kBlock < sp.nvec) op.apply(r[u], i + u * kBlock);
  }
  if (blockIdx.x == 0) {
    const int64_t e = scalar_index(sp);
    if (e >= 0) op.scalar(e);
  }
}

template <class T, int V>
struct Base {
  using S = Storage<T>;
  using E = typename S::E;
  using C = typename S::C;
  using Vec = typename dev::VecOf<E, V>::type;
  // packet j of the operand that starts at p (after the scalar head); every
  // packet is touched once, so the accesses are nontemporal
  __device__ static Vec ld(const E* p, int64_t j) { return dev::ld_nt(reinterpret_cast<const Vec*>(p) + j); }
  __device__ static void st(E* p, int64_t j, const Vec& v) { dev::st_nt(reinterpret_cast<Vec*>(p) + j, v); }
};

// ---------------------------------------------------------------- BS1 copy

template <class T, int V>
struct CopyOp : Base<T, V> {
  using B = Base<T, V>;
  using E = typename B::E;
  struct Regs {
    typename B::Vec a;
  };
  const E* x;
  E* y;
  int32_t head;
  __device__ void load(Regs& r, int64_t j) const { r.a = B::ld(x + head, j); }
  __device__ void apply(Regs& r, int64_t j) const { B::st(y + head, j, r.a); }
  __device__ void scalar(int64_t e) const { y[e] = x[e]; }
};

template <class T, int V, int U>
__global__ __launch_bounds__(kBlock) void k_copy(const typename Storage<T>::E* __restrict__ x,
                                                 typename Storage<T>::E* __restrict__ y, Span sp) {
  CopyOp<T, V> op{{}, x, y, sp.head};
  stream_loop<U>(op, sp);
}

// ---------------------------------------------------------------- BS2 AXPY

template <class T, int V>
struct AxpyOp : Base<T, V> {
  using B = Base<T, V>;
  using S = typename B::S;
  using E = typename B::E;
  using C = typename B::C;
  struct Regs {
    typename B::Vec a, b;
  };
  C alpha, beta;
  const E* x;
  E* y;
  int32_t head;
  __device__ C f(E xe, E ye) const { return alpha * S::load(xe) + beta * S::load(ye); }
  __device__ void load(Regs& r, int64_t j) const {
    r.a = B::ld(x + head, j);
    r.b = B::ld(y + head, j);
  }
  __device__ void apply(Regs& r, int64_t j) const {
#pragma unroll
    for (int k = 0; k < V; ++k) vset(r.b, k, S::store(f(vget<typename B::Vec, E>(r.a, k), vget<typename B::Vec, E>(r.b, k))));
    B::st(y + head, j, r.b);
  }
  __device__ void scalar(int64_t e) const { y[e] = S::store(f(x[e], y[e])); }
};

template <class T, int V, int U>
__global__ __launch_bounds__(kBlock) void k_axpy(typename Storage<T>::C alpha, const typename Storage<T>::E* __restrict__ x,
                                                 typename Storage<T>::C beta, typename Storage<T>::E* __restrict__ y,
                                                 Span sp) {
  AxpyOp<T, V> op{{}, alpha, beta, x, y, sp.head};
  stream_loop<U>(op, sp);
}

// ---------------------------------------------------------------- BS3 norm

template <class T, int V, bool W>
struct NormOp : Base<T, V> {
  using B = Base<T, V>;
  using S = typename B::S;
  using E = typename B::E;
  using C = typename B::C;
  using Vec = typename B::Vec;
  struct Regs {
    Vec a, b;
  };
  const E* x;
  const E* w;
  int32_t head;
  DW<C> acc;
  // term fl(x*x), or fl(w*fl(x*x))
  __device__ void add(E xe, E we) {
    const C xk = S::load(xe);
    C t = xk * xk;
    if (W) t = S::load(we) * t;
    dev::dw_acc(acc, t);
  }
  __device__ void load(Regs& r, int64_t j) const {
    r.a = B::ld(x + head, j);
    if (W) r.b = B::ld(w + head, j);
  }
  __device__ void apply(Regs& r, int64_t) {
#pragma unroll
    for (int k = 0; k < V; ++k) add(vget<Vec, E>(r.a, k), W ? vget<Vec, E>(r.b, k) : E{});
  }
  __device__ void scalar(int64_t e) { add(x[e], W ? w[e] : E{}); }
};

template <class T, int V, int U, bool W>
__global__ __launch_bounds__(kBlock) void k_norm(const typename Storage<T>::E* __restrict__ x,
                                                 const typename Storage<T>::E* __restrict__ w, Span sp,
                                                 double* partials, double* out) {
  using C = typename Storage<T>::C;
  NormOp<T, V, W> op{{}, x, w, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U>(op, sp);
  dev::block_store_pair<kBlock>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, out);
}

// ---------------------------------------------------------------- BS4 inner product

template <class T, int V>
struct DotOp : Base<T, V> {
  using B = Base<T, V>;
  using S = typename B::S;
  using E = typename B::E;
  using C = typename B::C;
  using Vec = typename B::Vec;
  struct Regs {
    Vec a, b;
  };
  const E* x;
  const E* y;
  int32_t head;
  DW<C> acc;
  __device__ void load(Regs& r, int64_t j) const {
    r.a = B::ld(x + head, j);
    r.b = B::ld(y + head, j);
  }
  __device__ void apply(Regs& r, int64_t) {
#pragma unroll
    for (int k = 0; k < V; ++k) dev::dw_acc_prod(acc, S::load(vget<Vec, E>(r.a, k)), S::load(vget<Vec, E>(r.b, k)));
  }
  __device__ void scalar(int64_t e) { dev::dw_acc_prod(acc, S::load(x[e]), S::load(y[e])); }
};

template <class T, int V, int U>
__global__ __launch_bounds__(kBlock) void k_dot(const typename Storage<T>::E* __restrict__ x,
                                                const typename Storage<T>::E* __restrict__ y, Span sp,
                                                double* partials, double* out) {
  using C = typename Storage<T>::C;
  DotOp<T, V> op{{}, x, y, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U>(op, sp);
  dev::block_store_pair<kBlock>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, out);
}

// ---------------------------------------------------------------- BS5 fused CG update

template <class T, int V, bool W>
struct CgOp : Base<T, V> {
  using B = Base<T, V>;
  using S = typename B::S;
  using E = typename B::E;
  using C = typename B::C;
  using Vec = typename B::Vec;
  struct Regs {
    Vec x, p, r, a, w;
  };
  C alpha;
  E* x;
  const E* p;
  E* r;
  const E* Ap;
  const E* w;
  int32_t head;
  DW<C> acc;
  // updates one entry in place; the reduction uses the stored new residual
  __device__ void one(E& xe, E pe, E& re, E ae, E we) {
    xe = S::store(S::load(xe) + alpha * S::load(pe));
    re = S::store(S::load(re) - alpha * S::load(ae));
    const C rk = S::load(re);
    C t = rk * rk;
    if (W) t = S::load(we) * t;
    dev::dw_acc(acc, t);
  }
  __device__ void load(Regs& g, int64_t j) const {
    g.x = B::ld(x + head, j);
    g.p = B::ld(p + head, j);
    g.r = B::ld(r + head, j);
    g.a = B::ld(Ap + head, j);
    if (W) g.w = B::ld(w + head, j);
  }
  __device__ void apply(Regs& g, int64_t j) {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      E xe = vget<Vec, E>(g.x, k), re = vget<Vec, E>(g.r, k);
      one(xe, vget<Vec, E>(g.p, k), re, vget<Vec, E>(g.a, k), W ? vget<Vec, E>(g.w, k) : E{});
      vset(g.x, k, xe);
      vset(g.r, k, re);
    }
    B::st(x + head, j, g.x);
    B::st(r + head, j, g.r);
  }
  __device__ void scalar(int64_t e) {
    E xe = x[e], re = r[e];
    one(xe, p[e], re, Ap[e], W ? w[e] : E{});
    x[e] = xe;
    r[e] = re;
  }
};

template <class T, int V, int U, bool W>
__global__ __launch_bounds__(kBlock) void k_cg_update(typename Storage<T>::C alpha, typename Storage<T>::E* __restrict__ x,
                                                      const typename Storage<T>::E* __restrict__ p,
                                                      typename Storage<T>::E* __restrict__ r,
                                                      const typename Storage<T>::E* __restrict__ Ap,
                                                      const typename Storage<T>::E* __restrict__ w, Span sp,
                                                      double* partials, double* out) {
  using C = typename Storage<T>::C;
  CgOp<T, V, W> op{{}, alpha, x, p, r, Ap, w, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U>(op, sp);
  dev::block_store_pair<kBlock>(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials, out);
}

// ---------------------------------------------------------------- host side

// Packet layout for a set of same-typed operands: 16-byte packets when all
// operands share their address modulo 16, one-element packets otherwise.
template <class T>
Span make_span(int64_t n, std::initializer_list<const void*> ptrs) {
  constexpr int V = Storage<T>::V;
  const void* first = *ptrs.begin();
  const uintptr_t m = reinterpret_cast<uintptr_t>(first) % 16;
  using E = typename Storage<T>::E;
  bool same = true;
  for (const void* q : ptrs)
    if (q && reinterpret_cast<uintptr_t>(q) % 16 != m) same = false;
  Span sp;
  sp.n = n;
  if (same) {
    int64_t head = m ? static_cast<int64_t>((16 - m) / sizeof(E)) : 0;
    if (head > n) head = n;
    sp.head = static_cast<int32_t>(head);
    sp.vwidth = V;
    sp.nvec = (n - head) / V;
  } else {
    sp.head = 0;
    sp.vwidth = 1;
    sp.nvec = n;
  }
  return sp;
}

inline int grid_for(const Span& sp, int unroll, int cap) {
  const int64_t per = static_cast<int64_t>(kBlock) * unroll;
  int64_t g = (sp.nvec + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

// Second stage of every reduction: one workgroup adds the G per-workgroup
// pairs, thread t taking pairs t, t + 1024, ... in order.
__global__ __launch_bounds__(kFinishBlock) void k_finish(const double* __restrict__ partials, int G,
                                                          double* __restrict__ out) {
  DW<double> r{0.0, 0.0};
  for (int i = threadIdx.x; i < G; i += kFinishBlock) r = dev::dw_add(r, DW<double>{partials[2 * i], partials[2 * i + 1]});
  r = dev::block_reduce<kFinishBlock>(r);
  if (threadIdx.x == 0) *out = r.s + r.c;
}

bs_status finish(bs_ctx* ctx, int grid, double* out, hipStream_t st, const char* op) {
  bs_status s = check_launch(op);
  if (s || grid == 1) return s;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, st, ctx->partials, grid, out);
  return check_launch(op);
}

inline int norm_unroll(int u) { return (u >= 8) ? 8 : (u >= 4) ? 4 : (u >= 2) ? 2 : 1; }

// Launch `K<T, V, U>` for the runtime unroll and packet width.
#define BS_DISPATCH(KERNEL, T, sp, u, grid, stream, ...)                                                  \
  do {                                                                                                     \
    constexpr int VN = Storage<T>::V;                                                                      \
    if ((sp).vwidth == 1) {                                                                                \
      hipLaunchKernelGGL((KERNEL<T, 1, 4>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);             \
    } else if ((u) == 8) {                                                                                 \
      hipLaunchKernelGGL((KERNEL<T, VN, 8>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);            \
    } else if ((u) == 4) {                                                                                 \
      hipLaunchKernelGGL((KERNEL<T, VN, 4>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);            \
    } else if ((u) == 2) {                                                                                 \
      hipLaunchKernelGGL((KERNEL<T, VN, 2>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);            \
    } else {                                                                                               \
      hipLaunchKernelGGL((KERNEL<T, VN, 1>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);            \
    }                                                                                                      \
  } while (0)

// The same with an extra bool template argument (weighted or not).
#define BS_DISPATCH_B(KERNEL, T, B, sp, u, grid, stream, ...)                                             \
  do {                                                                                                     \
    constexpr int VN = Storage<T>::V;                                                                      \
    if ((sp).vwidth == 1) {                                                                                \
      hipLaunchKernelGGL((KERNEL<T, 1, 4, B>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);          \
    } else if ((u) == 8) {                                                                                 \
      hipLaunchKernelGGL((KERNEL<T, VN, 8, B>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);         \
    } else if ((u) == 4) {                                                                                 \
      hipLaunchKernelGGL((KERNEL<T, VN, 4, B>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);         \
    } else if ((u) == 2) {                                                                                 \
      hipLaunchKernelGGL((KERNEL<T, VN, 2, B>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);         \
    } else {                                                                                               \
      hipLaunchKernelGGL((KERNEL<T, VN, 1, B>), dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);         \
    }                                                                                                      \
  } while (0)

template <class T>
bs_status run_copy(bs_ctx* ctx, int64_t n, const void* x, void* y, hipStream_t st) {
  const Span sp = make_span<T>(n, {x, y});
  const Tune& tn = ctx->tune[OP_COPY][0];
  const int u = norm_unroll(tn.unroll);
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, tn.grid_cap);
  BS_DISPATCH(k_copy, T, sp, u, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<typename Storage<T>::E*>(y), sp);
  return check_launch("bs_copy");
}

template <class T>
bs_status run_axpy(bs_ctx* ctx, int64_t n, double alpha, const void* x, double beta, void* y, hipStream_t st) {
  using C = typename Storage<T>::C;
  const Span sp = make_span<T>(n, {x, y});
  const Tune& tn = ctx->tune[OP_AXPY][0];
  const int u = norm_unroll(tn.unroll);
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, tn.grid_cap);
  BS_DISPATCH(k_axpy, T, sp, u, g, st, static_cast<C>(alpha), static_cast<const typename Storage<T>::E*>(x), static_cast<C>(beta),
              static_cast<typename Storage<T>::E*>(y), sp);
  return check_launch("bs_axpy");
}

template <class T>
bs_status run_norm(bs_ctx* ctx, int64_t n, const void* x, const void* w, double* out, hipStream_t st) {
  const Span sp = make_span<T>(n, {x, w});
  const Tune& tn = ctx->tune[OP_NORM][0];
  const int u = norm_unroll(tn.unroll);
  const int cap = tn.grid_cap < kMaxReduceBlocks ? tn.grid_cap : kMaxReduceBlocks;
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap);
  if (w)
    BS_DISPATCH_B(k_norm, T, true, sp, u, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<const typename Storage<T>::E*>(w), sp,
                  ctx->partials, out);
  else
    BS_DISPATCH_B(k_norm, T, false, sp, u, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<const typename Storage<T>::E*>(x), sp,
                  ctx->partials, out);
  return finish(ctx, g, out, st, "bs_norm");
}

template <class T>
bs_status run_dot(bs_ctx* ctx, int64_t n, const void* x, const void* y, double* out, hipStream_t st) {
  const Span sp = make_span<T>(n, {x, y});
  const Tune& tn = ctx->tune[OP_DOT][0];
  const int u = norm_unroll(tn.unroll);
  const int cap = tn.grid_cap < kMaxReduceBlocks ? tn.grid_cap : kMaxReduceBlocks;
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap);
  BS_DISPATCH(k_dot, T, sp, u, g, st, static_cast<const typename Storage<T>::E*>(x), static_cast<const typename Storage<T>::E*>(y), sp, ctx->partials, out);
  return finish(ctx, g, out, st, "bs_dot");
}

template <class T>
bs_status run_cg_update(bs_ctx* ctx, int64_t n, double alpha, void* x, const void* p, void* r, const void* Ap,
                        const void* w, double* out, hipStream_t st) {
  using C = typename Storage<T>::C;
  const Span sp = make_span<T>(n, {x, p, r, Ap, w});
  const Tune& tn = ctx->tune[OP_CG_UPDATE][0];
  const int u = norm_unroll(tn.unroll);
  const int cap = tn.grid_cap < kMaxReduceBlocks ? tn.grid_cap : kMaxReduceBlocks;
  const int g = grid_for(sp, sp.vwidth == 1 ? 4 : u, cap);
  if (w)
    BS_DISPATCH_B(k_cg_update, T, true, sp, u, g, st, static_cast<C>(alpha), static_cast<typename Storage<T>::E*>(x),
                  static_cast<const typename Storage<T>::E*>(p), static_cast<typename Storage<T>::E*>(r), static_cast<const typename Storage<T>::E*>(Ap),
                  static_cast<const typename Storage<T>::E*>(w), sp, ctx->partials, out);
  else
    BS_DISPATCH_B(k_cg_update, T, false, sp, u, g, st, static_cast<C>(alpha), static_cast<typename Storage<T>::E*>(x),
                  static_cast<const typename Storage<T>::E*>(p), static_cast<typename Storage<T>::E*>(r), static_cast<const typename Storage<T>::E*>(Ap),
                  static_cast<const typename Storage<T>::E*>(p), sp, ctx->partials, out);
  return finish(ctx, g, out, st, "bs_cg_update");
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
