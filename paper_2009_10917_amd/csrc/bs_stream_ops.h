// Streaming building blocks shared by the operation kernels: the packet
// layout of a vector operation, the grid-stride loop that moves 16-byte
// packets, and the per-element bodies of BS1-BS5.
#pragma once

#include <initializer_list>

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace ops {

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
  int32_t order;  // workgroup order, see logical_block
};

// Which packets workgroup blockIdx.x streams: its number under the tune's
// workgroup order.  Order 0 keeps the dispatch order, so the 8 XCDs
// interleave 4 KB slices of every operand; order 1 gives each XCD 1 MB runs
// (dev::group_block); order 2 one contiguous range per XCD (dev::xcd_block).
__device__ __forceinline__ int64_t logical_block(const Span& sp) {
  return dev::block_order(blockIdx.x, gridDim.x, sp.order);
}

// Element handled by thread threadIdx.x of workgroup 0 in the scalar head or
// tail, or -1.  head < V <= 8 and tail < V, so 32 threads cover both.
__device__ __forceinline__ int64_t scalar_index(const Span& sp) {
  const int t = threadIdx.x;
  const int64_t tail_start = sp.head + sp.nvec * sp.vwidth;
  if (t < sp.head) return t;
  if (t >= 16 && t < 32 && tail_start + (t - 16) < sp.n) return tail_start + (t - 16);
  return -1;
}

// The streaming loop shared by BS1-BS5.  Thread t of workgroup b (the
// logical block number) of NB threads owns packets i, i + NB, ...,
// i + (U-1)*NB with i = b*NB*U + t and strides by the whole grid.  Each trip first issues
// all of its loads (op.load), then computes and stores (op.apply), so U
// packets per operand are in flight.
// Trips that are entirely in range run without bounds checks; only the last
// (ragged) trip of a thread checks each packet.
template <int U, int NB = kBlock, class Op>
__device__ __forceinline__ void stream_loop(Op& op, const Span& sp) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * NB * U;
  int64_t i = logical_block(sp) * NB * U + threadIdx.x;
  for (; i + static_cast<int64_t>(U - 1) * NB < sp.nvec; i += step) {
    typename Op::Regs r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) op.load(r[u], i + u * NB);
#pragma unroll
    for (int u = 0; u < U; ++u) op.apply(r[u], i + u * NB);
  }
  if (i < sp.nvec) {
    typename Op::Regs r[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * NB < sp.nvec) op.load(r[u], i + u * NB);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * NB < sp.nvec) op.apply(r[u], i + u * NB);
  }
  if (blockIdx.x == 0) {
    const int64_t e = scalar_index(sp);
    if (e >= 0) op.scalar(e);
  }
}

// NT: every packet is touched once per call, so by default the accesses
// are nontemporal; vectors that the next calls will touch again while they
// still fit the 256 MB last-level cache (the small-size regime) run faster
// with ordinary cached accesses (NT = false).
template <class T, int V, bool NT = true>
struct Base {
  using S = Storage<T>;
  using E = typename S::E;
  using C = typename S::C;
  using Vec = typename dev::VecOf<E, V>::type;
  // packet j of the operand that starts at p (after the scalar head)
  __device__ static Vec ld(const E* p, int64_t j) {
    if constexpr (NT) return dev::ld_nt(reinterpret_cast<const Vec*>(p) + j);
    else return reinterpret_cast<const Vec*>(p)[j];
  }
  __device__ static void st(E* p, int64_t j, const Vec& v) {
    if constexpr (NT) dev::st_nt(reinterpret_cast<Vec*>(p) + j, v);
    else reinterpret_cast<Vec*>(p)[j] = v;
  }
};

// ---------------------------------------------------------------- BS1 copy

template <class T, int V, bool NT = true>
struct CopyOp : Base<T, V, NT> {
  using B = Base<T, V, NT>;
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

template <class T, int V, bool NT = true>
struct AxpyOp : Base<T, V, NT> {
  using B = Base<T, V, NT>;
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

template <class T, int V, bool W, bool NT = true>
struct NormOp : Base<T, V, NT> {
  using B = Base<T, V, NT>;
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

template <class T, int V, bool NT = true>
struct DotOp : Base<T, V, NT> {
  using B = Base<T, V, NT>;
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

template <class T, int V, bool W, bool NT = true>
struct CgOp : Base<T, V, NT> {
  using B = Base<T, V, NT>;
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
  sp.order = 0;
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

inline int grid_for(const Span& sp, int unroll, int cap, int block = kBlock) {
  const int64_t per = static_cast<int64_t>(block) * unroll;
  int64_t g = (sp.nvec + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

}  // namespace ops
}  // namespace bs
