// Conjugate gradients (Algorithm 1) built from the streaming operations, on
// the 7-point finite-difference operator (kernels in bs_stencil.h) and on
// the assembled Helmholtz operator of the spectral elements (bs_elem.hip),
// and mixed-precision iterative refinement around the former.
//
// One CG iteration runs on the device without returning to the host.
// Binary64 (five launches):
//   Ap = A p with the partial sums of p.Ap               (operator + BS4)
//   alpha = r.r / p.Ap                                   (1 workgroup)
//   x += alpha p, r -= alpha Ap, partial sums of r.r     (BS5)
//   beta = r'.r' / r.r, convergence test                 (1 workgroup)
//   p = r + beta p                                       (BS2)
// Binary32 and bfloat16 storage (two launches): the direction update is
// folded into the next operator application -- that kernel forms beta and
// the convergence test at its head from the update's partial sums, reads r
// and the old p, forms the new p with the same rounded operations the AXPY
// uses, writes it to a second buffer (p alternates between two buffers) and
// applies the operator to it -- and the update kernel forms alpha at its head
// from the operator's partial sums; the first iteration runs with beta = 0
// on p = r.  Every workgroup of such a kernel adds all the pairs itself, in
// one fixed order, so the update's grid stays small (kUpdateBlocks).  In
// binary64 the four vectors of the fused kernel outgrow the 256 MB
// last-level cache on the benchmark grid and its halo re-reads cost more than
// the separate AXPY, and the streaming kernels run fastest on full grids,
// whose pairs are too many to add at every workgroup's head: binary64 keeps
// the one-workgroup scalar kernels.
//
// The scalars live in a device-side state; once it says done, the remaining
// kernels of a batch return at once.  Batches of 16, 8, 4 or 2 iterations
// are captured into HIP graphs and replayed; the host reads the state after
// each group of batches and sizes the next group from the rate at which r.r
// has fallen (struct Batches).
//
// Iterative refinement (binary64 outer loop, inner CG in binary32 or
// bfloat16 storage with binary32 arithmetic): r = b - A x and ||r|| in
// binary64; inner CG on A d = r/||r|| to a relative residual theta (or
// max_inner iterations); x += ||r|| d in binary64; stop when the true
// relative residual ||b - A x|| / ||b|| <= tol.  theta is inner_tol, or the
// looser 0.5 tol ||b|| / ||r|| when that already meets the outer target, so
// the last refinement step is not solved further than needed.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>

#include "bs_stencil.h"
#include "bs_stream_ops.h"

namespace bs {
namespace {

using namespace ops;
using stencil::cg_alpha;
using stencil::cg_beta;
using stencil::CgLink;
using stencil::CgState;
using stencil::Op7;
using stencil::store_partial;

// Workgroups of the update kernel when the next kernel forms beta at its
// head (grid-stride): every workgroup of that kernel adds their partial
// sums, so they stay few.
constexpr int kUpdateBlocks = 1024;

// Size of the last-level cache (MALL) of the device the solver is built for.
constexpr double kLastLevelCache = 256.0 * 1024 * 1024;

// Storage types whose CG folds the direction update into the operator.
template <class T>
constexpr bool kFuseDirection = !std::is_same<T, double>::value;

inline unsigned int blocks_for(int64_t n) { return static_cast<unsigned int>((n + kBlock - 1) / kBlock); }

template <class T> struct DtypeOf;
template <> struct DtypeOf<double> { static constexpr bs_dtype v = BS_F64; };
template <> struct DtypeOf<float> { static constexpr bs_dtype v = BS_F32; };
template <> struct DtypeOf<dev::bf16> { static constexpr bs_dtype v = BS_BF16; };
template <class T>
constexpr bs_dtype dtype_of() {
  return DtypeOf<T>::v;
}

template <class T>
bs_status launch_stencil(int64_t m, double shift, const void* x, void* y, hipStream_t st) {
  using E = typename Storage<T>::E;
  int device = 0;
  if (bs_status s = check_hip(hipGetDevice(&device), "bs_stencil7")) return s;
  Op7<T, false, false> op;
  if (!op.prepare(m, device)) return fail(BS_ERR_INVALID_ARG, "bs_stencil7: grid side %lld is too large", static_cast<long long>(m));
  op.enqueue(st, shift, static_cast<const E*>(x), nullptr, nullptr, static_cast<E*>(y), nullptr, nullptr);
  return check_launch("bs_stencil7");
}

// ---------------------------------------------------------------- scalar steps

__global__ void k_cg_init(CgState* st, const double* rr, double stop_rr, int32_t max_iters) {
  if (threadIdx.x == 0) {
    st->rr_slot[0] = st->rr_slot[1] = st->rr = st->rr0 = *rr;
    st->stop_rr = stop_rr;
    st->iters = 0;
    st->max_iters = max_iters;
    st->fresh = 1;
    st->done = (*rr <= stop_rr || max_iters <= 0) ? 1 : 0;
    st->alpha = st->beta = st->pAp = 0.0;
  }
}

// Start of the inner solve of a refinement step, on the device: scal[2] is
// r.r of the binary64 residual, scal[0] rl.rl of its rounded direction.
// The inner tolerance theta = max(inner_tol, 0.5 sqrt(stop / r.r)) (the last
// step need not go below what the outer target asks for); the run is done
// at once when the outer residual already meets stop.
__global__ void k_ir_init(CgState* st, const double* scal, double stop, double inner_tol, int32_t max_inner) {
  if (threadIdx.x == 0) {
    const double rr = scal[2], rr0 = scal[0];
    const double theta = fmax(inner_tol, 0.5 * sqrt(stop / rr));
    const double stop_rr = theta * theta * rr0;
    st->rr_slot[0] = st->rr_slot[1] = st->rr = st->rr0 = rr0;
    st->outer_rr = rr;
    st->stop_rr = stop_rr;
    st->iters = 0;
    st->max_iters = max_inner;
    st->fresh = 1;
    st->done = (rr <= stop || rr0 <= stop_rr || max_inner <= 0) ? 1 : 0;
    st->alpha = st->beta = st->pAp = 0.0;
  }
}

// Algorithm 1 step 7 as a kernel of its own (one workgroup), for the
// binary64 engine: p.Ap from the operator's partial sums, alpha = r.r / p.Ap.
__global__ __launch_bounds__(kFinishBlock) void k_after_pAp(const double* __restrict__ partials, int G, CgState* st,
                                                             int slot) {
  if (st->done) return;
  DW<double> a{0.0, 0.0};
  for (int i = threadIdx.x; i < G; i += kFinishBlock) a = dev::dw_add(a, DW<double>{partials[2 * i], partials[2 * i + 1]});
  a = dev::block_reduce<kFinishBlock>(a);
  if (threadIdx.x == 0) {
    const double pAp = a.s + a.c;
    st->pAp = pAp;
    if (pAp > 0.0) {
      st->alpha = st->rr_slot[slot] / pAp;
      st->iters += 1;
    } else {
      st->done = 2;  // A is not positive definite on p (or p vanished)
    }
  }
}

// Algorithm 1 step 10 and the stopping test as a kernel of its own (one
// workgroup), for the binary64 engine: r'.r' from the update's partial
// sums, beta = r'.r' / r.r into the slot of the next iteration.
__global__ __launch_bounds__(kFinishBlock) void k_after_update(const double* __restrict__ partials, int G,
                                                                CgState* st, int slot) {
  if (st->done) return;
  DW<double> a{0.0, 0.0};
  for (int i = threadIdx.x; i < G; i += kFinishBlock) a = dev::dw_add(a, DW<double>{partials[2 * i], partials[2 * i + 1]});
  a = dev::block_reduce<kFinishBlock>(a);
  if (threadIdx.x == 0) {
    const double rr_new = a.s + a.c;
    st->beta = rr_new / st->rr_slot[slot ^ 1];
    st->rr_slot[slot] = rr_new;
    st->rr = rr_new;
    st->fresh = 0;
    if (!__builtin_isfinite(rr_new))
      st->done = 2;  // overflow or NaN: further iterations cannot recover
    else if (rr_new <= st->stop_rr || st->iters >= st->max_iters)
      st->done = 1;
  }
}

// x += alpha p, r -= alpha Ap and the partial sums of r.r.  With HEAD, alpha
// = r.r / p.Ap is formed at the head from the operator's partial sums;
// otherwise it is read from the state (k_after_pAp).
template <class T, int V, int U, bool HEAD, bool NT = true>
__global__ __launch_bounds__(kBlock) void k_cg_step(CgState* st, CgLink op_sums, typename Storage<T>::E* __restrict__ x,
                                                    const typename Storage<T>::E* __restrict__ p,
                                                    typename Storage<T>::E* __restrict__ r,
                                                    const typename Storage<T>::E* __restrict__ Ap, Span sp,
                                                    double* partials) {
  using C = typename Storage<T>::C;
  double alpha = 0.0;
  if constexpr (HEAD) {
    if (!cg_alpha(st, op_sums, &alpha)) return;
  } else {
    if (st->done) return;
    alpha = st->alpha;
  }
  CgOp<T, V, false, NT> op{{}, static_cast<C>(alpha), x, p, r, Ap, nullptr, sp.head, DW<C>{C(0), C(0)}};
  stream_loop<U>(op, sp);
  store_partial(DW<double>{static_cast<double>(op.acc.s), static_cast<double>(op.acc.c)}, partials);
}

// p = r + beta p.  With HEAD, beta = r'.r' / r.r and the stopping test are
// formed at the head from the update's partial sums; otherwise beta is read
// from the state (k_after_update).
template <class T, int V, int U, bool HEAD, bool NT = true>
__global__ __launch_bounds__(kBlock) void k_direction(CgState* st, CgLink upd_sums,
                                                      const typename Storage<T>::E* __restrict__ r,
                                                      typename Storage<T>::E* __restrict__ p, Span sp) {
  using C = typename Storage<T>::C;
  double beta = 0.0;
  if constexpr (HEAD) {
    if (!cg_beta(st, upd_sums, &beta)) return;
  } else {
    if (st->done) return;
    beta = st->beta;
  }
  AxpyOp<T, V, NT> op{{}, C(1), static_cast<C>(beta), r, p, sp.head};
  stream_loop<U>(op, sp);
}

// ---------------------------------------------------------------- precision changes

// binary64 -> binary32 rounded to odd: truncate, and set the last bit when
// the truncation was inexact.  Binary32 keeps 16 more significand bits than
// bfloat16, so rounding this value to nearest-even bfloat16 gives the
// binary64 value rounded once to nearest-even bfloat16 (Boldo and
// Melquiond, "Emulation of FMA and correctly rounded sums: proved
// algorithms using rounding to odd", IEEE Trans. Computers 2008).
__device__ __forceinline__ float to_f32_odd(double v) {
  const float t = __double2float_rz(v);
  if (static_cast<double>(t) == v || v != v) return t;
  return __uint_as_float(__float_as_uint(t) | 1u);
}

template <class T>
__device__ __forceinline__ typename Storage<T>::E round_once(double v) {
  if constexpr (std::is_same<T, dev::bf16>::value) {
    return Storage<T>::store(to_f32_odd(v));
  } else {
    return Storage<T>::store(static_cast<typename Storage<T>::C>(v));
  }
}

// Start of a refinement step: s = 1 / sqrt(*rr) (the binary64 residual's
// norm, read on the device), rl = r s rounded once to the storage type (to
// nearest, ties to even), p = rl, d = 0, and the partial sums of rl.rl over
// the stored values (binary32 arithmetic, compensated, as the norm of BS3).
template <class T>
__global__ __launch_bounds__(kBlock) void k_ir_prepare(const double* __restrict__ r, const double* __restrict__ rr,
                                                       int64_t n, typename Storage<T>::E* __restrict__ rl,
                                                       typename Storage<T>::E* __restrict__ p,
                                                       typename Storage<T>::E* __restrict__ d, double* partials) {
  using S = Storage<T>;
  using C = typename S::C;
  using E = typename S::E;
  const double s = 1.0 / sqrt(*rr);
  DW<C> acc{C(0), C(0)};
  const int64_t step = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += step) {
    const E e = round_once<T>(r[i] * s);
    rl[i] = e;
    p[i] = e;
    d[i] = E{};
    const C v = S::load(e);
    dev::dw_acc(acc, v * v);
  }
  store_partial(DW<double>{static_cast<double>(acc.s), static_cast<double>(acc.c)}, partials);
}

// x = x + sqrt(*rr) d  (binary64 x, narrow d; the refinement's correction)
template <class T>
__global__ __launch_bounds__(kBlock) void k_add_scaled(double* __restrict__ x, const double* __restrict__ rr,
                                                       const typename Storage<T>::E* __restrict__ d, int64_t n) {
  const double s = sqrt(*rr);
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) x[i] = x[i] + s * static_cast<double>(Storage<T>::load(d[i]));
}

// Tail of the binary64 residual: r = b - r (r holding A x on entry), rounded
// as BS2 rounds fl(1 b + (-1) r), and the compensated partial sums of r.r.
template <int V>
struct ResidualOp : ops::Base<double, V> {
  using B = ops::Base<double, V>;
  using Vec = typename B::Vec;
  struct Regs {
    Vec b, r;
  };
  const double* b;
  double* r;
  int32_t head;
  DW<double> acc;
  __device__ double one(double be, double re) {
    const double v = be - re;
    dev::dw_acc(acc, v * v);
    return v;
  }
  __device__ void load(Regs& g, int64_t j) const {
    g.b = B::ld(b + head, j);
    g.r = B::ld(r + head, j);
  }
  __device__ void apply(Regs& g, int64_t j) {
#pragma unroll
    for (int k = 0; k < V; ++k) ops::vset(g.r, k, one(ops::vget<Vec, double>(g.b, k), ops::vget<Vec, double>(g.r, k)));
    B::st(r + head, j, g.r);
  }
  __device__ void scalar(int64_t e) { r[e] = one(b[e], r[e]); }
};

template <int V>
__global__ __launch_bounds__(kBlock) void k_residual_tail(const double* __restrict__ b, double* __restrict__ r, Span sp,
                                                          double* partials) {
  ResidualOp<V> op{{}, b, r, sp.head, DW<double>{0.0, 0.0}};
  stream_loop<4>(op, sp);
  store_partial(DW<double>{op.acc.s, op.acc.c}, partials);
}

// *out = the G compensated pairs added in order (one workgroup).
__global__ __launch_bounds__(kFinishBlock) void k_sum_pairs(const double* __restrict__ partials, int G,
                                                             double* __restrict__ out) {
  DW<double> a{0.0, 0.0};
  for (int i = threadIdx.x; i < G; i += kFinishBlock) a = dev::dw_add(a, DW<double>{partials[2 * i], partials[2 * i + 1]});
  a = dev::block_reduce<kFinishBlock>(a);
  if (threadIdx.x == 0) *out = a.s + a.c;
}

// ---------------------------------------------------------------- host-side CG engine

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

// Captured batches of CG iterations, 16, 8, 4 and 2 long (even, so that
// the fused forms' direction is back in p after every batch).  A run starts
// with a batch of 16; after each read-back of the state the host launches
// at most 16 more, fewer when the mean rate at which r.r has fallen so far
// says the run ends sooner, so that few iterations are launched after the
// one that converges (each of those still costs a launch whose kernels
// return at their head).  Larger steps from an early rate misjudge: r.r
// need not fall steadily.
struct Batches {
  static constexpr int kCount = 4;
  static constexpr int kSize[kCount] = {16, 8, 4, 2};
  hipGraphExec_t exec[kCount] = {};

  ~Batches() {
    for (hipGraphExec_t e : exec)
      if (e) (void)hipGraphExecDestroy(e);
  }

  // Capture each size; a size the runtime cannot capture runs eagerly.
  template <class F>
  bs_status capture(hipStream_t st, F&& enqueue) {
    for (int w = 0; w < kCount; ++w) {
      hipGraph_t graph = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      bs_status s = BS_OK;
      for (int i = 0; i < kSize[w] && !s; ++i) s = enqueue(i & 1);
      const hipError_t e1 = hipStreamEndCapture(st, &graph);
      if (s) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
      }
      if (e1 != hipSuccess || !graph) {
        (void)hipGetLastError();
        continue;
      }
      const hipError_t e2 = hipGraphInstantiate(&exec[w], graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e2 != hipSuccess) {
        exec[w] = nullptr;
        (void)hipGetLastError();
      }
    }
    return BS_OK;
  }

  template <class F>
  bs_status launch(int w, hipStream_t st, F&& enqueue) {
    if (exec[w]) return check_hip(hipGraphLaunch(exec[w], st), "cg graph launch");
    bs_status s = BS_OK;
    for (int i = 0; i < kSize[w] && !s; ++i) s = enqueue(i & 1);
    return s ? s : check_launch("cg");
  }

  // Iterations to launch next: r.r fell from rr0 to rr over iters
  // iterations; at that mean rate, with a margin, until stop_rr.  (r.r
  // need not fall monotonically, and a read-back costs about as much as
  // five idle iterations, so the margin is generous.)
  static int64_t next_iterations(const CgState& c) {
    int64_t k = kSize[0];
    if (c.iters > 0 && c.rr > 0.0 && c.rr < c.rr0 && c.stop_rr > 0.0 && c.rr > c.stop_rr) {
      const double need = std::log(c.stop_rr / c.rr) / (std::log(c.rr / c.rr0) / c.iters);
      k = need < 4096.0 ? static_cast<int64_t>(std::ceil(need * 1.3)) + 4 : 4096;
    }
    return k;
  }

  // Launch at least k iterations (at most the state's limit): whole batches
  // of 16, the rest rounded up to one smaller batch (each graph launch adds
  // a gap of its own).
  template <class F>
  bs_status launch_at_least(int64_t k, const CgState* c, hipStream_t st, F&& enqueue) {
    if (c) {
      const int64_t left = static_cast<int64_t>(c->max_iters) - c->iters;
      if (k > left) k = left;
    }
    if (k < 1) k = 1;
    bs_status s = BS_OK;
    for (; k >= kSize[0] && !s; k -= kSize[0]) s = launch(0, st, enqueue);
    if (k > 0 && !s) {
      int w = kCount - 1;
      while (w > 0 && kSize[w] < k) --w;
      s = launch(w, st, enqueue);
    }
    return s;
  }

  // Iterate until the state reports done, starting with at least `first`
  // iterations (a caller that knows how many the last run took passes that);
  // returns the final state in *out.
  template <class F>
  bs_status run(hipStream_t st, CgState* state, CgState* out, F&& enqueue, int64_t first = kSize[0]) {
    bs_status s = launch_at_least(first, nullptr, st, enqueue);
    while (!s) {
      s = check_hip(hipMemcpyAsync(out, state, sizeof(CgState), hipMemcpyDeviceToHost, st), "cg");
      if (!s) s = check_hip(hipStreamSynchronize(st), "cg");
      if (s || out->done) break;
      const int64_t k = next_iterations(*out);
      // far from the end (at least 46 iterations to go at the mean rate), two
      // batches per read-back; near it, one
      const int64_t cap = k >= 4 * kSize[0] ? 2 * kSize[0] : kSize[0];
      s = launch_at_least(k < cap ? k : cap, out, st, enqueue);
    }
    return s;
  }
};

// Runs CG iterations in dtype T on vectors owned by the caller.  With the
// direction update folded into the operator, p alternates between p and p2:
// iteration i reads the old direction from one and writes the new one to
// the other.  Batches hold an even number of iterations, so the current
// direction is back in p after every batch.
template <class T>
struct CgEngine {
  using S = Storage<T>;
  using E = typename S::E;
  using C = typename S::C;
  static constexpr bool kFuse = kFuseDirection<T>;

  bs_ctx* ctx;
  hipStream_t st;
  int64_t m, n;
  double shift;
  E *x, *r, *p, *p2, *Ap;  // p2 is used only when the direction update is fused
  CgState* state;
  double* rr_dev;  // scratch scalar
  Span sp;
  Op7<T, true, kFuse> op;
  // the solve's vectors fit the 256 MB last-level cache: the streaming
  // steps use cached accesses (they find the operator's output there)
  bool cached = false;
  int g_upd = 1, g_dir = 1;
  Batches batches;

  // The operator's partial sums (p.Ap) go to the first kMaxReduceBlocks
  // pairs of the context's buffer, the update's (r.r) to the next ones.
  double* op_partials() const { return ctx->partials; }
  double* upd_partials() const { return ctx->partials + 2 * static_cast<size_t>(kMaxReduceBlocks); }

  // Binary32 and bfloat16 (direction folded into the operator): two
  // launches, the scalars formed at the heads of the kernels that use them.
  // Binary64: the operator, alpha (one workgroup), the update, beta (one
  // workgroup) and the direction, each streaming kernel on its full grid.
  void enqueue_iteration(int parity) {
    E* p_old = (kFuse && parity) ? p2 : p;
    E* p_cur = kFuse ? (parity ? p : p2) : p;
    const CgLink from_update{upd_partials(), g_upd, parity};  // the direction of this iteration
    const CgLink from_op{op_partials(), static_cast<int32_t>(op.blocks), parity};
    op.enqueue(st, shift, p_old, r, p_cur, Ap, op_partials(), state, from_update);
    if constexpr (kFuse) {
      if (sp.vwidth == 1)
        hipLaunchKernelGGL((k_cg_step<T, 1, 4, true>), dim3(g_upd), dim3(kBlock), 0, st, state, from_op, x, p_cur, r,
                           Ap, sp, upd_partials());
      else if (cached)
        hipLaunchKernelGGL((k_cg_step<T, S::V, 4, true, false>), dim3(g_upd), dim3(kBlock), 0, st, state, from_op, x,
                           p_cur, r, Ap, sp, upd_partials());
      else
        hipLaunchKernelGGL((k_cg_step<T, S::V, 4, true>), dim3(g_upd), dim3(kBlock), 0, st, state, from_op, x, p_cur,
                           r, Ap, sp, upd_partials());
    } else {
      hipLaunchKernelGGL(k_after_pAp, dim3(1), dim3(kFinishBlock), 0, st, op_partials(), static_cast<int>(op.blocks),
                         state, parity);
      if (sp.vwidth == 1)
        hipLaunchKernelGGL((k_cg_step<T, 1, 4, false>), dim3(g_upd), dim3(kBlock), 0, st, state, from_op, x, p_cur, r,
                           Ap, sp, upd_partials());
      else if (cached)
        hipLaunchKernelGGL((k_cg_step<T, S::V, 4, false, false>), dim3(g_upd), dim3(kBlock), 0, st, state, from_op, x,
                           p_cur, r, Ap, sp, upd_partials());
      else
        hipLaunchKernelGGL((k_cg_step<T, S::V, 4, false>), dim3(g_upd), dim3(kBlock), 0, st, state, from_op, x, p_cur,
                           r, Ap, sp, upd_partials());
      hipLaunchKernelGGL(k_after_update, dim3(1), dim3(kFinishBlock), 0, st, upd_partials(), g_upd, state, parity ^ 1);
      const CgLink none{nullptr, 0, parity ^ 1};
      if (sp.vwidth == 1)
        hipLaunchKernelGGL((k_direction<T, 1, 1, false>), dim3(g_dir), dim3(kBlock), 0, st, state, none, r, p, sp);
      else if (cached)
        hipLaunchKernelGGL((k_direction<T, S::V, 1, false, false>), dim3(g_dir), dim3(kBlock), 0, st, state, none, r,
                           p, sp);
      else
        hipLaunchKernelGGL((k_direction<T, S::V, 1, false>), dim3(g_dir), dim3(kBlock), 0, st, state, none, r, p, sp);
    }
  }

  bs_status prepare() {
    sp = make_span<T>(n, {x, r, p, p2, Ap});
    cached = static_cast<double>(kFuse ? 5 : 4) * n * sizeof(E) <= kLastLevelCache;
    if (!op.prepare(m, ctx->device))
      return fail(BS_ERR_INVALID_ARG, "cg: grid side %lld is too large", static_cast<long long>(m));
    // with the scalars formed at the kernels' heads every workgroup reads all
    // the previous kernel's pairs, so those grids stay small
    g_upd = grid_for(sp, 4, kFuse ? kUpdateBlocks : kMaxReduceBlocks);
    g_dir = grid_for(sp, 1, 1 << 30);
    return batches.capture(st, [this](int parity) {
      enqueue_iteration(parity);
      return BS_OK;
    });
  }

  // The same for a state some earlier kernel has initialised.
  bs_status run_initialised(CgState* out) {
    return batches.run(st, state, out, [this](int parity) {
      enqueue_iteration(parity);
      return BS_OK;
    });
  }

  // Iterate until the state reports done, launching at least `first`
  // iterations before the first read-back; returns the final state.
  bs_status run(double stop_rr, int32_t max_iters, CgState* out, int64_t first = Batches::kSize[0]) {
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, st, state, rr_dev, stop_rr, max_iters);
    if (bs_status s = check_launch("cg")) return s;
    return batches.run(
        st, state, out,
        [this](int parity) {
          enqueue_iteration(parity);
          return BS_OK;
        },
        first);
  }
};

// CG on y_G = Z^T A_L Z x_G, the assembled Helmholtz operator (Section 2,
// eqs. global_system, assembled_stiff, assembled_mass), binary64, six
// launches per iteration: the local operator applied to p (scatter fused
// into its load) with the partial sums of p.Ap formed there as the sum over
// elements of u_e . A^e u_e, the gather of the local results, alpha (one
// workgroup), the update with the partial sums of r.r (BS5), beta (one
// workgroup) and the direction (BS2).  The scalars stay on the device, and
// batches of iterations run as one captured graph.
struct HelmEngine {
  bs_ctx* ctx;
  hipStream_t st;
  const bs_elem* el;
  const bs_gs* gs;
  const double* geo;
  double lambda;
  int64_t n;
  double *x, *r, *p, *Ap, *yL;
  CgState* state;
  Span sp;
  int g_op = 1, g_upd = 1, g_dir = 1;
  Batches batches;

  double* op_partials() const { return ctx->partials; }
  double* upd_partials() const { return ctx->partials + 2 * static_cast<size_t>(kMaxReduceBlocks); }

  bs_status enqueue_iteration(int parity) {
    bs_status s = helm_apply_dot(ctx, el, gs, geo, lambda, p, yL, Ap, op_partials(), &state->done, st);
    if (s) return s;
    hipLaunchKernelGGL(k_after_pAp, dim3(1), dim3(kFinishBlock), 0, st, op_partials(), g_op, state, parity);
    const CgLink none{nullptr, 0, parity};
    if (sp.vwidth == 1)
      hipLaunchKernelGGL((k_cg_step<double, 1, 4, false>), dim3(g_upd), dim3(kBlock), 0, st, state, none, x, p, r, Ap,
                         sp, upd_partials());
    else
      hipLaunchKernelGGL((k_cg_step<double, 2, 4, false>), dim3(g_upd), dim3(kBlock), 0, st, state, none, x, p, r, Ap,
                         sp, upd_partials());
    hipLaunchKernelGGL(k_after_update, dim3(1), dim3(kFinishBlock), 0, st, upd_partials(), g_upd, state, parity ^ 1);
    if (sp.vwidth == 1)
      hipLaunchKernelGGL((k_direction<double, 1, 1, false>), dim3(g_dir), dim3(kBlock), 0, st, state, none, r, p, sp);
    else
      hipLaunchKernelGGL((k_direction<double, 2, 1, false>), dim3(g_dir), dim3(kBlock), 0, st, state, none, r, p, sp);
    return check_launch("bs_helmholtz_cg_solve");
  }

  bs_status prepare() {
    sp = make_span<double>(n, {x, r, p, Ap});
    g_op = helm_dot_blocks(gs->n_local / ((el->N + 1) * (el->N + 1) * (el->N + 1)));
    g_upd = grid_for(sp, 4, kMaxReduceBlocks);
    g_dir = grid_for(sp, 1, 1 << 30);
    return batches.capture(st, [this](int parity) { return enqueue_iteration(parity); });
  }

  bs_status run(const double* rr_dev, double stop_rr, int32_t max_iters, CgState* out) {
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, st, state, rr_dev, stop_rr, max_iters);
    if (bs_status s = check_launch("bs_helmholtz_cg_solve")) return s;
    return batches.run(st, state, out, [this](int parity) { return enqueue_iteration(parity); });
  }
};

// Solver workspace: one allocation, carved into aligned pieces.
struct Workspace {
  DevMem mem;
  char* cur = nullptr;
  size_t left = 0;
  bool alloc(size_t bytes) {
    if (hipMalloc(&mem.p, bytes) != hipSuccess) return false;
    cur = static_cast<char*>(mem.p);
    left = bytes;
    return true;
  }
  template <class X>
  X* take(int64_t count) {
    const size_t bytes = (static_cast<size_t>(count) * sizeof(X) + 255) & ~static_cast<size_t>(255);
    X* q = reinterpret_cast<X*>(cur);
    cur += bytes;
    left -= bytes;
    return q;
  }
};

inline size_t padded(size_t bytes) { return (bytes + 255) & ~static_cast<size_t>(255); }

bs_status check_solver_args(const char* op, bs_ctx* ctx, int64_t m, const double* b, const double* x, double tol) {
  bs_status s;
  if ((s = check_ctx(ctx, op))) return s;
  if (m < 1 || m > 4096 || m * m * m >= (int64_t(1) << 31))
    return fail(BS_ERR_INVALID_ARG, "%s: grid size m must lie in [1, 1290]", op);
  if (!b || !x) return fail(BS_ERR_INVALID_ARG, "%s: b or x is NULL", op);
  if (!aligned_to(b, 8) || !aligned_to(x, 8)) return fail(BS_ERR_INVALID_ARG, "%s: misaligned vector", op);
  if (!(tol > 0.0)) return fail(BS_ERR_INVALID_ARG, "%s: tolerance must be positive", op);
  return BS_OK;
}

// r = b - A x (binary64) with r.r left in *rr_dev; nothing is read back.
constexpr int kTailBlocks = 2048;  // workgroups of the residual tail and the step preparation
bs_status residual_dev(bs_ctx* ctx, int64_t m, double shift, const double* b, const double* x, double* r,
                       double* rr_dev, hipStream_t st) {
  const int64_t n = m * m * m;
  bs_status s = launch_stencil<double>(m, shift, x, r, st);
  if (s) return s;
  Span sp = make_span<double>(n, {b, r});
  const int g = grid_for(sp, 4, kTailBlocks);
  if (sp.vwidth == 1)
    hipLaunchKernelGGL(k_residual_tail<1>, dim3(g), dim3(kBlock), 0, st, b, r, sp, ctx->partials);
  else
    hipLaunchKernelGGL(k_residual_tail<2>, dim3(g), dim3(kBlock), 0, st, b, r, sp, ctx->partials);
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(kFinishBlock), 0, st, ctx->partials, g, rr_dev);
  return check_launch("residual");
}

// The same, returning r.r on the host.
bs_status residual(bs_ctx* ctx, int64_t m, double shift, const double* b, const double* x, double* r, double* rr_dev,
                   double* rr_host, hipStream_t st) {
  bs_status s = residual_dev(ctx, m, shift, b, x, r, rr_dev, st);
  if (!s) s = check_hip(hipMemcpyAsync(rr_host, rr_dev, sizeof(double), hipMemcpyDeviceToHost, st), "residual");
  if (!s) s = check_hip(hipStreamSynchronize(st), "residual");
  return s;
}

struct OwnStream {
  hipStream_t s = nullptr;
  ~OwnStream() {
    if (s) (void)hipStreamDestroy(s);
  }
};

template <class T>
bs_status ir_solve(bs_ctx* ctx, int64_t m, double shift, const double* b, double* x, double tol, double inner_tol,
                   int64_t max_inner, int64_t max_outer, bs_cg_result* res, hipStream_t caller) {
  using E = typename Storage<T>::E;
  const char* op = "bs_cg_ir_solve";
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = m * m * m;
  bs_status s = check_hip(hipStreamSynchronize(caller), op);
  if (s) return s;
  OwnStream own;
  if ((s = check_hip(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking), op))) return s;
  hipStream_t st = own.s;
  Workspace ws;
  const int vecs = kFuseDirection<T> ? 5 : 4;  // rl, d, p, Ap (+ p2)
  const size_t bytes = padded(n * 8) + vecs * padded(n * sizeof(E)) + 2 * padded(sizeof(CgState)) + 1024;
  if (!ws.alloc(bytes)) return fail(BS_ERR_ALLOC, "%s: cannot allocate %zu bytes of workspace", op, bytes);
  double* r64 = ws.take<double>(n);
  E* rl = ws.take<E>(n);
  E* d = ws.take<E>(n);
  E* p = ws.take<E>(n);
  E* p2 = kFuseDirection<T> ? ws.take<E>(n) : nullptr;
  E* Ap = ws.take<E>(n);
  CgState* state = ws.take<CgState>(1);
  double* scal = ws.take<double>(8);

  CgEngine<T> eng{ctx, st, m, n, shift, d, rl, p, p2, Ap, state, scal};
  if ((s = eng.prepare())) return s;

  double bb = 0.0;
  if ((s = bs_norm(ctx, BS_F64, n, b, nullptr, scal + 1, st))) return s;
  if ((s = check_hip(hipMemcpyAsync(&bb, scal + 1, 8, hipMemcpyDeviceToHost, st), op))) return s;
  if ((s = check_hip(hipStreamSynchronize(st), op))) return s;
  const double stop = tol * tol * bb;
  double hist[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
  int64_t outer = 0, inner = 0;
  double rr = 0.0;
  bool stagnated = false;
  // scal[2] = r.r of the binary64 residual, scal[0] = rl.rl of its rounded
  // direction; one read-back per refinement step
  if ((s = residual_dev(ctx, m, shift, b, x, r64, scal + 2, st))) return s;
  const unsigned int gp = blocks_for(n) < static_cast<unsigned int>(kTailBlocks) ? blocks_for(n) : kTailBlocks;
  while (true) {
    hipLaunchKernelGGL((k_ir_prepare<T>), dim3(gp), dim3(kBlock), 0, st, r64, scal + 2, n, rl, p, d, ctx->partials);
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(kFinishBlock), 0, st, ctx->partials, static_cast<int>(gp), scal);
    if ((s = check_launch(op))) return s;
    if (outer >= max_outer) {
      if ((s = check_hip(hipMemcpyAsync(&rr, scal + 2, sizeof(double), hipMemcpyDeviceToHost, st), op))) return s;
      if ((s = check_hip(hipStreamSynchronize(st), op))) return s;
      break;
    }
    // the inner tolerance and the outer test are taken on the device, so
    // the inner iterations follow without a read-back; the host learns the
    // outer residual from the state after the run (a run that starts done
    // costs one batch of kernels that return at their head)
    hipLaunchKernelGGL(k_ir_init, dim3(1), dim3(64), 0, st, state, scal, stop, inner_tol,
                       static_cast<int32_t>(max_inner));
    if ((s = check_launch(op))) return s;
    CgState fin{};
    if ((s = eng.run_initialised(&fin))) return s;
    rr = fin.outer_rr;
    inner += fin.iters;
    if (rr <= stop) break;
    // outer residual must halve within three refinement steps
    if (outer >= 3 && std::sqrt(rr) > 0.5 * std::sqrt(hist[(outer - 3) % 4])) {
      stagnated = true;
      break;
    }
    hist[outer % 4] = rr;
    hipLaunchKernelGGL((k_add_scaled<T>), dim3(blocks_for(n)), dim3(kBlock), 0, st, x, scal + 2,
                       static_cast<const E*>(d), n);
    if ((s = check_launch(op))) return s;
    if ((s = residual_dev(ctx, m, shift, b, x, r64, scal + 2, st))) return s;
    ++outer;
  }
  if ((s = check_hip(hipStreamSynchronize(st), op))) return s;
  if (res) {
    res->iterations = inner;
    res->outer_iterations = outer;
    res->restarts = 0;
    res->rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (stagnated || rr > stop)
    return fail(BS_ERR_NO_CONVERGENCE, "%s: relative residual %.3e after %lld refinement steps", op,
                bb > 0.0 ? std::sqrt(rr / bb) : 0.0, static_cast<long long>(outer));
  return BS_OK;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" bs_status bs_stencil7(bs_ctx* ctx, bs_dtype dtype, int64_t m, double shift, const void* x, void* y,
                                 void* stream) {
  bs_status s;
  const char* op = "bs_stencil7";
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype))) return s;
  if (m < 0 || m > 46340 || (m > 0 && m * m * m >= (int64_t(1) << 40)))
    return fail(BS_ERR_INVALID_ARG, "%s: bad grid size %lld", op, static_cast<long long>(m));
  const int64_t n = m * m * m;
  if ((s = check_vec(op, "x", x, n, dtype)) || (s = check_vec(op, "y", y, n, dtype))) return s;
  const uintptr_t a = reinterpret_cast<uintptr_t>(x), b = reinterpret_cast<uintptr_t>(y);
  const uintptr_t nb = static_cast<uintptr_t>(n) * dtype_size(dtype);
  if (n && a < b + nb && b < a + nb) return fail(BS_ERR_INVALID_ARG, "%s: y overlaps x", op);
  if (n == 0) return BS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case BS_F64: return launch_stencil<double>(m, shift, x, y, st);
    case BS_F32: return launch_stencil<float>(m, shift, x, y, st);
    case BS_BF16: return launch_stencil<dev::bf16>(m, shift, x, y, st);
  }
  return fail(BS_ERR_INVALID_ARG, "%s: unknown dtype", op);
}

extern "C" bs_status bs_cg_solve(bs_ctx* ctx, int64_t m, double shift, const double* d_b, double* d_x, double tol,
                                 int64_t max_iter, bs_cg_result* res, void* stream) {
  const char* op = "bs_cg_solve";
  bs_status s;
  if ((s = check_solver_args(op, ctx, m, d_b, d_x, tol))) return s;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = m * m * m;
  hipStream_t caller = static_cast<hipStream_t>(stream);
  if ((s = check_hip(hipStreamSynchronize(caller), op))) return s;
  OwnStream own;
  if ((s = check_hip(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking), op))) return s;
  hipStream_t st = own.s;
  Workspace ws;
  const size_t bytes = 3 * padded(n * 8) + padded(sizeof(CgState)) + 1024;
  if (!ws.alloc(bytes)) return fail(BS_ERR_ALLOC, "%s: cannot allocate %zu bytes of workspace", op, bytes);
  double* r = ws.take<double>(n);
  double* p = ws.take<double>(n);
  double* Ap = ws.take<double>(n);
  CgState* state = ws.take<CgState>(1);
  double* scal = ws.take<double>(8);
  CgEngine<double> eng{ctx, st, m, n, shift, d_x, r, p, nullptr, Ap, state, scal};
  if ((s = eng.prepare())) return s;
  double bb = 0.0;
  if ((s = bs_norm(ctx, BS_F64, n, d_b, nullptr, scal + 1, st))) return s;
  if ((s = check_hip(hipMemcpyAsync(&bb, scal + 1, 8, hipMemcpyDeviceToHost, st), op))) return s;
  if ((s = check_hip(hipStreamSynchronize(st), op))) return s;
  const double stop = tol * tol * bb;
  int64_t iters = 0, restarts = 0;
  double rr = 0.0;
  bool breakdown = false;
  while (true) {
    // (re)start from the true residual
    if ((s = residual(ctx, m, shift, d_b, d_x, r, scal, &rr, st))) return s;
    if (rr <= stop || iters >= max_iter || breakdown) break;
    if ((s = bs_copy(ctx, BS_F64, n, r, p, st))) return s;
    CgState fin{};
    const int64_t left = max_iter - iters;
    if ((s = eng.run(stop, static_cast<int32_t>(left < INT32_MAX ? left : INT32_MAX), &fin))) return s;
    iters += fin.iters;
    breakdown = fin.done == 2;
    ++restarts;
  }
  if (res) {
    res->iterations = iters;
    res->outer_iterations = 0;
    res->restarts = restarts > 0 ? restarts - 1 : 0;
    res->rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (rr > stop)
    return fail(BS_ERR_NO_CONVERGENCE, "%s: relative residual %.3e after %lld iterations", op,
                bb > 0.0 ? std::sqrt(rr / bb) : 0.0, static_cast<long long>(iters));
  return BS_OK;
}

extern "C" bs_status bs_cg_ir_solve(bs_ctx* ctx, bs_dtype inner, int64_t m, double shift, const double* d_b,
                                    double* d_x, double tol, double inner_tol, int64_t max_inner, int64_t max_outer,
                                    bs_cg_result* res, void* stream) {
  const char* op = "bs_cg_ir_solve";
  bs_status s;
  if ((s = check_solver_args(op, ctx, m, d_b, d_x, tol)) || (s = check_dtype(op, inner))) return s;
  if (!(inner_tol > 0.0 && inner_tol < 1.0)) return fail(BS_ERR_INVALID_ARG, "%s: inner_tol must lie in (0, 1)", op);
  if (max_inner < 1 || max_inner > INT32_MAX || max_outer < 0)
    return fail(BS_ERR_INVALID_ARG, "%s: bad iteration limits", op);
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (inner) {
    case BS_F64: return ir_solve<double>(ctx, m, shift, d_b, d_x, tol, inner_tol, max_inner, max_outer, res, st);
    case BS_F32: return ir_solve<float>(ctx, m, shift, d_b, d_x, tol, inner_tol, max_inner, max_outer, res, st);
    case BS_BF16: return ir_solve<dev::bf16>(ctx, m, shift, d_b, d_x, tol, inner_tol, max_inner, max_outer, res, st);
  }
  return fail(BS_ERR_INVALID_ARG, "%s: unknown dtype", op);
}

extern "C" bs_status bs_helmholtz_cg_solve(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* d_geo,
                                           double lambda, const double* d_b, double* d_x, double tol, int64_t max_iter,
                                           bs_cg_result* res, void* stream) {
  const char* op = "bs_helmholtz_cg_solve";
  bs_status s;
  if ((s = check_ctx(ctx, op))) return s;
  if (!el || !gs) return fail(BS_ERR_INVALID_ARG, "%s: element object or plan is NULL", op);
  if (el->device != ctx->device || gs->device != ctx->device)
    return fail(BS_ERR_INVALID_ARG, "%s: element object or plan on another device", op);
  if (el->N > 7) return fail(BS_ERR_UNSUPPORTED, "%s: the local operator is built for degrees N <= 7", op);
  const int64_t P = static_cast<int64_t>(el->N + 1) * (el->N + 1) * (el->N + 1);
  if (gs->n_local % P != 0) return fail(BS_ERR_INVALID_ARG, "%s: plan length is not a whole number of elements", op);
  const int64_t n = gs->n_global, n_elem = gs->n_local / P;
  if ((s = check_vec(op, "geo", d_geo, 7 * n_elem, BS_F64)) || (s = check_vec(op, "b", d_b, n, BS_F64)) ||
      (s = check_vec(op, "x", d_x, n, BS_F64)))
    return s;
  if (n > 0 && (!d_b || !d_x)) return fail(BS_ERR_INVALID_ARG, "%s: b or x is NULL", op);
  if (!(tol > 0.0)) return fail(BS_ERR_INVALID_ARG, "%s: tolerance must be positive", op);
  if (max_iter < 0) return fail(BS_ERR_INVALID_ARG, "%s: max_iter must be >= 0", op);
  const uintptr_t xa = reinterpret_cast<uintptr_t>(d_x), ba = reinterpret_cast<uintptr_t>(d_b);
  if (n > 0 && xa < ba + static_cast<uintptr_t>(n) * 8 && ba < xa + static_cast<uintptr_t>(n) * 8)
    return fail(BS_ERR_INVALID_ARG, "%s: x overlaps b", op);
  const auto t0 = std::chrono::steady_clock::now();
  if (n == 0) {
    if (res) *res = bs_cg_result{0, 0, 0, 0.0, 0.0};
    return BS_OK;
  }
  hipStream_t caller = static_cast<hipStream_t>(stream);
  if ((s = check_hip(hipStreamSynchronize(caller), op))) return s;
  OwnStream own;
  if ((s = check_hip(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking), op))) return s;
  hipStream_t st = own.s;
  Workspace ws;
  const size_t bytes = 3 * padded(n * 8) + padded(gs->n_local * 8) + padded(sizeof(CgState)) + 1024;
  if (!ws.alloc(bytes)) return fail(BS_ERR_ALLOC, "%s: cannot allocate %zu bytes of workspace", op, bytes);
  double* r = ws.take<double>(n);
  double* p = ws.take<double>(n);
  double* Ap = ws.take<double>(n);
  double* yL = ws.take<double>(gs->n_local);
  CgState* state = ws.take<CgState>(1);
  double* scal = ws.take<double>(8);
  HelmEngine eng{ctx, st, el, gs, d_geo, lambda, n, d_x, r, p, Ap, yL, state};
  if ((s = eng.prepare())) return s;
  double bb = 0.0;
  if ((s = bs_norm(ctx, BS_F64, n, d_b, nullptr, scal + 1, st))) return s;
  if ((s = check_hip(hipMemcpyAsync(&bb, scal + 1, 8, hipMemcpyDeviceToHost, st), op))) return s;
  if ((s = check_hip(hipStreamSynchronize(st), op))) return s;
  const double stop = tol * tol * bb;
  int64_t iters = 0, restarts = 0;
  double rr = 0.0;
  bool breakdown = false;
  while (true) {
    // (re)start from the true residual r = b - A x, in binary64
    if ((s = bs_helmholtz_apply(ctx, el, gs, d_geo, lambda, d_x, yL, r, st)) ||
        (s = bs_axpy(ctx, BS_F64, n, 1.0, d_b, -1.0, r, st)) || (s = bs_norm(ctx, BS_F64, n, r, nullptr, scal, st)))
      return s;
    if ((s = check_hip(hipMemcpyAsync(&rr, scal, 8, hipMemcpyDeviceToHost, st), op))) return s;
    if ((s = check_hip(hipStreamSynchronize(st), op))) return s;
    if (rr <= stop || iters >= max_iter || breakdown) break;
    if ((s = bs_copy(ctx, BS_F64, n, r, p, st))) return s;
    CgState fin{};
    const int64_t left = max_iter - iters;
    if ((s = eng.run(scal, stop, static_cast<int32_t>(left < INT32_MAX ? left : INT32_MAX), &fin))) return s;
    iters += fin.iters;
    breakdown = fin.done == 2;
    ++restarts;
  }
  if (res) {
    res->iterations = iters;
    res->outer_iterations = 0;
    res->restarts = restarts > 0 ? restarts - 1 : 0;
    res->rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (rr > stop)
    return fail(BS_ERR_NO_CONVERGENCE, "%s: relative residual %.3e after %lld iterations", op,
                bb > 0.0 ? std::sqrt(rr / bb) : 0.0, static_cast<long long>(iters));
  return BS_OK;
}
