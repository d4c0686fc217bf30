// Batched execution over many independent instances of uneven size.
//
// Every instance has global vectors x, y, p, r, Ap and local vectors xL, pL,
// wL, stored back to back in instance order, and a scatter map whose ids
// refer to its own global nodes.  The batch shifts each instance's ids by
// its global offset, which makes Z block-diagonal over the concatenation;
// the CSR of Z^T is then the single-instance plan of that map.
//
// One step applies, to every instance, the seven streaming operations once
// each and one CG iteration with A = Z^T Z:
//    1 y = x                           BS1
//    2 y = alpha x + beta y            BS2
//    3 norm = sum wL xL^2              BS3
//    4 dot = x . y                     BS4
//    5 x += alpha p, r -= alpha Ap     BS5, rr = r . r
//    6 xL = Z x, 8 pL = Z p            BS7
//    7 y = Z^T xL, 9 Ap = Z^T pL       BS6
//   10 pAp = p . Ap, a = rr / pAp      BS4
//   11 x += a p, r -= a Ap             BS5, rr2 = r . r
//   12 p = r + (rr2 / rr) p            BS2
// alpha and beta are shared; a and b = rr2 / rr belong to each instance.
//
// Work is cut into chunks of 2048 consecutive elements that never cross an
// instance.  A workgroup handles one chunk at a time (8 elements per
// thread); reductions leave one compensated pair per chunk, and an
// instance's value is the sum of its chunks' pairs in chunk order, formed by
// one wave.  The steps are grouped into eleven intervals separated by the
// data dependencies; the forms run the same interval code on the same
// chunks, so they give identical bits:
//   per instance  eleven launches per instance, each over its chunks;
//   per phase     eleven launches in all, each over every chunk.
// A per-phase step neither allocates nor synchronises, so a caller can
// capture it in a HIP graph.  The persistent form (one launch, intervals
// separated by grid barriers) is not offered: a grid barrier whose waiters
// poll with agent-scope acquire loads did not complete on gfx950, and the
// form returns BS_ERR_UNSUPPORTED until a barrier-free schedule replaces it.

#include <algorithm>
#include <vector>

#include "bs_device.h"
#include "bs_internal.h"

using bs::dev::DW;
using bs::dev::kWave;
using bs::dev::Storage;

namespace bs {
namespace {

constexpr int kPer = 8;                    // elements per thread in a chunk
constexpr int kChunk = kBlock * kPer;      // elements per chunk
constexpr int kIntervals = 11;
constexpr int kSlots = 8;                  // output doubles per instance
enum Slot { S_NORM = 0, S_DOT, S_RR, S_PAP, S_ALPHA, S_RR2, S_BETA };

template <class T> struct DtypeOf;
template <> struct DtypeOf<double> { static constexpr bs_dtype v = BS_F64; };
template <> struct DtypeOf<float> { static constexpr bs_dtype v = BS_F32; };
template <> struct DtypeOf<dev::bf16> { static constexpr bs_dtype v = BS_BF16; };

struct Chunk {
  int64_t start;  // first element (index into the concatenated vectors)
  int32_t len;    // 1 .. kChunk
  int32_t inst;
};

template <class T>
struct Args {
  using E = typename Storage<T>::E;
  using C = typename Storage<T>::C;
  E *x, *y, *p, *r, *Ap, *xL, *pL;
  const E* wL;
  const Chunk* cg;  // chunks of the global vectors
  const Chunk* cl;  // chunks of the local vectors
  int64_t g0, g1, l0, l1;  // chunk ranges to process
  int32_t i0, i1;          // instance range to finish
  const int64_t* fg;       // first global chunk of each instance [n_inst + 1]
  const int64_t* fl;       // first local chunk of each instance [n_inst + 1]
  const int32_t* map;      // scatter ids, shifted to the concatenated global vector
  const int32_t* rs;       // CSR of Z^T
  const int32_t* ci;
  double* part_a;          // compensated pairs, one per chunk
  double* part_b;
  double* out;             // [n_inst][kSlots]
  C alpha, beta;
};

// ---------------------------------------------------------------- chunk bodies

template <class T, class F>
__device__ __forceinline__ void each(const Chunk& ch, F f) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = threadIdx.x + kBlock * k;
    if (e < ch.len) f(ch.start + e);
  }
}

// One pair per chunk.  The trailing barrier lets a workgroup call this again
// for its next chunk: block_reduce's LDS slots are free once thread 0 has
// read them.
__device__ __forceinline__ void put_pair(double* part, int64_t c, DW<double> a) {
  a = dev::block_reduce<kBlock>(a);
  if (threadIdx.x == 0) {
    part[2 * c] = a.s;
    part[2 * c + 1] = a.c;
  }
  __syncthreads();
}

template <class C>
__device__ __forceinline__ DW<double> widen(DW<C> a) {
  return DW<double>{static_cast<double>(a.s), static_cast<double>(a.c)};
}

template <class T>
__device__ void ch_copy(const Args<T>& a, const Chunk& ch) {
  each<T>(ch, [&](int64_t e) { a.y[e] = a.x[e]; });
}

template <class T>
__device__ void ch_axpy(const Args<T>& a, const Chunk& ch) {
  using S = Storage<T>;
  each<T>(ch, [&](int64_t e) { a.y[e] = S::store(a.alpha * S::load(a.x[e]) + a.beta * S::load(a.y[e])); });
}

template <class T>
__device__ void ch_norm(const Args<T>& a, const Chunk& ch, int64_t c) {
  using S = Storage<T>;
  using C = typename S::C;
  DW<C> acc{C(0), C(0)};
  each<T>(ch, [&](int64_t e) {
    const C xk = S::load(a.xL[e]);
    dev::dw_acc(acc, S::load(a.wL[e]) * (xk * xk));
  });
  put_pair(a.part_a, c, widen(acc));
}

template <class T>
__device__ void ch_dot(const typename Storage<T>::E* u, const typename Storage<T>::E* v, double* part,
                       const Chunk& ch, int64_t c) {
  using S = Storage<T>;
  using C = typename S::C;
  DW<C> acc{C(0), C(0)};
  each<T>(ch, [&](int64_t e) { dev::dw_acc_prod(acc, S::load(u[e]), S::load(v[e])); });
  put_pair(part, c, widen(acc));
}

template <class T>
__device__ void ch_update(const Args<T>& a, typename Storage<T>::C alpha, double* part, const Chunk& ch, int64_t c) {
  using S = Storage<T>;
  using C = typename S::C;
  DW<C> acc{C(0), C(0)};
  each<T>(ch, [&](int64_t e) {
    a.x[e] = S::store(S::load(a.x[e]) + alpha * S::load(a.p[e]));
    const typename S::E rn = S::store(S::load(a.r[e]) - alpha * S::load(a.Ap[e]));
    a.r[e] = rn;
    const C rk = S::load(rn);
    dev::dw_acc_prod(acc, rk, rk);
  });
  put_pair(part, c, widen(acc));
}

template <class T>
__device__ void ch_scatter(const Args<T>& a, const typename Storage<T>::E* g, typename Storage<T>::E* l,
                           const Chunk& ch) {
  each<T>(ch, [&](int64_t e) { l[e] = g[a.map[e]]; });
}

// each row from +0.0, its local copies added in ascending local index
template <class T>
__device__ void ch_gather(const Args<T>& a, const typename Storage<T>::E* l, typename Storage<T>::E* g,
                          const Chunk& ch) {
  using S = Storage<T>;
  using C = typename S::C;
  each<T>(ch, [&](int64_t e) {
    C s = C(0);
    for (int32_t j = a.rs[e]; j < a.rs[e + 1]; ++j) s = s + S::load(l[a.ci[j]]);
    g[e] = S::store(s);
  });
}

template <class T>
__device__ void ch_direction(const Args<T>& a, const Chunk& ch) {
  using S = Storage<T>;
  using C = typename S::C;
  const C b = static_cast<C>(a.out[ch.inst * kSlots + S_BETA]);
  each<T>(ch, [&](int64_t e) { a.p[e] = S::store(C(1) * S::load(a.r[e]) + b * S::load(a.p[e])); });
}

// Sum of one instance's chunk pairs in chunk order, by one wave; every lane
// ends with the same value.
__device__ __forceinline__ double wave_sum(const double* part, int64_t c0, int64_t c1) {
  DW<double> acc{0.0, 0.0};
  for (int64_t c = c0 + threadIdx.x % kWave; c < c1; c += kWave)
    acc = dev::dw_add(acc, DW<double>{part[2 * c], part[2 * c + 1]});
  acc = dev::wave_reduce(acc);
  return acc.s + acc.c;
}

// ---------------------------------------------------------------- intervals

template <class T, class F>
__device__ __forceinline__ void over_chunks(const Chunk* table, int64_t c0, int64_t c1, F f) {
  for (int64_t c = c0 + blockIdx.x; c < c1; c += gridDim.x) f(table[c], c);
}

template <class F>
__device__ __forceinline__ void over_instances(int32_t i0, int32_t i1, F f) {
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
  for (int64_t i = i0 + static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave; i < i1; i += waves)
    f(static_cast<int32_t>(i));
}

template <class T>
__device__ void interval(int k, const Args<T>& a) {
  using C = typename Storage<T>::C;
  switch (k) {
    case 0:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t) { ch_copy(a, ch); });
      break;
    case 1:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t) { ch_axpy(a, ch); });
      over_chunks<T>(a.cl, a.l0, a.l1, [&](const Chunk& ch, int64_t c) { ch_norm(a, ch, c); });
      break;
    case 2:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t c) { ch_dot<T>(a.x, a.y, a.part_b, ch, c); });
      over_instances(a.i0, a.i1, [&](int32_t i) {
        const double v = wave_sum(a.part_a, a.fl[i], a.fl[i + 1]);
        if (threadIdx.x % kWave == 0) a.out[i * kSlots + S_NORM] = v;
      });
      break;
    case 3:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t c) { ch_update(a, a.alpha, a.part_a, ch, c); });
      over_instances(a.i0, a.i1, [&](int32_t i) {
        const double v = wave_sum(a.part_b, a.fg[i], a.fg[i + 1]);
        if (threadIdx.x % kWave == 0) a.out[i * kSlots + S_DOT] = v;
      });
      break;
    case 4:
      over_chunks<T>(a.cl, a.l0, a.l1, [&](const Chunk& ch, int64_t) { ch_scatter(a, a.x, a.xL, ch); });
      over_chunks<T>(a.cl, a.l0, a.l1, [&](const Chunk& ch, int64_t) { ch_scatter(a, a.p, a.pL, ch); });
      over_instances(a.i0, a.i1, [&](int32_t i) {
        const double v = wave_sum(a.part_a, a.fg[i], a.fg[i + 1]);
        if (threadIdx.x % kWave == 0) a.out[i * kSlots + S_RR] = v;
      });
      break;
    case 5:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t) { ch_gather(a, a.xL, a.y, ch); });
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t) { ch_gather(a, a.pL, a.Ap, ch); });
      break;
    case 6:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t c) { ch_dot<T>(a.p, a.Ap, a.part_b, ch, c); });
      break;
    case 7:
      over_instances(a.i0, a.i1, [&](int32_t i) {
        const double v = wave_sum(a.part_b, a.fg[i], a.fg[i + 1]);
        if (threadIdx.x % kWave == 0) {
          a.out[i * kSlots + S_PAP] = v;
          a.out[i * kSlots + S_ALPHA] = a.out[i * kSlots + S_RR] / v;
        }
      });
      break;
    case 8:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t c) {
        const C al = static_cast<C>(a.out[ch.inst * kSlots + S_ALPHA]);
        ch_update(a, al, a.part_a, ch, c);
      });
      break;
    case 9:
      over_instances(a.i0, a.i1, [&](int32_t i) {
        const double v = wave_sum(a.part_a, a.fg[i], a.fg[i + 1]);
        if (threadIdx.x % kWave == 0) {
          a.out[i * kSlots + S_RR2] = v;
          a.out[i * kSlots + S_BETA] = v / a.out[i * kSlots + S_RR];
        }
      });
      break;
    default:
      over_chunks<T>(a.cg, a.g0, a.g1, [&](const Chunk& ch, int64_t) { ch_direction(a, ch); });
      break;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_interval(int k, Args<T> a) {
  interval<T>(k, a);
}

}  // namespace
}  // namespace bs

// ---------------------------------------------------------------- plan

struct bs_batch {
  int device;
  int32_t n_inst;
  int64_t n_local, n_global;
  std::vector<int64_t> off_local, off_global;    // [n_inst + 1]
  std::vector<int64_t> first_local, first_global;  // first chunk of each instance [n_inst + 1]
  bs::Chunk* chunks_local;
  bs::Chunk* chunks_global;
  int64_t* d_first_local;
  int64_t* d_first_global;
  bs_gs* plan;
  double* partials;  // two buffers of 2 * max(chunks) doubles
};

using namespace bs;

namespace {

void free_batch(bs_batch* b) {
  if (!b) return;
  (void)hipFree(b->chunks_local);
  (void)hipFree(b->chunks_global);
  (void)hipFree(b->d_first_local);
  (void)hipFree(b->d_first_global);
  (void)hipFree(b->partials);
  if (b->plan) (void)bs_gs_destroy(b->plan);
  delete b;
}

// chunks of the concatenation with per-instance lengths len[i]
void make_chunks(const std::vector<int64_t>& off, std::vector<Chunk>& chunks, std::vector<int64_t>& first) {
  const size_t n = off.size() - 1;
  first.assign(n + 1, 0);
  chunks.clear();
  for (size_t i = 0; i < n; ++i) {
    first[i] = static_cast<int64_t>(chunks.size());
    for (int64_t s = off[i]; s < off[i + 1]; s += kChunk) {
      const int64_t len = std::min<int64_t>(kChunk, off[i + 1] - s);
      chunks.push_back(Chunk{s, static_cast<int32_t>(len), static_cast<int32_t>(i)});
    }
  }
  first[n] = static_cast<int64_t>(chunks.size());
}

__global__ void k_shift_map(const int32_t* in, int32_t* out, const Chunk* chunks, int64_t n_chunks,
                            const int64_t* off_global_dev, int* bad) {
  for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    const Chunk ch = chunks[c];
    const int64_t base = off_global_dev[ch.inst];
    const int64_t ng = off_global_dev[ch.inst + 1] - base;
    for (int e = threadIdx.x; e < ch.len; e += kBlock) {
      const int32_t id = in[ch.start + e];
      if (id < 0 || id >= ng) {
        *bad = 1;
        out[ch.start + e] = 0;
      } else {
        out[ch.start + e] = static_cast<int32_t>(base + id);
      }
    }
  }
}

template <class T>
bs_status run_step(bs_ctx* ctx, bs_batch* b, int mode, const bs_batch_vectors* v, double alpha, double beta,
                   double* d_out, hipStream_t st) {
  using E = typename Storage<T>::E;
  using C = typename Storage<T>::C;
  Args<T> a{};
  a.x = static_cast<E*>(v->x);
  a.y = static_cast<E*>(v->y);
  a.p = static_cast<E*>(v->p);
  a.r = static_cast<E*>(v->r);
  a.Ap = static_cast<E*>(v->Ap);
  a.xL = static_cast<E*>(v->xL);
  a.pL = static_cast<E*>(v->pL);
  a.wL = static_cast<const E*>(v->wL);
  a.cg = b->chunks_global;
  a.cl = b->chunks_local;
  a.fg = b->d_first_global;
  a.fl = b->d_first_local;
  a.map = b->plan->map;
  a.rs = b->plan->row_starts;
  a.ci = b->plan->col_ids;
  const int64_t nch = std::max(b->first_global.back(), b->first_local.back());
  a.part_a = b->partials;
  a.part_b = b->partials + 2 * nch;
  a.out = d_out;
  a.alpha = static_cast<C>(alpha);
  a.beta = static_cast<C>(beta);
  (void)ctx;
  auto grid_of = [](int64_t g, int64_t l, int64_t inst) {
    int64_t n = std::max(g, l);
    n = std::max(n, (inst + kBlock / kWave - 1) / (kBlock / kWave));
    return static_cast<unsigned int>(std::max<int64_t>(1, std::min<int64_t>(n, 1 << 20)));
  };
  if (mode == BS_BATCH_PER_INSTANCE) {
    for (int32_t i = 0; i < b->n_inst; ++i) {
      a.g0 = b->first_global[i];
      a.g1 = b->first_global[i + 1];
      a.l0 = b->first_local[i];
      a.l1 = b->first_local[i + 1];
      a.i0 = i;
      a.i1 = i + 1;
      const unsigned int grid = grid_of(a.g1 - a.g0, a.l1 - a.l0, 1);
      for (int k = 0; k < kIntervals; ++k) hipLaunchKernelGGL(k_interval<T>, dim3(grid), dim3(kBlock), 0, st, k, a);
    }
    return check_launch("bs_batch_step");
  }
  a.g0 = 0;
  a.g1 = b->first_global.back();
  a.l0 = 0;
  a.l1 = b->first_local.back();
  a.i0 = 0;
  a.i1 = b->n_inst;
  if (mode == BS_BATCH_PER_PHASE) {
    const unsigned int grid = grid_of(a.g1, a.l1, b->n_inst);
    for (int k = 0; k < kIntervals; ++k) hipLaunchKernelGGL(k_interval<T>, dim3(grid), dim3(kBlock), 0, st, k, a);
    return check_launch("bs_batch_step");
  }
  return fail(BS_ERR_UNSUPPORTED, "bs_batch_step: the persistent form is not available");
}

}  // namespace

extern "C" bs_status bs_mesh_box_map_host(int64_t E, int N, int32_t* map, int64_t* n_global) {
  const char* op = "bs_mesh_box_map_host";
  if (E < 1 || N < 1) return fail(BS_ERR_INVALID_ARG, "%s: need E >= 1 and N >= 1", op);
  if (!map) return fail(BS_ERR_INVALID_ARG, "%s: map is NULL", op);
  int64_t m = 1;
  while (m * m * m < E) ++m;
  const int64_t Np = N + 1, M = m * N + 1;
  if (M * M * M >= (int64_t(1) << 31) || E * Np * Np * Np >= (int64_t(1) << 31))
    return fail(BS_ERR_INVALID_ARG, "%s: mesh too large for 32-bit ids", op);
  std::vector<int32_t> rank(static_cast<size_t>(M * M * M), -1);
  auto key = [&](int64_t e, int64_t i, int64_t j, int64_t k) {
    const int64_t X = N * (e % m) + i, Y = N * ((e / m) % m) + j, Z = N * (e / (m * m)) + k;
    return X + M * (Y + M * Z);
  };
  for (int64_t e = 0; e < E; ++e)
    for (int64_t k = 0; k < Np; ++k)
      for (int64_t j = 0; j < Np; ++j)
        for (int64_t i = 0; i < Np; ++i) rank[static_cast<size_t>(key(e, i, j, k))] = 0;
  int32_t next = 0;
  for (auto& r : rank)
    if (r == 0) r = next++;
  int64_t l = 0;
  for (int64_t e = 0; e < E; ++e)
    for (int64_t k = 0; k < Np; ++k)
      for (int64_t j = 0; j < Np; ++j)
        for (int64_t i = 0; i < Np; ++i) map[l++] = rank[static_cast<size_t>(key(e, i, j, k))];
  if (n_global) *n_global = next;
  return BS_OK;
}

extern "C" bs_status bs_batch_create(bs_ctx* ctx, int32_t n_inst, const int64_t* h_n_local,
                                     const int64_t* h_n_global, const int32_t* d_map, void* stream, bs_batch** out) {
  const char* op = "bs_batch_create";
  bs_status s;
  if ((s = check_ctx(ctx, op))) return s;
  if (!out) return fail(BS_ERR_INVALID_ARG, "%s: out is NULL", op);
  *out = nullptr;
  if (n_inst < 1 || !h_n_local || !h_n_global || !d_map)
    return fail(BS_ERR_INVALID_ARG, "%s: need n_inst >= 1 and non-NULL sizes and map", op);
  if (!aligned_to(d_map, 4)) return fail(BS_ERR_INVALID_ARG, "%s: misaligned map", op);
  bs_batch* b = new bs_batch{};
  b->device = ctx->device;
  b->n_inst = n_inst;
  b->off_local.assign(n_inst + 1, 0);
  b->off_global.assign(n_inst + 1, 0);
  for (int32_t i = 0; i < n_inst; ++i) {
    if (h_n_local[i] < 1 || h_n_global[i] < 1) {
      delete b;
      return fail(BS_ERR_INVALID_ARG, "%s: instance %d has an empty vector", op, i);
    }
    b->off_local[i + 1] = b->off_local[i] + h_n_local[i];
    b->off_global[i + 1] = b->off_global[i] + h_n_global[i];
  }
  b->n_local = b->off_local.back();
  b->n_global = b->off_global.back();
  if (b->n_local >= (int64_t(1) << 31) || b->n_global >= (int64_t(1) << 31)) {
    delete b;
    return fail(BS_ERR_INVALID_ARG, "%s: totals must stay below 2^31", op);
  }
  std::vector<Chunk> cl, cgl;
  make_chunks(b->off_local, cl, b->first_local);
  make_chunks(b->off_global, cgl, b->first_global);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nch = std::max<int64_t>(cl.size(), cgl.size());
  int32_t* shifted = nullptr;
  int64_t* d_off_global = nullptr;
  int* bad = nullptr;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
  bool ok = alloc(reinterpret_cast<void**>(&b->chunks_local), cl.size() * sizeof(Chunk)) &&
            alloc(reinterpret_cast<void**>(&b->chunks_global), cgl.size() * sizeof(Chunk)) &&
            alloc(reinterpret_cast<void**>(&b->d_first_local), (n_inst + 1) * sizeof(int64_t)) &&
            alloc(reinterpret_cast<void**>(&b->d_first_global), (n_inst + 1) * sizeof(int64_t)) &&
            alloc(reinterpret_cast<void**>(&b->partials), 4 * nch * sizeof(double)) &&
            alloc(reinterpret_cast<void**>(&shifted), b->n_local * sizeof(int32_t)) &&
            alloc(reinterpret_cast<void**>(&d_off_global), (n_inst + 1) * sizeof(int64_t)) &&
            alloc(reinterpret_cast<void**>(&bad), sizeof(int));
  if (!ok) {
    (void)hipFree(shifted);
    (void)hipFree(d_off_global);
    (void)hipFree(bad);
    free_batch(b);
    return fail(BS_ERR_ALLOC, "%s: device allocation failed", op);
  }
  s = check_hip(hipMemcpyAsync(b->chunks_local, cl.data(), cl.size() * sizeof(Chunk), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemcpyAsync(b->chunks_global, cgl.data(), cgl.size() * sizeof(Chunk), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemcpyAsync(b->d_first_local, b->first_local.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemcpyAsync(b->d_first_global, b->first_global.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemcpyAsync(d_off_global, b->off_global.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemsetAsync(bad, 0, sizeof(int), st), op);
  if (!s) {
    const unsigned int grid = static_cast<unsigned int>(std::min<int64_t>(static_cast<int64_t>(cl.size()), 65536));
    hipLaunchKernelGGL(k_shift_map, dim3(grid), dim3(kBlock), 0, st, d_map, shifted, b->chunks_local,
                       static_cast<int64_t>(cl.size()), d_off_global, bad);
    s = check_launch(op);
  }
  int h_bad = 0;
  if (!s) s = check_hip(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st), op);
  if (!s) s = check_hip(hipStreamSynchronize(st), op);
  if (!s && h_bad) s = fail(BS_ERR_INVALID_ARG, "%s: a map entry lies outside its instance's global range", op);
  if (!s) s = bs_gs_create(ctx, shifted, b->n_local, b->n_global, stream, &b->plan);
  (void)hipFree(shifted);
  (void)hipFree(d_off_global);
  (void)hipFree(bad);
  if (s) {
    free_batch(b);
    return s;
  }
  *out = b;
  return BS_OK;
}

extern "C" bs_status bs_batch_destroy(bs_batch* b) {
  free_batch(b);
  return BS_OK;
}

extern "C" bs_status bs_batch_info(const bs_batch* b, int64_t* n_local, int64_t* n_global, int64_t* n_chunks_local,
                                   int64_t* n_chunks_global, int32_t* persistent_blocks_f64) {
  if (!b) return fail(BS_ERR_INVALID_ARG, "bs_batch_info: batch is NULL");
  if (n_local) *n_local = b->n_local;
  if (n_global) *n_global = b->n_global;
  if (n_chunks_local) *n_chunks_local = b->first_local.back();
  if (n_chunks_global) *n_chunks_global = b->first_global.back();
  if (persistent_blocks_f64) *persistent_blocks_f64 = 0;
  return BS_OK;
}

extern "C" bs_status bs_batch_offsets(const bs_batch* b, int64_t* h_off_local, int64_t* h_off_global) {
  if (!b) return fail(BS_ERR_INVALID_ARG, "bs_batch_offsets: batch is NULL");
  if (h_off_local) std::copy(b->off_local.begin(), b->off_local.end(), h_off_local);
  if (h_off_global) std::copy(b->off_global.begin(), b->off_global.end(), h_off_global);
  return BS_OK;
}

extern "C" bs_status bs_batch_barrier_timeouts(const bs_batch* b, int32_t* count, void* stream) {
  if (!b || !count) return fail(BS_ERR_INVALID_ARG, "bs_batch_barrier_timeouts: NULL argument");
  (void)stream;
  *count = 0;  // no form waits on a grid barrier
  return BS_OK;
}

extern "C" bs_status bs_batch_step(bs_ctx* ctx, bs_batch* b, bs_dtype dtype, int mode, const bs_batch_vectors* v,
                                   double alpha, double beta, double* d_out, void* stream) {
  const char* op = "bs_batch_step";
  bs_status s;
  if ((s = check_ctx(ctx, op)) || (s = check_dtype(op, dtype))) return s;
  if (!b || !v || !d_out) return fail(BS_ERR_INVALID_ARG, "%s: NULL batch, vectors or output", op);
  if (mode < BS_BATCH_PER_INSTANCE || mode > BS_BATCH_PERSISTENT)
    return fail(BS_ERR_INVALID_ARG, "%s: unknown mode %d", op, mode);
  const void* g[] = {v->x, v->y, v->p, v->r, v->Ap};
  const void* l[] = {v->xL, v->pL, v->wL};
  for (const void* q : g)
    if ((s = check_vec(op, "global vector", q, b->n_global, dtype))) return s;
  for (const void* q : l)
    if ((s = check_vec(op, "local vector", q, b->n_local, dtype))) return s;
  if (!aligned_to(d_out, 8)) return fail(BS_ERR_INVALID_ARG, "%s: misaligned output", op);
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case BS_F64: return run_step<double>(ctx, b, mode, v, alpha, beta, d_out, st);
    case BS_F32: return run_step<float>(ctx, b, mode, v, alpha, beta, d_out, st);
    case BS_BF16: return run_step<dev::bf16>(ctx, b, mode, v, alpha, beta, d_out, st);
  }
  return fail(BS_ERR_INVALID_ARG, "%s: unknown dtype", op);
}
