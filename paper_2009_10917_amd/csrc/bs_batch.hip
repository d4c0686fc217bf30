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
// instance, and chunks into items: up to 8 chunks of one instance in one
// part of a phase (or one instance's final sum of a reduction).  The step's
// phases are grouped into eleven intervals by data dependence; within an
// interval no item depends on another.  Reductions leave one compensated
// pair per chunk in a buffer of their own, and an instance's value is the
// sum of its chunks' pairs in chunk order, formed by one wave.  Three forms
// run the same item code on the same chunks, so they give identical bits:
//   per instance  one launch per interval and instance (11 per instance),
//                 one chunk per workgroup;
//   per phase     one launch per interval for the whole batch, one chunk
//                 per workgroup;
//   persistent    one launch.  Workgroups claim items with an atomic ticket
//                 in list order (intervals ascending); before an item of
//                 interval k of instance i runs, its workgroup waits until
//                 every interval k-1 item of instance i is done.  Those
//                 items come earlier in the list, so they were claimed
//                 earlier by running workgroups and the wait ends however
//                 many workgroups are resident.  Waits poll with relaxed
//                 loads; a wait longer than a wall-clock limit sets a sticky
//                 abort flag that ends every workgroup, so the kernel always
//                 finishes.  The last workgroup out resets the ticket and
//                 the counters for the next launch.
// Per-phase and persistent steps neither allocate nor synchronise, so a
// caller can capture them in a HIP graph.

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
constexpr int kItemChunks = 8;             // chunks per item
constexpr int kClaimMax = 8;               // items per ticket of the persistent form, at most (tune op "batch")
constexpr int kSlots = 8;                  // output doubles per instance
enum Slot { S_NORM = 0, S_DOT, S_RR, S_PAP, S_ALPHA, S_RR2, S_BETA };

// Parts of the step; kInterval gives each part's interval, kTable whether it
// runs over global chunks (0), local chunks (1) or finishes an instance (2).
enum Part {
  P_COPY, P_AXPY, P_NORM, P_DOT_XY, F_NORM, P_UPDATE_A, F_DOT, P_SCATTER, F_RR, P_GATHER, P_DOT_PAP, F_PAP,
  P_UPDATE_B, F_RR2, P_DIRECTION, N_PARTS
};
constexpr int kInterval[N_PARTS] = {0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 6, 7, 8, 9, 10};
constexpr int kTable[N_PARTS] = {0, 0, 1, 0, 2, 0, 2, 1, 2, 0, 0, 2, 0, 2, 0};

template <class T> struct DtypeOf;
template <> struct DtypeOf<double> { static constexpr bs_dtype v = BS_F64; };
template <> struct DtypeOf<float> { static constexpr bs_dtype v = BS_F32; };
template <> struct DtypeOf<dev::bf16> { static constexpr bs_dtype v = BS_BF16; };

struct Chunk {
  int64_t start;  // first element (index into the concatenated vectors)
  int32_t len;    // 1 .. kChunk
  int32_t inst;
};

// One unit of work: chunks [c0, c1) of the part's table, all of instance
// `inst` (or, for a finishing part, that instance's sum).
struct Item {
  int32_t part;
  int32_t inst;
  int32_t c0, c1;
};

// One chunk of a part of one instance (chunk -1: the instance's finish).
struct Unit {
  int32_t part;
  int32_t inst;
  int32_t chunk;
  int32_t pad;
};

// Shared state of the persistent form.
struct Sched {
  unsigned int* ticket;     // next claim
  unsigned int* exits;      // workgroups that have left
  int* abort;               // sticky: a wait outlived the limit
  unsigned int* done;       // [kIntervals][n_inst] items completed
  const unsigned int* need; // [kIntervals][n_inst] items in all
  int64_t n_items;
  int32_t n_inst;
  int32_t claim;            // items per ticket (1 .. kClaimMax)
  uint64_t wait_ticks;      // wall-clock limit of one wait
};

template <class T>
struct Args {
  using E = typename Storage<T>::E;
  using C = typename Storage<T>::C;
  E *x, *y, *p, *r, *Ap, *xL, *pL;
  const E* wL;
  const Chunk* cg;  // chunks of the global vectors
  const Chunk* cl;  // chunks of the local vectors
  const Item* items;
  const Unit* units;
  const int64_t* fg;       // first global chunk of each instance [n_inst + 1]
  const int64_t* fl;       // first local chunk of each instance [n_inst + 1]
  const int32_t* map;      // scatter ids, shifted to the concatenated global vector
  const int32_t* rs;       // CSR of Z^T
  const int32_t* ci;
  double* part_norm;       // compensated pairs per chunk, one buffer per reduction
  double* part_dot;
  double* part_rr;
  double* part_pap;
  double* part_rr2;
  double* out;             // [n_inst][kSlots]
  C alpha, beta;
};

// ---------------------------------------------------------------- chunk bodies

// A chunk's elements are e = threadIdx.x + kBlock k (k < kPer).  Each body
// issues every load of the chunk before it computes or stores anything (a
// store between two loads would order them: the vectors may alias as far as
// the compiler knows), with lanes past the chunk's end loading its last
// element; results are then formed and stored for the elements inside the
// chunk, in k order, so that sums add in the same order as an element-wise
// loop would.
__device__ __forceinline__ int64_t elem(const Chunk& ch, int k) {
  return ch.start + min(static_cast<int32_t>(threadIdx.x) + kBlock * k, ch.len - 1);
}
__device__ __forceinline__ bool inside(const Chunk& ch, int k) {
  return static_cast<int32_t>(threadIdx.x) + kBlock * k < ch.len;
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
  typename Storage<T>::E v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) v[k] = a.x[elem(ch, k)];
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (inside(ch, k)) a.y[elem(ch, k)] = v[k];
}

template <class T>
__device__ void ch_axpy(const Args<T>& a, const Chunk& ch) {
  using S = Storage<T>;
  typename S::E u[kPer], v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    u[k] = a.x[elem(ch, k)];
    v[k] = a.y[elem(ch, k)];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (inside(ch, k)) a.y[elem(ch, k)] = S::store(a.alpha * S::load(u[k]) + a.beta * S::load(v[k]));
}

template <class T>
__device__ void ch_norm(const Args<T>& a, const Chunk& ch, int64_t c) {
  using S = Storage<T>;
  using C = typename S::C;
  typename S::E u[kPer], w[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    u[k] = a.xL[elem(ch, k)];
    w[k] = a.wL[elem(ch, k)];
  }
  DW<C> acc{C(0), C(0)};
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const C xk = S::load(u[k]);
    if (inside(ch, k)) dev::dw_acc(acc, S::load(w[k]) * (xk * xk));
  }
  put_pair(a.part_norm, c, widen(acc));
}

template <class T>
__device__ void ch_dot(const typename Storage<T>::E* u, const typename Storage<T>::E* v, double* part,
                       const Chunk& ch, int64_t c) {
  using S = Storage<T>;
  using C = typename S::C;
  typename S::E p[kPer], q[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    p[k] = u[elem(ch, k)];
    q[k] = v[elem(ch, k)];
  }
  DW<C> acc{C(0), C(0)};
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (inside(ch, k)) dev::dw_acc_prod(acc, S::load(p[k]), S::load(q[k]));
  put_pair(part, c, widen(acc));
}

template <class T>
__device__ void ch_update(const Args<T>& a, typename Storage<T>::C alpha, double* part, const Chunk& ch, int64_t c) {
  using S = Storage<T>;
  using C = typename S::C;
  typename S::E xv[kPer], pv[kPer], rv[kPer], av[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t e = elem(ch, k);
    xv[k] = a.x[e];
    pv[k] = a.p[e];
    rv[k] = a.r[e];
    av[k] = a.Ap[e];
  }
  DW<C> acc{C(0), C(0)};
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (!inside(ch, k)) continue;
    const int64_t e = elem(ch, k);
    a.x[e] = S::store(S::load(xv[k]) + alpha * S::load(pv[k]));
    const typename S::E rn = S::store(S::load(rv[k]) - alpha * S::load(av[k]));
    a.r[e] = rn;
    const C rk = S::load(rn);
    dev::dw_acc_prod(acc, rk, rk);
  }
  put_pair(part, c, widen(acc));
}

template <class T>
__device__ void ch_scatter(const Args<T>& a, const typename Storage<T>::E* g, typename Storage<T>::E* l,
                           const Chunk& ch) {
  int32_t id[kPer];
  typename Storage<T>::E v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) id[k] = a.map[elem(ch, k)];
#pragma unroll
  for (int k = 0; k < kPer; ++k) v[k] = g[id[k]];
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (inside(ch, k)) l[elem(ch, k)] = v[k];
}

// Each row from +0.0, its local copies added in ascending local index.  The
// chunk's rows own the CSR positions [rs[first row], rs[last row + 1]);
// these are walked in windows of kChunk: column ids loaded contiguously,
// then every value of the window at once, staged in LDS, and each row adds
// the copies it has in the window (a row's partial sum carries over to the
// next window, so the additions keep their order).
template <class T>
__device__ void ch_gather(const Args<T>& a, const typename Storage<T>::E* l, typename Storage<T>::E* g,
                          const Chunk& ch) {
  using S = Storage<T>;
  using C = typename S::C;
  __shared__ C stage[kChunk];
  int32_t j0[kPer], j1[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t e = elem(ch, k);
    j0[k] = a.rs[e];
    j1[k] = a.rs[e + 1];
  }
  const int32_t n0 = a.rs[ch.start], n1 = a.rs[ch.start + ch.len];
  C s[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) s[k] = C(0);
  for (int32_t w0 = n0; w0 < n1; w0 += kChunk) {
    const int32_t wn = min(kChunk, n1 - w0);
    int32_t col[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) col[k] = a.ci[w0 + min(static_cast<int32_t>(threadIdx.x) + kBlock * k, wn - 1)];
    typename S::E v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = l[col[k]];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t q = threadIdx.x + kBlock * k;
      if (q < wn) stage[q] = S::load(v[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int32_t lo = max(j0[k], w0), hi = min(j1[k], w0 + wn);
      for (int32_t j = lo; j < hi; ++j) s[k] = s[k] + stage[j - w0];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (inside(ch, k)) g[elem(ch, k)] = S::store(s[k]);
}

template <class T>
__device__ void ch_direction(const Args<T>& a, const Chunk& ch) {
  using S = Storage<T>;
  using C = typename S::C;
  const C b = static_cast<C>(a.out[ch.inst * kSlots + S_BETA]);
  typename S::E rv[kPer], pv[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    rv[k] = a.r[elem(ch, k)];
    pv[k] = a.p[elem(ch, k)];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (inside(ch, k)) a.p[elem(ch, k)] = S::store(C(1) * S::load(rv[k]) + b * S::load(pv[k]));
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

// ---------------------------------------------------------------- items

// Finishing an instance's sum: wave 0 of the workgroup.
template <class T>
__device__ void run_finish(int part, int32_t i, const Args<T>& a) {
  if (threadIdx.x >= kWave) return;
  double* o = a.out + static_cast<int64_t>(i) * kSlots;
  switch (part) {
    case F_NORM: {
      const double v = wave_sum(a.part_norm, a.fl[i], a.fl[i + 1]);
      if (threadIdx.x == 0) o[S_NORM] = v;
      break;
    }
    case F_DOT: {
      const double v = wave_sum(a.part_dot, a.fg[i], a.fg[i + 1]);
      if (threadIdx.x == 0) o[S_DOT] = v;
      break;
    }
    case F_RR: {
      const double v = wave_sum(a.part_rr, a.fg[i], a.fg[i + 1]);
      if (threadIdx.x == 0) o[S_RR] = v;
      break;
    }
    case F_PAP: {
      const double v = wave_sum(a.part_pap, a.fg[i], a.fg[i + 1]);
      if (threadIdx.x == 0) {
        o[S_PAP] = v;
        o[S_ALPHA] = o[S_RR] / v;
      }
      break;
    }
    default: {  // F_RR2
      const double v = wave_sum(a.part_rr2, a.fg[i], a.fg[i + 1]);
      if (threadIdx.x == 0) {
        o[S_RR2] = v;
        o[S_BETA] = v / o[S_RR];
      }
      break;
    }
  }
}

// One chunk of a part, by the whole workgroup.
template <class T>
__device__ void run_chunk(int part, int32_t i, int32_t c, const Args<T>& a) {
  using C = typename Storage<T>::C;
  const Chunk ch = (kTable[part] == 0 ? a.cg : a.cl)[c];
  switch (part) {
    case P_COPY: ch_copy(a, ch); break;
    case P_AXPY: ch_axpy(a, ch); break;
    case P_NORM: ch_norm(a, ch, c); break;
    case P_DOT_XY: ch_dot<T>(a.x, a.y, a.part_dot, ch, c); break;
    case P_UPDATE_A: ch_update(a, a.alpha, a.part_rr, ch, c); break;
    case P_SCATTER:
      ch_scatter(a, a.x, a.xL, ch);
      ch_scatter(a, a.p, a.pL, ch);
      break;
    case P_GATHER:
      ch_gather(a, a.xL, a.y, ch);
      ch_gather(a, a.pL, a.Ap, ch);
      break;
    case P_DOT_PAP: ch_dot<T>(a.p, a.Ap, a.part_pap, ch, c); break;
    case P_UPDATE_B:
      ch_update(a, static_cast<C>(a.out[static_cast<int64_t>(i) * kSlots + S_ALPHA]), a.part_rr2, ch, c);
      break;
    default: ch_direction(a, ch); break;
  }
}

// One item: its chunks in order, or its instance's finish.
template <class T>
__device__ void run_item(const Item& it, const Args<T>& a) {
  if (kTable[it.part] == 2) {
    run_finish(it.part, it.inst, a);
    return;
  }
  for (int32_t c = it.c0; c < it.c1; ++c) run_chunk(it.part, it.inst, c, a);
}

// Units [u0, u1): one chunk of an item, or one finish, per workgroup at a
// time (per-instance and per-phase forms; the launch boundary orders the
// intervals).
template <class T>
__global__ __launch_bounds__(kBlock) void k_units(int64_t u0, int64_t u1, Args<T> a) {
  for (int64_t u = u0 + blockIdx.x; u < u1; u += gridDim.x) {
    const Unit un = a.units[u];
    if (un.chunk < 0)
      run_finish(un.part, un.inst, a);
    else
      run_chunk(un.part, un.inst, un.chunk, a);
    __syncthreads();
  }
}

__device__ __forceinline__ unsigned int load_relaxed(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait until instance i has finished interval k - 1, counting
// `local` items of that interval which this workgroup has run but not yet
// published.  Returns false when the form has been aborted.
__device__ bool wait_ready(const Sched& sc, int k, int32_t i, unsigned int local) {
  if (k == 0) return __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  const int64_t slot = static_cast<int64_t>(k - 1) * sc.n_inst + i;
  const unsigned int need = sc.need[slot] - local;
  const uint64_t t0 = wall_clock64();
  bool waited = false;
  while (load_relaxed(sc.done + slot) < need) {
    if (__hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (wall_clock64() - t0 > sc.wait_ticks) {
      __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    waited = true;
    __builtin_amdgcn_s_sleep(4);
  }
  // what the finished items of other workgroups wrote is visible from here on
  if (waited || need > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Each claim of sc.claim consecutive items runs in list order; its completions
// are published together after one release fence (an item may depend on an
// earlier item of the same claim, whose writes this workgroup already sees).
template <class T>
__global__ __launch_bounds__(kBlock) void k_persistent(Args<T> a, Sched sc) {
  __shared__ int64_t s_claim;
  __shared__ int s_go;
  while (true) {
    if (threadIdx.x == 0) {
      const bool stop = __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      s_claim = stop ? sc.n_items
                     : static_cast<int64_t>(__hip_atomic_fetch_add(sc.ticket, 1u, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT)) * sc.claim;
    }
    __syncthreads();
    const int64_t first = s_claim;
    if (first >= sc.n_items) break;
    const int64_t last = first + sc.claim < sc.n_items ? first + sc.claim : sc.n_items;
    bool stop = false;
    for (int64_t t = first; t < last; ++t) {
      const Item it = a.items[t];
      const int k = kInterval[it.part];
      if (threadIdx.x == 0) {
        unsigned int local = 0;  // earlier items of this claim that (k - 1, inst) is waiting for
        for (int64_t u = first; u < t; ++u) {
          const Item e = a.items[u];
          local += (kInterval[e.part] == k - 1 && e.inst == it.inst) ? 1u : 0u;
        }
        s_go = wait_ready(sc, k, it.inst, local) ? 1 : 0;
      }
      __syncthreads();
      if (!s_go) {
        stop = true;
        break;
      }
      run_item(it, a);
      __syncthreads();  // every thread's writes of the item are complete
    }
    if (stop) break;
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      int64_t t = first;
      while (t < last) {  // one increment per run of items with the same (interval, instance)
        const Item it = a.items[t];
        const int k = kInterval[it.part];
        unsigned int n = 0;
        while (t < last && kInterval[a.items[t].part] == k && a.items[t].inst == it.inst) {
          ++n;
          ++t;
        }
        __hip_atomic_fetch_add(sc.done + static_cast<int64_t>(k) * sc.n_inst + it.inst, n, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
  // the last workgroup out resets the schedule for the next launch
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    s_go = __hip_atomic_fetch_add(sc.exits, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  }
  __syncthreads();
  if (s_go) {
    for (int64_t j = threadIdx.x; j < static_cast<int64_t>(kIntervals) * sc.n_inst; j += kBlock) sc.done[j] = 0;
    if (threadIdx.x == 0) {
      *sc.ticket = 0;
      *sc.exits = 0;
    }
  }
}

}  // namespace
}  // namespace bs

// ---------------------------------------------------------------- plan

struct bs_batch {
  int device;
  int32_t n_inst;
  int64_t n_local, n_global;
  std::vector<int64_t> off_local, off_global;      // [n_inst + 1]
  std::vector<int64_t> first_local, first_global;  // first chunk of each instance [n_inst + 1]
  std::vector<int64_t> first_item;                 // [kIntervals * n_inst + 1]: items of (interval, instance)
  bs::Chunk* chunks_local;
  bs::Chunk* chunks_global;
  bs::Item* items;
  int64_t n_items;
  bs::Unit* units;
  std::vector<int64_t> first_unit;                 // [n_items + 1]
  int64_t* d_first_local;
  int64_t* d_first_global;
  bs_gs* plan;
  double* partials;  // one buffer per reduction: 2 pairs-worth per chunk of its table
  unsigned int* sched;  // ticket, exits, abort, then done[kIntervals * n_inst]
  unsigned int* need;   // [kIntervals * n_inst]
  int resident[3];      // workgroups of one persistent launch per dtype
  uint64_t wait_ticks;
};

using namespace bs;

namespace {

void free_batch(bs_batch* b) {
  if (!b) return;
  (void)hipFree(b->chunks_local);
  (void)hipFree(b->chunks_global);
  (void)hipFree(b->items);
  (void)hipFree(b->units);
  (void)hipFree(b->d_first_local);
  (void)hipFree(b->d_first_global);
  (void)hipFree(b->partials);
  (void)hipFree(b->sched);
  (void)hipFree(b->need);
  if (b->plan) (void)bs_gs_destroy(b->plan);
  delete b;
}

// chunks of the concatenation with per-instance lengths from the offsets
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

// The item list, sorted by (interval, instance, part), and the number of
// items of every (interval, instance).
void make_items(const bs_batch* b, std::vector<Item>& items, std::vector<int64_t>& first,
                std::vector<unsigned int>& need) {
  const int32_t n = b->n_inst;
  items.clear();
  first.assign(static_cast<size_t>(kIntervals) * n + 1, 0);
  need.assign(static_cast<size_t>(kIntervals) * n, 0);
  for (int k = 0; k < kIntervals; ++k) {
    for (int32_t i = 0; i < n; ++i) {
      first[static_cast<size_t>(k) * n + i] = static_cast<int64_t>(items.size());
      for (int p = 0; p < N_PARTS; ++p) {
        if (kInterval[p] != k) continue;
        if (kTable[p] == 2) {
          items.push_back(Item{p, i, 0, 0});
          continue;
        }
        const std::vector<int64_t>& f = kTable[p] == 0 ? b->first_global : b->first_local;
        for (int64_t c = f[i]; c < f[i + 1]; c += kItemChunks)
          items.push_back(Item{p, i, static_cast<int32_t>(c), static_cast<int32_t>(std::min<int64_t>(c + kItemChunks, f[i + 1]))});
      }
      need[static_cast<size_t>(k) * n + i] =
          static_cast<unsigned int>(items.size() - first[static_cast<size_t>(k) * n + i]);
    }
  }
  first.back() = static_cast<int64_t>(items.size());
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
int resident_blocks(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<T>, kBlock, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    return 256;
  }
  return per_cu * cus;
}

template <class T>
bs_status run_step(bs_ctx* ctx, bs_batch* b, int mode, const bs_batch_vectors* v, double alpha, double beta,
                   double* d_out,
                   hipStream_t st) {
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
  a.items = b->items;
  a.units = b->units;
  a.fg = b->d_first_global;
  a.fl = b->d_first_local;
  a.map = b->plan->map;
  a.rs = b->plan->row_starts;
  a.ci = b->plan->col_ids;
  const int64_t ncl = b->first_local.back(), ncg = b->first_global.back();
  a.part_norm = b->partials;
  a.part_dot = a.part_norm + 2 * ncl;
  a.part_rr = a.part_dot + 2 * ncg;
  a.part_pap = a.part_rr + 2 * ncg;
  a.part_rr2 = a.part_pap + 2 * ncg;
  a.out = d_out;
  a.alpha = static_cast<C>(alpha);
  a.beta = static_cast<C>(beta);
  const int32_t n = b->n_inst;
  // units of items [i0, i1)
  auto launch = [&](int64_t i0, int64_t i1) {
    const int64_t u0 = b->first_unit[i0], u1 = b->first_unit[i1];
    if (u1 <= u0) return;
    const unsigned int grid = static_cast<unsigned int>(std::min<int64_t>(u1 - u0, 1 << 20));
    hipLaunchKernelGGL(k_units<T>, dim3(grid), dim3(kBlock), 0, st, u0, u1, a);
  };
  if (mode == BS_BATCH_PER_INSTANCE) {
    for (int32_t i = 0; i < n; ++i)
      for (int k = 0; k < kIntervals; ++k)
        launch(b->first_item[static_cast<size_t>(k) * n + i], b->first_item[static_cast<size_t>(k) * n + i + 1]);
    return check_launch("bs_batch_step");
  }
  if (mode == BS_BATCH_PER_PHASE) {
    for (int k = 0; k < kIntervals; ++k)
      launch(b->first_item[static_cast<size_t>(k) * n], b->first_item[static_cast<size_t>(k + 1) * n]);
    return check_launch("bs_batch_step");
  }
  Sched sc{};
  sc.ticket = b->sched;
  sc.exits = b->sched + 1;
  sc.abort = reinterpret_cast<int*>(b->sched + 2);
  sc.done = b->sched + 4;
  sc.need = b->need;
  sc.n_items = b->n_items;
  sc.n_inst = n;
  sc.wait_ticks = b->wait_ticks;
  const int dt = static_cast<int>(DtypeOf<T>::v);
  // items per claim and a cap on the workgroups from the tune entry of op "batch"
  const Tune& tn = tune_for(ctx, OP_BATCH, dt, b->n_items);
  sc.claim = tn.unroll < 1 ? 1 : (tn.unroll > kClaimMax ? kClaimMax : tn.unroll);
  const int64_t claims = (b->n_items + sc.claim - 1) / sc.claim;
  const unsigned int grid = static_cast<unsigned int>(
      std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(b->resident[dt], claims), tn.grid_cap)));
  hipLaunchKernelGGL(k_persistent<T>, dim3(grid), dim3(kBlock), 0, st, a, sc);
  return check_launch("bs_batch_step");
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
  std::vector<Item> items;
  std::vector<unsigned int> need;
  make_items(b, items, b->first_item, need);
  b->n_items = static_cast<int64_t>(items.size());
  if (b->n_items >= (int64_t(1) << 31)) {
    delete b;
    return fail(BS_ERR_INVALID_ARG, "%s: too many work items", op);
  }
  std::vector<Unit> units;
  b->first_unit.assign(items.size() + 1, 0);
  for (size_t t = 0; t < items.size(); ++t) {
    b->first_unit[t] = static_cast<int64_t>(units.size());
    const Item& it = items[t];
    if (kTable[it.part] == 2)
      units.push_back(Unit{it.part, it.inst, -1, 0});
    else
      for (int32_t c = it.c0; c < it.c1; ++c) units.push_back(Unit{it.part, it.inst, c, 0});
  }
  b->first_unit.back() = static_cast<int64_t>(units.size());
  const size_t n_sched = 4 + static_cast<size_t>(kIntervals) * n_inst;
  const size_t n_part = 2 * cl.size() + 8 * cgl.size();
  int32_t* shifted = nullptr;
  int64_t* d_off_global = nullptr;
  int* bad = nullptr;
  auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
  bool ok = alloc(reinterpret_cast<void**>(&b->chunks_local), cl.size() * sizeof(Chunk)) &&
            alloc(reinterpret_cast<void**>(&b->chunks_global), cgl.size() * sizeof(Chunk)) &&
            alloc(reinterpret_cast<void**>(&b->d_first_local), (n_inst + 1) * sizeof(int64_t)) &&
            alloc(reinterpret_cast<void**>(&b->d_first_global), (n_inst + 1) * sizeof(int64_t)) &&
            alloc(reinterpret_cast<void**>(&b->partials), n_part * sizeof(double)) &&
            alloc(reinterpret_cast<void**>(&b->items), items.size() * sizeof(Item)) &&
            alloc(reinterpret_cast<void**>(&b->units), units.size() * sizeof(Unit)) &&
            alloc(reinterpret_cast<void**>(&b->sched), n_sched * sizeof(unsigned int)) &&
            alloc(reinterpret_cast<void**>(&b->need), need.size() * sizeof(unsigned int)) &&
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
  if (!s) s = check_hip(hipMemcpyAsync(b->items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemcpyAsync(b->units, units.data(), units.size() * sizeof(Unit), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemcpyAsync(b->need, need.data(), need.size() * sizeof(unsigned int), hipMemcpyHostToDevice, st), op);
  if (!s) s = check_hip(hipMemsetAsync(b->sched, 0, n_sched * sizeof(unsigned int), st), op);
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
  b->resident[BS_F64] = resident_blocks<double>(b->device);
  b->resident[BS_F32] = resident_blocks<float>(b->device);
  b->resident[BS_BF16] = resident_blocks<dev::bf16>(b->device);
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) != hipSuccess || khz <= 0) {
    (void)hipGetLastError();
    khz = 100000;  // 100 MHz
  }
  b->wait_ticks = static_cast<uint64_t>(khz) * 500;  // half a second
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
  if (persistent_blocks_f64) *persistent_blocks_f64 = b->resident[BS_F64];
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
  hipStream_t st = static_cast<hipStream_t>(stream);
  bs_status s = check_hip(hipMemcpyAsync(count, b->sched + 2, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                          "bs_batch_barrier_timeouts");
  if (!s) s = check_hip(hipStreamSynchronize(st), "bs_batch_barrier_timeouts");
  return s;
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
