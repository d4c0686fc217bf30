// Device-side building blocks for gfx950 (wave64, 8 XCDs).
//
// Every kernel translation unit that includes this header is compiled with
// floating-point contraction off, so `a*b + c` is two roundings unless a
// fused multiply-add is written out with __builtin_fma.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#pragma clang fp contract(off)

namespace bs {
namespace dev {

constexpr int kWave = 64;

// ---------------------------------------------------------------- storage

// Tag type of the bfloat16 dtype; its elements are stored as 16-bit patterns.
struct bf16 {};

// Storage type E, arithmetic type C and native packet width V (elements per
// 16 bytes) of each dtype, with the conversions between E and C.
template <class T> struct Storage;
template <> struct Storage<double> {
  using E = double;
  using C = double;
  static constexpr int V = 2;
  __device__ static double load(double x) { return x; }
  __device__ static double store(double x) { return x; }
};
template <> struct Storage<float> {
  using E = float;
  using C = float;
  static constexpr int V = 4;
  __device__ static float load(float x) { return x; }
  __device__ static float store(float x) { return x; }
};
template <> struct Storage<bf16> {
  using E = uint16_t;
  using C = float;
  static constexpr int V = 8;
  __device__ static float load(uint16_t x) { return __uint_as_float(static_cast<uint32_t>(x) << 16); }
  // binary32 -> bfloat16, round to nearest, ties to even; NaN stays NaN.
  // gfx950 converts in one instruction (v_cvt_pk_bf16_f32).
  __device__ static uint16_t store(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
};

// Register packet of V storage elements: a native vector, so that a full
// packet is one 16-byte (dwordx4) access and stays in VGPRs.
template <class E, int V>
struct VecOf {
  typedef E type __attribute__((ext_vector_type(V)));
};
template <class E>
struct VecOf<E, 1> {
  typedef E type;
};

template <class Vec, class E>
__device__ __forceinline__ E vget(const Vec& v, int k) {
  if constexpr (sizeof(Vec) == sizeof(E)) {
    return v;
  } else {
    return v[k];
  }
}
template <class Vec, class E>
__device__ __forceinline__ void vset(Vec& v, int k, E e) {
  if constexpr (sizeof(Vec) == sizeof(E)) {
    v = e;
  } else {
    v[k] = e;
  }
}

// ---------------------------------------------------------------- compensated sums

// Unevaluated pair s + c carrying a running sum and its accumulated
// rounding errors (the cascaded "Sum2"/"Dot2" scheme of Ogita, Rump & Oishi,
// SIAM J. Sci. Comput. 2005).
template <class C>
struct DW {
  C s;
  C c;
};

// Knuth's branch-free TwoSum: t + e == a + b exactly.
template <class C>
__device__ __forceinline__ void two_sum(C a, C b, C& t, C& e) {
  t = a + b;
  C z = t - a;
  e = (a - (t - z)) + (b - z);
}

template <class C>
__device__ __forceinline__ void dw_acc(DW<C>& a, C v) {
  C t, e;
  two_sum(a.s, v, t, e);
  a.s = t;
  a.c += e;
}

// Accumulate the exact product x*y: p + q == x*y (q from a fused multiply-add).
template <class C>
__device__ __forceinline__ void dw_acc_prod(DW<C>& a, C x, C y) {
  C p = x * y;
  C q = __builtin_fma(x, y, -p);
  dw_acc(a, p);
  a.c += q;
}

template <class C>
__device__ __forceinline__ DW<C> dw_add(DW<C> a, DW<C> b) {
  C t, e;
  two_sum(a.s, b.s, t, e);
  return DW<C>{t, (a.c + b.c) + e};
}

template <class C>
__device__ __forceinline__ DW<C> wave_reduce(DW<C> a) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    DW<C> b{__shfl_xor(a.s, off, kWave), __shfl_xor(a.c, off, kWave)};
    a = dw_add(a, b);
  }
  return a;
}

// Workgroup-wide reduction in a fixed order; the result is valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ DW<double> block_reduce(DW<double> a) {
  constexpr int NW = BLOCK / kWave;
  __shared__ double s_s[NW], s_c[NW];
  a = wave_reduce(a);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (lane == 0) {
    s_s[w] = a.s;
    s_c[w] = a.c;
  }
  __syncthreads();
  DW<double> r{0.0, 0.0};
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NW; ++i) r = dw_add(r, DW<double>{s_s[i], s_c[i]});
  }
  return r;
}

// End of the first stage of a grid reduction: the workgroup's compensated
// pair goes to partials[blockIdx.x]; a grid of one workgroup writes the
// rounded sum to *out directly.  The second stage (a separate launch, so the
// kernel boundary orders it after every workgroup of the first) adds the
// pairs in index order.  The result depends only on the grid size, never on
// the order in which workgroups ran, and no atomics or fences are involved.
template <int BLOCK>
__device__ __forceinline__ void block_store_pair(DW<double> a, double* partials, double* out) {
  a = block_reduce<BLOCK>(a);
  if (threadIdx.x == 0) {
    if (gridDim.x == 1) {
      *out = a.s + a.c;
    } else {
      partials[2 * blockIdx.x] = a.s;
      partials[2 * blockIdx.x + 1] = a.c;
    }
  }
}

// The same with the second stage folded into the launch (the small-size
// regime: one launch instead of two): with a counter, each workgroup
// publishes its pair and takes a ticket, and the workgroup that arrives last
// adds all gridDim.x pairs in index order (thread t takes pairs t, t + BLOCK,
// ..., then the workgroup tree), writes *out and resets the counter for the
// next launch.  No workgroup waits for another.  A NULL counter keeps the
// two-launch form.
template <int BLOCK>
__device__ __forceinline__ void block_finish(DW<double> a, double* partials, unsigned int* counter, double* out) {
  if (!counter || gridDim.x == 1) {
    block_store_pair<BLOCK>(a, partials, out);
    return;
  }
  __shared__ int s_last;
  a = block_reduce<BLOCK>(a);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a.s;
    partials[2 * blockIdx.x + 1] = a.c;
    // release: the pair is visible before the ticket; only the last
    // workgroup needs the acquire that makes every pair visible to it
    const unsigned int prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == gridDim.x - 1;
    if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (!s_last) return;
  DW<double> r{0.0, 0.0};
  for (int i = threadIdx.x; i < static_cast<int>(gridDim.x); i += BLOCK)
    r = dw_add(r, DW<double>{partials[2 * i], partials[2 * i + 1]});
  r = block_reduce<BLOCK>(r);
  if (threadIdx.x == 0) {
    *out = r.s + r.c;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Streaming (nontemporal) accesses for data touched exactly once.
template <class T>
__device__ __forceinline__ T ld_nt(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void st_nt(T* p, const T& v) {
  __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------- launch geometry

// Workgroups are dispatched round-robin over the 8 XCDs (hardware id p runs
// on XCD p % 8).  Renumber them so that each XCD works through one
// contiguous range of logical blocks: neighbouring blocks, which touch
// neighbouring data, then share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t p, uint32_t G) {
  constexpr uint32_t X = 8;
  const uint32_t q = G / X, r = G % X;
  const uint32_t x = p % X, i = p / X;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// In each group of 2048 dispatch ids, the 256 that one XCD receives (the same
// p % 8) take 256 consecutive block numbers; a ragged last group keeps the
// dispatch order.  Each XCD works through runs of neighbouring blocks while
// the grid as a whole still sweeps the data front to back.
__device__ __forceinline__ uint32_t group_block(uint32_t p, uint32_t G) {
  constexpr uint32_t kGroup = 2048, X = 8;
  if (p >= G / kGroup * kGroup) return p;
  const uint32_t r = p % kGroup;
  return (p - r) + (r % X) * (kGroup / X) + r / X;
}

// Block number of dispatch id p under workgroup order 0 (as dispatched),
// 1 (group_block) or 2 (xcd_block).
__device__ __forceinline__ uint32_t block_order(uint32_t p, uint32_t G, int order) {
  return order == 1 ? group_block(p, G) : order == 2 ? xcd_block(p, G) : p;
}

}  // namespace dev
}  // namespace bs
