// The shifted 7-point operator y = (6 + shift) x - (six neighbours) on an m^3
// grid of unknowns (index i + m(j + m k), zero Dirichlet ghosts), with an
// optional fused direction update and p.Ap reduction for CG.
//
// The additions run in a fixed order: centre term, then the neighbours at
// i-1, i+1, j-1, j+1, k-1, k+1 (absent neighbours skipped), with the diagonal
// computed in binary64 and rounded once to the working precision.  Every
// kernel here follows that order, so all of them give the same bits.
//
// Plane-chunk kernel.  Flatten a plane to the index f = i + m j.  A
// workgroup owns 256 S consecutive points of it (a run of whole or partial
// rows) and one chunk of k planes.  Its window [a - m, a + P + m) of each
// plane -- own points plus one row on either side -- is contiguous in
// memory, so each plane is fetched as whole cache lines and staged in LDS
// (two buffers, one per plane parity); i-1, i+1, j-1 and j+1 are read from
// LDS and k-1, k+1 stay in registers while the workgroup marches through its
// k chunk.  Loads run D planes ahead of the plane being computed (a ring of
// registers).  Every LDS read is in bounds, so the neighbour terms are read
// unconditionally and selected; only the last chunk of a plane is partial,
// and only it pays for per-point guards.  The number of k chunks is chosen
// so that every workgroup is resident at once.
#pragma once

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace stencil {

using dev::DW;
using dev::Storage;

// Scalars of a CG solve, kept on the device.  The kernels of an iteration
// compute the scalars they need from the previous kernel's partial sums
// (each workgroup adds them itself, in one fixed order, so all get the same
// bits); the values an iteration writes go to the slot of its parity, so
// that no kernel reads a field that another workgroup of the same kernel
// writes (done aside: it only ever changes from 0, every workgroup takes the
// same decision, and it is read and written atomically).
struct CgState {
  double rr_slot[2];  // r.r at the start of the iterations of parity 0 and 1
  double rr;          // the latest r.r (for the host)
  double pAp;         // p.Ap of the latest direction
  double alpha;
  double beta;
  double stop_rr;     // iterate while rr > stop_rr
  int32_t done;       // 0 running, 1 converged or out of iterations, 2 breakdown
  int32_t iters;      // completed updates, written by the update kernel only
  int32_t max_iters;
  int32_t fresh;      // 1 until the first update of a run (its direction is p = r)
  double rr0;         // r.r at the start of the run (for the host's batch sizes)
  double outer_rr;    // refinement: r.r of the binary64 residual the run started from
};

// Where a kernel finds the partial sums of the previous one: G compensated
// pairs, and the parity slot it reads or writes.
struct CgLink {
  const double* partials;
  int32_t G;
  int32_t slot;
};

// The done flag as thread 0 read it and, while it is 0, the sum of G
// compensated pairs added in index order per thread and then across the
// workgroup (the same order in every workgroup), both given to every thread.
struct Bcast {
  double v;
  int32_t done;
};

__device__ __forceinline__ Bcast block_sum_bcast(const double* __restrict__ partials, int G, const int32_t* done) {
  __shared__ double s_v;
  __shared__ int32_t s_done;
  // once the solve is over (the rest of a captured batch) the pairs are not read
  if (threadIdx.x == 0) s_done = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int32_t d = s_done;
  if (d) return Bcast{0.0, d};
  DW<double> r{0.0, 0.0};
  for (int i = threadIdx.x; i < G; i += kBlock) r = dev::dw_add(r, DW<double>{partials[2 * i], partials[2 * i + 1]});
  r = dev::block_reduce<kBlock>(r);
  if (threadIdx.x == 0) s_v = r.s + r.c;
  __syncthreads();
  return Bcast{s_v, 0};
}

__device__ __forceinline__ void set_done(CgState* st, int32_t v) {
  __hip_atomic_store(&st->done, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Algorithm 1 step 10 and the stopping test, at the head of the kernel that
// forms the next direction: r'.r' from the update's partial sums, beta =
// r'.r' / r.r (0 for the first direction of a run).  Returns false when the
// solve is over; every thread of a workgroup returns the same.
__device__ __forceinline__ bool cg_beta(CgState* st, CgLink in, double* beta) {
  const Bcast b = block_sum_bcast(in.partials, in.G, &st->done);
  if (b.done) return false;
  if (st->fresh) {
    *beta = 0.0;
    return true;
  }
  const double rr_new = b.v, rr_old = st->rr_slot[in.slot ^ 1];
  int32_t done = 0;
  if (!__builtin_isfinite(rr_new))
    done = 2;  // overflow or NaN: further iterations cannot recover
  else if (rr_new <= st->stop_rr || st->iters >= st->max_iters)
    done = 1;
  const double bt = rr_new / rr_old;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rr_slot[in.slot] = rr_new;
    st->rr = rr_new;
    st->beta = bt;
    if (done) set_done(st, done);
  }
  *beta = bt;
  return done == 0;
}

// Algorithm 1 step 7 at the head of the update kernel: p.Ap from the
// operator's partial sums, alpha = r.r / p.Ap.  Returns false when the solve
// is over or p.Ap is not positive (breakdown).
__device__ __forceinline__ bool cg_alpha(CgState* st, CgLink in, double* alpha) {
  const Bcast b = block_sum_bcast(in.partials, in.G, &st->done);
  if (b.done) return false;
  const double pAp = b.v;
  const bool ok = pAp > 0.0;  // A is positive definite on p unless p vanished
  const double a = st->rr_slot[in.slot] / pAp;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->pAp = pAp;
    if (ok) {
      st->alpha = a;
      st->iters += 1;
      st->fresh = 0;
    } else {
      set_done(st, 2);
    }
  }
  *alpha = a;
  return ok;
}

// Values the operator is applied to: the stored p, or (DIR) the new
// direction r + beta p rounded to storage exactly as an AXPY rounds it.
template <class T, bool DIR>
struct Source {
  using S = Storage<T>;
  using E = typename S::E;
  using C = typename S::C;
  const E* __restrict__ p;
  const E* __restrict__ r;
  C beta;
  __device__ __forceinline__ C at(int64_t g) const {
    if constexpr (DIR) {
      return S::load(S::store(C(1) * S::load(r[g]) + beta * S::load(p[g])));
    } else {
      return S::load(p[g]);
    }
  }
};

// First stage of a reduction whose second stage is a separate launch.
__device__ __forceinline__ void store_partial(DW<double> a, double* partials) {
  a = dev::block_reduce<kBlock>(a);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a.s;
    partials[2 * blockIdx.x + 1] = a.c;
  }
}

// Halo values per thread and plane: 2m <= H * 256.
template <int H>
inline bool halo_fits(int64_t m) {
  return 2 * m <= static_cast<int64_t>(H) * kBlock;
}

// Geometry of one launch: each plane is cut into chunks of 256 S points of
// the flattened index i + m j, and the k range into chunks of klen planes.
struct Plan7 {
  int32_t m;       // grid side
  int32_t nchunk;  // point chunks per plane
  int32_t klen;    // planes per k chunk
  int32_t pad;
};

constexpr size_t kPlaneLdsMax = 65536;

// LDS bytes of one workgroup: two plane windows of 256 S + 2m values.
template <class T, int S>
inline size_t plane_lds_bytes(int64_t m) {
  return 2 * static_cast<size_t>(kBlock * S + 2 * m) * sizeof(typename Storage<T>::E);
}

template <class T, int S, int H>
inline bool plane_fits(int64_t m) {
  return m >= 1 && halo_fits<H>(m) && plane_lds_bytes<T, S>(m) <= kPlaneLdsMax;
}

// Cut the grid so that all workgroups are resident at once.
template <int S>
inline Plan7 plan7_for(int64_t m, int64_t resident_blocks, int64_t* blocks) {
  Plan7 g{};
  g.m = static_cast<int32_t>(m);
  const int64_t per = static_cast<int64_t>(kBlock) * S;
  g.nchunk = static_cast<int32_t>((m * m + per - 1) / per);
  int64_t nkc = resident_blocks / g.nchunk;
  if (nkc > m) nkc = m;
  if (nkc < 1) nkc = 1;
  g.klen = static_cast<int32_t>((m + nkc - 1) / nkc);
  nkc = (m + g.klen - 1) / g.klen;
  *blocks = static_cast<int64_t>(g.nchunk) * nkc;
  return g;
}

// Loads of one plane into the register ring: the thread's own points (as
// storage values) and its halo values.
template <class T, bool DIR, int S, int H>
struct PlaneRegs {
  typename Storage<T>::E own[S];
  typename Storage<T>::E halo[H];
};

template <class T, bool DIR>
__device__ __forceinline__ typename Storage<T>::E fetch(const Source<T, DIR>& src, int64_t g) {
  using St = Storage<T>;
  if constexpr (DIR) {
    return St::store(typename St::C(1) * St::load(src.r[g]) + src.beta * St::load(src.p[g]));
  } else {
    return src.p[g];
  }
}

// The march of one workgroup.  FULL: the chunk holds 256 S points, so no
// point needs a guard.
template <class T, bool DOT, bool DIR, int S, int H, int D, bool FULL>
__device__ __forceinline__ void march7(const Plan7& pl, typename Storage<T>::C c, const Source<T, DIR>& src,
                                       typename Storage<T>::E* __restrict__ p_new,
                                       typename Storage<T>::E* __restrict__ y, int64_t a, int32_t P, int32_t k0,
                                       int32_t k1, typename Storage<T>::E* cur, typename Storage<T>::E* nxt,
                                       DW<typename Storage<T>::C>& acc) {
  using St = Storage<T>;
  using C = typename St::C;
  using E = typename St::E;
  const int t = threadIdx.x;
  const int32_t m = pl.m;
  const int64_t plane = static_cast<int64_t>(m) * m;
  // window of one plane in LDS: slot m + (f - a) for flattened f in [a - m, a + P + m)
  int32_t q[S];
  bool has_l[S], has_r[S], has_d[S], has_u[S], ok[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    q[s] = t + kBlock * s;
    ok[s] = FULL || q[s] < P;
    const int64_t f = a + (ok[s] ? q[s] : P - 1);
    const int32_t i = static_cast<int32_t>(f % m), j = static_cast<int32_t>(f / m);
    has_l[s] = i > 0;
    has_r[s] = i < m - 1;
    has_d[s] = j > 0;
    has_u[s] = j < m - 1;
    if (!FULL && !ok[s]) q[s] = P - 1;  // guarded points load a valid value and store nothing
  }
  int64_t hf[H];   // flattened index of halo value u, clamped into the plane
  int32_t hs[H];   // its LDS slot, or -1
#pragma unroll
  for (int u = 0; u < H; ++u) {
    const int32_t h = t + kBlock * u;
    const int64_t f = h < m ? a - m + h : a + P + (h - m);
    hs[u] = h < 2 * m ? static_cast<int32_t>(m + (f - a)) : -1;
    hf[u] = f < 0 ? 0 : (f >= plane ? plane - 1 : f);
  }
  // own values are needed up to plane k1 (the last k+1 term), halo values
  // only for planes the chunk stages; the tests are the same for the whole
  // workgroup, and skipped values are never read
  auto load_plane = [&](int32_t kp, PlaneRegs<T, DIR, S, H>& o) {
    const int64_t kpp = plane * kp;
    if (kp <= k1 && kp < m) {
#pragma unroll
      for (int s = 0; s < S; ++s) o.own[s] = fetch(src, a + q[s] + kpp);
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) o.own[s] = E{};
    }
    if (kp < k1) {
#pragma unroll
      for (int u = 0; u < H; ++u) o.halo[u] = fetch(src, hf[u] + kpp);
    } else {
#pragma unroll
      for (int u = 0; u < H; ++u) o.halo[u] = E{};
    }
  };
  auto stage = [&](E* buf, const PlaneRegs<T, DIR, S, H>& o) {
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (ok[s]) buf[m + q[s]] = o.own[s];
#pragma unroll
    for (int u = 0; u < H; ++u)
      if (hs[u] >= 0) buf[hs[u]] = o.halo[u];
  };

  E xm[S], xc[S];
  PlaneRegs<T, DIR, S, H> ring[D];
  {
    PlaneRegs<T, DIR, S, H> first;
#pragma unroll
    for (int s = 0; s < S; ++s) xm[s] = k0 > 0 ? fetch(src, a + q[s] + plane * (k0 - 1)) : E{};
    load_plane(k0, first);
#pragma unroll
    for (int s = 0; s < S; ++s) xc[s] = first.own[s];
#pragma unroll
    for (int d = 0; d < D; ++d) load_plane(k0 + 1 + d, ring[d]);
    stage(cur, first);
  }
  __syncthreads();

  for (int32_t k = k0; k < k1; ++k) {
    PlaneRegs<T, DIR, S, H> nx;
    load_plane(k + 1 + D, nx);
    const int64_t gk = a + plane * k;
    const bool has_b = k > 0, has_f = k + 1 < m;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int32_t l = m + q[s];
      const C il = St::load(cur[l - 1]), ir = St::load(cur[l + 1]);
      const C jd = St::load(cur[l - m]), ju = St::load(cur[l + m]);
      const C x0 = St::load(xc[s]);
      C v = c * x0;
      v = has_l[s] ? v - il : v;
      v = has_r[s] ? v - ir : v;
      v = has_d[s] ? v - jd : v;
      v = has_u[s] ? v - ju : v;
      if (has_b) v -= St::load(xm[s]);
      if (has_f) v -= St::load(ring[0].own[s]);
      const E ys = St::store(v);
      if (ok[s]) {
        y[gk + q[s]] = ys;
        if constexpr (DIR) p_new[gk + q[s]] = xc[s];
        if constexpr (DOT) dev::dw_acc_prod(acc, x0, St::load(ys));
      }
    }
    if (k + 1 < k1) stage(nxt, ring[0]);
    __syncthreads();
    E* tmp = cur;
    cur = nxt;
    nxt = tmp;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      xm[s] = xc[s];
      xc[s] = ring[0].own[s];
    }
#pragma unroll
    for (int d = 0; d + 1 < D; ++d) ring[d] = ring[d + 1];
    ring[D - 1] = nx;
  }
}

// S points per thread, H halo values per thread, loads issued D planes ahead.
template <class T, bool DOT, bool DIR, int S, int H, int D>
__global__ __launch_bounds__(kBlock) void k_plane7(Plan7 pl, typename Storage<T>::C c,
                                                   const typename Storage<T>::E* __restrict__ p,
                                                   const typename Storage<T>::E* __restrict__ r,
                                                   typename Storage<T>::E* __restrict__ p_new,
                                                   typename Storage<T>::E* __restrict__ y, double* partials,
                                                   CgState* st, CgLink link) {
  using St = Storage<T>;
  using C = typename St::C;
  using E = typename St::E;
  extern __shared__ __align__(16) unsigned char plane_lds[];
  double beta = 0.0;
  if constexpr (DIR) {
    if (!cg_beta(st, link, &beta)) return;
  } else {
    if (st && st->done) return;
  }
  const Source<T, DIR> src{p, r, static_cast<C>(beta)};
  const int32_t m = pl.m;
  const int64_t plane = static_cast<int64_t>(m) * m;
  const uint32_t b = dev::xcd_block(blockIdx.x, gridDim.x);
  const int32_t chunk = static_cast<int32_t>(b % pl.nchunk);
  const int32_t kc = static_cast<int32_t>(b / pl.nchunk);
  const int64_t a = static_cast<int64_t>(chunk) * kBlock * S;
  const int32_t P = static_cast<int32_t>(plane - a < kBlock * S ? plane - a : kBlock * S);
  const int32_t k0 = kc * pl.klen;
  const int32_t k1 = (k0 + pl.klen < m) ? k0 + pl.klen : m;
  E* cur = reinterpret_cast<E*>(plane_lds);
  E* nxt = cur + (kBlock * S + 2 * m);
  DW<C> acc{C(0), C(0)};
  if (P == kBlock * S)
    march7<T, DOT, DIR, S, H, D, true>(pl, c, src, p_new, y, a, P, k0, k1, cur, nxt, acc);
  else
    march7<T, DOT, DIR, S, H, D, false>(pl, c, src, p_new, y, a, P, k0, k1, cur, nxt, acc);
  if constexpr (DOT) store_partial(DW<double>{static_cast<double>(acc.s), static_cast<double>(acc.c)}, partials);
}

// ---------------------------------------------------------------- row-segment march

// Fallback for grids too wide for the plane-chunk window.  A wave owns a
// 64-point segment of one grid row and marches through a chunk of k planes,
// keeping k-1, k and k+1 in registers; i-1 and i+1 come from the neighbouring
// lanes (one extra load at each end of the segment) and j-1, j+1 from the
// caches.  Item w has j = w mod m, then segment, then chunk.
constexpr int kMarchUnroll = 4;

struct March {
  int32_t m, nseg, klen;
  int64_t items;
};

inline March march_for(int64_t m, int64_t resident_waves, int64_t* blocks) {
  March g;
  g.m = static_cast<int32_t>(m);
  g.nseg = static_cast<int32_t>((m + 63) / 64);
  const int64_t cols = m * g.nseg;
  int64_t nkc = resident_waves / cols;
  if (nkc > m) nkc = m;
  if (nkc < 1) nkc = 1;
  g.klen = static_cast<int32_t>((m + nkc - 1) / nkc);
  nkc = (m + g.klen - 1) / g.klen;
  g.items = cols * nkc;
  *blocks = (g.items + 3) / 4;
  return g;
}

template <class T, bool DOT, bool DIR>
__global__ __launch_bounds__(kBlock) void k_march7(March gm, typename Storage<T>::C c,
                                                   const typename Storage<T>::E* __restrict__ p,
                                                   const typename Storage<T>::E* __restrict__ r,
                                                   typename Storage<T>::E* __restrict__ p_new,
                                                   typename Storage<T>::E* __restrict__ y, double* partials,
                                                   CgState* st, CgLink link) {
  using St = Storage<T>;
  using C = typename St::C;
  using E = typename St::E;
  double beta = 0.0;
  if constexpr (DIR) {
    if (!cg_beta(st, link, &beta)) return;
  } else {
    if (st && st->done) return;
  }
  const Source<T, DIR> src{p, r, static_cast<C>(beta)};
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t w = static_cast<int64_t>(dev::xcd_block(blockIdx.x, gridDim.x)) * 4 + wave;
  const int32_t m = gm.m;
  const int32_t j = static_cast<int32_t>(w % m);
  const int64_t rest = w / m;
  const int32_t seg = static_cast<int32_t>(rest % gm.nseg);
  const int32_t kc = static_cast<int32_t>(rest / gm.nseg);
  const int32_t i = seg * 64 + lane;
  const int32_t k0 = kc * gm.klen;
  const int32_t k1 = (k0 + gm.klen < m) ? k0 + gm.klen : m;
  const int64_t plane = static_cast<int64_t>(m) * m;
  const bool active = w < gm.items;  // the same for every lane of the wave
  const bool valid = active && i < m;
  DW<C> acc{C(0), C(0)};
  if (active) {
    int64_t g = i + static_cast<int64_t>(m) * j + plane * k0;
    C xm = (valid && k0 > 0) ? src.at(g - plane) : C(0);
    C xc = valid ? src.at(g) : C(0);
    for (int32_t k = k0; k < k1; k += kMarchUnroll) {
      C xn[kMarchUnroll], jm[kMarchUnroll], jp[kMarchUnroll], lf[kMarchUnroll], rt[kMarchUnroll];
#pragma unroll
      for (int u = 0; u < kMarchUnroll; ++u) {
        const int32_t kk = k + u;
        const int64_t gg = g + plane * u;
        const bool act = valid && kk < k1;
        xn[u] = (act && kk + 1 < m) ? src.at(gg + plane) : C(0);
        jm[u] = (act && j > 0) ? src.at(gg - m) : C(0);
        jp[u] = (act && j < m - 1) ? src.at(gg + m) : C(0);
        lf[u] = (act && lane == 0 && i > 0) ? src.at(gg - 1) : C(0);
        rt[u] = (act && lane == 63 && i + 1 < m) ? src.at(gg + 1) : C(0);
      }
#pragma unroll
      for (int u = 0; u < kMarchUnroll; ++u) {
        const int32_t kk = k + u;
        if (kk >= k1) break;
        // every lane takes part in both shuffles: a lane that sat one out
        // would leave its neighbour nothing to read
        const C up = __shfl_up(xc, 1, 64);
        const C down = __shfl_down(xc, 1, 64);
        const C left = lane == 0 ? lf[u] : up;
        const C right = lane == 63 ? rt[u] : down;
        if (valid) {
          C v = c * xc;
          if (i > 0) v -= left;
          if (i < m - 1) v -= right;
          if (j > 0) v -= jm[u];
          if (j < m - 1) v -= jp[u];
          if (kk > 0) v -= xm;
          if (kk < m - 1) v -= xn[u];
          const E ys = St::store(v);
          y[g] = ys;
          if constexpr (DIR) p_new[g] = St::store(xc);
          if constexpr (DOT) dev::dw_acc_prod(acc, xc, St::load(ys));
        }
        xm = xc;
        xc = xn[u];
        g += plane;
      }
    }
  }
  if constexpr (DOT) store_partial(DW<double>{static_cast<double>(acc.s), static_cast<double>(acc.c)}, partials);
}

// ---------------------------------------------------------------- host-side launch

// Points per thread and planes in flight of the plane-chunk kernel, per
// storage type (measured on the 225^3 grid).
template <class T> struct PlaneCfg;
template <> struct PlaneCfg<double> { static constexpr int S = 4, D = 1; };
template <> struct PlaneCfg<float> { static constexpr int S = 4, D = 2; };
template <> struct PlaneCfg<dev::bf16> { static constexpr int S = 4, D = 2; };

// Workgroups of a kernel that fit on the device at once.
template <class K>
inline int64_t resident_blocks(K kernel, size_t lds, int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 256;
  }
  return static_cast<int64_t>(per_cu) * cus;
}

// One prepared operator application for grid side m: the plane-chunk kernel
// with 2, 4 or 12 halo registers, or the row-segment march beyond that.
template <class T, bool DOT, bool DIR>
struct Op7 {
  using St = Storage<T>;
  using E = typename St::E;
  using C = typename St::C;
  static constexpr int S = PlaneCfg<T>::S, D = PlaneCfg<T>::D;
  int kind = 0;
  Plan7 plan{};
  March march{};
  unsigned int blocks = 0;
  size_t lds = 0;

  template <int H>
  bool try_plane(int64_t m, int device, int k) {
    if (!plane_fits<T, S, H>(m)) return false;
    int64_t b = 0;
    lds = plane_lds_bytes<T, S>(m);
    plan = plan7_for<S>(m, resident_blocks(k_plane7<T, DOT, DIR, S, H, D>, lds, device), &b);
    blocks = static_cast<unsigned int>(b);
    kind = k;
    return true;
  }

  // Returns false if the grid needs more workgroups than a reduction takes.
  bool prepare(int64_t m, int device) {
    if (!(try_plane<2>(m, device, 0) || try_plane<4>(m, device, 1) || try_plane<12>(m, device, 2))) {
      int64_t b = 0;
      march = march_for(m, 4 * resident_blocks(k_march7<T, DOT, DIR>, 0, device), &b);
      if (b > 0x7fffffff) return false;
      blocks = static_cast<unsigned int>(b);
      lds = 0;
      kind = 3;
    }
    return !DOT || blocks <= static_cast<unsigned int>(kMaxReduceBlocks);
  }

  void enqueue(hipStream_t st, double shift, const E* p, const E* r, E* p_new, E* y, double* partials,
               CgState* cs, CgLink link = CgLink{nullptr, 0, 0}) const {
    const C c = static_cast<C>(6.0 + shift);
    switch (kind) {
      case 0:
        hipLaunchKernelGGL((k_plane7<T, DOT, DIR, S, 2, D>), dim3(blocks), dim3(kBlock), lds, st, plan, c, p, r, p_new,
                           y, partials, cs, link);
        break;
      case 1:
        hipLaunchKernelGGL((k_plane7<T, DOT, DIR, S, 4, D>), dim3(blocks), dim3(kBlock), lds, st, plan, c, p, r, p_new,
                           y, partials, cs, link);
        break;
      case 2:
        hipLaunchKernelGGL((k_plane7<T, DOT, DIR, S, 12, D>), dim3(blocks), dim3(kBlock), lds, st, plan, c, p, r,
                           p_new, y, partials, cs, link);
        break;
      default:
        hipLaunchKernelGGL((k_march7<T, DOT, DIR>), dim3(blocks), dim3(kBlock), 0, st, march, c, p, r, p_new, y,
                           partials, cs, link);
        break;
    }
  }
};

}  // namespace stencil
}  // namespace bs
