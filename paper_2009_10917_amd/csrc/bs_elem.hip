// Element operators of the Helmholtz problem (Section 2, eqs. helm_var,
// global_system, assembled_stiff, assembled_mass) inside the scattered form
// of CG: y_G = Z^T A_L Z x_G with A_L block diagonal.
//
// Basis: the tensor-product Lagrange polynomials through the N+1
// Gauss-Lobatto-Legendre (GLL) points of each axis; element integrals with
// the Q = N+1 point Gauss-Legendre rule, exact for products of two
// degree-N polynomials, on affine hexahedra.  Per element the factors
// (G11, G12, G13, G22, G23, G33, |J|), G = |J| J^-1 J^-T, give
//   A^e u = sum_{d,d'} A_d^T W G_dd' A_d' u + lambda |J| Bq^T W Bq u
// with Bq = B x B x B, A_1 = B x B x D (derivative along the first local
// axis), A_2 = B x D x B, A_3 = D x B x B, W the product Gauss weights,
// B[a][i] = l_i(xi_a) and D[a][i] = l_i'(xi_a).
//
// The local operator is applied by sum factorisation in collocated form:
// with Dh = D B^-1, the differentiation matrix of the Lagrange basis through
// the Gauss points (computed from its closed form, no inversion),
//   U = (B, B, B) u,  G1 = (B, B, D) u,  G2 = Dh_j U,  G3 = Dh_k U,
//   V0 = lambda |J| W U,  V_d = W sum_d' G_dd' G_d',
//   y = (B, B, B)^T (V0 + Dh_k^T V3 + Dh_j^T V2) + (B, B, D)^T V1,
// ten one-axis contractions of 8 x 8 matrices with the 8^3 element tensor
// (degrees below 7 are padded with zeros to 8 points per axis).  Each
// contraction runs on the matrix cores: V_MFMA_F64_16X16X4F64 multiplies a
// 16 x 4 block of the 1D matrix (two stacked 8-row matrices, or one with
// zero rows) by a 4 x 16 block of the tensor viewed as 8 x 64, so a
// contraction is eight MFMAs.  One wave holds one element; the tensor moves
// between contractions through the wave's own LDS, padded (one spare
// double per 8) so that every access pattern is free of bank conflicts.
//
// The scatter is fused into the load (x_L is never written): a wave reads
// its element's map entries and the x_G values they name.  The local result
// y_L is written once and summed by the gather (Listing 4), which adds the
// copies of each global node in ascending local index as BS6 does.
//
// The lumped mass (the GLL rule put on the nodes, so the block is diagonal
// with d_l = |J_e| w_i w_j w_k) needs no local vector at all: y_G[g] adds
// d_l x_G[g] over the copies l of g in ascending l, one fused pass over the
// CSR of Z^T that reads x_G once and writes y_G once.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

typedef double dvec4 __attribute__((ext_vector_type(4)));

constexpr int kAx = 8;                 // points per axis of the padded tensor
constexpr int kTen = kAx * kAx * kAx;  // 512
constexpr int kTenPad = kTen + kTen / 8;  // one spare double per 8: 576
constexpr int kWavesPerBlock = 4;

// Operand matrices, each stored as 16 rows x 16 columns (row-major) so that
// lane l of chunk h reads row l % 16, column 4h + l / 16.
enum { kTabB = 0, kTabBD, kTabDh, kTabDhT, kTabBtDt, kTabBt, kTabCount };
constexpr int kTabSize = 16 * 16;

// ---------------------------------------------------------------- host: 1D rules

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, long double x, long double& p, long double& dp) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) {
    p = 1.0L;
    dp = 0.0L;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const long double pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0L);  // valid off the end points
}

// Gauss-Legendre: roots of P_q by Newton from the Chebyshev-like guesses
// cos(pi (a + 3/4) / (q + 1/2)); weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_rule(int q, double* x, double* w) {
  for (int a = 0; a < q; ++a) {
    long double r = cosl(3.14159265358979323846264338327950288L * (a + 0.75L) / (q + 0.5L));
    long double p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(q, r, p, dp);
      const long double d = p / dp;
      r -= d;
      if (fabsl(d) < 1e-19L) break;
    }
    legendre(q, r, p, dp);
    x[q - 1 - a] = static_cast<double>(r);  // ascending
    w[q - 1 - a] = static_cast<double>(2.0L / ((1.0L - r * r) * dp * dp));
  }
}

// GLL: the end points and the roots of P_N' (Newton on P_N', whose
// derivative follows from the Legendre equation), weights
// 2 / (N (N+1) P_N(x)^2).
void gll_rule(int N, double* x, double* w) {
  x[0] = -1.0;
  x[N] = 1.0;
  for (int a = 1; a < N; ++a) {
    long double r = -cosl(3.14159265358979323846264338327950288L * a / N);  // Chebyshev-Lobatto guess
    for (int it = 0; it < 100; ++it) {
      long double p, dp;
      legendre(N, r, p, dp);
      // (1 - x^2) P'' = 2 x P' - N (N+1) P
      const long double d2 = (2.0L * r * dp - N * (N + 1.0L) * p) / (1.0L - r * r);
      const long double d = dp / d2;
      r -= d;
      if (fabsl(d) < 1e-19L) break;
    }
    x[a] = static_cast<double>(r);
  }
  for (int a = 0; a <= N; ++a) {
    long double p, dp;
    legendre(N, static_cast<long double>(x[a]), p, dp);
    w[a] = static_cast<double>(2.0L / (N * (N + 1.0L) * p * p));
  }
}

// Lagrange basis through nodes[0..n) at point t: value and derivative of l_j.
void lagrange(const long double* nodes, int n, int j, long double t, long double& v, long double& dv) {
  long double den = 1.0L, num = 1.0L, dnum = 0.0L;
  for (int m = 0; m < n; ++m) {
    if (m == j) continue;
    den *= nodes[j] - nodes[m];
    dnum = dnum * (t - nodes[m]) + num;  // product rule, accumulated
    num *= t - nodes[m];
  }
  v = num / den;
  dv = dnum / den;
}

// The operand tables of degree N (N <= 7), padded to 8 points per axis.
void build_tables(const bs_elem& el, double* tab) {
  const int P1 = el.N + 1, Q = el.N + 1;
  long double xg[16], xq[16];
  for (int a = 0; a < P1; ++a) xg[a] = el.gll_x[a];
  for (int a = 0; a < Q; ++a) xq[a] = el.gauss_x[a];
  long double B[8][8] = {}, D[8][8] = {}, Dh[8][8] = {};
  for (int a = 0; a < Q; ++a)
    for (int i = 0; i < P1; ++i) lagrange(xg, P1, i, xq[a], B[a][i], D[a][i]);
  // Dh[a][b] = lh_b'(xi_a), lh the Lagrange basis through the Gauss points
  for (int a = 0; a < Q; ++a)
    for (int b = 0; b < Q; ++b) {
      long double v, dv;
      lagrange(xq, Q, b, xq[a], v, dv);
      Dh[a][b] = dv;
    }
  std::memset(tab, 0, sizeof(double) * kTabCount * kTabSize);
  auto at = [&](int t, int r, int c) -> double& { return tab[t * kTabSize + r * 16 + c]; };
  for (int r = 0; r < 8; ++r)
    for (int c = 0; c < 8; ++c) {
      at(kTabB, r, c) = static_cast<double>(B[r][c]);
      at(kTabBD, r, c) = static_cast<double>(B[r][c]);
      at(kTabBD, r + 8, c) = static_cast<double>(D[r][c]);
      at(kTabDh, r, c) = static_cast<double>(Dh[r][c]);
      at(kTabDhT, r, c) = static_cast<double>(Dh[c][r]);
      at(kTabBtDt, r, c) = static_cast<double>(B[c][r]);
      at(kTabBtDt, r, c + 8) = static_cast<double>(D[c][r]);
      at(kTabBt, r, c) = static_cast<double>(B[c][r]);
    }
}

// ---------------------------------------------------------------- device: local operator

struct Geo {
  double g11, g12, g13, g22, g23, g33, detj;
};

struct Rule8 {
  double w[kAx];  // Gauss weights, zero beyond Q
};

// Address of tensor entry (i, j, k) in the padded layout.
__device__ __forceinline__ int tad(int i, int j, int k) { return i + 9 * j + 72 * k; }

// Entry (s along the contracted axis X, col = the two other indices, the
// lower one fastest) of a tensor, for X = 0 (i), 1 (j) or 2 (k).
template <int X>
__device__ __forceinline__ int pad_at(int s, int col) {
  const int lo = col & 7, hi = col >> 3;
  if constexpr (X == 0) return tad(s, lo, hi);
  if constexpr (X == 1) return tad(lo, s, hi);
  return tad(lo, hi, s);
}

// acc[t] (+)= A * In for the 4 column tiles of one contraction along X:
// chunk h reads In at (s = 4h + l/16, col = 16t + l%16); A's operand for
// chunk h is a[h].  The binary64 accumulator is interleaved: register v of
// lane l holds row l/16 + 4v of column 16t + l%16.
template <int X, int KC>
__device__ __forceinline__ void contract(const double* __restrict__ in, const double (&a)[KC], dvec4 (&acc)[4]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int h = 0; h < KC; ++h) {
      const double b = in[pad_at<X>(4 * h + (l >> 4), 16 * t + (l & 15))];
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], b, acc[t], 0, 0, 0);
    }
  }
}

// Rows row_off .. row_off + 7 of the accumulator go to rows 0..7 of out
// (row_off is 0 or 8, so registers v = row_off / 4 and row_off / 4 + 1).
template <int X>
__device__ __forceinline__ void store_rows(double* __restrict__ out, const dvec4 (&acc)[4], int row_off) {
  const int l = threadIdx.x & 63;
  const int v0 = row_off >> 2;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 2; ++v) out[pad_at<X>((l >> 4) + 4 * v, 16 * t + (l & 15))] = acc[t][v0 + v];
}

template <int X>
__device__ __forceinline__ void load_rows(const double* __restrict__ in, dvec4 (&acc)[4]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[t][v] = in[pad_at<X>((l >> 4) + 4 * v, 16 * t + (l & 15))];
    acc[t][2] = 0.0;
    acc[t][3] = 0.0;
  }
}

__device__ __forceinline__ void zero(dvec4 (&acc)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = dvec4{0.0, 0.0, 0.0, 0.0};
}

template <int KC>
__device__ __forceinline__ void operand(const double* __restrict__ tab, int which, double (&a)[KC]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int h = 0; h < KC; ++h) a[h] = tab[which * kTabSize + (l & 15) * 16 + 4 * h + (l >> 4)];
}

// Each element's tensor lives in its wave's own LDS buffers, so only the
// lanes of one wave exchange data between contractions: a wave's LDS
// operations are performed in order, and the fences and the wave barrier keep
// the compiler from moving them across this point (the waves of a workgroup
// never wait for one another).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per element, four elements per workgroup, the workgroups
// striding over the elements.  map/xG give the element's values (the fused
// scatter), yL receives A^e u.  With DOT (the CG form) the workgroup also
// leaves in partials[blockIdx.x] the compensated sum of u . A^e u over its
// elements, which adds up to p . Z^T A_L Z p since masked copies read u = 0;
// it returns at once when *done is set.
template <bool DOT>
__global__ __launch_bounds__(kWavesPerBlock * 64) void k_helm_local(
    const double* __restrict__ tab, Rule8 rule, const int32_t* __restrict__ map, int64_t n_global,
    const double* __restrict__ geo, double lambda, const double* __restrict__ xG, double* __restrict__ yL,
    int64_t n_elem, int P1, const int32_t* __restrict__ done, double* __restrict__ partials) {
  __shared__ double lds[kWavesPerBlock][4][kTenPad];
  if constexpr (DOT) {
    if (*done) return;  // set only between launches: every workgroup leaves here or none
  }
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  double* b0 = lds[wave][0];
  double* b1 = lds[wave][1];
  double* b2 = lds[wave][2];
  double* b3 = lds[wave][3];
  const int64_t P = static_cast<int64_t>(P1) * P1 * P1;
  double aB[2], aBD[2], aDh[2], aDhT[2], aBtDt[4], aBt[2];
  operand(tab, kTabB, aB);
  operand(tab, kTabBD, aBD);
  operand(tab, kTabDh, aDh);
  operand(tab, kTabDhT, aDhT);
  operand(tab, kTabBtDt, aBtDt);
  operand(tab, kTabBt, aBt);
  dev::DW<double> dot{0.0, 0.0};

  // The loads of an element are issued an iteration ahead of its work (its
  // map ids two ahead, since the x_G loads need them), so that their
  // latency hides behind the contractions of the element before.
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
  auto load_ids = [&](int64_t e, int32_t (&id)[8]) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int f = l + 64 * m, i = f & 7, j = (f >> 3) & 7, k = f >> 6;
      id[m] = (e < n_elem && i < P1 && j < P1 && k < P1) ? map[e * P + i + P1 * (j + P1 * k)] : -1;
    }
  };
  // masked, padding and out-of-range ids read 0
  auto load_vals = [&](const int32_t (&id)[8], double (&u)[8]) {
#pragma unroll
    for (int m = 0; m < 8; ++m) u[m] = (id[m] >= 0 && id[m] < n_global) ? xG[id[m]] : 0.0;
  };
  auto load_geo = [&](int64_t e) {
    if (e >= n_elem) return Geo{};
    const double* q = geo + 7 * e;
    return Geo{q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
  };
  const int64_t e_first = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave;
  int32_t id_next[8];
  double u_cur[8];
  Geo g_cur;
  load_ids(e_first, id_next);
  load_vals(id_next, u_cur);
  g_cur = load_geo(e_first);
  load_ids(e_first + stride, id_next);

  for (int64_t e0 = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock; e0 < n_elem; e0 += stride) {
    const int64_t e = e0 + wave;
    const bool live = e < n_elem;
    double u[8], u_next[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) u[m] = u_cur[m];
    const Geo g = g_cur;
    load_vals(id_next, u_next);
    g_cur = load_geo(e + stride);
    load_ids(e + 2 * stride, id_next);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int f = l + 64 * m;
      b0[tad(f & 7, (f >> 3) & 7, f >> 6)] = u[m];
    }
    wave_sync();
    dvec4 acc[4];
    // U = (B, B, B) u and G1 = (B, B, D) u: along k, along j, then [B; D] along i
    zero(acc);
    contract<2, 2>(b0, aB, acc);
    store_rows<2>(b1, acc, 0);
    wave_sync();
    zero(acc);
    contract<1, 2>(b1, aB, acc);
    store_rows<1>(b0, acc, 0);
    wave_sync();
    zero(acc);
    contract<0, 2>(b0, aBD, acc);
    store_rows<0>(b1, acc, 0);  // U
    store_rows<0>(b2, acc, 8);  // G1
    wave_sync();
    // G2 = Dh along j of U, G3 = Dh along k of U
    zero(acc);
    contract<1, 2>(b1, aDh, acc);
    store_rows<1>(b0, acc, 0);
    zero(acc);
    contract<2, 2>(b1, aDh, acc);
    store_rows<2>(b3, acc, 0);
    wave_sync();
    // quadrature-point values: V0 (b1), V1 (b2), V2 (b0), V3 (b3), in place
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int f = l + 64 * m, a = f & 7, b = (f >> 3) & 7, c = f >> 6;
      const int ad = tad(a, b, c);
      const double W = (rule.w[a] * rule.w[b]) * rule.w[c];
      const double U = b1[ad], d1 = b2[ad], d2 = b0[ad], d3 = b3[ad];
      b1[ad] = ((lambda * g.detj) * W) * U;
      b2[ad] = W * ((g.g11 * d1 + g.g12 * d2) + g.g13 * d3);
      b0[ad] = W * ((g.g12 * d1 + g.g22 * d2) + g.g23 * d3);
      b3[ad] = W * ((g.g13 * d1 + g.g23 * d2) + g.g33 * d3);
    }
    wave_sync();
    // W1 = V0 + Dh_k^T V3, then W2 = W1 + Dh_j^T V2 (accumulated in place in b1)
    load_rows<2>(b1, acc);
    contract<2, 2>(b3, aDhT, acc);
    wave_sync();
    store_rows<2>(b1, acc, 0);
    wave_sync();
    load_rows<1>(b1, acc);
    contract<1, 2>(b0, aDhT, acc);
    wave_sync();
    store_rows<1>(b1, acc, 0);
    wave_sync();
    // Y3 = B^T W2 + D^T V1 along i (K = 16: W2 then V1)
    zero(acc);
    {
      double lo[2] = {aBtDt[0], aBtDt[1]}, hi[2] = {aBtDt[2], aBtDt[3]};
      contract<0, 2>(b1, lo, acc);
      contract<0, 2>(b2, hi, acc);
    }
    store_rows<0>(b0, acc, 0);
    wave_sync();
    zero(acc);
    contract<1, 2>(b0, aBt, acc);
    store_rows<1>(b3, acc, 0);
    wave_sync();
    zero(acc);
    contract<2, 2>(b3, aBt, acc);
    if constexpr (DOT) {
      // y back through LDS into the load's layout, beside the lane's u
      store_rows<2>(b1, acc, 0);
      wave_sync();
      if (live) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int f = l + 64 * m, i = f & 7, j = (f >> 3) & 7, k = f >> 6;
          if (i < P1 && j < P1 && k < P1) {
            const double y = b1[tad(i, j, k)];
            dev::st_nt(yL + e * P + i + P1 * (j + P1 * k), y);
            dev::dw_acc_prod(dot, u[m], y);
          }
        }
      }
    } else if (live) {
      // y along k: register v < 2 of lane l holds node k = l/16 + 4v at
      // (i, j) = (col % 8, col / 8); registers 2 and 3 hold the padding rows
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = 16 * t + (l & 15), i = col & 7, j = col >> 3;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int k = (l >> 4) + 4 * v;
          if (i < P1 && j < P1 && k < P1) dev::st_nt(yL + e * P + i + P1 * (j + P1 * k), acc[t][v]);
        }
      }
    }
    wave_sync();  // this element's LDS reads before the next element's writes
#pragma unroll
    for (int m = 0; m < 8; ++m) u_cur[m] = u_next[m];
  }
  if constexpr (DOT) {
    dot = dev::block_reduce<kWavesPerBlock * 64>(dot);
    if (threadIdx.x == 0) {
      partials[2 * blockIdx.x] = dot.s;
      partials[2 * blockIdx.x + 1] = dot.c;
    }
  }
}

// ---------------------------------------------------------------- device: lumped mass

struct Gll16 {
  double w[16];
};

// Rows of the CSR of Z^T in global order, nonzero-balanced blocks (the
// gather's blockStarts split): the workgroup computes d_l of every column of
// its window from the column's element and node, stages them in LDS, and
// each thread adds d_l x_G[g] over its rows' copies in CSR order from +0.0.
__global__ __launch_bounds__(kBlock) void k_mass_lumped(const int32_t* __restrict__ rs, const int32_t* __restrict__ ci,
                                                        const int32_t* __restrict__ bstart, const double* __restrict__ geo,
                                                        Gll16 gw, int P1, const double* __restrict__ xG,
                                                        double* __restrict__ yG, int64_t chunk, int64_t nnz) {
  constexpr int L = kStage / kBlock;
  __shared__ double lds[kStage];
  const int64_t b = blockIdx.x;
  const int64_t w0 = b * chunk;
  const int P = P1 * P1 * P1;
  if (w0 < nnz) {
    int32_t col[L];
#pragma unroll
    for (int k = 0; k < L; ++k) col[k] = dev::ld_nt(ci + min(w0 + threadIdx.x + k * kBlock, nnz - 1));
    double dj[L];
#pragma unroll
    for (int k = 0; k < L; ++k) dj[k] = geo[7 * static_cast<int64_t>(col[k] / P) + 6];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int q = col[k] % P;
      const int i = q % P1, j = (q / P1) % P1, kk = q / (P1 * P1);
      const double d = ((gw.w[i] * gw.w[j]) * gw.w[kk]) * dj[k];
      if (w0 + threadIdx.x + k * kBlock < nnz) lds[threadIdx.x + k * kBlock] = d;
    }
  }
  const int32_t r0 = bstart[b], r1 = bstart[b + 1];
  __syncthreads();
  for (int32_t q = r0 + threadIdx.x; q < r1; q += kBlock) {
    const int32_t a = rs[q], z = rs[q + 1];
    const double x = xG[q];
    double s = 0.0;
    if (a >= w0 && z <= w0 + kStage) {
      for (int32_t c = a; c < z; ++c) s += lds[c - w0] * x;
    } else {
      for (int32_t c = a; c < z; ++c) {
        const int32_t l = ci[c], qq = l % P;
        const int i = qq % P1, j = (qq / P1) % P1, kk = qq / (P1 * P1);
        s += (((gw.w[i] * gw.w[j]) * gw.w[kk]) * geo[7 * static_cast<int64_t>(l / P) + 6]) * x;
      }
    }
    dev::st_nt(yG + q, s);
  }
}

inline unsigned int ceil_div(int64_t a, int64_t b) { return static_cast<unsigned int>((a + b - 1) / b); }

bs_status check_elem(const char* op, bs_ctx* ctx, const bs_elem* el) {
  bs_status s;
  if ((s = check_ctx(ctx, op))) return s;
  if (!el) return fail(BS_ERR_INVALID_ARG, "%s: element object is NULL", op);
  if (el->device != ctx->device) return fail(BS_ERR_INVALID_ARG, "%s: element object on another device", op);
  return BS_OK;
}

bs_status check_f64(const char* op, const char* name, const void* p, int64_t n) {
  return check_vec(op, name, p, n, BS_F64);
}

// Workgroups of the local operator: every resident one (two fit a CU's
// LDS), each striding over the elements so that its loads run ahead of its
// work, and no more than there are groups of four elements.
template <bool DOT>
int helm_blocks(int64_t n_elem) {
  int device = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&device) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_helm_local<DOT>, kWavesPerBlock * 64, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    (void)hipGetLastError();
    per_cu = 2;
    cus = 256;
  }
  const int64_t resident = static_cast<int64_t>(per_cu < 1 ? 1 : per_cu) * (cus < 1 ? 1 : cus);
  const int64_t g = (n_elem + kWavesPerBlock - 1) / kWavesPerBlock;
  return static_cast<int>(g < 1 ? 1 : (g < resident ? g : resident));
}

bs_status launch_local(bs_ctx* ctx, const bs_elem* el, int64_t n_elem, const int32_t* map, int64_t n_global,
                       const double* geo, double lambda, const double* xG, double* yL, hipStream_t st) {
  (void)ctx;
  if (n_elem == 0) return BS_OK;
  Rule8 rule{};
  for (int a = 0; a <= el->N; ++a) rule.w[a] = el->gauss_w[a];
  hipLaunchKernelGGL(k_helm_local<false>, dim3(helm_blocks<false>(n_elem)), dim3(kWavesPerBlock * 64), 0, st,
                     el->tables, rule, map, n_global, geo, lambda, xG, yL, n_elem, el->N + 1, nullptr, nullptr);
  return check_launch("bs_helmholtz_local");
}

}  // namespace

int helm_dot_blocks(int64_t n_elem) { return helm_blocks<true>(n_elem); }

bs_status helm_apply_dot(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* geo, double lambda,
                         const double* p, double* yL, double* Ap, double* partials, const int32_t* done,
                         hipStream_t st) {
  const int64_t P = static_cast<int64_t>(el->N + 1) * (el->N + 1) * (el->N + 1);
  const int64_t n_elem = gs->n_local / P;
  Rule8 rule{};
  for (int a = 0; a <= el->N; ++a) rule.w[a] = el->gauss_w[a];
  hipLaunchKernelGGL(k_helm_local<true>, dim3(helm_dot_blocks(n_elem)), dim3(kWavesPerBlock * 64), 0, st, el->tables,
                     rule, gs->map, gs->n_global, geo, lambda, p, yL, n_elem, el->N + 1, done, partials);
  if (bs_status s = check_launch("helmholtz cg")) return s;
  return bs_gather(ctx, gs, BS_F64, yL, Ap, st);
}

}  // namespace bs

using namespace bs;

extern "C" bs_status bs_elem_create(bs_ctx* ctx, int N, bs_elem** out) {
  const char* op = "bs_elem_create";
  bs_status s;
  if (!out) return fail(BS_ERR_INVALID_ARG, "%s: out is NULL", op);
  *out = nullptr;
  if ((s = check_ctx(ctx, op))) return s;
  if (N < 1 || N > 15) return fail(BS_ERR_INVALID_ARG, "%s: degree N must lie in [1, 15]", op);
  bs_elem* el = new bs_elem();
  el->device = ctx->device;
  el->N = N;
  gll_rule(N, el->gll_x, el->gll_w);
  gauss_rule(N + 1, el->gauss_x, el->gauss_w);
  el->tables = nullptr;
  if (N <= 7) {
    double host[kTabCount * kTabSize];
    build_tables(*el, host);
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(host)) != hipSuccess) {
      delete el;
      return fail(BS_ERR_ALLOC, "%s: cannot allocate the basis tables", op);
    }
    el->tables = static_cast<double*>(p);
    s = check_hip(hipMemcpy(p, host, sizeof(host), hipMemcpyHostToDevice), op);
    if (s) {
      (void)hipFree(p);
      delete el;
      return s;
    }
  }
  *out = el;
  return BS_OK;
}

extern "C" bs_status bs_elem_destroy(bs_elem* el) {
  if (!el) return BS_OK;
  hipError_t e = hipSuccess;
  if (el->tables) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(el->device);
    e = hipFree(el->tables);
    (void)hipSetDevice(prev);
  }
  delete el;
  return check_hip(e, "bs_elem_destroy");
}

extern "C" bs_status bs_elem_rules(const bs_elem* el, double* gll_x, double* gll_w, double* gauss_x,
                                   double* gauss_w) {
  if (!el) return fail(BS_ERR_INVALID_ARG, "bs_elem_rules: element object is NULL");
  for (int a = 0; a <= el->N; ++a) {
    if (gll_x) gll_x[a] = el->gll_x[a];
    if (gll_w) gll_w[a] = el->gll_w[a];
    if (gauss_x) gauss_x[a] = el->gauss_x[a];
    if (gauss_w) gauss_w[a] = el->gauss_w[a];
  }
  return BS_OK;
}

extern "C" bs_status bs_helmholtz_local(bs_ctx* ctx, const bs_elem* el, int64_t n_elem, const int32_t* d_map,
                                        int64_t n_global, const double* d_geo, double lambda, const double* xG,
                                        double* yL, void* stream) {
  const char* op = "bs_helmholtz_local";
  bs_status s;
  if ((s = check_elem(op, ctx, el))) return s;
  if (el->N > 7) return fail(BS_ERR_UNSUPPORTED, "%s: the local operator is built for degrees N <= 7", op);
  if (n_elem < 0 || n_global < 0) return fail(BS_ERR_INVALID_ARG, "%s: negative size", op);
  const int64_t P = static_cast<int64_t>(el->N + 1) * (el->N + 1) * (el->N + 1);
  if (n_elem > 0 && (!d_map || !aligned_to(d_map, 4))) return fail(BS_ERR_INVALID_ARG, "%s: bad map pointer", op);
  if ((s = check_f64(op, "geo", d_geo, 7 * n_elem)) || (s = check_f64(op, "xG", xG, n_global)) ||
      (s = check_f64(op, "yL", yL, n_elem * P)))
    return s;
  const uintptr_t y0 = reinterpret_cast<uintptr_t>(yL), y1 = y0 + static_cast<uintptr_t>(n_elem * P * 8);
  for (const void* q : {static_cast<const void*>(xG), static_cast<const void*>(d_geo), static_cast<const void*>(d_map)}) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(q);
    if (n_elem > 0 && q && a >= y0 && a < y1) return fail(BS_ERR_INVALID_ARG, "%s: yL overlaps an input", op);
  }
  return launch_local(ctx, el, n_elem, d_map, n_global, d_geo, lambda, xG, yL, static_cast<hipStream_t>(stream));
}

extern "C" bs_status bs_helmholtz_apply(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* d_geo,
                                        double lambda, const double* xG, double* yL_work, double* yG,
                                        void* stream) {
  const char* op = "bs_helmholtz_apply";
  bs_status s;
  if ((s = check_elem(op, ctx, el))) return s;
  if (!gs) return fail(BS_ERR_INVALID_ARG, "%s: plan is NULL", op);
  if (gs->device != ctx->device) return fail(BS_ERR_INVALID_ARG, "%s: plan on another device", op);
  const int64_t P = static_cast<int64_t>(el->N + 1) * (el->N + 1) * (el->N + 1);
  if (gs->n_local % P != 0) return fail(BS_ERR_INVALID_ARG, "%s: plan length is not a whole number of elements", op);
  if ((s = check_f64(op, "yG", yG, gs->n_global))) return s;
  const uintptr_t a = reinterpret_cast<uintptr_t>(xG), b = reinterpret_cast<uintptr_t>(yG);
  const uintptr_t nb = static_cast<uintptr_t>(gs->n_global) * 8;
  if (gs->n_global > 0 && a < b + nb && b < a + nb) return fail(BS_ERR_INVALID_ARG, "%s: yG overlaps xG", op);
  if ((s = bs_helmholtz_local(ctx, el, gs->n_local / P, gs->map, gs->n_global, d_geo, lambda, xG, yL_work, stream)))
    return s;
  return bs_gather(ctx, gs, BS_F64, yL_work, yG, stream);
}

extern "C" bs_status bs_mass_lumped(bs_ctx* ctx, const bs_elem* el, const bs_gs* gs, const double* d_geo,
                                    const double* xG, double* yG, void* stream) {
  const char* op = "bs_mass_lumped";
  bs_status s;
  if ((s = check_elem(op, ctx, el))) return s;
  if (!gs) return fail(BS_ERR_INVALID_ARG, "%s: plan is NULL", op);
  if (gs->device != ctx->device) return fail(BS_ERR_INVALID_ARG, "%s: plan on another device", op);
  const int P1 = el->N + 1;
  const int64_t P = static_cast<int64_t>(P1) * P1 * P1;
  if (gs->n_local % P != 0) return fail(BS_ERR_INVALID_ARG, "%s: plan length is not a whole number of elements", op);
  const int64_t E = gs->n_local / P;
  if ((s = check_f64(op, "geo", d_geo, 7 * E)) || (s = check_f64(op, "xG", xG, gs->n_global)) ||
      (s = check_f64(op, "yG", yG, gs->n_global)))
    return s;
  const uintptr_t a = reinterpret_cast<uintptr_t>(xG), b = reinterpret_cast<uintptr_t>(yG);
  const uintptr_t nb = static_cast<uintptr_t>(gs->n_global) * 8;
  if (gs->n_global > 0 && a < b + nb && b < a + nb) return fail(BS_ERR_INVALID_ARG, "%s: yG overlaps xG", op);
  if (gs->n_global == 0) return BS_OK;
  Gll16 gw{};
  for (int i = 0; i < P1; ++i) gw.w[i] = el->gll_w[i];
  hipLaunchKernelGGL(k_mass_lumped, dim3(static_cast<unsigned int>(gs->n_blocks)), dim3(kBlock), 0,
                     static_cast<hipStream_t>(stream), gs->row_starts, gs->col_ids, gs->block_starts, d_geo, gw, P1,
                     xG, yG, gs->chunk, gs->n_unmasked);
  return check_launch(op);
}
