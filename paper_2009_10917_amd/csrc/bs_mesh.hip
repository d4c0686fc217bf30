// Scatter map of a structured hex mesh (Section 2, eq. scatter_def): the
// element-to-global index map of K x K x K hexahedra carrying (N+1)^3
// Gauss-Lobatto-Legendre nodes each, with element slots permuted and each
// element's local frame turned by one of the 24 proper rotations of the cube.
// The paper leaves the numbering open; the conventions are stated in bs.h.

#include <algorithm>

#include "bs_device.h"
#include "bs_internal.h"

namespace bs {
namespace {

inline unsigned int blocks_for(int64_t n) { return static_cast<unsigned int>((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------- orientations

// The 24 proper rotations of the hex as (axis permutation, flips), axis
// permutations in lexicographic order, flip masks ascending, improper ones
// (odd permutation parity xor odd number of flips) skipped.
struct OrientTable {
  int8_t pi[24][3];
  int8_t flip[24][3];
};

OrientTable make_orient_table() {
  OrientTable t{};
  int p[3] = {0, 1, 2};
  int n = 0;
  do {
    const int inv = (p[0] > p[1]) + (p[0] > p[2]) + (p[1] > p[2]);
    for (int f = 0; f < 8; ++f) {
      const int f0 = f & 1, f1 = (f >> 1) & 1, f2 = (f >> 2) & 1;
      if (((inv & 1) ^ f0 ^ f1 ^ f2) != 0) continue;
      for (int d = 0; d < 3; ++d) t.pi[n][d] = static_cast<int8_t>(p[d]);
      t.flip[n][0] = static_cast<int8_t>(f0);
      t.flip[n][1] = static_cast<int8_t>(f1);
      t.flip[n][2] = static_cast<int8_t>(f2);
      ++n;
    }
  } while (std::next_permutation(p, p + 3));
  return t;
}

// Global id of local node l, or -1 when the slot's element or orientation
// is out of range.
__host__ __device__ inline int32_t hex_node(int64_t l, int64_t K, int N, const int32_t* perm,
                                            const uint8_t* orient, const OrientTable& T) {
  const int64_t Np = N + 1, Np3 = Np * Np * Np, M = K * N + 1, E = K * K * K;
  const int64_t s = l / Np3, rem = l - s * Np3;
  const int64_t t[3] = {rem % Np, (rem / Np) % Np, rem / (Np * Np)};
  const int64_t e = perm ? perm[s] : s;
  const int o = orient ? orient[s] : 0;
  if (e < 0 || e >= E || o >= 24) return -1;
  int64_t off[3];
  for (int d = 0; d < 3; ++d) {
    const int64_t v = t[T.pi[o][d]];
    off[d] = T.flip[o][d] ? N - v : v;
  }
  const int64_t X = N * (e % K) + off[0], Y = N * ((e / K) % K) + off[1], Z = N * (e / (K * K)) + off[2];
  return static_cast<int32_t>(X + M * (Y + M * Z));
}

__global__ __launch_bounds__(kBlock) void k_hex_map(int64_t K, int N, const int32_t* __restrict__ perm,
                                                    const uint8_t* __restrict__ orient, OrientTable T,
                                                    int32_t* __restrict__ map, int64_t n_local,
                                                    int* __restrict__ bad) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= n_local) return;
  const int32_t g = hex_node(l, K, N, perm, orient, T);
  map[l] = g;
  if (g < 0) atomicOr(bad, 1);
}

bs_status check_mesh(int64_t K, int N, int64_t* n_local) {
  if (K < 1 || N < 1) return fail(BS_ERR_INVALID_ARG, "hex map: K and N must be >= 1");
  const double ng = static_cast<double>(K * N + 1), nl = static_cast<double>(K) * K * K * (N + 1.0) * (N + 1) * (N + 1);
  if (ng * ng * ng >= 2147483648.0 || nl >= 2147483648.0)
    return fail(BS_ERR_INVALID_ARG, "hex map: mesh K=%lld N=%d exceeds 32-bit node ids", (long long)K, N);
  *n_local = K * K * K * (N + 1) * (N + 1) * (N + 1);
  return BS_OK;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" bs_status bs_mesh_hex_map_host(int64_t K, int N, const int32_t* perm, const uint8_t* orient,
                                          int32_t* map) {
  int64_t n_local = 0;
  bs_status s;
  if ((s = check_mesh(K, N, &n_local))) return s;
  if (!map) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map_host: map is NULL");
  const OrientTable T = make_orient_table();
  bool bad = false;
  for (int64_t l = 0; l < n_local; ++l) {
    map[l] = hex_node(l, K, N, perm, orient, T);
    bad |= map[l] < 0;
  }
  if (bad) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map_host: perm or orientation entry out of range");
  return BS_OK;
}

extern "C" bs_status bs_mesh_hex_map(int64_t K, int N, const int32_t* d_perm, const uint8_t* d_orient, int32_t* d_map,
                                     void* stream) {
  int64_t n_local = 0;
  bs_status s;
  if ((s = check_mesh(K, N, &n_local))) return s;
  if (!d_map) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map: d_map is NULL");
  if (!aligned_to(d_map, 4) || (d_perm && !aligned_to(d_perm, 4)))
    return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map: misaligned int32 array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* bad = nullptr;
  if (hipMalloc(&bad, sizeof(int)) != hipSuccess) return fail(BS_ERR_ALLOC, "bs_mesh_hex_map: flag allocation");
  int h_bad = 0;
  s = check_hip(hipMemsetAsync(bad, 0, sizeof(int), st), "bs_mesh_hex_map");
  if (!s) {
    hipLaunchKernelGGL(k_hex_map, dim3(blocks_for(n_local)), dim3(kBlock), 0, st, K, N, d_perm, d_orient,
                       make_orient_table(), d_map, n_local, bad);
    s = check_launch("bs_mesh_hex_map");
  }
  if (!s) s = check_hip(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st), "bs_mesh_hex_map");
  if (!s) s = check_hip(hipStreamSynchronize(st), "bs_mesh_hex_map");
  (void)hipFree(bad);
  if (s) return s;
  if (h_bad) return fail(BS_ERR_INVALID_ARG, "bs_mesh_hex_map: perm or orientation entry out of range");
  return BS_OK;
}

