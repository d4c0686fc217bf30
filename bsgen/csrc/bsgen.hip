// Device form of the seeded input generator (see bsgen/__init__.py for the
// definition).  Value i of stream k under seed S is F(key + (i+1)*GAMMA) with
// F the SplitMix64 output function and key = F(S xor F(k)) (Steele, Lea &
// Flood, OOPSLA 2014).  Uniform [0,1) takes the top 53 bits times 2^-53;
// uniform [-1,1) is 2u - 1.  Narrow storage rounds the binary64 value to
// binary32 (nearest even) and then to bfloat16 (nearest even).
//
// Input generation only: no part of the streaming operations lives here.

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double draw(uint64_t key, int64_t i, int sym) {
  const uint64_t x = mix(key + static_cast<uint64_t>(i + 1) * kGamma);
  const double u = static_cast<double>(x >> 11) * 0x1.0p-53;
  return sym ? 2.0 * u - 1.0 : u;
}

__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

__global__ void k_uniform_f64(uint64_t key, int64_t start, int64_t n, int sym, double* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = draw(key, start + i, sym);
}

__global__ void k_uniform_f32(uint64_t key, int64_t start, int64_t n, int sym, float* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<float>(draw(key, start + i, sym));
}

__global__ void k_uniform_bf16(uint64_t key, int64_t start, int64_t n, int sym, uint16_t* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = to_bf16(static_cast<float>(draw(key, start + i, sym)));
}

}  // namespace

// dtype: 0 binary64, 1 binary32, 2 bfloat16.  sym: 1 for [-1,1), 0 for [0,1).
// Fills out[0..n) with values start..start+n-1 of the stream.  Returns 0 on
// success, the HIP error code otherwise.
extern "C" int bsgen_uniform(uint64_t seed, uint64_t stream, int64_t start, int64_t n, int sym, int dtype, void* out,
                             void* hip_stream) {
  if (n <= 0) return 0;
  if (!out) return static_cast<int>(hipErrorInvalidValue);
  const uint64_t key = mix(seed ^ mix(stream));
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(k_uniform_f64, dim3(blocks), dim3(256), 0, st, key, start, n, sym, static_cast<double*>(out));
      break;
    case 1:
      hipLaunchKernelGGL(k_uniform_f32, dim3(blocks), dim3(256), 0, st, key, start, n, sym, static_cast<float*>(out));
      break;
    case 2:
      hipLaunchKernelGGL(k_uniform_bf16, dim3(blocks), dim3(256), 0, st, key, start, n, sym,
                         static_cast<uint16_t*>(out));
      break;
    default:
      return static_cast<int>(hipErrorInvalidValue);
  }
  return static_cast<int>(hipGetLastError());
}
