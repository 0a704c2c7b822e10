// datagen.hip -- seeded synthetic inputs on the GPU (libmsgen.so).
//
// Holds none of the compression or operator arithmetic.  It reproduces, bit for bit,
// the counter-based generators of datagen.py: SplitMix64 (Steele, Lea, Flood 2014)
// keyed by mix64(seed), x_i = mix64(key + (i + 1) * GAMMA).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t mix64_h(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t xs(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

__global__ void k_uniform_bits(uint64_t key, uint64_t start, uint64_t n, unsigned b, uint32_t *out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = b ? (uint32_t)(xs(key, start + i) >> (64 - b)) : 0u;
}

__global__ void k_uniform_range(uint64_t key, uint64_t start, uint64_t n, uint64_t lo, uint64_t span,
                                uint32_t *out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)(lo + (((xs(key, start + i) >> 32) * span) >> 32));
}

// gaps for the sorted distribution: g_0 = start value, g_i = x_i >> 61
__global__ void k_gaps(uint64_t key, uint64_t n, uint64_t first, int64_t *out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = i ? (int64_t)(xs(key, i) >> 61) : (int64_t)first;
}

// run-start flags of the runs distribution: row i > 0 starts a run when x_i >> 58 == 0
__global__ void k_run_flags(uint64_t key, uint64_t n, int64_t *out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (i && (xs(key, i) >> 58) == 0) ? 1 : 0;
}

// value of run r = 2 * (x'_r >> 49) + (r & 1)
__global__ void k_run_values(uint64_t key1, const int64_t *run_id, uint64_t n, uint32_t *out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = (uint64_t)run_id[i];
    out[i] = (uint32_t)(2 * (xs(key1, r) >> 49) + (r & 1));
  }
}

unsigned blocks_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

extern "C" {

int msgen_uniform_bits(uint64_t seed, uint64_t start, uint64_t n, unsigned b, uint32_t *out, void *stream) {
  if (b > 32) return 1;
  if (!n) return 0;
  hipLaunchKernelGGL(k_uniform_bits, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, mix64_h(seed), start,
                     n, b, out);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}

int msgen_uniform_range(uint64_t seed, uint64_t start, uint64_t n, uint64_t lo, uint64_t span, uint32_t *out,
                        void *stream) {
  if (span == 0 || span > (1ull << 32) || lo + span > (1ull << 32)) return 1;
  if (!n) return 0;
  hipLaunchKernelGGL(k_uniform_range, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, mix64_h(seed), start,
                     n, lo, span, out);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}

int msgen_gaps(uint64_t seed, uint64_t n, int64_t *out, void *stream) {
  if (!n) return 0;
  const uint64_t first = mix64_h(mix64_h(seed + 1) + kGamma) >> 44;  // x'_0 of the stream of seed + 1
  hipLaunchKernelGGL(k_gaps, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, mix64_h(seed), n, first, out);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}

int msgen_run_flags(uint64_t seed, uint64_t n, int64_t *out, void *stream) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_run_flags, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, mix64_h(seed), n, out);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}

int msgen_run_values(uint64_t seed, const int64_t *run_id, uint64_t n, uint32_t *out, void *stream) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_run_values, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, mix64_h(seed + 1), run_id,
                     n, out);
  return hipGetLastError() == hipSuccess ? 0 : 8;
}

}  // extern "C"
