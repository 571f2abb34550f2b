// Explicit candidate bytes written straight into device memory (input
// generation only; none of the bound's arithmetic).  Same bytes as
// wl_alloc_bytes in gen.c: the counter-based draw documented there,
//   key  = mix(seed ^ mix(d * GOLDEN))
//   word = mix(key ^ ((c << 32) | (v >> 2)))
//   h16  = (word >> (16 * (v & 3))) & 0xFFFF
//   r    = 1 + ((h16 * range) >> 16),  range = min(p_v, M, 255),
// candidate 0 all zeros, byte (d, c, v) at K * node_off[d] + c * N_d + v.
// Lets a benchmark place tens of GB of candidate bytes in HBM without
// staging them through host memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int THREADS = 256;
constexpr int MAX_N = 8192;  // nodes of one DAG held in LDS (ranges)

// One workgroup per DAG: the node ranges in LDS, then the K * N bytes of the
// DAG's rows written in order, four consecutive bytes per thread and store
// (one hash word covers four nodes of a candidate).
__global__ __launch_bounds__(THREADS) void k_alloc_bytes(uint64_t seed, int64_t d0, int64_t count,
                                                         const int64_t* node_off, const int32_t* par,
                                                         int32_t M, int32_t K, uint8_t* out) {
  __shared__ uint8_t s_range[MAX_N];
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const int64_t n0 = node_off[i] - node_off[0];
    const int32_t N = (int32_t)(node_off[i + 1] - node_off[i]);
    __syncthreads();
    for (int v = threadIdx.x; v < N; v += THREADS) {
      const int32_t p = par[n0 + v];
      const int32_t r = p < M ? p : M;
      s_range[v] = (uint8_t)(r > 255 ? 255 : r);
    }
    __syncthreads();
    const uint64_t key = mix64(seed ^ mix64((uint64_t)(d0 + i) * GOLDEN));
    uint8_t* o = out + (int64_t)K * n0;
    // row c of the DAG: bytes [c * N, c * N + N); quads of nodes v = 4q .. 4q + 3
    const int32_t quads = (N + 3) >> 2;
    const uint32_t total = (uint32_t)K * (uint32_t)quads;  // below 2^32: K <= 2^16, quads <= 2^11
    for (uint32_t j = threadIdx.x; j < total; j += THREADS) {
      const int32_t c = (int32_t)(j / (uint32_t)quads);
      const int32_t q = (int32_t)(j - (uint32_t)c * (uint32_t)quads);
      uint8_t* row = o + (int64_t)c * N;
      const uint64_t word = c == 0 ? 0ull : mix64(key ^ (((uint64_t)c << 32) | (uint64_t)q));
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int32_t v = 4 * q + k;
        if (v < N) {
          const uint32_t h16 = (uint32_t)(word >> (16 * k)) & 0xFFFFu;
          row[v] = c == 0 ? (uint8_t)0 : (uint8_t)(1u + ((h16 * (uint32_t)s_range[v]) >> 16));
        }
      }
    }
  }
}

}  // namespace

// DAGs d0 .. d0 + count - 1 (device arrays: node_off [count + 1], relative
// offsets taken from node_off[0]; par [N]) into out (device, K * N bytes),
// on `stream`.  Returns a hipError_t (0 on success); DAGs above 8,192 nodes
// are rejected.
extern "C" int wl_alloc_bytes_device(uint64_t seed, int64_t d0, int64_t count, const int64_t* node_off,
                                     const int32_t* par, int32_t M, int32_t K, int32_t max_n, uint8_t* out,
                                     void* stream) {
  if (count <= 0) return 0;
  if (max_n > MAX_N || K < 1 || K > 65536 || M < 1) return (int)hipErrorInvalidValue;
  const int64_t grid = count < 65536 ? count : 65536;
  hipLaunchKernelGGL(k_alloc_bytes, dim3((unsigned)grid), dim3(THREADS), 0, (hipStream_t)stream, seed, d0,
                     count, node_off, par, M, K, out);
  return (int)hipGetLastError();
}
