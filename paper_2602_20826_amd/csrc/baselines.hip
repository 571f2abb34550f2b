// Comparison bounds of the evaluation (Section 5.2), per DAG, from the
// batch's tables.  With t_min = 1 the most useful parallelism of a node is
// m^max = min(p, C_hat) (the table mx).
//   Greedy:          sum of Eq. 1 times at m = min(m^max, M).
//   Greedy+unaware:  sum of Eq. 1 times at m = m^max (ceil(m/M) waves).
//   Graham_para:     node v as m^max unit-SM nodes of ceil(C_hat/m^max)
//                    ticks; Graham's list-scheduling bound on M SMs,
//                    len + floor((vol - len) / M), len the longest path in
//                    ticks, vol the SM-ticks of all unit nodes.
// One wavefront per DAG.  The sums are lane-parallel over nodes.  The
// longest path walks the sigma ranks upward: W^anc grows along every edge,
// so a node's successors have smaller ranks and are final when the node is
// reached; every lane reads a short successor list whole (no cross-lane
// reduction), a long one is split over the lanes.
#include "internal.h"

namespace dagbound {
namespace {

constexpr int WAVE = 64;

__device__ inline int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ inline int64_t wave_max64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(x, o);
    x = y > x ? y : x;
  }
  return x;
}

// STAGE: the DAG's successor offsets and lists are copied into LDS first
// (coalesced), so the walk over the ranks waits on LDS only.
template <bool STAGE>
__global__ __launch_bounds__(WAVE) void k_baselines(Tables t, int32_t M, int64_t* greedy, int64_t* unaware,
                                                    int64_t* graham, int32_t max_n) {
  extern __shared__ int64_t s_len[];  // [max_n]: longest path of unit ticks starting at the node
  const int d = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t n0 = t.node_off[d];
  const int N = (int)(t.node_off[d + 1] - n0);
  const int64_t e0 = t.edge_off[d];
  const int E = (int)(t.edge_off[d + 1] - e0);
  const uint32_t* soff = t.soff + n0 + d;
  const uint16_t* succ = t.succ + e0;
  if (STAGE) {
    uint32_t* l_soff = (uint32_t*)(s_len + max_n);
    uint16_t* l_succ = (uint16_t*)(l_soff + max_n + 1);
    for (int i = lane; i <= N; i += WAVE) l_soff[i] = soff[i];
    for (int i = lane; i < E; i += WAVE) l_succ[i] = succ[i];
    soff = l_soff;
    succ = l_succ;
  }
  int64_t g = 0, u = 0, vol = 0;
  for (int s = lane; s < N; s += WAVE) {
    const uint64_t c = t.wc[n0 + s];
    const uint64_t mm = t.mx[n0 + s];
    const uint64_t mg = mm < (uint64_t)M ? mm : (uint64_t)M;
    g += (int64_t)((c + mg - 1) / mg);                    // Eq. 1, one wave
    const uint64_t waves = (mm + M - 1) / (uint64_t)M;
    u += (int64_t)((waves * c + mm - 1) / mm);           // Eq. 1, ceil(m/M) waves
    const uint64_t ell = (c + mm - 1) / mm;
    vol += (int64_t)(mm * ell);
    s_len[s] = (int64_t)ell;
  }
  g = wave_sum64(g);
  u = wave_sum64(u);
  vol = wave_sum64(vol);
  __syncthreads();
  int64_t longest = 0;
  for (int s = 0; s < N; s++) {
    const uint32_t a = soff[s], b = soff[s + 1];
    int64_t best = 0;
    if (b - a <= 8) {
      // few successors (the common case): every lane reads them all (the
      // same addresses, one broadcast each), no cross-lane reduction
      for (uint32_t k = a; k < b; k++) {
        const int64_t x = s_len[succ[k]];
        best = x > best ? x : best;
      }
    } else {
      for (uint32_t k = a + lane; k < b; k += WAVE) {
        const int64_t x = s_len[succ[k]];
        best = x > best ? x : best;
      }
      best = wave_max64(best);
    }
    const int64_t l = s_len[s] + best;
    longest = l > longest ? l : longest;
    // one wavefront: its LDS accesses complete in order, so every lane has
    // read s_len[s] before this write, and the barrier waits for the write
    if (lane == 0) s_len[s] = l;
    __syncthreads();
  }
  if (lane == 0) {
    if (greedy) greedy[d] = g;
    if (unaware) unaware[d] = u;
    if (graham) graham[d] = N ? longest + (vol - longest) / M : 0;
  }
}

// LDS of one workgroup: the path lengths, and with staging the successor
// offsets and lists of the largest DAG.  Staging is used while it stays
// within STAGE_LDS, so that several DAGs share a compute unit.
constexpr size_t STAGE_LDS = 32 * 1024;
size_t baselines_lds_bytes(int32_t max_n, int32_t max_e, bool stage) {
  const size_t n = (size_t)(max_n > 0 ? max_n : 1);
  return stage ? ((n * 8 + (n + 1) * 4 + (size_t)max_e * 2 + 15) & ~(size_t)15) : n * 8;
}

}  // namespace

hipError_t launch_baselines(const Tables& t, int32_t D, int32_t M, int32_t max_n, int32_t max_e, int64_t* greedy,
                            int64_t* unaware, int64_t* graham, hipStream_t stream) {
  if (D <= 0) return hipSuccess;
  const bool stage = baselines_lds_bytes(max_n, max_e, true) <= STAGE_LDS;
  const size_t lds = baselines_lds_bytes(max_n, max_e, stage);
  const void* fn = stage ? (const void*)k_baselines<true> : (const void*)k_baselines<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (stage)
    hipLaunchKernelGGL(k_baselines<true>, dim3(D), dim3(WAVE), lds, stream, t, M, greedy, unaware, graham, max_n);
  else
    hipLaunchKernelGGL(k_baselines<false>, dim3(D), dim3(WAVE), lds, stream, t, M, greedy, unaware, graham, max_n);
  return hipGetLastError();
}

}  // namespace dagbound
