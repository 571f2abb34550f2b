// Realization of one schedule on this GPU as a HIP graph, the counterpart
// of the paper's case study (Sections 5.1 and 5.3: one busy kernel with per-node
// iteration counts, m_i set through the launch shape, the DAG run as a CUDA
// graph).  Each launched part of the schedule becomes one kernel node of m
// workgroups; a workgroup reserves more than half of a compute unit's LDS,
// so it holds one compute unit alone, and spins for C ticks on the GPU's
// constant-rate clock (Eq. 1's block model: m blocks of C ticks, one SM
// each).  With one barrier per slot boundary, a slot's parts are one launch
// of all their blocks (kernels of one graph level do not all run at once on
// a few hardware queues, the blocks of one launch do), each slot after the
// one before.  Without barriers each part is its own kernel node, after the
// DAG's edges, the chain of a segmented node's parts and the extra
// dependencies of Section 4.1.
#include <algorithm>
#include <map>
#include <utility>
#include <vector>

#include "internal.h"

namespace dagbound {
namespace {

// Dynamic LDS of a busy workgroup: above half of the 160 KB of a compute
// unit, so no two busy workgroups share one.
constexpr size_t BUSY_LDS = 96 * 1024;

__global__ __launch_bounds__(64) void k_busy(int64_t ticks) {
  extern __shared__ int busy_lds[];
  if (threadIdx.x == 0) {
    const int64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(2);
    busy_lds[0] = 0;
  }
  __syncthreads();
}

// One slot as one launch: workgroup i spins ticks[i] (the C of the part it
// belongs to), so every block of the slot starts together, as the slot's
// parts do under one barrier per slot boundary.
__global__ __launch_bounds__(64) void k_busy_slot(const int64_t* ticks) {
  extern __shared__ int busy_lds[];
  if (threadIdx.x == 0) {
    const int64_t t0 = wall_clock64();
    const int64_t n = ticks[blockIdx.x];
    while (wall_clock64() - t0 < n) __builtin_amdgcn_s_sleep(2);
    busy_lds[0] = 0;
  }
  __syncthreads();
}

struct Part {
  int64_t slot, node, part, m, C;
};

}  // namespace

hipError_t realize_schedule(const int64_t* rec, int64_t nrec, int32_t n, const int32_t* esrc,
                            const int32_t* edst, int32_t ne, int64_t tick_ns, bool barriers, int32_t reps,
                            int64_t* makespan_ns, int32_t* nparts_out) {
  int dev = 0, rate_khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_busy, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)BUSY_LDS);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_busy_slot, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)BUSY_LDS);
  if (e != hipSuccess) return e;
  const int64_t ticks_per_tick = std::max<int64_t>(1, tick_ns * (int64_t)rate_khz / 1000000);

  std::vector<Part> parts;
  std::vector<int64_t> ex_raw;  // extra dependencies: from node, from part, to node, to part
  int64_t nslots = 0;
  for (int64_t i = 0; i < nrec; i++) {
    // records as the schedule dump writes them: PART {2, slot, node, part,
    // kind, m, C, load}, SLOT {1, slot, ...}, EDGE {3, slot, from node,
    // from part, to node, to part, 0, 0}
    const int64_t* r = rec + 8 * i;
    if (r[0] == 2 && r[2] >= 0 && r[2] < n && r[1] >= 0 && r[5] >= 1) parts.push_back({r[1], r[2], r[3], r[5], r[6]});
    else if (r[0] == 1) nslots = std::max(nslots, r[1] + 1);
    else if (r[0] == 3) ex_raw.insert(ex_raw.end(), {r[2], r[3], r[4], r[5]});
  }
  if (nparts_out) *nparts_out = (int32_t)parts.size();
  std::map<std::pair<int64_t, int64_t>, size_t> index;  // (node, part) -> part
  std::vector<int64_t> last_part(n, -1);
  for (size_t k = 0; k < parts.size(); k++) {
    index[{parts[k].node, parts[k].part}] = k;
    last_part[parts[k].node] = std::max(last_part[parts[k].node], parts[k].part);
  }

  hipGraph_t g = nullptr;
  e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  std::vector<hipGraphNode_t> pn(parts.size(), nullptr);
  std::vector<hipGraphNode_t> bar(nslots, nullptr);
  std::vector<std::vector<size_t>> by_slot(nslots);
  for (size_t k = 0; k < parts.size(); k++)
    if (parts[k].slot < nslots) by_slot[parts[k].slot].push_back(k);
  auto add_part = [&](size_t k, const hipGraphNode_t* deps, size_t nd) -> hipError_t {
    int64_t ticks = parts[k].C * ticks_per_tick;
    void* args[] = {&ticks};
    hipKernelNodeParams p = {};
    p.func = (void*)k_busy;
    p.gridDim = dim3((unsigned)parts[k].m);
    p.blockDim = dim3(64);
    p.sharedMemBytes = (unsigned)BUSY_LDS;
    p.kernelParams = args;
    p.extra = nullptr;
    return hipGraphAddKernelNode(&pn[k], g, deps, nd, &p);
  };
  int64_t* d_ticks = nullptr;
  if (barriers) {
    // one launch per slot holding the blocks of all its parts, each slot
    // after the one before (the launches of one graph branch run in order)
    std::vector<int64_t> wt;
    std::vector<size_t> first(nslots + 1, 0);
    for (int64_t j = 0; j < nslots; j++) {
      first[j] = wt.size();
      for (size_t k : by_slot[j])
        for (int64_t b = 0; b < parts[k].m; b++) wt.push_back(parts[k].C * ticks_per_tick);
    }
    first[nslots] = wt.size();
    if (!wt.empty()) e = hipMalloc((void**)&d_ticks, wt.size() * 8);
    if (e == hipSuccess && !wt.empty()) e = hipMemcpy(d_ticks, wt.data(), wt.size() * 8, hipMemcpyHostToDevice);
    for (int64_t j = 0; j < nslots && e == hipSuccess; j++) {
      if (first[j + 1] == first[j]) continue;
      hipGraphNode_t prev = j > 0 ? bar[j - 1] : nullptr;
      for (int64_t i = j - 1; i >= 0 && !prev; i--) prev = bar[i];
      const int64_t* tp = d_ticks + first[j];
      void* args[] = {(void*)&tp};
      hipKernelNodeParams p = {};
      p.func = (void*)k_busy_slot;
      p.gridDim = dim3((unsigned)(first[j + 1] - first[j]));
      p.blockDim = dim3(64);
      p.sharedMemBytes = (unsigned)BUSY_LDS;
      p.kernelParams = args;
      p.extra = nullptr;
      e = hipGraphAddKernelNode(&bar[j], g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
    }
  } else {
    // the DAG's edges (last part of u before the first part of v), the
    // chain of a segmented node's parts, and the extra dependencies
    std::vector<std::vector<size_t>> deps(parts.size());
    auto part_of = [&](int64_t node, int64_t part) -> int64_t {
      auto it = index.find({node, part});
      return it == index.end() ? -1 : (int64_t)it->second;
    };
    for (int32_t k = 0; k < ne; k++) {
      const int64_t a = esrc[k] >= 0 && esrc[k] < n ? part_of(esrc[k], last_part[esrc[k]]) : -1;
      const int64_t b = edst[k] >= 0 && edst[k] < n ? part_of(edst[k], 0) : -1;
      if (a >= 0 && b >= 0) deps[b].push_back((size_t)a);
    }
    for (size_t k = 0; k < parts.size(); k++) {
      const int64_t a = parts[k].part > 0 ? part_of(parts[k].node, parts[k].part - 1) : -1;
      if (a >= 0) deps[k].push_back((size_t)a);
    }
    for (size_t i = 0; i + 3 < ex_raw.size(); i += 4) {
      const int64_t a = part_of(ex_raw[i], ex_raw[i + 1]), b = part_of(ex_raw[i + 2], ex_raw[i + 3]);
      if (a >= 0 && b >= 0) deps[b].push_back((size_t)a);
    }
    // every dependency lies in an earlier slot or earlier in the same slot's
    // launch order, so adding the parts in slot order adds it first
    for (int64_t j = 0; j < nslots && e == hipSuccess; j++) {
      for (size_t k : by_slot[j]) {
        // a graph node takes each dependency once
        std::sort(deps[k].begin(), deps[k].end());
        deps[k].erase(std::unique(deps[k].begin(), deps[k].end()), deps[k].end());
        std::vector<hipGraphNode_t> d;
        for (size_t x : deps[k])
          if (x != k && pn[x]) d.push_back(pn[x]);
        e = add_part(k, d.data(), d.size());
        if (e != hipSuccess) break;
      }
    }
  }
  hipGraphExec_t ge = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  hipStream_t st = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipGraphLaunch(ge, st);  // warm-up
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int32_t r = 0; r < reps && e == hipSuccess; r++) {
    e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = hipGraphLaunch(ge, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e == hipSuccess) makespan_ns[r] = (int64_t)((double)ms * 1e6);
  }
  if (st) (void)hipStreamSynchronize(st);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st) (void)hipStreamDestroy(st);
  if (ge) (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  if (d_ticks) (void)hipFree(d_ticks);
  return e;
}

}  // namespace dagbound
