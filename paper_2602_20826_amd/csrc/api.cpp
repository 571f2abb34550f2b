// C-ABI of libdagbound (declared in include/dagbound.h): argument checks,
// device memory, and the order of the kernel launches.  Every step of the
// method runs in the gfx950 kernels of prep.hip and sweep.hip; this file only
// moves buffers and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dagbound.h"
#include "internal.h"

using namespace dagbound;

namespace {

thread_local std::string g_err;

dagbound_status fail(dagbound_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

dagbound_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? DAGBOUND_E_OOM : DAGBOUND_E_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Device memory: freed batch blocks are kept per device and handed to the next
// batch of similar size, so repeated create/destroy cycles do not go back to
// the HIP allocator each time.
struct CachedBlock {
  void* p;
  size_t size;
  int device;
};
std::mutex g_mu;
std::vector<CachedBlock> g_cache;
size_t g_cached_bytes = 0;
constexpr size_t CACHE_CAP = 16ull << 30;
constexpr size_t GRAIN = 2ull << 20;

void cache_trim_locked(size_t cap) {
  while (g_cached_bytes > cap && !g_cache.empty()) {
    CachedBlock b = g_cache.front();
    g_cache.erase(g_cache.begin());
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(b.device);
    (void)hipFree(b.p);
    (void)hipSetDevice(cur);
    g_cached_bytes -= b.size;
  }
}

hipError_t dev_alloc(void** p, size_t* size, int device) {
  size_t need = std::max<size_t>(GRAIN, (*size + GRAIN - 1) / GRAIN * GRAIN);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    int best = -1;
    for (size_t i = 0; i < g_cache.size(); i++) {
      const CachedBlock& b = g_cache[i];
      if (b.device == device && b.size >= need && b.size <= 2 * need &&
          (best < 0 || b.size < g_cache[best].size))
        best = (int)i;
    }
    if (best >= 0) {
      *p = g_cache[best].p;
      *size = g_cache[best].size;
      g_cached_bytes -= g_cache[best].size;
      g_cache.erase(g_cache.begin() + best);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, need);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(g_mu);
      cache_trim_locked(0);
    }
    e = hipMalloc(p, need);
  }
  if (e == hipSuccess) *size = need;
  return e;
}

void dev_release(void* p, size_t size, int device) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.push_back({p, size, device});
  g_cached_bytes += size;
  cache_trim_locked(CACHE_CAP);
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Bump allocator over one device block.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = (T*)(base + off);
    off += count * sizeof(T);
    return p;
  }
};

size_t table_bytes(int64_t D, int64_t tn, int64_t te, size_t gres_words, bool mrec) {
  return 24 * 256 + (size_t)(D + 1) * 8 * 2 + (size_t)tn * 8 + (size_t)D * 8 + 24 + (mrec ? (size_t)tn * 32 : 0) +
         (size_t)tn * 4 * 2 + (size_t)(tn + D) * 4 + (size_t)D * 4 + (size_t)tn * 2 * 4 +
         (size_t)te * 2 + gres_words * 4 + (size_t)D * 4;
}

// Side streams of each device for the size-class launches (created once,
// default priority, kept until the process ends).
std::mutex g_stream_mu;
std::vector<std::array<hipStream_t, NUM_CLASSES>> g_side;

hipError_t side_streams(int device, hipStream_t out[NUM_CLASSES]) {
  std::lock_guard<std::mutex> lk(g_stream_mu);
  if ((int)g_side.size() <= device) g_side.resize(device + 1, std::array<hipStream_t, NUM_CLASSES>{});
  for (int c = 0; c < NUM_CLASSES; c++) {
    if (!g_side[device][c]) {
      hipError_t e = hipStreamCreateWithFlags(&g_side[device][c], hipStreamNonBlocking);
      if (e != hipSuccess) {
        g_side[device][c] = nullptr;
        return e;
      }
    }
    out[c] = g_side[device][c];
  }
  return hipSuccess;
}

}  // namespace

struct dagbound_batch {
  int device = 0;
  int32_t D = 0, M = 1;
  int64_t tn = 0, te = 0;
  int32_t max_n = 0, max_e = 0;
  std::vector<int64_t> node_off, edge_off;  // host copies
  void* block = nullptr;
  size_t block_size = 0;
  Tables t{};
  unsigned long long* best = nullptr;  // [D] packed per-DAG minimum
  unsigned long long* err = nullptr;   // [3] first failing DAG, any load >= 2^20, large-DAG work counter
  uint32_t* gres = nullptr;            // residual tables of the global evaluation pass
  bool small_loads = false;            // every load < 2^20
  bool small_indeg = false;            // every in-degree < 256
  // DAG ids grouped by size class (the evaluation launches one kernel per class)
  int32_t* order = nullptr;
  std::vector<int32_t> order_host;
  int32_t class_off[NUM_CLASSES + 1] = {};
  int32_t class_max_n[NUM_CLASSES] = {};
  bool size_classes = true;
  bool class_streams = true;           // class launches on side streams
  bool persistent = false;             // first pass as a persistent kernel
  int32_t node_lanes_class = LARGE_CLASS;  // first class run by the lane-per-node kernel
  bool autotune_pending = false;       // time the launch plans on the next evaluation
  // "graph": the evaluation's launches recorded once into a HIP graph and
  // replayed while the outputs, stream, allocation set and tuning stay the same
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  const void* g_key[4] = {nullptr, nullptr, nullptr, nullptr};  // bounds, cp, intf, stream
  uint64_t g_gen = ~0ull, g_tune = ~0ull;
  uint64_t tune_gen = 0;
  float plan_ms[8] = {};               // last autotune: (node lanes from 257 nodes, persistent, class_streams) = (l, p, s) at 4l + 2p + s
  size_t gres_off[NUM_CLASSES] = {};
  uint64_t* grows = nullptr;           // residual-slot map regions for DAGs of 129-512 nodes
  int32_t adj_uniform_nw = 0;          // the adjacency rows' words: 0 per size class, else this for every DAG
  size_t rows_off[NUM_CLASSES + 1] = {};
  hipEvent_t ev[NUM_CLASSES + 1] = {};  // fork, joins
  // per-allocation-set scratch: tiles handed to the global pass
  void* ovf_block = nullptr;
  size_t ovf_block_size = 0;
  uint32_t* ovf_list = nullptr;
  uint32_t* ovf_count = nullptr;
  // tuning
  int32_t res_slots = RES_SLOTS;
  int32_t eval_path = EVAL_PATH_AUTO;
  // candidate allocations
  bool has_alloc = false;
  int32_t K = 0;
  uint32_t mode = DAGBOUND_ALLOC_EXPLICIT;
  int32_t para_mode = DAGBOUND_PARA_SPATIAL;  // reading of the launching loop
  const uint8_t* alloc = nullptr;
  void* alloc_owned = nullptr;
  size_t alloc_owned_size = 0;
  uint64_t seed = 0;
  uint64_t alloc_gen = 0;
  uint64_t best_gen = ~0ull;
};

namespace {

// Host arrays of released batches, kept for the next batch: a fresh array
// of a few MB is paged in on first touch, which would cost more than
// create_batch's own host work.
std::mutex g_host_mu;
std::vector<std::vector<int64_t>> g_host64;
std::vector<std::vector<int32_t>> g_host32;
constexpr size_t HOST_POOL = 8;

template <class T>
std::vector<T> host_take(std::vector<std::vector<T>>& pool, size_t n) {
  std::vector<T> v;
  {
    std::lock_guard<std::mutex> lk(g_host_mu);
    int best = -1;
    for (size_t i = 0; i < pool.size(); i++)
      if (pool[i].capacity() >= n && (best < 0 || pool[i].capacity() < pool[best].capacity())) best = (int)i;
    if (best >= 0) {
      v = std::move(pool[best]);
      pool.erase(pool.begin() + best);
    }
  }
  v.resize(n);
  return v;
}

template <class T>
void host_give(std::vector<std::vector<T>>& pool, std::vector<T>&& v) {
  if (v.capacity() == 0) return;
  v.clear();
  std::lock_guard<std::mutex> lk(g_host_mu);
  if (pool.size() < HOST_POOL) pool.push_back(std::move(v));
}

void batch_free(dagbound_batch* b) {
  if (!b) return;
  {
    DeviceGuard g(b->device);
    (void)hipDeviceSynchronize();
  }
  dev_release(b->block, b->block_size, b->device);
  dev_release(b->alloc_owned, b->alloc_owned_size, b->device);
  dev_release(b->ovf_block, b->ovf_block_size, b->device);
  for (hipEvent_t ev : b->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  host_give(g_host64, std::move(b->node_off));
  host_give(g_host64, std::move(b->edge_off));
  host_give(g_host32, std::move(b->order_host));
  delete b;
}

SweepArgs sweep_args(const dagbound_batch* b) {
  SweepArgs a{};
  a.t = b->t;
  a.D = b->D;
  a.M = b->M;
  a.K = b->K;
  a.kalloc = b->K;
  a.alloc = b->mode == DAGBOUND_ALLOC_EXPLICIT ? b->alloc : nullptr;
  a.seed = b->seed;
  a.temporal = b->para_mode;
  a.max_n = b->max_n;
  a.max_e = b->max_e;
  a.order = b->size_classes ? b->order : nullptr;
  for (int c = 0; c <= NUM_CLASSES; c++) a.class_off[c] = b->class_off[c];
  for (int c = 0; c < NUM_CLASSES; c++) a.class_max_n[c] = b->class_max_n[c];
  for (int c = 0; c < NUM_CLASSES; c++) a.gres_off[c] = b->gres_off[c];
  a.grows = b->grows;
  for (int c = 0; c <= NUM_CLASSES; c++) a.rows_off[c] = b->rows_off[c];
  a.ovf_list = b->ovf_list;
  a.ovf_count = b->ovf_count;
  a.gres = b->gres;
  a.res_slots = b->res_slots;
  a.path = b->eval_path;
  a.small_loads = b->small_loads ? 1 : 0;
  a.small_indeg = b->small_indeg ? 1 : 0;
  a.persistent = b->persistent ? 1 : 0;
  a.node_lanes_class = b->node_lanes_class;
  return a;
}

hipError_t run_sweep_plan(dagbound_batch* b, const SweepArgs& a, hipStream_t st);

// One evaluation launch of a batch.  After set_tuning("autotune", 1) the
// next call runs every launch plan (persistent first pass or not, class
// launches concurrent or not, and, when the batch holds DAGs of 257-512
// nodes, their lane-per-candidate or lane-per-node kernel) once, timed with
// events on `st`, and keeps the fastest; the results of every plan are
// identical.
hipError_t run_sweep(dagbound_batch* b, const SweepArgs& a, hipStream_t st) {
  if (!b->autotune_pending) return run_sweep_plan(b, a, st);
  b->autotune_pending = false;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  const int nplans = b->class_off[4] > b->class_off[3] ? 8 : 4;
  float best = -1.f;
  int best_plan = (b->node_lanes_class == 3 ? 4 : 0) + (b->persistent ? 2 : 0) + (b->class_streams ? 1 : 0);
  for (int plan = 0; plan < nplans && e == hipSuccess; plan++) {
    b->persistent = plan & 2;
    b->class_streams = plan & 1;
    b->node_lanes_class = plan & 4 ? 3 : LARGE_CLASS;
    SweepArgs ap = a;
    ap.persistent = b->persistent ? 1 : 0;
    ap.node_lanes_class = b->node_lanes_class;
    e = hipEventRecord(t0, st);
    if (e == hipSuccess) e = run_sweep_plan(b, ap, st);
    if (e == hipSuccess) e = hipEventRecord(t1, st);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e != hipSuccess) break;
    b->plan_ms[plan] = ms;
    if (best < 0.f || ms < best) { best = ms; best_plan = plan; }
  }
  b->persistent = best_plan & 2;
  b->class_streams = best_plan & 1;
  b->node_lanes_class = best_plan & 4 ? 3 : LARGE_CLASS;
  b->tune_gen++;
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  return e;
}

// Side streams and fork/join events of a batch (created before any capture).
hipError_t plan_resources(dagbound_batch* b, SweepStreams* ss) {
  hipError_t e = side_streams(b->device, ss->side);
  for (int i = 0; i <= NUM_CLASSES && e == hipSuccess; i++)
    if (!b->ev[i]) e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
  return e;
}

// One evaluation launch of a batch: the size classes on the device's side
// streams when there is more than one class to run.
// Words of a bitset row of a DAG of n <= 512 nodes.
int row_words(int64_t n) { return n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : 8; }

// The adjacency rows in the layout the next launch reads: rows of each
// size class's words, or, while the batch runs as one launch over DAGs of up
// to 512 nodes, rows of the largest DAG's words for every DAG.  Rewritten
// (on `st`) only when that layout changes.
hipError_t ensure_adj(dagbound_batch* b, hipStream_t st) {
  if (!b->t.adj) return hipSuccess;
  const int want = !b->size_classes && b->max_n <= 512 ? row_words(b->max_n) : 0;
  if (want == b->adj_uniform_nw) return hipSuccess;
  const hipError_t e = launch_adj(b->t, b->order, b->class_off, b->class_max_n, want, st);
  if (e == hipSuccess) b->adj_uniform_nw = want;
  return e;
}

hipError_t run_sweep_plan(dagbound_batch* b, const SweepArgs& a, hipStream_t st) {
  const hipError_t ea = ensure_adj(b, st);
  if (ea != hipSuccess) return ea;
  // Concurrent class launches pay off when a class runs the persistent form
  // (DAGs above 128 nodes), whose grid is capped by its occupancy; the
  // one-workgroup-per-tile launches of the smaller classes each fill the
  // device alone and run faster one after the other (100,000 batched-layered
  // DAGs: 4.13 against 4.26 ms per evaluation).
  int classes = 0;
  bool wide = false;
  for (int c = 0; c < NUM_CLASSES; c++) {
    classes += b->class_off[c + 1] > b->class_off[c];
    wide = wide || (c >= 2 && b->class_off[c + 1] > b->class_off[c]);
  }
  if (!a.order || !b->class_streams || classes < 2 || !wide) return launch_sweep(a, st, nullptr);
  SweepStreams ss;
  hipError_t e = plan_resources(b, &ss);
  if (e != hipSuccess) return e;
  ss.fork = b->ev[0];
  for (int c = 0; c < NUM_CLASSES; c++) ss.join[c] = b->ev[c + 1];
  return launch_sweep(a, st, &ss);
}

}  // namespace

dagbound_status surrogate_best(dagbound_batch* b, dagbound_model* m, int32_t top_k, int32_t* best_idx,
                               int64_t* best_bound, uint32_t ptr_kind, hipStream_t st);

extern "C" {

const char* dagbound_last_error(void) { return g_err.c_str(); }

const char* dagbound_version(void) { return "libdagbound 0.1 (gfx950)"; }

dagbound_status dagbound_create_batch(int32_t num_dags, const int64_t* node_off,
                                      const int64_t* edge_off, const int32_t* edge_src,
                                      const int32_t* edge_dst, const int64_t* wcet,
                                      const int32_t* max_par, int32_t num_cus, uint32_t ptr_kind,
                                      void* hip_stream, dagbound_batch** out) {
  g_err.clear();
  if (!out) return fail(DAGBOUND_E_ARG, "out is NULL");
  if (num_dags < 0) return fail(DAGBOUND_E_ARG, "num_dags < 0");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (num_cus < 1 || num_cus > 65535) return fail(DAGBOUND_E_ARG, "num_cus %d outside [1, 65535]", num_cus);
  if (!node_off || !edge_off) return fail(DAGBOUND_E_ARG, "node_off/edge_off is NULL");
  int device = 0;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(DAGBOUND_E_DEVICE, "no HIP device");
  }
  if (hipGetDevice(&device) != hipSuccess) return fail(DAGBOUND_E_DEVICE, "hipGetDevice failed");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t D = num_dags;

  std::vector<int64_t> no = host_take(g_host64, (size_t)D + 1), eo = host_take(g_host64, (size_t)D + 1);
  if (ptr_kind == DAGBOUND_PTR_HOST) {
    memcpy(no.data(), node_off, (D + 1) * sizeof(int64_t));
    memcpy(eo.data(), edge_off, (D + 1) * sizeof(int64_t));
  } else {
    hipError_t e = hipMemcpyAsync(no.data(), node_off, (D + 1) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(eo.data(), edge_off, (D + 1) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading node_off/edge_off");
  }
  if (no[0] != 0 || eo[0] != 0) return fail(DAGBOUND_E_ARG, "node_off[0] and edge_off[0] must be 0");
  // checks, largest sizes, and the size class of each DAG (a byte per DAG
  // for the grouping below) in one pass
  static_assert(NUM_CLASSES == 5 && LARGE_CLASS == 4, "class bounds 64, 128, 256, 512");
  static thread_local std::vector<uint8_t> cls;
  cls.resize((size_t)D);
  int64_t max_n = 0, max_e = 0;
  for (int64_t d = 0; d < D; d++) {
    const int64_t n = no[d + 1] - no[d], e = eo[d + 1] - eo[d];
    if (n < 0 || e < 0) return fail(DAGBOUND_E_ARG, "DAG %lld: offsets decrease", (long long)d);
    if (n > DAGBOUND_MAX_NODES_PER_DAG)
      return fail(DAGBOUND_E_UNSUPPORTED, "DAG %lld has %lld nodes; the library handles at most %d",
                  (long long)d, (long long)n, DAGBOUND_MAX_NODES_PER_DAG);
    max_n = std::max(max_n, n);
    max_e = std::max(max_e, e);
    cls[(size_t)d] = (uint8_t)((n > 64) + (n > 128) + (n > 256) + (n > 512));
  }
  const int64_t tn = no[D], te = eo[D];
  if (tn > 0 && (!wcet || !max_par)) return fail(DAGBOUND_E_ARG, "wcet/max_par is NULL");
  if (te > 0 && (!edge_src || !edge_dst)) return fail(DAGBOUND_E_ARG, "edge_src/edge_dst is NULL");

  dagbound_batch* b = new dagbound_batch();
  b->device = device;
  b->D = num_dags;
  b->M = num_cus;
  b->tn = tn;
  b->te = te;
  b->max_n = (int32_t)max_n;
  b->max_e = (int32_t)std::min<int64_t>(max_e, INT32_MAX);
  b->node_off = std::move(no);
  b->edge_off = std::move(eo);
  const int64_t* nh = b->node_off.data();
  const int64_t* eh = b->edge_off.data();
  int32_t class_max_e[NUM_CLASSES] = {};  // most edges of a DAG of each class
  {
    // DAG ids grouped by size class, in id order within a class: a
    // counting sort over the class bytes (four interleaved counters, so no
    // counter waits on its own last store), then the largest DAG of each
    // class from its own range
    int64_t c4[4][NUM_CLASSES] = {};
    const int64_t D4 = D & ~(int64_t)3;
    for (int64_t d = 0; d < D4; d += 4) {
      c4[0][cls[(size_t)d]]++;
      c4[1][cls[(size_t)d + 1]]++;
      c4[2][cls[(size_t)d + 2]]++;
      c4[3][cls[(size_t)d + 3]]++;
    }
    for (int64_t d = D4; d < D; d++) c4[0][cls[(size_t)d]]++;
    int64_t pos[NUM_CLASSES];
    b->class_off[0] = 0;
    for (int c = 0; c < NUM_CLASSES; c++) {
      pos[c] = b->class_off[c];
      b->class_off[c + 1] = (int32_t)(b->class_off[c] + c4[0][c] + c4[1][c] + c4[2][c] + c4[3][c]);
    }
    b->order_host = host_take(g_host32, (size_t)D);
    int32_t* ord = b->order_host.data();
    for (int64_t d = 0; d < D; d++) ord[pos[cls[(size_t)d]]++] = (int32_t)d;
    for (int c = 0; c < NUM_CLASSES; c++) {
      int64_t mn = 0, me = 0;
      for (int64_t i = b->class_off[c]; i < b->class_off[c + 1]; i++) {
        const int32_t d = ord[i];
        mn = std::max(mn, nh[d + 1] - nh[d]);
        me = std::max(me, eh[d + 1] - eh[d]);
      }
      b->class_max_n[c] = (int32_t)mn;
      class_max_e[c] = (int32_t)std::min<int64_t>(me, INT32_MAX);
    }
  }
  const int32_t n_records = b->class_off[LARGE_CLASS + 1] - b->class_off[3];
  const size_t gres_words = sweep_gres_words(b->class_max_n, b->class_off, (int32_t)max_n, b->gres_off);
  const size_t rows_words = sweep_rows_words(b->class_max_n, b->class_off, (int32_t)max_n, b->rows_off);
  // adjacency rows: 2 * (words of the largest DAG up to 512 nodes) per node
  int32_t adj_max_n = 0;
  for (int c = 0; c < LARGE_CLASS; c++)
    if (b->class_off[c + 1] > b->class_off[c]) adj_max_n = std::max(adj_max_n, b->class_max_n[c]);
  const int32_t adj_node = adj_max_n > 0 ? 2 * row_words(adj_max_n) : 0;
  const size_t adj_words = (size_t)adj_node * (size_t)tn;
  b->block_size = table_bytes(D, tn, te, gres_words, n_records > 0) + rows_words * 8 + adj_words * 8 + 512;
  hipError_t e = dev_alloc(&b->block, &b->block_size, device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "allocating batch tables");
  }
  Carve cv(b->block);
  int64_t* d_no = cv.take<int64_t>(D + 1);
  int64_t* d_eo = cv.take<int64_t>(D + 1);
  b->t.node_off = d_no;
  b->t.edge_off = d_eo;
  b->t.wanc = cv.take<int64_t>(tn);
  b->best = cv.take<unsigned long long>(D);
  b->err = cv.take<unsigned long long>(3);
  b->gres = cv.take<uint32_t>(gres_words);
  if (rows_words) b->grows = cv.take<uint64_t>(rows_words);
  b->t.adj = adj_words ? cv.take<uint64_t>(adj_words) : nullptr;
  b->t.adj_node = adj_node;
  b->t.wc = cv.take<uint32_t>(tn);
  b->t.soff = cv.take<uint32_t>(tn + D);
  b->t.ngroups = cv.take<int32_t>(D);
  b->t.gl = cv.take<uint16_t>(tn);
  b->t.pp = cv.take<uint16_t>(tn);
  b->t.mx = cv.take<uint32_t>(tn);
  b->t.indeg = cv.take<uint16_t>(tn);
  b->t.inv = cv.take<uint16_t>(tn);
  b->t.succ = cv.take<uint16_t>(te);
  b->order = cv.take<int32_t>(D);
  if (n_records > 0) {  // DAGs above 256 nodes may run the lane-per-node kernel
    b->t.nrec = cv.take<uint4>(tn);
    b->t.mrec = cv.take<uint4>(tn);
  }

  // Inputs: device pointers are read in place; host arrays go through a
  // staging block that is released when this call returns.
  PrepInputs in{edge_src, edge_dst, wcet, max_par};
  void* stage = nullptr;
  size_t stage_size = 0;
  // the offsets are already on the device when the caller passes device
  // pointers: copy them there instead of back from the host copies
  const hipMemcpyKind okind = ptr_kind == DAGBOUND_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  e = hipMemcpyAsync(d_no, ptr_kind == DAGBOUND_PTR_DEVICE ? (const void*)node_off : (const void*)nh, (D + 1) * 8, okind, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_eo, ptr_kind == DAGBOUND_PTR_DEVICE ? (const void*)edge_off : (const void*)eh, (D + 1) * 8, okind, st);
  if (e == hipSuccess && D > 0)
    e = hipMemcpyAsync(b->order, b->order_host.data(), (size_t)D * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && ptr_kind == DAGBOUND_PTR_HOST && (tn + te) > 0) {
    stage_size = 4 * 256 + (size_t)te * 8 + (size_t)tn * 12;
    e = dev_alloc(&stage, &stage_size, device);
    if (e == hipSuccess) {
      Carve sc(stage);
      int32_t* s_src = sc.take<int32_t>(te);
      int32_t* s_dst = sc.take<int32_t>(te);
      int64_t* s_w = sc.take<int64_t>(tn);
      int32_t* s_p = sc.take<int32_t>(tn);
      e = hipMemcpyAsync(s_src, edge_src, te * 4, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(s_dst, edge_dst, te * 4, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(s_w, wcet, tn * 8, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(s_p, max_par, tn * 4, hipMemcpyHostToDevice, st);
      in = PrepInputs{s_src, s_dst, s_w, s_p};
    }
  }
  if (e == hipSuccess) e = hipMemsetAsync(b->err, 0xFF, sizeof(unsigned long long), st);
  if (e == hipSuccess) e = hipMemsetAsync(b->err + 1, 0, 2 * sizeof(unsigned long long), st);
  // global scratch of the workgroup-per-DAG preprocessing (DAGs above 256
  // nodes), released with the staging
  void* lscratch = nullptr;
  size_t lscratch_size = 0;
  for (int c = 3; c <= LARGE_CLASS; c++)
    lscratch_size = std::max(lscratch_size, prep_large_scratch_bytes(b->class_off[c + 1] - b->class_off[c],
                                                                     b->class_max_n[c], class_max_e[c]));
  if (e == hipSuccess && lscratch_size > 0) {
    e = dev_alloc(&lscratch, &lscratch_size, device);
    if (e != hipSuccess) lscratch = nullptr;
  }
  // the size classes' preprocessing launches run beside each other on the
  // side streams (their events are the batch's, later used by the evaluation)
  hipStream_t side[NUM_CLASSES] = {};
  bool fork_ok = e == hipSuccess && side_streams(device, side) == hipSuccess;
  for (int i = 0; i <= NUM_CLASSES && fork_ok; i++)
    if (!b->ev[i]) fork_ok = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) == hipSuccess;
  if (!fork_ok) (void)hipGetLastError();
  if (e == hipSuccess)
    e = launch_prep(b->t, in, num_dags, num_cus, (int32_t)max_n, b->order, b->class_off, b->err, lscratch,
                    b->class_max_n, class_max_e, fork_ok ? side : nullptr, fork_ok ? b->ev[0] : nullptr,
                    fork_ok ? b->ev + 1 : nullptr, st);
  // adjacency rows of each size class (they read the successor lists
  // clamped to each DAG's ranges: safe before the validation below)
  if (e == hipSuccess && b->t.adj) e = launch_adj(b->t, b->order, b->class_off, b->class_max_n, 0, st);
  unsigned long long errw[2] = {~0ull, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(errw, b->err, sizeof errw, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dev_release(stage, stage_size, device);
  dev_release(lscratch, lscratch_size, device);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "preprocessing");
  }
  const unsigned long long err = errw[0];
  b->small_loads = (errw[1] & 1) == 0;
  b->small_indeg = (errw[1] & 2) == 0;
  if (err != ~0ull) {
    const long long d = (long long)(err >> 8);
    const unsigned code = (unsigned)(err & 0xFF);
    batch_free(b);
    switch (code) {
      case PREP_E_CYCLE: return fail(DAGBOUND_E_CYCLE, "DAG %lld has a cycle or a self-loop", d);
      case PREP_E_RANGE: return fail(DAGBOUND_E_RANGE, "DAG %lld: node id, load or parallelism out of range", d);
      case PREP_E_DUP: return fail(DAGBOUND_E_DUP_EDGE, "DAG %lld lists an edge twice", d);
      case PREP_E_OVERFLOW: return fail(DAGBOUND_E_OVERFLOW, "DAG %lld: summed load reaches 2^40", d);
      default: return fail(DAGBOUND_E_DEVICE, "DAG %lld: internal preprocessing error %u", d, code);
    }
  }
  // Checked after validation, so an invalid DAG reports its own error first.
  if (sweep_lds_need((int)max_n, (int)b->max_e) > LDS_LIMIT) {
    batch_free(b);
    return fail(DAGBOUND_E_UNSUPPORTED,
                "largest DAG (%lld nodes, %lld edges) exceeds the evaluation kernel's LDS budget",
                (long long)max_n, (long long)max_e);
  }
  *out = b;
  return DAGBOUND_OK;
}

dagbound_status dagbound_set_allocations(dagbound_batch* b, int32_t K, uint32_t mode,
                                         const uint8_t* alloc, uint64_t seed, uint32_t ptr_kind) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (K < 1 || K > DAGBOUND_MAX_CANDIDATES) return fail(DAGBOUND_E_ARG, "K = %d outside [1, %d]", K, DAGBOUND_MAX_CANDIDATES);
  if (mode > DAGBOUND_ALLOC_SEEDED) return fail(DAGBOUND_E_ARG, "bad mode %u", mode);
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  DeviceGuard g(b->device);
  if (mode == DAGBOUND_ALLOC_EXPLICIT) {
    if (b->tn > 0 && !alloc) return fail(DAGBOUND_E_ARG, "alloc is NULL");
    const size_t bytes = (size_t)K * (size_t)b->tn;
    if (ptr_kind == DAGBOUND_PTR_HOST && bytes > 0) {
      if (b->alloc_owned_size < bytes) {
        dev_release(b->alloc_owned, b->alloc_owned_size, b->device);
        b->alloc_owned = nullptr;
        b->alloc_owned_size = bytes;
        hipError_t e = dev_alloc(&b->alloc_owned, &b->alloc_owned_size, b->device);
        if (e != hipSuccess) {
          b->alloc_owned = nullptr;
          b->alloc_owned_size = 0;
          b->has_alloc = false;
          return hip_fail(e, "allocating candidate bytes");
        }
      }
      hipError_t e = hipMemcpy(b->alloc_owned, alloc, bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        b->has_alloc = false;
        return hip_fail(e, "copying candidate bytes");
      }
      b->alloc = (const uint8_t*)b->alloc_owned;
    } else {
      b->alloc = alloc;
    }
  } else {
    b->alloc = nullptr;
    b->seed = seed;
  }
  const size_t tiles = (size_t)b->D * (size_t)((K + 63) / 64);
  const size_t need = 512 + COUNTERS_PER_CLASS * NUM_CLASSES * 4 + tiles * 4;
  if (b->ovf_block_size < need) {
    dev_release(b->ovf_block, b->ovf_block_size, b->device);
    b->ovf_block = nullptr;
    b->ovf_block_size = need;
    hipError_t e = dev_alloc(&b->ovf_block, &b->ovf_block_size, b->device);
    if (e != hipSuccess) {
      b->ovf_block = nullptr;
      b->ovf_block_size = 0;
      b->has_alloc = false;
      return hip_fail(e, "allocating evaluation scratch");
    }
  }
  Carve oc(b->ovf_block);
  b->ovf_count = oc.take<uint32_t>(COUNTERS_PER_CLASS * NUM_CLASSES);
  b->ovf_list = oc.take<uint32_t>(tiles);
  b->K = K;
  b->mode = mode;
  b->has_alloc = true;
  b->alloc_gen++;
  return DAGBOUND_OK;
}

dagbound_status dagbound_eval_bounds(dagbound_batch* b, int64_t* bounds, int64_t* cp_term,
                                     int64_t* intf_term, uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  const size_t n = (size_t)b->D * (size_t)b->K;
  if (!bounds && n > 0) return fail(DAGBOUND_E_ARG, "bounds is NULL");
  DeviceGuard g(b->device);
  hipStream_t st = (hipStream_t)hip_stream;
  SweepArgs a = sweep_args(b);
  void* tmp = nullptr;
  size_t tmp_size = 0;
  hipError_t e = hipSuccess;
  if (ptr_kind == DAGBOUND_PTR_HOST && n > 0) {
    tmp_size = 3 * 256 + n * 8 * (1 + (cp_term != nullptr) + (intf_term != nullptr));
    e = dev_alloc(&tmp, &tmp_size, b->device);
    if (e != hipSuccess) return hip_fail(e, "allocating output staging");
    Carve c(tmp);
    a.bounds = c.take<int64_t>(n);
    a.cp = cp_term ? c.take<int64_t>(n) : nullptr;
    a.intf = intf_term ? c.take<int64_t>(n) : nullptr;
  } else {
    a.bounds = bounds;
    a.cp = cp_term;
    a.intf = intf_term;
  }
  a.best = b->best;
  if (b->use_graph && ptr_kind == DAGBOUND_PTR_DEVICE && st && !b->autotune_pending) {
    // record the launches once for these outputs, stream, candidates and
    // tuning; replay the graph afterwards
    const void* key[4] = {bounds, cp_term, intf_term, st};
    bool same = b->gexec && b->g_gen == b->alloc_gen && b->g_tune == b->tune_gen;
    for (int i = 0; i < 4; i++) same = same && b->g_key[i] == key[i];
    if (!same) {
      if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
      SweepStreams ss;
      e = plan_resources(b, &ss);
      hipGraph_t graph = nullptr;
      if (e == hipSuccess) e = ensure_adj(b, st);  // outside the graph
      if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        const hipError_t el = run_sweep_plan(b, a, st);
        e = hipStreamEndCapture(st, &graph);
        if (e == hipSuccess) e = el;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e == hipSuccess) {
        for (int i = 0; i < 4; i++) b->g_key[i] = key[i];
        b->g_gen = b->alloc_gen;
        b->g_tune = b->tune_gen;
      } else {
        b->gexec = nullptr;
      }
    }
    if (e == hipSuccess) e = hipGraphLaunch(b->gexec, st);
  } else {
    e = run_sweep(b, a, st);
  }
  if (e == hipSuccess && ptr_kind == DAGBOUND_PTR_HOST && n > 0) {
    e = hipMemcpyAsync(bounds, a.bounds, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && cp_term) e = hipMemcpyAsync(cp_term, a.cp, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && intf_term) e = hipMemcpyAsync(intf_term, a.intf, n * 8, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess && (ptr_kind == DAGBOUND_PTR_HOST || !st)) e = hipStreamSynchronize(st);
  if (tmp) {
    if (e != hipSuccess) (void)hipDeviceSynchronize();
    dev_release(tmp, tmp_size, b->device);
  }
  if (e != hipSuccess) {
    b->best_gen = ~0ull;
    return hip_fail(e, "evaluating bounds");
  }
  b->best_gen = b->alloc_gen;
  return DAGBOUND_OK;
}

dagbound_status dagbound_best_allocation(dagbound_batch* b, uint32_t search, int32_t top_k,
                                         const dagbound_model* model, int32_t* best_idx,
                                         int64_t* best_bound, uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  (void)top_k;
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if ((!best_idx || !best_bound) && b->D > 0) return fail(DAGBOUND_E_ARG, "best_idx/best_bound is NULL");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (search == DAGBOUND_SEARCH_SURROGATE) {
    if (!model) return fail(DAGBOUND_E_ARG, "surrogate search needs a model");
    if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
    if (b->mode != DAGBOUND_ALLOC_SEEDED) return fail(DAGBOUND_E_ARG, "surrogate search needs seeded candidates");
    if (top_k < 1 || top_k > 255 || top_k >= b->K)
      return fail(DAGBOUND_E_ARG, "top_k = %d outside [1, min(255, K-1)]", top_k);
    return surrogate_best(b, const_cast<dagbound_model*>(model), top_k, best_idx, best_bound, ptr_kind,
                          (hipStream_t)hip_stream);
  }
  if (search != DAGBOUND_SEARCH_EXHAUSTIVE) return fail(DAGBOUND_E_ARG, "bad search %u", search);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  DeviceGuard g(b->device);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = hipSuccess;
  if (b->best_gen != b->alloc_gen) {
    SweepArgs a = sweep_args(b);
    a.best = b->best;
    e = run_sweep(b, a, st);
    if (e != hipSuccess) {
      b->best_gen = ~0ull;
      return hip_fail(e, "evaluating bounds");
    }
    b->best_gen = b->alloc_gen;
  }
  void* tmp = nullptr;
  size_t tmp_size = 0;
  int32_t* oi = best_idx;
  int64_t* ob = best_bound;
  if (ptr_kind == DAGBOUND_PTR_HOST && b->D > 0) {
    tmp_size = 512 + (size_t)b->D * 12;
    e = dev_alloc(&tmp, &tmp_size, b->device);
    if (e != hipSuccess) return hip_fail(e, "allocating output staging");
    Carve c(tmp);
    ob = c.take<int64_t>(b->D);
    oi = c.take<int32_t>(b->D);
  }
  e = launch_best_final(b->best, b->D, oi, ob, nullptr, 0, st);
  if (e == hipSuccess && ptr_kind == DAGBOUND_PTR_HOST && b->D > 0) {
    e = hipMemcpyAsync(best_idx, oi, (size_t)b->D * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(best_bound, ob, (size_t)b->D * 8, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess && (ptr_kind == DAGBOUND_PTR_HOST || !st)) e = hipStreamSynchronize(st);
  if (tmp) {
    if (e != hipSuccess) (void)hipDeviceSynchronize();
    dev_release(tmp, tmp_size, b->device);
  }
  if (e != hipSuccess) return hip_fail(e, "selecting best candidates");
  return DAGBOUND_OK;
}

dagbound_status dagbound_get_division(dagbound_batch* b, int32_t d, int64_t* wanc,
                                      int32_t* group_of, int32_t* order, int32_t* num_groups) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (d < 0 || d >= b->D) return fail(DAGBOUND_E_ARG, "DAG index %d outside [0, %d)", d, b->D);
  DeviceGuard g(b->device);
  const int64_t n0 = b->node_off[d];
  const int n = (int)(b->node_off[d + 1] - n0);
  std::vector<uint16_t> gl(n), inv(n);
  std::vector<int64_t> w(n);
  int32_t ng = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && n > 0) e = hipMemcpy(gl.data(), b->t.gl + n0, n * 2, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n > 0) e = hipMemcpy(inv.data(), b->t.inv + n0, n * 2, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n > 0) e = hipMemcpy(w.data(), b->t.wanc + n0, n * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&ng, b->t.ngroups + d, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "reading division tables");
  std::vector<int32_t> perm(n);
  for (int v = 0; v < n; v++) perm[inv[v]] = v;
  int gi = 0;
  for (int i = 0; i < n; i++) {
    const int v = perm[gl[i] & 0x7FFF];
    if (order) order[i] = v;
    if (group_of) group_of[v] = gi;
    if (gl[i] & 0x8000) gi++;
  }
  if (wanc) std::copy(w.begin(), w.end(), wanc);
  if (num_groups) *num_groups = ng;
  return DAGBOUND_OK;
}

// Every record of the schedule of (d, c) into `rec` (host), and its terms.
static hipError_t schedule_all(dagbound_batch* b, int32_t d, int32_t c, std::vector<int64_t>& rec,
                               int64_t terms[3]) {
  int64_t cap = 4096;
  for (int attempt = 0; attempt < 2; attempt++) {
    void* tmp = nullptr;
    size_t tmp_size = 256 + 64 + (size_t)cap * 64;
    hipError_t e = dev_alloc(&tmp, &tmp_size, b->device);
    if (e != hipSuccess) return e;
    Carve cv(tmp);
    int64_t* d_out = cv.take<int64_t>(4);
    int64_t* d_rec = cv.take<int64_t>((size_t)cap * 8);
    e = hipDeviceSynchronize();
    if (e == hipSuccess)
      e = launch_schedule(b->t, d, c, b->K, b->M, b->mode == DAGBOUND_ALLOC_EXPLICIT ? b->alloc : nullptr, b->seed,
                          b->max_n, d_rec, cap, d_out, b->para_mode, nullptr);
    int64_t out[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpy(out, d_out, sizeof out, hipMemcpyDeviceToHost);
    if (e == hipSuccess && out[0] <= cap) {
      rec.resize((size_t)out[0] * 8);
      if (out[0] > 0) e = hipMemcpy(rec.data(), d_rec, (size_t)out[0] * 64, hipMemcpyDeviceToHost);
      for (int i = 0; i < 3; i++) terms[i] = out[i + 1];
      dev_release(tmp, tmp_size, b->device);
      return e;
    }
    dev_release(tmp, tmp_size, b->device);
    if (e != hipSuccess) return e;
    cap = out[0];
  }
  return hipErrorUnknown;
}

dagbound_status dagbound_run_schedule(dagbound_batch* b, int32_t d, int32_t c, int64_t tick_ns, int32_t barriers,
                                      int32_t reps, int64_t* makespan_ns, int64_t* terms) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (d < 0 || d >= b->D) return fail(DAGBOUND_E_ARG, "DAG index %d outside [0, %d)", d, b->D);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  if (c < 0 || c >= b->K) return fail(DAGBOUND_E_ARG, "candidate %d outside [0, %d)", c, b->K);
  if (tick_ns < 1000 || tick_ns > 10000000) return fail(DAGBOUND_E_ARG, "tick_ns %lld outside [1000, 1e7]", (long long)tick_ns);
  if (reps < 1 || reps > 100000 || !makespan_ns) return fail(DAGBOUND_E_ARG, "bad reps or makespan buffer");
  if (barriers != 0 && barriers != 1) return fail(DAGBOUND_E_ARG, "barriers must be 0 or 1");
  DeviceGuard g(b->device);
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) return hip_fail(e, "device attributes");
  if (b->M > cus) return fail(DAGBOUND_E_ARG, "M = %d exceeds the device's %d compute units", b->M, cus);
  std::vector<int64_t> rec;
  int64_t t3[3] = {0, 0, 0};
  e = schedule_all(b, d, c, rec, t3);
  if (e != hipSuccess) return hip_fail(e, "schedule dump");
  // the expected run time, bound x tick per run, stays within two minutes
  if ((double)t3[0] * (double)tick_ns * (double)(reps + 1) > 120e9)
    return fail(DAGBOUND_E_ARG, "bound %lld x tick x runs exceeds two minutes", (long long)t3[0]);
  const int64_t n0 = b->node_off[d], n1 = b->node_off[d + 1];
  const int32_t N = (int32_t)(n1 - n0);
  std::vector<int32_t> es, ed;
  if (!barriers && N > 0) {
    // the DAG's edges in local ids, from the tables by sigma rank
    const int64_t e0 = b->edge_off[d], e1 = b->edge_off[d + 1];
    std::vector<uint32_t> soff((size_t)N + 1);
    std::vector<uint16_t> succ((size_t)(e1 - e0) + 1), inv((size_t)N);
    e = hipMemcpy(soff.data(), b->t.soff + n0 + d, ((size_t)N + 1) * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && e1 > e0) e = hipMemcpy(succ.data(), b->t.succ + e0, (size_t)(e1 - e0) * 2, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(inv.data(), b->t.inv + n0, (size_t)N * 2, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the DAG's tables");
    std::vector<int32_t> perm((size_t)N, 0);
    for (int32_t v = 0; v < N; v++) perm[inv[v]] = v;
    for (int32_t s = 0; s < N; s++)
      for (uint32_t k = soff[s]; k < soff[s + 1]; k++) {
        es.push_back(perm[s]);
        ed.push_back(perm[succ[k]]);
      }
  }
  int32_t nparts = 0;
  e = realize_schedule(rec.data(), (int64_t)(rec.size() / 8), N, es.data(), ed.data(), (int32_t)es.size(), tick_ns,
                       barriers != 0, reps, makespan_ns, &nparts);
  if (e != hipSuccess) return hip_fail(e, "running the schedule's graph");
  if (terms) {
    for (int i = 0; i < 3; i++) terms[i] = t3[i];
    terms[3] = nparts;
  }
  return DAGBOUND_OK;
}

dagbound_status dagbound_get_schedule(dagbound_batch* b, int32_t d, int32_t c, int64_t* records, int64_t cap,
                                      int64_t* count, int64_t* terms) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (d < 0 || d >= b->D) return fail(DAGBOUND_E_ARG, "DAG index %d outside [0, %d)", d, b->D);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  if (c < 0 || c >= b->K) return fail(DAGBOUND_E_ARG, "candidate %d outside [0, %d)", c, b->K);
  if (cap < 0 || (cap > 0 && !records)) return fail(DAGBOUND_E_ARG, "bad record buffer");
  DeviceGuard g(b->device);
  void* tmp = nullptr;
  size_t tmp_size = 256 + 64 + (size_t)cap * 64;
  hipError_t e = dev_alloc(&tmp, &tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "allocating schedule records");
  Carve cv(tmp);
  int64_t* d_out = cv.take<int64_t>(4);
  int64_t* d_rec = cv.take<int64_t>((size_t)cap * 8);
  e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = launch_schedule(b->t, d, c, b->K, b->M, b->mode == DAGBOUND_ALLOC_EXPLICIT ? b->alloc : nullptr, b->seed,
                        b->max_n, d_rec, cap, d_out, b->para_mode, nullptr);
  int64_t out[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpy(out, d_out, sizeof out, hipMemcpyDeviceToHost);
  if (e == hipSuccess && cap > 0 && out[0] > 0)
    e = hipMemcpy(records, d_rec, (size_t)std::min<int64_t>(out[0], cap) * 64, hipMemcpyDeviceToHost);
  dev_release(tmp, tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "schedule dump");
  if (count) *count = out[0];
  if (terms) {
    terms[0] = out[1];
    terms[1] = out[2];
    terms[2] = out[3];
  }
  return DAGBOUND_OK;
}

dagbound_status dagbound_baselines(dagbound_batch* b, int64_t* greedy, int64_t* greedy_unaware,
                                  int64_t* graham_para, uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  const size_t n = (size_t)b->D;
  int64_t* out[3] = {greedy, greedy_unaware, graham_para};
  if (n == 0 || (!greedy && !greedy_unaware && !graham_para)) return DAGBOUND_OK;
  DeviceGuard g(b->device);
  hipStream_t st = (hipStream_t)hip_stream;
  int64_t* dv[3] = {greedy, greedy_unaware, graham_para};
  void* tmp = nullptr;
  size_t tmp_size = 0;
  hipError_t e = hipSuccess;
  if (ptr_kind == DAGBOUND_PTR_HOST) {
    tmp_size = 3 * 256 + 3 * n * 8;
    e = dev_alloc(&tmp, &tmp_size, b->device);
    if (e != hipSuccess) return hip_fail(e, "allocating output staging");
    Carve c(tmp);
    for (int i = 0; i < 3; i++) dv[i] = out[i] ? c.take<int64_t>(n) : nullptr;
  }
  e = launch_baselines(b->t, b->D, b->M, b->max_n, b->max_e, dv[0], dv[1], dv[2], st);
  for (int i = 0; i < 3 && e == hipSuccess && ptr_kind == DAGBOUND_PTR_HOST; i++)
    if (out[i]) e = hipMemcpyAsync(out[i], dv[i], n * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && (ptr_kind == DAGBOUND_PTR_HOST || !st)) e = hipStreamSynchronize(st);
  if (tmp) {
    if (e != hipSuccess) (void)hipDeviceSynchronize();
    dev_release(tmp, tmp_size, b->device);
  }
  if (e != hipSuccess) return hip_fail(e, "comparison bounds");
  return DAGBOUND_OK;
}

dagbound_status dagbound_set_para_launch(dagbound_batch* b, uint32_t mode) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (mode != DAGBOUND_PARA_SPATIAL && mode != DAGBOUND_PARA_TEMPORAL) return fail(DAGBOUND_E_ARG, "bad mode %u", mode);
  if (b->para_mode != (int32_t)mode) {
    b->para_mode = (int32_t)mode;
    b->best_gen = ~0ull;  // results change: the cached minimum and any recorded graph are stale
    b->tune_gen++;
  }
  return DAGBOUND_OK;
}

dagbound_status dagbound_set_tuning(dagbound_batch* b, const char* key, int64_t value) {
  g_err.clear();
  if (!b || !key) return fail(DAGBOUND_E_ARG, "batch or key is NULL");
  if (!strcmp(key, "residual_slots")) {
    if (value < 1 || value > RES_SLOTS) return fail(DAGBOUND_E_ARG, "residual_slots outside [1, %d]", RES_SLOTS);
    b->res_slots = (int32_t)value;
  } else if (!strcmp(key, "eval_path")) {
    if (value != EVAL_PATH_AUTO && value != EVAL_PATH_GLOBAL) return fail(DAGBOUND_E_ARG, "eval_path must be 0 or 1");
    b->eval_path = (int32_t)value;
  } else if (!strcmp(key, "size_classes")) {
    if (value != 0 && value != 1) return fail(DAGBOUND_E_ARG, "size_classes must be 0 or 1");
    b->size_classes = value != 0;
  } else if (!strcmp(key, "class_streams")) {
    if (value != 0 && value != 1) return fail(DAGBOUND_E_ARG, "class_streams must be 0 or 1");
    b->class_streams = value != 0;
  } else if (!strcmp(key, "persistent")) {
    if (value != 0 && value != 1) return fail(DAGBOUND_E_ARG, "persistent must be 0 or 1");
    b->persistent = value != 0;
  } else if (!strcmp(key, "autotune")) {
    if (value != 0 && value != 1) return fail(DAGBOUND_E_ARG, "autotune must be 0 or 1");
    b->autotune_pending = value != 0;
  } else if (!strcmp(key, "node_lanes")) {
    if (value != 256 && value != 512) return fail(DAGBOUND_E_ARG, "node_lanes must be 256 or 512");
    b->node_lanes_class = value == 256 ? 3 : LARGE_CLASS;
  } else if (!strcmp(key, "graph")) {
    if (value != 0 && value != 1) return fail(DAGBOUND_E_ARG, "graph must be 0 or 1");
    b->use_graph = value != 0;
  } else {
    return fail(DAGBOUND_E_ARG, "unknown tuning key '%s'", key);
  }
  b->best_gen = ~0ull;
  b->tune_gen++;
  return DAGBOUND_OK;
}

dagbound_status dagbound_eval_listed(dagbound_batch* b, int32_t L, const int32_t* cand, int64_t* bounds,
                                     int64_t* cp_term, int64_t* intf_term, uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  if (L < 1 || L > DAGBOUND_MAX_CANDIDATES) return fail(DAGBOUND_E_ARG, "L = %d outside [1, %d]", L, DAGBOUND_MAX_CANDIDATES);
  const size_t n = (size_t)b->D * (size_t)L;
  if (n > 0 && (!cand || !bounds)) return fail(DAGBOUND_E_ARG, "cand/bounds is NULL");
  if (n == 0) return DAGBOUND_OK;
  DeviceGuard g(b->device);
  hipStream_t st = (hipStream_t)hip_stream;
  const bool host = ptr_kind == DAGBOUND_PTR_HOST;
  if (host) {
    for (size_t i = 0; i < n; i++)
      if (cand[i] < 0 || cand[i] >= b->K)
        return fail(DAGBOUND_E_ARG, "cand[%zu] = %d outside [0, %d)", i, cand[i], b->K);
  }
  void* tmp = nullptr;
  // tiles handed to the second evaluation pass are listed per call: the
  // batch's list holds the allocation set's tiles, a list may have more
  const size_t tiles = (size_t)b->D * (size_t)((L + 63) / 64);
  size_t tmp_size = 6 * 256 + n * 4 + 4 + tiles * 4 +
                    (host ? n * 8 * (1 + (cp_term != nullptr) + (intf_term != nullptr)) : 0);
  hipError_t e = dev_alloc(&tmp, &tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "allocating list scratch");
  Carve c(tmp);
  uint32_t* bad = c.take<uint32_t>(1);
  SweepArgs a = sweep_args(b);
  a.K = L;
  a.ovf_list = c.take<uint32_t>(tiles);
  a.best = b->best;
  if (host) {
    int32_t* dl = c.take<int32_t>(n);
    e = hipMemcpyAsync(dl, cand, n * 4, hipMemcpyHostToDevice, st);
    a.cand_list = dl;
    a.bounds = c.take<int64_t>(n);
    a.cp = cp_term ? c.take<int64_t>(n) : nullptr;
    a.intf = intf_term ? c.take<int64_t>(n) : nullptr;
  } else {
    // ids out of range are an argument error: checked on the device first
    uint32_t nbad = 0;
    e = launch_check_list(cand, (int64_t)n, b->K, bad, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && nbad) {
      dev_release(tmp, tmp_size, b->device);
      return fail(DAGBOUND_E_ARG, "%u entries of cand outside [0, %d)", nbad, b->K);
    }
    a.cand_list = cand;
    a.bounds = bounds;
    a.cp = cp_term;
    a.intf = intf_term;
  }
  if (e == hipSuccess) e = run_sweep(b, a, st);
  b->best_gen = ~0ull;  // the per-DAG minimum now holds list positions
  if (e == hipSuccess && host) {
    e = hipMemcpyAsync(bounds, a.bounds, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && cp_term) e = hipMemcpyAsync(cp_term, a.cp, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && intf_term) e = hipMemcpyAsync(intf_term, a.intf, n * 8, hipMemcpyDeviceToHost, st);
  }
  // the list scratch is released below, so the work is waited for
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  dev_release(tmp, tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "evaluating listed candidates");
  return DAGBOUND_OK;
}

dagbound_status dagbound_eval_conditional(dagbound_batch* b, const int32_t* cond_of, const int32_t* branch_of,
                                          int64_t* bounds, int32_t* worst, uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  if (!b) return fail(DAGBOUND_E_ARG, "batch is NULL");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  if (b->para_mode != DAGBOUND_PARA_SPATIAL)
    return fail(DAGBOUND_E_UNSUPPORTED, "conditional DAGs are evaluated under the spatial launching reading only");
  if (b->max_n > 512) return fail(DAGBOUND_E_UNSUPPORTED, "conditional DAGs of more than 512 nodes are not supported");
  const int64_t D = b->D, K = b->K, T = b->tn;
  if (D * K == 0) return DAGBOUND_OK;
  if (!bounds) return fail(DAGBOUND_E_ARG, "bounds is NULL");
  if (T > 0 && (!cond_of || !branch_of)) return fail(DAGBOUND_E_ARG, "cond_of/branch_of is NULL");
  DeviceGuard g(b->device);
  hipStream_t st = (hipStream_t)hip_stream;
  const bool host = ptr_kind == DAGBOUND_PTR_HOST;
  std::vector<int32_t> co((size_t)T), br((size_t)T);
  std::vector<uint16_t> inv((size_t)T);
  hipError_t e = hipSuccess;
  if (host) {
    std::copy(cond_of, cond_of + T, co.begin());
    std::copy(branch_of, branch_of + T, br.begin());
  } else {
    e = hipMemcpyAsync(co.data(), cond_of, (size_t)T * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(br.data(), branch_of, (size_t)T * 4, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(inv.data(), b->t.inv, (size_t)T * 2, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "reading the conditional structure");
  // per DAG: branches of each conditional, mixed-radix place values, realizations
  std::vector<int32_t> R((size_t)D);
  std::vector<uint32_t> tab((size_t)T);
  int32_t Rmax = 1;
  for (int64_t d = 0; d < D; d++) {
    const int64_t n0 = b->node_off[d], n1 = b->node_off[d + 1];
    int32_t nq = 0;
    for (int64_t v = n0; v < n1; v++) {
      if (co[v] < -1 || co[v] >= COND_MAX_REALIZATIONS)
        return fail(DAGBOUND_E_RANGE, "cond_of[%lld] = %d outside [-1, %d)", (long long)v, co[v], COND_MAX_REALIZATIONS);
      if (co[v] >= 0 && (br[v] < 0 || br[v] > 254))
        return fail(DAGBOUND_E_RANGE, "branch_of[%lld] = %d outside [0, 254]", (long long)v, br[v]);
      nq = std::max(nq, co[v] + 1);
    }
    std::vector<int32_t> nb((size_t)nq, 1), pre((size_t)nq, 1);
    for (int64_t v = n0; v < n1; v++)
      if (co[v] >= 0) nb[co[v]] = std::max(nb[co[v]], br[v] + 1);
    int64_t r = 1;
    for (int32_t q = 0; q < nq; q++) {
      pre[q] = (int32_t)r;
      r *= nb[q];
      if (r > COND_MAX_REALIZATIONS)
        return fail(DAGBOUND_E_RANGE, "DAG %lld has more than %d realizations", (long long)d, COND_MAX_REALIZATIONS);
    }
    R[d] = (int32_t)r;
    Rmax = std::max(Rmax, (int32_t)r);
    for (int64_t v = n0; v < n1; v++) {
      const int64_t s = n0 + inv[v];
      tab[s] = co[v] < 0 ? 1u
                         : (uint32_t)pre[co[v]] | ((uint32_t)nb[co[v]] << 13) | ((uint32_t)br[v] << 21);
    }
  }
  const int64_t L = K * Rmax;  // list entries per DAG: candidate c's realizations at c * Rmax + rho
  if (L > INT32_MAX / 2 || D * ((L + 63) / 64) > INT32_MAX)
    return fail(DAGBOUND_E_RANGE, "K x realizations = %lld per DAG is too large", (long long)L);
  void* tmp = nullptr;
  const size_t tiles = (size_t)D * (size_t)((L + 63) / 64);  // the second pass's list, per call
  size_t tmp_size = 7 * 256 + (size_t)T * 4 + (size_t)D * 4 + (size_t)(D * L) * 4 + (size_t)(D * L) * 8 +
                    tiles * 4 + (host ? (size_t)(D * K) * 12 : 0);
  e = dev_alloc(&tmp, &tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "allocating conditional scratch");
  Carve c(tmp);
  uint32_t* dtab = c.take<uint32_t>((size_t)T);
  int32_t* dR = c.take<int32_t>((size_t)D);
  int32_t* list = c.take<int32_t>((size_t)(D * L));
  int64_t* rb = c.take<int64_t>((size_t)(D * L));
  uint32_t* ovf = c.take<uint32_t>(tiles);
  int64_t* ob = host ? c.take<int64_t>((size_t)(D * K)) : bounds;
  int32_t* ow = host ? (worst ? c.take<int32_t>((size_t)(D * K)) : nullptr) : worst;
  e = hipMemcpyAsync(dtab, tab.data(), (size_t)T * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dR, R.data(), (size_t)D * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_cond_list(list, D * L, L, Rmax, st);
  if (e == hipSuccess) {
    SweepArgs a = sweep_args(b);
    a.K = (int32_t)L;
    a.ovf_list = ovf;
    a.cand_list = list;
    a.bounds = rb;
    a.cp = a.intf = nullptr;
    a.best = b->best;  // reset by the launch; the conditional kernels leave it alone
    a.cond_tab = dtab;
    a.cond_R = Rmax;
    a.node_lanes_class = LARGE_CLASS;  // the lane-per-candidate kernels of every class up to 512 nodes
    e = run_sweep_plan(b, a, st);
    b->best_gen = ~0ull;
  }
  if (e == hipSuccess) e = launch_cond_reduce(rb, dR, (int32_t)D, (int32_t)K, Rmax, ob, ow, st);
  if (e == hipSuccess && host) {
    e = hipMemcpyAsync(bounds, ob, (size_t)(D * K) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && worst) e = hipMemcpyAsync(worst, ow, (size_t)(D * K) * 4, hipMemcpyDeviceToHost, st);
  }
  // the scratch is released below, so the work is waited for
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  dev_release(tmp, tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "evaluating conditional DAGs");
  return DAGBOUND_OK;
}

void dagbound_destroy_batch(dagbound_batch* b) { batch_free(b); }

void dagbound_shutdown(void) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    cache_trim_locked(0);
  }
  std::lock_guard<std::mutex> lk(g_stream_mu);
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (size_t dev = 0; dev < g_side.size(); dev++) {
    bool any = false;
    for (hipStream_t s : g_side[dev]) any = any || s;
    if (!any) continue;
    (void)hipSetDevice((int)dev);
    for (hipStream_t& s : g_side[dev]) {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        s = nullptr;
      }
    }
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  g_side.clear();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned candidate proposal.

struct dagbound_model {
  int device = 0;
  void* block = nullptr;  // parameters, gradient, Adam moments, BF16 weights
  size_t block_size = 0;
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
  __bf16 *wfwd = nullptr, *wbwd = nullptr;
  int64_t step = 0;
  void* ws = nullptr;  // activations for the last batch size
  size_t ws_size = 0;
};

namespace {

// Glorot-uniform initial weights from the SplitMix64 finalizer of (seed, i);
// biases start at zero.
void model_init_params(uint64_t seed, std::vector<float>& h) {
  h.assign((size_t)SUR_PARAMS, 0.f);
  auto mix = [](uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  // count entries from offset off, scaled for a layer of fan_in inputs and
  // fan_out outputs (the message-passing layers see 2 * HID inputs)
  auto fill = [&](int64_t off, int64_t count, int fan_in, int fan_out) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    for (int64_t i = 0; i < count; i++) {
      const double u = (double)(mix(seed ^ mix((uint64_t)(off + i))) >> 11) / 9007199254740992.0;
      h[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * a);
    }
  };
  fill(SUR_OFF_W0, SUR_FIN * SUR_HID, SUR_FIN, SUR_HID);
  for (int l = 0; l < SUR_LAYERS; l++) {
    const int64_t o = SUR_OFF_L1 + l * SUR_LAYER_STRIDE;
    fill(o, SUR_HID * SUR_HID, 2 * SUR_HID, SUR_HID);
    fill(o + SUR_HID * SUR_HID, SUR_HID * SUR_HID, 2 * SUR_HID, SUR_HID);
  }
  fill(SUR_OFF_WA, SUR_HID * SUR_OUT, SUR_HID, SUR_OUT);
}

// Activation workspace of a batch; returns the argument block.  Inference
// (train = false) leaves out the gradient buffers (about half the bytes).
// With may_alloc = false a workspace too small for the batch is E_STATE
// instead of being replaced.
dagbound_status model_workspace(dagbound_model* m, const dagbound_batch* b, SurArgs* s, bool train,
                                bool may_alloc = true) {
  const int64_t R = b->tn, D = b->D;
  const int64_t nchunk = train ? (R + SUR_CHUNK - 1) / SUR_CHUNK : 0;
  const size_t node = train ? sur_node_bytes() : sur_node_bytes() - sur_node_grad_bytes();
  const size_t need = 32 * 256 + (size_t)R * node + (size_t)(R + D) * 4 + (size_t)b->te * 4 +
                      (size_t)nchunk * (256 * 128 + 128) * 4 + (size_t)D * 4;
  if (m->ws_size < need && !may_alloc)
    return fail(DAGBOUND_E_STATE,
                "the model's workspace (%zu bytes) is too small for this batch (%zu bytes); a call that may "
                "allocate (dagbound_best_allocation, dagbound_model_select or dagbound_model_forward) sizes it",
                m->ws_size, need);
  if (m->ws_size < need) {
    dev_release(m->ws, m->ws_size, m->device);
    m->ws = nullptr;
    m->ws_size = need;
    hipError_t e = dev_alloc(&m->ws, &m->ws_size, m->device);
    if (e != hipSuccess) {
      m->ws = nullptr;
      m->ws_size = 0;
      return hip_fail(e, "allocating surrogate activations");
    }
  }
  Carve c(m->ws);
  *s = SurArgs{};
  s->t = b->t;
  s->D = b->D;
  s->M = b->M;
  s->max_n = b->max_n;
  s->rows = R;
  s->p = m->p;
  s->g = m->g;
  s->m1 = m->m1;
  s->m2 = m->m2;
  s->wfwd = m->wfwd;
  s->wbwd = m->wbwd;
  s->X = c.take<float>((size_t)R * SUR_FIN);
  s->A = c.take<float>((size_t)R * SUR_OUT);
  for (int l = 0; l <= SUR_LAYERS; l++) s->H[l] = c.take<__bf16>((size_t)R * SUR_HID);
  s->G[0] = c.take<__bf16>((size_t)R * SUR_HID);
  s->dag_of = c.take<int32_t>((size_t)R);
  s->nboff = c.take<uint32_t>((size_t)(R + D));
  s->nb = c.take<uint16_t>((size_t)b->te * 2);
  s->loss_part = c.take<float>((size_t)D);
  if (train) {
    for (int l = 1; l < SUR_LAYERS; l++) s->G[l] = c.take<__bf16>((size_t)R * SUR_HID);
    s->dA = c.take<float>((size_t)R * SUR_OUT);
    s->dZ[0] = c.take<__bf16>((size_t)R * SUR_HID);
    s->dZ[1] = c.take<__bf16>((size_t)R * SUR_HID);
    s->DT = c.take<float>((size_t)R * 256);
    s->partial = c.take<float>((size_t)nchunk * 256 * 128);
    s->partial2 = c.take<float>((size_t)nchunk * 128);
  }
  return DAGBOUND_OK;
}

}  // namespace

extern "C" {

dagbound_status dagbound_model_create(uint64_t seed, dagbound_model** out) {
  g_err.clear();
  if (!out) return fail(DAGBOUND_E_ARG, "out is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(DAGBOUND_E_DEVICE, "no HIP device");
  }
  dagbound_model* m = new dagbound_model();
  (void)hipGetDevice(&m->device);
  m->block_size = 8 * 256 + (size_t)SUR_PARAMS * 4 * 4 + (size_t)SUR_LAYERS * 256 * 128 * 2 * 2;
  hipError_t e = dev_alloc(&m->block, &m->block_size, m->device);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "allocating the model");
  }
  Carve c(m->block);
  m->p = c.take<float>(SUR_PARAMS);
  m->g = c.take<float>(SUR_PARAMS);
  m->m1 = c.take<float>(SUR_PARAMS);
  m->m2 = c.take<float>(SUR_PARAMS);
  m->wfwd = c.take<__bf16>((size_t)SUR_LAYERS * 256 * 128);
  m->wbwd = c.take<__bf16>((size_t)SUR_LAYERS * 256 * 128);
  std::vector<float> h;
  model_init_params(seed, h);
  e = hipMemcpy(m->p, h.data(), h.size() * 4, hipMemcpyHostToDevice);
  // gradient and both Adam moments start at zero (three separate 256-byte
  // aligned arrays, so one memset over the first would miss the gaps' tail)
  for (float* z : {m->g, m->m1, m->m2})
    if (e == hipSuccess) e = hipMemset(z, 0, (size_t)SUR_PARAMS * 4);
  SurArgs s{};
  s.p = m->p;
  s.wfwd = m->wfwd;
  s.wbwd = m->wbwd;
  if (e == hipSuccess) e = sur_refresh_weights(s, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    dev_release(m->block, m->block_size, m->device);
    delete m;
    return hip_fail(e, "initialising the model");
  }
  *out = m;
  return DAGBOUND_OK;
}

void dagbound_model_destroy(dagbound_model* m) {
  if (!m) return;
  {
    DeviceGuard g(m->device);
    (void)hipDeviceSynchronize();
  }
  dev_release(m->block, m->block_size, m->device);
  dev_release(m->ws, m->ws_size, m->device);
  delete m;
}

dagbound_status dagbound_model_params(dagbound_model* m, float* get, const float* set, float* grad,
                                      int64_t* step) {
  g_err.clear();
  if (!m) return fail(DAGBOUND_E_ARG, "model is NULL");
  DeviceGuard g(m->device);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && get) e = hipMemcpy(get, m->p, (size_t)SUR_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && grad) e = hipMemcpy(grad, m->g, (size_t)SUR_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && set) {
    e = hipMemcpy(m->p, set, (size_t)SUR_PARAMS * 4, hipMemcpyHostToDevice);
    SurArgs s{};
    s.p = m->p;
    s.wfwd = m->wfwd;
    s.wbwd = m->wbwd;
    if (e == hipSuccess) e = sur_refresh_weights(s, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) return hip_fail(e, "model parameters");
  if (step) *step = m->step;
  return DAGBOUND_OK;
}

}  // extern "C"

namespace {

// Checkpoint file: a fixed header, then the FP32 parameters and both Adam
// moments (DAGBOUND_MODEL_PARAMS floats each, little-endian as in memory).
// The checksum is FNV-1a (64-bit) over the three arrays.
constexpr char MODEL_MAGIC[8] = {'D', 'A', 'G', 'B', 'M', 'D', 'L', '\0'};
constexpr uint32_t MODEL_FILE_VERSION = 1;
struct ModelFileHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  int64_t params;
  int64_t step;
  int32_t fin, hid, layers, out;
  uint64_t checksum;
};
static_assert(sizeof(ModelFileHeader) == 56, "checkpoint header layout");

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; i++) {
    h ^= c[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

}  // namespace

extern "C" {

dagbound_status dagbound_model_save(const dagbound_model* m, const char* path) {
  g_err.clear();
  if (!m || !path) return fail(DAGBOUND_E_ARG, "model or path is NULL");
  DeviceGuard g(m->device);
  std::vector<float> buf((size_t)SUR_PARAMS * 3);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(buf.data(), m->p, (size_t)SUR_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + SUR_PARAMS, m->m1, (size_t)SUR_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * SUR_PARAMS, m->m2, (size_t)SUR_PARAMS * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "reading the model");
  ModelFileHeader h{};
  memcpy(h.magic, MODEL_MAGIC, 8);
  h.version = MODEL_FILE_VERSION;
  h.header_bytes = (uint32_t)sizeof h;
  h.params = SUR_PARAMS;
  h.step = m->step;
  h.fin = SUR_FIN;
  h.hid = SUR_HID;
  h.layers = SUR_LAYERS;
  h.out = SUR_OUT;
  h.checksum = fnv1a(buf.data(), buf.size() * 4, 0xCBF29CE484222325ull);
  // written under a temporary name and renamed, so a failed save leaves any
  // earlier file at `path` intact
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return fail(DAGBOUND_E_IO, "cannot open %s for writing", tmp.c_str());
  bool ok = fwrite(&h, sizeof h, 1, f) == 1 && fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    (void)remove(tmp.c_str());
    return fail(DAGBOUND_E_IO, "writing %s failed", path);
  }
  return DAGBOUND_OK;
}

dagbound_status dagbound_model_load(dagbound_model* m, const char* path) {
  g_err.clear();
  if (!m || !path) return fail(DAGBOUND_E_ARG, "model or path is NULL");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(DAGBOUND_E_IO, "cannot open %s", path);
  ModelFileHeader h{};
  std::vector<float> buf((size_t)SUR_PARAMS * 3);
  const bool head = fread(&h, sizeof h, 1, f) == 1;
  bool body = false;
  if (head && !memcmp(h.magic, MODEL_MAGIC, 8) && h.version == MODEL_FILE_VERSION &&
      h.header_bytes == sizeof h && h.params == SUR_PARAMS && h.fin == SUR_FIN && h.hid == SUR_HID &&
      h.layers == SUR_LAYERS && h.out == SUR_OUT && h.step >= 0) {
    body = fread(buf.data(), 4, buf.size(), f) == buf.size();
    char extra;
    body = body && fread(&extra, 1, 1, f) == 0;  // nothing after the moments
  }
  fclose(f);
  if (!head) return fail(DAGBOUND_E_IO, "%s: short header", path);
  if (memcmp(h.magic, MODEL_MAGIC, 8)) return fail(DAGBOUND_E_IO, "%s is not a libdagbound model file", path);
  if (h.version != MODEL_FILE_VERSION)
    return fail(DAGBOUND_E_IO, "%s: file version %u, this library reads version %u", path, h.version, MODEL_FILE_VERSION);
  if (!body) return fail(DAGBOUND_E_IO, "%s: wrong architecture or size", path);
  if (fnv1a(buf.data(), buf.size() * 4, 0xCBF29CE484222325ull) != h.checksum)
    return fail(DAGBOUND_E_IO, "%s: checksum mismatch", path);
  DeviceGuard g(m->device);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(m->p, buf.data(), (size_t)SUR_PARAMS * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->m1, buf.data() + SUR_PARAMS, (size_t)SUR_PARAMS * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->m2, buf.data() + 2 * SUR_PARAMS, (size_t)SUR_PARAMS * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->g, 0, (size_t)SUR_PARAMS * 4);
  SurArgs s{};
  s.p = m->p;
  s.wfwd = m->wfwd;
  s.wbwd = m->wbwd;
  if (e == hipSuccess) e = sur_refresh_weights(s, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "loading the model");
  m->step = h.step;
  return DAGBOUND_OK;
}

dagbound_status dagbound_model_forward(dagbound_model* m, dagbound_batch* b, float* node_out,
                                       uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  if (!m || !b) return fail(DAGBOUND_E_ARG, "model or batch is NULL");
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (!node_out && b->tn > 0) return fail(DAGBOUND_E_ARG, "node_out is NULL");
  if (m->device != b->device) return fail(DAGBOUND_E_ARG, "model and batch live on different devices");
  DeviceGuard g(m->device);
  hipStream_t st = (hipStream_t)hip_stream;
  SurArgs s;
  dagbound_status rc = model_workspace(m, b, &s, false);
  if (rc != DAGBOUND_OK) return rc;
  hipError_t e = sur_features(s, st);
  if (e == hipSuccess) e = sur_forward(s, st);
  // A rows are in sigma order: the caller gets them in local-id order
  float* dout = node_out;
  void* tmp = nullptr;
  size_t tmp_size = 0;
  if (e == hipSuccess && ptr_kind == DAGBOUND_PTR_HOST && b->tn > 0) {
    tmp_size = (size_t)b->tn * 12;
    e = dev_alloc(&tmp, &tmp_size, m->device);
    dout = (float*)tmp;
  }
  if (e == hipSuccess) e = sur_output_local(s, dout, st);
  if (e == hipSuccess && ptr_kind == DAGBOUND_PTR_HOST && b->tn > 0)
    e = hipMemcpyAsync(node_out, dout, (size_t)b->tn * 12, hipMemcpyDeviceToHost, st);
  const hipError_t es = hipStreamSynchronize(st);  // documented to wait for its work
  if (e == hipSuccess) e = es;
  if (tmp) dev_release(tmp, tmp_size, m->device);
  if (e != hipSuccess) return hip_fail(e, "surrogate forward");
  return DAGBOUND_OK;
}

dagbound_status dagbound_model_train_step(dagbound_model* m, dagbound_batch* b, int32_t K, uint64_t seed,
                                          const int64_t* bounds, float lr, float* loss, uint32_t ptr_kind,
                                          void* hip_stream) {
  g_err.clear();
  if (!m || !b || !bounds) return fail(DAGBOUND_E_ARG, "model, batch or bounds is NULL");
  if (K < 2 || K > 16384) return fail(DAGBOUND_E_ARG, "K = %d outside [2, 16384]", K);
  if (ptr_kind > DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "bad ptr_kind %u", ptr_kind);
  if (m->device != b->device) return fail(DAGBOUND_E_ARG, "model and batch live on different devices");
  DeviceGuard g(m->device);
  hipStream_t st = (hipStream_t)hip_stream;
  SurArgs s;
  dagbound_status rc = model_workspace(m, b, &s, true);
  if (rc != DAGBOUND_OK) return rc;
  const int64_t* dbounds = bounds;
  void* tmp = nullptr;
  size_t tmp_size = 0;
  hipError_t e = hipSuccess;
  if (ptr_kind == DAGBOUND_PTR_HOST) {
    tmp_size = (size_t)b->D * K * 8;
    e = dev_alloc(&tmp, &tmp_size, m->device);
    if (e == hipSuccess) e = hipMemcpy(tmp, bounds, (size_t)b->D * K * 8, hipMemcpyHostToDevice);
    dbounds = (const int64_t*)tmp;
  }
  const float scale = 1.f / (float)((int64_t)b->D * (K - 1));
  if (e == hipSuccess) e = sur_features(s, st);
  if (e == hipSuccess) e = sur_forward(s, st);
  if (e == hipSuccess) e = sur_head_train(s, K, seed, dbounds, scale, st);
  if (e == hipSuccess) e = sur_backward(s, st);
  if (e == hipSuccess && lr > 0.f) {
    m->step++;
    e = sur_adam(s, lr, m->step, st);
    if (e == hipSuccess) e = sur_refresh_weights(s, st);
  }
  std::vector<float> lp((size_t)b->D);
  if (e == hipSuccess && b->D > 0) e = hipMemcpyAsync(lp.data(), s.loss_part, lp.size() * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dev_release(tmp, tmp_size, m->device);
  if (e != hipSuccess) return hip_fail(e, "surrogate training step");
  double sum = 0;
  for (float x : lp) sum += x;
  if (loss) *loss = (float)sum;
  return DAGBOUND_OK;
}

dagbound_status dagbound_model_select(dagbound_model* m, dagbound_batch* b, int32_t K, uint64_t seed,
                                      int32_t top_k, int32_t nodes, int32_t* cand, float* scores,
                                      uint32_t ptr_kind, void* hip_stream) {
  g_err.clear();
  if (!m || !b || !cand) return fail(DAGBOUND_E_ARG, "model, batch or cand is NULL");
  if (K < 1 || K > 16384) return fail(DAGBOUND_E_ARG, "K = %d outside [1, 16384]", K);
  if (top_k < 0 || top_k > 255 || top_k >= K) return fail(DAGBOUND_E_ARG, "top_k = %d outside [0, min(255, K-1)]", top_k);
  if (nodes < 1 || nodes > 64) return fail(DAGBOUND_E_ARG, "nodes = %d outside [1, 64]", nodes);
  if (ptr_kind != DAGBOUND_PTR_DEVICE) return fail(DAGBOUND_E_ARG, "model_select takes device pointers");
  if (m->device != b->device) return fail(DAGBOUND_E_ARG, "model and batch live on different devices");
  DeviceGuard g(m->device);
  hipStream_t st = (hipStream_t)hip_stream;
  SurArgs s;
  dagbound_status rc = model_workspace(m, b, &s, false);
  if (rc != DAGBOUND_OK) return rc;
  hipError_t e = sur_features(s, st);
  if (e == hipSuccess) e = sur_forward(s, st);
  if (e == hipSuccess) e = sur_select(s, K, seed, nodes, top_k, scores, cand, st);
  if (e == hipSuccess && !st) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "surrogate selection");
  return DAGBOUND_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free surrogate search (dagbound_best_allocation_static).  The
// candidate lists live in one file-scope device array; every device the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: its device address is taken once per device with
// hipGetSymbolAddress (that device current) and kept in g_scratch_dev.
namespace {

static __device__ __align__(256) int32_t scratch[DAGBOUND_STATIC_LIST_ENTRIES];

std::mutex g_scratch_mu;
std::vector<int32_t*> g_scratch_dev;  // per device, nullptr until looked up

// Device address of `scratch` on `device` (which must be current).
hipError_t scratch_on(int device, int32_t** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize((size_t)device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = (int32_t*)p;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

}  // namespace

extern "C" dagbound_status dagbound_best_allocation_static(dagbound_batch* b, const dagbound_model* model,
                                                           int32_t top_k, int32_t* best_idx, int64_t* best_bound,
                                                           void* hip_stream) {
  g_err.clear();
  if (!b || !model) return fail(DAGBOUND_E_ARG, "batch or model is NULL");
  dagbound_model* m = const_cast<dagbound_model*>(model);
  if (!b->has_alloc) return fail(DAGBOUND_E_STATE, "set_allocations has not been called");
  if (b->mode != DAGBOUND_ALLOC_SEEDED) return fail(DAGBOUND_E_ARG, "surrogate search needs seeded candidates");
  if (top_k < 1 || top_k > 255 || top_k >= b->K)
    return fail(DAGBOUND_E_ARG, "top_k = %d outside [1, min(255, K-1)]", top_k);
  if (m->device != b->device) return fail(DAGBOUND_E_ARG, "model and batch live on different devices");
  const int32_t kk = top_k + 1;
  const size_t entries = (size_t)b->D * (size_t)kk;
  if (entries > (size_t)DAGBOUND_STATIC_LIST_ENTRIES)
    return fail(DAGBOUND_E_ARG, "D x (top_k + 1) = %zu list entries exceed the static scratch (%d entries)", entries,
                DAGBOUND_STATIC_LIST_ENTRIES);
  if (b->D == 0) return DAGBOUND_OK;
  if (!best_idx || !best_bound) return fail(DAGBOUND_E_ARG, "best_idx/best_bound is NULL");
  if (b->autotune_pending)
    return fail(DAGBOUND_E_STATE, "an autotune is pending; it runs in a call that may allocate");
  DeviceGuard g(b->device);
  hipStream_t st = (hipStream_t)hip_stream;
  SurArgs s;
  dagbound_status rc = model_workspace(m, b, &s, false, false);
  if (rc != DAGBOUND_OK) return rc;
  int32_t* cand = nullptr;
  hipError_t e = scratch_on(b->device, &cand);
  if (e != hipSuccess) return hip_fail(e, "device address of the static scratch");
  e = sur_features(s, st);
  if (e == hipSuccess) e = sur_forward(s, st);
  if (e == hipSuccess) e = sur_select(s, b->K, b->seed, SUR_HEAD_NODES, top_k, nullptr, cand, st);
  if (e == hipSuccess) {
    SweepArgs a = sweep_args(b);
    a.K = kk;
    a.cand_list = cand;
    a.best = b->best;
    // the size classes one after another on the caller's stream (no side
    // streams or events to create)
    e = ensure_adj(b, st);
    if (e == hipSuccess) e = launch_sweep(a, st, nullptr);
    b->best_gen = ~0ull;  // the per-DAG minimum now holds list positions
  }
  if (e == hipSuccess) e = launch_best_final(b->best, b->D, best_idx, best_bound, cand, kk, st);
  if (e == hipSuccess && !st) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "allocation-free surrogate search");
  return DAGBOUND_OK;
}

// Surrogate-guided search: score every seeded candidate from the encoder's
// per-node coefficients over a bounded node set, evaluate the paper's rule
// and the top_k best-scored candidates exactly, keep the least bound.
dagbound_status surrogate_best(dagbound_batch* b, dagbound_model* m, int32_t top_k, int32_t* best_idx,
                               int64_t* best_bound, uint32_t ptr_kind, hipStream_t st) {
  if (m->device != b->device) return fail(DAGBOUND_E_ARG, "model and batch live on different devices");
  DeviceGuard g(b->device);
  SurArgs s;
  dagbound_status rc = model_workspace(m, b, &s, false);
  if (rc != DAGBOUND_OK) return rc;
  const int32_t kk = top_k + 1;
  void* tmp = nullptr;
  size_t tmp_size = 512 * 3 + (size_t)b->D * (kk * 4 + 12);
  hipError_t e = dev_alloc(&tmp, &tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "allocating surrogate scratch");
  Carve c(tmp);
  int32_t* cand = c.take<int32_t>((size_t)b->D * kk);
  int64_t* ob = c.take<int64_t>((size_t)b->D);
  int32_t* oi = c.take<int32_t>((size_t)b->D);
  e = sur_features(s, st);
  if (e == hipSuccess) e = sur_forward(s, st);
  if (e == hipSuccess) e = sur_select(s, b->K, b->seed, SUR_HEAD_NODES, top_k, nullptr, cand, st);
  if (e == hipSuccess) {
    SweepArgs a = sweep_args(b);
    a.K = kk;
    a.cand_list = cand;
    a.best = b->best;
    e = run_sweep(b, a, st);
    b->best_gen = ~0ull;  // the per-DAG minimum now holds list positions
  }
  if (e == hipSuccess) {
    const bool host = ptr_kind == DAGBOUND_PTR_HOST;
    e = launch_best_final(b->best, b->D, host ? oi : best_idx, host ? ob : best_bound, cand, kk, st);
    if (e == hipSuccess && host && b->D > 0) {
      e = hipMemcpyAsync(best_idx, oi, (size_t)b->D * 4, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(best_bound, ob, (size_t)b->D * 8, hipMemcpyDeviceToHost, st);
    }
  }
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  dev_release(tmp, tmp_size, b->device);
  if (e != hipSuccess) return hip_fail(e, "surrogate search");
  return DAGBOUND_OK;
}
