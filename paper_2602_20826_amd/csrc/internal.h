// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dagbound {

// Allocation-independent per-DAG tables written by the preprocessing kernel.
// Node-indexed arrays use the batch's global node offsets (node_off[d] + i);
// "sigma order" is the order of descending W^anc, ties by smaller local id,
// which is both the Top_M order of Algorithm 1 and the launch order of
// parallel nodes in Section 4.1.
struct Tables {
  const int64_t* node_off;  // [D+1]
  const int64_t* edge_off;  // [D+1]
  uint16_t* gl;             // [T_N] sigma ranks in group order; bit 15 marks a group's last member
  uint32_t* wc;             // [T_N] load C_hat by sigma rank
  uint16_t* pp;             // [T_N] min(p, M) by sigma rank
  uint32_t* mx;             // [T_N] m^max = min(p, C_hat) by sigma rank (t_min = 1)
  uint16_t* indeg;          // [T_N] predecessor count by sigma rank
  uint16_t* inv;            // [T_N] sigma rank of each local node id
  uint32_t* soff;           // [T_N + D] successor offsets by sigma rank, N_d + 1 per DAG at node_off[d] + d
  uint16_t* succ;           // [T_E] successor sigma ranks, DAG d at edge_off[d]
  int64_t* wanc;            // [T_N] W^anc by local node id (inspection)
  int32_t* ngroups;         // [D] |Pi|
  // Node records for the lane-per-node evaluation, written only when the
  // batch holds a DAG above 256 nodes: {C_hat, min(p, M) | sigma << 16 | last << 31,
  // first successor (offset in the DAG's succ), local id | out-degree << 16}.
  uint4* nrec;              // [T_N] by sigma rank (last = 0)
  uint4* mrec;              // [T_N] in group order (last marks a group's last member)
  // Adjacency rows of the DAGs of up to 512 nodes: N_d predecessor bitsets,
  // then N_d successor bitsets, by sigma rank, nw 64-bit words each (nw of
  // the DAG's size class, or of the batch's largest DAG while the batch runs
  // as one launch), DAG d's from adj + adj_node * node_off[d].
  uint64_t* adj;            // [adj_node * T_N]
  int32_t adj_node;         // words per node: 2 * nw of the largest DAG up to 512 nodes
};

struct PrepInputs {
  const int32_t* src;
  const int32_t* dst;
  const int64_t* wcet;
  const int32_t* par;
};

// Error word of the preprocessing kernel: atomicMin of (d << 8 | code), so
// the smallest failing DAG is reported.  Codes are the negated status values.
enum : uint32_t { PREP_E_CYCLE = 2, PREP_E_RANGE = 3, PREP_E_DUP = 4, PREP_E_OVERFLOW = 8,
                  PREP_E_INTERNAL = 9 };

// err[0]: first failing DAG and code; err[1]: bit 0 if some load is 2^20 or
// more, bit 1 if some in-degree is 256 or more; err[2]: work counter of the
// large-DAG preprocessing (zeroed).
// With `order` (DAG ids grouped by size class, class c at class_off[c]),
// one launch per class; without, one launch sized for max_n.  DAGs above
// 512 nodes use `lscratch` (prep_large_scratch_bytes of their largest size).
// DAGs above 256 nodes (classes 3 and 4, one launch each) use `lscratch`,
// which holds the larger of the two classes' prep_large_scratch_bytes.
// With `side` (NUM_CLASSES streams, a fork event and one join event per
// class), the launches of DAGs up to 256 nodes run on their own streams,
// forked from and joined back to `stream`.
hipError_t launch_prep(const Tables& t, const PrepInputs& in, int32_t D, int32_t M, int32_t max_n,
                       const int32_t* order, const int32_t* class_off, unsigned long long* err,
                       void* lscratch, const int32_t* class_max_n, const int32_t* class_max_e,
                       const hipStream_t* side, hipEvent_t fork, const hipEvent_t* join, hipStream_t stream);

// Largest DAG the large-DAG kernels take, and the most workgroups of a
// workgroup-per-DAG preprocessing launch (each with its own scratch region):
// DAGs of 257-512 nodes take workgroups of four wavefronts, six per compute
// unit (six wavefronts per SIMD); larger DAGs take sixteen wavefronts, one
// per compute unit.
constexpr int LARGE_MAX_N = 8000;
constexpr int PREP_LARGE_GRID = 1536;
constexpr int PREP_LARGE_GRID_BIG = 256;
// Global scratch of a workgroup-per-DAG preprocessing launch over `count`
// DAGs of up to max_n nodes and max_e edges.
size_t prep_large_scratch_bytes(int32_t count, int32_t max_n, int32_t max_e);
// Workgroup-per-DAG preprocessing of `count` DAGs (ids from `list`, or
// 0..count-1); resets the work counter err[2] on the stream first.
hipError_t launch_prep_large(const Tables& t, const PrepInputs& in, int32_t count, int32_t M, const int32_t* list,
                             unsigned long long* err, void* scratch, int32_t max_n, int32_t max_e,
                             hipStream_t stream);

// Comparison bounds of Section 5.2 (Greedy, Greedy+unaware, Graham_para)
// per DAG into the non-null outputs ([D] each); the largest DAG's nodes and
// edges size the LDS.
hipError_t launch_baselines(const Tables& t, int32_t D, int32_t M, int32_t max_n, int32_t max_e, int64_t* greedy,
                            int64_t* unaware, int64_t* graham, hipStream_t stream);

// Runs the part graph of one schedule (records of the schedule dump; edges
// esrc -> edst of the DAG, local ids, used without barriers) `reps` times
// after one warm-up, with parts of C ticks of tick_ns nanoseconds; writes
// each run's makespan.  Blocks until done.
hipError_t realize_schedule(const int64_t* rec, int64_t nrec, int32_t n, const int32_t* esrc,
                            const int32_t* edst, int32_t ne, int64_t tick_ns, bool barriers, int32_t reps,
                            int64_t* makespan_ns, int32_t* nparts_out);

// Slots of the per-lane table of segmented residuals in the first
// evaluation pass; a tile that needs more goes to the global-memory pass.
// DAGs of up to 128 nodes keep RES_SLOTS_SMALL of them, which leaves their
// wavefronts' LDS small enough for one more wavefront per compute unit.
constexpr int RES_SLOTS = 12;
constexpr int RES_SLOTS_SMALL = 10;
__host__ __device__ constexpr int res_slots_of(int nw) { return nw <= 2 ? RES_SLOTS_SMALL : RES_SLOTS; }
// Global-memory residual tables (max_n * 64 words each): a first-pass tile
// that overflows its LDS table takes one and finishes at once; the second
// pass (one workgroup per table) takes the tiles left when all are taken.
constexpr int GLOBAL_PASS_GRID = 256;
// Global-memory regions for the residual-slot maps of DAGs of 129-512 nodes:
// one per workgroup of the persistent first pass (at most this many) and of
// the second pass; enough that the persistent grid reaches the occupancy
// limit.
constexpr int ROW_REGIONS = 4096;
enum : int32_t { EVAL_PATH_AUTO = 0, EVAL_PATH_GLOBAL = 1 };

// DAGs are evaluated in size classes (up to 64, 128, 256, 512 nodes, and
// larger), one launch per class, so that a small DAG never pays for a large
// one's bitsets and LDS.  The last class runs one wavefront per (DAG,
// candidate) with its lanes over nodes.
constexpr int NUM_CLASSES = 5;
constexpr int LARGE_CLASS = 4;
constexpr int COUNTERS_PER_CLASS = 4;  // 16 bytes per class, so the lane-per-node kernel's 64-bit counter is aligned
__host__ __device__ constexpr int class_of(int n) {
  return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 3 : LARGE_CLASS;
}
// Residual-load regions of the large-DAG evaluation (one per running
// wavefront, class_max_n words each); the persistent grid is the smaller of
// this and what the occupancy allows (about 19 wavefronts per compute unit).
constexpr int LARGE_SLOTS = 8192;

struct SweepArgs {
  Tables t;
  int32_t D, M, K;              // K: evaluations per DAG (candidates, or list entries with cand_list)
  int32_t kalloc;               // candidate rows per DAG in the explicit bytes (the allocation set's K)
  const int32_t* order;         // [D] DAG ids grouped by size class, or nullptr (one class: all DAGs)
  int32_t class_off[NUM_CLASSES + 1];  // host: class c holds order[class_off[c] .. class_off[c + 1])
  int32_t class_max_n[NUM_CLASSES];    // host: largest DAG of each class
  const int32_t* dag_list;      // device: the DAGs of the launch (set per class), or nullptr
  int32_t list_len;             // DAGs in the launch
  const uint8_t* alloc;         // explicit bytes, or nullptr when seeded
  uint64_t seed;
  int32_t temporal;             // launching loop (Eqs. 6-7): 0 spatial, 1 temporal (chained) reading
  int64_t* bounds;              // [D*K] or nullptr
  int64_t* cp;                  // [D*K] or nullptr
  int64_t* intf;                // [D*K] or nullptr
  unsigned long long* best;     // [D] packed (bound << 22 | c), atomicMin
  uint32_t* ovf_list;           // [D * ceil(K/64)] tiles handed to the global pass
  uint32_t* ovf_count;          // [COUNTERS_PER_CLASS * NUM_CLASSES]: per class, tiles listed,
                                // global tables taken, tiles taken by the persistent pass
  uint32_t* gres;               // residual tables: class c < LARGE_CLASS owns GLOBAL_PASS_GRID
                                // tables of class_max_n[c] * 64 words from gres + gres_off[c];
                                // the large class owns LARGE_SLOTS regions of class_max_n words
  size_t gres_off[NUM_CLASSES]; // host: word offset of each class's tables
  uint64_t* grows;              // map regions (residual-slot maps kept in global memory): class c
                                // owns ROW_REGIONS regions of 4 * (class_max_n[c] + 7) words from
                                // grows + rows_off[c]; rows_off[NUM_CLASSES] is the one-launch pool
  size_t rows_off[NUM_CLASSES + 1];
  int32_t max_n, max_e;
  const int32_t* cand_list;     // [D][K] candidate ids to evaluate, or nullptr (ids 0..K-1)
  int32_t res_slots;            // <= RES_SLOTS
  int32_t path;                 // EVAL_PATH_*
  int32_t small_loads;          // every C_hat < 2^20
  int32_t small_indeg;          // every in-degree < 256
  int32_t persistent;           // first pass as a persistent kernel over a work counter
  int32_t node_lanes_class;     // classes from this one on run the lane-per-node kernel (3 or 4)
  // Conditional DAGs (spatial reading, DAGs up to 512 nodes): per node by
  // sigma rank, pre | nb << 13 | branch << 21 (nb = 0: always executes;
  // else the node runs in realization rho iff (rho / pre) mod nb == branch),
  // or nullptr.  List position p evaluates realization p mod cond_R.
  const uint32_t* cond_tab;
  int32_t cond_R;
};
// Writes the adjacency rows (Tables::adj) of the DAGs of classes 0-3, each
// class's DAGs with rows of the class's words, or with `uniform_nw` words
// when it is nonzero (the one-launch mode).  Reads only soff/succ, clamped
// to each DAG's own ranges, so a batch that failed validation cannot make
// it read out of bounds.
hipError_t launch_adj(const Tables& t, const int32_t* order, const int32_t class_off[NUM_CLASSES + 1],
                      const int32_t class_max_n[NUM_CLASSES], int uniform_nw, hipStream_t stream);

// Largest number of realizations of one conditional DAG.
constexpr int COND_MAX_REALIZATIONS = 4096;
// bounds[d * K + c] = max over rho < R[d] of rb[(d * K + c) * Rmax + rho];
// worst (nullable) the first rho reaching it.
// list[i] = (i mod L) / Rmax for i < n: each candidate's realizations in turn.
hipError_t launch_cond_list(int32_t* list, int64_t n, int64_t L, int32_t Rmax, hipStream_t stream);
hipError_t launch_cond_reduce(const int64_t* rb, const int32_t* R, int32_t D, int32_t K, int32_t Rmax,
                              int64_t* bounds, int32_t* worst, hipStream_t stream);

// Packing of the per-DAG minimum: bound < 2^42 (the summed load is < 2^40)
// and candidate < 2^22.
constexpr int BEST_SHIFT = 22;

// Dynamic LDS bytes one evaluation workgroup needs for the batch's largest DAG.
size_t sweep_lds_need(int max_n, int max_e);
constexpr size_t LDS_LIMIT = 160 * 1024;

// The large-DAG evaluation of one launch (DAGs a.dag_list, or all), on the
// work counter `counter` (zeroed by k_eval_init).
hipError_t launch_eval_large(const SweepArgs& a, uint32_t* counter, hipStream_t stream);
size_t eval_large_lds_bytes(int max_n);

// Side streams for the size classes: each class launch runs on its own
// stream, forked from and joined back to the caller's stream by events, so
// that one class's tail overlaps the others' work.
struct SweepStreams {
  hipStream_t side[NUM_CLASSES];
  hipEvent_t fork;
  hipEvent_t join[NUM_CLASSES];
};

// Words of map regions a batch needs, and each pool's offset.
size_t sweep_rows_words(const int32_t class_max_n[NUM_CLASSES], const int32_t class_off[NUM_CLASSES + 1],
                        int32_t max_n, size_t rows_off[NUM_CLASSES + 1]);

// Words of residual tables a batch needs (the one-launch pool first, then
// every class with DAGs), and each class's offset.
size_t sweep_gres_words(const int32_t class_max_n[NUM_CLASSES], const int32_t class_off[NUM_CLASSES + 1],
                        int32_t max_n, size_t gres_off[NUM_CLASSES]);

// Evaluates every (DAG, candidate) pair; also resets `best` and fills it.
// With `ss`, the class launches run concurrently on its side streams.
hipError_t launch_sweep(const SweepArgs& a, hipStream_t stream, const SweepStreams* ss = nullptr);
// With `list` ([D][K] candidate ids), the packed index is a list position and
// is translated to the candidate id.
hipError_t launch_best_final(const unsigned long long* best, int32_t D, int32_t* idx, int64_t* bound,
                             const int32_t* list, int32_t K, hipStream_t stream);
// Counts the entries of list [n] outside [0, K) into *bad (zeroed first).
hipError_t launch_check_list(const int32_t* list, int64_t n, int32_t K, uint32_t* bad, hipStream_t stream);

// Schedule dump of DAG d under candidate c (schedule.hip): records of 8
// int64 into rec[cap][8]; out = {records the schedule has, bound, critical-
// path term, interference term}.  alloc = explicit bytes (K per DAG) or
// nullptr for the seeded candidates of `seed`; temporal selects the chained
// reading of the launching loop.
hipError_t launch_schedule(const Tables& t, int32_t d, int32_t c, int32_t K, int32_t M, const uint8_t* alloc,
                           uint64_t seed, int32_t max_n, int64_t* rec, int64_t cap, int64_t* out, int32_t temporal,
                           hipStream_t stream);

// ---------------------------------------------------------------------------
// Learned candidate proposal (surrogate.hip).
constexpr int SUR_FIN = 8, SUR_HID = 128, SUR_LAYERS = 3, SUR_OUT = 4;
constexpr int64_t SUR_OFF_W0 = 0;
constexpr int64_t SUR_OFF_B0 = SUR_OFF_W0 + SUR_FIN * SUR_HID;
constexpr int64_t SUR_OFF_L1 = SUR_OFF_B0 + SUR_HID;
constexpr int64_t SUR_LAYER_STRIDE = 2 * SUR_HID * SUR_HID + SUR_HID;  // Ws, Wm, b
constexpr int64_t SUR_OFF_WA = SUR_OFF_L1 + SUR_LAYERS * SUR_LAYER_STRIDE;
constexpr int64_t SUR_OFF_BA = SUR_OFF_WA + SUR_HID * SUR_OUT;
constexpr int64_t SUR_PARAMS = SUR_OFF_BA + SUR_OUT;
constexpr int64_t SUR_CHUNK = 8192;  // node rows per partial weight-gradient sum
constexpr int32_t SUR_HEAD_NODES = 32;  // nodes the search head reads per candidate

struct SurArgs {
  Tables t;
  int32_t D, M, max_n;
  int64_t rows;            // T_N
  float* p;                // master parameters
  float* g;                // gradient
  float *m1, *m2;          // Adam moments
  __bf16 *wfwd, *wbwd;     // BF16 layer weights (see k_weights_bf16)
  float* X;                // [rows][8]
  float *A, *dA;           // [rows][4]
  __bf16* H[SUR_LAYERS + 1];
  __bf16* G[SUR_LAYERS];
  __bf16* dZ[2];
  float* DT;               // [rows][256]
  int32_t* dag_of;         // [rows]
  uint32_t* nboff;         // [rows + D]
  uint16_t* nb;            // [2 * T_E]
  float *partial, *partial2;
  float* loss_part;        // [D]
};

size_t sur_node_bytes();
size_t sur_node_grad_bytes();  // the part only training uses
hipError_t sur_features(const SurArgs& s, hipStream_t st);
hipError_t sur_forward(const SurArgs& s, hipStream_t st);
hipError_t sur_head_train(const SurArgs& s, int32_t K, uint64_t seed, const int64_t* bounds, float scale,
                          hipStream_t st);
hipError_t sur_backward(const SurArgs& s, hipStream_t st);
hipError_t sur_adam(const SurArgs& s, float lr, int64_t step, hipStream_t st);
hipError_t sur_refresh_weights(const SurArgs& s, hipStream_t st);
// Head coefficients [T_N][3] in local-id order (device pointer).
hipError_t sur_output_local(const SurArgs& s, float* out, hipStream_t st);
hipError_t sur_select(const SurArgs& s, int32_t K, uint64_t seed, int32_t T, int32_t top_k, float* scores,
                      int32_t* cand, hipStream_t st);

}  // namespace dagbound
