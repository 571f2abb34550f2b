/*
 * libdagbound -- batched exact evaluation of the makespan bound of
 * DAG-structured GPU tasks on AMD Instinct MI355X (gfx950).
 *
 * Method: Zhang et al., "Exploiting Dependency and Parallelism: Real-Time
 * Scheduling and Analysis for GPU Tasks" (DAC 2026).
 *   - Task model (Section 2.1): a DAG G = (V, E); node v is a kernel with
 *     load C_hat_v (its execution time on one compute unit, integer ticks,
 *     t_min = 1) and maximum parallelism p_v; the GPU has M compute units.
 *   - Sub-graph division (Section 3, Eqs. 2-4, Algorithm 1) splits G into an
 *     ordered list of balanced groups.
 *   - Scheduling (Section 4.1, Eqs. 1, 5-7, Algorithm 2) sets each kernel's
 *     parallelism, launches parallel nodes into spare compute units, splits
 *     nodes that do not fit (segmentation) and adds extra dependencies.
 *   - Analysis (Section 4.2, Lemma 1, Theorem 1): the makespan is bounded by
 *     the sum of the groups' responses.
 * A candidate allocation r (one byte per node) replaces the paper's
 * parallelism rule for nodes with r_v > 0: as a group member the node runs
 * with m = min(r_v, p_v, remaining load, M) instead of Eq. 5; as a parallel
 * node its greedy target min(m^max, S) uses r_v instead of m^max.  r_v = 0
 * keeps the paper's rule.  Candidate 0 of every DAG is the paper's own
 * schedule (its bytes are ignored).  The bound of a group whose compute-unit
 * demand exceeds M (Eq. 5 rounding, or explicit r) adds the list-scheduling
 * interference term floor((A - maxC) / M), A = sum of m * C over the group.
 *
 * All results are exact int64, bit-identical to the plain CPU definition.
 *
 * Beyond the bound: the comparison bounds of the evaluation (Section 5.2:
 * Greedy, Greedy + unaware, Graham_para; dagbound_baselines), the other
 * reading of the launching loop (WS_j as an area, launched nodes chained;
 * dagbound_set_para_launch), and a schedule run on this GPU as a HIP graph
 * (the case study of Section 5.3; dagbound_run_schedule).
 *
 * Conventions shared by every call:
 *   - Status: 0 on success, a negative DAGBOUND_E_* code on failure;
 *     dagbound_last_error() then returns a message (per thread).  On failure
 *     outputs are not written and the batch is unchanged.
 *   - ptr_kind: DAGBOUND_PTR_HOST (host memory) or DAGBOUND_PTR_DEVICE
 *     (device memory of the current HIP device, e.g. a torch tensor's
 *     data_ptr()).  It applies to every array argument of the call.
 *   - hip_stream: a hipStream_t, or NULL.  With NULL, and for any call with
 *     host pointers, the call returns after the work is complete.  With a
 *     stream and device pointers the work is ordered on that stream and the
 *     call may return before it completes.  Calls on one batch must be
 *     ordered (one stream, or synchronized by the caller).
 *   - A batch is bound to the HIP device that was current at creation.
 */
#ifndef DAGBOUND_H
#define DAGBOUND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dagbound_batch dagbound_batch; /* opaque; owns its device memory */
typedef struct dagbound_model dagbound_model; /* opaque learned candidate proposal */
typedef int32_t dagbound_status;

enum {
  DAGBOUND_OK = 0,
  DAGBOUND_E_ARG = -1,        /* bad argument (null pointer, negative count, bad enum) */
  DAGBOUND_E_CYCLE = -2,      /* a DAG has a cycle or a self-loop */
  DAGBOUND_E_RANGE = -3,      /* a node id, load or parallelism is out of range */
  DAGBOUND_E_DUP_EDGE = -4,   /* a DAG lists the same edge twice */
  DAGBOUND_E_OOM = -5,        /* device memory exhausted */
  DAGBOUND_E_DEVICE = -6,     /* HIP runtime error, or no usable device */
  DAGBOUND_E_STATE = -7,      /* call out of order (e.g. eval before set_allocations) */
  DAGBOUND_E_OVERFLOW = -8,   /* a DAG's summed load reaches 2^40 */
  DAGBOUND_E_UNSUPPORTED = -9, /* valid input the library does not handle */
  DAGBOUND_E_IO = -10          /* a model file cannot be opened, read or written, or is not a
                                  model file of this version and architecture */
};
enum { DAGBOUND_PTR_HOST = 0, DAGBOUND_PTR_DEVICE = 1 };
enum { DAGBOUND_ALLOC_EXPLICIT = 0, DAGBOUND_ALLOC_SEEDED = 1 };
enum { DAGBOUND_SEARCH_EXHAUSTIVE = 0, DAGBOUND_SEARCH_SURROGATE = 1 };
enum { DAGBOUND_PARA_SPATIAL = 0, DAGBOUND_PARA_TEMPORAL = 1 };

/* Limits of the library. */
#define DAGBOUND_MAX_NODES_PER_DAG 8000  /* N_d, source and sink included */
#define DAGBOUND_MAX_CANDIDATES (1 << 22)

/*
 * dagbound_create_batch -- ingest num_dags DAG tasks and run the
 * allocation-independent part of the method on the GPU: input validation,
 * the ancestor closure and cumulative ancestor workload W^anc (Eq. 2), the
 * join-node list Theta, blocks (Eq. 3), local complete paths (Eq. 4) and the
 * balanced groups of Algorithm 1 (Rules 1-2), for M = num_cus compute units.
 *
 *   num_dags   D >= 0.
 *   node_off   int64 [D+1]: DAG d owns nodes node_off[d] .. node_off[d+1]-1
 *              of wcet/max_par; node_off[0] = 0, nondecreasing.  A DAG may be
 *              empty (bound 0).  N_d <= DAGBOUND_MAX_NODES_PER_DAG.
 *   edge_off   int64 [D+1]: DAG d owns edges edge_off[d] .. edge_off[d+1]-1;
 *              edge_off[0] = 0, nondecreasing.
 *   edge_src, edge_dst  int32 [edge_off[D]]: DAG-local node ids in
 *              [0, N_d); edge (u, v) means v starts after u completes.
 *              Any order; a single source/sink is not required.
 *   wcet       int64 [node_off[D]]: load C_hat_v, 1 <= C_hat_v <= 2^31-1;
 *              per DAG the sum must stay below 2^40.
 *   max_par    int32 [node_off[D]]: p_v >= 1.
 *   num_cus    M, 1 <= M <= 65535.
 *   out        receives the batch handle (untouched on failure).
 * Errors: E_ARG, E_CYCLE (cycle or self-loop), E_RANGE, E_DUP_EDGE,
 * E_OVERFLOW, E_OOM, E_DEVICE, E_UNSUPPORTED (a DAG above the node limit);
 * the message names the first failing DAG.  The batch copies what it needs;
 * the caller may free or reuse the inputs when the call returns.  This call
 * always waits for its GPU work (it must see the validation result).
 */
dagbound_status dagbound_create_batch(int32_t num_dags, const int64_t* node_off,
                                      const int64_t* edge_off, const int32_t* edge_src,
                                      const int32_t* edge_dst, const int64_t* wcet,
                                      const int32_t* max_par, int32_t num_cus, uint32_t ptr_kind,
                                      void* hip_stream, dagbound_batch** out);

/*
 * dagbound_set_allocations -- define K candidate allocations per DAG.
 *
 *   K      1 <= K <= DAGBOUND_MAX_CANDIDATES.
 *   mode   DAGBOUND_ALLOC_EXPLICIT: `alloc` holds K * node_off[D] bytes; the
 *          byte r of (DAG d, candidate c, local node v) sits at
 *          K * node_off[d] + c * N_d + v.  Bytes of candidate 0 are ignored.
 *          With PTR_HOST the bytes are copied into the batch.  With
 *          PTR_DEVICE the batch keeps the pointer and reads the bytes in
 *          place at each later evaluation: the caller keeps that memory
 *          alive and unchanged until the last evaluation that uses it.
 *          DAGBOUND_ALLOC_SEEDED: `alloc` is ignored; for c >= 1 the byte is
 *          drawn on the GPU by the counter-based hash
 *            mix(z): z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
 *                    z *= 0x94D049BB133111EB; z ^= z>>31   (SplitMix64
 *                    finalizer, Steele, Lea and Flood, OOPSLA 2014)
 *            key  = mix(seed ^ mix(d * 0x9E3779B97F4A7C15))
 *            word = mix(key ^ ((c << 32) | (v >> 2)))
 *            h16  = (word >> (16 * (v & 3))) & 0xFFFF
 *            r    = 1 + ((h16 * range) >> 16),  range = min(p_v, M, 255)
 *          (d is the DAG's index in the batch, all arithmetic mod 2^64).
 *   seed   used by SEEDED only.
 * Errors: E_ARG.  Replaces any earlier allocation set.
 */
dagbound_status dagbound_set_allocations(dagbound_batch* batch, int32_t K, uint32_t mode,
                                         const uint8_t* alloc, uint64_t seed, uint32_t ptr_kind);

/*
 * dagbound_eval_bounds -- the bound of every (DAG, candidate) pair: the
 * scheduling of Algorithm 2 (Eqs. 1, 5-7, segmentation, extra dependencies
 * as slot order) and the analysis of Lemma 1 / Theorem 1.
 *
 *   bounds     int64 [D * K]: bounds[d * K + c] = sum over groups of R_j
 *              (may be NULL only when D * K = 0).
 *   cp_term    int64 [D * K] or NULL: sum over groups of max C (the Lemma 1
 *              terms); intf_term int64 [D * K] or NULL: sum of the
 *              interference terms.  bounds = cp_term + intf_term.
 * Errors: E_ARG, E_STATE (no allocations set), E_DEVICE.
 */
dagbound_status dagbound_eval_bounds(dagbound_batch* batch, int64_t* bounds, int64_t* cp_term,
                                     int64_t* intf_term, uint32_t ptr_kind, void* hip_stream);

/*
 * dagbound_best_allocation -- per DAG, the candidate of least bound (ties to
 * the smallest candidate index) and that bound.
 *
 *   search     DAGBOUND_SEARCH_EXHAUSTIVE: every candidate is evaluated
 *              exactly (when dagbound_eval_bounds already ran on the current
 *              allocation set, its per-DAG minimum is reused).
 *              DAGBOUND_SEARCH_SURROGATE: seeded candidates only; `model`
 *              scores every candidate (dagbound_model_select with 32 nodes),
 *              and candidate 0 plus the top_k best-scored ones are evaluated
 *              exactly.  The result is exact for the candidates evaluated;
 *              ties go to the candidate listed first (0, then by score).
 *   top_k      SURROGATE: 1..min(255, K-1); ignored by EXHAUSTIVE.
 *   model      NULL for EXHAUSTIVE.
 *   best_idx   int32 [D]; best_bound int64 [D] (NULL only when D = 0).  An
 *              empty DAG reports candidate 0 with bound 0.
 * Errors: E_ARG, E_STATE, E_DEVICE.
 */
dagbound_status dagbound_best_allocation(dagbound_batch* batch, uint32_t search, int32_t top_k,
                                         const dagbound_model* model, int32_t* best_idx,
                                         int64_t* best_bound, uint32_t ptr_kind, void* hip_stream);

/*
 * dagbound_eval_listed -- the bounds of listed candidates of the current
 * allocation set: for each DAG d, the L candidate ids cand[d * L + i] in
 * [0, K) (repeats allowed), evaluated exactly as dagbound_eval_bounds
 * evaluates them (Algorithm 2, Lemma 1 / Theorem 1).  This is the exact
 * verification step of a proposal that picked a few candidates per DAG.
 *   L          entries per DAG, 1 <= L <= DAGBOUND_MAX_CANDIDATES.
 *   cand       int32 [D * L] candidate ids (same memory kind as the outputs).
 *   bounds     int64 [D * L]: bounds[d * L + i] is the bound of candidate
 *              cand[d * L + i] of DAG d; cp_term / intf_term as for
 *              dagbound_eval_bounds (each may be NULL).
 * An id outside [0, K) is E_ARG (device lists are checked on the device
 * before anything is evaluated).  The call waits for its work.  A later
 * exhaustive best_allocation evaluates the whole set again.
 * Errors: E_ARG, E_STATE (no allocations set), E_OOM, E_DEVICE.
 */
dagbound_status dagbound_eval_listed(dagbound_batch* batch, int32_t L, const int32_t* cand, int64_t* bounds,
                                     int64_t* cp_term, int64_t* intf_term, uint32_t ptr_kind, void* hip_stream);

/*
 * dagbound_eval_conditional -- makespan bounds of conditional DAG tasks (the
 * extension the paper names as future work in Section 6), for every
 * (DAG, candidate) of the current allocation set.  A conditional is a set of
 * alternative branches of which exactly one executes at run time; a
 * realization picks one branch of every conditional of a DAG.  The schedule
 * is the method's schedule of the DAG with every branch present (Algorithms
 * 1 and 2, spatial reading); in a realization the nodes of the branches not
 * taken hold no SM and no time, and each slot's response is Lemma 1 over the
 * slot's executed parts (members, parallel nodes launched whole, parallel
 * segments), 0 for a slot with none.  The result is the largest
 * realization bound.
 *   cond_of    int32 [node_off[D]]: the node's conditional within its DAG
 *              (0, 1, ...), or -1 for a node that always executes.
 *   branch_of  int32 [node_off[D]]: its branch within that conditional,
 *              0..254 (ignored for -1).  A conditional has max branch + 1
 *              branches; conditionals do not nest.
 *   bounds     int64 [D*K]: bounds[d*K + c] the largest realization bound.
 *   worst      int32 [D*K] or NULL: the first realization reaching it, as a
 *              mixed-radix index with conditional 0 the least significant
 *              digit.
 * Same memory kind (ptr_kind) for all four arrays.  With every node at -1
 * the result equals dagbound_eval_bounds.  The call waits for its work.
 * Limits: DAGs of up to 512 nodes, at most 4,096 realizations per DAG, the
 * spatial reading of the launching loop.
 * Errors: E_ARG, E_STATE (no allocations set), E_RANGE (ids outside the
 * ranges above, too many realizations), E_UNSUPPORTED (a DAG above 512
 * nodes, the temporal reading), E_OOM, E_DEVICE.
 */
dagbound_status dagbound_eval_conditional(dagbound_batch* batch, const int32_t* cond_of, const int32_t* branch_of,
                                          int64_t* bounds, int32_t* worst, uint32_t ptr_kind, void* hip_stream);

/*
 * dagbound_set_para_launch -- the reading of the launching loop of
 * Section 4.1 (Eqs. 6-7, Algorithm 2) used by every later evaluation of the
 * batch (eval_bounds, best_allocation, get_schedule, run_schedule).
 *   DAGBOUND_PARA_SPATIAL (default): the spare SMs S shrink by each launched
 *     parallel node's m; a node that does not fit in maxC * m is segmented
 *     there and launching stops.
 *   DAGBOUND_PARA_TEMPORAL: WS_j read as an area of S SMs for the slot's
 *     time maxC; every parallel node takes m = min(its target, S), the
 *     launched nodes run one after another on those SMs (chain edges, in
 *     the schedule dump as EDGE records inside the slot), and the budget is
 *     the time left; a node that does not fit in (time left) * m is
 *     segmented there and launching stops.  Both readings keep every slot
 *     within M SMs, so Lemma 1 holds for either.
 * Errors: E_ARG.
 */
dagbound_status dagbound_set_para_launch(dagbound_batch* batch, uint32_t mode);

/*
 * dagbound_run_schedule -- runs the schedule of DAG d under candidate c on
 * this GPU as a HIP graph, the counterpart of the paper's case study
 * (Sections 5.1 and 5.3: one busy kernel, m_i set through the launch shape, the DAG
 * as a graph) in the execution model of Section 2.2: every launched part
 * (member, parallel node, segment) is m workgroups, each holding one compute
 * unit alone for C ticks of tick_ns nanoseconds on the GPU's constant-rate
 * clock.
 *   barriers     1: a barrier at every slot boundary, the realization the
 *                bound covers: each slot is one launch of the blocks of all
 *                its parts, after the slot before; 0: each part is its own
 *                kernel node, after the DAG's edges (last part before first
 *                part), the chain of a segmented node's parts and the extra
 *                dependencies of Section 4.1 only.
 *   reps         runs timed after one warm-up run (1..100000).
 *   makespan_ns  int64 [reps] host: each run's time from graph launch to
 *                completion (HIP events), launch overhead included.
 *   terms        int64 [4] or NULL: {bound, critical-path term,
 *                interference term, parts}; the bound in ticks.
 * Requires M <= the device's compute units (a device with more can only
 * finish earlier), tick_ns in [1000, 1e7], and bound x tick x (reps + 1)
 * within two minutes.  Blocks until done.  Errors: E_ARG, E_STATE, E_DEVICE.
 */
dagbound_status dagbound_run_schedule(dagbound_batch* batch, int32_t d, int32_t c, int64_t tick_ns,
                                      int32_t barriers, int32_t reps, int64_t* makespan_ns, int64_t* terms);

/*
 * dagbound_baselines -- the comparison bounds of Section 5.2 for every DAG of
 * the batch, independent of any allocation set.  With t_min = 1 a node's
 * most useful parallelism is m^max = min(p_v, C_hat_v) (Section 2.2).
 *   greedy          int64 [D] or NULL: Greedy, nodes run one after another
 *                   at m = min(m^max, M): the sum of their Eq. 1 times.
 *   greedy_unaware  int64 [D] or NULL: Greedy + unaware, the same at
 *                   m = m^max (Eq. 1 with ceil(m/M) waves); the paper's
 *                   normalisation reference.
 *   graham_para     int64 [D] or NULL: Graham_para, each node as m^max
 *                   unit-SM nodes of ceil(C_hat/m^max) ticks and Graham's
 *                   list-scheduling bound on M SMs for that DAG,
 *                   len + floor((vol - len) / M): len the longest path in
 *                   ticks, vol the SM-ticks of all unit nodes.
 * An empty DAG gives 0 for all three; all outputs NULL is a no-op.
 * Errors: E_ARG, E_DEVICE.
 */
dagbound_status dagbound_baselines(dagbound_batch* batch, int64_t* greedy, int64_t* greedy_unaware,
                                  int64_t* graham_para, uint32_t ptr_kind, void* hip_stream);

/*
 * dagbound_get_schedule -- inspection of the schedule of DAG d under
 * candidate c of the current allocation set (Algorithm 2 and Lemma 1 as the
 * evaluation runs them), with the extra dependencies of Section 4.1 that
 * the evaluation keeps implicit in the slot order.  Records of 8 int64,
 * node ids DAG-local, a node's parts numbered from 0 in launch order:
 *   PART {2, slot, node, part, kind (0 member, 1 parallel node launched
 *         whole, 2 parallel segment), m, C, load}
 *   SLOT {1, slot, members, maxC, sum m, A = sum m*C, R_j, v_R} after the
 *         slot's parts (members 0 and v_R = -1 when every member finished
 *         earlier)
 *   EDGE {3, slot, from node, from part, to node, to part, 0, 0} after the
 *         slot record: v_R to each parallel node not launched whole, and each
 *         launched part to v_R's successors.
 *   records  int64 [cap][8] host buffer (may be NULL when cap = 0); the first
 *            min(cap, count) records are written.
 *   count    receives the number of records of the schedule.
 *   terms    int64 [3] or NULL: {bound, critical-path term, interference term}.
 * Waits for the batch's work.  Errors: E_ARG, E_STATE, E_DEVICE.
 */
dagbound_status dagbound_get_schedule(dagbound_batch* batch, int32_t d, int32_t c, int64_t* records, int64_t cap,
                                      int64_t* count, int64_t* terms);

/*
 * dagbound_get_division -- inspection of DAG d's sub-graph division as the
 * GPU computed it (host outputs, each may be NULL).
 *   wanc       int64 [N_d]: W^anc of each local node (Eq. 2).
 *   group_of   int32 [N_d]: index of the balanced group holding each node.
 *   order      int32 [N_d]: the nodes in group order (groups in Pi order,
 *              members of a group by descending W^anc, ties smaller id).
 *   num_groups receives |Pi|.
 * Waits for the batch's work.  Errors: E_ARG, E_DEVICE.
 */
dagbound_status dagbound_get_division(dagbound_batch* batch, int32_t d, int64_t* wanc,
                                      int32_t* group_of, int32_t* order, int32_t* num_groups);

/*
 * dagbound_set_tuning -- launch-plan options of the evaluation kernels; they
 * never change results.
 *   "residual_slots"  1..12 (default 12; DAGs up to 128 nodes use at most
 *                     10): per-candidate LDS table slots for
 *                     the remaining loads of segmented nodes; a 64-candidate
 *                     tile that needs more restarts with a table in global
 *                     memory that holds every node (256 such tables per
 *                     batch; further tiles wait for a second pass).
 *   "eval_path"       0 (default): LDS tables first, as above; 1: global
 *                     tables for every tile.
 *   "size_classes"    1 (default): one launch per DAG size class (up to 64,
 *                     128, 256, 512 nodes, and larger); 0: one launch over
 *                     all DAGs, sized for the largest.  DAGs above 512 nodes
 *                     run one wavefront per (DAG, candidate); "residual_slots",
 *                     "eval_path" and "persistent" do not apply to them.
 *   "class_streams"   1 (default): when the batch holds DAGs above 128 nodes,
 *                     the class launches run concurrently on side streams of
 *                     the device (forked from and joined back to the caller's
 *                     stream with events), else in turn on the caller's
 *                     stream; 0: always in turn on the caller's stream.
 *   "persistent"      0 (default): one workgroup per 64-candidate tile;
 *                     1: as many workgroups as fit on the device, each taking
 *                     tiles from a work counter.
 *   "node_lanes"      512 (default): DAGs above 512 nodes run one wavefront
 *                     per (DAG, candidate) with lanes over nodes; 256: so do
 *                     DAGs of 257-512 nodes (instead of one wavefront per
 *                     (DAG, 64 candidates), lane per candidate).
 *   "autotune"        1: the next evaluation (eval_bounds, or the sweep of an
 *                     exhaustive best_allocation) runs each combination of
 *                     "persistent", "class_streams" and, when the batch holds
 *                     DAGs of 257-512 nodes, "node_lanes" once, timed with
 *                     events on its stream (so that call synchronizes and must
 *                     not be captured in a graph), and keeps the fastest.
 *   "graph"           0 (default); 1: eval_bounds on device pointers and a
 *                     non-null stream records its launches (every class, the
 *                     fork/join events of the side streams, the second pass)
 *                     into a HIP graph on its first call and replays that graph
 *                     while the output pointers, stream, allocation set and
 *                     tuning stay the same (a change records a new one).
 * Errors: E_ARG (unknown key or value).
 */
dagbound_status dagbound_set_tuning(dagbound_batch* batch, const char* key, int64_t value);

/* ------------------------------------------------------------------------
 * Learned candidate proposal.  Not part of the paper: it ranks candidate
 * allocations so that only the best-ranked ones need exact evaluation.
 *
 * Model (per DAG, N(v) = predecessors and successors of v, hidden width 128):
 *   x_v  8 features: log2 C_hat/16, log2 min(p,M)/8, log2 W^anc/24,
 *        log2 |group|/8, group position in [0,1], log2(1+in-degree)/6,
 *        log2(1+out-degree)/6, C_hat / load of the node's group;
 *   H0 = relu(X W0 + b0); G_l = mean over N(v) of H_{l-1} (0 without
 *   neighbours); H_l = relu(H_{l-1} Ws_l + G_l Wm_l + b_l), l = 1..3;
 *   A = H3 Wa + ba, a_v = A[v][0..2].
 *   Score of candidate bytes r (lower = smaller predicted bound):
 *   (1/N) sum_v a_v . (t, t^2, 1/t), t = r_v / min(p_v, M, 255).
 * Layer GEMMs run in BF16 on the matrix cores with FP32 accumulation;
 * parameters are FP32 (Adam).  The flat parameter vector holds W0 [8x128],
 * b0 [128], then per layer Ws [128x128], Wm [128x128], b [128], then
 * Wa [128x4], ba [4]; matrices row-major, input index first.
 * Calls on one model must be ordered; the model keeps activation scratch
 * sized for the last batch it saw.
 */
#define DAGBOUND_MODEL_PARAMS 100356

/* New model on the current device, weights Glorot-uniform from `seed`. */
dagbound_status dagbound_model_create(uint64_t seed, dagbound_model** out);
void dagbound_model_destroy(dagbound_model* model);

/* Host copies of the parameters (get, [DAGBOUND_MODEL_PARAMS]) and of the
 * last gradient (grad); `set` replaces the parameters; step receives the
 * number of optimizer steps taken.  Each pointer may be NULL. */
dagbound_status dagbound_model_params(dagbound_model* model, float* get, const float* set, float* grad,
                                      int64_t* step);

/* Checkpoint of a model: dagbound_model_save writes its FP32 parameters,
 * both Adam moments and its optimizer step count to the file `path`
 * (versioned header with the architecture, FNV-1a checksum; written under
 * `path`.tmp and renamed, so a failed save leaves an earlier file intact);
 * dagbound_model_load replaces a model's parameters, moments and step by a
 * file's (gradient cleared), so training resumes exactly where the saved
 * model stopped.  Both wait for the model's work.
 * Errors: E_ARG (NULL), E_IO (cannot open / read / write; not a model file;
 * other version, architecture or size; checksum mismatch), E_DEVICE. */
dagbound_status dagbound_model_save(const dagbound_model* model, const char* path);
dagbound_status dagbound_model_load(dagbound_model* model, const char* path);

/* Per-node head coefficients a_v (float [node_off[D]][3], the batch's node
 * numbering).  Waits for its work. */
dagbound_status dagbound_model_forward(dagbound_model* model, dagbound_batch* batch, float* node_out,
                                       uint32_t ptr_kind, void* hip_stream);

/* One training step on a batch whose seeded candidates (K per DAG, seed)
 * have exact bounds `bounds` [D*K] (as dagbound_eval_bounds writes them):
 * the loss is the mean over c >= 1 of (score_c - (ln bound_c - ln bound_0))^2;
 * gradient by the hand-written backward pass; Adam (0.9, 0.999, 1e-8) with
 * learning rate lr (lr = 0: gradient only).  loss receives the loss before
 * the update.  Waits for its work. */
dagbound_status dagbound_model_train_step(dagbound_model* model, dagbound_batch* batch, int32_t K,
                                          uint64_t seed, const int64_t* bounds, float lr, float* loss,
                                          uint32_t ptr_kind, void* hip_stream);

/* Candidate selection for a seeded candidate set (K, seed): scores from the
 * `nodes` (1..64) nodes of largest |a0| + |a1| + range*|a2|, then per DAG
 * cand [D][top_k+1] = {0, the top_k smallest-scored candidates >= 1}
 * (ties to the smaller index); scores [D*K] may be NULL.  Device pointers. */
dagbound_status dagbound_model_select(dagbound_model* model, dagbound_batch* batch, int32_t K, uint64_t seed,
                                      int32_t top_k, int32_t nodes, int32_t* cand, float* scores,
                                      uint32_t ptr_kind, void* hip_stream);

/*
 * dagbound_best_allocation_static -- the surrogate search of
 * dagbound_best_allocation (SURROGATE) without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same results as that call.
 *   The candidate lists (D x (top_k + 1) int32 entries) live in a static
 *   device array of DAGBOUND_STATIC_LIST_ENTRIES entries (16 MiB) that each
 *   GPU holds until the process ends; every call on a GPU shares it, so
 *   calls that overlap on one GPU race.  The model's activation workspace
 *   must already be sized for the batch by an earlier allocating call
 *   (dagbound_best_allocation with SURROGATE, dagbound_model_select or
 *   dagbound_model_forward on this batch or a larger one).
 *   best_idx int32 [D], best_bound int64 [D]: device pointers.  The size
 *   classes run one after another on hip_stream (NULL: the call waits).
 * Errors: E_ARG (NULL, top_k outside [1, min(255, K-1)], explicit candidates,
 * D x (top_k + 1) above DAGBOUND_STATIC_LIST_ENTRIES), E_STATE (no
 * allocations set, workspace too small, autotune pending), E_DEVICE.
 */
#define DAGBOUND_STATIC_LIST_ENTRIES (4 << 20)
dagbound_status dagbound_best_allocation_static(dagbound_batch* batch, const dagbound_model* model, int32_t top_k,
                                                int32_t* best_idx, int64_t* best_bound, void* hip_stream);

/* Release the batch and its device memory (waits for its work).  NULL is a
 * no-op. */
void dagbound_destroy_batch(dagbound_batch* batch);

/* Releases the library's process-wide device resources: freed device
 * blocks it keeps for reuse and its per-device side streams (after waiting
 * for their work).  Call after every batch and model is destroyed, while the
 * HIP runtime is still up (the Python binding calls it at interpreter exit);
 * later calls recreate what they need. */
void dagbound_shutdown(void);

/* Message of the last failing call on this thread ("" if none). */
const char* dagbound_last_error(void);

/* Library version string. */
const char* dagbound_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DAGBOUND_H */
