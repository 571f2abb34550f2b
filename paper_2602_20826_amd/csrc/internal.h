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
  uint16_t* indeg;          // [T_N] predecessor count by sigma rank
  uint16_t* inv;            // [T_N] sigma rank of each local node id
  uint32_t* soff;           // [T_N + D] successor offsets by sigma rank, N_d + 1 per DAG at node_off[d] + d
  uint16_t* succ;           // [T_E] successor sigma ranks, DAG d at edge_off[d]
  int64_t* wanc;            // [T_N] W^anc by local node id (inspection)
  int32_t* ngroups;         // [D] |Pi|
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

// err[0]: first failing DAG and code; err[1]: largest load of the batch.
hipError_t launch_prep(const Tables& t, const PrepInputs& in, int32_t D, int32_t M, int32_t max_n,
                       unsigned long long* err, hipStream_t stream);

// Slots of the per-lane table of segmented residuals in the first
// evaluation pass; a tile that needs more goes to the global-memory pass.
constexpr int RES_SLOTS = 12;
// Workgroups of the global-memory pass (each owns max_n * 64 residual words).
constexpr int GLOBAL_PASS_GRID = 256;
enum : int32_t { EVAL_PATH_AUTO = 0, EVAL_PATH_GLOBAL = 1 };

struct SweepArgs {
  Tables t;
  int32_t D, M, K;
  const uint8_t* alloc;         // explicit bytes, or nullptr when seeded
  uint64_t seed;
  int64_t* bounds;              // [D*K] or nullptr
  int64_t* cp;                  // [D*K] or nullptr
  int64_t* intf;                // [D*K] or nullptr
  unsigned long long* best;     // [D] packed (bound << 22 | c), atomicMin
  uint32_t* ovf_list;           // [D * ceil(K/64)] tiles handed to the global pass
  uint32_t* ovf_count;          // [1]
  uint32_t* gres;               // [GLOBAL_PASS_GRID][max_n][64] residual tables
  int32_t max_n, max_e;
  int32_t res_slots;            // <= RES_SLOTS
  int32_t path;                 // EVAL_PATH_*
  int32_t small_loads;          // every C_hat < 2^22
};

// Packing of the per-DAG minimum: bound < 2^42 (the summed load is < 2^40)
// and candidate < 2^22.
constexpr int BEST_SHIFT = 22;

// Dynamic LDS bytes one evaluation workgroup needs for the batch's largest DAG.
size_t sweep_lds_need(int max_n, int max_e);
constexpr size_t LDS_LIMIT = 160 * 1024;

// Evaluates every (DAG, candidate) pair; also resets `best` and fills it.
hipError_t launch_sweep(const SweepArgs& a, hipStream_t stream);
hipError_t launch_best_final(const unsigned long long* best, int32_t D, int32_t* idx, int64_t* bound,
                             hipStream_t stream);

}  // namespace dagbound
