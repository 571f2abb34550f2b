// Allocation-independent preprocessing on gfx950: input validation, ancestor
// closure and W^anc (Eq. 2), the join-node list Theta and blocks (Eq. 3),
// the in-block forests whose root-to-leaf paths are the local complete paths
// (Eq. 4), and the balanced groups of Algorithm 1 (Rules 1 and 2).
//
// One 64-lane wavefront per DAG.  Node sets are bitsets of NW 64-bit words in
// LDS (NW = ceil(N_d / 64)).  The tables it writes are indexed by sigma rank,
// the order of descending W^anc with ties to the smaller local id; that order
// is the Top_M order of Algorithm 1 and the launch order of parallel nodes in
// Section 4.1, so the evaluation kernel never sorts.
#include <climits>

#include "internal.h"

namespace dagbound {
namespace {

constexpr int WAVE = 64;

// Wave reductions and the inclusive scan through DPP: row shifts build the
// prefix within each row of 16 lanes, two row broadcasts carry it across
// rows; lane 63 ends with the total.  Lanes without a source take the
// operation's identity.
template <class Op>
__device__ inline uint32_t wave_scan_dpp(uint32_t x, uint32_t id, Op op) {
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x111, 0xf, 0xf, false));  // row_shr:1
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x112, 0xf, 0xf, false));  // row_shr:2
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x114, 0xf, 0xf, false));  // row_shr:4
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x118, 0xf, 0xf, false));  // row_shr:8
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x142, 0xa, 0xf, false));  // row_bcast:15
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return x;
}
__device__ inline int wave_min_i32(int x) {
  const uint32_t b = (uint32_t)x ^ 0x80000000u;  // order-preserving map to unsigned
  const uint32_t r = wave_scan_dpp(b, 0xffffffffu, [](uint32_t p, uint32_t q) { return p < q ? p : q; });
  return (int)((uint32_t)__builtin_amdgcn_readlane((int)r, 63) ^ 0x80000000u);
}
__device__ inline uint32_t wave_max_u32(uint32_t x) {
  const uint32_t r = wave_scan_dpp(x, 0u, [](uint32_t p, uint32_t q) { return p > q ? p : q; });
  return (uint32_t)__builtin_amdgcn_readlane((int)r, 63);
}
__device__ inline uint32_t wave_incl_scan_u32(uint32_t x) {
  return wave_scan_dpp(x, 0u, [](uint32_t p, uint32_t q) { return p + q; });
}
__device__ inline uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Bytes of dynamic LDS the kernel carves for NW words per bitset.
__host__ __device__ constexpr size_t prep_lds_bytes(int NW) {
  return (size_t)NW * 64 * NW * 8 * 2   // pred, anc bitsets
         + (size_t)NW * 64 * 8          // wanc
         + (size_t)NW * 8 + 8           // done bitset, summed load
         + (size_t)NW * 64 * 4 * 6      // wcet, par, indeg, outdeg/cursor, block, parent
         + 8 * 4                        // misc scalars
         + (size_t)NW * 64 * 2 * 3      // sig, perm, theta
         + (size_t)NW * 64;             // closure state bytes
}

// Word w of node v's bitset row: rows of NW words with the word index XOR-ed
// by v's low bits, so lanes reading the same word of consecutive rows hit
// different LDS banks.
template <int NW>
__device__ inline int rw(int v, int w) { return v * NW + (w ^ (v & (NW - 1))); }

template <int NW>
__global__ __launch_bounds__(64) void k_prep(Tables t, PrepInputs in, int32_t M, const int32_t* list,
                                            unsigned long long* err) {
  constexpr int NMAX = NW * 64;
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* s_pred = (uint64_t*)smem;                // [NMAX][NW]: predecessors of v
  uint64_t* s_anc = s_pred + NMAX * NW;              // [NMAX][NW]: ance(v)
  int64_t* s_wanc = (int64_t*)(s_anc + NMAX * NW);   // [NMAX]
  uint64_t* s_done = (uint64_t*)(s_wanc + NMAX);     // [NW]
  unsigned long long* s_sum = (unsigned long long*)(s_done + NW);
  uint32_t* s_wcet = (uint32_t*)(s_sum + 1);         // [NMAX]
  uint32_t* s_par = s_wcet + NMAX;                   // [NMAX] p, saturated at 2^31-1
  uint32_t* s_indeg = s_par + NMAX;
  uint32_t* s_cursor = s_indeg + NMAX;               // out-degree, then fill cursor
  int32_t* s_block = (int32_t*)(s_cursor + NMAX);
  int32_t* s_parent = s_block + NMAX;
  uint32_t* s_misc = (uint32_t*)(s_parent + NMAX);   // [0] error code, [1] theta count
  uint16_t* s_sig = (uint16_t*)(s_misc + 8);         // sigma rank of local id
  uint16_t* s_perm = s_sig + NMAX;                   // local id of sigma rank
  uint16_t* s_theta = s_perm + NMAX;                 // join nodes in Theta order
  uint8_t* s_state = (uint8_t*)(s_theta + NMAX);     // closure state: 0 open, 1 done, 2 new

  const int d = list ? list[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t n0 = t.node_off[d];
  const int N = (int)(t.node_off[d + 1] - n0);
  const int64_t e0 = t.edge_off[d];
  const int64_t E = t.edge_off[d + 1] - e0;

  // the first loads of node and edge data are issued before the LDS is
  // cleared, so their latency overlaps it
  constexpr int EPRE = 4;
  int64_t w_first = 1;
  int32_t p_first = 1;
  if (lane < N) {
    w_first = in.wcet[n0 + lane];
    p_first = in.par[n0 + lane];
  }
  int32_t eu[EPRE], ev[EPRE];
#pragma unroll
  for (int q = 0; q < EPRE; q++) {
    const int64_t k = lane + (int64_t)q * WAVE;
    eu[q] = k < E ? in.src[e0 + k] : 0;
    ev[q] = k < E ? in.dst[e0 + k] : 0;
  }
  if (lane == 0) { s_misc[0] = 0; s_misc[1] = 0; *s_sum = 0; }
  for (int i = lane; i < N * NW; i += WAVE) { s_pred[i] = 0; s_anc[i] = 0; }
  for (int w = lane; w < NW; w += WAVE) s_done[w] = 0;
  for (int v = lane; v < N; v += WAVE) {
    s_indeg[v] = 0; s_cursor[v] = 0; s_state[v] = 0;
  }
  __syncthreads();

  // Task model (Section 2.1): loads and parallelism.
  uint32_t wmax = 0;
  unsigned long long lsum = 0;  // summed per lane, then over the wave
  for (int v = lane; v < N; v += WAVE) {
    int64_t w = v == lane ? w_first : in.wcet[n0 + v];
    int32_t p = v == lane ? p_first : in.par[n0 + v];
    if (w < 1 || w > 0x7fffffffLL || p < 1) { atomicCAS(&s_misc[0], 0u, (uint32_t)PREP_E_RANGE); w = 1; p = 1; }
    s_wcet[v] = (uint32_t)w;
    s_par[v] = (uint32_t)p;
    lsum += (unsigned long long)w;
    wmax = max(wmax, (uint32_t)w);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
  if (lane == 0) *s_sum = lsum;
  wmax = wave_max_u32(wmax);
  // err[1] bit 0 flags a load of 2^20 or more somewhere in the batch (set
  // rarely, so DAGs do not queue on one global address)
  if (lane == 0 && wmax >= (1u << 20)) atomicOr(&err[1], 1ull);
  // Edges: range, self-loop, duplicates (an LDS bitset of predecessors).
  // The first EPRE rounds come from the loads issued above; later rounds
  // load EPRE at a time.
  for (int64_t kb = 0; kb < E; kb += (int64_t)EPRE * WAVE) {
    if (kb > 0) {
#pragma unroll
      for (int q = 0; q < EPRE; q++) {
        const int64_t k = kb + lane + (int64_t)q * WAVE;
        eu[q] = k < E ? in.src[e0 + k] : 0;
        ev[q] = k < E ? in.dst[e0 + k] : 0;
      }
    }
#pragma unroll
    for (int q = 0; q < EPRE; q++) {
      const int64_t k = kb + lane + (int64_t)q * WAVE;
      if (k >= E) continue;
      const int32_t u = eu[q], v = ev[q];
      if (u < 0 || u >= N || v < 0 || v >= N) { atomicCAS(&s_misc[0], 0u, (uint32_t)PREP_E_RANGE); continue; }
      if (u == v) { atomicCAS(&s_misc[0], 0u, (uint32_t)PREP_E_CYCLE); continue; }
      uint64_t bit = 1ull << (u & 63);
      uint64_t old = atomicOr((unsigned long long*)&s_pred[rw<NW>(v, u >> 6)], (unsigned long long)bit);
      if (old & bit) { atomicCAS(&s_misc[0], 0u, (uint32_t)PREP_E_DUP); continue; }
      atomicAdd(&s_indeg[v], 1u);
      atomicAdd(&s_cursor[u], 1u);
    }
  }
  __syncthreads();
  {
    uint32_t dmax = 0;
    for (int v = lane; v < N; v += WAVE) dmax = max(dmax, s_indeg[v]);
    dmax = wave_max_u32(dmax);
    if (lane == 0 && dmax >= 256) atomicOr(&err[1], 2ull);
  }
  if (s_misc[0] == 0 && *s_sum >= (1ull << 40)) {
    if (lane == 0) s_misc[0] = PREP_E_OVERFLOW;
  }
  __syncthreads();
  if (s_misc[0]) {
    if (lane == 0) atomicMin(err, ((unsigned long long)d << 8) | s_misc[0]);
    return;
  }

  // Ancestor closure in topological waves: a node whose predecessors are all
  // closed takes ance(v) = union of (ance(u) + u) over its predecessors u.
  for (;;) {
    for (int v = lane; v < N; v += WAVE) {
      if (s_state[v]) continue;
      bool ready = true;
#pragma unroll
      for (int w = 0; w < NW; w++) ready = ready && !(s_pred[rw<NW>(v, w)] & ~s_done[w]);
      if (!ready) continue;
      uint64_t acc[NW];
#pragma unroll
      for (int w = 0; w < NW; w++) acc[w] = s_pred[rw<NW>(v, w)];
#pragma unroll
      for (int w = 0; w < NW; w++) {
        uint64_t b = s_pred[rw<NW>(v, w)];
        while (b) {
          int u = w * 64 + __builtin_ctzll(b);
          b &= b - 1;
#pragma unroll
          for (int x = 0; x < NW; x++) acc[x] |= s_anc[rw<NW>(u, x)];
        }
      }
#pragma unroll
      for (int w = 0; w < NW; w++) s_anc[rw<NW>(v, w)] = acc[w];
      s_state[v] = 2;
    }
    __syncthreads();
    bool fresh = false;
    for (int v = lane; v < N; v += WAVE)
      if (s_state[v] == 2) {
        s_state[v] = 1;
        atomicOr((unsigned long long*)&s_done[v >> 6], 1ull << (v & 63));
        fresh = true;
      }
    const bool any_fresh = __ballot(fresh) != 0;
    __syncthreads();
    if (!any_fresh) break;
  }
  {
    int closed = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) closed += __popcll(s_done[w]);
    if (closed != N) {  // some node never became ready: a cycle
      if (lane == 0) atomicMin(err, ((unsigned long long)d << 8) | PREP_E_CYCLE);
      return;
    }
  }

  // Eq. 2: W^anc(v) = C_hat_v + sum of C_hat over ance(v).
  // Four ancestors per step, so that their loads are in flight together.
  for (int v = lane; v < N; v += WAVE) {
    int64_t sum = s_wcet[v];
#pragma unroll
    for (int w = 0; w < NW; w++) {
      uint64_t b = s_anc[rw<NW>(v, w)];
      while (b) {
        uint32_t x[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
          x[t] = 0;
          if (b) {
            x[t] = s_wcet[w * 64 + __builtin_ctzll(b)];
            b &= b - 1;
          }
        }
        sum += (int64_t)x[0] + x[1] + x[2] + x[3];
      }
    }
    s_wanc[v] = sum;
  }
  __syncthreads();

  // Sigma rank (descending W^anc, ties to the smaller id) and the Theta rank
  // of join nodes (in-degree >= 2; ascending W^anc, ties to the smaller id).
  for (int v = lane; v < N; v += WAVE) {
    const int64_t wv = s_wanc[v];
    const bool join = s_indeg[v] >= 2;
    int r = 0, th = 0;
    for (int u = 0; u < N; u++) {
      const int64_t wu = s_wanc[u];
      r += (wu > wv) | ((wu == wv) & (u < v));
      th += (s_indeg[u] >= 2) & ((wu < wv) | ((wu == wv) & (u < v)));
    }
    s_sig[v] = (uint16_t)r;
    s_perm[r] = (uint16_t)v;
    if (join) { s_theta[th] = (uint16_t)v; atomicAdd(&s_misc[1], 1u); }
  }
  __syncthreads();
  const int nth = (int)s_misc[1];

  // Eq. 3: B_k = ance(theta_k) minus earlier blocks, i.e. v lands in the
  // first block (in Theta order) whose join node has v as an ancestor; the
  // rest form the residual block (index nth).
  // The join nodes are walked in Theta order (wave-uniform); each lane
  // assigns its nodes (v = lane, lane + 64, ...) to the first join node whose
  // ancestor row holds them, and the walk ends once every node is assigned.
  {
    int blk[NW];
    uint64_t open[NW];
#pragma unroll
    for (int j = 0; j < NW; j++) {
      blk[j] = nth;
      open[j] = __ballot(j * 64 + lane < N);
    }
    // Theta ids 64 at a time in registers; the next join node's row is
    // read one step ahead.
    uint32_t chunk = lane < nth ? s_theta[lane] : 0u;
    uint64_t row[NW];
    if (nth > 0) {
      const int th0 = __builtin_amdgcn_readlane((int)chunk, 0);
#pragma unroll
      for (int j = 0; j < NW; j++) row[j] = s_anc[rw<NW>(th0, j)];
    }
    for (int k = 0; k < nth; k++) {
      bool any = false;
#pragma unroll
      for (int j = 0; j < NW; j++) any = any || open[j] != 0;
      if (!any) break;
      uint64_t cur[NW];
#pragma unroll
      for (int j = 0; j < NW; j++) cur[j] = row[j];
      if (k + 1 < nth) {
        if (((k + 1) & 63) == 0) chunk = k + 1 + lane < nth ? s_theta[k + 1 + lane] : 0u;
        const int thn = __builtin_amdgcn_readlane((int)chunk, (k + 1) & 63);
#pragma unroll
        for (int j = 0; j < NW; j++) row[j] = s_anc[rw<NW>(thn, j)];
      }
#pragma unroll
      for (int j = 0; j < NW; j++) {
        const bool hit = ((open[j] >> lane) & 1) && ((cur[j] >> lane) & 1);
        if (hit) blk[j] = k;
        open[j] &= ~__ballot(hit);
      }
    }
#pragma unroll
    for (int j = 0; j < NW; j++)
      if (j * 64 + lane < N) s_block[j * 64 + lane] = blk[j];
  }
  __syncthreads();
  // In-block parent: a node has at most one predecessor in its own block, so
  // each block is a forest whose root-to-leaf paths are its local complete
  // paths (Eq. 4).
  for (int v = lane; v < N; v += WAVE) {
    int parent = -1, cnt = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
      uint64_t b = s_pred[rw<NW>(v, w)];
      while (b) {
        int u = w * 64 + __builtin_ctzll(b);
        b &= b - 1;
        if (s_block[u] == s_block[v]) { parent = u; cnt++; }
      }
    }
    if (cnt > 1) atomicCAS(&s_misc[0], 0u, (uint32_t)PREP_E_INTERNAL);
    s_parent[v] = parent;
  }
  __syncthreads();
  if (s_misc[0]) {
    if (lane == 0) atomicMin(err, ((unsigned long long)d << 8) | s_misc[0]);
    return;
  }

  // Algorithm 1, balanced groups.  Blocks are taken in order; within the
  // current block the heads of the local complete paths are the ungrouped
  // nodes whose in-block parent is grouped (or absent).  Lane l holds sigma
  // ranks l, l+64, ... with their block, parent (as a sigma rank) and
  // m^max = min(p, C_hat) in registers; G is the set of grouped sigma ranks.
  // Heads are picked in sigma order (Top_M, Rule 1) and Rule 2 keeps only
  // the first node of largest m^max when that reaches M.
  int blk[NW], psig[NW];
  uint32_t mmax[NW];
  bool grouped[NW];
  uint8_t* s_gflag = s_state;  // grouped flag by sigma rank (the closure state is dead here)
#pragma unroll
  for (int k = 0; k < NW; k++) {
    const int s = k * 64 + lane;
    grouped[k] = s >= N;
    blk[k] = INT_MAX;
    psig[k] = -1;
    mmax[k] = 0;
    if (s < N) {
      const int v = s_perm[s];
      blk[k] = s_block[v];
      psig[k] = s_parent[v] < 0 ? -1 : (int)s_sig[s_parent[v]];
      mmax[k] = min(s_par[v], s_wcet[v]);
      s_gflag[s] = 0;
    }
  }
  __syncthreads();
  uint16_t* gl = t.gl + n0;
  int gpos = 0, ng = 0;
  for (;;) {
    int bmin = INT_MAX;
#pragma unroll
    for (int k = 0; k < NW; k++)
      if (!grouped[k]) bmin = min(bmin, blk[k]);
    bmin = wave_min_i32(bmin);
    if (bmin == INT_MAX) break;
    bool head[NW];
    uint64_t hb[NW];
    int nh = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
      const bool pg = psig[k] < 0 || s_gflag[psig[k]] != 0;
      head[k] = !grouped[k] && blk[k] == bmin && pg;
      hb[k] = __ballot(head[k]);
      nh += __popcll(hb[k]);
    }
    const int take = min(nh, (int)M);
    bool sel[NW];
    uint64_t sb[NW];
    int before = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
      sel[k] = head[k] && (before + __popcll(hb[k] & lanes_below(lane)) < take);
      sb[k] = __ballot(sel[k]);
      before += __popcll(hb[k]);
    }
    if (take > 1) {
      uint32_t mx = 0;
#pragma unroll
      for (int k = 0; k < NW; k++)
        if (sel[k]) mx = max(mx, mmax[k]);
      mx = wave_max_u32(mx);
      if (mx >= (uint32_t)M) {
        bool found = false;
#pragma unroll
        for (int k = 0; k < NW; k++) {
          const uint64_t hbits = __ballot(sel[k] && mmax[k] == mx);
          uint64_t keep = 0;
          if (!found && hbits) { keep = hbits & (~hbits + 1); found = true; }
          sb[k] = keep;
          sel[k] = (keep >> lane) & 1;
        }
      }
    }
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) cnt += __popcll(sb[k]);
    int base = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
      if (sel[k]) {
        const int s = k * 64 + lane;
        const int pos = gpos + base + __popcll(sb[k] & lanes_below(lane));
        const uint32_t last = pos == gpos + cnt - 1 ? 0x8000u : 0u;
        gl[pos] = (uint16_t)(s | last);
        grouped[k] = true;
        s_gflag[s] = 1;
      }
      base += __popcll(sb[k]);
    }
    gpos += cnt;
    ng++;
    __syncthreads();
  }
  if (lane == 0) t.ngroups[d] = ng;

  // Tables by sigma rank.
  for (int s = lane; s < N; s += WAVE) {
    const int v = s_perm[s];
    t.wc[n0 + s] = s_wcet[v];
    t.pp[n0 + s] = (uint16_t)min(s_par[v], (uint32_t)M);
    t.mx[n0 + s] = min(s_par[v], s_wcet[v]);
    t.indeg[n0 + s] = (uint16_t)s_indeg[v];
  }
  for (int v = lane; v < N; v += WAVE) {
    t.inv[n0 + v] = s_sig[v];
    t.wanc[n0 + v] = s_wanc[v];
  }
  // Successor lists in sigma order: offsets by an exclusive scan of the
  // out-degrees, then each edge drops its head's sigma rank into its tail's
  // list.
  uint32_t* soff = t.soff + n0 + d;
  uint32_t carry = 0;
  for (int b = 0; b < N; b += WAVE) {
    const int s = b + lane;
    const uint32_t x = s < N ? s_cursor[s_perm[s]] : 0u;
    const uint32_t incl = wave_incl_scan_u32(x);
    if (s < N) soff[s] = carry + incl - x;
    carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  }
  if (lane == 0) soff[N] = carry;
  __syncthreads();
  for (int s = lane; s < N; s += WAVE) s_cursor[s_perm[s]] = soff[s];
  __syncthreads();
  for (int64_t k = lane; k < E; k += WAVE) {
    const int32_t u = in.src[e0 + k], v = in.dst[e0 + k];
    const uint32_t pos = atomicAdd(&s_cursor[u], 1u);
    t.succ[e0 + pos] = s_sig[v];
  }
  // Node records of the large-DAG evaluation (kept when the batch also
  // holds DAGs above 512 nodes, which may run every DAG in that kernel).
  if (t.nrec) {
    __syncthreads();
    for (int s = lane; s < N; s += WAVE) {
      const int v = s_perm[s];
      const uint32_t deg = soff[s + 1] - soff[s];
      t.nrec[n0 + s] = make_uint4(s_wcet[v], min(s_par[v], (uint32_t)M) | ((uint32_t)s << 16), soff[s],
                                  (uint32_t)v | (deg << 16));
    }
    __syncthreads();
    for (int k = lane; k < N; k += WAVE) {
      const uint32_t g = gl[k];
      uint4 r = t.nrec[n0 + (g & 0x7FFF)];
      r.y |= (g & 0x8000u) << 16;
      t.mrec[n0 + k] = r;
    }
  }
}

template <int NW>
hipError_t launch_prep_nw(const Tables& t, const PrepInputs& in, int32_t count, int32_t M, const int32_t* list,
                          unsigned long long* err, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const size_t lds = prep_lds_bytes(NW);
  hipError_t e = hipFuncSetAttribute((const void*)k_prep<NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep<NW>, dim3(count), dim3(64), lds, stream, t, in, M, list, err);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prep(const Tables& t, const PrepInputs& in, int32_t D, int32_t M, int32_t max_n,
                       const int32_t* order, const int32_t* class_off, unsigned long long* err,
                       void* lscratch, const int32_t* class_max_n, const int32_t* class_max_e,
                       const hipStream_t* side, hipEvent_t fork, const hipEvent_t* join, hipStream_t stream) {
  if (D <= 0) return hipSuccess;
  if (max_n > LARGE_MAX_N) return hipErrorInvalidValue;
  if (!order) {  // one launch sized for the largest DAG
    switch (class_of(max_n)) {
      case 0: return launch_prep_nw<1>(t, in, D, M, nullptr, err, stream);
      case 1: return launch_prep_nw<2>(t, in, D, M, nullptr, err, stream);
      case 2: return launch_prep_nw<4>(t, in, D, M, nullptr, err, stream);
      case 3: return launch_prep_nw<8>(t, in, D, M, nullptr, err, stream);
      default: return hipErrorInvalidValue;  // large DAGs need their class's scratch sizes
    }
  }
  // DAGs above 256 nodes go to the workgroup-per-DAG kernel (large.hip), one
  // launch per class, largest first; each smaller class gets a launch sized
  // for its own bitset width (one-word rows for DAGs up to 64 nodes)
  hipError_t e = hipSuccess;
  // the small classes' launches touch only the failure words (atomics), so
  // they may run beside each other and beside the large classes, which stay
  // in order on `stream` (they share the work counter err[2])
  bool forked[3] = {false, false, false};
  if (side && fork && join) e = hipEventRecord(fork, stream);
  for (int c = 2; c >= 0 && e == hipSuccess; c--) {
    const int32_t n = class_off[c + 1] - class_off[c];
    if (n <= 0) continue;
    hipStream_t sc = stream;
    if (side && fork && join) {
      sc = side[c];
      e = hipStreamWaitEvent(sc, fork, 0);
      if (e != hipSuccess) break;
    }
    const int32_t* list = order + class_off[c];
    e = c == 2 ? launch_prep_nw<4>(t, in, n, M, list, err, sc)
               : c == 1 ? launch_prep_nw<2>(t, in, n, M, list, err, sc) : launch_prep_nw<1>(t, in, n, M, list, err, sc);
    if (e == hipSuccess && sc != stream) {
      e = hipEventRecord(join[c], sc);
      forked[c] = e == hipSuccess;
    }
  }
  for (int c = LARGE_CLASS; c >= 3 && e == hipSuccess; c--)
    e = launch_prep_large(t, in, class_off[c + 1] - class_off[c], M, order + class_off[c], err, lscratch,
                          class_max_n[c], class_max_e[c], stream);
  for (int c = 0; c < 3; c++) {  // join every forked stream, even after an error
    if (!forked[c]) continue;
    const hipError_t w = hipStreamWaitEvent(stream, join[c], 0);
    if (e == hipSuccess) e = w;
  }
  return e;
}

}  // namespace dagbound
