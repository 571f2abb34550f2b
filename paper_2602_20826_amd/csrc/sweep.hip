// Exact evaluation of the bound on gfx950: Algorithm 2 (parallelism scaling,
// Eq. 5; spare capacity and parallel nodes, Eqs. 6-7; node segmentation;
// extra dependencies as slot order) and the analysis of Lemma 1 and
// Theorem 1, for every (DAG, candidate allocation) pair.
//
// Mapping: one 64-lane wavefront per (DAG, tile of 64 candidates); lane c
// runs candidate c.  The group sequence is the same for every candidate, so
// the slot loop and the member loop are wave-uniform (member data is read
// once per wave and broadcast); only the parallel-node launches and the
// releases they cause diverge.
//
// Per-candidate state:
//   - released / finished / segmented sets: bitsets in registers, indexed by
//     sigma rank (descending W^anc), so the next parallel node to launch is
//     the lowest set bit;
//   - remaining loads: a node's remaining load differs from C_hat only after
//     it was segmented, so each lane keeps the remaining loads of its
//     segmented nodes in a small table ordered by sigma rank ([slot][lane] in
//     LDS; the slot of a node is its rank within the segmented set).  A tile
//     whose table would overflow is handed to a second pass of the same code
//     whose table lives in global memory and holds every node;
//   - candidate bytes: [node][lane] bytes in LDS.
// Releases use per-candidate counters of unfinished predecessors, packed in
// LDS dwords [node][lane].  All arithmetic is integer.
#include "internal.h"

namespace dagbound {
namespace {

constexpr int WAVE = 64;

template <int NW>
__device__ inline uint64_t word_of(const uint64_t (&b)[NW], int v) {
  uint64_t w = b[0];
#pragma unroll
  for (int k = 1; k < NW; k++) w = (v >> 6) == k ? b[k] : w;
  return w;
}
template <int NW>
__device__ inline bool bit_get(const uint64_t (&b)[NW], int v) {
  return (word_of<NW>(b, v) >> (v & 63)) & 1;
}
template <int NW>
__device__ inline void bit_set(uint64_t (&b)[NW], int v) {
#pragma unroll
  for (int k = 0; k < NW; k++) b[k] |= (v >> 6) == k ? (1ull << (v & 63)) : 0ull;
}
template <int NW>
__device__ inline void bit_clear(uint64_t (&b)[NW], int v) {
#pragma unroll
  for (int k = 0; k < NW; k++) b[k] &= (v >> 6) == k ? ~(1ull << (v & 63)) : ~0ull;
}
template <int NW>
__device__ inline int bit_first(const uint64_t (&b)[NW]) {
  int r = -1;
#pragma unroll
  for (int k = NW - 1; k >= 0; k--) r = b[k] ? k * 64 + __builtin_ctzll(b[k]) : r;
  return r;
}
// Index of the lowest set bit (or -1), cleared in place.
template <int NW>
__device__ inline int pop_first(uint64_t (&b)[NW]) {
  int r = -1;
  bool done = false;
#pragma unroll
  for (int k = 0; k < NW; k++) {
    const bool take = !done && b[k] != 0;
    if (take) {
      r = k * 64 + __builtin_ctzll(b[k]);
      b[k] &= b[k] - 1;
    }
    done = done || take;
  }
  return r;
}
template <int NW>
__device__ inline bool bits_any(const uint64_t (&b)[NW]) {
  uint64_t x = 0;
#pragma unroll
  for (int k = 0; k < NW; k++) x |= b[k];
  return x != 0;
}
// Number of set bits below bit v.
template <int NW>
__device__ inline int bit_rank(const uint64_t (&b)[NW], int v) {
  int r = 0;
#pragma unroll
  for (int k = 0; k < NW; k++) {
    const int hi = v - k * 64;
    const uint64_t m = hi >= 64 ? ~0ull : (hi <= 0 ? 0ull : (~0ull >> (64 - hi)));
    r += __popcll(b[k] & m);
  }
  return r;
}
template <int NW>
__device__ inline int bit_count(const uint64_t (&b)[NW]) {
  int r = 0;
#pragma unroll
  for (int k = 0; k < NW; k++) r += __popcll(b[k]);
  return r;
}

__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// ceil(a / b) for a < 2^22, b >= 1: a single-precision estimate is within one
// of the quotient; one integer step corrects it.
__device__ inline uint32_t ceil_div_small(uint32_t a, uint32_t b) {
  uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
  int32_t r = (int32_t)(a - q * b);
  if (r < 0) { q--; r += (int32_t)b; }
  else if (r >= (int32_t)b) { q++; r -= (int32_t)b; }
  return q + (r != 0);
}
template <bool SMALL>
__device__ inline uint32_t ceil_div(uint32_t a, uint32_t b) {
  if (SMALL) return ceil_div_small(a, b);
  return (uint32_t)(((uint64_t)a + b - 1) / b);
}

// round(cv * M / W), half up, exactly: floor((2 cv M + W) / (2 W)).  The
// quotient is at most M + 1/2 < 2^16; a double estimate is within one of it
// and one integer step corrects it.
__device__ inline uint32_t round_share(uint32_t cv, uint32_t M, uint64_t W) {
  const uint64_t num = 2ull * cv * M + W;
  const uint64_t den = 2ull * W;
  uint32_t q = (uint32_t)((double)num / (double)den);
  if ((uint64_t)(q + 1) * den <= num) q++;
  else if ((uint64_t)q * den > num) q--;
  return q;
}

// Counter-based candidate byte (the hash documented for seeded allocations).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// OR over the wavefront: row shifts within each row of 16 lanes, then row
// broadcasts; lane 63 ends with the OR of all 64 lanes.
__device__ inline uint32_t wave_or32(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}
__device__ inline uint64_t wave_or64(uint64_t x) {
  return ((uint64_t)wave_or32((uint32_t)(x >> 32)) << 32) | wave_or32((uint32_t)x);
}

// Unfinished-predecessor counters, packed into dwords laid out [node / P][lane]
// so a lane always hits its own bank: P = 4 byte counters while every
// in-degree fits (N <= 256), P = 2 half-word counters above.  A decrement is
// one LDS atomic subtract on the node's field (it never borrows: a counter is
// positive until its last predecessor finishes).
template <int NW> struct Cnt { static constexpr int PER = 4, BITS = 8; };
template <> struct Cnt<8> { static constexpr int PER = 2, BITS = 16; };

// LDS layout of one wavefront (bytes), for the batch's largest DAG.
struct Lds {
  size_t mem, node, soff, succ, ppv, res, r, npr, total;
};
__host__ __device__ inline Lds lds_layout(int maxn, int maxe, int nw, bool big) {
  Lds l;
  size_t o = 0;
  l.mem = o;  o += (size_t)maxn * 16;           // members in group order
  l.node = o; o += (size_t)maxn * 8;            // node info by sigma rank
  l.soff = o; o += (size_t)(maxn + 1) * 4;      // successor offsets by sigma rank
  l.succ = o; o += ((size_t)maxe * 2 + 15) & ~(size_t)15;  // successor sigma ranks
  l.ppv = o;  o += ((size_t)maxn * 2 + 15) & ~(size_t)15;  // min(p, M) by local id
  l.res = o;  o += big ? 0 : (size_t)RES_SLOTS * WAVE * 4;  // residual table
  l.r = o;    o += (size_t)maxn * WAVE;         // candidate bytes [local id][lane]
  l.npr = o;  o += (size_t)((maxn + 3) / 4 + 1) * WAVE * 4 * (nw == 8 ? 2 : 1);  // packed counters
  l.total = (o + 15) & ~(size_t)15;
  return l;
}

// One (DAG, 64-candidate tile).  Returns true if the lane tables overflowed
// (nothing was written; the tile must be redone by the global-table pass).
template <int NW, bool BIG, bool SMALL>
__device__ bool eval_tile(const SweepArgs& a, int item, unsigned char* smem, uint32_t* gres) {
  constexpr int CP = Cnt<NW>::PER, CB = Cnt<NW>::BITS;
  constexpr uint32_t CMASK = (1u << CB) - 1u;
  const int ntile = (a.K + WAVE - 1) / WAVE;
  const int d = item / ntile;
  const int tile = item - d * ntile;
  const int lane = threadIdx.x;
  const int slot = tile * WAVE + lane;  // output position
  const bool active = slot < a.K;
  const int c = a.cand_list ? (active ? a.cand_list[(int64_t)d * a.K + slot] : 0) : slot;  // candidate id
  const int64_t n0 = a.t.node_off[d];
  const int N = (int)(a.t.node_off[d + 1] - n0);
  const int64_t e0 = a.t.edge_off[d];
  const int E = (int)(a.t.edge_off[d + 1] - e0);
  const uint32_t M = (uint32_t)a.M;
  const Lds L = lds_layout(a.max_n, a.max_e, NW, BIG);
  uint4* s_mem = (uint4*)(smem + L.mem);       // {C_hat, pp | v << 16, s | last << 31, 0}
  uint2* s_node = (uint2*)(smem + L.node);     // {C_hat, pp | v << 16} by sigma rank
  uint32_t* s_soff = (uint32_t*)(smem + L.soff);
  uint16_t* s_succ = (uint16_t*)(smem + L.succ);
  uint16_t* s_ppv = (uint16_t*)(smem + L.ppv); // [local id]
  uint32_t* res = BIG ? gres : (uint32_t*)(smem + L.res);  // [slot][lane]
  uint8_t* s_r = smem + L.r;                   // [local id][lane]
  uint32_t* s_cnt = (uint32_t*)(smem + L.npr); // [sigma / CP][lane]
  const int qcap = BIG ? a.max_n : a.res_slots;

  // ---- DAG tables (shared by the 64 candidates)
  for (int s = lane; s < N; s += WAVE) s_node[s] = make_uint2(a.t.wc[n0 + s], a.t.pp[n0 + s]);
  for (int s = lane; s <= N; s += WAVE) s_soff[s] = a.t.soff[n0 + d + s];
  for (int e = lane; e < E; e += WAVE) s_succ[e] = a.t.succ[e0 + e];
  __syncthreads();
  for (int v = lane; v < N; v += WAVE) {
    const int s = a.t.inv[n0 + v];
    const uint32_t y = s_node[s].y;
    s_node[s].y = y | ((uint32_t)v << 16);
    s_ppv[v] = (uint16_t)y;
  }
  __syncthreads();
  for (int k = lane; k < N; k += WAVE) {
    const uint32_t g = a.t.gl[n0 + k];
    const int s = g & 0x7FFF;
    const uint2 nd = s_node[s];
    s_mem[k] = make_uint4(nd.x, nd.y, (uint32_t)s | ((g & 0x8000u) << 16), 0u);
  }
  // per-candidate unfinished-predecessor counters; sources are released
  uint64_t rel[NW], seg[NW];
#pragma unroll
  for (int w = 0; w < NW; w++) { rel[w] = 0; seg[w] = 0; }
  for (int s0 = 0; s0 < N; s0 += CP) {
    uint32_t packed = 0;
#pragma unroll
    for (int i = 0; i < CP; i++) {
      const int s = s0 + i;
      if (s < N) {
        const uint32_t np = a.t.indeg[n0 + s];
        packed |= np << (CB * i);
        if (np == 0) bit_set<NW>(rel, s);
      }
    }
    s_cnt[(s0 / CP) * WAVE + lane] = packed;
  }
  // ---- candidate bytes of this lane, by local id.  Candidate 0 is the
  // paper's own rule (all zero); lanes past K run zeros and store nothing.
  if (a.alloc) {
    if (c > 0 && active) {
      // 16-byte aligned loads over the lane's row; an aligned chunk holding a
      // byte of the row never leaves that byte's page.
      const uint8_t* row = a.alloc + (int64_t)a.K * n0 + (int64_t)c * N;
      const uintptr_t rb = (uintptr_t)row;
      const uintptr_t p0 = rb & ~(uintptr_t)15;
      const uintptr_t pe = rb + (uintptr_t)N;
      for (uintptr_t p = p0; p < pe; p += 16) {
        const uint4 q = *(const uint4*)p;
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 16; j++) {
          const int64_t idx = (int64_t)(p + j) - (int64_t)rb;
          if (idx >= 0 && idx < N) s_r[idx * WAVE + lane] = (uint8_t)(w4[j >> 2] >> (8 * (j & 3)));
        }
      }
    } else {
      for (int v = 0; v < N; v++) s_r[v * WAVE + lane] = 0;
    }
  } else {
    const uint64_t key = mix64(a.seed ^ mix64((uint64_t)d * 0x9E3779B97F4A7C15ull));
    uint64_t word = 0;
    for (int v = 0; v < N; v++) {
      if ((v & 3) == 0) word = mix64(key ^ (((uint64_t)c << 32) | (uint64_t)(v >> 2)));
      const uint32_t range = min((uint32_t)s_ppv[v], 255u);
      const uint32_t h16 = (uint32_t)(word >> (16 * (v & 3))) & 0xFFFFu;
      const uint32_t r = 1u + ((h16 * range) >> 16);
      s_r[v * WAVE + lane] = (c > 0 && active) ? (uint8_t)r : (uint8_t)0;
    }
  }
  __syncthreads();

  // ---- per-candidate sweep (Algorithm 2 and Theorem 1).  rel: released
  // and unfinished (Algorithm 2's Released_nodes); seg: segmented nodes
  // whose remaining load sits in the residual table.
  uint64_t bound = 0, cp = 0;
  bool ovf = false;
  int k = 0;
  while (k < N) {
    // Pass 1 over the group: its extent, member set, and W(pi_j), the
    // remaining load of the members unfinished in this lane (Eq. 5).
    uint64_t gm[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) gm[w] = 0;
    uint64_t W = 0;
    int kend = k;
    for (;;) {
      const uint4 mm = s_mem[kend];
      const int s = (int)(uni(mm.z) & 0x7FFFu);
      bit_set<NW>(gm, s);
      if (bit_get<NW>(rel, s)) {
        uint32_t cv = uni(mm.x);
        if (bit_get<NW>(seg, s)) cv = res[bit_rank<NW>(seg, s) * WAVE + lane];
        W += cv;
      }
      kend++;
      if ((uni(mm.z) >> 31) || kend >= N) break;
    }
    if (!__ballot(W != 0)) { k = kend; continue; }  // every member finished earlier
    // Pass 2: parallelism of each unfinished member (Eq. 5, or the candidate
    // byte) and its execution time (Eq. 1, t_min = 1, m <= M).
    uint32_t maxC = 0, sm = 0;
    uint64_t A = 0;
    for (int q = k; q < kend; q++) {
      const uint4 mm = s_mem[q];
      const int s = (int)(uni(mm.z) & 0x7FFFu);
      if (!bit_get<NW>(rel, s)) continue;
      uint32_t cv = uni(mm.x);
      if (bit_get<NW>(seg, s)) cv = res[bit_rank<NW>(seg, s) * WAVE + lane];
      const uint32_t rv = s_r[(uni(mm.y) >> 16) * WAVE + lane];
      const uint32_t mx = min(uni(mm.y) & 0xFFFFu, cv);
      uint32_t m;
      if (rv) m = min(rv, mx);
      else m = max(1u, min(mx, round_share(cv, M, W)));
      const uint32_t C = ceil_div<SMALL>(cv, m);
      maxC = max(maxC, C);
      sm += m;
      A += (uint64_t)m * C;
    }
    // Eqs. 6-7: parallel nodes (released, outside the group) take the S spare
    // compute units, largest W^anc first; a node that does not fit in
    // maxC * m is segmented there and the launching stops.  The nodes taken
    // from Q and not segmented are the ones launched whole.
    uint32_t S = (W != 0 && sm < M) ? M - sm : 0u;
    uint64_t Q[NW], Lw[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) { Q[w] = rel[w] & ~gm[w]; Lw[w] = Q[w]; }
    int cseg = -1;
    while (S) {
      const int cn = pop_first<NW>(Q);
      if (cn < 0) break;
      const uint2 nd = s_node[cn];
      const bool sg = bit_get<NW>(seg, cn);
      int rk = 0;
      uint32_t cc = nd.x;
      if (sg) {
        rk = bit_rank<NW>(seg, cn);
        cc = res[rk * WAVE + lane];
      }
      const uint32_t rc = s_r[(nd.y >> 16) * WAVE + lane];
      const uint32_t mx = min(nd.y & 0xFFFFu, cc);
      const uint32_t mc = min(rc ? min(rc, mx) : mx, S);
      const uint64_t cap = (uint64_t)maxC * mc;
      if ((uint64_t)cc > cap) {
        const uint32_t left = cc - (uint32_t)cap;
        cseg = cn;
        if (sg) {
          res[rk * WAVE + lane] = left;
        } else {
          rk = bit_rank<NW>(seg, cn);
          const int cnt = bit_count<NW>(seg);
          if (cnt >= qcap) {
            ovf = true;
          } else {
            for (int i = cnt; i > rk; i--) res[i * WAVE + lane] = res[(i - 1) * WAVE + lane];
            res[rk * WAVE + lane] = left;
            bit_set<NW>(seg, cn);
          }
        }
        break;
      }
      S -= mc;
    }
#pragma unroll
    for (int w = 0; w < NW; w++) Lw[w] &= ~Q[w];
    if (cseg >= 0) bit_clear<NW>(Lw, cseg);
    // Lemma 1, plus the list-scheduling term if the members oversubscribe.
    if (W != 0) {
      uint64_t R = maxC;
      if (sm > M) R += (A - maxC) / M;
      bound += R;
      cp += maxC;
    }
    // Finished now: the unfinished members and the nodes launched whole.
    uint64_t Dn[NW], gone[NW], Fu[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) {
      Dn[w] = (rel[w] & gm[w]) | Lw[w];
      gone[w] = seg[w] & Dn[w];
      rel[w] &= ~Dn[w];
      Fu[w] = gm[w] | wave_or64(Lw[w]);  // finished now in some lane
    }
    while (bits_any<NW>(gone)) {  // drop finished nodes from the residual table
      const int x = pop_first<NW>(gone);
      const int rk = bit_rank<NW>(seg, x);
      const int cnt = bit_count<NW>(seg);
      for (int i = rk; i + 1 < cnt; i++) res[i * WAVE + lane] = res[(i + 1) * WAVE + lane];
      bit_clear<NW>(seg, x);
    }
    // Releases: every node finished now decrements its successors' counters
    // in the lanes where it finished; a counter reaching zero releases its
    // node.  The walk is wave-uniform over the nodes finished in some lane.
    while (bits_any<NW>(Fu)) {
      const int x = pop_first<NW>(Fu);
      const bool mine = bit_get<NW>(Dn, x);
      const uint32_t e1 = uni(s_soff[x + 1]);
      for (uint32_t e = uni(s_soff[x]); e < e1; e++) {
        const int u = (int)uni(s_succ[e]);
        if (mine) {
          const int sh = CB * (u % CP);
          const uint32_t old = atomicSub(&s_cnt[(u / CP) * WAVE + lane], 1u << sh);
          if (((old >> sh) & CMASK) == 1u) bit_set<NW>(rel, u);
        }
      }
    }
    if (__ballot(ovf)) return true;
    k = kend;
  }

  if (active) {
    const int64_t o = (int64_t)d * a.K + slot;
    if (a.bounds) a.bounds[o] = (int64_t)bound;
    if (a.cp) a.cp[o] = (int64_t)cp;
    if (a.intf) a.intf[o] = (int64_t)(bound - cp);
  }
  if (a.best) {
    unsigned long long key = active ? ((bound << BEST_SHIFT) | (uint64_t)slot) : ~0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long y = __shfl_xor(key, o);
      key = y < key ? y : key;
    }
    if (lane == 0) atomicMin(&a.best[d], key);
  }
  return false;
}

// First pass: one tile per workgroup, residual tables in LDS.
template <int NW, bool SMALL>
__global__ __launch_bounds__(64) void k_eval(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = blockIdx.x;
  if (eval_tile<NW, false, SMALL>(a, item, smem, nullptr)) {
    if (threadIdx.x == 0) a.ovf_list[atomicAdd(a.ovf_count, 1u)] = (uint32_t)item;
  }
}

// Second pass: the tiles the first pass handed over (or every tile when
// `direct`), residual tables in global memory sized to hold every node.
template <int NW, bool SMALL>
__global__ __launch_bounds__(64) void k_eval_global(SweepArgs a, int direct, int total) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int count = direct ? total : (int)*a.ovf_count;
  uint32_t* gres = a.gres + (size_t)blockIdx.x * (size_t)a.max_n * WAVE;
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int item = direct ? q : (int)a.ovf_list[q];
    eval_tile<NW, true, SMALL>(a, item, smem, gres);
    __syncthreads();
  }
}

__global__ void k_eval_init(unsigned long long* best, int32_t D, uint32_t* ovf_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D) best[i] = ~0ull;
  if (i == 0) *ovf_count = 0;
}

__global__ void k_best_final(const unsigned long long* best, int32_t D, int32_t* idx, int64_t* bnd,
                             const int32_t* list, int32_t K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D) {
    const unsigned long long k = best[i];
    const int32_t pos = (int32_t)(k & ((1ull << BEST_SHIFT) - 1));
    if (idx) idx[i] = list ? list[(int64_t)i * K + pos] : pos;
    if (bnd) bnd[i] = (int64_t)(k >> BEST_SHIFT);
  }
}

template <int NW, bool SMALL>
hipError_t launch_nw(const SweepArgs& a, hipStream_t stream) {
  const int ntile = (a.K + WAVE - 1) / WAVE;
  const int total = a.D * ntile;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(k_eval_init, dim3((a.D + 255) / 256), dim3(256), 0, stream, a.best, a.D,
                     a.ovf_count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.path != EVAL_PATH_GLOBAL) {
    const size_t lds = lds_layout(a.max_n, a.max_e, NW, false).total;
    e = hipFuncSetAttribute((const void*)k_eval<NW, SMALL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_eval<NW, SMALL>), dim3(total), dim3(WAVE), lds, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const size_t lds = lds_layout(a.max_n, a.max_e, NW, true).total;
  e = hipFuncSetAttribute((const void*)k_eval_global<NW, SMALL>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = a.path == EVAL_PATH_GLOBAL ? min(total, GLOBAL_PASS_GRID) : GLOBAL_PASS_GRID;
  if (grid > 0) {
    hipLaunchKernelGGL((k_eval_global<NW, SMALL>), dim3(grid), dim3(WAVE), lds, stream, a,
                       a.path == EVAL_PATH_GLOBAL ? 1 : 0, total);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

size_t sweep_lds_need(int max_n, int max_e) {
  const int nw = (max_n + 63) / 64;
  return lds_layout(max_n, max_e, nw <= 1 ? 1 : nw <= 2 ? 2 : nw <= 4 ? 4 : 8, false).total;
}

hipError_t launch_sweep(const SweepArgs& a, hipStream_t stream) {
  if (a.D <= 0) return hipSuccess;
  const bool small = a.small_loads != 0;
  if (a.max_n <= 64) return small ? launch_nw<1, true>(a, stream) : launch_nw<1, false>(a, stream);
  if (a.max_n <= 128) return small ? launch_nw<2, true>(a, stream) : launch_nw<2, false>(a, stream);
  if (a.max_n <= 256) return small ? launch_nw<4, true>(a, stream) : launch_nw<4, false>(a, stream);
  if (a.max_n <= 512) return small ? launch_nw<8, true>(a, stream) : launch_nw<8, false>(a, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_best_final(const unsigned long long* best, int32_t D, int32_t* idx, int64_t* bound,
                             const int32_t* list, int32_t K, hipStream_t stream) {
  if (D <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best_final, dim3((D + 255) / 256), dim3(256), 0, stream, best, D, idx, bound, list,
                     K);
  return hipGetLastError();
}

}  // namespace dagbound
