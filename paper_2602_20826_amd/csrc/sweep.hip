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
//   - candidate bytes: explicit ones read from the lane's own row in device
//     memory where they are used; seeded ones drawn from the counter hash
//     (into LDS as [node][lane] bytes for DAGs of up to 128 nodes).
// Releases use per-candidate counters of unfinished predecessors, packed in
// LDS dwords [node][lane].  All arithmetic is integer.
#include "internal.h"

namespace dagbound {
namespace {

constexpr int WAVE = 64;

// Word v / 64 of a bitset held in registers; a masked OR rather than an
// indexed read keeps the array in registers.
template <int NW>
__device__ inline uint64_t word_of(const uint64_t (&b)[NW], int v) {
  if constexpr (NW == 1) return b[0];
  uint64_t w = 0;
  const int q = v >> 6;
#pragma unroll
  for (int k = 0; k < NW; k++) w |= b[k] & (0ull - (uint64_t)(q == k));
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
// The same with a wave-uniform index: the word is addressed directly (GPR
// indexing) instead of through a select over every word.
template <int NW>
__device__ inline bool bit_get_u(const uint64_t (&b)[NW], int v) {
  const int u = __builtin_amdgcn_readfirstlane(v);
  if constexpr (NW == 1) return (b[0] >> (u & 63)) & 1;
  return (b[u >> 6] >> (u & 63)) & 1;
}
template <int NW>
__device__ inline void bit_set_u(uint64_t (&b)[NW], int v) {
  const int u = __builtin_amdgcn_readfirstlane(v);
  if constexpr (NW == 1) b[0] |= 1ull << (u & 63);
  else b[u >> 6] |= 1ull << (u & 63);
}
// Index of the lowest set bit (or -1), cleared in place.
template <int NW>
__device__ inline int pop_first(uint64_t (&b)[NW]) {
  if constexpr (NW == 1) {
    const uint64_t w = b[0];
    b[0] = w & (w - 1);
    return w ? (int)__builtin_ctzll(w) : -1;
  } else if constexpr (NW == 2) {
    const bool lo = b[0] != 0;
    const uint64_t w = lo ? b[0] : b[1];
    const uint64_t w2 = w & (w - 1);
    if (lo) b[0] = w2;
    else b[1] = w2;
    return w ? (lo ? 0 : 64) + (int)__builtin_ctzll(w) : -1;
  }
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
// Pops the set bits of a bitset in increasing order through a cursor word,
// so a pop touches one word; the bitset itself is updated by rest().
template <int NW>
struct Popper {
  uint64_t cw;
  int kw;
  __device__ void init(const uint64_t (&b)[NW]) { kw = 0; cw = b[0]; }
  __device__ int pop(const uint64_t (&b)[NW]) {
    while (cw == 0) {
      if (++kw >= NW) { kw = NW; return -1; }
      cw = word_of<NW>(b, kw * 64);
    }
    const int r = kw * 64 + (int)__builtin_ctzll(cw);
    cw &= cw - 1;
    return r;
  }
  // leaves in b the bits not popped yet
  __device__ void rest(uint64_t (&b)[NW]) const {
#pragma unroll
    for (int k = 0; k < NW; k++) b[k] = k < kw ? 0ull : (k == kw ? cw : b[k]);
  }
};
// Index of the highest set bit, or -1.
template <int NW>
__device__ inline int bit_last(const uint64_t (&b)[NW]) {
  int r = -1;
#pragma unroll
  for (int k = 0; k < NW; k++) r = b[k] ? k * 64 + 63 - __builtin_clzll(b[k]) : r;
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
// (a & ~b) | c in one instruction per dword; OR-accumulates the bits of a
// row r outside a set f into o.
__device__ inline uint32_t andn_or(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xBA);
}
__device__ inline uint32_t outside(uint64_t r, uint64_t f, uint32_t o) {
  o = andn_or((uint32_t)r, (uint32_t)f, o);
  return andn_or((uint32_t)(r >> 32), (uint32_t)(f >> 32), o);
}
__device__ inline uint64_t readlane64(uint64_t x, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
}

// ceil(a / b) for 1 <= a < 2^20 and 1 <= b < 2^16, exactly: with a - 1 =
// q b + r, (a - 1/2) / b lies in [q + 1/(2b), q + 1 - 1/(2b)], and the
// single-precision product (a - 1/2) * rcp(b) (reciprocal within one ulp) is
// off by less than a * 2^-22.4 / b < 1/(5b), so it truncates to q.
__device__ inline uint32_t ceil_div_small(uint32_t a, uint32_t b) {
  return (uint32_t)(((float)a - 0.5f) * __builtin_amdgcn_rcpf((float)b)) + 1u;
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

// With the candidate bytes out of LDS (RS), the residual-slot map of DAGs
// above 128 nodes lives in a global-memory region of the workgroup instead
// of LDS, which keeps the workgroup's LDS small enough for several waves per
// compute unit.
template <int NW, bool RS> struct MapInGlobal { static constexpr bool value = NW >= 4 && RS; };
// 64-bit words of one workgroup's region (the map) for DAGs of up to max_n
// nodes.
__host__ __device__ inline size_t row_region_words(int max_n, int nw, bool rs) {
  return nw >= 4 && rs ? 4 * ((size_t)max_n + 7) : 0;
}

// LDS layout of one wavefront (bytes), for the batch's largest DAG.
struct Lds {
  size_t mem, node, ppv, inv, res, r, map, stage, uni, total;
};
__host__ __device__ inline Lds lds_layout(int maxn, int nw, bool big, bool rs) {
  Lds l;
  size_t o = 0;
  // members in group order, sigma | last << 15 (above 256 nodes: device memory)
  l.mem = o;  o += nw == 8 ? 0 : ((size_t)maxn * 2 + 15) & ~(size_t)15;
  l.node = o; o += (size_t)maxn * 8;            // node info by sigma rank
  const size_t idb = ((size_t)maxn * 2 + 15) & ~(size_t)15;
  if (big) {
    l.ppv = o;  o += idb;                       // min(p, M) by local id
    l.inv = o;  o += idb;                       // sigma rank by local id
    l.res = o;
  } else {
    // the two id tables serve the set-up only, before the residual table
    // is first written: they share its space (12 * 64 words hold 2 * 512
    // ids, 10 * 64 words the 2 * 128 of DAGs up to 128 nodes)
    l.res = o;  o += (size_t)res_slots_of(nw) * WAVE * 4;  // residual table [slot][lane]
    l.ppv = l.res;
    l.inv = l.res + idb;
    static_assert(RES_SLOTS * WAVE * 4 >= 2 * 512 * 2 && RES_SLOTS_SMALL * WAVE * 4 >= 2 * 128 * 2,
                  "id tables fit in the residual table");
  }
  l.r = o;    o += rs ? 0 : (size_t)maxn * WAVE;  // candidate bytes [sigma][lane] (none when drawn on the fly)
  l.map = o;  o += (big || (nw >= 4 && rs)) ? 0 : (size_t)((maxn + 7) / 8) * WAVE * 4;  // residual slot of a node, 4 bits
  o = (o + 15) & ~(size_t)15;
  l.stage = o; o += nw <= 2 ? 0 : (size_t)WAVE * nw * 8;  // predecessor rows of release candidates [lane][nw]
                                                          // (rows of DAGs up to 128 nodes stay in registers)
  l.uni = o;  o += nw <= 2 ? 0 : (size_t)2 * nw * 8;     // wave-uniform sets above 128 nodes: FO, members
  l.total = (o + 15) & ~(size_t)15;
  return l;
}

// Eq. 5's half-up share floor((2 cv M + W) / (2 W)) for loads below 2^20
// and M below 2^12: cv M < 2^32 and W < 2^29 then.  A float estimate from
// the slot's reciprocal of 2W is within one of the quotient; the remainder
// 2 cv M + W - 2 W q then lies in [-2W, 4W), inside the signed 32-bit range,
// so wrapping 32-bit arithmetic gives it exactly and one signed test
// corrects the estimate.
__device__ inline uint32_t round_share_small(uint32_t cv, uint32_t M, uint32_t W, float rw2) {
  const uint32_t num = __umul24(2u * cv, M) + W;  // modulo 2^32
  const uint32_t den = 2u * W;
  uint32_t q = (uint32_t)(__builtin_fmaf(2.0f * (float)cv, (float)M, (float)W) * rw2);
  const int32_t r = (int32_t)(num - q * den);
  if (r < 0) q--;
  else if (r >= (int32_t)den) q++;
  return q;
}

// One (DAG, 64-candidate tile).  Returns true if a lane's residual table
// overflowed (nothing was written; the tile must be redone by the
// global-table pass).  LM: the launching loop's reading, spatial (0) or
// temporal (1); 2 is the spatial reading of a conditional DAG, where lane
// (list position) p evaluates realization p mod a.cond_R of its candidate:
// the same schedule, and each slot's response over its executed parts.
template <int NW, bool BIG, bool SMALL, bool RS, int LM>
__device__ bool eval_tile(const SweepArgs& a, int item, unsigned char* smem, uint32_t* gres, uint64_t* grows) {
  constexpr bool TP = LM == 1;
  constexpr bool CD = LM == 2;
  const int ntile = (a.K + WAVE - 1) / WAVE;
  const int li = item / ntile;
  const int tile = item - li * ntile;
  const int d = a.dag_list ? a.dag_list[li] : li;
  const int lane = threadIdx.x;
  const int slot = tile * WAVE + lane;  // output position
  const bool active = slot < a.K;
  const int c = a.cand_list ? (active ? a.cand_list[(int64_t)d * a.K + slot] : 0) : slot;  // candidate id
  const int64_t n0 = a.t.node_off[d];
  const int N = (int)uni((uint32_t)(a.t.node_off[d + 1] - n0));
  const uint32_t M = (uint32_t)a.M;
  const bool mpow2 = (M & (M - 1u)) == 0u;  // division by M as a shift
  const uint32_t msh = (uint32_t)__builtin_ctz(M);
  const Lds L = lds_layout(a.max_n, NW, BIG, RS);
  uint16_t* s_mem = (uint16_t*)(smem + L.mem); // sigma | last << 15, in group order
  uint2* s_node = (uint2*)(smem + L.node);     // {C_hat, pp | local id << 16} by sigma rank
  uint16_t* s_ppv = (uint16_t*)(smem + L.ppv); // [local id]
  uint16_t* s_inv = (uint16_t*)(smem + L.inv); // [local id]
  uint32_t* res = BIG ? gres : (uint32_t*)(smem + L.res);  // [slot][lane], or [sigma][lane] when BIG
  uint8_t* s_r = smem + L.r;                   // [sigma][lane]
  uint32_t* s_map = MapInGlobal<NW, RS>::value ? (uint32_t*)grows
                                               : (uint32_t*)(smem + L.map); // [sigma / 8][lane], 4 bits per node: slot + 1

  // ---- DAG tables (shared by the 64 candidates)
  for (int s = lane; s < N; s += WAVE) s_node[s] = make_uint2(a.t.wc[n0 + s], a.t.pp[n0 + s]);
  for (int v = lane; v < N; v += WAVE) s_inv[v] = a.t.inv[n0 + v];
  __syncthreads();
  for (int v = lane; v < N; v += WAVE) {
    const int s = s_inv[v];
    const uint32_t y = s_node[s].y;
    s_ppv[v] = (uint16_t)y;
    s_node[s].y = y | ((uint32_t)v << 16);
  }
  // Member records in group order.  Above 256 nodes (GREC) they are read
  // from the batch's member records in device memory, the next group's
  // first 64 one group ahead, which leaves their LDS to more wavefronts;
  // smaller DAGs keep only the group order (sigma ranks) in LDS and take
  // the rest of a record from the node table.
  constexpr bool GREC = NW == 8;
  const uint4* mrec = GREC ? a.t.mrec + n0 : nullptr;
  auto mem_rec = [&](int i) -> uint2 {
    if constexpr (GREC) {
      const uint4 r = mrec[i];
      return make_uint2(r.x, r.y);
    } else {
      // {C_hat, pp | s << 16 | last << 31} from the node's record
      const uint32_t g = s_mem[i];
      const uint2 nd = s_node[g & 0x7FFFu];
      return make_uint2(nd.x, (nd.y & 0xFFFFu) | ((g & 0x7FFFu) << 16) | ((g & 0x8000u) << 16));
    }
  };
  if (!GREC) {
    for (int k = lane; k < N; k += WAVE) s_mem[k] = a.t.gl[n0 + k];
  }
  __syncthreads();
  // Predecessor and successor rows of the DAG's nodes (NW words each, by
  // sigma rank) come from the batch's adjacency rows.
  const uint64_t* prow_v = a.t.adj + (size_t)a.t.adj_node * (size_t)n0;
  const uint64_t* srow_v = prow_v + (size_t)N * NW;
  uint64_t* s_stage = (uint64_t*)(smem + L.stage);  // [lane][NW] rows of the release candidates
  // released: the sources; finished: none.  Predecessor rows of DAGs up to
  // 128 nodes stay in registers (REG): lane x keeps those of nodes w * 64 + x.
  constexpr bool REG = NW <= 2;
  uint64_t rel[NW], fin[NW], seg[NW];
  uint64_t PB[REG ? NW : 1][REG ? NW : 1];
#pragma unroll
  for (int w = 0; w < NW; w++) {
    const int u = w * WAVE + lane;
    rel[w] = __ballot(u < N && a.t.indeg[n0 + u] == 0);
    fin[w] = 0;
    seg[w] = 0;
    if constexpr (REG) {
#pragma unroll
      for (int k2 = 0; k2 < NW; k2++) {
        PB[w][k2] = u < N ? prow_v[(size_t)u * NW + k2] : 0ull;
      }
    }
  }
  if (!BIG) {
    for (int i = 0; i < (N + 7) / 8; i++) s_map[i * WAVE + lane] = 0;
  }
  uint32_t freem = (1u << min(a.res_slots, res_slots_of(NW))) - 1u;  // free residual slots
  // ---- candidate bytes of this lane, by sigma rank.  Candidate 0 is the
  // paper's own rule (all zero); lanes past K run zeros and store nothing.
  // With RS the bytes stay out of LDS: seeded bytes are drawn where they are
  // used (r_of), explicit ones (XB) are read from the lane's row in device
  // memory one use ahead (the row's bytes stay in the caches: each lane's
  // row is N bytes).
  const bool rlive = c > 0 && active;
  const bool XB = RS && a.alloc != nullptr;
  const uint64_t rkey = a.alloc ? 0ull : mix64(a.seed ^ mix64((uint64_t)d * 0x9E3779B97F4A7C15ull));
  auto r_of = [&](uint32_t v, uint32_t pp) -> uint32_t {
    const uint64_t word = mix64(rkey ^ (((uint64_t)c << 32) | (uint64_t)(v >> 2)));
    const uint32_t h16 = (uint32_t)(word >> (16 * (v & 3))) & 0xFFFFu;
    return rlive ? 1u + ((h16 * min(pp, 255u)) >> 16) : 0u;
  };
  // the lane's explicit row (lanes of candidate 0 or past K read row 0 and
  // use zero)
  const uint8_t* xrow = XB ? a.alloc + (int64_t)a.kalloc * n0 + (int64_t)(rlive ? c : 0) * N : nullptr;
  if (RS) {
  } else if (a.alloc) {
    if (c > 0 && active) {
      // 16-byte aligned loads over the lane's row; an aligned chunk holding a
      // byte of the row never leaves that byte's page.
      const uint8_t* row = a.alloc + (int64_t)a.kalloc * n0 + (int64_t)c * N;
      const uintptr_t rb = (uintptr_t)row;
      const uintptr_t p0 = rb & ~(uintptr_t)15;
      const uintptr_t pe = rb + (uintptr_t)N;
      for (uintptr_t p = p0; p < pe; p += 16) {
        const uint4 q = *(const uint4*)p;
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 16; j++) {
          const int64_t idx = (int64_t)(p + j) - (int64_t)rb;
          if (idx >= 0 && idx < N) s_r[s_inv[idx] * WAVE + lane] = (uint8_t)(w4[j >> 2] >> (8 * (j & 3)));
        }
      }
    } else {
      for (int v = 0; v < N; v++) s_r[v * WAVE + lane] = 0;
    }
  } else {
    uint64_t word = 0;
    for (int v = 0; v < N; v++) {
      if ((v & 3) == 0) word = mix64(rkey ^ (((uint64_t)c << 32) | (uint64_t)(v >> 2)));
      const uint32_t range = min((uint32_t)s_ppv[v], 255u);
      const uint32_t h16 = (uint32_t)(word >> (16 * (v & 3))) & 0xFFFFu;
      const uint32_t r = 1u + ((h16 * range) >> 16);
      s_r[s_inv[v] * WAVE + lane] = (c > 0 && active) ? (uint8_t)r : (uint8_t)0;
    }
  }
  __syncthreads();

  // Conditional DAGs: the nodes of this lane's realization that execute.
  uint64_t xm[NW];
  if constexpr (CD) {
#pragma unroll
    for (int w = 0; w < NW; w++) xm[w] = 0;
    const uint32_t rho = active ? (uint32_t)(slot % a.cond_R) : 0u;
    for (int s = 0; s < N; s++) {
      const uint32_t t = a.cond_tab[n0 + s];
      const uint32_t nb = (t >> 13) & 255u;
      const bool ex = nb == 0 || (rho / (t & 0x1FFFu)) % nb == (t >> 21);
      if (ex) bit_set_u<NW>(xm, s);
    }
  }

  // Remaining load of a segmented node.
  auto res_at = [&](int s) -> uint32_t* {
    if (BIG) return &res[s * WAVE + lane];
    const uint32_t sl = ((s_map[(s >> 3) * WAVE + lane] >> (4 * (s & 7))) & 15u) - 1u;
    return &res[sl * WAVE + lane];
  };

  // ---- per-candidate sweep (Algorithm 2 and Theorem 1).  rel: released
  // and unfinished (Algorithm 2's Released_nodes); fin: finished; seg:
  // segmented and unfinished, remaining load in the residual table.
  uint64_t bound = 0, cp = 0;
  uint64_t xbound = 0, xcp = 0;  // conditional: the realization's bound and maxC terms
  bool ovf = false;
  // FO: nodes finished in some lane (wave-uniform).  Above 128 nodes FO and
  // the group's member set wait in LDS while they are not needed, which
  // leaves their registers to the walk and the release.
  constexpr bool ULDS = NW >= 4;
  uint64_t FO[ULDS ? 1 : NW];
  uint64_t* s_uni = (uint64_t*)(smem + L.uni);  // [0, NW): FO, [NW, 2 NW): members
  if constexpr (ULDS) {
    if (lane < NW) s_uni[lane] = 0;
  } else {
#pragma unroll
    for (int w = 0; w < NW; w++) FO[w] = 0;
  }
  int k = 0;
  uint2 nxt = make_uint2(0u, 0u);
  if (GREC && lane < N) nxt = mem_rec(lane);
  while (k < N) {
    // The group's extent from the members' end marks, 64 records at a time;
    // the first 64 records stay in registers (lane i holds member k + i).
    uint2 rec0 = make_uint2(0u, 0u);
    if (GREC) rec0 = nxt;
    else if (k + lane < N) rec0 = mem_rec(k + lane);
    int kend;
    {
      const uint64_t ends = __ballot(k + lane < N && (rec0.y >> 31));
      if (ends) {
        kend = k + 1 + __builtin_ctzll(ends);
      } else {
        kend = k + WAVE;
        while (kend < N) {
          const bool e = kend + lane < N && (mem_rec(kend + lane).y >> 31);
          const uint64_t m = __ballot(e);
          if (m) { kend += 1 + __builtin_ctzll(m); break; }
          kend += WAVE;
        }
        kend = min(kend, N);
      }
    }
    if (GREC) {
      nxt = make_uint2(0u, 0u);
      if (kend + lane < N) nxt = mem_rec(kend + lane);
    }
    // Pass 1: member set and W(pi_j), the remaining load of the members
    // unfinished in this lane (Eq. 5).
    uint64_t gm[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) gm[w] = 0;
    uint64_t W = 0;
    uint32_t W32 = 0;  // loads below 2^20: up to 512 of them sum below 2^29
    for (int base = k; base < kend; base += WAVE) {
      uint2 rec = rec0;
      if (base != k && base + lane < kend) rec = mem_rec(base + lane);
      const int cnt = min(WAVE, kend - base);
      for (int i = 0; i < cnt; i++) {
        const int s = ((uint32_t)__builtin_amdgcn_readlane((int)rec.y, i) >> 16) & 0x7FFF;
        bit_set_u<NW>(gm, s);
        if (bit_get_u<NW>(rel, s)) {
          uint32_t cv = (uint32_t)__builtin_amdgcn_readlane((int)rec.x, i);
          if (bit_get_u<NW>(seg, s)) cv = *res_at(s);
          if (SMALL) W32 += cv;
          else W += cv;
        }
      }
    }
    if (SMALL) W = W32;
    if (!__ballot(W != 0)) { k = kend; continue; }  // every member finished earlier
    // Pass 2: parallelism of each unfinished member (Eq. 5, or the candidate
    // byte) and its execution time (Eq. 1, t_min = 1, m <= M).  The byte of
    // the next member is read one step ahead.
    const float rw2 = SMALL ? __builtin_amdgcn_rcpf((float)(2ull * W)) : 0.0f;
    uint32_t maxC = 0, sm = 0;
    uint32_t xmaxC = 0, xsm = 0;  // conditional: over the slot's executed parts
    uint64_t xA = 0;
    // with loads below 2^20, m C < load + m < 2^21 per member and the sums
    // of up to 512 members stay below 2^30: 32-bit arithmetic
    uint64_t A = 0;
    uint32_t A32 = 0;
    for (int base = k; base < kend; base += WAVE) {
      uint2 rec = rec0;
      if (base != k && base + lane < kend) rec = mem_rec(base + lane);
      const int cnt = min(WAVE, kend - base);
      uint32_t rnext = 0, recv = 0;
      if (RS) {  // local ids of the chunk's members
        if (base + lane < kend) recv = s_node[(rec.y >> 16) & 0x7FFF].y >> 16;
        if (XB) rnext = xrow[(uint32_t)__builtin_amdgcn_readlane((int)recv, 0)];
      } else {
        rnext = s_r[(((uint32_t)__builtin_amdgcn_readlane((int)rec.y, 0) >> 16) & 0x7FFF) * WAVE + lane];
      }
      for (int i = 0; i < cnt; i++) {
        const int s = ((uint32_t)__builtin_amdgcn_readlane((int)rec.y, i) >> 16) & 0x7FFF;
        uint32_t rv = rnext;
        if (XB) {
          rv = rlive ? rnext : 0u;
          if (i + 1 < cnt) rnext = xrow[(uint32_t)__builtin_amdgcn_readlane((int)recv, i + 1)];
        } else if (RS) {
          rv = r_of((uint32_t)__builtin_amdgcn_readlane((int)recv, i),
                    (uint32_t)__builtin_amdgcn_readlane((int)rec.y, i) & 0xFFFFu);
        } else if (i + 1 < cnt) {
          rnext = s_r[(((uint32_t)__builtin_amdgcn_readlane((int)rec.y, i + 1) >> 16) & 0x7FFF) * WAVE + lane];
        }
        if (!bit_get_u<NW>(rel, s)) continue;
        uint32_t cv = (uint32_t)__builtin_amdgcn_readlane((int)rec.x, i);
        if (bit_get_u<NW>(seg, s)) {
          // a segmented member: its remaining load, and its residual slot
          // is free again (the member finishes in this slot)
          if (BIG) {
            cv = res[s * WAVE + lane];
          } else {
            const uint32_t sl = ((s_map[(s >> 3) * WAVE + lane] >> (4 * (s & 7))) & 15u) - 1u;
            cv = res[sl * WAVE + lane];
            freem |= 1u << sl;
          }
        }
        const uint32_t mx = min((uint32_t)__builtin_amdgcn_readlane((int)rec.y, i) & 0xFFFFu, cv);
        uint32_t m;
        if (rv) m = min(rv, mx);
        else m = max(1u, min(mx, SMALL ? round_share_small(cv, M, W32, rw2) : round_share(cv, M, W)));
        const uint32_t C = ceil_div<SMALL>(cv, m);
        maxC = max(maxC, C);
        sm += m;
        if (SMALL) A32 += __umul24(m, C);
        else A += (uint64_t)m * C;
        if (CD && bit_get_u<NW>(xm, s)) {
          xmaxC = max(xmaxC, C);
          xsm += m;
          xA += (uint64_t)m * C;
        }
      }
    }
    // Eqs. 6-7: parallel nodes (released, outside the group) take the S spare
    // compute units, largest W^anc first; a node that does not fit in
    // maxC * m is segmented there and the launching stops.  Each lane walks
    // its own parallel set; the next node's data are read one step ahead.
    // The nodes taken from Q and not segmented are the ones launched whole.
    uint32_t S = (W != 0 && sm < M) ? M - sm : 0u;
    uint64_t Q[NW], Lw[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) Q[w] = rel[w] & ~gm[w];
    if constexpr (ULDS) {
      if (lane == 0) {
#pragma unroll
        for (int w = 0; w < NW; w++) s_uni[NW + w] = gm[w];
      }
    }
    int cseg = -1;
    bool csg = false;
    uint32_t cleft = 0;
    constexpr bool CURSOR = NW >= 4;
    Popper<NW> pq;
    pq.init(Q);
    int cn = S ? (CURSOR ? pq.pop(Q) : pop_first<NW>(Q)) : -1;
    int ci = max(cn, 0);
    uint2 nd = s_node[ci];
    uint32_t rc = RS ? (XB ? (uint32_t)xrow[nd.y >> 16] : 0u) : s_r[ci * WAVE + lane];
    uint32_t mw = BIG ? 0u : s_map[(ci >> 3) * WAVE + lane];
    bool go = cn >= 0;
    const bool walked = go;
    // temporal reading: S stays for every node, the launched nodes run one
    // after another and spend the slot's time maxC
    uint32_t T = maxC;
    while (go) {
      const int cur = cn;
      const uint2 ndc = nd;
      const uint32_t rcc = XB ? (rlive ? rc : 0u) : RS ? r_of(ndc.y >> 16, ndc.y & 0xFFFFu) : rc, mwc = mw;
      // remaining load of cur: read before the next node's data, so that
      // waiting for it leaves those reads in flight
      bool sg;
      uint32_t cc = ndc.x;
      uint32_t nib = 0;
      if (BIG) {
        sg = bit_get<NW>(seg, cur);
        if (sg) cc = res[cur * WAVE + lane];
      } else {
        nib = (mwc >> (4 * (cur & 7))) & 15u;
        sg = nib != 0;
        const uint32_t rv = res[(sg ? nib - 1u : 0u) * WAVE + lane];
        cc = sg ? rv : cc;
      }
      cn = CURSOR ? pq.pop(Q) : pop_first<NW>(Q);
      ci = max(cn, 0);
      nd = s_node[ci];
      if (!RS) rc = s_r[ci * WAVE + lane];
      else if (XB) rc = xrow[nd.y >> 16];
      if (!BIG) mw = s_map[(ci >> 3) * WAVE + lane];
      const uint32_t mx = min(ndc.y & 0xFFFFu, cc);
      const uint32_t mc = min(rcc ? min(rcc, mx) : mx, S);
      // capacity (time left) * m; with loads below 2^20 and M below 2^12 the
      // product stays below 2^32.  Below the load it is exact in 32 bits.
      const uint32_t tl = TP ? T : maxC;
      uint32_t cap32;
      bool fits;
      if (SMALL) {
        cap32 = __umul24(tl, mc);
        fits = cc <= cap32;
      } else {
        const uint64_t cap = (uint64_t)tl * mc;
        fits = (uint64_t)cc <= cap;
        cap32 = (uint32_t)cap;
      }
      if (!fits) {
        cseg = cur;
        csg = sg;
        cleft = cc - cap32;
      } else if (!BIG && sg) {
        freem |= 1u << (nib - 1u);  // a segmented node launched whole: its slot is free again
      }
      if (CD && bit_get<NW>(xm, cur)) {
        // launched whole (C = ceil(load / m)) or as a segment (C = maxC)
        const uint32_t Cp = fits ? ceil_div<SMALL>(cc, mc) : maxC;
        xmaxC = max(xmaxC, Cp);
        xsm += mc;
        xA += (uint64_t)mc * Cp;
      }
      if (TP) {
        T -= fits ? ceil_div<SMALL>(cc, mc) : 0u;
        go = fits && T != 0 && cn >= 0;
      } else {
        S -= fits ? mc : 0u;
        go = fits && S != 0 && cn >= 0;
      }
    }
    // Launched whole: the nodes of Q before the first one not launched
    // whole (the segmented one, else the one read ahead), or all of Q when
    // the walk ran out of nodes.
    {
      const int stop = cseg >= 0 ? cseg : (cn >= 0 ? cn : (walked ? NW * WAVE : 0));
#pragma unroll
      for (int w = 0; w < NW; w++) {
        const int t = min(max(stop - w * WAVE, 0), WAVE);
        Lw[w] = rel[w] & ~(ULDS ? s_uni[NW + w] : gm[w]) & (t ? ~0ull >> (WAVE - t) : 0ull);
      }
    }
    if (cseg >= 0) {
      if (csg) {
        *res_at(cseg) = cleft;
      } else if (BIG) {
        res[cseg * WAVE + lane] = cleft;
        bit_set<NW>(seg, cseg);
      } else if (freem == 0) {
        ovf = true;
      } else {
        const uint32_t sl = (uint32_t)__builtin_ctz(freem);
        freem &= freem - 1u;
        res[sl * WAVE + lane] = cleft;
        uint32_t* mp = &s_map[(cseg >> 3) * WAVE + lane];
        const int sh = 4 * (cseg & 7);
        *mp = (*mp & ~(15u << sh)) | ((sl + 1u) << sh);
        bit_set<NW>(seg, cseg);
      }
    }
    // Lemma 1, plus the list-scheduling term if the members oversubscribe.
    if (W != 0) {
      uint64_t R = maxC;
      if (sm > M) R += SMALL ? (uint64_t)(mpow2 ? (A32 - maxC) >> msh : (A32 - maxC) / M) : (A - maxC) / M;
      bound += R;
      cp += maxC;
      if (CD) {
        uint64_t xR = xmaxC;
        if (xsm > M) xR += (xA - xmaxC) / M;
        xbound += xR;
        xcp += xmaxC;
      }
    }
    // Finished now: the unfinished members and the nodes launched whole.
    uint64_t Dn[NW], Fu[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) {
      const uint64_t g = ULDS ? s_uni[NW + w] : gm[w];
      Dn[w] = (rel[w] & g) | Lw[w];
      seg[w] &= ~Dn[w];
      rel[w] &= ~Dn[w];
      fin[w] |= Dn[w];
      Fu[w] = g | (__ballot(Lw[w] != 0) ? wave_or64(Lw[w]) : 0ull);  // finished now in some lane
    }
    // Releases: a successor of a node finished now (in some lane) is
    // released in the lanes where all its predecessors have finished.
    // Lane-parallel over nodes (lane x takes node w * 64 + x): the successor
    // rows of the nodes finished now are OR-ed into the candidates; the
    // candidates' predecessor rows are read, and those with a predecessor
    // unfinished in every lane (outside FO, the nodes finished in some lane)
    // dropped; the rest go through LDS, from where every lane reads each
    // candidate's row (one broadcast read) and tests it against its own
    // finished set.
    {
      uint64_t cand[NW];
#pragma unroll
      for (int k2 = 0; k2 < NW; k2++)
        if (!ULDS) FO[ULDS ? 0 : k2] |= Fu[k2];
      if constexpr (ULDS) {
        if (lane == 0) {
#pragma unroll
          for (int k2 = 0; k2 < NW; k2++) s_uni[k2] |= Fu[k2];
        }
      }
      if constexpr (REG) {
        // lane x holds node w * 64 + x's predecessor row: a candidate when
        // one of its predecessors finished now in some lane
#pragma unroll
        for (int w = 0; w < NW; w++) {
          uint32_t hit = 0;
#pragma unroll
          for (int k2 = 0; k2 < NW; k2++)
            hit |= ((uint32_t)PB[w][k2] & (uint32_t)Fu[k2]) | ((uint32_t)(PB[w][k2] >> 32) & (uint32_t)(Fu[k2] >> 32));
          cand[w] = __ballot(hit != 0);
        }
      } else {
        uint64_t acc[NW];
#pragma unroll
        for (int k2 = 0; k2 < NW; k2++) acc[k2] = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
          if ((Fu[w] >> lane) & 1) {
            const uint64_t* r = srow_v + (size_t)(w * WAVE + lane) * NW;
#pragma unroll
            for (int k2 = 0; k2 < NW; k2++) acc[k2] |= r[k2];
          }
        }
#pragma unroll
        for (int k2 = 0; k2 < NW; k2++) cand[k2] = __ballot(acc[k2] != 0) ? wave_or64(acc[k2]) : 0ull;
      }
      // A node found ready is added to rel even where it has finished
      // already; rel is cut back to the unfinished nodes below.
#pragma unroll
      for (int w = 0; w < NW; w++) {
        if (cand[w] == 0) continue;
        uint64_t pr[NW];
#pragma unroll
        for (int k2 = 0; k2 < NW; k2++) pr[k2] = 0;
        if ((cand[w] >> lane) & 1) {
          const uint64_t* r = prow_v + (size_t)(w * WAVE + lane) * NW;
#pragma unroll
          for (int k2 = 0; k2 < NW; k2++) pr[k2] = REG ? PB[w][k2] : r[k2];
        }
        uint32_t open = 0;
#pragma unroll
        for (int k2 = 0; k2 < NW; k2++) open = outside(pr[k2], ULDS ? s_uni[k2] : FO[ULDS ? 0 : k2], open);
        uint64_t cw = cand[w] & ~__ballot(open != 0);
        if (!cw) continue;
        if constexpr (REG) {
          // rows in registers: broadcast from the lane holding each
          while (cw) {
            const int ul = __builtin_ctzll(cw);
            cw &= cw - 1;
            uint32_t o = 0;
#pragma unroll
            for (int k2 = 0; k2 < NW; k2++) o = outside(readlane64(PB[w][k2], ul), fin[k2], o);
            if (o == 0) rel[w] |= 1ull << ul;
          }
          continue;
        }
        if ((cw >> lane) & 1) {
#pragma unroll
          for (int k2 = 0; k2 < NW; k2++) s_stage[lane * NW + k2] = pr[k2];
        }
        __builtin_amdgcn_wave_barrier();
        while (cw) {
          const int ul = __builtin_ctzll(cw);
          cw &= cw - 1;
          uint32_t o = 0;
#pragma unroll
          for (int k2 = 0; k2 < NW; k2++) o = outside(s_stage[ul * NW + k2], fin[k2], o);
          if (o == 0) rel[w] |= 1ull << ul;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
#pragma unroll
    for (int w = 0; w < NW; w++) rel[w] &= ~fin[w];
    if (__ballot(ovf)) return true;
    k = kend;
  }

  if (CD) {
    bound = xbound;
    cp = xcp;
  }
  if (active) {
    const int64_t o = (int64_t)d * a.K + slot;
    if (a.bounds) a.bounds[o] = (int64_t)bound;
    if (a.cp) a.cp[o] = (int64_t)cp;
    if (a.intf) a.intf[o] = (int64_t)(bound - cp);
  }
  if (a.best && !CD) {
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

// First pass: one tile per workgroup, residual table in LDS.  A tile that
// overflows it restarts at once with one of the global-memory tables, or,
// when all are taken, is listed for the second pass.
template <int NW, bool SMALL, bool RS, int LM>
__device__ void first_pass_tile(const SweepArgs& a, int item, unsigned char* smem, uint32_t* counters,
                                uint32_t* list, uint64_t* grows) {
  if (eval_tile<NW, false, SMALL, RS, LM>(a, item, smem, nullptr, grows)) {
    uint32_t g = 0;
    if (threadIdx.x == 0) g = atomicAdd(&counters[1], 1u);
    g = __shfl(g, 0);
    __syncthreads();
    if (g < (uint32_t)GLOBAL_PASS_GRID) {
      eval_tile<NW, true, SMALL, RS, LM>(a, item, smem, a.gres + (size_t)g * (size_t)a.max_n * WAVE, grows);
    } else if (threadIdx.x == 0) {
      list[atomicAdd(&counters[0], 1u)] = (uint32_t)item;
    }
  }
}

// Region of workgroup `slot` (maps in global memory only).
template <int NW, bool RS>
__device__ inline uint64_t* rows_of(const SweepArgs& a, int slot) {
  return a.grows ? a.grows + (size_t)slot * row_region_words(a.max_n, NW, RS) : nullptr;
}

template <int NW, bool SMALL, bool RS, int LM>
__global__ __launch_bounds__(64) void k_eval(SweepArgs a, uint32_t* counters, uint32_t* list) {
  extern __shared__ __align__(16) unsigned char smem[];
  // maps in global memory run the persistent form only (their regions
  // are per running workgroup)
  if constexpr (!MapInGlobal<NW, RS>::value)
    first_pass_tile<NW, SMALL, RS, LM>(a, blockIdx.x, smem, counters, list, nullptr);
}

// Persistent form of the first pass: as many workgroups as fit on the device
// at once, each taking tiles from a work counter until all `total` are taken.
// Every workgroup leaves the loop when the counter passes `total`.
// At least three waves per SIMD: the eight-word-row class would otherwise
// take two (the registers it spills cost less than the lost latency hiding).
template <int NW, bool SMALL, bool RS, int LM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_eval_persistent(SweepArgs a, uint32_t* counters, uint32_t* list,
                                                        int total) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* grows = rows_of<NW, RS>(a, blockIdx.x);
  for (;;) {
    uint32_t item = 0;
    if (threadIdx.x == 0) item = atomicAdd(&counters[2], 1u);
    item = __shfl(item, 0);
    if (item >= (uint32_t)total) break;
    first_pass_tile<NW, SMALL, RS, LM>(a, (int)item, smem, counters, list, grows);
    __syncthreads();
  }
}

// Second pass: the tiles the first pass listed (or every tile when
// `direct`), residual tables in global memory sized to hold every node.
template <int NW, bool SMALL, bool RS, int LM>
__global__ __launch_bounds__(64) void k_eval_global(SweepArgs a, const uint32_t* counters, const uint32_t* list,
                                                    int direct, int total) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int count = direct ? total : (int)counters[0];
  uint32_t* gres = a.gres + (size_t)blockIdx.x * (size_t)a.max_n * WAVE;
  uint64_t* grows = rows_of<NW, RS>(a, blockIdx.x);
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int item = direct ? q : (int)list[q];
    eval_tile<NW, true, SMALL, RS, LM>(a, item, smem, gres, grows);
    __syncthreads();
  }
}

// Adjacency rows of one DAG per wavefront: lane x builds the successor row
// of node x in registers and sets x in its successors' predecessor rows in
// LDS; both go out with NW-word rows.
template <int NW>
__global__ __launch_bounds__(64) void k_adj(Tables t, const int32_t* list) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* s_pb = (uint64_t*)smem;
  const int d = list[blockIdx.x];
  const int lane = threadIdx.x;
  const int64_t n0 = t.node_off[d];
  const int N = (int)(t.node_off[d + 1] - n0);
  const int64_t e0 = t.edge_off[d];
  const uint32_t E = (uint32_t)(t.edge_off[d + 1] - e0);
  uint64_t* pb = t.adj + (size_t)t.adj_node * (size_t)n0;
  uint64_t* sb = pb + (size_t)N * NW;
  for (int i = lane; i < N * NW; i += WAVE) s_pb[i] = 0;
  __syncthreads();
  for (int x = lane; x < N; x += WAVE) {
    uint64_t row[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) row[w] = 0;
    const uint32_t ea = min(t.soff[n0 + d + x], E);
    const uint32_t eb = min(max(t.soff[n0 + d + x + 1], ea), E);
    for (uint32_t e = ea; e < eb; e++) {
      const int u = t.succ[e0 + e];
      if (u >= N) continue;
      bit_set<NW>(row, u);
      atomicOr((unsigned long long*)&s_pb[u * NW + (x >> 6)], 1ull << (x & 63));
    }
#pragma unroll
    for (int w = 0; w < NW; w++) sb[(size_t)x * NW + w] = row[w];
  }
  __syncthreads();
  for (int i = lane; i < N * NW; i += WAVE) pb[i] = s_pb[i];
}

template <int NW>
hipError_t launch_adj_nw(const Tables& t, const int32_t* list, int count, int max_n, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj<NW>, dim3(count), dim3(WAVE), (size_t)max_n * NW * 8, stream, t, list);
  return hipGetLastError();
}

__global__ void k_eval_init(unsigned long long* best, int32_t D, uint32_t* counters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D) best[i] = ~0ull;
  if (i < COUNTERS_PER_CLASS * NUM_CLASSES) counters[i] = 0;
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

template <int NW, bool SMALL, bool RS, int LM>
hipError_t launch_nw(const SweepArgs& a, uint32_t* counters, uint32_t* list, hipStream_t stream) {
  const int ntile = (a.K + WAVE - 1) / WAVE;
  const int total = a.list_len * ntile;
  hipError_t e = hipSuccess;
  if (total <= 0) return e;
  // eight-word rows read the member records of the batch (written whenever
  // it holds a DAG above 256 nodes, which such a launch implies)
  if (NW == 8 && !a.t.mrec) return hipErrorInvalidValue;
  constexpr bool GROWS = MapInGlobal<NW, RS>::value;
  // maps in global memory need a region per running workgroup: persistent only
  if (a.path != EVAL_PATH_GLOBAL && (a.persistent || GROWS)) {
    const size_t lds = lds_layout(a.max_n, NW, false, RS).total;
    const void* fn = (const void*)k_eval_persistent<NW, SMALL, RS, LM>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0, dev = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WAVE, lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int grid = max(1, min(total, max(1, per_cu) * max(1, cus)));
    if (GROWS) grid = min(grid, ROW_REGIONS);
    hipLaunchKernelGGL((k_eval_persistent<NW, SMALL, RS, LM>), dim3(grid), dim3(WAVE), lds, stream, a, counters, list,
                       total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else if (a.path != EVAL_PATH_GLOBAL) {
    const size_t lds = lds_layout(a.max_n, NW, false, RS).total;
    e = hipFuncSetAttribute((const void*)k_eval<NW, SMALL, RS, LM>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_eval<NW, SMALL, RS, LM>), dim3(total), dim3(WAVE), lds, stream, a, counters, list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const size_t lds = lds_layout(a.max_n, NW, true, RS).total;
  e = hipFuncSetAttribute((const void*)k_eval_global<NW, SMALL, RS, LM>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = a.path == EVAL_PATH_GLOBAL ? min(total, GLOBAL_PASS_GRID) : GLOBAL_PASS_GRID;
  hipLaunchKernelGGL((k_eval_global<NW, SMALL, RS, LM>), dim3(grid), dim3(WAVE), lds, stream, a, counters, list,
                     a.path == EVAL_PATH_GLOBAL ? 1 : 0, total);
  return hipGetLastError();
}

// Explicit candidate bytes stay out of LDS (each lane reads its row from
// device memory one use ahead), which keeps more wavefronts per compute
// unit; seeded bytes of DAGs above 128 nodes are drawn where they are used,
// smaller DAGs' seeded bytes are drawn once into LDS.
template <bool SMALL, int LM>
hipError_t launch_class_tp(int cls, const SweepArgs& a, uint32_t* counters, uint32_t* list, hipStream_t stream) {
  switch (cls) {
    case 0: return a.alloc ? launch_nw<1, SMALL, true, LM>(a, counters, list, stream)
                           : launch_nw<1, SMALL, false, LM>(a, counters, list, stream);
    case 1: return a.alloc ? launch_nw<2, SMALL, true, LM>(a, counters, list, stream)
                           : launch_nw<2, SMALL, false, LM>(a, counters, list, stream);
    case 2: return launch_nw<4, SMALL, true, LM>(a, counters, list, stream);
    default: return launch_nw<8, SMALL, true, LM>(a, counters, list, stream);
  }
}

// The two readings of the launching loop are separate kernels, so the
// spatial one keeps its code and registers.
template <bool SMALL>
hipError_t launch_class(int cls, const SweepArgs& a, uint32_t* counters, uint32_t* list, hipStream_t stream) {
  if (a.cond_tab) return launch_class_tp<SMALL, 2>(cls, a, counters, list, stream);
  return a.temporal ? launch_class_tp<SMALL, 1>(cls, a, counters, list, stream)
                    : launch_class_tp<SMALL, 0>(cls, a, counters, list, stream);
}

}  // namespace

hipError_t launch_adj(const Tables& t, const int32_t* order, const int32_t class_off[NUM_CLASSES + 1],
                      const int32_t class_max_n[NUM_CLASSES], int uniform_nw, hipStream_t stream) {
  hipError_t e = hipSuccess;
  for (int c = 0; c < LARGE_CLASS && e == hipSuccess; c++) {
    const int count = class_off[c + 1] - class_off[c];
    const int32_t* list = order + class_off[c];
    switch (uniform_nw ? uniform_nw : 1 << c) {
      case 1: e = launch_adj_nw<1>(t, list, count, class_max_n[c], stream); break;
      case 2: e = launch_adj_nw<2>(t, list, count, class_max_n[c], stream); break;
      case 4: e = launch_adj_nw<4>(t, list, count, class_max_n[c], stream); break;
      case 8: e = launch_adj_nw<8>(t, list, count, class_max_n[c], stream); break;
      default: e = hipErrorInvalidValue;
    }
  }
  return e;
}

size_t sweep_lds_need(int max_n, int max_e) {
  (void)max_e;
  if (class_of(max_n) == LARGE_CLASS) return eval_large_lds_bytes(max_n);
  const int nw = 1 << class_of(max_n);
  return lds_layout(max_n, nw, false, nw >= 4).total;
}

size_t sweep_rows_words(const int32_t class_max_n[NUM_CLASSES], const int32_t class_off[NUM_CLASSES + 1],
                        int32_t max_n, size_t rows_off[NUM_CLASSES + 1]) {
  size_t w = 0;
  for (int c = 0; c < NUM_CLASSES; c++) {
    rows_off[c] = w;
    if (c >= 2 && c < LARGE_CLASS && class_off[c + 1] > class_off[c])
      w += (size_t)ROW_REGIONS * row_region_words(class_max_n[c], 4 << (c - 2), true);
  }
  rows_off[NUM_CLASSES] = w;  // the one-launch mode's pool
  const int cls = class_of(max_n);
  if (cls >= 2 && cls < LARGE_CLASS) w += (size_t)ROW_REGIONS * row_region_words(max_n, 4 << (cls - 2), true);
  return w;
}

// Residual words of one class's launch: GLOBAL_PASS_GRID tables of n * 64
// words, or LARGE_SLOTS regions of n words for the large class.
static size_t gres_pool_words(int cls, int32_t n) {
  return cls == LARGE_CLASS ? (size_t)LARGE_SLOTS * (size_t)n : (size_t)GLOBAL_PASS_GRID * (size_t)n * WAVE;
}

size_t sweep_gres_words(const int32_t class_max_n[NUM_CLASSES], const int32_t class_off[NUM_CLASSES + 1],
                        int32_t max_n, size_t gres_off[NUM_CLASSES]) {
  size_t w = gres_pool_words(class_of(max_n), max_n);  // one pool for the one-launch mode
  for (int c = 0; c < NUM_CLASSES; c++) {
    gres_off[c] = w;
    if (class_off[c + 1] > class_off[c]) w += gres_pool_words(c, class_max_n[c]);
  }
  return w;
}

hipError_t launch_sweep(const SweepArgs& a, hipStream_t stream, const SweepStreams* ss) {
  if (a.D <= 0) return hipSuccess;
  if (a.max_n > LARGE_MAX_N) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eval_init, dim3((a.D + 255) / 256), dim3(256), 0, stream, a.best, a.D, a.ovf_count);
  hipError_t e = hipGetLastError();
  const int ntile = (a.K + WAVE - 1) / WAVE;
  int launched[NUM_CLASSES] = {};
  const bool fork = ss != nullptr && a.order != nullptr;
  if (e == hipSuccess && fork) e = hipEventRecord(ss->fork, stream);
  // largest DAGs first: their tiles are the longest
  for (int c = NUM_CLASSES - 1; c >= 0 && e == hipSuccess; c--) {
    SweepArgs ac = a;
    if (a.order) {
      ac.dag_list = a.order + a.class_off[c];
      ac.list_len = a.class_off[c + 1] - a.class_off[c];
      ac.max_n = a.class_max_n[c];
      ac.gres = a.gres + a.gres_off[c];
      ac.grows = a.grows ? a.grows + a.rows_off[c] : nullptr;
    } else {
      // one launch over all DAGs, sized by the largest, with the shared pool
      if (c != class_of(a.max_n)) continue;
      ac.dag_list = nullptr;
      ac.list_len = a.D;
      ac.grows = a.grows ? a.grows + a.rows_off[NUM_CLASSES] : nullptr;
    }
    if (ac.list_len <= 0) continue;
    hipStream_t sc = stream;
    if (fork) {
      sc = ss->side[c];
      e = hipStreamWaitEvent(sc, ss->fork, 0);
      if (e != hipSuccess) break;
    }
    uint32_t* counters = a.ovf_count + COUNTERS_PER_CLASS * c;
    uint32_t* list = a.ovf_list + (size_t)(a.order ? a.class_off[c] : 0) * ntile;
    if (c >= a.node_lanes_class) e = launch_eval_large(ac, counters, sc);
    else e = a.small_loads && a.M < 4096 ? launch_class<true>(c, ac, counters, list, sc)
                                         : launch_class<false>(c, ac, counters, list, sc);
    if (e == hipSuccess && fork) {
      e = hipEventRecord(ss->join[c], sc);
      launched[c] = 1;
    }
  }
  if (fork) {  // join every side stream that was forked, even after an error
    for (int c = 0; c < NUM_CLASSES; c++) {
      if (!launched[c]) continue;
      const hipError_t w = hipStreamWaitEvent(stream, ss->join[c], 0);
      if (e == hipSuccess) e = w;
    }
  }
  return e;
}

namespace {
__global__ void k_check_list(const int32_t* list, int64_t n, int32_t K, uint32_t* bad) {
  uint32_t cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    cnt += (list[i] < 0 || list[i] >= K) ? 1u : 0u;
  if (cnt) atomicAdd(bad, cnt);
}
__global__ void k_zero_word(uint32_t* w) { *w = 0u; }
}  // namespace

hipError_t launch_check_list(const int32_t* list, int64_t n, int32_t K, uint32_t* bad, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, stream, bad);
  if (n > 0) {
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_check_list, dim3((unsigned)blocks), dim3(256), 0, stream, list, n, K, bad);
  }
  return hipGetLastError();
}

namespace {
__global__ void k_cond_reduce(const int64_t* rb, const int32_t* R, int32_t D, int32_t K, int32_t Rmax,
                              int64_t* bounds, int32_t* worst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)D * K) return;
  const int d = (int)(i / K);
  const int64_t* x = rb + i * Rmax;
  int64_t best = -1;
  int32_t arg = 0;
  for (int r = 0; r < R[d]; r++)
    if (x[r] > best) { best = x[r]; arg = r; }
  bounds[i] = best < 0 ? 0 : best;
  if (worst) worst[i] = arg;
}
}  // namespace

namespace {
__global__ void k_cond_list(int32_t* list, int64_t n, int64_t L, int32_t Rmax) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    list[i] = (int32_t)((i % L) / Rmax);
}
}  // namespace

hipError_t launch_cond_list(int32_t* list, int64_t n, int64_t L, int32_t Rmax, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_cond_list, dim3((unsigned)blocks), dim3(256), 0, stream, list, n, L, Rmax);
  return hipGetLastError();
}

hipError_t launch_cond_reduce(const int64_t* rb, const int32_t* R, int32_t D, int32_t K, int32_t Rmax,
                              int64_t* bounds, int32_t* worst, hipStream_t stream) {
  const int64_t n = (int64_t)D * K;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cond_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, rb, R, D, K, Rmax, bounds,
                     worst);
  return hipGetLastError();
}

hipError_t launch_best_final(const unsigned long long* best, int32_t D, int32_t* idx, int64_t* bound,
                             const int32_t* list, int32_t K, hipStream_t stream) {
  if (D <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best_final, dim3((D + 255) / 256), dim3(256), 0, stream, best, D, idx, bound, list,
                     K);
  return hipGetLastError();
}

}  // namespace dagbound
