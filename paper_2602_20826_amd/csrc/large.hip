// DAGs above 512 nodes on gfx950.
//
// Preprocessing (k_prep_large): one workgroup per DAG (4 wavefronts up to
// 512 nodes, 16 above), each workgroup looping over DAGs from a work
// counter.  The ancestor bit-matrix
// (N x ceil(N/64) words, too large for LDS) lives in a global-memory region
// of the workgroup; the tables it writes are the ones the small-DAG kernel
// writes (prep.hip), plus the member records in group order.
//   edges      range, self-loop and duplicate checks (predecessor bits set
//              with atomics in the matrix rows), in/out degrees, CSR lists
//   closure    Kahn levels; a level's rows are the OR of their predecessors'
//              rows, which are final (Eq. 2 needs ance(v))
//   W^anc      one wavefront per node sums C_hat over its row (Eq. 2)
//   orders     sigma (descending W^anc, smaller id first) and Theta (join
//              nodes, ascending W^anc, smaller id first) by bitonic sorts in LDS
//   blocks     the first join node in Theta order whose row holds v (Eq. 3):
//              a minimum over Theta, so the Theta list is cut into chunks
//              scanned in parallel and combined with atomicMin
//   groups     Algorithm 1 runs block by block, and blocks are independent:
//              each block's groups fill the positions of its nodes in
//              (block, sigma) order, so wavefronts take blocks in parallel
//
// Evaluation (k_eval_large): one wavefront per (DAG, candidate), lanes over
// nodes, persistent over a 64-bit work counter.  Per candidate the LDS holds
// the released / segmented / member / released-in-this-slot bitsets, the
// counts of unfinished predecessors (8 or 16 bits per node) and, for
// explicit bytes, the candidate bytes by sigma rank (seeded bytes are drawn
// where they are used); residual loads of segmented nodes are in a global
// region of the wavefront.  Node data come from one 16-byte record per node
// (in sigma order for parallel nodes, in group order for members).  A slot (Algorithm 2 for one group, then Lemma 1):
// the members are one lane each (W(pi_j), Eq. 5, Eq. 1 through wave
// reductions); the parallel nodes are taken 64 at a time in sigma order and
// Eqs. 6-7 become a prefix sum: the node at prefix P_i is reached while
// P_i < S, takes min(m, S - P_i) units, and the first reached node that does
// not fit in maxC * m is segmented, which stops the launching; finished
// nodes decrement their successors' counts at once, and a count reaching
// zero releases the successor when the slot ends.  All arithmetic is integer.
#include <algorithm>
#include <climits>

#include "internal.h"

namespace dagbound {
namespace {

constexpr int WAVE = 64;
constexpr int PT_MAX = 1024;  // threads of the largest preprocessing workgroup
constexpr int ID_BITS = 13;  // local ids below 8192 in sort keys
constexpr uint64_t ID_MASK = (1ull << ID_BITS) - 1;

__device__ inline uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// DPP steps of a wave scan: row shifts within rows of 16 lanes, then row
// broadcasts; lanes without a source take `id`.  Lane 63 ends with the total.
template <int CTRL, int RM>
__device__ inline uint32_t dpp32(uint32_t x, uint32_t id) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM>
__device__ inline uint64_t dpp64(uint64_t x, uint64_t id) {
  return ((uint64_t)dpp32<CTRL, RM>((uint32_t)(x >> 32), (uint32_t)(id >> 32)) << 32) |
         dpp32<CTRL, RM>((uint32_t)x, (uint32_t)id);
}
template <class T, class Op>
__device__ inline T wave_scan(T x, T id, Op op) {
  if constexpr (sizeof(T) == 8) {
    x = op(x, dpp64<0x111, 0xf>(x, id));
    x = op(x, dpp64<0x112, 0xf>(x, id));
    x = op(x, dpp64<0x114, 0xf>(x, id));
    x = op(x, dpp64<0x118, 0xf>(x, id));
    x = op(x, dpp64<0x142, 0xa>(x, id));
    x = op(x, dpp64<0x143, 0xc>(x, id));
  } else {
    x = op(x, dpp32<0x111, 0xf>(x, id));
    x = op(x, dpp32<0x112, 0xf>(x, id));
    x = op(x, dpp32<0x114, 0xf>(x, id));
    x = op(x, dpp32<0x118, 0xf>(x, id));
    x = op(x, dpp32<0x142, 0xa>(x, id));
    x = op(x, dpp32<0x143, 0xc>(x, id));
  }
  return x;
}
__device__ inline uint32_t lane63(uint32_t x) { return (uint32_t)__builtin_amdgcn_readlane((int)x, 63); }
__device__ inline uint64_t readlane64(uint64_t x, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
}
__device__ inline uint32_t wave_incl_sum(uint32_t x) {
  return wave_scan<uint32_t>(x, 0u, [](uint32_t p, uint32_t q) { return p + q; });
}
__device__ inline uint32_t wave_sum(uint32_t x) { return lane63(wave_incl_sum(x)); }
__device__ inline uint64_t wave_sum64(uint64_t x) {
  return readlane64(wave_scan<uint64_t>(x, 0ull, [](uint64_t p, uint64_t q) { return p + q; }), 63);
}
__device__ inline uint32_t wave_max(uint32_t x) {
  return lane63(wave_scan<uint32_t>(x, 0u, [](uint32_t p, uint32_t q) { return p > q ? p : q; }));
}
__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__host__ __device__ inline int pow2_at_least(int n) {
  int p = 64;
  while (p < n) p <<= 1;
  return p;
}

// ---------------------------------------------------------------------------
// Preprocessing.

// Global scratch of one preprocessing workgroup, for DAGs of up to NL nodes
// and EL edges.
struct PrepScratch {
  uint64_t* anc;      // [NL][NW] ancestor rows (first the predecessor bits)
  uint16_t* predl;    // [EL] predecessor lists (local ids)
  uint16_t* succl;    // [EL] successor lists (local ids)
  uint32_t* predoff;  // [NL + 1]
  uint32_t* succoff;  // [NL + 1]
  uint32_t* outc;     // [NL] out-degree, then fill cursor
  uint32_t* par;      // [NL] p by local id
  uint16_t* topo;     // [NL] Kahn order; later the block segment starts
  uint16_t* perm;     // [NL] local id of each sigma rank
  int32_t* psig;      // [NL] sigma rank of the in-block parent, by sigma rank (-1: none)
  uint32_t* mmax;     // [NL] min(p, C_hat) by sigma rank
  uint32_t* blk;      // [NL] block by sigma rank
  uint16_t* blist;    // [NL] sigma ranks in (block, sigma) order
  uint32_t* segs;     // [NL] segment counts (exclusive scan)
  size_t bytes;
};
__host__ __device__ inline PrepScratch prep_scratch(unsigned char* base, int NL, int EL) {
  PrepScratch s;
  size_t o = 0;
  auto take = [&](size_t n) {
    o = (o + 255) & ~(size_t)255;
    unsigned char* p = base ? base + o : nullptr;
    o += n;
    return p;
  };
  const size_t nw = (size_t)(NL + 63) / 64;
  s.anc = (uint64_t*)take((size_t)NL * nw * 8);
  s.predl = (uint16_t*)take((size_t)EL * 2);
  s.succl = (uint16_t*)take((size_t)EL * 2);
  s.predoff = (uint32_t*)take((size_t)(NL + 1) * 4);
  s.succoff = (uint32_t*)take((size_t)(NL + 1) * 4);
  s.outc = (uint32_t*)take((size_t)NL * 4);
  s.par = (uint32_t*)take((size_t)NL * 4);
  s.topo = (uint16_t*)take((size_t)NL * 2);
  s.perm = (uint16_t*)take((size_t)NL * 2);
  s.psig = (int32_t*)take((size_t)NL * 4);
  s.mmax = (uint32_t*)take((size_t)NL * 4);
  s.blk = (uint32_t*)take((size_t)NL * 4);
  s.blist = (uint16_t*)take((size_t)NL * 2);
  s.segs = (uint32_t*)take((size_t)NL * 4);
  s.bytes = (o + 255) & ~(size_t)255;
  return s;
}

// LDS of the preprocessing workgroup (bytes), for DAGs of up to NL nodes.
struct PrepLds {
  size_t key, wcl, cnt, gflag, sel, misc, total;
};
__host__ __device__ inline PrepLds prep_lds(int NL) {
  PrepLds l;
  size_t o = 0;
  const int P = pow2_at_least(NL);
  l.key = o;   o += (size_t)P * 8;                          // sort keys
  l.wcl = o;   o += (size_t)NL * 4;                         // C_hat by local id
  l.cnt = o;   o += (size_t)NL * 4;                         // counts, cursors, blocks
  l.gflag = o; o += ((size_t)NL + 15) & ~(size_t)15;        // grouped flag by sigma rank
  l.sel = o;   o += (size_t)(PT_MAX / WAVE) * ((NL + 63) / 64) * 8;  // per-wave selection masks
  l.misc = o;  o += 64 * 4;
  l.total = o;
  return l;
}

enum { M_ERR = 0, M_ITEM, M_TAIL, M_NTH, M_NG, M_SEG, M_NSEG, M_WTOT = 16 };  // misc words

// Ascending bitonic sort of key[0, P) (P a power of two) by the workgroup.
template <int PT>
__device__ void bitonic_sort(uint64_t* key, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P / 2; i += PT) {
        const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = key[lo], b = key[hi];
        if ((a > b) == up) {
          key[lo] = b;
          key[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Exclusive prefix sums of f(0..n-1) into out[], by the workgroup; returns
// the total.  Each thread takes a run of consecutive items.
template <int PT, class F>
__device__ uint32_t block_scan(int n, F f, uint32_t* out, uint32_t* wtot) {
  constexpr int PWAVES = PT / WAVE;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int per = (n + PT - 1) / PT;
  const int i0 = tid * per, i1 = min(n, i0 + per);
  uint32_t loc = 0;
  for (int i = i0; i < i1; i++) loc += f(i);
  const uint32_t incl = wave_incl_sum(loc);
  if (lane == 63) wtot[wid] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int w = 0; w < PWAVES; w++) {
      const uint32_t x = wtot[w];
      wtot[w] = run;
      run += x;
    }
    wtot[PWAVES] = run;
  }
  __syncthreads();
  uint32_t run = wtot[wid] + incl - loc;
  for (int i = i0; i < i1; i++) {
    const uint32_t x = f(i);
    out[i] = run;
    run += x;
  }
  const uint32_t total = wtot[PWAVES];
  __syncthreads();
  return total;
}

// Algorithm 1 on one block: its nodes are blist[a, b) in sigma order.  The
// heads are the ungrouped nodes whose in-block parent is grouped (or
// absent); a step takes the first M of them in sigma order (Top_M, Rule 1),
// or, when two or more are taken and the largest m^max among them reaches
// M, only the first node of that m^max (Rule 2).  Groups fill positions
// a .. b - 1 of the group list in order.  One wavefront; returns the number
// of groups, or -1 if a step finds no head.
__device__ int group_block(const Tables& t, int64_t n0, int a, int b, int32_t M, const PrepScratch& S,
                           uint8_t* gflag, uint64_t* sel) {
  const int lane = threadIdx.x & 63;
  const int nc = (b - a + 63) >> 6;
  int gpos = a, ng = 0;
  while (gpos < b) {
    int before = 0, take = 0;
    uint32_t mxl = 0;
    for (int c = 0; c < nc; c++) {
      const int pos = a + c * 64 + lane;
      const bool in = pos < b;
      const int s = in ? S.blist[pos] : 0;
      bool head = false;
      if (in && !gflag[s]) {
        const int ps = S.psig[s];
        head = ps < 0 || gflag[ps] != 0;
      }
      const uint64_t hb = __ballot(head);
      const bool sl = head && before + __popcll(hb & lanes_below(lane)) < M;
      const uint64_t sb = __ballot(sl);
      if (lane == 0) sel[c] = sb;
      if (sl) mxl = max(mxl, S.mmax[s]);
      before += __popcll(hb);
      take += __popcll(sb);
    }
    if (take == 0) return -1;  // no head in an ungrouped block: not a forest
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t mx = wave_max(mxl);
    if (take > 1 && mx >= (uint32_t)M) {
      bool found = false;
      for (int c = 0; c < nc; c++) {
        const uint64_t sb = sel[c];
        const int pos = a + c * 64 + lane;
        const bool on = (sb >> lane) & 1;
        const uint64_t hit = __ballot(on && S.mmax[S.blist[pos]] == mx);
        uint64_t keep = 0;
        if (!found && hit) {
          keep = hit & (~hit + 1);
          found = true;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) sel[c] = keep;
      }
      take = 1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    int base = 0;
    for (int c = 0; c < nc && base < take; c++) {
      const uint64_t sb = sel[c];
      if (!sb) continue;
      if ((sb >> lane) & 1) {
        const int pos = a + c * 64 + lane;
        const int s = S.blist[pos];
        const int g = gpos + base + __popcll(sb & lanes_below(lane));
        const uint32_t last = g == gpos + take - 1 ? 0x8000u : 0u;
        t.gl[n0 + g] = (uint16_t)(s | last);
        gflag[s] = 1;
      }
      base += __popcll(sb);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    gpos += take;
    ng++;
  }
  return ng;
}

// One DAG.  Every thread of the workgroup calls it and returns together.
template <int PT>
__device__ void prep_one(const Tables& t, const PrepInputs& in, int32_t M, int d, unsigned long long* err,
                         const PrepScratch& S, unsigned char* smem, const PrepLds& L) {
  constexpr int PWAVES = PT / WAVE;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  uint64_t* key = (uint64_t*)(smem + L.key);
  uint32_t* wcl = (uint32_t*)(smem + L.wcl);
  uint32_t* cnt = (uint32_t*)(smem + L.cnt);
  uint8_t* gflag = smem + L.gflag;
  uint32_t* misc = (uint32_t*)(smem + L.misc);
  uint32_t* wtot = misc + M_WTOT;
  unsigned long long* s_sum = (unsigned long long*)(misc + 8);

  const int64_t n0 = t.node_off[d];
  const int N = (int)(t.node_off[d + 1] - n0);
  const int64_t e0 = t.edge_off[d];
  const int E = (int)(t.edge_off[d + 1] - e0);
  const int NW = (N + 63) >> 6;
  const int P = pow2_at_least(N);

  if (tid == 0) {
    misc[M_ERR] = 0;
    misc[M_TAIL] = 0;
    misc[M_NTH] = 0;
    misc[M_NG] = 0;
    misc[M_SEG] = 0;
    *s_sum = 0;
  }
  __syncthreads();

  // Task model (Section 2.1): loads and parallelism.
  unsigned long long lsum = 0;
  uint32_t wmax = 0;
  for (int v = tid; v < N; v += PT) {
    int64_t w = in.wcet[n0 + v];
    int32_t p = in.par[n0 + v];
    if (w < 1 || w > 0x7fffffffLL || p < 1) {
      atomicCAS(&misc[M_ERR], 0u, (uint32_t)PREP_E_RANGE);
      w = 1;
      p = 1;
    }
    wcl[v] = (uint32_t)w;
    S.par[v] = (uint32_t)p;
    cnt[v] = 0;
    S.outc[v] = 0;
    gflag[v] = 0;
    lsum += (unsigned long long)w;
    wmax = max(wmax, (uint32_t)w);
  }
  for (size_t i = tid; i < (size_t)N * NW; i += PT) S.anc[i] = 0;
  lsum = wave_sum64(lsum);
  wmax = wave_max(wmax);
  if (lane == 0) {
    atomicAdd(s_sum, lsum);
    if (wmax >= (1u << 20)) atomicOr(&err[1], 1ull);
  }
  __syncthreads();
  // Edges: range, self-loop, duplicates (predecessor bits in the rows).
  for (int k = tid; k < E; k += PT) {
    const int32_t u = in.src[e0 + k], v = in.dst[e0 + k];
    if (u < 0 || u >= N || v < 0 || v >= N) {
      atomicCAS(&misc[M_ERR], 0u, (uint32_t)PREP_E_RANGE);
      continue;
    }
    if (u == v) {
      atomicCAS(&misc[M_ERR], 0u, (uint32_t)PREP_E_CYCLE);
      continue;
    }
    const uint64_t bit = 1ull << (u & 63);
    const uint64_t old = atomicOr((unsigned long long*)&S.anc[(size_t)v * NW + (u >> 6)], (unsigned long long)bit);
    if (old & bit) {
      atomicCAS(&misc[M_ERR], 0u, (uint32_t)PREP_E_DUP);
      continue;
    }
    atomicAdd(&cnt[v], 1u);
    atomicAdd(&S.outc[u], 1u);
  }
  __syncthreads();
  {
    uint32_t code = misc[M_ERR];
    if (code == 0 && *s_sum >= (1ull << 40)) code = PREP_E_OVERFLOW;
    if (code) {
      if (tid == 0) atomicMin(err, ((unsigned long long)d << 8) | code);
      return;
    }
  }

  // CSR lists of predecessors and successors.
  const uint32_t ne = block_scan<PT>(N, [&](int i) { return cnt[i]; }, S.predoff, wtot);
  block_scan<PT>(N, [&](int i) { return S.outc[i]; }, S.succoff, wtot);
  if (tid == 0) {
    S.predoff[N] = ne;
    S.succoff[N] = ne;
  }
  for (int v = tid; v < N; v += PT) {
    cnt[v] = S.predoff[v];
    S.outc[v] = S.succoff[v];
  }
  __syncthreads();
  for (int k = tid; k < E; k += PT) {
    const int32_t u = in.src[e0 + k], v = in.dst[e0 + k];
    S.predl[atomicAdd(&cnt[v], 1u)] = (uint16_t)u;
    S.succl[atomicAdd(&S.outc[u], 1u)] = (uint16_t)v;
  }
  __syncthreads();
  uint32_t dmax = 0;
  for (int v = tid; v < N; v += PT) {
    const uint32_t deg = S.predoff[v + 1] - S.predoff[v];
    cnt[v] = deg;
    dmax = max(dmax, deg);
    if (deg == 0) S.topo[atomicAdd(&misc[M_TAIL], 1u)] = (uint16_t)v;
  }
  dmax = wave_max(dmax);
  if (lane == 0 && dmax >= 256) atomicOr(&err[1], 2ull);  // in-degrees need 16-bit counts
  __syncthreads();

  // Ancestor closure by Kahn levels: the rows of a level are final once
  // their predecessors' rows are, and the level's successors whose count
  // reaches zero form the next level.
  int lo = 0, hi = (int)misc[M_TAIL];
  __syncthreads();
  while (lo < hi) {
    const int cl = hi - lo;
    for (int p = tid; p < cl * NW; p += PT) {
      const int i = lo + p / NW, w = p - (p / NW) * NW;
      const int v = S.topo[i];
      uint64_t acc = S.anc[(size_t)v * NW + w];
      const uint32_t ea = S.predoff[v], eb = S.predoff[v + 1];
      uint32_t e = ea;
      for (; e + 4 <= eb; e += 4) {
        const int u0 = S.predl[e], u1 = S.predl[e + 1], u2 = S.predl[e + 2], u3 = S.predl[e + 3];
        acc |= S.anc[(size_t)u0 * NW + w] | S.anc[(size_t)u1 * NW + w] | S.anc[(size_t)u2 * NW + w] |
               S.anc[(size_t)u3 * NW + w];
      }
      for (; e < eb; e++) acc |= S.anc[(size_t)S.predl[e] * NW + w];
      S.anc[(size_t)v * NW + w] = acc;
    }
    for (int i = lo + tid; i < hi; i += PT) {
      const int v = S.topo[i];
      for (uint32_t e = S.succoff[v]; e < S.succoff[v + 1]; e++) {
        const int x = S.succl[e];
        if (atomicSub(&cnt[x], 1u) == 1u) S.topo[atomicAdd(&misc[M_TAIL], 1u)] = (uint16_t)x;
      }
    }
    __syncthreads();
    lo = hi;
    hi = (int)misc[M_TAIL];
    __syncthreads();
  }
  if (lo != N) {  // some node never became ready: a cycle
    if (tid == 0) atomicMin(err, ((unsigned long long)d << 8) | PREP_E_CYCLE);
    return;
  }

  // Eq. 2: W^anc(v) = C_hat_v + sum of C_hat over ance(v), one wavefront per
  // node; then the sigma order by sorting (2^40 - 1 - W^anc, id).
  for (int v = wid; v < N; v += PWAVES) {
    uint64_t sum = 0;
    for (int w = lane; w < NW; w += WAVE) {
      uint64_t b = S.anc[(size_t)v * NW + w];
      while (b) {
        uint32_t x[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          x[q] = 0;
          if (b) {
            x[q] = wcl[w * 64 + __builtin_ctzll(b)];
            b &= b - 1;
          }
        }
        sum += (uint64_t)x[0] + x[1] + x[2] + x[3];
      }
    }
    sum = wave_sum64(sum) + wcl[v];
    if (lane == 0) {
      t.wanc[n0 + v] = (int64_t)sum;
      key[v] = ((((1ull << 40) - 1) - sum) << ID_BITS) | (uint64_t)v;
    }
  }
  for (int v = N + tid; v < P; v += PT) key[v] = ~0ull;
  __syncthreads();
  bitonic_sort<PT>(key, P);
  for (int s = tid; s < N; s += PT) {
    const int v = (int)(key[s] & ID_MASK);
    S.perm[s] = (uint16_t)v;
    t.inv[n0 + v] = (uint16_t)s;
  }
  __syncthreads();
  // Theta: join nodes (in-degree >= 2) by ascending (W^anc, id).
  for (int v = tid; v < P; v += PT) {
    uint64_t k = ~0ull;
    if (v < N && S.predoff[v + 1] - S.predoff[v] >= 2) {
      k = ((uint64_t)t.wanc[n0 + v] << ID_BITS) | (uint64_t)v;
      atomicAdd(&misc[M_NTH], 1u);
    }
    key[v] = k;
  }
  __syncthreads();
  bitonic_sort<PT>(key, P);
  const int nth = (int)misc[M_NTH];

  // Eq. 3: the block of v is the first k (Theta order) with v in
  // ance(theta_k), else the residual block nth.  Thread (chunk, word)
  // scans its chunk of Theta in order for the bits of its word.
  for (int v = tid; v < N; v += PT) cnt[v] = (uint32_t)nth;
  __syncthreads();
  if (nth > 0) {
    const int nch = PT / NW;
    const int w = tid % NW, ch = tid / NW;
    if (ch < nch) {
      const int k0 = (int)((int64_t)nth * ch / nch), k1 = (int)((int64_t)nth * (ch + 1) / nch);
      uint64_t open = (w == NW - 1 && (N & 63)) ? ((1ull << (N & 63)) - 1) : ~0ull;
      for (int k = k0; k < k1 && open; k += 4) {
        uint64_t x[4];
#pragma unroll
        for (int q = 0; q < 4; q++)
          x[q] = k + q < k1 ? S.anc[(size_t)(key[k + q] & ID_MASK) * NW + w] : 0ull;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          uint64_t h = x[q] & open;
          open &= ~h;
          while (h) {
            atomicMin(&cnt[w * 64 + __builtin_ctzll(h)], (uint32_t)(k + q));
            h &= h - 1;
          }
        }
      }
    }
  }
  __syncthreads();
  // In-block parent: at most one predecessor in the node's own block, so a
  // block is a forest whose root-to-leaf paths are its local complete paths
  // (Eq. 4).  Tables by sigma rank for Algorithm 1.
  for (int v = tid; v < N; v += PT) {
    const uint32_t bv = cnt[v];
    int parent = -1, c = 0;
    for (uint32_t e = S.predoff[v]; e < S.predoff[v + 1]; e++) {
      const int u = S.predl[e];
      if (cnt[u] == bv) {
        parent = u;
        c++;
      }
    }
    if (c > 1) atomicCAS(&misc[M_ERR], 0u, (uint32_t)PREP_E_INTERNAL);
    const int s = t.inv[n0 + v];
    S.blk[s] = bv;
    S.psig[s] = parent < 0 ? -1 : (int)t.inv[n0 + parent];
    S.mmax[s] = min(S.par[v], wcl[v]);
  }
  __syncthreads();
  if (misc[M_ERR]) {
    if (tid == 0) atomicMin(err, ((unsigned long long)d << 8) | misc[M_ERR]);
    return;
  }

  // Algorithm 1, block by block: nodes in (block, sigma) order, one segment
  // per nonempty block, segments taken by wavefronts.
  for (int s = tid; s < P; s += PT) key[s] = s < N ? (((uint64_t)S.blk[s] << ID_BITS) | (uint64_t)s) : ~0ull;
  __syncthreads();
  bitonic_sort<PT>(key, P);
  for (int i = tid; i < N; i += PT) S.blist[i] = (uint16_t)(key[i] & ID_MASK);
  auto starts = [&](int i) -> uint32_t {
    return (i == 0 || (key[i] >> ID_BITS) != (key[i - 1] >> ID_BITS)) ? 1u : 0u;
  };
  const uint32_t nseg = block_scan<PT>(N, starts, S.segs, wtot);
  for (int i = tid; i < N; i += PT)
    if (starts(i)) S.topo[S.segs[i]] = (uint16_t)i;
  __syncthreads();
  {
    uint64_t* sel = (uint64_t*)(smem + L.sel) + (size_t)wid * NW;
    int ng = 0;
    for (;;) {
      uint32_t sg = 0;
      if (lane == 0) sg = atomicAdd(&misc[M_SEG], 1u);
      sg = uni(sg);
      if (sg >= nseg) break;
      const int a = S.topo[sg];
      const int b = sg + 1 < nseg ? (int)S.topo[sg + 1] : N;
      const int g = group_block(t, n0, a, b, M, S, gflag, sel);
      if (g < 0) {
        if (lane == 0) atomicCAS(&misc[M_ERR], 0u, (uint32_t)PREP_E_INTERNAL);
        break;
      }
      ng += g;
    }
    if (lane == 0) atomicAdd(&misc[M_NG], (uint32_t)ng);
  }
  __syncthreads();
  if (misc[M_ERR]) {
    if (tid == 0) atomicMin(err, ((unsigned long long)d << 8) | misc[M_ERR]);
    return;
  }
  if (tid == 0) t.ngroups[d] = (int32_t)misc[M_NG];

  // Tables by sigma rank, successor lists in sigma order (each list sorted,
  // so the tables do not depend on the order of the atomics above).
  for (int s = tid; s < N; s += PT) {
    const int v = S.perm[s];
    t.wc[n0 + s] = wcl[v];
    t.pp[n0 + s] = (uint16_t)min(S.par[v], (uint32_t)M);
    t.mx[n0 + s] = min(S.par[v], wcl[v]);
    t.indeg[n0 + s] = (uint16_t)(S.predoff[v + 1] - S.predoff[v]);
  }
  uint32_t* soff = t.soff + n0 + d;
  const uint32_t tot =
      block_scan<PT>(N, [&](int s) { const int v = S.perm[s]; return S.succoff[v + 1] - S.succoff[v]; }, soff, wtot);
  if (tid == 0) soff[N] = tot;
  for (int s = tid; s < N; s += PT) {
    const int u = S.perm[s];
    const uint32_t a0 = S.succoff[u], a1 = S.succoff[u + 1];
    uint16_t* out = t.succ + e0 + soff[s];
    if (a1 - a0 <= 16) {
      // up to 16 successors: loaded together and sorted in registers by a
      // bitonic network (padding above every sigma rank sorts last)
      const uint32_t deg = a1 - a0;
      uint32_t b[16];
#pragma unroll
      for (int j = 0; j < 16; j++) b[j] = (uint32_t)j < deg ? (uint32_t)t.inv[n0 + S.succl[a0 + j]] : 0xFFFFu;
#pragma unroll
      for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
          for (int i = 0; i < 16; i++) {
            const int l = i ^ j;
            if (l > i) {
              const uint32_t lo = min(b[i], b[l]), hi = max(b[i], b[l]);
              const bool up = (i & k) == 0;
              b[i] = up ? lo : hi;
              b[l] = up ? hi : lo;
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 16; j++)
        if ((uint32_t)j < deg) out[j] = (uint16_t)b[j];
    } else {
      for (uint32_t e = a0; e < a1; e++) {
        const uint16_t x = t.inv[n0 + S.succl[e]];
        uint32_t j = e - a0;
        while (j > 0 && out[j - 1] > x) {
          out[j] = out[j - 1];
          j--;
        }
        out[j] = x;
      }
    }
    if (t.nrec)
      t.nrec[n0 + s] = make_uint4(wcl[u], min(S.par[u], (uint32_t)M) | ((uint32_t)s << 16), soff[s],
                                  (uint32_t)u | ((a1 - a0) << 16));
  }
  __syncthreads();
  // member records in group order (batches with DAGs above 512 nodes)
  if (!t.mrec) return;
  for (int k = tid; k < N; k += PT) {
    const uint32_t g = t.gl[n0 + k];
    uint4 r = t.nrec[n0 + (g & 0x7FFF)];
    r.y |= (g & 0x8000u) << 16;
    t.mrec[n0 + k] = r;
  }
}

template <int PT>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(6))) void k_prep_large(
    Tables t, PrepInputs in, int32_t M, const int32_t* list, int32_t count, unsigned long long* err,
    unsigned char* scratch, int32_t NL, int32_t EL) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PrepLds L = prep_lds(NL);
  const PrepScratch S0 = prep_scratch(nullptr, NL, EL);
  const PrepScratch S = prep_scratch(scratch + (size_t)blockIdx.x * S0.bytes, NL, EL);
  uint32_t* misc = (uint32_t*)(smem + L.misc);
  for (;;) {
    if (threadIdx.x == 0) misc[M_ITEM] = (uint32_t)atomicAdd(&err[2], 1ull);
    __syncthreads();
    const uint32_t item = misc[M_ITEM];
    if (item >= (uint32_t)count) break;
    prep_one<PT>(t, in, M, list ? list[item] : (int)item, err, S, smem, L);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Evaluation.

__device__ inline uint32_t ceil_div_small(uint32_t a, uint32_t b) {
  return (uint32_t)(((float)a - 0.5f) * __builtin_amdgcn_rcpf((float)b)) + 1u;
}
template <bool SMALL>
__device__ inline uint32_t ceil_div(uint32_t a, uint32_t b) {
  if (SMALL) return ceil_div_small(a, b);
  return (uint32_t)(((uint64_t)a + b - 1) / b);
}
// round(cv * M / W) half up, exactly: floor((2 cv M + W) / (2 W)) with
// cv <= W.  The quotient is at most M + 1/2 < 2^16; the single-precision
// estimate fma(2 cv, M, W) * rcp(2 W) has a relative error of a few 2^-24
// (each input rounded once, the reciprocal within one ulp), so it is off by
// less than 2^16 * 2^-21 < 1/32 and truncates to the quotient or one of its
// neighbours; one exact 64-bit step corrects it.
__device__ inline uint32_t round_share(uint32_t cv, uint32_t M, uint64_t W, float rw2) {
  const uint64_t num = 2ull * cv * M + W;
  const uint64_t den = 2ull * W;
  uint32_t q = (uint32_t)(__builtin_fmaf(2.0f * (float)cv, (float)M, (float)W) * rw2);
  const uint64_t pq = (uint64_t)q * den;
  if (pq > num) q--;
  else if (pq + den <= num) q++;
  return q;
}
// Counter-based candidate byte (the hash documented for seeded allocations).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// LDS of one evaluation wavefront (bytes), for DAGs of up to maxn nodes:
// 8-bit counts when every in-degree is below 256, no byte table when the
// candidate bytes are drawn where they are used.
struct EvalLds {
  size_t rel, seg, gm, pend, cnt, r, total;
};
__host__ __device__ inline EvalLds eval_lds(int maxn, bool c8, bool rs) {
  EvalLds l;
  const size_t nw = (size_t)(maxn + 63) / 64;
  size_t o = 0;
  l.rel = o;  o += nw * 8;  // released, unfinished
  l.seg = o;  o += nw * 8;  // segmented, unfinished (remaining load in the residual region)
  l.gm = o;   o += nw * 8;  // members of the current group
  l.pend = o; o += nw * 8;  // released during the current slot
  l.cnt = o;  o += (c8 ? (size_t)(maxn + 3) / 4 : (size_t)(maxn + 1) / 2) * 4;  // unfinished predecessors
  l.r = o;    o += rs ? 0 : ((size_t)maxn + 15) & ~(size_t)15;  // candidate bytes by sigma rank
  l.total = o;
  return l;
}

// Orders the wavefront's LDS and global accesses (one wavefront per
// workgroup: lanes communicate through memory in program order).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <bool SMALL, bool RS, bool C8, bool TP>
__device__ void eval_one(const SweepArgs& a, uint64_t item, unsigned char* smem, uint32_t* res) {
  const int lane = threadIdx.x;
  const uint64_t li = item / (uint64_t)a.K;
  const int slot = (int)(item - li * (uint64_t)a.K);
  const int d = a.dag_list ? a.dag_list[li] : (int)li;
  const int c = a.cand_list ? a.cand_list[(int64_t)d * a.K + slot] : slot;
  const int64_t n0 = a.t.node_off[d];
  const int N = (int)uni((uint32_t)(a.t.node_off[d + 1] - n0));
  const int NW = (N + 63) >> 6;
  const uint32_t M = (uint32_t)a.M;
  const EvalLds L = eval_lds(a.max_n, C8, RS);
  uint64_t* relw = (uint64_t*)(smem + L.rel);
  uint64_t* segw = (uint64_t*)(smem + L.seg);
  uint64_t* gmw = (uint64_t*)(smem + L.gm);
  uint64_t* pendw = (uint64_t*)(smem + L.pend);
  uint32_t* cnt = (uint32_t*)(smem + L.cnt);
  uint8_t* rb = smem + L.r;
  const uint16_t* indeg = a.t.indeg + n0;
  const uint16_t* succ = a.t.succ + a.t.edge_off[d];
  const uint4* mrec = a.t.mrec + n0;
  const uint4* nrec = a.t.nrec + n0;

  // ---- state: sources released, nothing finished; counts of unfinished
  // predecessors (four 8-bit or two 16-bit counts per word).
  if (C8) {
    for (int i = lane; i < (N + 3) / 4; i += WAVE) {
      uint32_t w = 0;
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (4 * i + q < N) w |= (uint32_t)indeg[4 * i + q] << (8 * q);
      cnt[i] = w;
    }
  } else {
    for (int i = lane; i < (N + 1) / 2; i += WAVE) {
      const uint32_t lo = indeg[2 * i];
      const uint32_t hi = 2 * i + 1 < N ? (uint32_t)indeg[2 * i + 1] : 0u;
      cnt[i] = lo | (hi << 16);
    }
  }
  for (int base = 0; base < N; base += WAVE) {
    const int s = base + lane;
    const uint64_t src = __ballot(s < N && indeg[s] == 0);
    if (lane == 0) relw[base >> 6] = src;
  }
  for (int w = lane; w < NW; w += WAVE) {
    segw[w] = 0;
    gmw[w] = 0;
    pendw[w] = 0;
  }
  // candidate bytes: candidate 0 is the paper's own rule (all zero)
  const uint64_t rkey = mix64(a.seed ^ mix64((uint64_t)d * 0x9E3779B97F4A7C15ull));
  if (!RS) {
    const uint16_t* inv = a.t.inv + n0;
    if (c == 0 || !a.alloc) {
      for (int s = lane; s < N; s += WAVE) rb[s] = 0;
    } else {
      const uint8_t* row = a.alloc + (int64_t)a.kalloc * n0 + (int64_t)c * N;
      for (int v = lane; v < N; v += WAVE) rb[inv[v]] = row[v];
    }
  }
  // byte of node s (local id v, min(p, M) = pp)
  auto r_of = [&](int s, uint32_t v, uint32_t pp) -> uint32_t {
    if (!RS) return rb[s];
    const uint64_t word = mix64(rkey ^ (((uint64_t)c << 32) | (uint64_t)(v >> 2)));
    const uint32_t h16 = (uint32_t)(word >> (16 * (v & 3))) & 0xFFFFu;
    return c == 0 ? 0u : 1u + ((h16 * min(pp, 255u)) >> 16);
  };
  // One finished node's successors lose an unfinished predecessor; a count
  // reaching zero releases the successor (after the slot).
  auto dec = [&](int x) {
    if (C8) {
      const uint32_t sh = (x & 3) * 8;
      const uint32_t old = atomicSub(&cnt[x >> 2], 1u << sh);
      if (((old >> sh) & 0xFFu) == 1u) atomicOr((unsigned long long*)&pendw[x >> 6], 1ull << (x & 63));
    } else {
      const uint32_t sh = (x & 1) * 16;
      const uint32_t old = atomicSub(&cnt[x >> 1], 1u << sh);
      if (((old >> sh) & 0xFFFFu) == 1u) atomicOr((unsigned long long*)&pendw[x >> 6], 1ull << (x & 63));
    }
  };
  // Releases by the finished nodes held in `lanes` (record .z = first
  // successor, .w >> 16 = out-degree), two nodes' lists loaded together.
  auto release = [&](uint64_t lanes, uint32_t rz, uint32_t rw) {
    while (lanes) {
      const int b0 = __builtin_ctzll(lanes);
      lanes &= lanes - 1;
      const int b1 = lanes ? __builtin_ctzll(lanes) : b0;
      const bool two = lanes != 0;
      lanes &= lanes - 1;
      const uint32_t ea0 = (uint32_t)__builtin_amdgcn_readlane((int)rz, b0);
      const uint32_t dg0 = (uint32_t)__builtin_amdgcn_readlane((int)rw, b0) >> 16;
      const uint32_t ea1 = (uint32_t)__builtin_amdgcn_readlane((int)rz, b1);
      const uint32_t dg1 = two ? (uint32_t)__builtin_amdgcn_readlane((int)rw, b1) >> 16 : 0u;
      const int x0 = (uint32_t)lane < dg0 ? (int)succ[ea0 + lane] : -1;
      const int x1 = (uint32_t)lane < dg1 ? (int)succ[ea1 + lane] : -1;
      if (x0 >= 0) dec(x0);
      if (x1 >= 0) dec(x1);
      for (uint32_t o = WAVE; o < dg0; o += WAVE)
        if (o + lane < dg0) dec(succ[ea0 + o + lane]);
      for (uint32_t o = WAVE; o < dg1; o += WAVE)
        if (o + lane < dg1) dec(succ[ea1 + o + lane]);
    }
  };
  wave_sync();

  uint64_t bound = 0, cp = 0;
  int k = 0;
  // (records are picked by assignment, not by a conditional expression,
  // which would select between their addresses and spill them)
  uint4 rec = make_uint4(0u, 0u, 0u, 0u);
  if (lane < N) rec = mrec[lane];
  while (k < N) {
    // group extent from the end marks
    int kend;
    {
      const uint64_t ends = __ballot(k + lane < N && (rec.y >> 31));
      if (ends) {
        kend = k + 1 + __builtin_ctzll(ends);
      } else {
        kend = k + WAVE;
        while (kend < N) {
          const uint64_t m = __ballot(kend + lane < N && (mrec[kend + lane].y >> 31));
          if (m) {
            kend += 1 + __builtin_ctzll(m);
            break;
          }
          kend += WAVE;
        }
        kend = min(kend, N);
      }
    }
    auto chunk = [&](int base) {
      uint4 r1 = rec;
      if (base != k) {
        r1 = make_uint4(0u, 0u, 0u, 0u);
        if (base + lane < kend) r1 = mrec[base + lane];
      }
      return r1;
    };
    // Pass 1: member set and W(pi_j), the remaining load of the released
    // members (Eq. 5).  A group of at most 64 members keeps each lane's
    // remaining load for pass 2.
    uint64_t W = 0;
    uint32_t cv0 = 0;
    for (int base = k; base < kend; base += WAVE) {
      const uint4 r1 = chunk(base);
      const int s = (r1.y >> 16) & 0x7FFF;
      uint32_t cv = 0;
      if (base + lane < kend) {
        atomicOr((unsigned long long*)&gmw[s >> 6], 1ull << (s & 63));
        if ((relw[s >> 6] >> (s & 63)) & 1) cv = ((segw[s >> 6] >> (s & 63)) & 1) ? res[s] : r1.x;
      }
      if (base == k) cv0 = cv;
      // 64 loads below 2^20 sum below 2^26
      W += SMALL ? (uint64_t)wave_sum(cv) : wave_sum64(cv);
    }
    // Loads for later phases are issued only now, after the loads this
    // pass waited for (the vector-memory counter completes in order): the
    // next group's records and the first two members' successor lists.
    __builtin_amdgcn_sched_barrier(0);
    uint4 rnext = make_uint4(0u, 0u, 0u, 0u);
    if (kend + lane < N) rnext = mrec[kend + lane];
    const int nm = min(kend - k, 2);
    const uint32_t pz0 = (uint32_t)__builtin_amdgcn_readlane((int)rec.z, 0);
    const uint32_t pd0 = (uint32_t)__builtin_amdgcn_readlane((int)rec.w, 0) >> 16;
    const uint32_t pz1 = (uint32_t)__builtin_amdgcn_readlane((int)rec.z, 1);
    const uint32_t pd1 = nm > 1 ? (uint32_t)__builtin_amdgcn_readlane((int)rec.w, 1) >> 16 : 0u;
    int px0 = -1, px1 = -1;
    if (W != 0) {
      if ((uint32_t)lane < pd0) px0 = succ[pz0 + lane];
      if ((uint32_t)lane < pd1) px1 = succ[pz1 + lane];
    }
    wave_sync();
    if (W == 0) {
      // every member finished earlier (or is not released): nothing runs
      for (int base = k; base < kend; base += WAVE) {
        const uint4 r1 = chunk(base);
        if (base + lane < kend) gmw[((r1.y >> 16) & 0x7FFF) >> 6] = 0;
      }
      wave_sync();
      k = kend;
      rec = rnext;
      continue;
    }
    // the parallel-node candidates (released, outside the group) are fixed
    // now; their first word's records are loaded ahead
    const uint64_t pw0 = lane < NW ? relw[lane] & ~gmw[lane] : 0ull;
    const uint64_t pw1 = lane + WAVE < NW ? relw[lane + WAVE] & ~gmw[lane + WAVE] : 0ull;
    const uint64_t nz0 = __ballot(pw0 != 0), nz1 = __ballot(pw1 != 0);
    const int j0 = nz0 ? __builtin_ctzll(nz0) : (nz1 ? WAVE + __builtin_ctzll(nz1) : -1);
    uint4 pre = make_uint4(0u, 0u, 0u, 0u);
    if (j0 >= 0) {
      const uint64_t word = readlane64(j0 < WAVE ? pw0 : pw1, j0 & 63);
      if ((word >> lane) & 1) pre = nrec[j0 * WAVE + lane];
    }
    // Pass 2: parallelism (the candidate byte, or Eq. 5) and execution time
    // (Eq. 1) of each released member; the released members finish.
    const float rw2 = __builtin_amdgcn_rcpf((float)(2ull * W));
    uint32_t maxC = 0, sm = 0;
    uint64_t A = 0;
    for (int base = k; base < kend; base += WAVE) {
      const uint4 r1 = chunk(base);
      const int s = (r1.y >> 16) & 0x7FFF;
      const bool rl = base + lane < kend && ((relw[s >> 6] >> (s & 63)) & 1);
      uint64_t a1 = 0;
      if (rl) {
        uint32_t cv = cv0;
        if (base != k) cv = ((segw[s >> 6] >> (s & 63)) & 1) ? res[s] : r1.x;
        const uint32_t pp = r1.y & 0xFFFFu;
        const uint32_t mx = min(pp, cv);
        const uint32_t rv = r_of(s, r1.w & 0xFFFFu, pp);
        const uint32_t m = rv ? min(rv, mx) : max(1u, min(mx, round_share(cv, M, W, rw2)));
        const uint32_t C = ceil_div<SMALL>(cv, m);
        maxC = max(maxC, C);
        sm += m;
        a1 = (uint64_t)m * C;
      }
      // m C < load + m < 2^21 for loads below 2^20: 64 of them sum below 2^27
      A += SMALL ? (uint64_t)wave_sum((uint32_t)a1) : wave_sum64(a1);
      const uint64_t fl = __ballot(rl);
      if (rl) {
        const uint64_t bit = 1ull << (s & 63);
        atomicAnd((unsigned long long*)&relw[s >> 6], ~bit);
        atomicAnd((unsigned long long*)&segw[s >> 6], ~bit);
      }
      if (base == k && (fl & ~3ull) == 0 && pd0 <= WAVE && pd1 <= WAVE) {
        // the released members are among the first two: their lists are loaded
        if ((fl & 1) && px0 >= 0) dec(px0);
        if ((fl & 2) && px1 >= 0) dec(px1);
      } else {
        release(fl, r1.z, r1.w);
      }
    }
    maxC = wave_max(maxC);
    sm = wave_sum(sm);
    wave_sync();
    // Eqs. 6-7: parallel nodes in sigma order take the spare units S; the
    // node at prefix P_i is reached while P_i < S and takes min(m, S - P_i);
    // the first reached node that does not fit in maxC * m is segmented and
    // the launching stops.
    const uint32_t S = sm < M ? M - sm : 0u;
    if (TP && S > 0 && j0 >= 0) {
      // temporal reading: every node keeps the S spare units and the launched
      // nodes run one after another; the node whose time prefix T_i is below
      // maxC is reached, fits if its C = ceil(load / m) ends by maxC, and the
      // first reached node that does not is segmented at (maxC - T_i) * m
      uint32_t Tc = 0;
      bool stop = false;
      for (int h = j0 >> 6; h < 2 && !stop; h++) {
        const uint64_t pw = h ? pw1 : pw0;
        uint64_t nz = h ? nz1 : nz0;
        while (nz && !stop) {
          const int jl = __builtin_ctzll(nz);
          nz &= nz - 1;
          const int j = h * WAVE + jl;
          const uint64_t word = readlane64(pw, jl);
          const bool on = (word >> lane) & 1;
          const int s = j * WAVE + lane;
          uint4 r = pre;
          if (j != j0 && on) r = nrec[s];
          const uint64_t sw = segw[j];
          uint32_t cc = 0, mc = 1, ct = 0;
          if (on) {
            cc = ((sw >> lane) & 1) ? res[s] : r.x;
            const uint32_t pp = r.y & 0xFFFFu;
            const uint32_t mx = min(pp, cc);
            const uint32_t rr = r_of(s, r.w & 0xFFFFu, pp);
            mc = min(rr ? min(rr, mx) : mx, S);
            ct = ceil_div<SMALL>(cc, mc);
          }
          // time prefixes saturate at maxC (no node past it is reached), so
          // the sums stay in range for any load
          const uint32_t incl = wave_scan<uint32_t>(min(ct, maxC), 0u, [maxC](uint32_t p, uint32_t q) {
            return min(p + q, maxC);
          });
          // the prefix of the lanes below: a whole-wave shift right by one
          // lane (DPP, every lane active; lane 0 takes 0)
          const uint32_t excl = dpp32<0x138, 0xf>(incl, 0u);
          const uint32_t Ti = min(Tc + excl, maxC);
          const bool reached = on && Ti < maxC;
          const uint64_t cap = (uint64_t)(reached ? maxC - Ti : 0u) * mc;
          const bool fits = (uint64_t)cc <= cap;
          const uint64_t nofit = __ballot(reached && !fits);
          uint64_t launched = __ballot(reached && fits);
          uint64_t segbit = 0;
          if (nofit) {
            const int f = __builtin_ctzll(nofit);
            launched &= lanes_below(f);
            if (lane == f) res[s] = cc - (uint32_t)cap;
            segbit = 1ull << f;
            stop = true;
          } else {
            Tc = min(Tc + lane63(incl), maxC);
            stop = Tc >= maxC;
          }
          if (lane == 0) {
            relw[j] &= ~launched;
            segw[j] = (sw & ~launched) | segbit;
          }
          release(launched, r.z, r.w);
        }
      }
    }
    if (!TP && S > 0 && j0 >= 0) {
      uint32_t Pc = 0;
      bool stop = false;
      for (int h = j0 >> 6; h < 2 && !stop; h++) {
        const uint64_t pw = h ? pw1 : pw0;
        uint64_t nz = h ? nz1 : nz0;
        while (nz && !stop) {
          const int jl = __builtin_ctzll(nz);
          nz &= nz - 1;
          const int j = h * WAVE + jl;
          const uint64_t word = readlane64(pw, jl);
          const bool on = (word >> lane) & 1;
          const int s = j * WAVE + lane;
          uint4 r = pre;
          if (j != j0 && on) r = nrec[s];
          const uint64_t sw = segw[j];
          uint32_t cc = 0, mcp = 0;
          if (on) {
            cc = ((sw >> lane) & 1) ? res[s] : r.x;
            const uint32_t pp = r.y & 0xFFFFu;
            const uint32_t mx = min(pp, cc);
            const uint32_t rr = r_of(s, r.w & 0xFFFFu, pp);
            mcp = rr ? min(rr, mx) : mx;
          }
          const uint32_t incl = wave_incl_sum(mcp);
          const uint32_t Pi = Pc + incl - mcp;
          const bool reached = on && Pi < S;
          const uint32_t mc = reached ? min(mcp, S - Pi) : 0u;
          const uint64_t cap = (uint64_t)maxC * mc;
          const bool fits = (uint64_t)cc <= cap;
          const uint64_t nofit = __ballot(reached && !fits);
          uint64_t launched = __ballot(reached && fits);
          uint64_t segbit = 0;
          if (nofit) {
            // segmented: it runs maxC * m of its load, the rest stays released
            const int f = __builtin_ctzll(nofit);
            launched &= lanes_below(f);
            if (lane == f) res[s] = cc - (uint32_t)cap;
            segbit = 1ull << f;
            stop = true;
          } else {
            Pc = min(Pc + lane63(incl), S);
            stop = Pc >= S;
          }
          if (lane == 0) {
            relw[j] &= ~launched;
            segw[j] = (sw & ~launched) | segbit;
          }
          release(launched, r.z, r.w);
        }
      }
    }
    // Lemma 1, plus the list-scheduling term if the members oversubscribe.
    uint64_t R = maxC;
    if (sm > M) R += (A - maxC) / M;
    bound += R;
    cp += maxC;
    wave_sync();
    for (int w = lane; w < NW; w += WAVE) {
      relw[w] |= pendw[w];
      pendw[w] = 0;
      gmw[w] = 0;
    }
    wave_sync();
    k = kend;
    rec = rnext;
  }

  if (lane == 0) {
    const int64_t o = (int64_t)d * a.K + slot;
    if (a.bounds) a.bounds[o] = (int64_t)bound;
    if (a.cp) a.cp[o] = (int64_t)cp;
    if (a.intf) a.intf[o] = (int64_t)(bound - cp);
    if (a.best) atomicMin(&a.best[d], (bound << BEST_SHIFT) | (uint64_t)slot);
  }
}

template <bool SMALL, bool RS, bool C8, bool TP>
__global__ __launch_bounds__(64) void k_eval_large(SweepArgs a, unsigned long long* counter, uint64_t total) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* res = a.gres + (size_t)blockIdx.x * (size_t)a.max_n;
  for (;;) {
    uint64_t item = 0;
    if (threadIdx.x == 0) item = atomicAdd(counter, 1ull);
    item = ((uint64_t)uni((uint32_t)(item >> 32)) << 32) | uni((uint32_t)item);  // lane 0's
    if (item >= total) break;
    eval_one<SMALL, RS, C8, TP>(a, item, smem, res);
    wave_sync();
  }
}

template <bool SMALL, bool RS, bool C8, bool TP>
hipError_t launch_large_v(const SweepArgs& a, unsigned long long* counter, uint64_t total, hipStream_t stream) {
  const size_t lds = eval_lds(a.max_n, C8, RS).total;
  const void* fn = (const void*)k_eval_large<SMALL, RS, C8, TP>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WAVE, lds);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const uint64_t cap = (uint64_t)max(1, per_cu) * (uint64_t)max(1, cus);
  uint64_t g = total < cap ? total : cap;
  if (g > (uint64_t)LARGE_SLOTS) g = LARGE_SLOTS;
  hipLaunchKernelGGL((k_eval_large<SMALL, RS, C8, TP>), dim3((unsigned)g), dim3(WAVE), lds, stream, a, counter, total);
  return hipGetLastError();
}

template <bool SMALL, bool RS>
hipError_t launch_large_c(const SweepArgs& a, unsigned long long* counter, uint64_t total, hipStream_t stream) {
  if (a.temporal)
    return a.small_indeg ? launch_large_v<SMALL, RS, true, true>(a, counter, total, stream)
                         : launch_large_v<SMALL, RS, false, true>(a, counter, total, stream);
  return a.small_indeg ? launch_large_v<SMALL, RS, true, false>(a, counter, total, stream)
                       : launch_large_v<SMALL, RS, false, false>(a, counter, total, stream);
}

}  // namespace

// Workgroups of one preprocessing launch: 256 threads (six workgroups per
// compute unit) for DAGs up to 512 nodes, 1024 threads (one per compute
// unit, whose LDS the largest DAGs fill) above.
static int prep_large_grid(int32_t count, int32_t max_n) {
  return std::max(0, std::min(count, max_n <= 512 ? PREP_LARGE_GRID : PREP_LARGE_GRID_BIG));
}

size_t prep_large_scratch_bytes(int32_t count, int32_t max_n, int32_t max_e) {
  return (size_t)prep_large_grid(count, max_n) * prep_scratch(nullptr, max_n, std::max(max_e, 1)).bytes;
}

size_t eval_large_lds_bytes(int max_n) { return eval_lds(max_n, false, false).total; }

template <int PT>
static hipError_t launch_prep_pt(const Tables& t, const PrepInputs& in, int32_t count, int32_t M, const int32_t* list,
                                 unsigned long long* err, void* scratch, int32_t NL, int32_t EL, hipStream_t stream) {
  const size_t lds = prep_lds(NL).total;
  hipError_t e = hipFuncSetAttribute((const void*)k_prep_large<PT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep_large<PT>, dim3(prep_large_grid(count, NL)), dim3(PT), lds, stream, t, in, M, list,
                     count, err, (unsigned char*)scratch, NL, std::max(EL, 1));
  return hipGetLastError();
}

hipError_t launch_prep_large(const Tables& t, const PrepInputs& in, int32_t count, int32_t M, const int32_t* list,
                             unsigned long long* err, void* scratch, int32_t NL, int32_t EL, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (NL > LARGE_MAX_N || !scratch) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(err + 2, 0, sizeof(unsigned long long), stream);  // work counter
  if (e != hipSuccess) return e;
  return NL <= 512 ? launch_prep_pt<256>(t, in, count, M, list, err, scratch, NL, EL, stream)
                   : launch_prep_pt<1024>(t, in, count, M, list, err, scratch, NL, EL, stream);
}

hipError_t launch_eval_large(const SweepArgs& a, uint32_t* counter, hipStream_t stream) {
  const uint64_t total = (uint64_t)a.list_len * (uint64_t)a.K;
  if (total == 0) return hipSuccess;
  if (a.max_n > LARGE_MAX_N || !a.t.mrec || !a.t.nrec) return hipErrorInvalidValue;
  unsigned long long* ctr = (unsigned long long*)counter;
  // seeded bytes are drawn where they are used: N bytes of LDS per
  // wavefront would cost more in occupancy (measured) than the hashing
  const bool rs = a.alloc == nullptr;
  if (a.small_loads)
    return rs ? launch_large_c<true, true>(a, ctr, total, stream) : launch_large_c<true, false>(a, ctr, total, stream);
  return rs ? launch_large_c<false, true>(a, ctr, total, stream) : launch_large_c<false, false>(a, ctr, total, stream);
}

}  // namespace dagbound
