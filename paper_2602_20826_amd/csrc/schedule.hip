// Schedule dump of one (DAG, candidate) on gfx950, for dagbound_get_schedule:
// the slot loop of Algorithm 2 and the slot responses of Lemma 1 with every
// launched part, every slot and the extra dependencies of Section 4.1
// (edges from the slot's longest member to the parallel nodes not launched
// whole, and from each launched part to that member's successors) written
// out as records.  The evaluation kernels keep these edges implicit in the
// slot order; this inspection call makes them explicit.
//
// One wavefront: the lanes set up the per-node state in LDS, then lane 0
// walks the slots (a debug call for one schedule, not a throughput path).
// Node state is indexed by sigma rank; records carry local node ids.
#include "internal.h"

namespace dagbound {
namespace {

constexpr int WAVE = 64;
enum : uint8_t { F_REL = 1, F_DONE = 2, F_INP = 4, F_WHOLE = 8 };

__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct SchedLds {
  size_t rel, cur, npred, nparts, perm, plist, llist, flags, rb, total;
};
__host__ __device__ inline SchedLds sched_lds(int maxn) {
  SchedLds l;
  size_t o = 0;
  auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
  l.rel = o;    o += al((size_t)(maxn + 63) / 64 * 8);  // released bitset by sigma rank
  l.cur = o;    o += al((size_t)maxn * 4);              // remaining load
  l.npred = o;  o += al((size_t)maxn * 2);              // unfinished predecessors
  l.nparts = o; o += al((size_t)maxn * 2);              // parts launched so far
  l.perm = o;   o += al((size_t)maxn * 2);              // local id of each sigma rank
  l.plist = o;  o += al((size_t)maxn * 2);              // the slot's incomplete members
  l.llist = o;  o += al((size_t)maxn * 2);              // the slot's launched parallel nodes
  l.flags = o;  o += al((size_t)maxn);
  l.rb = o;     o += al((size_t)maxn);                  // candidate byte
  l.total = o;
  return l;
}

struct SchedArgs {
  Tables t;
  int32_t d, c, K, M;
  const uint8_t* alloc;  // explicit bytes, or nullptr (seeded)
  uint64_t seed;
  int64_t* rec;          // [cap][8]
  int64_t cap;
  int64_t* out;          // {records, bound, critical-path term, interference term}
  int32_t temporal;      // launching loop: 0 spatial, 1 temporal (chained) reading
};

__global__ __launch_bounds__(64) void k_schedule(SchedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int d = a.d, c = a.c;
  const int64_t n0 = a.t.node_off[d];
  const int N = (int)(a.t.node_off[d + 1] - n0);
  const int NW = (N + 63) >> 6;
  const SchedLds L = sched_lds(N > 0 ? N : 1);
  uint64_t* relw = (uint64_t*)(smem + L.rel);
  uint32_t* cur = (uint32_t*)(smem + L.cur);
  uint16_t* npred = (uint16_t*)(smem + L.npred);
  uint16_t* nparts = (uint16_t*)(smem + L.nparts);
  uint16_t* perm = (uint16_t*)(smem + L.perm);
  uint16_t* plist = (uint16_t*)(smem + L.plist);
  uint16_t* llist = (uint16_t*)(smem + L.llist);
  uint8_t* flags = smem + L.flags;
  uint8_t* rb = smem + L.rb;
  const uint16_t* gl = a.t.gl + n0;
  const uint16_t* pp = a.t.pp + n0;
  const uint32_t* soff = a.t.soff + n0 + d;
  const uint16_t* succ = a.t.succ + a.t.edge_off[d];
  const uint64_t rkey = mix64(a.seed ^ mix64((uint64_t)d * 0x9E3779B97F4A7C15ull));
  for (int v = lane; v < N; v += WAVE) perm[a.t.inv[n0 + v]] = (uint16_t)v;
  for (int s = lane; s < N; s += WAVE) {
    cur[s] = a.t.wc[n0 + s];
    npred[s] = a.t.indeg[n0 + s];
    nparts[s] = 0;
    flags[s] = a.t.indeg[n0 + s] == 0 ? F_REL : 0;
  }
  for (int w = 0; w < NW; w++) {
    const int s = w * WAVE + lane;
    const uint64_t b = __ballot(s < N && a.t.indeg[n0 + s] == 0);
    if (lane == 0) relw[w] = b;
  }
  __syncthreads();
  for (int s = lane; s < N; s += WAVE) {
    const uint32_t v = perm[s];
    uint32_t r = 0;
    if (c > 0) {
      if (a.alloc) {
        r = a.alloc[(int64_t)a.K * n0 + (int64_t)c * N + v];
      } else {
        const uint64_t word = mix64(rkey ^ (((uint64_t)c << 32) | (uint64_t)(v >> 2)));
        const uint32_t h16 = (uint32_t)(word >> (16 * (v & 3))) & 0xFFFFu;
        r = 1u + ((h16 * min((uint32_t)pp[s], 255u)) >> 16);
      }
    }
    rb[s] = (uint8_t)r;
  }
  __syncthreads();
  if (lane != 0) return;

  const int64_t M = a.M;
  int64_t nrec = 0;
  auto put = [&](int64_t r0, int64_t r1, int64_t r2, int64_t r3, int64_t r4, int64_t r5, int64_t r6,
                 int64_t r7) {
    if (nrec < a.cap) {
      int64_t* p = a.rec + nrec * 8;
      p[0] = r0; p[1] = r1; p[2] = r2; p[3] = r3; p[4] = r4; p[5] = r5; p[6] = r6; p[7] = r7;
    }
    nrec++;
  };
  auto cdiv = [](int64_t x, int64_t y) { return (x + y - 1) / y; };
  int64_t bound = 0, cp = 0;
  int k = 0, j = 0;
  while (k < N) {
    int kend = k;
    while (kend < N && !(gl[kend] & 0x8000u)) kend++;
    kend = min(kend + 1, N);
    // the group's incomplete members, in group order, and W(pi_j) (Eq. 5)
    int nP = 0;
    int64_t W = 0;
    for (int i = k; i < kend; i++) {
      const int s = gl[i] & 0x7FFF;
      if (flags[s] & F_DONE) continue;
      plist[nP++] = (uint16_t)s;
      flags[s] |= F_INP;
      W += cur[s];
    }
    if (nP == 0) {
      put(1, j, 0, 0, 0, 0, 0, -1);
      k = kend;
      j++;
      continue;
    }
    // parallelism (the candidate byte, or Eq. 5's half-up share) and
    // execution time (Eq. 1); v_R is the member of largest C, smaller id first
    int64_t maxC = 0, sum_m = 0, A = 0;
    int vR = -1, vRs = -1;
    for (int i = 0; i < nP; i++) {
      const int s = plist[i];
      const int v = perm[s];
      const int64_t mmax = min((int64_t)pp[s], (int64_t)cur[s]);
      const int64_t mv = rb[s] ? min((int64_t)rb[s], mmax)
                               : max((int64_t)1, min(mmax, (2 * (int64_t)cur[s] * M + W) / (2 * W)));
      const int64_t C = cdiv(cur[s], mv);
      sum_m += mv;
      A += mv * C;
      if (C > maxC || (C == maxC && v < vR)) {
        maxC = C;
        vR = v;
        vRs = s;
      }
      put(2, j, v, nparts[s], 0, mv, C, cur[s]);
    }
    // Eqs. 6-7: released non-members in sigma order fill the S spare units;
    // one that does not fit in maxC * m is segmented there and launching stops
    int64_t S = M - sum_m > 0 ? M - sum_m : 0;
    int nl = 0;
    if (a.temporal && S > 0) {
      // temporal reading: every node keeps the S spare units, the launched
      // nodes run one after another within the slot's time maxC
      int64_t T = maxC, peak = 0;
      for (int w = 0; w < NW && T > 0; w++) {
        uint64_t bits = relw[w];
        while (bits && T > 0) {
          const int s = w * WAVE + __builtin_ctzll(bits);
          bits &= bits - 1;
          if (flags[s] & F_INP) continue;
          const int64_t mmax = min((int64_t)pp[s], (int64_t)cur[s]);
          const int64_t mc = min(rb[s] ? min((int64_t)rb[s], mmax) : mmax, S);
          const int64_t capc = T * mc;
          peak = max(peak, mc);
          llist[nl++] = (uint16_t)s;
          if ((int64_t)cur[s] > capc) {
            put(2, j, perm[s], nparts[s], 2, mc, T, capc);
            nparts[s]++;
            cur[s] -= (uint32_t)capc;
            A += mc * T;
            T = 0;
            break;
          }
          const int64_t Cc = cdiv(cur[s], mc);
          put(2, j, perm[s], nparts[s], 1, mc, Cc, cur[s]);
          flags[s] |= F_WHOLE;
          A += mc * Cc;
          T -= Cc;
        }
      }
      sum_m += peak;
      S = 0;
    }
    for (int w = 0; w < NW && S > 0; w++) {
      uint64_t bits = relw[w];
      while (bits && S > 0) {
        const int s = w * WAVE + __builtin_ctzll(bits);
        bits &= bits - 1;
        if (flags[s] & F_INP) continue;
        const int64_t mmax = min((int64_t)pp[s], (int64_t)cur[s]);
        const int64_t mc = min(rb[s] ? min((int64_t)rb[s], mmax) : mmax, S);
        const int64_t capc = maxC * mc;
        llist[nl++] = (uint16_t)s;
        if ((int64_t)cur[s] > capc) {
          put(2, j, perm[s], nparts[s], 2, mc, maxC, capc);
          nparts[s]++;
          cur[s] -= (uint32_t)capc;
          A += mc * cdiv(capc, mc);
          sum_m += mc;
          S = 0;
          break;
        }
        const int64_t Cc = cdiv(cur[s], mc);
        put(2, j, perm[s], nparts[s], 1, mc, Cc, cur[s]);
        flags[s] |= F_WHOLE;
        A += mc * Cc;
        sum_m += mc;
        S -= mc;
      }
    }
    // Lemma 1, with the list-scheduling term when the slot oversubscribes
    const int64_t Rj = sum_m > M ? maxC + (A - maxC) / M : maxC;
    bound += Rj;
    cp += maxC;
    put(1, j, nP, maxC, sum_m, A, Rj, vR);
    // extra dependencies (Section 4.1)
    const int vR_part = nparts[vRs];
    for (int w = 0; w < NW; w++) {
      uint64_t bits = relw[w];
      while (bits) {
        const int s = w * WAVE + __builtin_ctzll(bits);
        bits &= bits - 1;
        if (flags[s] & (F_INP | F_WHOLE)) continue;
        put(3, j, vR, vR_part, perm[s], nparts[s], 0, 0);
      }
    }
    for (int i = 0; i < nl; i++) {
      const int s = llist[i];
      const int part = (flags[s] & F_WHOLE) ? nparts[s] : nparts[s] - 1;
      for (uint32_t e = soff[vRs]; e < soff[vRs + 1]; e++) put(3, j, perm[s], part, perm[succ[e]], 0, 0, 0);
    }
    for (int i = 1; a.temporal && i < nl; i++) {
      // the chain of the temporal reading: each launched part after the one before
      const int q = llist[i - 1], s = llist[i];
      put(3, j, perm[q], nparts[q], perm[s], (flags[s] & F_WHOLE) ? nparts[s] : nparts[s] - 1, 0, 0);
    }
    // completion: the members and the nodes launched whole; then releases
    for (int pass = 0; pass < 2; pass++) {
      const int cnt = pass ? nl : nP;
      for (int i = 0; i < cnt; i++) {
        const int s = pass ? llist[i] : plist[i];
        if (pass && !(flags[s] & F_WHOLE)) continue;
        flags[s] = (uint8_t)((flags[s] | F_DONE) & ~F_REL);
        relw[s >> 6] &= ~(1ull << (s & 63));
        nparts[s]++;
      }
    }
    for (int pass = 0; pass < 2; pass++) {
      const int cnt = pass ? nl : nP;
      for (int i = 0; i < cnt; i++) {
        const int s = pass ? llist[i] : plist[i];
        if (pass && !(flags[s] & F_WHOLE)) continue;
        for (uint32_t e = soff[s]; e < soff[s + 1]; e++) {
          const int x = succ[e];
          if (--npred[x] == 0) {
            flags[x] |= F_REL;
            relw[x >> 6] |= 1ull << (x & 63);
          }
        }
      }
    }
    for (int i = 0; i < nP; i++) flags[plist[i]] &= (uint8_t)~F_INP;
    for (int i = 0; i < nl; i++) flags[llist[i]] &= (uint8_t)~F_WHOLE;
    k = kend;
    j++;
  }
  a.out[0] = nrec;
  a.out[1] = bound;
  a.out[2] = cp;
  a.out[3] = bound - cp;
}

}  // namespace

hipError_t launch_schedule(const Tables& t, int32_t d, int32_t c, int32_t K, int32_t M, const uint8_t* alloc,
                           uint64_t seed, int32_t max_n, int64_t* rec, int64_t cap, int64_t* out, int32_t temporal,
                           hipStream_t stream) {
  if (max_n > LARGE_MAX_N) return hipErrorInvalidValue;
  SchedArgs a{t, d, c, K, M, alloc, seed, rec, cap, out, temporal};
  const size_t lds = sched_lds(max_n > 0 ? max_n : 1).total;
  hipError_t e = hipFuncSetAttribute((const void*)k_schedule, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_schedule, dim3(1), dim3(WAVE), lds, stream, a);
  return hipGetLastError();
}

}  // namespace dagbound
