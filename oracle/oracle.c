/*
 * CPU ORACLE for the makespan bound of DAG-structured GPU tasks
 * (Zhang et al., "Exploiting Dependency and Parallelism: Real-Time Scheduling
 * and Analysis for GPU Tasks", DAC 2026).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, step-by-step
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * It follows the paper's steps in the paper's order:
 *   task model and execution time ............ Section 2.2, Eq. 1
 *   cumulative ancestor workload W^anc ....... Section 3.1, Eq. 2
 *   join-node list Theta, blocks B_k ......... Section 3.1, Eq. 3
 *   local complete paths Lambda_k ............ Section 3.1, Eq. 4
 *   balanced groups Pi (Rules 1-2) ........... Section 3.2, Algorithm 1
 *   parallelism scaling ...................... Section 4.1, Eq. 5
 *   spare capacity, parallel nodes ........... Section 4.1, Eqs. 6-7
 *   node segmentation, extra dependencies .... Section 4.1, Algorithm 2
 *   group response and makespan bound ........ Section 4.2, Lemma 1, Theorem 1
 *   comparison bounds (Greedy, Greedy +
 *   unaware, Graham_para) .................... Section 5.2
 * with these readings of passages that are informal or inconsistent
 * (each one is listed with its reason in the design notes):
 *   - Theta is sorted by ASCENDING W^anc, ties by smaller id (the worked
 *     example of Section 3.2 and the in-block in-degree claim need it).
 *   - Time is integer ticks, t_min = 1: C = ceil(load / m) for m <= M;
 *     the effective maximum parallelism is min(p_v, current load).
 *   - Eq. 5 "round" is half-up on exact integers, clamped to >= 1.
 *   - Top_M takes the largest W^anc first, ties by smaller id.
 *   - Rule 2: if a group of >1 nodes holds a node whose maximum parallelism
 *     reaches M, the group becomes that node alone (the first such node of
 *     largest maximum parallelism, in Top order).
 *   - para(pi_j) = released nodes not in pi_j, launched largest W^anc first;
 *     the spare SM count S shrinks by each launched node's m; a node that does
 *     not fit within max C of the group is cut at capacity max C * m and the
 *     launching stops (spatial reading of Eqs. 6-7).
 *   - A candidate allocation r (one byte per node) replaces Eq. 5 (as a group
 *     member) and the greedy m^max (as a parallel node) for nodes with r > 0;
 *     r = 0 keeps the paper's rule.
 *   - If a slot's SM demand exceeds M (rounding, or explicit r), its response
 *     is max C + floor((A - max C) / M), A = sum of m*C over the slot (a list-
 *     scheduling bound in the block model); otherwise it is max C (Lemma 1).
 * All arithmetic is int64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_E_ARG -1
#define O_E_CYCLE -2
#define O_E_RANGE -3
#define O_E_DUP_EDGE -4
#define O_E_OOM -5
#define O_E_OVERFLOW -8

/* ------------------------------------------------------------------ */
/* Task model (Section 2.1) and integer execution time (Eq. 1).        */
/* ------------------------------------------------------------------ */

static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/* Eq. 1 with t_min = 1 and integer ticks: C = max(1, ceil(ceil(m/M) * load / m)).
 * For m <= M this is ceil(load/m). */
int64_t oracle_exec_time(int64_t load, int64_t m, int64_t M) {
  int64_t waves = ceil_div(m, M);
  return max64(1, ceil_div(waves * load, m));
}

typedef struct {
  int n, e, M;
  const int32_t *src, *dst;
  const int64_t* wcet;   /* \hat C_v, load on one SM */
  const int32_t* par;    /* p_v, maximum parallelism of the kernel */
  /* derived */
  int *pred_off, *pred, *succ_off, *succ;
  unsigned char* anc;    /* anc[v*n+u] != 0  <=>  u in ance(v) */
  int64_t* wanc;         /* Eq. 2 */
  int ntheta;
  int* theta;            /* join nodes in Theta order */
  int nblocks;           /* ntheta + 1 (residual block last) */
  int* block;            /* block index of each node */
  int ngroups;
  int* goff;             /* [ngroups+1] */
  int* gmem;             /* members in group order, each group in Top order */
} odag;

static void odag_free(odag* g) {
  free(g->pred_off); free(g->pred); free(g->succ_off); free(g->succ);
  free(g->anc); free(g->wanc); free(g->theta); free(g->block);
  free(g->goff); free(g->gmem);
  memset(g, 0, sizeof(*g));
}

/* Build adjacency and check the inputs (task model, Section 2.1). */
static int odag_init(odag* g, int n, int e, const int32_t* src, const int32_t* dst,
                     const int64_t* wcet, const int32_t* par, int M) {
  memset(g, 0, sizeof(*g));
  g->n = n; g->e = e; g->M = M; g->src = src; g->dst = dst; g->wcet = wcet; g->par = par;
  if (n < 0 || e < 0 || M < 1 || M > 65535) return O_E_ARG;
  int64_t total = 0;
  for (int v = 0; v < n; v++) {
    if (wcet[v] < 1 || wcet[v] > 2147483647LL || par[v] < 1) return O_E_RANGE;
    total += wcet[v];
  }
  if (total >= (1LL << 40)) return O_E_OVERFLOW;
  for (int k = 0; k < e; k++) {
    if (src[k] < 0 || src[k] >= n || dst[k] < 0 || dst[k] >= n) return O_E_RANGE;
    if (src[k] == dst[k]) return O_E_CYCLE;
  }
  g->pred_off = calloc((size_t)n + 1, sizeof(int));
  g->succ_off = calloc((size_t)n + 1, sizeof(int));
  g->pred = malloc(sizeof(int) * (size_t)(e + 1));
  g->succ = malloc(sizeof(int) * (size_t)(e + 1));
  if (!g->pred_off || !g->succ_off || !g->pred || !g->succ) return O_E_OOM;
  for (int k = 0; k < e; k++) { g->pred_off[dst[k] + 1]++; g->succ_off[src[k] + 1]++; }
  for (int v = 0; v < n; v++) { g->pred_off[v + 1] += g->pred_off[v]; g->succ_off[v + 1] += g->succ_off[v]; }
  int* pf = malloc(sizeof(int) * (size_t)(n + 1));
  int* sf = malloc(sizeof(int) * (size_t)(n + 1));
  if (!pf || !sf) { free(pf); free(sf); return O_E_OOM; }
  memcpy(pf, g->pred_off, sizeof(int) * (size_t)n);
  memcpy(sf, g->succ_off, sizeof(int) * (size_t)n);
  for (int k = 0; k < e; k++) { g->pred[pf[dst[k]]++] = src[k]; g->succ[sf[src[k]]++] = dst[k]; }
  free(pf); free(sf);
  /* duplicate edges would fake join nodes: reject them */
  for (int v = 0; v < n; v++)
    for (int a = g->pred_off[v]; a < g->pred_off[v + 1]; a++)
      for (int b = a + 1; b < g->pred_off[v + 1]; b++)
        if (g->pred[a] == g->pred[b]) return O_E_DUP_EDGE;
  /* acyclicity: Kahn's algorithm must visit every node */
  int* indeg = malloc(sizeof(int) * (size_t)(n + 1));
  int* q = malloc(sizeof(int) * (size_t)(n + 1));
  if (!indeg || !q) { free(indeg); free(q); return O_E_OOM; }
  int qh = 0, qt = 0;
  for (int v = 0; v < n; v++) { indeg[v] = g->pred_off[v + 1] - g->pred_off[v]; if (!indeg[v]) q[qt++] = v; }
  while (qh < qt) {
    int u = q[qh++];
    for (int a = g->succ_off[u]; a < g->succ_off[u + 1]; a++)
      if (--indeg[g->succ[a]] == 0) q[qt++] = g->succ[a];
  }
  free(indeg); free(q);
  if (qt != n) return O_E_CYCLE;
  return O_OK;
}

/* ance(v): every transitive predecessor of v, by a backward search from v. */
static int oracle_ancestors(odag* g) {
  int n = g->n;
  g->anc = calloc((size_t)n * (size_t)n + 1, 1);
  int* stack = malloc(sizeof(int) * (size_t)(n + 1));
  if (!g->anc || !stack) { free(stack); return O_E_OOM; }
  for (int v = 0; v < n; v++) {
    unsigned char* a = g->anc + (size_t)v * n;
    int sp = 0;
    for (int k = g->pred_off[v]; k < g->pred_off[v + 1]; k++)
      if (!a[g->pred[k]]) { a[g->pred[k]] = 1; stack[sp++] = g->pred[k]; }
    while (sp) {
      int u = stack[--sp];
      for (int k = g->pred_off[u]; k < g->pred_off[u + 1]; k++)
        if (!a[g->pred[k]]) { a[g->pred[k]] = 1; stack[sp++] = g->pred[k]; }
    }
  }
  free(stack);
  return O_OK;
}

/* Eq. 2: W^anc(v) = sum of \hat C over ance(v) and v itself. */
static int oracle_wanc(odag* g) {
  int n = g->n;
  g->wanc = malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!g->wanc) return O_E_OOM;
  for (int v = 0; v < n; v++) {
    int64_t s = g->wcet[v];
    for (int u = 0; u < n; u++) if (g->anc[(size_t)v * n + u]) s += g->wcet[u];
    g->wanc[v] = s;
  }
  return O_OK;
}

/* Orders used by the method. */
static __thread const odag* g_cmp;  /* comparator context (per thread) */
/* Theta: ascending W^anc, ties by smaller id. */
static int cmp_theta(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  if (g_cmp->wanc[x] != g_cmp->wanc[y]) return g_cmp->wanc[x] < g_cmp->wanc[y] ? -1 : 1;
  return x - y;
}
/* Top order (Top_M of Algorithm 1, para order of Section 4.1):
 * descending W^anc, ties by smaller id. */
static int cmp_top(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  if (g_cmp->wanc[x] != g_cmp->wanc[y]) return g_cmp->wanc[x] > g_cmp->wanc[y] ? -1 : 1;
  return x - y;
}

/* Section 3.1: join nodes sorted into Theta; blocks B_k = ance(theta_k)
 * minus earlier blocks (Eq. 3); the rest forms the residual block. */
static int oracle_blocks(odag* g) {
  int n = g->n;
  g->theta = malloc(sizeof(int) * (size_t)(n + 1));
  g->block = malloc(sizeof(int) * (size_t)(n + 1));
  if (!g->theta || !g->block) return O_E_OOM;
  g->ntheta = 0;
  for (int v = 0; v < n; v++)
    if (g->pred_off[v + 1] - g->pred_off[v] >= 2) g->theta[g->ntheta++] = v;
  g_cmp = g;
  qsort(g->theta, (size_t)g->ntheta, sizeof(int), cmp_theta);
  g->nblocks = g->ntheta + 1;
  for (int v = 0; v < n; v++) g->block[v] = -1;
  for (int k = 0; k < g->ntheta; k++) {
    int t = g->theta[k];
    for (int u = 0; u < n; u++)
      if (g->anc[(size_t)t * n + u] && g->block[u] < 0) g->block[u] = k;
  }
  for (int v = 0; v < n; v++) if (g->block[v] < 0) g->block[v] = g->ntheta;
  return O_OK;
}

/* Section 3.1, Eq. 4: local complete paths of block k, from local sources
 * (no predecessor inside the block) along in-block edges to local sinks (no
 * successor inside the block).  Paths are written as node lists into
 * `paths` (each of length plen[i]).  Returns the number of paths, or -1. */
static int local_paths(const odag* g, int k, int** paths, int* plen, int maxpaths) {
  int n = g->n, np = 0;
  int* stack = malloc(sizeof(int) * (size_t)(n + 1));
  int* it = malloc(sizeof(int) * (size_t)(n + 1));
  if (!stack || !it) { free(stack); free(it); return -1; }
  for (int s = 0; s < n; s++) {
    if (g->block[s] != k) continue;
    int local_src = 1;
    for (int a = g->pred_off[s]; a < g->pred_off[s + 1]; a++)
      if (g->block[g->pred[a]] == k) local_src = 0;
    if (!local_src) continue;
    /* depth-first enumeration of in-block paths from s */
    int sp = 0;
    stack[sp] = s; it[sp] = g->succ_off[s]; sp++;
    while (sp) {
      int v = stack[sp - 1];
      int advanced = 0, has_in_block_succ = 0;
      for (int a = g->succ_off[v]; a < g->succ_off[v + 1]; a++)
        if (g->block[g->succ[a]] == k) has_in_block_succ = 1;
      if (!has_in_block_succ) {
        /* v is a local sink: emit the path on the stack */
        if (np >= maxpaths) { free(stack); free(it); return -1; }
        paths[np] = malloc(sizeof(int) * (size_t)sp);
        if (!paths[np]) { free(stack); free(it); return -1; }
        for (int i = 0; i < sp; i++) paths[np][i] = stack[i];
        plen[np] = sp; np++;
        sp--;
        continue;
      }
      while (it[sp - 1] < g->succ_off[v + 1]) {
        int w = g->succ[it[sp - 1]++];
        if (g->block[w] == k) { stack[sp] = w; it[sp] = g->succ_off[w]; sp++; advanced = 1; break; }
      }
      if (!advanced) sp--;
    }
  }
  free(stack); free(it);
  return np;
}

/* Section 3.2, Algorithm 1: per block, repeatedly take the heads of the local
 * complete paths, keep the Top_M by W^anc (Rule 1), apply Rule 2, remove them
 * from every path and append the group to Pi. */
static int oracle_groups(odag* g) {
  int n = g->n, M = g->M;
  g->goff = malloc(sizeof(int) * (size_t)(n + 2));
  g->gmem = malloc(sizeof(int) * (size_t)(n + 1));
  int* heads = malloc(sizeof(int) * (size_t)(n + 1));
  unsigned char* removed = calloc((size_t)n + 1, 1);
  unsigned char* is_head = calloc((size_t)n + 1, 1);
  int maxpaths = n + 1;
  int** paths = calloc((size_t)maxpaths, sizeof(int*));
  int* plen = malloc(sizeof(int) * (size_t)maxpaths);
  int* pfirst = malloc(sizeof(int) * (size_t)maxpaths); /* index of the first unremoved element */
  if (!g->goff || !g->gmem || !heads || !removed || !is_head || !paths || !plen || !pfirst) {
    free(heads); free(removed); free(is_head); free(paths); free(plen); free(pfirst);
    return O_E_OOM;
  }
  int ng = 0, nm = 0, rc = O_OK;
  g->goff[0] = 0;
  for (int k = 0; k < g->nblocks && rc == O_OK; k++) {
    int np = local_paths(g, k, paths, plen, maxpaths);
    if (np < 0) { rc = O_E_OOM; break; }
    for (int i = 0; i < np; i++) pfirst[i] = 0;
    for (;;) {
      /* heads of the non-empty paths, distinct */
      int nh = 0;
      for (int i = 0; i < np; i++) {
        while (pfirst[i] < plen[i] && removed[paths[i][pfirst[i]]]) pfirst[i]++;
        if (pfirst[i] < plen[i]) {
          int h = paths[i][pfirst[i]];
          if (!is_head[h]) { is_head[h] = 1; heads[nh++] = h; }
        }
      }
      for (int i = 0; i < nh; i++) is_head[heads[i]] = 0;
      if (nh == 0) break;               /* Lambda_k is empty */
      g_cmp = g;
      qsort(heads, (size_t)nh, sizeof(int), cmp_top);
      int take = nh < M ? nh : M;       /* Rule 1 */
      if (take > 1) {                   /* Rule 2 */
        int pick = -1; int64_t best = -1;
        for (int i = 0; i < take; i++) {
          int v = heads[i];
          int64_t mmax = min64(g->par[v], g->wcet[v]);
          if (mmax >= M && mmax > best) { best = mmax; pick = v; }
        }
        if (pick >= 0) { heads[0] = pick; take = 1; }
      }
      for (int i = 0; i < take; i++) { removed[heads[i]] = 1; g->gmem[nm++] = heads[i]; }
      g->goff[++ng] = nm;
    }
    for (int i = 0; i < np; i++) { free(paths[i]); paths[i] = NULL; }
  }
  g->ngroups = ng;
  free(heads); free(removed); free(is_head); free(paths); free(plen); free(pfirst);
  if (rc == O_OK && nm != n) rc = O_E_ARG; /* every node must land in exactly one group */
  return rc;
}

static int oracle_prepare(odag* g, int n, int e, const int32_t* src, const int32_t* dst,
                          const int64_t* wcet, const int32_t* par, int M) {
  int rc = odag_init(g, n, e, src, dst, wcet, par, M);
  if (rc == O_OK) rc = oracle_ancestors(g);
  if (rc == O_OK) rc = oracle_wanc(g);
  if (rc == O_OK) rc = oracle_blocks(g);
  if (rc == O_OK) rc = oracle_groups(g);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Exported: sub-graph division (for the worked-example checks).       */
/* ------------------------------------------------------------------ */

/* Outputs (each may be NULL): wanc[n]; theta[n] (ntheta entries); block[n];
 * group_of[n]; gmem[n] and goff[n+1] (ngroups+1 entries); counts[2] =
 * {ntheta, ngroups}. */
int oracle_division(int n, int e, const int32_t* src, const int32_t* dst, const int64_t* wcet,
                    const int32_t* par, int M, int64_t* wanc, int32_t* theta, int32_t* block,
                    int32_t* group_of, int32_t* gmem, int32_t* goff, int32_t* counts) {
  odag g;
  int rc = oracle_prepare(&g, n, e, src, dst, wcet, par, M);
  if (rc == O_OK) {
    for (int v = 0; v < n; v++) {
      if (wanc) wanc[v] = g.wanc[v];
      if (block) block[v] = g.block[v];
    }
    if (theta) for (int k = 0; k < g.ntheta; k++) theta[k] = g.theta[k];
    for (int j = 0; j < g.ngroups; j++)
      for (int i = g.goff[j]; i < g.goff[j + 1]; i++) {
        if (group_of) group_of[g.gmem[i]] = j;
        if (gmem) gmem[i] = g.gmem[i];
      }
    if (goff) for (int j = 0; j <= g.ngroups; j++) goff[j] = g.goff[j];
    if (counts) { counts[0] = g.ntheta; counts[1] = g.ngroups; }
  }
  odag_free(&g);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Scheduling (Algorithm 2) and response-time analysis (Lemma 1,       */
/* Theorem 1).                                                         */
/* ------------------------------------------------------------------ */

/* Schedule trace records, 8 int64 each:
 *   SLOT: {1, j, |P_j|, maxC, sum m, A, R_j, v_R}
 *   PART: {2, j, node, part index, kind (0 member, 1 parallel whole,
 *          2 parallel segment), m, C, load}
 *   EDGE: {3, j, from node, from part, to node, to part, 0, 0}
 * Parts of a node are numbered from 0 in launch order. */
#define REC 8

typedef struct {
  int64_t* buf; int64_t cap, n;
} trace_t;

static void trace_put(trace_t* t, int64_t a0, int64_t a1, int64_t a2, int64_t a3, int64_t a4,
                      int64_t a5, int64_t a6, int64_t a7) {
  if (t && t->buf && t->n < t->cap) {
    int64_t* r = t->buf + t->n * REC;
    r[0] = a0; r[1] = a1; r[2] = a2; r[3] = a3; r[4] = a4; r[5] = a5; r[6] = a6; r[7] = a7;
  }
  if (t) t->n++;
}

/* Runs Algorithm 2 under candidate r (r may be NULL: the paper's rule for
 * every node).  out3 = {bound, critical-path term, interference term}.
 * temporal selects the other reading of the launching loop (Eqs. 6-7 with
 * WS_j as an area): the S spare SMs stay S for every parallel node, the
 * launched nodes run one after another on them (chain edges), and the
 * budget is the slot's time maxC; a node that does not fit in the time left
 * is segmented at (time left) * m_c and the launching stops. */
static int oracle_schedule(const odag* g, const uint8_t* r, int64_t* out3, trace_t* tr, int temporal,
                           const uint8_t* xm) {
  int n = g->n;
  int64_t M = g->M;
  int64_t* cur = malloc(sizeof(int64_t) * (size_t)(n + 1));       /* remaining load, \hat C */
  unsigned char* complete = calloc((size_t)n + 1, 1);
  unsigned char* released = calloc((size_t)n + 1, 1);
  unsigned char* inP = calloc((size_t)n + 1, 1);
  int* npred = malloc(sizeof(int) * (size_t)(n + 1));
  int* nparts = calloc((size_t)n + 1, sizeof(int));
  int* P = malloc(sizeof(int) * (size_t)(n + 1));
  int64_t* m = malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* C = malloc(sizeof(int64_t) * (size_t)(n + 1));
  int* para = malloc(sizeof(int) * (size_t)(n + 1));
  int* done = malloc(sizeof(int) * (size_t)(n + 1));
  unsigned char* launched_whole = calloc((size_t)n + 1, 1);
  int* launched_part = malloc(sizeof(int) * (size_t)(n + 1));
  if (!cur || !complete || !released || !inP || !npred || !nparts || !P || !m || !C || !para ||
      !done || !launched_whole || !launched_part) {
    free(cur); free(complete); free(released); free(inP); free(npred); free(nparts); free(P);
    free(m); free(C); free(para); free(done); free(launched_whole); free(launched_part);
    return O_E_OOM;
  }
  for (int v = 0; v < n; v++) {
    cur[v] = g->wcet[v];
    npred[v] = g->pred_off[v + 1] - g->pred_off[v];
    released[v] = (npred[v] == 0);      /* Released_nodes <- src(G) */
  }
  int64_t bound = 0, cp = 0, intf = 0;
  /* conditional reading (xm != NULL): the same schedule, and each slot's
   * response from the parts of the nodes that execute (xm[v] != 0) */
  int64_t xbound = 0, xcp = 0;
  for (int j = 0; j < g->ngroups; j++) {
    /* members of pi_j that are not complete yet */
    int nP = 0;
    for (int i = g->goff[j]; i < g->goff[j + 1]; i++) {
      int v = g->gmem[i];
      if (!complete[v]) { P[nP++] = v; inP[v] = 1; }
    }
    if (nP == 0) { trace_put(tr, 1, j, 0, 0, 0, 0, 0, -1); continue; }
    /* Eq. 5: parallelism scaling, W(pi_j) = sum of the members' loads */
    int64_t W = 0;
    for (int i = 0; i < nP; i++) W += cur[P[i]];
    int64_t maxC = 0, sum_m = 0, A = 0;
    int64_t xmaxC = 0, xsum_m = 0, xA = 0;
    int vR = -1;
    for (int i = 0; i < nP; i++) {
      int v = P[i];
      int64_t mmax = min64(g->par[v], cur[v]);
      int64_t mv;
      if (r && r[v] > 0) {
        mv = min64(min64(r[v], mmax), M);
      } else {
        int64_t rounded = (2 * cur[v] * M + W) / (2 * W);   /* round(cur*M/W), half up */
        mv = max64(1, min64(mmax, rounded));
      }
      m[v] = mv;
      C[v] = ceil_div(cur[v], mv);                          /* Eq. 1, m <= M */
      sum_m += mv;
      A += mv * C[v];
      if (C[v] > maxC || (C[v] == maxC && v < vR)) { maxC = C[v]; vR = v; }
      if (!xm || xm[v]) { xsum_m += mv; xA += mv * C[v]; xmaxC = max64(xmaxC, C[v]); }
    }
    for (int i = 0; i < nP; i++)
      trace_put(tr, 2, j, P[i], nparts[P[i]], 0, m[P[i]], C[P[i]], cur[P[i]]);
    /* Eq. 7: parallel nodes = released nodes outside the group, Top order */
    int npara = 0;
    for (int v = 0; v < n; v++) if (released[v] && !inP[v]) para[npara++] = v;
    g_cmp = g;
    qsort(para, (size_t)npara, sizeof(int), cmp_top);
    /* Eq. 6 and the launching loop: S spare SMs next to the group */
    int64_t S = M - sum_m;
    if (S < 0) S = 0;
    int nl = 0, seg_node = -1;
    if (temporal) {
      int64_t T = maxC, peak = 0;     /* time left on the spare SMs */
      for (int i = 0; i < npara && S > 0 && T > 0; i++) {
        int c = para[i];
        int64_t mmax = min64(g->par[c], cur[c]);
        int64_t target = (r && r[c] > 0) ? min64(r[c], mmax) : mmax;
        int64_t mc = min64(target, S);
        int64_t cap = T * mc;
        peak = max64(peak, mc);
        if (cur[c] > cap) {
          trace_put(tr, 2, j, c, nparts[c], 2, mc, T, cap);
          launched_part[nl++] = c;
          nparts[c]++;
          cur[c] -= cap;
          A += mc * T;
          seg_node = c;
          break;
        }
        int64_t Cc = ceil_div(cur[c], mc);
        trace_put(tr, 2, j, c, nparts[c], 1, mc, Cc, cur[c]);
        launched_whole[c] = 1;
        launched_part[nl++] = c;
        A += mc * Cc;
        T -= Cc;
      }
      sum_m += peak;
      S = 0;
    }
    for (int i = 0; i < npara && S > 0; i++) {
      int c = para[i];
      int64_t mmax = min64(g->par[c], cur[c]);
      int64_t target = (r && r[c] > 0) ? min64(r[c], mmax) : mmax;
      int64_t mc = min64(target, S);
      int64_t cap = maxC * mc;
      if (cur[c] > cap) {
        /* node segmentation: the parallel segment fills the capacity */
        trace_put(tr, 2, j, c, nparts[c], 2, mc, maxC, cap);
        launched_part[nl++] = c;
        nparts[c]++;
        cur[c] -= cap;
        A += mc * ceil_div(cap, mc);
        sum_m += mc;
        if (!xm || xm[c]) { xsum_m += mc; xA += mc * ceil_div(cap, mc); xmaxC = max64(xmaxC, ceil_div(cap, mc)); }
        seg_node = c;
        break;
      }
      int64_t Cc = ceil_div(cur[c], mc);
      trace_put(tr, 2, j, c, nparts[c], 1, mc, Cc, cur[c]);
      launched_whole[c] = 1;
      launched_part[nl++] = c;
      A += mc * Cc;
      sum_m += mc;
      if (!xm || xm[c]) { xsum_m += mc; xA += mc * Cc; xmaxC = max64(xmaxC, Cc); }
      S -= mc;
    }
    /* Lemma 1, with the list-scheduling term when the slot oversubscribes */
    int64_t Rj = maxC;
    if (sum_m > M) Rj = maxC + (A - maxC) / M;
    bound += Rj; cp += maxC; intf += Rj - maxC;
    /* Lemma 1 over the executed parts only: they start together when they
     * fit, else list scheduling bounds them; no executed part: 0 */
    int64_t xRj = xmaxC;
    if (xsum_m > M) xRj = xmaxC + (xA - xmaxC) / M;
    xbound += xRj; xcp += xmaxC;
    trace_put(tr, 1, j, nP, maxC, sum_m, A, Rj, vR);
    /* extra dependencies (Section 4.1), recorded for inspection */
    int vR_part = nparts[vR];
    for (int i = 0; i < npara; i++) {
      int u = para[i];
      if (launched_whole[u]) continue;
      /* not launched whole (never launched, or the residual of the segment) */
      trace_put(tr, 3, j, vR, vR_part, u, nparts[u], 0, 0);
    }
    for (int i = 0; i < nl; i++) {
      int c = launched_part[i];
      int part = launched_whole[c] ? nparts[c] : nparts[c] - 1;
      for (int a = g->succ_off[vR]; a < g->succ_off[vR + 1]; a++)
        trace_put(tr, 3, j, c, part, g->succ[a], 0, 0, 0);
    }
    for (int i = 1; temporal && i < nl; i++) {
      /* the chain: each launched part after the one launched before it */
      int q = launched_part[i - 1], c = launched_part[i];
      trace_put(tr, 3, j, q, nparts[q], c, launched_whole[c] ? nparts[c] : nparts[c] - 1, 0, 0);
    }
    (void)seg_node;
    /* completion and release (Algorithm 2, "Update Released_nodes") */
    int nd = 0;
    for (int i = 0; i < nP; i++) done[nd++] = P[i];
    for (int i = 0; i < nl; i++) if (launched_whole[launched_part[i]]) done[nd++] = launched_part[i];
    for (int i = 0; i < nd; i++) {
      int v = done[i];
      complete[v] = 1; released[v] = 0; nparts[v]++;
    }
    for (int i = 0; i < nd; i++) {
      int v = done[i];
      for (int a = g->succ_off[v]; a < g->succ_off[v + 1]; a++)
        if (--npred[g->succ[a]] == 0) released[g->succ[a]] = 1;
    }
    for (int i = 0; i < nP; i++) inP[P[i]] = 0;
    for (int i = 0; i < nl; i++) launched_whole[launched_part[i]] = 0;
  }
  if (xm) { out3[0] = xbound; out3[1] = xcp; out3[2] = xbound - xcp; }
  else { out3[0] = bound; out3[1] = cp; out3[2] = intf; }
  free(cur); free(complete); free(released); free(inP); free(npred); free(nparts); free(P);
  free(m); free(C); free(para); free(done); free(launched_whole); free(launched_part);
  return O_OK;
}

/* Bound of one DAG under one candidate (r may be NULL).  out3 = {bound,
 * critical-path term, interference term}.  trace/trace_cap optional; the
 * number of records the schedule produced is stored in *trace_n.
 * para_mode 0: spatial launching loop, 1: temporal (chained) reading. */
int oracle_bound(int n, int e, const int32_t* src, const int32_t* dst, const int64_t* wcet,
                 const int32_t* par, int M, const uint8_t* r, int64_t* out3, int64_t* trace,
                 int64_t trace_cap, int64_t* trace_n, int para_mode) {
  odag g;
  int rc = oracle_prepare(&g, n, e, src, dst, wcet, par, M);
  if (rc == O_OK) {
    trace_t t = { trace, trace_cap, 0 };
    rc = oracle_schedule(&g, r, out3, &t, para_mode, NULL);
    if (trace_n) *trace_n = t.n;
  }
  odag_free(&g);
  return rc;
}

/* Conditional DAGs (the paper's future work, Section 6), spatial reading:
 * the schedule of the DAG with every branch present, and the makespan bound
 * of one realization, in which only the nodes with xm[v] != 0 execute (the
 * others take no SM and no time).  Each slot's response is Lemma 1 over
 * the slot's executed parts (members, parallel nodes launched whole and
 * parallel segments): their largest C when their SMs fit in M, else the
 * list-scheduling form; a slot with no executed part takes 0.  out3 =
 * {bound, critical-path term, interference term} of the realization. */
int oracle_cond_bound(int n, int e, const int32_t* src, const int32_t* dst, const int64_t* wcet,
                      const int32_t* par, int M, const uint8_t* r, const uint8_t* xm, int64_t* out3) {
  odag g;
  if (!xm) return O_E_ARG;
  int rc = oracle_prepare(&g, n, e, src, dst, wcet, par, M);
  if (rc == O_OK) rc = oracle_schedule(&g, r, out3, NULL, 0, xm);
  odag_free(&g);
  return rc;
}

/* All K candidates of one DAG: r holds K*n bytes, (c, v) at c*n + v; the
 * bytes of candidate 0 are ignored (candidate 0 is the paper's own rule).
 * bounds/cp/intf [K] (cp and intf may be NULL). */
int oracle_bounds_dag(int n, int e, const int32_t* src, const int32_t* dst, const int64_t* wcet,
                      const int32_t* par, int M, int K, const uint8_t* r, int64_t* bounds,
                      int64_t* cp, int64_t* intf, int para_mode) {
  odag g;
  int rc = oracle_prepare(&g, n, e, src, dst, wcet, par, M);
  for (int c = 0; c < K && rc == O_OK; c++) {
    int64_t o[3];
    rc = oracle_schedule(&g, c == 0 ? NULL : r + (int64_t)c * n, o, NULL, para_mode, NULL);
    bounds[c] = o[0];
    if (cp) cp[c] = o[1];
    if (intf) intf[c] = o[2];
  }
  odag_free(&g);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Comparison bounds of the evaluation (Section 5.2).                  */
/*                                                                     */
/* With t_min = 1 the maximum useful parallelism of v is               */
/* m^max = min(p_v, C_hat_v) (Section 2.2, with the input cap p_v).     */
/*   Greedy: every node at m = min(m^max, M), nodes run one after       */
/*     another: the sum of their Eq. 1 times.                          */
/*   Greedy + unaware: m = m^max, ceil(m/M) waves in Eq. 1, summed.     */
/*   Graham_para: node v becomes m^max unit-SM nodes of                 */
/*     ceil(C_hat/m^max) ticks, all with v's dependencies; Graham's     */
/*     list-scheduling bound on M SMs for that DAG is                  */
/*     len + floor((vol - len) / M), len = the longest path in ticks,   */
/*     vol = the SM-ticks of all unit nodes (floor: makespans are       */
/*     whole ticks).                                                   */
/* ------------------------------------------------------------------ */

/* out3 = {Greedy, Greedy + unaware, Graham_para} of one DAG. */
int oracle_baselines(int n, int e, const int32_t* src, const int32_t* dst, const int64_t* wcet,
                     const int32_t* par, int M, int64_t* out3) {
  odag g;
  int rc = odag_init(&g, n, e, src, dst, wcet, par, M);
  int64_t* len = NULL;
  int* indeg = NULL;
  int* order = NULL;
  if (rc == O_OK) {
    len = calloc((size_t)n + 1, sizeof(int64_t));
    indeg = malloc(sizeof(int) * (size_t)(n + 1));
    order = malloc(sizeof(int) * (size_t)(n + 1));
    if (!len || !indeg || !order) rc = O_E_OOM;
  }
  if (rc == O_OK) {
    int64_t greedy = 0, unaware = 0, vol = 0, longest = 0;
    for (int v = 0; v < n; v++) {
      int64_t mmax = min64(par[v], wcet[v]);
      greedy += oracle_exec_time(wcet[v], min64(mmax, M), M);
      unaware += oracle_exec_time(wcet[v], mmax, M);
      vol += mmax * ceil_div(wcet[v], mmax);
    }
    /* longest path of the expanded DAG, in a topological order (Kahn) */
    int qh = 0, qt = 0;
    for (int v = 0; v < n; v++) {
      indeg[v] = g.pred_off[v + 1] - g.pred_off[v];
      if (!indeg[v]) order[qt++] = v;
    }
    while (qh < qt) {
      int u = order[qh++];
      int64_t mmax = min64(par[u], wcet[u]);
      len[u] += ceil_div(wcet[u], mmax);  /* len[u] held the longest predecessor path */
      longest = max64(longest, len[u]);
      for (int a = g.succ_off[u]; a < g.succ_off[u + 1]; a++) {
        int w = g.succ[a];
        len[w] = max64(len[w], len[u]);
        if (--indeg[w] == 0) order[qt++] = w;
      }
    }
    out3[0] = greedy;
    out3[1] = unaware;
    out3[2] = n ? longest + (vol - longest) / M : 0;
  }
  free(len); free(indeg); free(order);
  odag_free(&g);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Block-level execution model, for safety checks of the bound.        */
/*                                                                     */
/* A launched part with parallelism m and execution time C is m thread  */
/* blocks, each holding one SM for C ticks (the waves of Eq. 1).  The   */
/* hardware block scheduler is a black box (Section 2.2): any ready     */
/* block may take a free SM, and an SM is never left idle while a block */
/* is ready (work-conserving).  Parts form a DAG through `pred`.        */
/* ------------------------------------------------------------------ */

typedef struct {
  int nparts, M;
  const int64_t *m, *C;
  const int32_t *pred_off, *pred;
  int64_t *started, *finished;
  int64_t* run_end;      /* finish times of running blocks */
  int* run_part;
  int nrun;
  int64_t best;
  int64_t nodes, node_limit;
} sim_t;

static int part_ready(sim_t* s, int x) {
  if (s->started[x] >= s->m[x]) return 0;
  for (int a = s->pred_off[x]; a < s->pred_off[x + 1]; a++)
    if (s->finished[s->pred[a]] < s->m[s->pred[a]]) return 0;
  return 1;
}

/* Depth-first search over every dispatch choice.  At one time instant the
 * blocks started are chosen in nondecreasing part index (the order of
 * simultaneous starts does not matter). */
static void sim_dfs(sim_t* s, int64_t t, int minpart) {
  if (s->node_limit && ++s->nodes > s->node_limit) return;
  int any = 0;
  if (s->nrun < s->M) {
    for (int x = 0; x < s->nparts; x++) {
      if (!part_ready(s, x)) continue;
      any = 1;
      if (x < minpart) continue;
      s->started[x]++;
      s->run_end[s->nrun] = t + s->C[x];
      s->run_part[s->nrun] = x;
      s->nrun++;
      sim_dfs(s, t, x);
      s->nrun--;
      s->started[x]--;
    }
    if (any) return; /* work-conserving: some block must start now */
  }
  if (s->nrun == 0) {
    /* nothing runs: either everything is done or nothing is ready */
    if (t > s->best) s->best = t;
    return;
  }
  /* advance to the next completion; the running list is put back exactly
   * as it was, since the caller removes the block it added last */
  int64_t tn = INT64_MAX;
  for (int i = 0; i < s->nrun; i++) if (s->run_end[i] < tn) tn = s->run_end[i];
  int64_t saved_end[64]; int saved_part[64];
  const int nsaved = s->nrun;
  memcpy(saved_end, s->run_end, sizeof(int64_t) * (size_t)nsaved);
  memcpy(saved_part, s->run_part, sizeof(int) * (size_t)nsaved);
  int k = 0;
  for (int i = 0; i < nsaved; i++) {
    if (saved_end[i] == tn) {
      s->finished[saved_part[i]]++;
    } else {
      s->run_end[k] = saved_end[i]; s->run_part[k] = saved_part[i]; k++;
    }
  }
  s->nrun = k;
  sim_dfs(s, tn, 0);
  for (int i = 0; i < nsaved; i++)
    if (saved_end[i] == tn) s->finished[saved_part[i]]--;
  memcpy(s->run_end, saved_end, sizeof(int64_t) * (size_t)nsaved);
  memcpy(s->run_part, saved_part, sizeof(int) * (size_t)nsaved);
  s->nrun = nsaved;
}

/* Worst makespan over all work-conserving dispatch orders of the parts
 * (each part: m blocks of C ticks; pred in CSR form).  M <= 64.  Returns
 * -1 if the search exceeded node_limit (0 = unlimited). */
int64_t oracle_worst_makespan(int nparts, int M, const int64_t* m, const int64_t* C,
                              const int32_t* pred_off, const int32_t* pred, int64_t node_limit) {
  if (M < 1 || M > 64) return -2;
  sim_t s;
  memset(&s, 0, sizeof(s));
  s.nparts = nparts; s.M = M; s.m = m; s.C = C; s.pred_off = pred_off; s.pred = pred;
  s.started = calloc((size_t)nparts + 1, sizeof(int64_t));
  s.finished = calloc((size_t)nparts + 1, sizeof(int64_t));
  s.run_end = calloc(65, sizeof(int64_t));
  s.run_part = calloc(65, sizeof(int));
  s.node_limit = node_limit;
  s.best = 0;
  if (!s.started || !s.finished || !s.run_end || !s.run_part) return -3;
  sim_dfs(&s, 0, 0);
  int64_t out = (node_limit && s.nodes > node_limit) ? -1 : s.best;
  free(s.started); free(s.finished); free(s.run_end); free(s.run_part);
  return out;
}

/* One random work-conserving dispatch with random early completion: each
 * block runs for a uniform duration in [1, C] when early != 0, else C.
 * Returns the makespan. */
int64_t oracle_random_makespan(int nparts, int M, const int64_t* m, const int64_t* C,
                               const int32_t* pred_off, const int32_t* pred, uint64_t seed,
                               int early) {
  int64_t* started = calloc((size_t)nparts + 1, sizeof(int64_t));
  int64_t* finished = calloc((size_t)nparts + 1, sizeof(int64_t));
  int64_t* run_end = malloc(sizeof(int64_t) * (size_t)(M + 1));
  int* run_part = malloc(sizeof(int) * (size_t)(M + 1));
  int* ready = malloc(sizeof(int) * (size_t)(nparts + 1));
  if (!started || !finished || !run_end || !run_part || !ready) return -3;
  uint64_t st = seed;
  int nrun = 0;
  int64_t t = 0;
  for (;;) {
    for (;;) {
      if (nrun >= M) break;
      int nr = 0;
      for (int x = 0; x < nparts; x++) {
        if (started[x] >= m[x]) continue;
        int ok = 1;
        for (int a = pred_off[x]; a < pred_off[x + 1]; a++)
          if (finished[pred[a]] < m[pred[a]]) { ok = 0; break; }
        if (ok) ready[nr++] = x;
      }
      if (!nr) break;
      st += 0x9E3779B97F4A7C15ULL;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z ^= z >> 31;
      int x = ready[z % (uint64_t)nr];
      int64_t dur = C[x];
      if (early && C[x] > 1) dur = 1 + (int64_t)((z >> 32) % (uint64_t)C[x]);
      started[x]++;
      run_end[nrun] = t + dur; run_part[nrun] = x; nrun++;
    }
    if (!nrun) break;
    int64_t tn = INT64_MAX;
    for (int i = 0; i < nrun; i++) if (run_end[i] < tn) tn = run_end[i];
    for (int i = 0; i < nrun;) {
      if (run_end[i] == tn) {
        finished[run_part[i]]++;
        run_end[i] = run_end[nrun - 1]; run_part[i] = run_part[nrun - 1]; nrun--;
      } else {
        i++;
      }
    }
    t = tn;
  }
  free(started); free(finished); free(run_end); free(run_part); free(ready);
  return t;
}
