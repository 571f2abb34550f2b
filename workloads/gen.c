/*
 * Seeded synthetic DAG-task generator.
 *
 * Produces batches of DAG tasks in the layout the bound library ingests
 * (per-DAG node and edge offsets, DAG-local edge endpoints, per-node load
 * (WCET, in integer ticks) and maximum parallelism), plus explicit candidate
 * allocation bytes.  It holds none of the bound's arithmetic: it only draws
 * random graphs and random integers.  Both the CPU oracle and the GPU path
 * consume its output.
 *
 * Random source: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  DAG d of a batch with base
 * seed B draws from its own stream whose state starts at mix(B ^ mix(d)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline uint64_t rnext(rng_t* r) { r->s += GOLDEN; return mix64(r->s); }
/* uniform double in [0,1) with 53 random bits */
static inline double runif(rng_t* r) { return (double)(rnext(r) >> 11) * (1.0 / 9007199254740992.0); }
/* uniform integer in [a, b] (inclusive), multiply-shift on 32 random bits */
static inline int64_t rint_ab(rng_t* r, int64_t a, int64_t b) {
  uint64_t span = (uint64_t)(b - a) + 1u;
  if (span <= 0xFFFFFFFFull) return a + (int64_t)(((rnext(r) >> 32) * span) >> 32);
  return a + (int64_t)(rnext(r) % span);
}

/* Shape and distribution parameters of one workload.  Mirrored field by
 * field in workloads/__init__.py (ctypes). */
typedef struct {
  int32_t shape;        /* 0 ER over a random order, 1 layered, 2 mixed 50/50 ER/layered */
  int32_t nmin, nmax;   /* internal node count range (source/sink not counted) */
  int32_t n_logu;       /* 1: node count log-uniform in [nmin,nmax], else uniform */
  int32_t width_max;    /* layered: width of each layer U{1..width_max} */
  int32_t skip_min, skip_max; /* layered: skip edges span skip_min..skip_max layers */
  int32_t wcet_kind;    /* 0 uniform int, 1 log-uniform int, 2 lognormal rounded */
  int32_t pmin, pmax;   /* max parallelism U{pmin..pmax} */
  int32_t add_src_sink; /* 1: add one source and one sink node */
  int32_t permute_ids;  /* 1: node ids are a random permutation (not topological) */
  int32_t pad0;
  double p_er;          /* ER edge probability per ordered pair */
  double p_adj;         /* layered: edge probability per adjacent-layer pair */
  double p_skip;        /* layered: edge probability per skip pair */
  int64_t wmin, wmax;   /* WCET range for kinds 0 and 1 */
  double mu, sigma;     /* lognormal parameters for kind 2 */
} wl_spec;

/* growable int32 pair buffer */
typedef struct { int32_t* a; int64_t n, cap; } ibuf;
static int ib_push2(ibuf* b, int32_t x, int32_t y) {
  if (b->n + 2 > b->cap) {
    int64_t nc = b->cap ? b->cap * 2 : 1024;
    while (nc < b->n + 2) nc *= 2;
    int32_t* na = (int32_t*)realloc(b->a, (size_t)nc * sizeof(int32_t));
    if (!na) return -1;
    b->a = na; b->cap = nc;
  }
  b->a[b->n++] = x; b->a[b->n++] = y;
  return 0;
}

/* Visit the indices of successes of T Bernoulli(p) trials by geometric skips. */
typedef struct { rng_t* r; double lq; double p; int64_t pos, T; } bern_t;
static void bern_init(bern_t* b, rng_t* r, double p, int64_t T) {
  b->r = r; b->p = p; b->T = T; b->pos = -1;
  b->lq = (p > 0.0 && p < 1.0) ? log1p(-p) : 0.0;
}
static int64_t bern_next(bern_t* b) {
  if (b->p <= 0.0) return -1;
  if (b->p >= 1.0) { b->pos++; return b->pos < b->T ? b->pos : -1; }
  double u = runif(b->r);
  double g = floor(log1p(-u) / b->lq);
  if (g > (double)(b->T)) return -1;
  b->pos += 1 + (int64_t)g;
  return b->pos < b->T ? b->pos : -1;
}

typedef struct {
  int32_t n;       /* total nodes */
  ibuf edges;      /* (src, dst) pairs, DAG-local ids */
  int64_t* wcet;
  int32_t* par;
} gdag;

static int64_t draw_wcet(const wl_spec* s, rng_t* r) {
  if (s->wcet_kind == 0) return rint_ab(r, s->wmin, s->wmax);
  if (s->wcet_kind == 1) {
    double lo = log((double)s->wmin), hi = log((double)s->wmax + 1.0);
    int64_t v = (int64_t)floor(exp(lo + (hi - lo) * runif(r)));
    if (v < s->wmin) v = s->wmin;
    if (v > s->wmax) v = s->wmax;
    return v;
  }
  /* lognormal: Box-Muller normal draw */
  double u1 = runif(r), u2 = runif(r);
  double z = sqrt(-2.0 * log1p(-u1)) * cos(6.283185307179586 * u2);
  double x = exp(s->mu + s->sigma * z);
  int64_t v = (int64_t)floor(x + 0.5);
  if (v < 1) v = 1;
  if (v > 2147483647LL) v = 2147483647LL;
  return v;
}

/* Generate DAG number d.  Returns 0 or -1 on allocation failure. */
static int gen_one(const wl_spec* s, uint64_t base, int64_t d, gdag* g) {
  rng_t r = { mix64(base ^ mix64((uint64_t)d)) };
  int32_t nin;
  if (s->n_logu) {
    double lo = log((double)s->nmin), hi = log((double)s->nmax + 1.0);
    nin = (int32_t)floor(exp(lo + (hi - lo) * runif(&r)));
    if (nin < s->nmin) nin = s->nmin;
    if (nin > s->nmax) nin = s->nmax;
  } else {
    nin = (int32_t)rint_ab(&r, s->nmin, s->nmax);
  }
  int shape = s->shape;
  if (shape == 2) shape = (rnext(&r) >> 63) ? 1 : 0;
  int extra = s->add_src_sink ? 2 : 0;
  int32_t n = nin + extra;
  g->n = n;
  g->edges.n = 0;
  /* internal node k (0..nin-1) gets local id ids[k + (extra?1:0)] */
  int32_t* ids = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* indeg = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  int32_t* outdeg = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  g->wcet = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  g->par = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!ids || !indeg || !outdeg || !g->wcet || !g->par) return -1;
  for (int32_t i = 0; i < n; i++) ids[i] = i;
  if (s->permute_ids)
    for (int32_t i = n - 1; i > 0; i--) {
      int32_t j = (int32_t)rint_ab(&r, 0, i);
      int32_t t = ids[i]; ids[i] = ids[j]; ids[j] = t;
    }
  const int32_t* in_id = ids + (extra ? 1 : 0);
  int rc = 0;
  if (shape == 0) {
    /* ER: internal index order is the topological order; pairs (i<j) */
    int64_t T = (int64_t)nin * (nin - 1) / 2;
    bern_t b; bern_init(&b, &r, s->p_er, T);
    int64_t k; int32_t i = 0; int64_t rowstart = 0; /* linear index of (i, i+1) */
    while ((k = bern_next(&b)) >= 0) {
      while (k >= rowstart + (nin - 1 - i)) { rowstart += nin - 1 - i; i++; }
      int32_t j = i + 1 + (int32_t)(k - rowstart);
      rc |= ib_push2(&g->edges, in_id[i], in_id[j]);
      outdeg[in_id[i]]++; indeg[in_id[j]]++;
    }
  } else {
    /* layered: widths U{1..width_max}; the last layer is truncated */
    int32_t* lstart = (int32_t*)malloc((size_t)(nin + 1) * sizeof(int32_t));
    if (!lstart) return -1;
    int32_t nl = 0, pos = 0;
    while (pos < nin) {
      int32_t w = (int32_t)rint_ab(&r, 1, s->width_max);
      if (w > nin - pos) w = nin - pos;
      lstart[nl++] = pos; pos += w;
    }
    lstart[nl] = nin;
    for (int32_t L = 0; L + 1 < nl; L++) {
      int32_t a0 = lstart[L], aw = lstart[L + 1] - a0;
      int32_t b0 = lstart[L + 1], bw = lstart[L + 2] - b0;
      bern_t b; bern_init(&b, &r, s->p_adj, (int64_t)aw * bw);
      int64_t k;
      while ((k = bern_next(&b)) >= 0) {
        int32_t u = in_id[a0 + (int32_t)(k / bw)], v = in_id[b0 + (int32_t)(k % bw)];
        rc |= ib_push2(&g->edges, u, v); outdeg[u]++; indeg[v]++;
      }
      if (s->p_skip > 0.0)
        for (int32_t span = s->skip_min; span <= s->skip_max; span++) {
          if (L + span >= nl) break;
          int32_t c0 = lstart[L + span], cw = lstart[L + span + 1] - c0;
          bern_t bs; bern_init(&bs, &r, s->p_skip, (int64_t)aw * cw);
          while ((k = bern_next(&bs)) >= 0) {
            int32_t u = in_id[a0 + (int32_t)(k / cw)], v = in_id[c0 + (int32_t)(k % cw)];
            rc |= ib_push2(&g->edges, u, v); outdeg[u]++; indeg[v]++;
          }
        }
    }
    free(lstart);
  }
  if (extra) {
    int32_t src = ids[0], snk = ids[n - 1];
    for (int32_t k = 0; k < nin; k++) {
      int32_t v = in_id[k];
      if (indeg[v] == 0) rc |= ib_push2(&g->edges, src, v);
    }
    for (int32_t k = 0; k < nin; k++) {
      int32_t v = in_id[k];
      if (outdeg[v] == 0) rc |= ib_push2(&g->edges, v, snk);
    }
  }
  /* per-node load and parallelism, drawn in local-id order */
  for (int32_t v = 0; v < n; v++) {
    g->wcet[v] = draw_wcet(s, &r);
    g->par[v] = (int32_t)rint_ab(&r, s->pmin, s->pmax);
  }
  free(ids); free(indeg); free(outdeg);
  return rc ? -1 : 0;
}

/* A generated batch held between the two calls below. */
typedef struct {
  int64_t count, total_nodes, total_edges;
  int64_t* nn;   /* [count] */
  int64_t* ne;   /* [count] */
  gdag* dags;    /* [count] */
} wl_batch;

/* Generate DAGs d0 .. d0+count-1 of a workload.  On success returns a handle
 * whose totals are filled in; copy out with wl_batch_take(). */
wl_batch* wl_batch_generate(const wl_spec* s, uint64_t base, int64_t d0, int64_t count,
                            int32_t nthreads) {
  if (count < 0) return NULL;
  wl_batch* b = (wl_batch*)calloc(1, sizeof(wl_batch));
  if (!b) return NULL;
  b->count = count;
  b->nn = (int64_t*)calloc((size_t)(count + 1), sizeof(int64_t));
  b->ne = (int64_t*)calloc((size_t)(count + 1), sizeof(int64_t));
  b->dags = (gdag*)calloc((size_t)(count + 1), sizeof(gdag));
  if (!b->nn || !b->ne || !b->dags) return NULL;
  int failed = 0;
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1) reduction(| : failed)
  for (int64_t i = 0; i < count; i++) {
    if (gen_one(s, base, d0 + i, &b->dags[i]) != 0) failed |= 1;
    b->nn[i] = b->dags[i].n;
    b->ne[i] = b->dags[i].edges.n / 2;
  }
  if (failed) return NULL;
  for (int64_t i = 0; i < count; i++) { b->total_nodes += b->nn[i]; b->total_edges += b->ne[i]; }
  return b;
}

int64_t wl_batch_nodes(const wl_batch* b) { return b->total_nodes; }
int64_t wl_batch_edges(const wl_batch* b) { return b->total_edges; }

/* Copy the batch into caller arrays: node_off/edge_off [count+1], src/dst
 * [edges], wcet/par [nodes].  Frees the handle. */
void wl_batch_take(wl_batch* b, int64_t* node_off, int64_t* edge_off, int32_t* src,
                   int32_t* dst, int64_t* wcet, int32_t* par, int32_t nthreads) {
  node_off[0] = 0; edge_off[0] = 0;
  for (int64_t i = 0; i < b->count; i++) {
    node_off[i + 1] = node_off[i] + b->nn[i];
    edge_off[i + 1] = edge_off[i] + b->ne[i];
  }
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < b->count; i++) {
    gdag* g = &b->dags[i];
    int64_t e0 = edge_off[i], n0 = node_off[i];
    for (int64_t k = 0; k < b->ne[i]; k++) {
      src[e0 + k] = g->edges.a[2 * k];
      dst[e0 + k] = g->edges.a[2 * k + 1];
    }
    memcpy(wcet + n0, g->wcet, (size_t)g->n * sizeof(int64_t));
    memcpy(par + n0, g->par, (size_t)g->n * sizeof(int32_t));
    free(g->edges.a); free(g->wcet); free(g->par);
  }
  free(b->nn); free(b->ne); free(b->dags); free(b);
}

void wl_batch_free(wl_batch* b) {
  if (!b) return;
  for (int64_t i = 0; i < b->count; i++) {
    free(b->dags[i].edges.a); free(b->dags[i].wcet); free(b->dags[i].par);
  }
  free(b->nn); free(b->ne); free(b->dags); free(b);
}

/* ------------------------------------------------------------------------
 * Candidate allocations.
 *
 * Counter-based draw (random access by (seed, d, c, v)):
 *   key  = mix(seed ^ mix(d * GOLDEN))
 *   word = mix(key ^ ((c << 32) | (v >> 2)))
 *   h16  = (word >> (16 * (v & 3))) & 0xFFFF
 *   r    = 1 + ((h16 * range) >> 16),  range = min(p_v, M, 255)
 * Candidate c = 0 is all zeros (the method's own parallelism rule).
 * ------------------------------------------------------------------------ */
static inline uint32_t cand_r(uint64_t seed, uint64_t d, uint64_t c, uint64_t v, uint32_t range) {
  uint64_t key = mix64(seed ^ mix64(d * GOLDEN));
  uint64_t word = mix64(key ^ ((c << 32) | (v >> 2)));
  uint32_t h16 = (uint32_t)((word >> (16 * (v & 3))) & 0xFFFFu);
  return 1u + ((h16 * range) >> 16);
}

/* Fill explicit candidate bytes for DAGs d0..d0+count-1: the byte of (d,c,v)
 * sits at K*node_off[d] + c*N_d + v (node_off relative to DAG d0). */
void wl_alloc_bytes(uint64_t seed, int64_t d0, int64_t count, const int64_t* node_off,
                    const int32_t* par, int32_t M, int32_t K, uint8_t* out, int32_t nthreads) {
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < count; i++) {
    int64_t n0 = node_off[i], nd = node_off[i + 1] - n0;
    uint8_t* o = out + (int64_t)K * n0;
    memset(o, 0, (size_t)nd);
    for (int32_t c = 1; c < K; c++)
      for (int64_t v = 0; v < nd; v++) {
        int64_t p = par[n0 + v];
        uint32_t range = (uint32_t)(p < M ? p : M);
        if (range > 255u) range = 255u;
        o[(int64_t)c * nd + v] = (uint8_t)cand_r(seed, (uint64_t)(d0 + i), (uint64_t)c, (uint64_t)v, range);
      }
  }
}

/* The bytes of listed candidates: row i of DAG d holds the bytes of
 * candidate list[d * L + i] (same draw as wl_alloc_bytes), at
 * L * node_off[d] + i * N_d + v (node_off relative to DAG d0). */
void wl_alloc_bytes_list(uint64_t seed, int64_t d0, int64_t count, const int64_t* node_off,
                         const int32_t* par, int32_t M, int32_t L, const int32_t* list, uint8_t* out,
                         int32_t nthreads) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < count; i++) {
    int64_t n0 = node_off[i], nd = node_off[i + 1] - n0;
    uint8_t* o = out + (int64_t)L * n0;
    for (int32_t j = 0; j < L; j++) {
      int64_t c = list[i * L + j];
      for (int64_t v = 0; v < nd; v++) {
        int64_t p = par[n0 + v];
        uint32_t range = (uint32_t)(p < M ? p : M);
        if (range > 255u) range = 255u;
        o[(int64_t)j * nd + v] = c == 0 ? 0 : (uint8_t)cand_r(seed, (uint64_t)(d0 + i), (uint64_t)c, (uint64_t)v, range);
      }
    }
  }
}
