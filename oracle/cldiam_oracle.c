/*
 * CPU oracle for the CL-DIAM decomposition, quotient graph and diameter
 * estimate.  TEST INFRASTRUCTURE ONLY: it exists to check the GPU library.
 * Only the test suite, the smoke entry point and the benchmark's CPU-baseline
 * leg may load it; the product path never does.
 *
 * Plain, sequential and slow on purpose.  It follows Ceccarello,
 * Pietracaprina, Pucci, Upfal, "A practical parallel algorithm for diameter
 * approximation of massive weighted graphs" (arXiv:1506.03265):
 *   - decomposition: Algorithm 1 (CLUSTER) with the Delta-growing step and
 *     Procedure Contract of Section 3;
 *   - quotient graph and estimate: Section 4;
 *   - single-source shortest paths for the Delta-stepping 2-approximation
 *     baseline of Section 5 (exact distances, here by Dijkstra).
 * It shares no code with the GPU library.
 *
 * Row offsets are 64-bit throughout, so the oracle also takes graphs of more
 * than 2^31 arcs (one GPU's share of the billion-edge graphs of Section 5).
 *
 * Readings taken where the paper is silent or ambiguous (each one is pinned
 * by a test against brute force or the mathematics):
 *   log is log2; gamma = 4 ln 2; the stage loop runs while
 *   |U| >= ceil(8 tau log2 n), U is not empty and n > 1 (a single node,
 *   where log2 n = 0 makes the selection probability 0, is its own cluster); the selection probability is
 *   p = ((gamma*tau)*log2 n)/|U| in IEEE double and node v of stage s is a new
 *   center iff word 0 of Philox4x32-10(counter (v, s, 0, 0), key seed) is
 *   below T = floor(p*2^32) (T = 2^32 when p >= 1).
 *   PartialGrowth runs each Delta to its fixpoint; ties between equal
 *   distances go to the smaller center id (lexicographic (d, c) minimum),
 *   which is the fixpoint of repeated Delta-growing steps.
 *   The contracted graph is not built: every node assigned in an earlier
 *   stage acts as a source at distance 0 with its cluster's label, which is
 *   what Contract's rewired edges (c_u, v) of weight w(u,v) provide.
 *   Delta starts at floor(sum of weights / arcs) unless given, persists across
 *   stages and doubles only while fewer than half of the uncovered nodes are
 *   covered and some uncovered node is still reachable (otherwise the stage
 *   keeps what it covered); Delta above 2^31 is an overflow error.
 *   The distance recorded for a node assigned in stage s is
 *   D = d + R_prev(c), where d is its stage-local growth distance and
 *   R_prev(c) the radius bound of its cluster after stage s-1, so D bounds
 *   dist(c, v) from above; the estimate is Phi(G_C) + 2 max D.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_EOVERFLOW -3
#define OR_ESTAGES -4

#define INF64 (~(uint64_t)0)
#define DELTA_MAX ((uint64_t)1 << 31)
#define MAX_STAGES 4096

/* ------------------------------------------------- Philox4x32-10 (SC'11) -- */

static void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int round = 0; round < 10; ++round) {
    if (round) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t a = (uint64_t)0xD2511F53u * c[0];
    uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t x0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
    uint32_t x2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)b;
    c[3] = (uint32_t)a;
    c[0] = x0;
    c[2] = x2;
  }
}

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  philox4x32_10(c, key[0], key[1]);
  memcpy(out, c, 16);
}

/* ------------------------------------------------------ binary min-heap -- */

typedef struct { uint64_t d; uint32_t c; uint32_t v; } item_t;
typedef struct { item_t *a; int64_t len, cap; } heap_t;

static int less(const item_t *x, const item_t *y) {
  return x->d < y->d || (x->d == y->d && x->c < y->c);
}

static int heap_push(heap_t *h, uint64_t d, uint32_t c, uint32_t v) {
  if (h->len == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 1024;
    item_t *na = realloc(h->a, (size_t)nc * sizeof(item_t));
    if (!na) return -1;
    h->a = na; h->cap = nc;
  }
  int64_t i = h->len++;
  item_t it = {d, c, v};
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!less(&it, &h->a[p])) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i] = it;
  return 0;
}

static item_t heap_pop(heap_t *h) {
  item_t top = h->a[0], last = h->a[--h->len];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    const item_t *cur = &last;
    if (l < h->len && less(&h->a[l], cur)) { s = l; cur = &h->a[l]; }
    if (r < h->len && less(&h->a[r], cur)) s = r;
    if (s == i) break;
    h->a[i] = h->a[s];
    i = s;
  }
  if (h->len) h->a[i] = last;
  return top;
}

/* ---------------------------------------------------------- decomposition -- */

typedef struct {
  int32_t stages;        /* executed stages of the outer loop */
  int32_t levels;        /* PartialGrowth calls (one per Delta value tried) */
  uint32_t delta0;
  uint32_t delta_end;
  int32_t stop;          /* ceil(8 tau log2 n) */
  int32_t num_clusters;
  int32_t singletons;
  int32_t pad;
  uint64_t radius;       /* max over nodes of D */
  /* work counts of this sequential run, used for algorithmic bytes */
  uint64_t sum_uncovered;  /* sum over stages of |U_s| */
  uint64_t sum_acting;     /* nodes whose rows are read: settled + boundary sources */
  uint64_t sum_arcs;       /* arcs read from those rows */
  uint64_t sum_covered;    /* nodes assigned during stages */
} or_stats;

/* per-stage log, caller arrays of length log_cap (may be NULL) */
typedef struct {
  int32_t *uncovered;   /* |U_s| */
  int32_t *centers;     /* new centers of stage s */
  int32_t *covered;     /* nodes assigned in stage s (centers included) */
  uint32_t *delta;      /* Delta in force when stage s assigned */
  int32_t cap;
} or_stage_log;

uint32_t or_default_delta(int64_t m, const uint32_t *w) {
  if (m <= 0) return 1;
  uint64_t s = 0;
  for (int64_t i = 0; i < m; ++i) s += w[i];
  uint64_t d = s / (uint64_t)m;
  return d < 1 ? 1u : (uint32_t)(d > 0xffffffffu ? 0xffffffffu : d);
}

int or_decompose(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *w,
                 uint32_t tau, uint32_t delta0, uint64_t seed,
                 int32_t *cluster, uint64_t *D, or_stats *st, or_stage_log *lg) {
  if (n < 1 || tau < 1 || !row_ptr || !cluster || !D || !st) return OR_EINVAL;
  memset(st, 0, sizeof *st);
  int64_t m = row_ptr[n];
  uint64_t delta = delta0 ? delta0 : or_default_delta(m, w);
  st->delta0 = (uint32_t)delta;
  if (delta > DELTA_MAX) return OR_EOVERFLOW;

  const double gamma = 4.0 * M_LN2;
  const double L = log2((double)n);
  const int64_t stop = (int64_t)ceil(8.0 * tau * L);
  st->stop = (int32_t)stop;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);

  int32_t *U = malloc((size_t)n * 4);
  int32_t *settled = malloc((size_t)n * 4);   /* stage stamp of settlement */
  int32_t *srcmark = malloc((size_t)n * 4);   /* stage stamp of boundary sources */
  uint32_t *loc = malloc((size_t)n * 4);
  uint32_t *lab = malloc((size_t)n * 4);
  uint64_t *R = calloc((size_t)n, 8);
  int32_t *newly = malloc((size_t)n * 4);
  heap_t h = {0};
  int rc = OR_OK;
  if (!U || !settled || !srcmark || !loc || !lab || !R || !newly) { rc = OR_ENOMEM; goto done; }
  for (int32_t v = 0; v < n; ++v) { U[v] = v; cluster[v] = -1; D[v] = 0; settled[v] = -1; srcmark[v] = -1; }
  int64_t nU = n;
  int32_t s = 0;

  while (n > 1 && nU > 0 && nU >= stop) {
    if (s >= MAX_STAGES) { rc = OR_ESTAGES; goto done; }
    /* new centers: each uncovered node independently with probability p */
    double p = gamma * tau * L / (double)nU;
    uint64_t T = p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(p * 4294967296.0);
    h.len = 0;
    int32_t ncent = 0;
    for (int64_t i = 0; i < nU; ++i) {
      uint32_t v = (uint32_t)U[i];
      uint32_t c[4] = {v, (uint32_t)s, 0, 0};
      philox4x32_10(c, k0, k1);
      if ((uint64_t)c[0] < T) {
        if (heap_push(&h, 0, v, v)) { rc = OR_ENOMEM; goto done; }
        ncent++;
      }
    }
    /* previously assigned nodes are sources at distance 0 (Contract); their
     * first relaxations into U are generated from U's side */
    for (int64_t i = 0; i < nU; ++i) {
      int32_t v = U[i];
      for (int64_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
        int32_t u = col[a];
        if (cluster[u] < 0) continue;
        if (heap_push(&h, w[a], (uint32_t)cluster[u], (uint32_t)v)) { rc = OR_ENOMEM; goto done; }
        if (srcmark[u] != s) {
          srcmark[u] = s;
          st->sum_acting++;
          st->sum_arcs += (uint64_t)(row_ptr[u + 1] - row_ptr[u]);
        }
      }
    }
    int64_t covered = 0;
    int32_t nnew = 0;
    /* PartialGrowth(Delta) to its fixpoint = lexicographic Dijkstra limited to
     * distance <= Delta; entries beyond Delta stay queued for a larger Delta */
    for (;;) {
      st->levels++;
      while (h.len && h.a[0].d <= delta) {
        item_t it = heap_pop(&h);
        if (settled[it.v] == s) continue;
        settled[it.v] = s;
        loc[it.v] = (uint32_t)it.d;
        lab[it.v] = it.c;
        newly[nnew++] = (int32_t)it.v;
        covered++;
        st->sum_acting++;
        st->sum_arcs += (uint64_t)(row_ptr[it.v + 1] - row_ptr[it.v]);
        for (int64_t a = row_ptr[it.v]; a < row_ptr[it.v + 1]; ++a) {
          int32_t x = col[a];
          if (cluster[x] >= 0 || settled[x] == s) continue;
          if (heap_push(&h, it.d + w[a], it.c, (uint32_t)x)) { rc = OR_ENOMEM; goto done; }
        }
      }
      while (h.len && settled[h.a[0].v] == s) heap_pop(&h);
      if (2 * covered >= nU) break;   /* at least half of U covered */
      if (h.len == 0) break;          /* no uncovered node reachable at any Delta */
      if (2 * delta > DELTA_MAX) { rc = OR_EOVERFLOW; goto done; }
      delta *= 2;
    }
    /* assign: D from the radius bounds of the previous stage, then update */
    for (int32_t i = 0; i < nnew; ++i) {
      int32_t v = newly[i];
      cluster[v] = (int32_t)lab[v];
      D[v] = (uint64_t)loc[v] + R[lab[v]];
    }
    for (int32_t i = 0; i < nnew; ++i) {
      int32_t v = newly[i];
      if (D[v] > R[lab[v]]) R[lab[v]] = D[v];
    }
    if (lg && s < lg->cap) {
      if (lg->uncovered) lg->uncovered[s] = (int32_t)nU;
      if (lg->centers) lg->centers[s] = ncent;
      if (lg->covered) lg->covered[s] = nnew;
      if (lg->delta) lg->delta[s] = (uint32_t)delta;
    }
    st->sum_uncovered += (uint64_t)nU;
    st->sum_covered += (uint64_t)nnew;
    int64_t k = 0;
    for (int64_t i = 0; i < nU; ++i)
      if (cluster[U[i]] < 0) U[k++] = U[i];
    nU = k;
    s++;
  }
  /* the few nodes left become singleton clusters */
  for (int64_t i = 0; i < nU; ++i) { cluster[U[i]] = U[i]; D[U[i]] = 0; }
  st->singletons = (int32_t)nU;
  st->stages = s;
  st->delta_end = (uint32_t)delta;
  for (int32_t v = 0; v < n; ++v) {
    if (cluster[v] == v) st->num_clusters++;
    if (D[v] > st->radius) st->radius = D[v];
  }
done:
  free(U); free(settled); free(srcmark); free(loc); free(lab); free(R); free(newly); free(h.a);
  return rc;
}

/* ------------------------------------ decomposition, literal growth steps -- */

/*
 * CLUSTER(G, tau) with Procedure PartialGrowth of Algorithm 1 taken
 * literally: each Delta-growing step is synchronous (all offers of a step are
 * computed from the state before the step), a node accepts an offer only if
 * its distance is strictly smaller than the node's current one (among the
 * offers of one step, the smallest distance and then the smallest center
 * wins), and PartialGrowth stops as soon as a step updates no state or at
 * least half of the stage's uncovered nodes are covered (threshold
 * |V_i - C_i| / 2, the outer loop's), or after step_cap steps (0 = no cap).
 * The outer loop doubles Delta one step at a time while fewer than half are
 * covered; a stage whose growth has stopped with no node reachable at any
 * Delta keeps what it covered.  If the new centers alone cover half, the
 * stage performs no step.
 *
 * Counters (the paper's experiments report rounds and work):
 *   rounds   = growing steps executed (including a final step that updates
 *              nothing);
 *   updates  = node states changed, summed over steps;
 *   messages = offers sent, summed over steps: in a step, each node of the
 *              active set sends one offer over every arc with d_u + w <=
 *              Delta.  The active set of a step is the set of nodes updated
 *              by the previous step; in the first step of a stage it is the
 *              new centers plus the previous stage's carried sources; in the
 *              first step after Delta doubles it is the nodes still active plus
 *              every node that, at a step of the previous Delta, had an arc
 *              with d_u + w > Delta.  The carried sources of a stage are the
 *              nodes still active when its growth stopped plus the nodes found
 *              with such an arc at the last Delta.  Nodes assigned in earlier
 *              stages send at distance 0 with their cluster's label (Contract).
 */
typedef struct {
  uint64_t rounds;
  uint64_t messages;
  uint64_t updates;
} or_step_stats;

int or_decompose_steps(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *w,
                       uint32_t tau, uint32_t delta0, uint64_t seed, uint32_t step_cap,
                       int32_t *cluster, uint64_t *D, or_stats *st, or_step_stats *ss, or_stage_log *lg) {
  if (n < 1 || tau < 1 || !row_ptr || !cluster || !D || !st || !ss) return OR_EINVAL;
  memset(st, 0, sizeof *st);
  memset(ss, 0, sizeof *ss);
  int64_t m = row_ptr[n];
  uint64_t delta = delta0 ? delta0 : or_default_delta(m, w);
  st->delta0 = (uint32_t)delta;
  if (delta > DELTA_MAX) return OR_EOVERFLOW;
  const double gamma = 4.0 * M_LN2;
  const double L = log2((double)n);
  const int64_t stop = (int64_t)ceil(8.0 * tau * L);
  st->stop = (int32_t)stop;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);

  const uint64_t UNSET = INF64;
  int32_t *U = malloc((size_t)n * 4);
  uint64_t *dist = malloc((size_t)n * 8);      /* stage-local d (UNSET = infinity) */
  uint32_t *lab = malloc((size_t)n * 4);       /* c */
  uint64_t *R = calloc((size_t)n, 8);
  int32_t *act = malloc((size_t)n * 4), *nxt = malloc((size_t)n * 4), *blk = malloc((size_t)n * 4);
  int64_t *amark = malloc((size_t)n * 8);      /* membership stamps of the three sets */
  int64_t *nmark = malloc((size_t)n * 8);
  int64_t *bmark = malloc((size_t)n * 8);
  uint64_t *bd = malloc((size_t)n * 8);        /* best offer of the current step */
  uint32_t *bl = malloc((size_t)n * 4);
  int rc = OR_OK;
  if (!U || !dist || !lab || !R || !act || !nxt || !blk || !amark || !nmark || !bmark || !bd || !bl) {
    rc = OR_ENOMEM;
    goto done;
  }
  for (int32_t v = 0; v < n; ++v) {
    U[v] = v; cluster[v] = -1; D[v] = 0; dist[v] = UNSET; lab[v] = 0;
    amark[v] = nmark[v] = bmark[v] = -1;
  }
  int64_t nU = n, nact = 0, nblk = 0;
  int64_t stamp = 0;       /* increases for every new set */
  int64_t aset = ++stamp;  /* stamp of the active set */
  int64_t bset = ++stamp;  /* stamp of the set of nodes with an arc beyond Delta */
  int32_t s = 0;

  while (n > 1 && nU > 0 && nU >= stop) {
    if (s >= MAX_STAGES) { rc = OR_ESTAGES; goto done; }
    double p = gamma * tau * L / (double)nU;
    uint64_t T = p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(p * 4294967296.0);
    int64_t covered = 0;
    int32_t ncent = 0;
    /* carried sources stay in the active set; the new centers join it */
    for (int64_t i = 0; i < nU; ++i) {
      uint32_t v = (uint32_t)U[i];
      uint32_t c[4] = {v, (uint32_t)s, 0, 0};
      philox4x32_10(c, k0, k1);
      if ((uint64_t)c[0] < T) {
        dist[v] = 0;
        lab[v] = v;
        ncent++;
        covered++;
        if (amark[v] != aset) { amark[v] = aset; act[nact++] = (int32_t)v; }
      }
    }
    while (2 * covered < nU) {
      st->levels++;
      uint32_t steps = 0;
      int moved = 0;
      /* PartialGrowth(G_i, Delta) */
      for (;;) {
        ss->rounds++;
        steps++;
        st->sum_acting += (uint64_t)nact;
        int64_t nset = ++stamp, nn = 0;
        for (int64_t i = 0; i < nact; ++i) {
          int32_t u = act[i];
          uint64_t du = dist[u];
          int heavy = 0;
          for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a) {
            uint64_t cand = du + w[a];
            if (cand > delta) { heavy = 1; continue; }
            ss->messages++;
            st->sum_arcs++;
            int32_t v = col[a];
            if (cand >= dist[v]) continue;        /* only a strictly smaller distance */
            if (nmark[v] != nset) {
              nmark[v] = nset;
              nxt[nn++] = v;
              bd[v] = cand;
              bl[v] = lab[u];
            } else if (cand < bd[v] || (cand == bd[v] && lab[u] < bl[v])) {
              bd[v] = cand;
              bl[v] = lab[u];
            }
          }
          if (heavy && bmark[u] != bset) { bmark[u] = bset; blk[nblk++] = u; }
        }
        for (int64_t i = 0; i < nn; ++i) {
          int32_t v = nxt[i];
          if (dist[v] == UNSET) covered++;
          dist[v] = bd[v];
          lab[v] = bl[v];
        }
        ss->updates += (uint64_t)nn;
        /* the updated nodes are the next active set */
        aset = ++stamp;
        for (int64_t i = 0; i < nn; ++i) { act[i] = nxt[i]; amark[act[i]] = aset; }
        nact = nn;
        moved = nn > 0;
        if (!moved || 2 * covered >= nU || (step_cap && steps >= step_cap)) break;
      }
      if (2 * covered >= nU) break;
      if (!moved) {
        /* fixpoint at this Delta: is any uncovered node reachable at all? */
        int reach = 0;
        for (int64_t i = 0; i < nblk && !reach; ++i) {
          int32_t u = blk[i];
          for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a)
            if (dist[col[a]] == UNSET) { reach = 1; break; }
        }
        if (!reach) break;
      }
      if (2 * delta > DELTA_MAX) { rc = OR_EOVERFLOW; goto done; }
      delta *= 2;
      /* the next PartialGrowth starts from the active nodes and every node
       * that had an arc beyond the old Delta */
      for (int64_t i = 0; i < nblk; ++i) {
        int32_t u = blk[i];
        if (amark[u] != aset) { amark[u] = aset; act[nact++] = u; }
      }
      bset = ++stamp;
      nblk = 0;
    }
    /* assign the covered nodes of U */
    int32_t nnew = 0;
    for (int64_t i = 0; i < nU; ++i) {
      int32_t v = U[i];
      if (dist[v] == UNSET) continue;
      cluster[v] = (int32_t)lab[v];
      D[v] = dist[v] + R[lab[v]];
      nnew++;
    }
    for (int64_t i = 0; i < nU; ++i) {
      int32_t v = U[i];
      if (cluster[v] >= 0 && D[v] > R[cluster[v]]) R[cluster[v]] = D[v];
    }
    if (lg && s < lg->cap) {
      if (lg->uncovered) lg->uncovered[s] = (int32_t)nU;
      if (lg->centers) lg->centers[s] = ncent;
      if (lg->covered) lg->covered[s] = nnew;
      if (lg->delta) lg->delta[s] = (uint32_t)delta;
    }
    st->sum_uncovered += (uint64_t)nU;
    st->sum_covered += (uint64_t)nnew;
    /* Contract: assigned nodes become distance-0 sources with their label */
    for (int64_t i = 0; i < nU; ++i) {
      int32_t v = U[i];
      if (cluster[v] >= 0) { dist[v] = 0; lab[v] = (uint32_t)cluster[v]; }
    }
    /* carried sources: the active set plus the nodes with an arc beyond Delta */
    for (int64_t i = 0; i < nblk; ++i) {
      int32_t u = blk[i];
      if (amark[u] != aset) { amark[u] = aset; act[nact++] = u; }
    }
    bset = ++stamp;
    nblk = 0;
    int64_t k = 0;
    for (int64_t i = 0; i < nU; ++i)
      if (cluster[U[i]] < 0) U[k++] = U[i];
    nU = k;
    s++;
  }
  for (int64_t i = 0; i < nU; ++i) { cluster[U[i]] = U[i]; D[U[i]] = 0; }
  st->singletons = (int32_t)nU;
  st->stages = s;
  st->delta_end = (uint32_t)delta;
  for (int32_t v = 0; v < n; ++v) {
    if (cluster[v] == v) st->num_clusters++;
    if (D[v] > st->radius) st->radius = D[v];
  }
done:
  free(U); free(dist); free(lab); free(R); free(act); free(nxt); free(blk);
  free(amark); free(nmark); free(bmark); free(bd); free(bl);
  return rc;
}

/* ------------------------------------------------ decomposition, CLUSTER2 -- */

/*
 * CLUSTER2(G, tau) of Algorithm 2 (Section 4).  R_CL is the radius bound
 * max D of CLUSTER(G, tau) above (same tau, seed and initial Delta); every
 * growth uses Delta2 = 2 R_CL.  Iterations i = 1 .. ceil(log2 n): each
 * uncovered node becomes a new center with probability 2^i / n (word 0 of
 * Philox4x32-10(counter (v, i, 0, 1), key seed) below floor(p 2^32), 2^32
 * once p >= 1, so the last iteration takes every uncovered node); then all
 * clusters grow to the fixpoint of Delta2-growing steps (PartialGrowth2,
 * lexicographic (d, c) minimum as in CLUSTER).  Procedure Contract2 is
 * implicit: a node u assigned in iteration i-1 at growth distance d_u offers
 * its cluster's label at distance d_u + w - Delta2 to every unassigned
 * neighbour over an edge with w <= Delta2 (such an edge has d_u + w > Delta2,
 * or the neighbour would have been reached); that is the rescaled edge
 * (c_u, v).  A node reached in iteration i by a cluster whose center was
 * drawn in iteration j has D = d + Delta2 (i - j): the length of a path from
 * the center, since each contraction shortens the paths behind it by exactly
 * Delta2.  Delta2 above 2^31 is an overflow error.  Stats: stages =
 * iterations, levels = iterations, delta0 = the CLUSTER run's, delta_end =
 * Delta2, radius = max D; *radius1 = R_CL.
 */
int or_decompose_cluster2(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *w,
                          uint32_t tau, uint32_t delta0, uint64_t seed,
                          int32_t *cluster, uint64_t *D, or_stats *st, uint64_t *radius1, or_stage_log *lg) {
  if (n < 1 || tau < 1 || !row_ptr || !cluster || !D || !st || !radius1) return OR_EINVAL;
  or_stats st1;
  int rc = or_decompose(n, row_ptr, col, w, tau, delta0, seed, cluster, D, &st1, NULL);
  if (rc != OR_OK) return rc;
  memset(st, 0, sizeof *st);
  st->delta0 = st1.delta0;
  st->stop = st1.stop;
  *radius1 = st1.radius;
  const uint64_t d2 = 2 * st1.radius;
  if (d2 > DELTA_MAX) return OR_EOVERFLOW;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  int32_t iters = 0;
  while (((int64_t)1 << iters) < (int64_t)n) iters++;   /* ceil(log2 n) */

  int32_t *U = malloc((size_t)n * 4);
  int32_t *settled = malloc((size_t)n * 4);
  uint32_t *loc = malloc((size_t)n * 4);
  uint32_t *lab = malloc((size_t)n * 4);
  int32_t *birth = malloc((size_t)n * 4);
  int32_t *prev = malloc((size_t)n * 4), *cur = malloc((size_t)n * 4);
  heap_t h = {0};
  if (!U || !settled || !loc || !lab || !birth || !prev || !cur) { rc = OR_ENOMEM; goto done; }
  for (int32_t v = 0; v < n; ++v) { U[v] = v; cluster[v] = -1; D[v] = 0; settled[v] = 0; birth[v] = 0; }
  int64_t nU = n, nprev = 0;
  for (int32_t i = 1; i <= iters; ++i) {
    const double p = ldexp(1.0, i) / (double)n;
    const uint64_t T = p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(p * 4294967296.0);
    h.len = 0;
    int32_t ncent = 0;
    for (int64_t k = 0; k < nU; ++k) {
      uint32_t v = (uint32_t)U[k];
      uint32_t c[4] = {v, (uint32_t)i, 0, 1};
      philox4x32_10(c, k0, k1);
      if ((uint64_t)c[0] < T) {
        birth[v] = i;
        if (heap_push(&h, 0, v, v)) { rc = OR_ENOMEM; goto done; }
        ncent++;
      }
    }
    /* Contract2's rescaled edges out of the clusters grown last iteration */
    for (int64_t k = 0; k < nprev; ++k) {
      int32_t u = prev[k];
      for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a) {
        int32_t v = col[a];
        if (cluster[v] >= 0 || w[a] > d2) continue;
        if (heap_push(&h, (uint64_t)loc[u] + w[a] - d2, (uint32_t)cluster[u], (uint32_t)v)) {
          rc = OR_ENOMEM;
          goto done;
        }
      }
    }
    /* PartialGrowth2 to the fixpoint: lexicographic Dijkstra within Delta2 */
    int64_t ncur = 0;
    while (h.len) {
      item_t it = heap_pop(&h);
      if (it.d > d2) break;
      if (settled[it.v] == i) continue;
      settled[it.v] = i;
      loc[it.v] = (uint32_t)it.d;
      lab[it.v] = it.c;
      cur[ncur++] = (int32_t)it.v;
      for (int64_t a = row_ptr[it.v]; a < row_ptr[it.v + 1]; ++a) {
        int32_t x = col[a];
        if (cluster[x] >= 0 || settled[x] == i) continue;
        if (it.d + w[a] > d2) continue;
        if (heap_push(&h, it.d + w[a], it.c, (uint32_t)x)) { rc = OR_ENOMEM; goto done; }
      }
    }
    uint64_t covered = 0;
    for (int64_t k = 0; k < ncur; ++k) {
      int32_t v = cur[k];
      cluster[v] = (int32_t)lab[v];
      D[v] = (uint64_t)loc[v] + d2 * (uint64_t)(i - birth[lab[v]]);
      covered++;
    }
    if (lg && i - 1 < lg->cap) {
      if (lg->uncovered) lg->uncovered[i - 1] = (int32_t)nU;
      if (lg->centers) lg->centers[i - 1] = ncent;
      if (lg->covered) lg->covered[i - 1] = (int32_t)covered;
      if (lg->delta) lg->delta[i - 1] = (uint32_t)d2;
    }
    st->sum_uncovered += (uint64_t)nU;
    st->sum_covered += covered;
    int32_t *t = prev; prev = cur; cur = t;
    nprev = ncur;
    int64_t k2 = 0;
    for (int64_t k = 0; k < nU; ++k)
      if (cluster[U[k]] < 0) U[k2++] = U[k];
    nU = k2;
  }
  /* only for n = 1 (no iteration): the node is its own cluster */
  for (int64_t k = 0; k < nU; ++k) { cluster[U[k]] = U[k]; D[U[k]] = 0; }
  st->singletons = (int32_t)nU;
  st->stages = iters;
  st->levels = iters;
  st->delta_end = (uint32_t)d2;
  for (int32_t v = 0; v < n; ++v) {
    if (cluster[v] == v) st->num_clusters++;
    if (D[v] > st->radius) st->radius = D[v];
  }
done:
  free(U); free(settled); free(loc); free(lab); free(birth); free(prev); free(cur); free(h.a);
  return rc;
}

/* ------------------------------------------------------------ quotient -- */

typedef struct { uint64_t key; uint64_t w; } qrec_t;

static int cmp_qrec(const void *a, const void *b) {
  const qrec_t *x = a, *y = b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->w < y->w ? -1 : (x->w > y->w);
}

/* Weighted quotient graph (Section 4): one node per cluster, numbered by
 * ascending center id; for every edge (u,v) with c_u != c_v an edge between
 * the two clusters of weight w(u,v) + D_u + D_v, keeping the lightest of
 * parallel edges.  Outputs:
 *   k, center[k]            cluster index -> center node id
 *   ne, ea[ne], eb[ne], ew[ne]  undirected edges a < b, sorted by (a, b)
 * Arrays are malloc'd here and freed with or_free. */
int or_quotient(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *w,
                const int32_t *cluster, const uint64_t *D,
                int32_t *k_out, int32_t **center_out, int64_t *ne_out,
                int32_t **ea_out, int32_t **eb_out, uint64_t **ew_out, int64_t *pairs_out) {
  int32_t *dense = malloc((size_t)n * 4);
  if (!dense) return OR_ENOMEM;
  int32_t k = 0;
  for (int32_t v = 0; v < n; ++v) dense[v] = (cluster[v] == v) ? k++ : -1;
  int32_t *center = malloc((size_t)(k ? k : 1) * 4);
  int64_t P = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a)
      if (u < col[a] && cluster[u] != cluster[col[a]]) P++;
  qrec_t *rec = malloc((size_t)(P ? P : 1) * sizeof(qrec_t));
  if (!center || !rec) { free(dense); free(center); free(rec); return OR_ENOMEM; }
  for (int32_t v = 0; v < n; ++v)
    if (dense[v] >= 0) center[dense[v]] = v;
  int64_t i = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a) {
      int32_t v = col[a];
      if (!(u < v) || cluster[u] == cluster[v]) continue;
      uint64_t x = (uint64_t)dense[cluster[u]], y = (uint64_t)dense[cluster[v]];
      if (x > y) { uint64_t t = x; x = y; y = t; }
      rec[i].key = (x << 32) | y;
      rec[i].w = (uint64_t)w[a] + D[u] + D[v];
      i++;
    }
  qsort(rec, (size_t)P, sizeof(qrec_t), cmp_qrec);
  int64_t ne = 0;
  for (int64_t j = 0; j < P; ++j)
    if (j == 0 || rec[j].key != rec[j - 1].key) ne++;
  int32_t *ea = malloc((size_t)(ne ? ne : 1) * 4), *eb = malloc((size_t)(ne ? ne : 1) * 4);
  uint64_t *ew = malloc((size_t)(ne ? ne : 1) * 8);
  if (!ea || !eb || !ew) { free(dense); free(center); free(rec); free(ea); free(eb); free(ew); return OR_ENOMEM; }
  int64_t e = 0;
  for (int64_t j = 0; j < P; ++j)
    if (j == 0 || rec[j].key != rec[j - 1].key) {
      ea[e] = (int32_t)(rec[j].key >> 32);
      eb[e] = (int32_t)(rec[j].key & 0xffffffffu);
      ew[e] = rec[j].w;   /* first of its run = minimum weight */
      e++;
    }
  free(rec); free(dense);
  *k_out = k; *center_out = center; *ne_out = ne; *ea_out = ea; *eb_out = eb; *ew_out = ew;
  if (pairs_out) *pairs_out = P;
  return OR_OK;
}

void or_free(void *p) { free(p); }

/* ---------------------------------------------------- shortest paths -- */

/* Dijkstra from src over a CSR with u64 weights; dist[v] = INF64 when
 * unreachable. */
static int dijkstra64(int32_t n, const int64_t *rp, const int32_t *col, const uint64_t *w, int32_t src,
                      uint64_t *dist, heap_t *h) {
  for (int32_t v = 0; v < n; ++v) dist[v] = INF64;
  h->len = 0;
  dist[src] = 0;
  if (heap_push(h, 0, 0, (uint32_t)src)) return OR_ENOMEM;
  while (h->len) {
    item_t it = heap_pop(h);
    if (it.d != dist[it.v]) continue;
    for (int64_t a = rp[it.v]; a < rp[it.v + 1]; ++a) {
      uint64_t nd = it.d + w[a];
      if (nd < dist[col[a]]) {
        dist[col[a]] = nd;
        if (heap_push(h, nd, 0, (uint32_t)col[a])) return OR_ENOMEM;
      }
    }
  }
  return OR_OK;
}

/* Exact weighted diameter of an undirected graph given as an edge list over
 * k nodes: max finite distance over all pairs, one Dijkstra per node. */
int or_diameter_edges(int32_t k, int64_t ne, const int32_t *ea, const int32_t *eb, const uint64_t *ew,
                      uint64_t *phi_out) {
  int64_t *rp = calloc((size_t)k + 1, 8);
  int32_t *col = malloc((size_t)(2 * ne + 1) * 4);
  uint64_t *ww = malloc((size_t)(2 * ne + 1) * 8);
  int64_t *cur = malloc(((size_t)k + 1) * 8);
  uint64_t *dist = malloc(((size_t)k + 1) * 8);
  heap_t h = {0};
  int rc = OR_OK;
  if (!rp || !col || !ww || !cur || !dist) { rc = OR_ENOMEM; goto out; }
  for (int64_t e = 0; e < ne; ++e) { rp[ea[e] + 1]++; rp[eb[e] + 1]++; }
  for (int32_t v = 0; v < k; ++v) rp[v + 1] += rp[v];
  memcpy(cur, rp, (size_t)k * 8);
  for (int64_t e = 0; e < ne; ++e) {
    col[cur[ea[e]]] = eb[e]; ww[cur[ea[e]]++] = ew[e];
    col[cur[eb[e]]] = ea[e]; ww[cur[eb[e]]++] = ew[e];
  }
  uint64_t phi = 0;
  for (int32_t s = 0; s < k; ++s) {
    if ((rc = dijkstra64(k, rp, col, ww, s, dist, &h))) goto out;
    for (int32_t v = 0; v < k; ++v)
      if (dist[v] != INF64 && dist[v] > phi) phi = dist[v];
  }
  *phi_out = phi;
out:
  free(rp); free(col); free(ww); free(cur); free(dist); free(h.a);
  return rc;
}

/* Single-source shortest paths on the input graph (the exact distances that
 * Delta-stepping computes).  dist is u32 with 0xFFFFFFFF for unreachable;
 * a finite distance that does not fit below that value is an overflow. */
int or_sssp(int32_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *w, int32_t src,
            uint32_t *dist_out, uint64_t *max_out) {
  if (src < 0 || src >= n) return OR_EINVAL;
  int64_t m = row_ptr[n];
  int64_t *rp = malloc(((size_t)n + 1) * 8);
  uint64_t *ww = malloc((size_t)(m ? m : 1) * 8);
  uint64_t *dist = malloc((size_t)n * 8);
  heap_t h = {0};
  int rc = OR_OK;
  if (!rp || !ww || !dist) { rc = OR_ENOMEM; goto out; }
  memcpy(rp, row_ptr, ((size_t)n + 1) * 8);
  for (int64_t a = 0; a < m; ++a) ww[a] = w[a];
  if ((rc = dijkstra64(n, rp, col, ww, src, dist, &h))) goto out;
  uint64_t mx = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (dist[v] == INF64) { dist_out[v] = 0xffffffffu; continue; }
    if (dist[v] >= 0xffffffffu) { rc = OR_EOVERFLOW; goto out; }
    dist_out[v] = (uint32_t)dist[v];
    if (dist[v] > mx) mx = dist[v];
  }
  *max_out = mx;
out:
  free(rp); free(ww); free(dist); free(h.a);
  return rc;
}
