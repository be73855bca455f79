/*
 * Seeded synthetic graph generators: the shared input module.
 *
 * This file holds only input generation (random topology, random weights,
 * largest connected component, canonical CSR).  It contains none of the
 * decomposition's arithmetic.  Both the CPU oracle and the GPU path consume
 * the CSR it produces.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), implemented here from that published
 * definition.  Every draw is addressed by a counter (item index, sub-index,
 * stream tag, 0) under key (seed_lo, seed_hi), so generation is order-free.
 *
 * Stream tags: 1 edge weights, 2 grid edge drops, 3 diagonal shortcuts,
 * 4 R-MAT quadrant draws, 5 R-MAT vertex permutation, 8 geometric points,
 * 9 geometric graph sizes.
 *
 * Output CSR is symmetric (each undirected edge appears as two arcs), node ids
 * are compacted in ascending original order after the largest component is
 * kept, and each row is sorted by column id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAG_WEIGHT 1u
#define TAG_DROP 2u
#define TAG_DIAG 3u
#define TAG_RMAT 4u
#define TAG_PERM 5u
#define TAG_POINT 8u
#define TAG_GSIZE 9u

/* ---------------------------------------------------------------- Philox -- */

static void philox(const uint32_t ctr_in[4], uint64_t seed, uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void gg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr, (uint64_t)key[0] | ((uint64_t)key[1] << 32), out);
}

static uint32_t draw(uint32_t a, uint32_t b, uint32_t tag, uint64_t seed, int word) {
  uint32_t c[4] = {a, b, tag, 0}, o[4];
  philox(c, seed, o);
  return o[word];
}

/* 53-bit uniform double in [0,1) from two 32-bit words. */
static double u53(uint32_t hi, uint32_t lo) {
  uint64_t x = ((uint64_t)hi << 21) ^ (uint64_t)(lo >> 11);
  x &= ((uint64_t)1 << 53) - 1;
  return (double)x * (1.0 / 9007199254740992.0);
}

/* -------------------------------------------------------- edge list type -- */

typedef struct {
  uint32_t *u, *v, *w;
  int64_t len, cap;
} edges_t;

static int edges_push(edges_t *e, uint32_t u, uint32_t v, uint32_t w) {
  if (e->len == e->cap) {
    int64_t nc = e->cap ? e->cap * 2 : 1024;
    uint32_t *nu = realloc(e->u, nc * 4), *nv = realloc(e->v, nc * 4), *nw = realloc(e->w, nc * 4);
    if (!nu || !nv || !nw) return -1;
    e->u = nu; e->v = nv; e->w = nw; e->cap = nc;
  }
  e->u[e->len] = u; e->v[e->len] = v; e->w[e->len] = w; e->len++;
  return 0;
}

static void edges_free(edges_t *e) { free(e->u); free(e->v); free(e->w); memset(e, 0, sizeof *e); }

/* ------------------------------------------- LCC + canonical symmetric CSR -- */

static uint32_t uf_find(uint32_t *p, uint32_t x) {
  while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
  return x;
}

/* Output produced by every generator; freed with gg_free. */
typedef struct {
  int32_t n;
  int64_t m; /* arcs = 2 x undirected edges */
  int32_t *row_ptr; /* n+1 in int32 (NULL from gg_mesh64, whose offsets pass 2^31) */
  int32_t *col;
  uint32_t *w;
  int64_t *row_ptr64; /* same offsets in int64, always filled */
} gg_csr;

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : x > y;
}

/* Builds the LCC's canonical CSR from an undirected simple edge list over
 * n0 nodes (no self loops, no duplicate pairs). */
static int finish_csr(int64_t n0, edges_t *e, gg_csr *out) {
  memset(out, 0, sizeof *out);
  uint32_t *par = malloc((size_t)n0 * 4);
  int64_t *sz = calloc((size_t)n0, 8);
  if (!par || !sz) { free(par); free(sz); return -1; }
  for (int64_t i = 0; i < n0; ++i) par[i] = (uint32_t)i;
  for (int64_t i = 0; i < e->len; ++i) {
    uint32_t a = uf_find(par, e->u[i]), b = uf_find(par, e->v[i]);
    if (a != b) { if (a < b) par[b] = a; else par[a] = b; }
  }
  for (int64_t i = 0; i < n0; ++i) sz[uf_find(par, (uint32_t)i)]++;
  /* largest component; ties go to the one whose smallest node id is smaller
   * (roots are the smallest id of their component by construction) */
  uint32_t best = 0; int64_t bsz = -1;
  for (int64_t i = 0; i < n0; ++i)
    if (par[i] == (uint32_t)i && sz[i] > bsz) { bsz = sz[i]; best = (uint32_t)i; }
  free(sz);
  int32_t *nid = malloc((size_t)n0 * 4);
  if (!nid) { free(par); return -1; }
  int32_t n = 0;
  for (int64_t i = 0; i < n0; ++i) nid[i] = (uf_find(par, (uint32_t)i) == best) ? n++ : -1;
  free(par);
  int64_t *deg = calloc((size_t)n + 1, 8);
  if (!deg) { free(nid); return -1; }
  int64_t me = 0;
  for (int64_t i = 0; i < e->len; ++i) {
    int32_t a = nid[e->u[i]];
    if (a < 0) continue;
    deg[a + 1]++; deg[nid[e->v[i]] + 1]++; me++;
  }
  for (int32_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  int64_t m = 2 * me;
  out->n = n; out->m = m;
  out->row_ptr = malloc(((size_t)n + 1) * 4);
  out->row_ptr64 = malloc(((size_t)n + 1) * 8);
  out->col = malloc((size_t)(m ? m : 1) * 4);
  out->w = malloc((size_t)(m ? m : 1) * 4);
  int64_t *cur = malloc(((size_t)n + 1) * 8);
  if (!out->row_ptr || !out->row_ptr64 || !out->col || !out->w || !cur) { free(nid); free(deg); free(cur); return -1; }
  for (int32_t i = 0; i <= n; ++i) { out->row_ptr64[i] = deg[i]; out->row_ptr[i] = (int32_t)deg[i]; cur[i] = deg[i]; }
  for (int64_t i = 0; i < e->len; ++i) {
    int32_t a = nid[e->u[i]];
    if (a < 0) continue;
    int32_t b = nid[e->v[i]];
    out->col[cur[a]] = b; out->w[cur[a]++] = e->w[i];
    out->col[cur[b]] = a; out->w[cur[b]++] = e->w[i];
  }
  free(cur); free(nid); free(deg);
  /* sort each row by column id */
  uint64_t *tmp = NULL; int64_t tcap = 0;
  for (int32_t r = 0; r < n; ++r) {
    int64_t s = out->row_ptr64[r], t = out->row_ptr64[r + 1], len = t - s;
    if (len < 2) continue;
    if (len <= 16) {
      for (int64_t i = s + 1; i < t; ++i) {
        int32_t c = out->col[i]; uint32_t ww = out->w[i]; int64_t j = i - 1;
        while (j >= s && out->col[j] > c) { out->col[j + 1] = out->col[j]; out->w[j + 1] = out->w[j]; --j; }
        out->col[j + 1] = c; out->w[j + 1] = ww;
      }
    } else {
      if (len > tcap) { free(tmp); tcap = len; tmp = malloc((size_t)tcap * 8); if (!tmp) return -1; }
      for (int64_t i = 0; i < len; ++i) tmp[i] = ((uint64_t)(uint32_t)out->col[s + i] << 32) | out->w[s + i];
      qsort(tmp, (size_t)len, 8, cmp_u64);
      for (int64_t i = 0; i < len; ++i) { out->col[s + i] = (int32_t)(tmp[i] >> 32); out->w[s + i] = (uint32_t)tmp[i]; }
    }
  }
  free(tmp);
  return 0;
}

void gg_free(gg_csr *g) {
  if (!g) return;
  free(g->row_ptr); free(g->row_ptr64); free(g->col); free(g->w);
  memset(g, 0, sizeof *g);
}

static uint32_t weight_draw(uint64_t idx, uint64_t seed, uint32_t wmax) {
  uint32_t x = draw((uint32_t)idx, (uint32_t)(idx >> 32), TAG_WEIGHT, seed, 0);
  return 1u + (uint32_t)(((uint64_t)x * wmax) >> 32);
}

/* ------------------------------------------------------------ 2D grids -- */

/* rows x cols 4-neighbour grid, node id r*cols+c.  Edge index: horizontal
 * edges row-major (r*(cols-1)+c), then vertical (H + r*cols + c), then the
 * optional diagonal of cell (r,c) (H + V + r*(cols-1) + c).  Each grid edge is
 * dropped when its tag-2 draw is below drop_thr; each cell gets a diagonal
 * when its tag-3 draw is below diag_thr, oriented by the low bit of the
 * second word.  Weights are 1 + floor(x*wmax/2^32) of the tag-1 draw of the
 * edge index, so they lie in [1, wmax]. */
int gg_grid(int32_t rows, int32_t cols, uint32_t wmax, uint64_t seed,
            uint32_t drop_thr, uint32_t diag_thr, gg_csr *out) {
  if (rows < 1 || cols < 1 || wmax < 1 || (int64_t)rows * cols > 0x7fffffff) return -1;
  edges_t e = {0};
  int64_t H = (int64_t)rows * (cols - 1), V = (int64_t)(rows - 1) * cols;
  for (int32_t r = 0; r < rows; ++r)
    for (int32_t c = 0; c + 1 < cols; ++c) {
      int64_t idx = (int64_t)r * (cols - 1) + c;
      if (drop_thr && draw((uint32_t)idx, 0, TAG_DROP, seed, 0) < drop_thr) continue;
      if (edges_push(&e, (uint32_t)(r * cols + c), (uint32_t)(r * cols + c + 1), weight_draw((uint64_t)idx, seed, wmax))) goto fail;
    }
  for (int32_t r = 0; r + 1 < rows; ++r)
    for (int32_t c = 0; c < cols; ++c) {
      int64_t idx = H + (int64_t)r * cols + c;
      if (drop_thr && draw((uint32_t)idx, 0, TAG_DROP, seed, 0) < drop_thr) continue;
      if (edges_push(&e, (uint32_t)(r * cols + c), (uint32_t)((r + 1) * cols + c), weight_draw((uint64_t)idx, seed, wmax))) goto fail;
    }
  if (diag_thr)
    for (int32_t r = 0; r + 1 < rows; ++r)
      for (int32_t c = 0; c + 1 < cols; ++c) {
        int64_t cell = (int64_t)r * (cols - 1) + c;
        uint32_t cc[4] = {(uint32_t)cell, 0, TAG_DIAG, 0}, o[4];
        philox(cc, seed, o);
        if (o[0] >= diag_thr) continue;
        uint32_t a, b;
        if (o[1] & 1u) { a = (uint32_t)(r * cols + c + 1); b = (uint32_t)((r + 1) * cols + c); }
        else { a = (uint32_t)(r * cols + c); b = (uint32_t)((r + 1) * cols + c + 1); }
        if (edges_push(&e, a, b, weight_draw((uint64_t)(H + V + cell), seed, wmax))) goto fail;
      }
  {
    int rc = finish_csr((int64_t)rows * cols, &e, out);
    edges_free(&e);
    return rc;
  }
fail:
  edges_free(&e);
  return -1;
}

/* rows x cols grid with every grid edge kept plus the diagonals of gg_grid
 * (same draws, same weights: for sizes gg_grid takes and drop_thr = 0 the
 * two produce the same CSR).  A full grid is connected, so the CSR is written
 * directly, two passes over the nodes (degrees, then arcs) with no edge list
 * and no component search; offsets are int64 (row_ptr64 only, row_ptr stays
 * NULL), for graphs of more than 2^31 arcs. */
int gg_mesh64(int32_t rows, int32_t cols, uint32_t wmax, uint64_t seed, uint32_t diag_thr, gg_csr *out) {
  memset(out, 0, sizeof *out);
  if (rows < 2 || cols < 2 || wmax < 1 || (int64_t)rows * cols > 0x7fffffff) return -1;
  const int64_t n = (int64_t)rows * cols, cells = (int64_t)(rows - 1) * (cols - 1);
  const int64_t H = (int64_t)rows * (cols - 1), V = (int64_t)(rows - 1) * cols;
  /* diagonal of each cell: 0 none, 1 (r,c)-(r+1,c+1), 2 (r,c+1)-(r+1,c) */
  uint8_t *dg = calloc((size_t)cells, 1);
  int64_t *rp = malloc(((size_t)n + 1) * 8);
  if (!dg || !rp) { free(dg); free(rp); return -1; }
  if (diag_thr) {
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < cells; ++cell) {
      uint32_t cc[4] = {(uint32_t)cell, 0, TAG_DIAG, 0}, o[4];
      philox(cc, seed, o);
      if (o[0] < diag_thr) dg[cell] = (o[1] & 1u) ? 2 : 1;
    }
  }
  /* neighbours of (r,c) in ascending id: up-left, up, up-right, left, right,
   * down-left, down, down-right; k-th entry valid when nb_ok */
#define CELL(r, c) ((int64_t)(r) * (cols - 1) + (c))
  rp[0] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const int32_t r = (int32_t)(v / cols), c = (int32_t)(v % cols);
    int d = 0;
    if (r > 0 && c > 0 && dg[CELL(r - 1, c - 1)] == 1) d++;
    if (r > 0) d++;
    if (r > 0 && c + 1 < cols && dg[CELL(r - 1, c)] == 2) d++;
    if (c > 0) d++;
    if (c + 1 < cols) d++;
    if (r + 1 < rows && c > 0 && dg[CELL(r, c - 1)] == 2) d++;
    if (r + 1 < rows) d++;
    if (r + 1 < rows && c + 1 < cols && dg[CELL(r, c)] == 1) d++;
    rp[v + 1] = d;
  }
  for (int64_t v = 0; v < n; ++v) rp[v + 1] += rp[v];
  const int64_t m = rp[n];
  int32_t *col = malloc((size_t)m * 4);
  uint32_t *w = malloc((size_t)m * 4);
  if (!col || !w) { free(dg); free(rp); free(col); free(w); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const int32_t r = (int32_t)(v / cols), c = (int32_t)(v % cols);
    int64_t a = rp[v];
#define ARC(nb, idx) do { col[a] = (int32_t)(nb); w[a] = weight_draw((uint64_t)(idx), seed, wmax); a++; } while (0)
    if (r > 0 && c > 0 && dg[CELL(r - 1, c - 1)] == 1) ARC(v - cols - 1, H + V + CELL(r - 1, c - 1));
    if (r > 0) ARC(v - cols, H + (int64_t)(r - 1) * cols + c);
    if (r > 0 && c + 1 < cols && dg[CELL(r - 1, c)] == 2) ARC(v - cols + 1, H + V + CELL(r - 1, c));
    if (c > 0) ARC(v - 1, (int64_t)r * (cols - 1) + c - 1);
    if (c + 1 < cols) ARC(v + 1, (int64_t)r * (cols - 1) + c);
    if (r + 1 < rows && c > 0 && dg[CELL(r, c - 1)] == 2) ARC(v + cols - 1, H + V + CELL(r, c - 1));
    if (r + 1 < rows) ARC(v + cols, H + (int64_t)r * cols + c);
    if (r + 1 < rows && c + 1 < cols && dg[CELL(r, c)] == 1) ARC(v + cols + 1, H + V + CELL(r, c));
#undef ARC
  }
#undef CELL
  free(dg);
  out->n = (int32_t)n;
  out->m = m;
  out->row_ptr = NULL;
  out->row_ptr64 = rp;
  out->col = col;
  out->w = w;
  return 0;
}

/* --------------------------------------------------------------- R-MAT -- */

static void radix_sort_u64(uint64_t *a, uint64_t *tmp, int64_t n, int bits) {
  for (int shift = 0; shift < bits; shift += 16) {
    int64_t *cnt = calloc(65537, 8);
    for (int64_t i = 0; i < n; ++i) cnt[((a[i] >> shift) & 0xffff) + 1]++;
    for (int i = 0; i < 65536; ++i) cnt[i + 1] += cnt[i];
    for (int64_t i = 0; i < n; ++i) tmp[cnt[(a[i] >> shift) & 0xffff]++] = a[i];
    memcpy(a, tmp, (size_t)n * 8);
    free(cnt);
  }
}

/* R-MAT(scale, edge_factor) with quadrant probabilities given as u32
 * thresholds ta, ta+tb, ta+tb+tc (Chakrabarti, Zhan, Faloutsos 2004).
 * Edge e draws its bit at level l from word l%4 of Philox(e, l/4, tag 4).
 * Vertices are relabelled by a seeded random permutation (order of the tag-5
 * draws), then the graph is symmetrised, self loops and duplicate pairs are
 * dropped, and the edge of rank i in (min,max) order gets weight
 * 1 + (x >> wshift) of its tag-1 draw. */
int gg_rmat(int32_t scale, int32_t edge_factor, uint32_t ta, uint32_t tb, uint32_t tc,
            uint32_t wshift, uint64_t seed, gg_csr *out) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return -1;
  int64_t N = (int64_t)1 << scale, M = N * edge_factor;
  uint64_t *key = malloc((size_t)N * 8), *tmp = malloc((size_t)(M > N ? M : N) * 8);
  uint32_t *perm = malloc((size_t)N * 4);
  uint64_t *pairs = malloc((size_t)M * 8);
  if (!key || !tmp || !perm || !pairs) { free(key); free(tmp); free(perm); free(pairs); return -1; }
  /* permutation: node i goes to the rank of (draw_i, i) */
  for (int64_t i = 0; i < N; ++i) key[i] = ((uint64_t)draw((uint32_t)i, 0, TAG_PERM, seed, 0) << 32) | (uint64_t)i;
  radix_sort_u64(key, tmp, N, 64);
  for (int64_t r = 0; r < N; ++r) perm[key[r] & 0xffffffffu] = (uint32_t)r;
  free(key);
  uint32_t tab = ta + tb, tabc = ta + tb + tc;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < M; ++e) {
    uint32_t u = 0, v = 0, o[4] = {0, 0, 0, 0};
    for (int l = 0; l < scale; ++l) {
      if ((l & 3) == 0) {
        uint32_t c[4] = {(uint32_t)e, (uint32_t)(l >> 2), TAG_RMAT, 0};
        philox(c, seed, o);
      }
      uint32_t x = o[l & 3];
      uint32_t rb = x >= tab, cb = (x >= ta && x < tab) || x >= tabc;
      u = (u << 1) | rb; v = (v << 1) | cb;
    }
    u = perm[u]; v = perm[v];
    pairs[e] = (u == v) ? ~(uint64_t)0 : (u < v ? ((uint64_t)u << 32 | v) : ((uint64_t)v << 32 | u));
  }
  free(perm);
  radix_sort_u64(pairs, tmp, M, 64);
  free(tmp);
  edges_t e = {0};
  int64_t uniq = 0;
  for (int64_t i = 0; i < M; ++i) {
    if (pairs[i] == ~(uint64_t)0) break;
    if (i && pairs[i] == pairs[i - 1]) continue;
    uint32_t x = draw((uint32_t)uniq, (uint32_t)((uint64_t)uniq >> 32), TAG_WEIGHT, seed, 0);
    if (edges_push(&e, (uint32_t)(pairs[i] >> 32), (uint32_t)pairs[i], 1u + (x >> wshift))) { free(pairs); edges_free(&e); return -1; }
    uniq++;
  }
  free(pairs);
  int rc = finish_csr(N, &e, out);
  edges_free(&e);
  return rc;
}

/* ----------------------------------------------- random geometric graph -- */

/* n points uniform in the unit square (coordinates from the tag-8 draw of
 * (point, graph_tag)), radius sqrt(avg_deg/(pi n)), weight
 * floor(wscale*len + 0.5) + 1. */
int gg_rgg(int32_t n, double avg_deg, double wscale, uint32_t graph_tag, uint64_t seed, gg_csr *out) {
  if (n < 2) return -1;
  double *x = malloc((size_t)n * 8), *y = malloc((size_t)n * 8);
  if (!x || !y) { free(x); free(y); return -1; }
  for (int32_t i = 0; i < n; ++i) {
    uint32_t c[4] = {(uint32_t)i, graph_tag, TAG_POINT, 0}, o[4];
    philox(c, seed, o);
    x[i] = u53(o[0], o[1]);
    y[i] = u53(o[2], o[3]);
  }
  double r = sqrt(avg_deg / (M_PI * (double)n));
  int32_t nc = (int32_t)floor(1.0 / r);
  if (nc < 1) nc = 1;
  int64_t ncell = (int64_t)nc * nc;
  int32_t *cell_start = calloc((size_t)ncell + 1, 4), *order = malloc((size_t)n * 4), *cid = malloc((size_t)n * 4);
  if (!cell_start || !order || !cid) { free(x); free(y); free(cell_start); free(order); free(cid); return -1; }
  for (int32_t i = 0; i < n; ++i) {
    int32_t cx = (int32_t)(x[i] * nc), cy = (int32_t)(y[i] * nc);
    if (cx >= nc) cx = nc - 1;
    if (cy >= nc) cy = nc - 1;
    cid[i] = cy * nc + cx;
    cell_start[cid[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
  {
    int32_t *cur = malloc((size_t)ncell * 4);
    memcpy(cur, cell_start, (size_t)ncell * 4);
    for (int32_t i = 0; i < n; ++i) order[cur[cid[i]]++] = i;
    free(cur);
  }
  edges_t e = {0};
  double r2 = r * r;
  for (int32_t i = 0; i < n; ++i) {
    int32_t cx = cid[i] % nc, cy = cid[i] / nc;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int32_t qx = cx + dx, qy = cy + dy;
        if (qx < 0 || qy < 0 || qx >= nc || qy >= nc) continue;
        int32_t q = qy * nc + qx;
        for (int32_t k = cell_start[q]; k < cell_start[q + 1]; ++k) {
          int32_t j = order[k];
          if (j <= i) continue;
          double ddx = x[i] - x[j], ddy = y[i] - y[j], d2 = ddx * ddx + ddy * ddy;
          if (d2 > r2) continue;
          uint32_t w = (uint32_t)floor(wscale * sqrt(d2) + 0.5) + 1u;
          if (edges_push(&e, (uint32_t)i, (uint32_t)j, w)) goto fail;
        }
      }
  }
  free(x); free(y); free(cell_start); free(order); free(cid);
  {
    int rc = finish_csr(n, &e, out);
    edges_free(&e);
    return rc;
  }
fail:
  free(x); free(y); free(cell_start); free(order); free(cid);
  edges_free(&e);
  return -1;
}

/* Size of geometric graph g of a batch: round(10^(lo + span*u)). */
int32_t gg_rgg_size(uint32_t g, double lo, double span, uint64_t seed) {
  uint32_t c[4] = {g, 0, TAG_GSIZE, 0}, o[4];
  philox(c, seed, o);
  return (int32_t)floor(pow(10.0, lo + span * u53(o[0], o[1])) + 0.5);
}

/* ------------------------------------------- generic edge list -> CSR -- */

/* Builds the LCC canonical CSR from a caller edge list (simple graph). */
int gg_from_edges(int64_t n0, int64_t ne, const uint32_t *u, const uint32_t *v, const uint32_t *w, gg_csr *out) {
  edges_t e = {0};
  for (int64_t i = 0; i < ne; ++i) {
    if (u[i] >= (uint64_t)n0 || v[i] >= (uint64_t)n0 || u[i] == v[i]) { edges_free(&e); return -1; }
    if (edges_push(&e, u[i], v[i], w[i])) { edges_free(&e); return -1; }
  }
  int rc = finish_csr(n0, &e, out);
  edges_free(&e);
  return rc;
}
