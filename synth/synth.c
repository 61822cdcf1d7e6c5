/*
 * Seeded synthetic graph generators (R-MAT, 2D / 3D random geometric graphs).
 *
 * This module produces the test and benchmark inputs only. It holds none of
 * the label-propagation, contraction or compression arithmetic, so both the
 * CPU oracle and the GPU library can consume its output without sharing any
 * of the method's code.
 *
 * Every random number is drawn from the SplitMix64 sequence (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
 * draw k of seed s is mix(s + (k + 1) * 0x9E3779B97F4A7C15). Draws are indexed
 * by a counter, so the output does not depend on the thread count.
 *
 * All generators return a simple undirected graph as a symmetric CSR with
 * 64-bit offsets and 32-bit neighbour IDs: no self-loops, no duplicate edges,
 * every neighbourhood sorted by increasing ID.
 */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t sm_draw(uint64_t seed, uint64_t k) {
  return sm_mix(seed + (k + 1) * GOLDEN);
}

static inline double sm_unit(uint64_t seed, uint64_t k) {
  return (double)(sm_draw(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

/* Phase messages on stderr for long generations (SYNTH_PROGRESS set). */
static void progress(const char *what, int64_t a, int64_t b) {
  if (!getenv("SYNTH_PROGRESS")) return;
  fprintf(stderr, "[synth] %s %lld %lld\n", what, (long long)a, (long long)b);
  fflush(stderr);
}

typedef struct {
  int64_t n;
  uint64_t two_m;
  uint64_t *xadj;   /* n + 1 */
  int32_t *adjncy;  /* two_m */
} synth_csr;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Ascending sort of non-negative int32 values: insertion sort for short runs,
 * quicksort (median of three, loop on the larger side) up to 2^14 values, LSD
 * radix sort with 11-bit digits beyond (scratch from malloc; qsort if that
 * fails). */
static void isort_i32(int32_t *a, int64_t d) {
  for (int64_t i = 1; i < d; ++i) {
    int32_t x = a[i];
    int64_t j = i;
    while (j > 0 && a[j - 1] > x) { a[j] = a[j - 1]; --j; }
    a[j] = x;
  }
}

static void qsort_i32(int32_t *a, int64_t d) {
  while (d > 24) {
    int32_t x = a[0], y = a[d / 2], z = a[d - 1];
    int32_t piv = x < y ? (y < z ? y : (x < z ? z : x)) : (x < z ? x : (y < z ? z : y));
    int64_t i = 0, j = d - 1;
    for (;;) {
      while (a[i] < piv) ++i;
      while (a[j] > piv) --j;
      if (i >= j) break;
      int32_t t = a[i]; a[i] = a[j]; a[j] = t;
      ++i; --j;
    }
    /* [0, j] <= piv <= [j + 1, d) */
    int64_t left = j + 1, right = d - left;
    if (left < right) { qsort_i32(a, left); a += left; d = right; }
    else { qsort_i32(a + left, right); d = left; }
  }
  isort_i32(a, d);
}

static void sort_i32(int32_t *a, int64_t d) {
  if (d <= (1 << 14)) { qsort_i32(a, d); return; }
  uint32_t *tmp = (uint32_t *)malloc((size_t)d * sizeof(uint32_t));
  if (!tmp) { qsort(a, (size_t)d, sizeof(int32_t), cmp_i32); return; }
  uint32_t *src = (uint32_t *)a, *dst = tmp;
  int64_t cnt[2048];
  for (int pass = 0; pass < 3; ++pass) {
    int sh = 11 * pass;
    memset(cnt, 0, sizeof(cnt));
    for (int64_t i = 0; i < d; ++i) cnt[(src[i] >> sh) & 2047]++;
    int64_t run = 0;
    for (int k = 0; k < 2048; ++k) { int64_t c = cnt[k]; cnt[k] = run; run += c; }
    for (int64_t i = 0; i < d; ++i) dst[cnt[(src[i] >> sh) & 2047]++] = src[i];
    uint32_t *t = src; src = dst; dst = t;
  }
  /* three passes: the result is in tmp */
  memcpy(a, src, (size_t)d * sizeof(uint32_t));
  free(tmp);
}

/* Build a symmetric, deduplicated, self-loop free CSR from a directed pair
 * source. `emit(ctx, i, &u, &v)` yields pair i (returns 0 to skip it); each
 * accepted pair is inserted in both directions. The pairs are cut into
 * fixed chunks; pass 1 counts, per chunk, the entries of every bucket of
 * 2^shift consecutive IDs (private counters, no atomics); pass 2 draws the
 * pairs again and scatters (ID within bucket, neighbour) entries to their
 * bucket; pass 3 places every bucket's entries by vertex, and every
 * neighbourhood is sorted and deduplicated. The result depends only on the
 * set of pairs, not on the thread count. */
typedef int (*pair_fn)(const void *ctx, int64_t i, int32_t *u, int32_t *v);

static int build_csr(int64_t n, int64_t npairs, pair_fn emit, const void *ctx,
                     synth_csr *out) {
  int shift = 0;
  while (n > 0 && ((n - 1) >> shift) >= (1 << 12)) ++shift;
  int64_t nb = n > 0 ? ((n - 1) >> shift) + 1 : 1;
  int64_t nc = 4 * (int64_t)omp_get_max_threads();
  if (nc < 1) nc = 1;
  uint64_t *hist = (uint64_t *)calloc((size_t)(nc * nb), sizeof(uint64_t));
  uint64_t *bstart = (uint64_t *)malloc((size_t)(nb + 1) * sizeof(uint64_t));
  uint64_t *vstart = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
  if (!hist || !bstart || !vstart) { free(hist); free(bstart); free(vstart); return -1; }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nc; ++c) {
    uint64_t *h = hist + c * nb;
    int64_t lo = npairs / nc * c + (c < npairs % nc ? c : npairs % nc);
    int64_t hi = lo + npairs / nc + (c < npairs % nc ? 1 : 0);
    for (int64_t i = lo; i < hi; ++i) {
      int32_t u, v;
      if (!emit(ctx, i, &u, &v) || u == v) continue;
      h[u >> shift]++;
      h[v >> shift]++;
    }
  }
  /* bucket-major positions: bucket b, then chunk c */
  uint64_t total = 0;
  for (int64_t b = 0; b < nb; ++b) {
    bstart[b] = total;
    for (int64_t c = 0; c < nc; ++c) {
      uint64_t k = hist[c * nb + b];
      hist[c * nb + b] = total;
      total += k;
    }
  }
  bstart[nb] = total;
  progress("degrees counted: vertices, directed pairs", n, (int64_t)total);
  uint64_t *ent = (uint64_t *)malloc((total ? total : 1) * sizeof(uint64_t));
  if (!ent) { free(hist); free(bstart); free(vstart); return -1; }
  uint64_t mask = ((uint64_t)1 << shift) - 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nc; ++c) {
    uint64_t *h = hist + c * nb;
    int64_t lo = npairs / nc * c + (c < npairs % nc ? c : npairs % nc);
    int64_t hi = lo + npairs / nc + (c < npairs % nc ? 1 : 0);
    for (int64_t i = lo; i < hi; ++i) {
      int32_t u, v;
      if (!emit(ctx, i, &u, &v) || u == v) continue;
      ent[h[u >> shift]++] = (((uint64_t)u & mask) << 32) | (uint32_t)v;
      ent[h[v >> shift]++] = (((uint64_t)v & mask) << 32) | (uint32_t)u;
    }
  }
  free(hist);
  progress("pairs scattered", n, (int64_t)total);
  int32_t *tmp = (int32_t *)malloc((total ? total : 1) * sizeof(int32_t));
  if (!tmp) { free(bstart); free(vstart); free(ent); return -1; }
  int64_t bw = (int64_t)1 << shift;
#pragma omp parallel
  {
    uint64_t *lc = (uint64_t *)malloc((size_t)(bw + 1) * sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
    for (int64_t b = 0; b < nb; ++b) {
      int64_t v0 = b << shift;
      int64_t vn = n - v0 < bw ? n - v0 : bw;
      memset(lc, 0, (size_t)(bw + 1) * sizeof(uint64_t));
      for (uint64_t e = bstart[b]; e < bstart[b + 1]; ++e) lc[(ent[e] >> 32) + 1]++;
      uint64_t run = bstart[b];
      for (int64_t k = 0; k < vn; ++k) {
        vstart[v0 + k] = run;
        run += lc[k + 1];
        lc[k + 1] = vstart[v0 + k];
      }
      for (uint64_t e = bstart[b]; e < bstart[b + 1]; ++e)
        tmp[lc[(ent[e] >> 32) + 1]++] = (int32_t)(uint32_t)ent[e];
    }
    free(lc);
  }
  vstart[n] = total;
  free(ent);
  free(bstart);
  /* sort + dedupe each neighbourhood in place; record new degrees */
  uint64_t *deg = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
  if (!deg) { free(vstart); free(tmp); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n; ++u) {
    uint64_t b = vstart[u], e = vstart[u + 1];
    uint64_t d = e - b;
    if (d > 1) sort_i32(tmp + b, (int64_t)d);
    uint64_t k = 0;
    for (uint64_t j = 0; j < d; ++j)
      if (k == 0 || tmp[b + j] != tmp[b + k - 1]) tmp[b + k++] = tmp[b + j];
    deg[u] = k;
  }
  progress("neighbourhoods sorted", n, 0);
  uint64_t *xadj = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
  if (!xadj) { free(vstart); free(tmp); free(deg); return -1; }
  xadj[0] = 0;
  for (int64_t u = 0; u < n; ++u) xadj[u + 1] = xadj[u] + deg[u];
  uint64_t two_m = xadj[n];
  int32_t *adj = (int32_t *)malloc((two_m ? two_m : 1) * sizeof(int32_t));
  if (!adj) { free(vstart); free(tmp); free(deg); free(xadj); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n; ++u)
    memcpy(adj + xadj[u], tmp + vstart[u], (xadj[u + 1] - xadj[u]) * sizeof(int32_t));
  free(vstart);
  free(tmp);
  free(deg);
  out->n = n;
  out->two_m = two_m;
  out->xadj = xadj;
  out->adjncy = adj;
  return 0;
}

/* ---------------------------------------------------------------- R-MAT -- */
typedef struct {
  int scale;
  int64_t n_limit;
  uint64_t seed;
  uint64_t ta, tab, tabc; /* quadrant thresholds on a 32-bit uniform */
} rmat_ctx;

static int rmat_pair(const void *c, int64_t i, int32_t *pu, int32_t *pv) {
  const rmat_ctx *x = (const rmat_ctx *)c;
  int draws = (x->scale + 1) / 2;
  uint64_t u = 0, v = 0;
  for (int j = 0; j < draws; ++j) {
    uint64_t r = sm_draw(x->seed, (uint64_t)i * (uint64_t)draws + (uint64_t)j);
    for (int h = 0; h < 2; ++h) {
      int level = 2 * j + h;
      if (level >= x->scale) break;
      uint64_t q = h ? (r >> 32) : (r & 0xffffffffULL);
      int bit = x->scale - 1 - level;
      /* quadrant a: neither bit; b: v's bit; c: u's bit; d: both
       * (branch-free: the quadrant is a coin the predictor cannot learn) */
      uint64_t bu = q >= x->tab;
      uint64_t bv = (uint64_t)((q >= x->ta) & (q < x->tab)) | (uint64_t)(q >= x->tabc);
      u |= bu << bit;
      v |= bv << bit;
    }
  }
  if ((int64_t)u >= x->n_limit || (int64_t)v >= x->n_limit) return 0;
  *pu = (int32_t)u;
  *pv = (int32_t)v;
  return 1;
}

/* R-MAT with `nsamples` edge samples over 2^scale IDs; samples with an
 * endpoint >= n_limit are rejected (n_limit <= 0 means 2^scale). No ID
 * permutation is applied. */
int synth_rmat(int scale, int64_t nsamples, double a, double b, double c,
               uint64_t seed, int64_t n_limit, synth_csr *out) {
  if (scale < 1 || scale > 31 || nsamples < 0) return -2;
  rmat_ctx x;
  x.scale = scale;
  x.n_limit = n_limit > 0 ? n_limit : (1LL << scale);
  x.seed = seed;
  x.ta = (uint64_t)(a * 4294967296.0);
  x.tab = (uint64_t)((a + b) * 4294967296.0);
  x.tabc = (uint64_t)((a + b + c) * 4294967296.0);
  return build_csr(x.n_limit, nsamples, rmat_pair, &x, out);
}

/* ------------------------------------------------------------------ RGG -- */
typedef struct {
  int dim;
  int64_t n;
  double r2;
  const double *pt;     /* n * dim, in final ID order */
  int64_t g;            /* cells per dimension */
  const int64_t *cstart; /* g^dim + 1 */
  /* enumerated candidate pairs are produced per point; see rgg_build */
} rgg_ctx;

static inline int64_t cell_of(double x, int64_t g) {
  int64_t c = (int64_t)(x * (double)g);
  if (c >= g) c = g - 1;
  if (c < 0) c = 0;
  return c;
}

typedef struct {
  int64_t key;   /* linear cell id */
  double x;
  int64_t idx;
} rgg_rec;

static int cmp_rec(const void *pa, const void *pb) {
  const rgg_rec *a = (const rgg_rec *)pa, *b = (const rgg_rec *)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->x != b->x) return a->x < b->x ? -1 : 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Random geometric graph: n points uniform in [0,1)^dim, an edge between two
 * points at Euclidean distance <= r. Vertex IDs follow the (cell_z, cell_y,
 * cell_x, x) order on a grid of cells at least r wide, for locality. */
int synth_rgg(int dim, int64_t n, double r, uint64_t seed, synth_csr *out) {
  if ((dim != 2 && dim != 3) || n < 1 || n > 2147483647LL || !(r > 0)) return -2;
  int64_t g = (int64_t)floor(1.0 / r);
  if (g < 1) g = 1;
  if (dim == 2 && g > 65536) g = 65536;
  if (dim == 3 && g > 2048) g = 2048;
  int64_t ncell = dim == 2 ? g * g : g * g * g;
  double *raw = (double *)malloc((size_t)n * dim * sizeof(double));
  rgg_rec *rec = (rgg_rec *)malloc((size_t)n * sizeof(rgg_rec));
  if (!raw || !rec) { free(raw); free(rec); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < dim; ++d) raw[i * dim + d] = sm_unit(seed, (uint64_t)(i * dim + d));
    int64_t cx = cell_of(raw[i * dim + 0], g), cy = cell_of(raw[i * dim + 1], g);
    int64_t key = cy * g + cx;
    if (dim == 3) key += cell_of(raw[i * dim + 2], g) * g * g;
    rec[i].key = key;
    rec[i].x = raw[i * dim + 0];
    rec[i].idx = i;
  }
  progress("points drawn", n, ncell);
  /* order by (cell, x, index): a counting sort by cell, then each cell's few
   * points sorted by (x, index) */
  double *pt = (double *)malloc((size_t)n * dim * sizeof(double));
  int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t *cpos = (int64_t *)malloc(((size_t)ncell + 1) * sizeof(int64_t));
  rgg_rec *ord = (rgg_rec *)malloc((size_t)n * sizeof(rgg_rec));
  if (!pt || !cstart || !cpos || !ord) {
    free(raw); free(rec); free(pt); free(cstart); free(cpos); free(ord);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
#pragma omp atomic
    cstart[rec[i].key + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  memcpy(cpos, cstart, ((size_t)ncell + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = __atomic_fetch_add(&cpos[rec[i].key], 1, __ATOMIC_RELAXED);
    ord[p] = rec[i];
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t c = 0; c < ncell; ++c) {
    int64_t b = cstart[c], e = cstart[c + 1];
    for (int64_t i = b + 1; i < e; ++i) { /* insertion sort: cells hold a few points */
      rgg_rec x = ord[i];
      int64_t j = i;
      while (j > b && cmp_rec(&ord[j - 1], &x) > 0) { ord[j] = ord[j - 1]; --j; }
      ord[j] = x;
    }
  }
  progress("points ordered by cell", n, ncell);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d) pt[i * dim + d] = raw[ord[i].idx * dim + d];
  free(raw);
  free(rec);
  free(ord);
  free(cpos);
  double r2 = r * r;
  /* count, then fill: neighbours of i come from the 3^dim surrounding cells */
  uint64_t *xadj = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
  if (!xadj) { free(pt); free(cstart); return -1; }
  for (int pass = 0; pass < 2; ++pass) {
    int32_t *adj = NULL;
    if (pass == 1) {
      for (int64_t i = 0; i < n; ++i) xadj[i + 1] += xadj[i];
      adj = (int32_t *)malloc((xadj[n] ? xadj[n] : 1) * sizeof(int32_t));
      if (!adj) { free(pt); free(cstart); free(xadj); return -1; }
      out->adjncy = adj;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      const double *p = pt + i * dim;
      int64_t c[3] = {cell_of(p[0], g), cell_of(p[1], g), dim == 3 ? cell_of(p[2], g) : 0};
      uint64_t k = 0;
      int64_t zlo = dim == 3 ? c[2] - 1 : 0, zhi = dim == 3 ? c[2] + 1 : 0;
      for (int64_t z = zlo; z <= zhi; ++z) {
        if (z < 0 || z >= (dim == 3 ? g : 1)) continue;
        for (int64_t y = c[1] - 1; y <= c[1] + 1; ++y) {
          if (y < 0 || y >= g) continue;
          for (int64_t x = c[0] - 1; x <= c[0] + 1; ++x) {
            if (x < 0 || x >= g) continue;
            int64_t cell = z * g * g + y * g + x;
            for (int64_t j = cstart[cell]; j < cstart[cell + 1]; ++j) {
              if (j == i) continue;
              const double *q = pt + j * dim;
              double s = 0;
              for (int d = 0; d < dim; ++d) s += (p[d] - q[d]) * (p[d] - q[d]);
              if (s <= r2) {
                if (pass == 1) adj[xadj[i] + k] = (int32_t)j;
                ++k;
              }
            }
          }
        }
      }
      if (pass == 0) xadj[i + 1] = k;
      else if (k > 1) sort_i32(adj + xadj[i], (int64_t)k);
    }
    progress(pass == 0 ? "neighbours counted" : "neighbours written", n, pass);
  }
  free(pt);
  free(cstart);
  out->n = n;
  out->two_m = xadj[n];
  out->xadj = xadj;
  return 0;
}

void synth_free(synth_csr *g) {
  free(g->xadj);
  free(g->adjncy);
  g->xadj = NULL;
  g->adjncy = NULL;
}

void synth_copy(const synth_csr *g, uint64_t *xadj, int32_t *adjncy) {
  memcpy(xadj, g->xadj, ((size_t)g->n + 1) * sizeof(uint64_t));
  memcpy(adjncy, g->adjncy, g->two_m * sizeof(int32_t));
}

/* Seeded integer weights in [lo, hi] for `count` items (draw k = item k of
 * stream `seed`). Used to make weighted test graphs. */
void synth_weights(int64_t count, int32_t lo, int32_t hi, uint64_t seed, int32_t *out) {
  uint64_t span = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k)
    out[k] = (int32_t)((int64_t)lo + (int64_t)(sm_draw(seed, (uint64_t)k) % span));
}

/* Symmetric seeded edge weights: weight of {u, v} depends on the unordered
 * pair only, so the CSR stays symmetric in weights too. */
void synth_edge_weights(int64_t n, const uint64_t *xadj, const int32_t *adjncy,
                        int32_t lo, int32_t hi, uint64_t seed, int32_t *out) {
  uint64_t span = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n; ++u)
    for (uint64_t e = xadj[u]; e < xadj[u + 1]; ++e) {
      uint64_t a = (uint64_t)u, b = (uint64_t)(uint32_t)adjncy[e];
      uint64_t lo_id = a < b ? a : b, hi_id = a < b ? b : a;
      uint64_t h = sm_mix(seed ^ sm_mix(lo_id * 0x100000001B3ULL + hi_id));
      out[e] = (int32_t)((int64_t)lo + (int64_t)(h % span));
    }
}

/* Counter-based uniform double for host-side recipes (sizes, coin flips). */
double synth_unit(uint64_t seed, uint64_t k) { return sm_unit(seed, k); }
uint64_t synth_draw(uint64_t seed, uint64_t k) { return sm_draw(seed, k); }
