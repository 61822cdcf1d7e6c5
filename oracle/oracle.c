/*
 * CPU ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously correct reference for everything the GPU library
 * computes. Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the library never does, and the two share no code.
 *
 * Contents, each following the paper (arxiv 2410.19119, "Tera-Scale
 * Multilevel Graph Partitioning") and the synchronous reading of it:
 *   - VarInt / zigzag codec and the gap-encoded neighbourhood format, with
 *     or without interval encoding (Section III-A, "Compression Scheme");
 *   - size-constrained label-propagation clustering in synchronous rounds
 *     (Section IV-A, Algorithm 1 for what one vertex computes; the
 *     batch-synchronous form follows Section II-B on the distributed LP);
 *   - cluster contraction into a quotient graph (Section IV-B, the weight
 *     definition of a coarse edge);
 *   - the edge cut (Section I, the partitioning objective);
 *   - the coarsening loop (Sections I and II-A: cluster, contract, repeat);
 *   - the uncoarsening slice (Section II-A: an initial partition of the
 *     coarsest graph, projected level by level and refined there with
 *     size-constrained LP as in Section II-B; the balance bound of
 *     Section I).
 *
 * Floating point is never used: IDs are int32, offsets uint64, input weights
 * int32 >= 1, ratings / gains / cluster weights int64.
 *
 * Parallelism: the per-vertex rating loop is an OpenMP parallel-for. Each
 * vertex reads only the round's snapshot, so the result does not depend on the
 * thread count. Everything else is sequential.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_EOVERFLOW -3
#define ORC_EFORMAT -4

/* Format constants: neighbourhoods with more than 10 000 neighbours are split
 * into independently coded chunks of 1 000 (Section III-A). Interval-coded
 * graphs split above 4 000 neighbours: the most neighbours one piece of the
 * GPU's high-degree path rates, so that pieces start at chunks. */
#define ORC_CHUNK_THRESHOLD 10000
#define ORC_ITV_CHUNK_THRESHOLD 4000
#define ORC_CHUNK_LEN 1000
#define CHUNK_THRESHOLD(itv) ((itv) ? ORC_ITV_CHUNK_THRESHOLD : ORC_CHUNK_THRESHOLD)

/* ------------------------------------------------------------ VarInt ---- */
/* VarInt (Section III-A): 7 payload bits per byte, least significant group
 * first; the high bit of a byte says another byte of the same number
 * follows. */
size_t orc_varint_put(uint8_t *out, uint64_t x) {
  size_t k = 0;
  while (x >= 0x80) {
    out[k++] = (uint8_t)(x & 0x7F) | 0x80;
    x >>= 7;
  }
  out[k++] = (uint8_t)x;
  return k;
}

/* Reads one VarInt at *pos (advancing it). Returns 0 on a malformed or
 * truncated number (more than 10 bytes or running past `end`). */
int orc_varint_get(const uint8_t *buf, uint64_t end, uint64_t *pos, uint64_t *value) {
  uint64_t x = 0;
  for (int shift = 0; shift < 70; shift += 7) {
    if (*pos >= end) return 0;
    uint8_t b = buf[(*pos)++];
    x |= (uint64_t)(b & 0x7F) << shift;
    if (!(b & 0x80)) {
      *value = x;
      return 1;
    }
  }
  return 0;
}

/* Signed values (the first neighbour relative to u, weight differences) are
 * mapped to unsigned ones so small magnitudes stay short: 0,-1,1,-2 -> 0,1,2,3. */
uint64_t orc_zigzag(int64_t x) { return ((uint64_t)x << 1) ^ (uint64_t)(x >> 63); }
int64_t orc_unzigzag(uint64_t z) { return (int64_t)(z >> 1) ^ -(int64_t)(z & 1); }

/* ------------------------------------------------------- compression ---- */
typedef struct {
  int32_t v, w;
} orc_nb;

static int cmp_nb(const void *a, const void *b) {
  const orc_nb *x = (const orc_nb *)a, *y = (const orc_nb *)b;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  return (x->w > y->w) - (x->w < y->w);
}

/* Upper bound of the compressed size, for buffer allocation. */
uint64_t orc_compress_bound(int32_t n, uint64_t two_m, int weighted) {
  return (uint64_t)n * 10 + two_m * (weighted ? 10 : 5) + (two_m / ORC_CHUNK_LEN + 1) * 4 + 16;
}

/* Encodes one neighbourhood, already sorted by (id, weight), at `out`.
 * Layout, in this order:
 *   VarInt(first edge ID of u)     -- gives degrees and edge IDs (Section III-A)
 *   if deg > 10 000 (4 000 with intervals): (ceil(deg/1000) - 1) little-endian
 *                    uint32 byte offsets, relative to the start of this
 *                    record, of chunks 2, 3, ...
 *   per chunk of up to 1 000 neighbours (the whole neighbourhood if it is not
 *   split), without intervals:
 *     VarInt(zigzag(v_0 - u)), then VarInt(v_i - v_{i-1}) for the rest (gap
 *     encoding); if weighted, each neighbour code is followed by
 *     VarInt(zigzag(w_i - w_{i-1})) with w_{-1} = 0 at the chunk start.
 *   with intervals (Section III-A: a run x, x+1, ..., x+l-1 of l >= 3
 *   consecutive IDs is kept as the pair (x, l)), per chunk:
 *     the chunk's neighbours are split, left to right, into maximal runs of
 *     IDs each one above the previous neighbour's; runs of length >= 3 are
 *     intervals, every other neighbour a residual;
 *     VarInt(k) = number of intervals;
 *     per interval j: VarInt(zigzag(x_j - u)), VarInt(l_j - 3);
 *     if weighted: the weights of the interval neighbours, interval by
 *       interval, each as VarInt(zigzag(w - w_prev)), w_prev = 0 at the
 *       chunk start;
 *     the residuals r_0 < r_1 ... (in neighbour order) gap encoded as above:
 *       VarInt(zigzag(r_0 - u)), then VarInt(r_i - r_{i-1}); if weighted each
 *       followed by VarInt(zigzag(w - w_prev)), the weight chain continuing
 *       from the interval weights.
 * Returns the number of bytes written. */
static uint64_t encode_chunk_gaps(int32_t u, const orc_nb *nb, uint64_t b, uint64_t e, int weighted,
                                  uint8_t *out) {
  uint64_t k = 0;
  int32_t wprev = 0;
  for (uint64_t i = b; i < e; ++i) {
    uint64_t code = (i == b) ? orc_zigzag((int64_t)nb[i].v - (int64_t)u)
                             : (uint64_t)((int64_t)nb[i].v - (int64_t)nb[i - 1].v);
    k += orc_varint_put(out + k, code);
    if (weighted) {
      k += orc_varint_put(out + k, orc_zigzag((int64_t)nb[i].w - (int64_t)wprev));
      wprev = nb[i].w;
    }
  }
  return k;
}

/* Marks the neighbours of nb[b..e) that belong to intervals (runs of >= 3
 * IDs, each exactly one above the previous neighbour, found left to right)
 * in in_run[i - b]; returns the number of intervals. */
static uint64_t find_intervals(const orc_nb *nb, uint64_t b, uint64_t e, uint8_t *in_run) {
  uint64_t count = 0;
  for (uint64_t i = b; i < e;) {
    uint64_t j = i + 1;
    while (j < e && (int64_t)nb[j].v == (int64_t)nb[j - 1].v + 1) ++j;
    const int is_interval = j - i >= 3;
    for (uint64_t t = i; t < (is_interval ? j : i + 1); ++t) in_run[t - b] = (uint8_t)is_interval;
    if (is_interval) {
      ++count;
      i = j;
    } else {
      ++i;
    }
  }
  return count;
}

static uint64_t encode_chunk_intervals(int32_t u, const orc_nb *nb, uint64_t b, uint64_t e, int weighted,
                                       uint8_t *in_run, uint8_t *out) {
  uint64_t k = orc_varint_put(out, find_intervals(nb, b, e, in_run));
  for (uint64_t i = b; i < e;) { /* the (start, length - 3) pairs */
    if (!in_run[i - b]) { ++i; continue; }
    uint64_t j = i + 1;
    while (j < e && in_run[j - b] && (int64_t)nb[j].v == (int64_t)nb[j - 1].v + 1) ++j;
    k += orc_varint_put(out + k, orc_zigzag((int64_t)nb[i].v - (int64_t)u));
    k += orc_varint_put(out + k, j - i - 3);
    i = j;
  }
  int32_t wprev = 0;
  if (weighted)
    for (uint64_t i = b; i < e; ++i)
      if (in_run[i - b]) {
        k += orc_varint_put(out + k, orc_zigzag((int64_t)nb[i].w - (int64_t)wprev));
        wprev = nb[i].w;
      }
  int first = 1;
  int32_t rprev = 0;
  for (uint64_t i = b; i < e; ++i) {
    if (in_run[i - b]) continue;
    uint64_t code = first ? orc_zigzag((int64_t)nb[i].v - (int64_t)u) : (uint64_t)((int64_t)nb[i].v - rprev);
    k += orc_varint_put(out + k, code);
    if (weighted) {
      k += orc_varint_put(out + k, orc_zigzag((int64_t)nb[i].w - (int64_t)wprev));
      wprev = nb[i].w;
    }
    rprev = nb[i].v;
    first = 0;
  }
  return k;
}

static uint64_t encode_nbh(int32_t u, uint64_t first_edge, const orc_nb *nb, uint64_t deg,
                           int weighted, int intervals, uint8_t *in_run, uint8_t *out) {
  uint64_t k = orc_varint_put(out, first_edge);
  uint64_t nchunks = deg > CHUNK_THRESHOLD(intervals) ? (deg + ORC_CHUNK_LEN - 1) / ORC_CHUNK_LEN : 1;
  uint64_t table = k;
  if (nchunks > 1) k += 4 * (nchunks - 1);
  for (uint64_t ch = 0; ch < nchunks; ++ch) {
    uint64_t b = ch * (nchunks > 1 ? ORC_CHUNK_LEN : 0);
    uint64_t e = nchunks > 1 ? b + ORC_CHUNK_LEN : deg;
    if (e > deg) e = deg;
    if (ch > 0) {
      uint32_t rel = (uint32_t)k;
      memcpy(out + table + 4 * (ch - 1), &rel, 4);
    }
    k += intervals ? encode_chunk_intervals(u, nb, b, e, weighted, in_run, out + k)
                   : encode_chunk_gaps(u, nb, b, e, weighted, out + k);
  }
  return k;
}

/* Compresses a CSR (neighbourhoods in any order; they are sorted here).
 * offs gets n+1 byte offsets; bytes must hold orc_compress_bound() bytes. */
int orc_compress_ex(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                    int intervals, uint64_t *offs, uint8_t *bytes, uint64_t *nbytes) {
  uint64_t maxdeg = 0;
  for (int32_t u = 0; u < n; ++u)
    if (xadj[u + 1] - xadj[u] > maxdeg) maxdeg = xadj[u + 1] - xadj[u];
  orc_nb *nb = (orc_nb *)malloc((maxdeg ? maxdeg : 1) * sizeof(orc_nb));
  uint8_t *in_run = (uint8_t *)malloc(maxdeg ? maxdeg : 1);
  if (!nb || !in_run) { free(nb); free(in_run); return ORC_ENOMEM; }
  uint64_t pos = 0;
  for (int32_t u = 0; u < n; ++u) {
    uint64_t d = xadj[u + 1] - xadj[u];
    for (uint64_t i = 0; i < d; ++i) {
      nb[i].v = adjncy[xadj[u] + i];
      nb[i].w = adjwgt ? adjwgt[xadj[u] + i] : 1;
    }
    qsort(nb, d, sizeof(orc_nb), cmp_nb);
    offs[u] = pos;
    pos += encode_nbh(u, xadj[u], nb, d, adjwgt != NULL, intervals, in_run, bytes + pos);
  }
  offs[n] = pos;
  *nbytes = pos;
  free(nb);
  free(in_run);
  return ORC_OK;
}

int orc_compress(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                 uint64_t *offs, uint8_t *bytes, uint64_t *nbytes) {
  return orc_compress_ex(n, xadj, adjncy, adjwgt, 0, offs, bytes, nbytes);
}

/* Decodes one chunk of `cnt` neighbours starting at byte *p (advancing it)
 * into ids / wts; returns 0 on a malformed stream. Interval chunks give the
 * interval neighbours first, then the residuals. */
static int decode_chunk(const uint8_t *bytes, uint64_t end, uint64_t *p, int32_t u, int32_t n, uint64_t cnt,
                        int weighted, int intervals, int32_t *ids, int32_t *wts) {
  uint64_t i = 0, code;
  int64_t wprev = 0;
  if (intervals) {
    uint64_t k;
    if (!orc_varint_get(bytes, end, p, &k) || k > cnt) return 0;
    for (uint64_t j = 0; j < k; ++j) {
      uint64_t zs, lm3;
      if (!orc_varint_get(bytes, end, p, &zs) || !orc_varint_get(bytes, end, p, &lm3)) return 0;
      int64_t x = (int64_t)u + orc_unzigzag(zs);
      uint64_t len = lm3 + 3;
      if (len > cnt - i || x < 0 || x + (int64_t)len > n) return 0;
      for (uint64_t t = 0; t < len; ++t) ids[i++] = (int32_t)(x + (int64_t)t);
    }
    for (uint64_t t = 0; t < i; ++t) {
      if (weighted) {
        if (!orc_varint_get(bytes, end, p, &code)) return 0;
        wprev += orc_unzigzag(code);
      } else {
        wprev = 1;
      }
      wts[t] = (int32_t)wprev;
    }
  }
  int64_t prev = 0;
  for (uint64_t r = 0; i < cnt; ++i, ++r) {
    if (!orc_varint_get(bytes, end, p, &code)) return 0;
    int64_t v = r == 0 ? (int64_t)u + orc_unzigzag(code) : prev + (int64_t)code;
    if (v < 0 || v >= n) return 0;
    ids[i] = (int32_t)v;
    prev = v;
    if (weighted) {
      if (!orc_varint_get(bytes, end, p, &code)) return 0;
      wprev += orc_unzigzag(code);
    } else {
      wprev = 1;
    }
    wts[i] = (int32_t)wprev;
  }
  return 1;
}

/* Decodes the compressed graph back to CSR. Degrees come from the first-edge
 * headers (deg(u) = fe(u+1) - fe(u), fe(n) = 2m). The chunk table of every
 * split neighbourhood is checked against where the chunks actually start.
 * Neighbourhoods come out sorted by (ID, weight), as they went in. */
int orc_decompress_ex(int32_t n, uint64_t two_m, int weighted, int intervals, const uint64_t *offs,
                      const uint8_t *bytes, uint64_t *xadj, int32_t *adjncy, int32_t *adjwgt) {
  uint64_t end = offs[n];
  uint64_t *fe = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
  if (!fe) return ORC_ENOMEM;
  for (int32_t u = 0; u < n; ++u) {
    uint64_t p = offs[u];
    if (!orc_varint_get(bytes, end, &p, &fe[u])) { free(fe); return ORC_EFORMAT; }
  }
  fe[n] = two_m;
  if (n > 0 && fe[0] != 0) { free(fe); return ORC_EFORMAT; }
  uint64_t maxdeg = 0;
  for (int32_t u = 0; u <= n; ++u) {
    if (u > 0 && fe[u] < fe[u - 1]) { free(fe); return ORC_EFORMAT; }
    if (u > 0 && fe[u] - fe[u - 1] > maxdeg) maxdeg = fe[u] - fe[u - 1];
    xadj[u] = fe[u];
  }
  orc_nb *nb = (orc_nb *)malloc((maxdeg ? maxdeg : 1) * sizeof(orc_nb));
  int32_t *ids = (int32_t *)malloc((maxdeg ? maxdeg : 1) * sizeof(int32_t));
  int32_t *wts = (int32_t *)malloc((maxdeg ? maxdeg : 1) * sizeof(int32_t));
  if (!nb || !ids || !wts) { free(fe); free(nb); free(ids); free(wts); return ORC_ENOMEM; }
  int status = ORC_OK;
  for (int32_t u = 0; u < n && status == ORC_OK; ++u) {
    uint64_t deg = fe[u + 1] - fe[u];
    uint64_t p = offs[u], hdr;
    orc_varint_get(bytes, end, &p, &hdr);
    uint64_t nchunks = deg > CHUNK_THRESHOLD(intervals) ? (deg + ORC_CHUNK_LEN - 1) / ORC_CHUNK_LEN : 1;
    uint64_t table = p;
    if (nchunks > 1) p += 4 * (nchunks - 1);
    for (uint64_t ch = 0; ch < nchunks; ++ch) {
      uint64_t b = nchunks > 1 ? ch * ORC_CHUNK_LEN : 0;
      uint64_t e = nchunks > 1 ? b + ORC_CHUNK_LEN : deg;
      if (e > deg) e = deg;
      if (ch > 0) {
        uint32_t rel;
        memcpy(&rel, bytes + table + 4 * (ch - 1), 4);
        if (offs[u] + rel != p) { status = ORC_EFORMAT; break; }
      }
      if (!decode_chunk(bytes, offs[u + 1], &p, u, n, e - b, weighted, intervals, ids + b, wts + b)) {
        status = ORC_EFORMAT;
        break;
      }
    }
    if (status != ORC_OK) break;
    if (p != offs[u + 1]) { status = ORC_EFORMAT; break; }
    for (uint64_t i = 0; i < deg; ++i) {
      nb[i].v = ids[i];
      nb[i].w = wts[i];
    }
    if (intervals) qsort(nb, deg, sizeof(orc_nb), cmp_nb);
    for (uint64_t i = 0; i < deg; ++i) {
      adjncy[fe[u] + i] = nb[i].v;
      if (adjwgt) adjwgt[fe[u] + i] = nb[i].w;
    }
  }
  free(fe);
  free(nb);
  free(ids);
  free(wts);
  return status;
}

int orc_decompress(int32_t n, uint64_t two_m, int weighted, const uint64_t *offs, const uint8_t *bytes,
                   uint64_t *xadj, int32_t *adjncy, int32_t *adjwgt) {
  return orc_decompress_ex(n, two_m, weighted, 0, offs, bytes, xadj, adjncy, adjwgt);
}

/* ---------------------------------------------- label propagation ---- */
/* Tie-break priority of cluster c in round r: the SplitMix64 output function
 * (Steele, Lea and Flood 2014) applied to seed XOR (r << 32) XOR c. It is a
 * bijection of c, so two distinct clusters never share a priority. The
 * smaller value wins a tie in rating. */
uint64_t orc_tiebreak_key(uint64_t seed, uint32_t round, uint32_t c) {
  uint64_t z = seed ^ ((uint64_t)round << 32) ^ (uint64_t)c;
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  int32_t c;
  int64_t r;
} orc_rating;

static int cmp_rating_label(const void *a, const void *b) {
  const orc_rating *x = (const orc_rating *)a, *y = (const orc_rating *)b;
  return (x->c > y->c) - (x->c < y->c);
}

typedef struct {
  int32_t u, target;
  int64_t gain, w;
} orc_prop;

static int cmp_prop(const void *a, const void *b) {
  const orc_prop *x = (const orc_prop *)a, *y = (const orc_prop *)b;
  if (x->target != y->target) return x->target < y->target ? -1 : 1;
  if (x->gain != y->gain) return x->gain > y->gain ? -1 : 1; /* gain descending */
  return (x->u > y->u) - (x->u < y->u);                      /* then vertex ascending */
}

typedef struct {
  int32_t rounds_run;       /* rounds that made at least one proposal */
  int64_t proposals[64];    /* per round (first 64 rounds) */
  int64_t moves[64];
} orc_lp_stats;

/* The best move of u under the snapshot (C0, W0), or none.
 * Rating of cluster c = sum of weights of the edges from u into c (Section
 * IV-A1). Own = rating of u's current cluster. Candidates: clusters other
 * than u's own with positive rating that can take u without exceeding the
 * cap. The winner has the largest rating, ties broken by the smaller
 * tie-break key. A move is proposed only if it strictly beats staying. */
static int best_move(int32_t u, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                     const int32_t *vwgt, const int32_t *C0, const int64_t *W0, int64_t cap,
                     uint64_t seed, uint32_t round, orc_rating *buf, int32_t *target, int64_t *gain) {
  uint64_t d = xadj[u + 1] - xadj[u];
  if (d == 0) return 0;
  for (uint64_t i = 0; i < d; ++i) {
    int32_t v = adjncy[xadj[u] + i];
    buf[i].c = C0[v];
    buf[i].r = adjwgt ? adjwgt[xadj[u] + i] : 1;
  }
  qsort(buf, d, sizeof(orc_rating), cmp_rating_label);
  /* sum runs of equal labels into one rating per distinct cluster */
  uint64_t k = 0;
  for (uint64_t i = 0; i < d; ++i) {
    if (k > 0 && buf[k - 1].c == buf[i].c) buf[k - 1].r += buf[i].r;
    else buf[k++] = buf[i];
  }
  int32_t own_c = C0[u];
  int64_t wu = vwgt ? vwgt[u] : 1;
  int64_t own = 0;
  int found = 0;
  int32_t best_c = 0;
  int64_t best_r = 0;
  uint64_t best_key = 0;
  for (uint64_t i = 0; i < k; ++i) {
    int32_t c = buf[i].c;
    if (c == own_c) {
      own = buf[i].r;
      continue;
    }
    if (buf[i].r <= 0) continue;
    if (W0[c] + wu > cap) continue;
    uint64_t key = orc_tiebreak_key(seed, round, (uint32_t)c);
    if (!found || buf[i].r > best_r || (buf[i].r == best_r && key < best_key)) {
      found = 1;
      best_c = c;
      best_r = buf[i].r;
      best_key = key;
    }
  }
  if (!found || best_r <= own) return 0;
  *target = best_c;
  *gain = best_r - own;
  return 1;
}

/* Sub-round of vertex u among S: the tie-break mix above applied to the
 * fixed salt ORC_SUBROUND_SALT and u (round 0), modulo S. It depends on u
 * only, so a vertex keeps its sub-round for the whole call. */
#define ORC_SUBROUND_SALT 0x6A09E667F3BCC909ull
uint32_t orc_subround(uint32_t u, uint32_t S) {
  return (uint32_t)(orc_tiebreak_key(ORC_SUBROUND_SALT, 0, u) % S);
}

/* The synchronous rounds shared by clustering and refinement, starting from
 * the labelling in `labels` (every label in [0, n)), each round split into S
 * sub-rounds (S = 1: one synchronous step per round).
 * Per sub-round s of round r: the vertices of sub-round s compute their best
 * move against the snapshot taken at the start of the sub-round (tie-break
 * keys of round r); then, for each target cluster, the proposals are taken
 * in (gain descending, vertex ascending) order and admitted while the
 * running sum of their weights, added to the cluster's weight at the start of
 * the sub-round, stays within the cap; admitted vertices move. A later
 * sub-round sees the moves of the earlier ones, as the paper's in-place
 * updates let later vertices see earlier moves (Algorithms 1 and 2), but in
 * a fixed order. A round with no proposal in any sub-round is a fixed point,
 * so the loop stops there. Cluster weights are recomputed from the labels.
 * Rounds are numbered from first_round (their tie-break keys); statistics are
 * indexed from the first round of the call. */
static int lp_rounds(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                     const int32_t *vwgt, int64_t cap, int32_t first_round, int32_t rounds, int32_t subrounds,
                     uint64_t seed, int32_t *labels, orc_lp_stats *stats) {
  if (stats) memset(stats, 0, sizeof(*stats));
  int32_t *C0 = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  int64_t *W = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int64_t *W0 = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int32_t *ptarget = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  int64_t *pgain = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  orc_prop *props = (orc_prop *)malloc(((size_t)n + 1) * sizeof(orc_prop));
  if (!C0 || !W || !W0 || !ptarget || !pgain || !props) {
    free(C0); free(W); free(W0); free(ptarget); free(pgain); free(props);
    return ORC_ENOMEM;
  }
  uint64_t maxdeg = 0;
  for (int32_t c = 0; c < n; ++c) W[c] = 0;
  for (int32_t u = 0; u < n; ++u) {
    W[labels[u]] += vwgt ? vwgt[u] : 1;
    if (xadj[u + 1] - xadj[u] > maxdeg) maxdeg = xadj[u + 1] - xadj[u];
  }
  int status = ORC_OK;
  const uint32_t S = (uint32_t)subrounds;
  for (int32_t r = 0; r < rounds; ++r) {
    int64_t round_props = 0;
    for (uint32_t sr = 0; sr < S; ++sr) {
      memcpy(C0, labels, (size_t)n * sizeof(int32_t));
      memcpy(W0, W, (size_t)n * sizeof(int64_t));
      int fail = 0;
#pragma omp parallel
      {
        orc_rating *buf = (orc_rating *)malloc((maxdeg ? maxdeg : 1) * sizeof(orc_rating));
        if (!buf) {
#pragma omp atomic write
          fail = 1;
        }
#pragma omp for schedule(dynamic, 256)
        for (int32_t u = 0; u < n; ++u) {
          ptarget[u] = -1;
          if (S > 1 && orc_subround((uint32_t)u, S) != sr) continue;
          if (buf && best_move(u, xadj, adjncy, adjwgt, vwgt, C0, W0, cap, seed, (uint32_t)(first_round + r), buf,
                               &ptarget[u], &pgain[u]) == 0)
            ptarget[u] = -1;
        }
        free(buf);
      }
      if (fail) { status = ORC_ENOMEM; break; }
      int64_t np = 0;
      for (int32_t u = 0; u < n; ++u) {
        if (ptarget[u] < 0) continue;
        props[np].u = u;
        props[np].target = ptarget[u];
        props[np].gain = pgain[u];
        props[np].w = vwgt ? vwgt[u] : 1;
        ++np;
      }
      if (np == 0) continue; /* nothing moves in this sub-round */
      round_props += np;
      qsort(props, (size_t)np, sizeof(orc_prop), cmp_prop);
      int64_t moves = 0;
      for (int64_t i = 0; i < np;) {
        int32_t c = props[i].target;
        int64_t sum = 0;
        int open = 1;
        int64_t j = i;
        for (; j < np && props[j].target == c; ++j) {
          sum += props[j].w;
          if (open && W0[c] + sum <= cap) {
            labels[props[j].u] = c;
            ++moves;
          } else {
            open = 0; /* longest admissible prefix: nothing after a rejection */
          }
        }
        i = j;
      }
      /* cluster weights from scratch: W[c] = sum of w(u) over members of c */
      for (int32_t c = 0; c < n; ++c) W[c] = 0;
      for (int32_t u = 0; u < n; ++u) W[labels[u]] += vwgt ? vwgt[u] : 1;
      if (stats && r < 64) {
        stats->proposals[r] += np;
        stats->moves[r] += moves;
      }
    }
    if (status != ORC_OK || round_props == 0) break;
    if (stats) stats->rounds_run = r + 1;
  }
  free(C0); free(W); free(W0); free(ptarget); free(pgain); free(props);
  return status;
}

/* Size-constrained LP clustering (Section IV-A): every vertex starts in its
 * own cluster (C[u] = u), then the synchronous rounds above.
 * labels (out): n cluster IDs in [0, n); not renumbered. */
int orc_lp_cluster_sub(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                       const int32_t *vwgt, int64_t cap, int32_t rounds, int32_t subrounds, uint64_t seed,
                       int32_t *labels, orc_lp_stats *stats) {
  if (n < 0 || cap < 1 || rounds < 0 || subrounds < 1 || subrounds > 64) return ORC_EINVAL;
  for (int32_t u = 0; u < n; ++u) labels[u] = u;
  return lp_rounds(n, xadj, adjncy, adjwgt, vwgt, cap, 0, rounds, subrounds, seed, labels, stats);
}

/* The same synchronous clustering rounds resumed from the labels a previous
 * call left (rounds first_round .. first_round + rounds - 1, one synchronous
 * step each): running rounds 0..R-1 in pieces gives exactly the labels of one
 * call with R rounds, since the state between rounds is the labelling alone
 * (cluster weights are recomputed from it). */
int orc_lp_rounds_from(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                       const int32_t *vwgt, int64_t cap, int32_t first_round, int32_t rounds, uint64_t seed,
                       int32_t *labels, orc_lp_stats *stats) {
  if (n < 0 || cap < 1 || first_round < 0 || rounds < 0) return ORC_EINVAL;
  for (int32_t u = 0; u < n; ++u)
    if (labels[u] < 0 || labels[u] >= n) return ORC_EINVAL;
  return lp_rounds(n, xadj, adjncy, adjwgt, vwgt, cap, first_round, rounds, 1, seed, labels, stats);
}

/* Size-constrained LP refinement of a k-way partition (Section II-B: the
 * refinement runs label propagation from the given partition, with the
 * blocks as the labels): the same synchronous rounds, started from the
 * blocks in `labels`, with the maximum block weight as the cap. A vertex
 * moves to the adjacent block with the most edge weight to it if that beats
 * its own block and the block can take it; moves into a block are admitted
 * while the block stays within the cap.
 * labels (in/out): the block of every vertex, in [0, k); 1 <= k <= n. */
int orc_lp_refine(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                  const int32_t *vwgt, int32_t k, int64_t max_block_weight, int32_t rounds, int32_t subrounds,
                  uint64_t seed, int32_t *labels, orc_lp_stats *stats) {
  if (n < 0 || k < 1 || (n > 0 && k > n) || max_block_weight < 1 || rounds < 0 || subrounds < 1 ||
      subrounds > 64)
    return ORC_EINVAL;
  for (int32_t u = 0; u < n; ++u)
    if (labels[u] < 0 || labels[u] >= k) return ORC_EINVAL;
  return lp_rounds(n, xadj, adjncy, adjwgt, vwgt, max_block_weight, 0, rounds, subrounds, seed, labels, stats);
}

/* Initial k-way partition by contiguous weight: the vertices, in ID order,
 * fill the blocks one after another; vertex u goes to block
 * floor(k * P_u / c(V)), where P_u is the total weight of the vertices
 * before u and c(V) the total weight. Every block then weighs less than
 * c(V)/k plus one vertex weight. k >= 1. */
int orc_initial_partition(int32_t n, const int32_t *vwgt, int32_t k, int32_t *labels) {
  if (n < 0 || k < 1) return ORC_EINVAL;
  unsigned __int128 total = 0, P = 0;
  for (int32_t u = 0; u < n; ++u) total += (unsigned __int128)(vwgt ? vwgt[u] : 1);
  for (int32_t u = 0; u < n; ++u) {
    labels[u] = (int32_t)(((unsigned __int128)k * P) / total);
    P += (unsigned __int128)(vwgt ? vwgt[u] : 1);
  }
  return ORC_OK;
}

int orc_lp_cluster(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                   const int32_t *vwgt, int64_t cap, int32_t rounds, uint64_t seed, int32_t *labels,
                   orc_lp_stats *stats) {
  return orc_lp_cluster_sub(n, xadj, adjncy, adjwgt, vwgt, cap, rounds, 1, seed, labels, stats);
}

/* The paper's asynchronous LP as a quality reference (Algorithms 1 and 2,
 * sequential): per round the vertices are visited in a random order (a
 * Fisher-Yates shuffle drawing index j for position i as the tie-break mix of
 * (seed ^ ORC_ORDER_SALT, round, i) modulo i + 1), and each moves at once to
 * its best cluster under the current labels and weights (same rating, cap,
 * tie-break and gain rules as the synchronous rounds). A round without a move
 * ends the call. stats: proposals = moves per round. */
#define ORC_ORDER_SALT 0xBB67AE8584CAA73Bull
int orc_lp_cluster_async(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                         const int32_t *vwgt, int64_t cap, int32_t rounds, uint64_t seed, int32_t *labels,
                         orc_lp_stats *stats) {
  if (n < 0 || cap < 1 || rounds < 0) return ORC_EINVAL;
  if (stats) memset(stats, 0, sizeof(*stats));
  int64_t *W = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int32_t *order = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  uint64_t maxdeg = 0;
  for (int32_t u = 0; u < n; ++u)
    if (xadj[u + 1] - xadj[u] > maxdeg) maxdeg = xadj[u + 1] - xadj[u];
  orc_rating *buf = (orc_rating *)malloc((maxdeg ? maxdeg : 1) * sizeof(orc_rating));
  if (!W || !order || !buf) {
    free(W); free(order); free(buf);
    return ORC_ENOMEM;
  }
  for (int32_t u = 0; u < n; ++u) {
    labels[u] = u;
    W[u] = vwgt ? vwgt[u] : 1;
  }
  for (int32_t r = 0; r < rounds; ++r) {
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
      const int32_t j = (int32_t)(orc_tiebreak_key(seed ^ ORC_ORDER_SALT, (uint32_t)r, (uint32_t)i) %
                                  (uint64_t)(i + 1));
      const int32_t t = order[i];
      order[i] = order[j];
      order[j] = t;
    }
    int64_t moves = 0;
    for (int32_t i = 0; i < n; ++i) {
      const int32_t u = order[i];
      int32_t target;
      int64_t gain;
      if (!best_move(u, xadj, adjncy, adjwgt, vwgt, labels, W, cap, seed, (uint32_t)r, buf, &target, &gain))
        continue;
      const int64_t wu = vwgt ? vwgt[u] : 1;
      W[labels[u]] -= wu;
      W[target] += wu;
      labels[u] = target;
      ++moves;
    }
    if (moves == 0) break;
    if (stats) {
      stats->rounds_run = r + 1;
      if (r < 64) stats->proposals[r] = stats->moves[r] = moves;
    }
  }
  free(W); free(order); free(buf);
  return ORC_OK;
}

/* One LP round from an arbitrary snapshot, for sampled checks: fills the
 * proposal (target or -1, gain) of each listed vertex. */
int orc_lp_proposals(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                     const int32_t *vwgt, const int32_t *C0, const int64_t *W0, int64_t cap,
                     uint64_t seed, int32_t round, int64_t count, const int32_t *vertices,
                     int32_t *target, int64_t *gain) {
  (void)n;
  uint64_t maxdeg = 0;
  for (int64_t i = 0; i < count; ++i) {
    int32_t u = vertices[i];
    if (xadj[u + 1] - xadj[u] > maxdeg) maxdeg = xadj[u + 1] - xadj[u];
  }
  orc_rating *buf = (orc_rating *)malloc((maxdeg ? maxdeg : 1) * sizeof(orc_rating));
  if (!buf) return ORC_ENOMEM;
  for (int64_t i = 0; i < count; ++i) {
    target[i] = -1;
    gain[i] = 0;
    best_move(vertices[i], xadj, adjncy, adjwgt, vwgt, C0, W0, cap, seed, (uint32_t)round, buf,
              &target[i], &gain[i]);
  }
  free(buf);
  return ORC_OK;
}

/* ------------------------------------------------------- contraction ---- */
typedef struct {
  int32_t b;
  int64_t w;
} orc_cedge;

static int cmp_cedge(const void *a, const void *b) {
  const orc_cedge *x = (const orc_cedge *)a, *y = (const orc_cedge *)b;
  return (x->b > y->b) - (x->b < y->b);
}

/* Quotient graph of the clustering (Section IV-B): one coarse vertex per
 * nonempty cluster, numbered by increasing cluster label; its weight is the
 * sum of its members' weights; the coarse edge (a, b) carries the summed
 * weight of all fine edges from members of a to members of b, for a != b
 * (edges inside a cluster vanish). Neighbourhoods are sorted by coarse ID.
 * Output arrays are allocated here (free with orc_free); map[u] = coarse ID
 * of u's cluster. Returns ORC_EOVERFLOW if a coarse edge weight exceeds
 * INT32_MAX. */
int orc_contract(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                 const int32_t *vwgt, const int32_t *labels, int32_t *n_out, uint64_t **cxadj,
                 int32_t **cadjncy, int32_t **cadjwgt, int32_t **cvwgt, int32_t *map) {
  int32_t *id = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  if (!id) return ORC_ENOMEM;
  for (int32_t c = 0; c < n; ++c) id[c] = 0;
  for (int32_t u = 0; u < n; ++u) {
    if (labels[u] < 0 || labels[u] >= n) { free(id); return ORC_EINVAL; }
    id[labels[u]] = 1;
  }
  int32_t nc = 0;
  for (int32_t c = 0; c < n; ++c) id[c] = id[c] ? nc++ : -1;
  /* members of each coarse vertex, in increasing fine ID */
  uint64_t *mstart = (uint64_t *)calloc((size_t)nc + 1, sizeof(uint64_t));
  int32_t *members = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  int32_t *vw = (int32_t *)calloc((size_t)nc + 1, sizeof(int32_t));
  int64_t *vw64 = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
  if (!mstart || !members || !vw || !vw64) { free(id); free(mstart); free(members); free(vw); free(vw64); return ORC_ENOMEM; }
  for (int32_t u = 0; u < n; ++u) mstart[id[labels[u]] + 1]++;
  for (int32_t a = 0; a < nc; ++a) mstart[a + 1] += mstart[a];
  {
    uint64_t *fill = (uint64_t *)malloc(((size_t)nc + 1) * sizeof(uint64_t));
    if (!fill) { free(id); free(mstart); free(members); free(vw); free(vw64); return ORC_ENOMEM; }
    memcpy(fill, mstart, ((size_t)nc + 1) * sizeof(uint64_t));
    for (int32_t u = 0; u < n; ++u) members[fill[id[labels[u]]]++] = u;
    free(fill);
  }
  int status = ORC_OK;
  for (int32_t u = 0; u < n; ++u) {
    int32_t a = id[labels[u]];
    map[u] = a;
    vw64[a] += vwgt ? vwgt[u] : 1;
  }
  for (int32_t a = 0; a < nc; ++a) {
    if (vw64[a] > INT32_MAX) status = ORC_EOVERFLOW;
    vw[a] = (int32_t)vw64[a];
  }
  free(vw64);
  /* per coarse vertex: gather (coarse neighbour, weight), sort, sum runs */
  uint64_t *cx = (uint64_t *)calloc((size_t)nc + 1, sizeof(uint64_t));
  uint64_t cap_edges = 1024, used = 0;
  int32_t *ca = (int32_t *)malloc(cap_edges * sizeof(int32_t));
  int32_t *cw = (int32_t *)malloc(cap_edges * sizeof(int32_t));
  uint64_t bufcap = 1024;
  orc_cedge *buf = (orc_cedge *)malloc(bufcap * sizeof(orc_cedge));
  if (!cx || !ca || !cw || !buf) { status = ORC_ENOMEM; goto done; }
  for (int32_t a = 0; a < nc; ++a) {
    uint64_t k = 0;
    for (uint64_t m = mstart[a]; m < mstart[a + 1]; ++m) {
      int32_t u = members[m];
      for (uint64_t e = xadj[u]; e < xadj[u + 1]; ++e) {
        int32_t b = id[labels[adjncy[e]]];
        if (b == a) continue;
        if (k == bufcap) {
          bufcap *= 2;
          orc_cedge *nb = (orc_cedge *)realloc(buf, bufcap * sizeof(orc_cedge));
          if (!nb) { status = ORC_ENOMEM; goto done; }
          buf = nb;
        }
        buf[k].b = b;
        buf[k].w = adjwgt ? adjwgt[e] : 1;
        ++k;
      }
    }
    qsort(buf, k, sizeof(orc_cedge), cmp_cedge);
    uint64_t j = 0;
    for (uint64_t i = 0; i < k; ++i) {
      if (j > 0 && buf[j - 1].b == buf[i].b) buf[j - 1].w += buf[i].w;
      else buf[j++] = buf[i];
    }
    while (used + j > cap_edges) {
      cap_edges *= 2;
      int32_t *na = (int32_t *)realloc(ca, cap_edges * sizeof(int32_t));
      if (!na) { status = ORC_ENOMEM; goto done; }
      ca = na;
      int32_t *nw = (int32_t *)realloc(cw, cap_edges * sizeof(int32_t));
      if (!nw) { status = ORC_ENOMEM; goto done; }
      cw = nw;
    }
    for (uint64_t i = 0; i < j; ++i) {
      if (buf[i].w > INT32_MAX) status = ORC_EOVERFLOW;
      ca[used + i] = buf[i].b;
      cw[used + i] = (int32_t)buf[i].w;
    }
    used += j;
    cx[a + 1] = used;
  }
done:
  free(buf);
  free(id);
  free(mstart);
  free(members);
  if (status == ORC_ENOMEM) { free(cx); free(ca); free(cw); free(vw); return status; }
  *n_out = nc;
  *cxadj = cx;
  *cadjncy = ca;
  *cadjwgt = cw;
  *cvwgt = vw;
  return status;
}

void orc_free(void *p) { free(p); }

/* Edge cut (Section I): total weight of edges whose endpoints lie in
 * different clusters. Each undirected edge appears twice in the CSR, hence
 * the halving. */
int64_t orc_edge_cut(int32_t n, const uint64_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                     const int32_t *labels) {
  int64_t s = 0;
  for (int32_t u = 0; u < n; ++u)
    for (uint64_t e = xadj[u]; e < xadj[u + 1]; ++e)
      if (labels[u] != labels[adjncy[e]]) s += adjwgt ? adjwgt[e] : 1;
  return s / 2;
}
