/*
 * lp.h — C ABI of the MI355X label-propagation coarsening library.
 *
 * The library implements the coarsening hot path of the multilevel graph
 * partitioner in "Tera-Scale Multilevel Graph Partitioning" (arxiv 2410.19119):
 * size-constrained label-propagation (LP) clustering run directly on a
 * gap + VarInt compressed adjacency (Section III-A), with the two-phase split
 * of low- and high-degree vertices (Section IV-A2), followed by cluster
 * contraction (Section IV-B); on top of the coarsening hierarchy, the
 * uncoarsening steps of a k-way partition (initial partition, projection,
 * size-constrained LP refinement; Section II) and the sparse gain table of
 * Section V. Every step runs in hand-written HIP kernels for gfx950.
 *
 * Conventions shared by every entry point:
 *  - Pointers named *_dev are device pointers on the current HIP device; all
 *    other pointers are host pointers. No pointer is retained after a call
 *    returns, except inside the lp_graph handles the library creates.
 *  - `stream` is a hipStream_t (NULL = the default stream). Calls enqueue
 *    their work on it; results written to device buffers are valid once the
 *    stream has reached that point. Calls that return host values
 *    (lp_graph_info, lp_edge_cut, lp_cluster_ex with stats, lp_compress,
 *    lp_contract) synchronise the stream before returning; so do the calls
 *    that check their arguments on the device (lp_refine, lp_gain_table_create,
 *    lp_gain_table_move).
 *  - Scratch memory comes from the caller's allocator when one is set
 *    (lp_set_allocator), else from the library's per-device memory cache,
 *    in the order of `stream`, and goes back to it before the call returns.
 *    The cache hands memory released by one call to the next (at once on
 *    the same stream, on another stream once the release has completed)
 *    instead of returning it to HIP, keeping up to half of the device's
 *    memory (lp_trim_memory returns it; lp_memory_info reports it).
 *  - Errors are returned as lp_status codes; no exception crosses the ABI.
 *    Argument errors are detected before any work is enqueued. A device
 *    fault surfaces as LP_EDEVICE from the next synchronising call.
 *  - Handles are immutable after creation; one handle may be used from
 *    several streams at once. Each handle must be freed with lp_graph_free.
 *    Handles made by lp_compress and lp_graph_from_csr use plain device
 *    allocations. Handles made inside a call on a stream (lp_contract's
 *    coarse graph, lp_batch_create's batch) take their buffers from the
 *    memory cache on that stream ("its stream") and are released in that
 *    stream's order: work on any other stream that uses such a handle must
 *    be ordered before its stream (an event, or a synchronisation) by the
 *    caller before lp_graph_free.
 *  - Integer widths: vertex IDs and labels int32 (n < 2^31), edge counts
 *    and offsets uint64, input edge / vertex weights int32 >= 1, ratings,
 *    gains, cluster weights and caps int64.
 */
#ifndef LP_H_
#define LP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_graph lp_graph;
typedef int32_t lp_status;

#define LP_OK 0
#define LP_EINVAL (-1)       /* bad argument or malformed input graph */
#define LP_ENOMEM (-2)       /* device allocation failed */
#define LP_EOVERFLOW (-3)    /* a coarse weight would exceed INT32_MAX */
#define LP_EDEVICE (-4)      /* a HIP call or kernel failed */
#define LP_EUNSUPPORTED (-5) /* input outside the supported range (see the call) */

/* Neighbourhoods longer than this are split into independently decodable
 * chunks of LP_CHUNK_LEN neighbours (Section III-A). Fixed by the format. */
#define LP_CHUNK_THRESHOLD 10000
#define LP_CHUNK_LEN 1000
/* Interval-coded graphs (lp_compress_ex with LP_COMPRESS_INTERVALS) split
 * neighbourhoods longer than this instead: the most neighbours the GPU's
 * hub path rates in one piece, so that a piece always starts at a chunk. */
#define LP_ITV_CHUNK_THRESHOLD 4000

/* Human-readable name of a status code (static string). */
const char *lp_strerror(lp_status s);

/* Library version string. */
const char *lp_version(void);

/*
 * lp_compress — build a compressed graph handle from a CSR (Section III-A).
 *
 * Input (device pointers, read only, owned by the caller):
 *   n            number of vertices, 0 <= n < 2^31
 *   xadj_dev     uint64[n+1], xadj[0] = 0, non-decreasing; neighbours of u
 *                are adjncy[xadj[u] .. xadj[u+1])
 *   adjncy_dev   int32[2m] neighbour IDs
 *   adjwgt_dev   int32[2m] edge weights >= 1, or NULL for unit weights
 *   vwgt_dev     int32[n] vertex weights >= 1, or NULL for unit weights
 * The graph must be symmetric (u in N(v) iff v in N(u), with equal weights;
 * this is not checked), without self-loops, with every neighbourhood sorted
 * by (neighbour ID, weight); duplicate neighbours are allowed.
 *
 * Encoding of vertex u's record (byte offset offs[u], offs uint64[n+1]):
 *   VarInt(first edge ID of u)   (degrees come from consecutive headers)
 *   if deg(u) > LP_CHUNK_THRESHOLD: ceil(deg/LP_CHUNK_LEN) - 1 little-endian
 *     uint32 byte offsets, relative to offs[u], of chunks 2, 3, ...
 *   per chunk (the whole neighbourhood if not split): VarInt(zigzag(v0 - u)),
 *     then VarInt(v_i - v_{i-1}) per further neighbour (gap encoding); if
 *     adjwgt is given, every neighbour code is followed by
 *     VarInt(zigzag(w_i - w_{i-1})), w_{-1} = 0 at each chunk start.
 * VarInt = LEB128: 7 data bits per byte, low group first, bit 7 set when
 * another byte follows (Section III-A). Interval encoding: lp_compress_ex.
 *
 * Output: *out receives a new handle owning device copies of the compressed
 * bytes, offsets and vertex weights. Synchronises `stream`.
 * Errors: LP_EINVAL for a neighbour ID out of range, a self-loop, a weight
 * < 1, or an unsorted neighbourhood; LP_ENOMEM; LP_EDEVICE.
 */
lp_status lp_compress(int32_t n, const uint64_t *xadj_dev, const int32_t *adjncy_dev,
                      const int32_t *adjwgt_dev, const int32_t *vwgt_dev, void *stream,
                      lp_graph **out);

/*
 * lp_compress_ex — lp_compress with format flags. LP_COMPRESS_INTERVALS adds
 * the interval encoding of Section III-A: a run x, x+1, ..., x+l-1 of l >= 3
 * consecutive neighbour IDs is stored as the pair (x, l). Per chunk (records
 * of more than LP_ITV_CHUNK_THRESHOLD neighbours are split into chunks of
 * LP_CHUNK_LEN, each coded on its own) the chunk's sorted neighbours are cut,
 * left to right, into maximal runs of IDs each one above the previous
 * neighbour's; runs of at least three are intervals, every other neighbour a
 * residual. Chunk layout:
 *   VarInt(k), the number of intervals;
 *   per interval: VarInt(zigzag(x - u)), VarInt(l - 3);
 *   if adjwgt is given: the weights of the interval neighbours, interval by
 *     interval, each VarInt(zigzag(w - w_prev)), w_prev = 0 at the chunk start;
 *   the residuals r_0 < r_1 < ...: VarInt(zigzag(r_0 - u)), then
 *     VarInt(r_i - r_{i-1}); with weights, each followed by
 *     VarInt(zigzag(w - w_prev)), the chain continuing from the interval
 *     weights.
 * Decoding yields a chunk's interval neighbours first, then its residuals;
 * lp_decompress merges them back into sorted order. Other flags: LP_EINVAL.
 * Everything else as lp_compress; every entry point accepts both formats.
 */
#define LP_COMPRESS_INTERVALS 1
lp_status lp_compress_ex(int32_t n, const uint64_t *xadj_dev, const int32_t *adjncy_dev,
                         const int32_t *adjwgt_dev, const int32_t *vwgt_dev, int32_t flags, void *stream,
                         lp_graph **out);

/*
 * lp_graph_from_csr — plain (uncompressed) CSR handle, same input contract
 * as lp_compress. The library copies the arrays. Coarse graphs produced by
 * lp_contract are handles of this kind (the paper compresses only the input
 * graph, Section II-C).
 */
lp_status lp_graph_from_csr(int32_t n, const uint64_t *xadj_dev, const int32_t *adjncy_dev,
                            const int32_t *adjwgt_dev, const int32_t *vwgt_dev, void *stream,
                            lp_graph **out);

/* Sizes of a handle (host outputs; any may be NULL). nbytes = compressed
 * adjacency bytes (0 for plain handles); is_compressed = 0 (plain CSR),
 * 1 (gap + VarInt) or 2 (gap + VarInt with intervals); total_vwgt = sum of
 * vertex weights. */
lp_status lp_graph_info(const lp_graph *g, int32_t *n, uint64_t *two_m, uint64_t *nbytes,
                        int32_t *is_compressed, int32_t *has_edge_weights, int64_t *total_vwgt);

/* Copies the compressed representation of a compressed handle into caller
 * buffers: offs_dev uint64[n+1], bytes_dev uint8[nbytes]. LP_EINVAL for a
 * plain handle. */
lp_status lp_graph_export(const lp_graph *g, uint64_t *offs_dev, uint8_t *bytes_dev, void *stream);

/*
 * lp_decompress — decode a handle back to CSR (the inverse of the gap +
 * VarInt coding, and of the interval coding, of Section III-A; plain handles
 * are copied). Device outputs, caller sized: xadj_dev uint64[n+1],
 * adjncy_dev int32[2m], adjwgt_dev int32[2m] (may be NULL; unit weights are
 * written as 1), vwgt_dev int32[n] (may be NULL). Neighbourhoods come out
 * sorted by (ID, weight). Synchronises `stream`. Errors: LP_EINVAL for a
 * null argument or a malformed compressed stream (the outputs are then
 * unspecified), LP_EUNSUPPORTED for a batch handle, LP_ENOMEM, LP_EDEVICE.
 */
lp_status lp_decompress(const lp_graph *g, uint64_t *xadj_dev, int32_t *adjncy_dev,
                        int32_t *adjwgt_dev, int32_t *vwgt_dev, void *stream);

/*
 * Options of lp_cluster_ex. The first four are result-invariant tuning
 * knobs, the degree-bucket thresholds: vertices of degree 1..t_lane are
 * rated one per lane; up to t_tile in edge-balanced tiles (one workgroup
 * rates up to 2048 neighbours of up to 80 vertices at once); up to t_block in
 * tiles of up to 4096 neighbours of up to 4 vertices (all with LDS rating
 * tables, Section IV-A2 first phase); higher-degree vertices go to the
 * chunk-parallel hub path (second phase). Any valid setting gives identical
 * labels. `subrounds` changes the method: with S > 1 every round is split
 * into S sub-rounds, vertex u (its ID inside its graph) acting in sub-round
 * sub(u) = SplitMix64 output of (0x6A09E667F3BCC909 xor u), the mix of the
 * tie-break keys, modulo S; each sub-round is one synchronous step (rating
 * with the round's tie-break keys, acceptance, moves) over its vertices
 * against the labels and weights the earlier sub-rounds left, so that
 * neighbours in different sub-rounds no longer move at once (a pair of
 * vertices then merges instead of swapping every round). A round without a
 * proposal in any sub-round ends the call; statistics sum over the
 * sub-rounds of a round. Zero fields mean "default".
 */
typedef struct {
  int32_t t_lane;    /* 0..16, default 16 */
  int32_t t_tile;    /* t_lane..2048, default 2048 */
  int32_t t_block;   /* t_tile..4096, default 4096 */
  int32_t hub_part;  /* target edges per hub partition, 256..8192, default 2048 */
  int32_t timing;    /* nonzero: time each phase with HIP events (stats must be given) */
  int32_t subrounds; /* sub-rounds per round, 1..64, default 1 (plain synchronous rounds) */
  int32_t gain_table; /* lp_refine only: nonzero rates from a sparse gain table (see lp_gain_table);
                         result-invariant; lp_cluster rejects it (LP_EINVAL) */
  int32_t overlap;   /* nonzero: the four rating paths of a round run on concurrent side streams
                        instead of one after another on `stream` (result-invariant) */
  int32_t reorder;   /* result-invariant: rate on a degree-ordered copy of the graph, built on the
                        first call and kept with the handle until lp_graph_free (about the size of
                        the graph again; the build synchronises the stream and takes one-time
                        scratch of about 28 bytes per directed edge). Random label gathers then
                        find the labels of the vertices most edges point to in fewer cache lines.
                        0: automatic: from the second lp_cluster(_ex) call on a handle made by
                        lp_compress(_ex) or lp_graph_from_csr (not on coarse graphs) with at least
                        2^20 vertices and a largest degree of at least 32 times the average, for
                        calls that start from singletons with one sub-round (a graph clustered
                        once would not repay the build); 1: always where it applies, from the
                        first call; 2: never.
                        lp_refine(_ex), sub-rounds, batches and the gain table always rate on the
                        graph as given. */
} lp_config;

/* Phases timed when lp_config.timing is set (milliseconds summed over rounds). */
#define LP_PHASE_SETUP 0  /* degrees, buckets, tiles, hub metadata, initial labels */
#define LP_PHASE_LANE 1   /* rating, lane-per-vertex bucket */
#define LP_PHASE_TILE 2   /* rating, edge-balanced tile bucket */
#define LP_PHASE_BLOCK 3  /* rating, workgroup-per-vertex bucket */
#define LP_PHASE_HUB 4    /* rating, hub path (whole hubs, pieces, reduction, combine) */
#define LP_PHASE_ACCEPT 5 /* proposal compaction, sort, admission, apply */
#define LP_PHASE_ROUND 6  /* whole rounds (rating, acceptance, apply) */
/* the kernels of the hub path, each timed alone (within LP_PHASE_HUB) */
#define LP_PHASE_HUB_WHOLE 7   /* hubs rated whole, one workgroup each */
#define LP_PHASE_HUB_PIECES 8  /* pieces of the larger hubs */
#define LP_PHASE_HUB_REDUCE 9  /* reduction of the pieces' partial ratings, and combine */
#define LP_NUM_PHASES 10

/* Per-call statistics (host struct, filled when requested). */
typedef struct {
  int32_t rounds_run;         /* rounds that had at least one proposal */
  int32_t n_lane, n_tile, n_block, n_hub; /* bucket sizes (vertices) */
  int64_t proposals[64];      /* per round */
  int64_t moves[64];          /* per round */
  uint64_t bucket_edges[4];   /* adjacency entries per bucket (lane, tile, block, hub) */
  uint64_t bucket_bytes[4];   /* compressed record bytes per bucket (0 for plain graphs) */
  float phase_ms[LP_NUM_PHASES]; /* filled when lp_config.timing is set */
  int32_t phase_launches[LP_NUM_PHASES]; /* rounds in which the phase ran */
  float round_ms[64];         /* per round (first 64), filled when lp_config.timing is set */
} lp_cluster_stats;

/*
 * lp_cluster — size-constrained label-propagation clustering.
 *
 * Semantics (Section IV-A, Algorithm 1 for what a vertex computes; rounds
 * are synchronous as in the batch-synchronous distributed LP of Section II-B):
 *   Start: C[u] = u, W[c] = weight of vertex c.
 *   Each round r = 0..rounds-1 reads the snapshot (C0, W0) of the previous
 *   round. For every u with neighbours: rating R(c) = sum of weights of the
 *   edges from u to vertices v with C0[v] = c (Section IV-A1); own =
 *   R(C0[u]). The best c != C0[u] with W0[c] + w(u) <= max_cluster_weight
 *   maximises R(c), ties broken by the smaller SplitMix64 key of
 *   (seed ^ (r << 32) ^ c). u proposes it iff R(c) > own, with gain
 *   R(c) - own. Proposals to each target are ordered by (gain desc, u asc)
 *   and admitted while W0[c] + the running sum of their weights stays
 *   <= max_cluster_weight; admitted vertices move. A round without any
 *   proposal ends the call early (the state is a fixed point).
 * Arguments: g (compressed or plain handle), max_cluster_weight >= 1,
 * rounds >= 0, seed, labels_dev int32[n] (output; labels are vertex IDs in
 * [0, n), not renumbered).
 * Errors: LP_EINVAL (cap < 1, rounds < 0, NULL labels); LP_ENOMEM;
 * LP_EUNSUPPORTED if a vertex's weighted degree needs more than 64 - log2(n)
 * bits.
 */
lp_status lp_cluster(const lp_graph *g, int64_t max_cluster_weight, int32_t rounds, uint64_t seed,
                     int32_t *labels_dev, void *stream);

/* lp_cluster with knobs (cfg may be NULL) and optional statistics (stats may
 * be NULL; when given the call synchronises `stream`). */
lp_status lp_cluster_ex(const lp_graph *g, int64_t max_cluster_weight, int32_t rounds, uint64_t seed,
                        int32_t *labels_dev, const lp_config *cfg, lp_cluster_stats *stats,
                        void *stream);

/*
 * Batches of graphs (many uneven graphs in one launch sequence).
 *
 * lp_batch_create — the disjoint union of G >= 1 graph handles as one batch
 * handle (all plain or all compressed in one format, all with or all without edge
 * weights, else LP_EUNSUPPORTED; total vertices < 2^31). Graph i's vertices
 * occupy [vbase[i], vbase[i+1]) of the union. The inputs are copied (they
 * stay owned by the caller and may be freed afterwards); the batch handle is
 * freed with lp_graph_free. The call synchronises `stream`.
 * A batch handle is accepted by lp_batch_cluster_ex, lp_contract and
 * lp_edge_cut (which see the union as one graph); lp_cluster(_ex),
 * lp_decompress and lp_graph_export reject it (LP_EINVAL / LP_EUNSUPPORTED).
 */
lp_status lp_batch_create(int32_t G, const lp_graph *const *graphs, void *stream, lp_graph **batch_out);

/* Number of graphs of a batch handle (0 for a single graph) and, if vbase is
 * not NULL, their first vertices (host int32[G + 1]). */
lp_status lp_batch_info(const lp_graph *batch, int32_t *G, int32_t *vbase);

/*
 * lp_batch_cluster_ex — lp_cluster on every graph of a batch at once.
 * caps, seeds: host arrays of G values (cap of graph i >= 1). Each graph
 * follows the rules of lp_cluster with its own cap and seed, and its
 * tie-break keys use labels local to the graph, so the labels of graph i are
 * exactly those lp_cluster gives for it alone. labels_dev: int32[n of the
 * union]; graph i's labels are written at [vbase[i], vbase[i+1]) as IDs
 * local to graph i. A round without proposals in any graph ends the call
 * (graphs without proposals are at a fixed point and stay there). Knobs and
 * statistics as in lp_cluster_ex (statistics sum over the graphs).
 */
lp_status lp_batch_cluster_ex(const lp_graph *batch, const int64_t *caps, int32_t rounds,
                              const uint64_t *seeds, int32_t *labels_dev, const lp_config *cfg,
                              lp_cluster_stats *stats, void *stream);

/*
 * lp_batch_cluster — G separate handles in, G label arrays out: builds the
 * batch, clusters it and writes graph i's labels to labels_dev[i] (host
 * array of G device pointers, int32[n_i] each). Synchronises `stream`.
 */
lp_status lp_batch_cluster(int32_t G, const lp_graph *const *graphs, const int64_t *caps, int32_t rounds,
                           const uint64_t *seeds, int32_t *const *labels_dev, void *stream);

/*
 * lp_contract — quotient graph of a clustering (Section IV-B).
 * Coarse vertex IDs are the ranks of the nonempty labels in increasing order;
 * the weight of a coarse vertex is the sum of its members' weights; the
 * coarse edge (a, b), a != b, carries the summed weight of all fine edges
 * between members of a and members of b; edges inside a cluster vanish.
 * Neighbourhoods are sorted by coarse ID.
 * Arguments: g, labels_dev int32[n] with values in [0, n), map_dev int32[n]
 * (output, fine vertex -> coarse vertex; may be NULL), *coarse_out receives a
 * new plain handle. Synchronises `stream`.
 * Errors: LP_EINVAL (label out of range), LP_EOVERFLOW (a coarse edge or
 * vertex weight exceeds INT32_MAX), LP_ENOMEM.
 */
lp_status lp_contract(const lp_graph *g, const int32_t *labels_dev, int32_t *map_dev, void *stream,
                      lp_graph **coarse_out);

/*
 * lp_edge_cut — total weight of the edges whose endpoints carry different
 * labels (the cut of Section I, each undirected edge counted once).
 * *cut_out is a host int64. Synchronises `stream`.
 */
lp_status lp_edge_cut(const lp_graph *g, const int32_t *labels_dev, int64_t *cut_out, void *stream);

/*
 * lp_edge_cut_noalloc — lp_edge_cut for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the same edge
 * visit, but no allocation of any kind and no synchronisation.
 * Arguments: g, labels_dev int32[n] as for lp_edge_cut; cut_dev receives the
 * cut as a device int64 once `stream` reaches the end of the call.
 * Scratch: a fixed 256-byte array of device memory per device, kept by the
 * library until the process ends (the cut accumulator and the edge visit's
 * counters); there is no size limit, since its size does not depend on the
 * graph. Every call on one device shares that array and the last call's
 * contents stay in it (each call clears it first): calls that overlap on one
 * device (on different streams, or from different threads) race and must be
 * ordered by the caller.
 * The handle's degree-bucket plan (memory of the handle, built once on the
 * first lp_cluster with default thresholds, lp_edge_cut or lp_contract on it)
 * must exist, since building it allocates.
 * Errors: LP_EINVAL (null arguments, or a handle without its plan),
 * LP_EUNSUPPORTED (device index above 63), LP_EDEVICE.
 */
lp_status lp_edge_cut_noalloc(const lp_graph *g, const int32_t *labels_dev, int64_t *cut_dev, void *stream);

/*
 * Uncoarsening slice of the multilevel scheme (Section II-A): an initial
 * partition of the coarsest graph, projected to each finer level and refined
 * there by size-constrained label propagation (Section II-B). Blocks are
 * labels in [0, k); a partition is balanced when every block weighs at most
 * the bound of Section I, passed in as max_block_weight.
 */

/*
 * lp_initial_partition — contiguous-weight k-way partition: the vertices, in
 * ID order, fill blocks 0..k-1; vertex u goes to block floor(k * P_u / c(V)),
 * where P_u is the total weight of the vertices before u and c(V) the total
 * weight. Every block weighs less than c(V)/k plus one vertex weight.
 * Arguments: g (single graph), k >= 1, labels_dev int32[n] (output).
 * Errors: LP_EINVAL (k < 1, NULL labels, batch handle); LP_EUNSUPPORTED if
 * k * c(V) >= 2^63.
 */
lp_status lp_initial_partition(const lp_graph *g, int32_t k, int32_t *labels_dev, void *stream);

/*
 * lp_project — blocks of a finer graph from those of its quotient graph
 * (Section II-A, uncoarsening): labels_dev[u] = coarse_labels_dev[map_dev[u]]
 * for u < n, with map_dev the fine-to-coarse map lp_contract writes. A map
 * entry outside [0, coarse_n) gives -1, which lp_refine rejects.
 * Errors: LP_EINVAL (n < 0, coarse_n < 0, NULL pointer with n > 0).
 */
lp_status lp_project(int32_t n, const int32_t *map_dev, int32_t coarse_n, const int32_t *coarse_labels_dev,
                     int32_t *labels_dev, void *stream);

/*
 * lp_refine — size-constrained label-propagation refinement of a k-way
 * partition (Section II-B): the rounds of lp_cluster (rating, tie-break keys
 * of (seed, round, block), gain, admission in (gain desc, u asc) order and the
 * early exit) started from the blocks in labels_dev instead of singletons,
 * with max_block_weight as the cap and W starting as the block weights. A
 * block that starts within max_block_weight stays within it (moves into a
 * block are admitted against its weight at the start of the round;
 * departures are not credited).
 * Arguments: g (single graph), 1 <= k <= n, max_block_weight >= 1,
 * rounds >= 0, seed, labels_dev int32[n] (in: the block of every vertex, in
 * [0, k); out: the refined blocks). The call synchronises `stream` once,
 * after checking the blocks on the device and before the first round.
 * Errors: LP_EINVAL (k out of range, a block outside [0, k), cap < 1,
 * rounds < 0, batch handle); LP_ENOMEM; LP_EUNSUPPORTED as lp_cluster.
 */
lp_status lp_refine(const lp_graph *g, int32_t k, int64_t max_block_weight, int32_t rounds, uint64_t seed,
                    int32_t *labels_dev, void *stream);

/* lp_refine with knobs and optional statistics, as lp_cluster_ex. */
lp_status lp_refine_ex(const lp_graph *g, int32_t k, int64_t max_block_weight, int32_t rounds, uint64_t seed,
                       int32_t *labels_dev, const lp_config *cfg, lp_cluster_stats *stats, void *stream);

/*
 * Sparse gain table (Section V): the affinity omega(u, b) of every vertex u
 * to every block b, i.e. the total weight of u's edges into b, kept in O(m)
 * memory. A vertex whose hash slice (pow2(2 deg(u)) slots of (block,
 * affinity)) would hold at least k slots keeps a dense row of k affinities
 * instead; affinities are int32 unless a weighted degree needs int64. The
 * gain of moving u to b is omega(u, b) - omega(u, block(u)). lp_refine with
 * lp_config.gain_table set builds one per call and rates from it, updating
 * it after every round instead of decoding every neighbourhood again.
 *
 * lp_gain_table_create — builds the table of `g` (single graph) for the
 * partition blocks_dev (int32[n] in [0, k), 1 <= k <= n; copied). The table
 * refers to g, which must outlive it. Synchronises `stream` (block check and
 * sizing). Errors: LP_EINVAL (bad k, a block out of range), LP_ENOMEM.
 */
typedef struct lp_gain_table lp_gain_table;
lp_status lp_gain_table_create(const lp_graph *g, const int32_t *blocks_dev, int32_t k, void *stream,
                               lp_gain_table **out);

/* Affinities of count (vertex, block) pairs (device arrays) into out_dev
 * int64[count]; -1 for a pair out of range. */
lp_status lp_gain_table_affinity(const lp_gain_table *t, int64_t count, const int32_t *vertices_dev,
                                 const int32_t *blocks_dev, int64_t *out_dev, void *stream);

/* Moves count distinct vertices to the given blocks at once (device arrays)
 * and updates the affinities of their neighbours. Synchronises `stream` to
 * check the batch. Errors: LP_EINVAL (a vertex or block out of range, a
 * vertex listed twice, count > n); nothing is changed then. */
lp_status lp_gain_table_move(lp_gain_table *t, int64_t count, const int32_t *vertices_dev, const int32_t *to_dev,
                             void *stream);

/* Slots over all slices, device bytes held, the number of missing entries
 * met by updates (0 unless the table is corrupt), and the number of slices
 * rebuilt so far because stale zero entries had filled them (outputs may
 * be NULL; synchronises when either count is asked for). */
lp_status lp_gain_table_info(const lp_gain_table *t, uint64_t *entries, uint64_t *bytes, int64_t *missing,
                             int64_t *rebuilds);

/* Frees a table (NULL is ignored), in its stream's order. */
void lp_gain_table_free(lp_gain_table *t);

/* Returns every block of the library's memory cache to HIP, on every device
 * (waiting for each device to be idle first). Handles stay valid; later calls
 * fill the cache again. For callers that share the device with other
 * allocators, e.g. between phases of a job. */
void lp_trim_memory(void);

/*
 * The caller's device allocator (the boundary's allocator of scratch memory;
 * e.g. a framework's caching allocator). alloc returns `bytes` of device
 * memory on the current device usable in the order of `stream` (NULL when
 * out of memory: the call then fails with LP_ENOMEM); free releases a block
 * in the order of `stream` (the stream of the library's last use of it).
 * Both are called from the thread of the library call, with no lock of the
 * library held, and must be thread-safe if several threads call the library.
 */
typedef struct {
  void *(*alloc)(size_t bytes, void *stream, void *ctx);
  void (*free)(void *ptr, void *stream, void *ctx);
  void *ctx;
} lp_allocator;

/*
 * lp_set_allocator — every later scratch allocation, and every buffer of a
 * handle made inside a call (lp_contract's coarse graph, batch handles),
 * comes from *a (copied; NULL restores the library's memory cache). Blocks
 * are always released to the allocator that made them. Handles made by
 * lp_compress and lp_graph_from_csr keep plain device allocations. Call it
 * while no other library call is running. LP_EINVAL if a function is NULL.
 */
lp_status lp_set_allocator(const lp_allocator *a);

/*
 * lp_memory_info — device memory the library holds: bytes of the current
 * device's memory cache handed out to calls and handles (*live_bytes) and
 * kept for reuse (*cached_bytes), and bytes obtained from the caller's
 * allocator and not yet released (*external_bytes, all devices). Any output
 * may be NULL.
 */
lp_status lp_memory_info(uint64_t *live_bytes, uint64_t *cached_bytes, uint64_t *external_bytes);

/* Frees a handle (NULL is ignored). A handle with plain allocations waits
 * for the device to be idle first; a handle made on a stream returns its
 * buffers to the library's memory cache in that stream's order, without
 * waiting: work already queued on the stream runs first, and a later call
 * reuses the buffers only after it. */
void lp_graph_free(lp_graph *g);

#ifdef __cplusplus
}
#endif

#endif /* LP_H_ */
