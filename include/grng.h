/*
 * grng.h -- C ABI of the MI355X (gfx950) exact RNG / GRNG library.
 *
 * Method: Foster, Sevilmis & Kimia, "Generalized Relative Neighborhood Graph
 * (GRNG) for Similarity Search" (arXiv 2208.10022).  The library builds
 *   - the GRNG of one or more nested pivot layers (Section 2, Definition 1;
 *     Section 3 for a layer guided by a coarser one, Theorem 2), and
 *   - the exact RNG of the points (Section 1, the RNG definition equation),
 *     guided by the finest pivot layer (Section 2, Theorem 1, Propositions 1-4,
 *     Algorithm 1),
 * and answers the paper's two uses of the index: incremental insertion
 * (Section 2, Stages I-VII) and RNG-neighbour queries (Algorithm 1 output).
 *
 * Exactness contract.  Results are the exact real-number answers for the
 * float32 inputs as given.  This needs every coordinate and radius to lie on a
 * dyadic grid: x = k * 2^-q with integer |k| < 2^24 (q = options.grid_exp),
 * and d * kmax^2 < 2^51 where kmax is the largest |k| over all coordinates and
 * d the dimension.  Under it every squared distance is exact in float64, so
 * the library decides each lune test exactly; tests that involve a distance
 * minus a radius are decided with an exact 128-bit integer predicate.  Inputs
 * that break the contract are rejected with GRNG_ENOTGRID.
 *
 * Conventions.
 *   - Pointers named *_dev are device pointers (HIP device memory of the
 *     current device); other pointers are host pointers.
 *   - The caller owns every buffer it passes.  The library copies what it
 *     keeps into its own device memory, so inputs may be freed after the call
 *     returns.  The library owns all device memory it allocates, released by
 *     grng_destroy.
 *   - All device work is enqueued on the stream given to grng_create.  Calls
 *     that return host-visible counts synchronize that stream before returning.
 *   - Errors: every call returns a grng_status; on failure grng_last_error()
 *     describes it (thread-local) and the index is left as it was before the
 *     call, except after GRNG_EDEVICE, after which only grng_destroy is valid.
 *   - An index is used by one host thread at a time.
 *   - Point ids are 0-based positions in the order points were given:
 *     grng_create's points first, then each insert_batch appended in order.
 *   - Edge output is canonical: pairs (u, v) with u < v, sorted by u then v,
 *     so two edge sets are equal iff their arrays are byte-equal.
 */
#ifndef GRNG_H
#define GRNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRNG_ABI_VERSION 1

typedef struct grng_index grng_index;

typedef enum grng_status {
    GRNG_OK = 0,
    GRNG_EINVAL = -1,    /* invalid argument (null pointer, size out of range, bad id, unsorted...) */
    GRNG_ENOMEM = -2,    /* a device or host allocation failed */
    GRNG_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed */
    GRNG_ENOTGRID = -4,  /* an input is not finite, not on the 2^-q grid, or too large (see above) */
    GRNG_ECAPACITY = -5, /* caller buffer too small; *needed / *num_edges holds the required size */
    GRNG_ESTATE = -6     /* call out of order (e.g. layer 1 before layer 0) */
} grng_status;

/* Arithmetic of the exhaustive witness scan (Section 2, Stage VI), where most
 * witness tests are spent.  Every kept/eliminated decision is exact in all
 * modes; the pivot and in-tile certificates before the scan always compare
 * float32 roundings (or upper bounds) of exact float64 tiles and only
 * eliminate on a proven witness. */
enum {
    GRNG_PREC_FP64 = 0, /* exact float64 squared distance for every witness test */
    GRNG_PREC_FP32 = 1, /* float32 rows with an error-bounded screen; undecided tests are recomputed in float64 */
    GRNG_PREC_BF16 = 2, /* GRNG_PREC_FP32, but the pair kernel's distance tiles come from bf16 MFMA with
                           float32 accumulation on cell-centred coordinates split into two bf16 parts
                           (three products per tile), with a per-tile error bound; a certificate kills a
                           pair only outside the bound, and pairs within it go on to the exhaustive scan,
                           which re-decides them exactly */
    GRNG_PREC_AUTO = 3  /* GRNG_PREC_FP32 or GRNG_PREC_BF16, i.e. the pair kernel's tile shape (float64
                           16x16x4 MFMA tiles or split bf16 16x16x32 tiles), chosen per index: by trial
                           builds of the autotuner when autotune = 1, else bf16 from a padded dimension
                           of 32 (one bf16 MFMA step; below it half of each step is padding).  Both give
                           the same edges; stats.precision_used tells which ran */
};

enum {
    GRNG_ORDER_DISTANCE = 0, /* witnesses visited nearest-first (Section 2, Stages III and V) */
    GRNG_ORDER_LEARNED = 1,  /* witness domains ranked by the learned scorer (grng_set_scorer) */
    GRNG_ORDER_LUNE = 2      /* within each group of 64 domains taken nearest-first, a pair visits them by
                                increasing max(d(x,p), d(y,p)) (pays off in high dimensions, where a
                                witness test reads a long row: 12% less build time on 1M x 96-D
                                points; 16-D builds run faster in distance order) */
};

typedef struct grng_options {
    int32_t grid_exp;      /* q: every coordinate and radius is an integer multiple of 2^-q; 0..60 */
    int32_t precision;     /* GRNG_PREC_* */
    int32_t witness_order; /* GRNG_ORDER_* */
    int32_t use_graph;     /* must be 0: graph capture is not implemented (grng_create returns GRNG_EINVAL
                              for any other value) */
    int32_t autotune;      /* 1: the first grng_build_rng with a pivot layer times complete builds over a
                              small set of choices (with GRNG_PREC_AUTO the pair kernel's tile shape first,
                              then the witness-pivot counts vgrng_pivots and stage4_pivots) and keeps the
                              fastest for later builds, insertions and queries of this index; 0: use the
                              fields below */
    int32_t stage4_pivots; /* pivot witnesses tested per pair before the exhaustive scan: 0 = default (16), 1..16 */
    int32_t vgrng_pivots;  /* Proposition 1 witnesses per 64-point block: the pivots nearest the block's home
                              cell, 0 = default (256), values >= the layer size use every pivot.  Any subset
                              of pivots is a valid witness set (fewer only prunes less), so edges never
                              depend on it. */
    int32_t metric;        /* GRNG_METRIC_*: the distance of the RNG (0 = Euclidean) */
    int32_t graph;         /* GRNG_GRAPH_*: the empty-region graph to build (0 = RNG) */
    int32_t beta_quarters; /* GRNG_GRAPH_BETA: beta = beta_quarters / 4, in [4, 64] (beta 1 to 16); 0 otherwise */
    uint64_t reserved[3];  /* must be 0 */
} grng_options;

/* Other metrics and empty-region graphs (Section 1: a general metric space;
 * the RNG is one of a family of empty-region graphs).  They are built by the
 * exhaustive path only: an index with metric != GRNG_METRIC_L2 or graph !=
 * GRNG_GRAPH_RNG takes no pivot layer (grng_build_grng_layer returns
 * GRNG_EINVAL), and build_rng, insert_batch and query_neighbors test every
 * pair against every point (at most 65,535 points, as for the Euclidean RNG
 * without a layer).  Under the grid contract every L1 and L-infinity
 * distance is exact in float64, so the decisions stay exact. */
enum {
    GRNG_METRIC_L2 = 0,   /* Euclidean */
    GRNG_METRIC_L1 = 1,   /* sum of absolute coordinate differences */
    GRNG_METRIC_LINF = 2  /* largest absolute coordinate difference */
};
enum {
    GRNG_GRAPH_RNG = 0,     /* u, v linked iff no z has max(d(u,z), d(v,z)) < d(u,v) */
    GRNG_GRAPH_GABRIEL = 1, /* Euclidean only: u, v linked iff no z has d(u,z)^2 + d(v,z)^2 < d(u,v)^2 */
    GRNG_GRAPH_BETA = 2     /* Euclidean only, the lune-based beta-skeleton (the beta-skeleton graph Section 1
                               names, in the lune-based form of its cited work), beta = beta_quarters / 4 >= 1:
                               u, v linked iff no z lies in both open balls of radius beta d(u,v) / 2 centred at
                               (1 - beta/2) u + (beta/2) v and (beta/2) u + (1 - beta/2) v.  beta 1 gives the
                               Gabriel graph, 2 the RNG; larger beta, fewer edges.  Exact: integer sums of
                               squares in 128 bits. */
};

typedef struct grng_stats {
    int64_t n_points;             /* points currently indexed */
    int64_t n_edges;              /* exemplar RNG edges (after build_rng / insert_batch) */
    int64_t n_layers;             /* pivot layers built */
    int64_t orphans;              /* points in no pivot domain of the finest layer */
    int64_t tile_pairs;           /* 64-point tile pairs scanned for candidate pairs */
    int64_t vgrng_pivots;         /* Proposition 1 witness pivots per block used by the last build */
    int64_t stage4_pivots;        /* Stage IV pivot witnesses used by the last build */
    int64_t unsorted_cell_rows;   /* rows of the last build whose witness-cell list was longer than the
                                     4,096 entries sorted on chip, and was scanned in pivot order */
    double distance_computations; /* squared distances produced (the paper's cost unit, Section 1): every
                                     point-pivot entry, every entry of the pair kernel's distance tiles
                                     (D(T,U), the pivot blocks, D(T,T), D(U,U) when computed), one per
                                     partner-pass test, and two per witness test of the exhaustive scan
                                     (plus one per witness cell's pivot) */
    double witness_tests;         /* (pair, witness) lune predicates evaluated, pivots included */
    double candidate_pairs;       /* pairs left after Stages I-III (Theorem 1, Propositions 1-2) */
    double stage4_survivors;      /* pairs left after pivot witnesses (Stage IV) */
    double exhaustive_pairs;      /* pairs left after Stage V in the tiles (the partner pass below takes
                                     them first, the exhaustive scan what it leaves) */
    double lune_tests;            /* witness predicates evaluated by the exhaustive scan */
    double rechecks;              /* comparisons re-decided in float64 / exact integers */
    double ms_layers;             /* device time of the last layer build */
    double ms_rng;                /* device time of the last build_rng */
    double ms_insert;             /* device time of the last insert_batch */
    double ms_query;              /* device time of the last query_neighbors */
    double ms_vgrng;              /* device time of the virtual-pivot (min,max) kernel in the last build */
    double ms_pairs;              /* device time of the tiled candidate-pair kernel in the last build */
    double ms_lune;               /* device time of the exhaustive lune kernel in the last build */
    double vgrng_ops;             /* (min,max) pairs evaluated by the virtual-pivot kernel: 2 n m kw, kw the
                                     Proposition 1 witness pivots per block (vgrng_pivots) */
    double pairs_flops;           /* MFMA flops of the pair kernel: 2 dp (64*64 + 2*64*16) per tile pair,
                                     plus 2 dp * 64*64 per tile pair that reaches Stage V (D(U,U)) and per
                                     D(T,T) computed (kept while consecutive tile pairs share T) */
    double lune_bytes;            /* algorithmic bytes read by the lune kernel: per witness test the
                                     witness row and its cell bound, 4 dp + 4 with the float32 screen,
                                     8 dp + 8 in float64 (a test ending early on a partial sum reads less) */
    double stage4_ops;            /* (min,max) operations of Stage IV in the pair kernel: 2*64*64*K'
                                     per tile pair, K' = pivot witnesses rounded up to a multiple of 4 */
    double ms_autotune;           /* device time of the autotuner's trial builds (0 when it has not run) */
    double ms_pair_masks;         /* device time of the candidate-mask pass before the pair kernel (last build);
                                     ms_pairs is the pair kernel alone */
    double screen_uncertain;      /* GRNG_PREC_BF16: pairs the pair kernel passed on to the exhaustive scan
                                     although an in-tile witness lay within the bf16 tiles' error bound (the scan
                                     re-decides them exactly); 0 in the other modes */
    double pair_tile_entries;     /* entries of the pair kernel's distance tiles computed in the last build:
                                     D(T,U), the pivot blocks, and D(U,U), D(T,T) where Stage V ran */
    double pair_method_distances; /* of those, the ones the method uses: candidate pairs' d(x,y), the pivot
                                     blocks and the Stage V witness matrices */
    double lune_tests_kept;       /* of lune_tests, those spent on pairs that stayed edges (each such pair
                                     tests every witness its cells hold; no visit order saves them) */
    double partner_tests;         /* Stage V with the row's other candidates (Algorithm 1, Stage 5): witness
                                     predicates evaluated, each pair of exhaustive_pairs against the 64
                                     partners nearest to each of its ends in that list (and the pairs left
                                     against the next 64 when at least 1% of the kills needed the last
                                     quarter of the lists) */
    double partner_kills;         /* of exhaustive_pairs, those this pass proved non-edges (the exhaustive
                                     scan skips them) */
    double ms_partner;            /* device time of that pass in the last build */
    int64_t precision_used;       /* GRNG_PREC_* form in effect (the autotuner's choice under GRNG_PREC_AUTO) */
} grng_stats;

/* ABI version the library was built with (GRNG_ABI_VERSION). */
int32_t grng_abi_version(void);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *grng_last_error(void);

/* Create an index over n points of dimension d (row-major float32 [n][d],
 * device memory).  Copies the points.  stream: a hipStream_t (NULL = null
 * stream).  opt: host pointer, required.  Validates the grid contract on the
 * device.  Errors: EINVAL (n < 1, d < 1 or d > 1024, null pointers, reserved
 * fields non-zero, grid_exp out of range), ENOTGRID, ENOMEM, EDEVICE. */
grng_status grng_create(grng_index **out, const float *points_dev, int64_t n, int32_t d,
                        void *stream, const grng_options *opt);

/* Build the GRNG of pivot layer `layer` (Section 2, Definition 1): pivots i, j
 * are linked iff no pivot k has d(k,i) < d(i,j) - (2 r_i + r_j) and
 * d(k,j) < d(i,j) - (r_i + 2 r_j).  Layer 0 is the coarsest and is built by
 * brute force over all pivot triples; layer l > 0 is guided by layer l-1:
 * fine pivots whose coarse relative-domain parents are unlinked are never
 * linked (Section 3, Theorem 2), and coarse pivots are tried first as
 * witnesses (Section 3, Stage IV).
 * pivot_ids_dev: int32 [m] point ids, distinct, ascending.  radii_dev: float32
 * [m] ball radii r_i >= 0 on the grid (a point x is in the domain of pivot p
 * iff d(x,p) <= r_p; Section 1, pivot domain equation).  Layers must be built
 * in order 0, 1, ...; building layer l again discards layers > l and the RNG.
 * The pivots of layer l-1 must be a subset of those of layer l (Section 3,
 * Theorem 2 needs nested layers).  Errors: EINVAL, ENOTGRID, ESTATE, ENOMEM,
 * EDEVICE. */
grng_status grng_build_grng_layer(grng_index *idx, int32_t layer, const int32_t *pivot_ids_dev,
                                  const float *radii_dev, int64_t m);

/* Add nb pivots to the built layer `layer` (Section 2, Stage I promotes a
 * point without parents to a pivot; Section 3 inserts pivots into a GRNG
 * layer with Stages I-VI and unlinks old pivots with Stage VII): the layer's
 * GRNG becomes GRNG(P u B) under Definition 1.  Old links are re-tested
 * against the new pivots only (adding pivots can only unlink a pair), pairs
 * with a new pivot against every pivot.  pivot_ids_dev: int32 [nb] point ids,
 * strictly ascending, none a pivot of this layer yet; each must already be a
 * pivot of every finer layer (layers stay nested).  radii_dev: float32 [nb]
 * radii >= 0 on the grid; old pivots keep theirs.  The exemplar RNG does not
 * change; when the finest layer changes after grng_build_rng, the index
 * recomputes its per-point tables against it, so later insertions and
 * queries use the new pivots.  On error the index is unchanged.  Errors:
 * EINVAL, ENOTGRID, ESTATE, ENOMEM, EDEVICE. */
grng_status grng_insert_pivots(grng_index *idx, int32_t layer, const int32_t *pivot_ids_dev, const float *radii_dev,
                               int64_t nb);

/* Ids (int32, ascending, device) of the points without a parent in the
 * finest layer (no pivot domain holds them: the candidates for promotion
 * with grng_insert_pivots).  *count = their number; if it exceeds capacity,
 * returns ECAPACITY and copies nothing (ids_dev may be NULL with capacity 0).
 * Requires a pivot layer and a prior grng_build_rng.  Errors: EINVAL,
 * ESTATE, ECAPACITY, EDEVICE. */
grng_status grng_get_orphans(grng_index *idx, int32_t *ids_dev, int64_t capacity, int64_t *count);

/* Build the exact RNG of all indexed points (Section 1, RNG definition:
 * u, v linked iff no z has max(d(u,z), d(v,z)) < d(u,v); ties keep the edge).
 * With at least one layer built, candidate pairs and witnesses are pruned by
 * the finest layer (Section 2: Theorem 1, Propositions 1-2 for candidates,
 * Stage IV pivot witnesses, Propositions 3-4 for witness domains); without a
 * layer, every pair is tested against every point.  The kernels keep rows in
 * LDS: guided builds, insertions and queries need d <= 104, the brute-force
 * build d <= 128 (EINVAL above that).  Errors: EINVAL, ESTATE, ENOMEM,
 * EDEVICE. */
grng_status grng_build_rng(grng_index *idx);

/* Insert nb points (float32 [nb][d], device) with ids n..n+nb-1 and update
 * the RNG to RNG(S u B) (Section 2: localization Stages I-VI for each new
 * point against S u B, then Stage VII invalidation of existing edges by the
 * new points, Proposition 5).  Pivot layers stay as built.  Requires a prior
 * grng_build_rng.  The index keeps its per-point tables between calls (the
 * point-pivot squared distances, float64 [n][m] with room for growth, home
 * cells, parents, virtual-pivot bits): an insertion computes them for the
 * batch only and merges them in, redoing only the cell bits of home cells
 * whose radius grew.  The result equals a rebuild over S u B.  On error the
 * index is unchanged.  Errors: EINVAL, ENOTGRID, ESTATE, ENOMEM, EDEVICE. */
grng_status grng_insert_batch(grng_index *idx, const float *points_dev, int64_t nb);

/* RNG neighbours of nq query points (float32 [nq][d], device) within S u {Q}
 * for each query separately, without inserting them (Algorithm 1 output):
 * x in S is a neighbour of Q iff no z in S \ {x} has
 * max(d(Q,z), d(x,z)) < d(Q,x).  Output in CSR form: offsets_dev int64
 * [nq+1] and nbrs_dev int32 [capacity], neighbours of each query ascending.
 * If the total exceeds capacity, returns ECAPACITY with *needed set and
 * offsets_dev filled; call again with a larger nbrs_dev.  Requires a prior
 * grng_build_rng.  Errors: EINVAL, ENOTGRID, ESTATE, ECAPACITY, ENOMEM,
 * EDEVICE. */
grng_status grng_query_neighbors(grng_index *idx, const float *q_dev, int64_t nq, int64_t *offsets_dev,
                                 int32_t *nbrs_dev, int64_t capacity, int64_t *needed);

/* Copy an edge set into uv_dev (int32 [2*E], device): layer >= 0 gives the
 * GRNG of that pivot layer, layer = -1 the exemplar RNG, both as point ids
 * (pivots are points, Section 1).  Canonical order (u < v, sorted).
 * If E > capacity (in pairs), returns ECAPACITY with *num_edges = E and
 * copies nothing.  uv_dev may be NULL with capacity 0 to query E.
 * Errors: EINVAL, ESTATE, ECAPACITY, EDEVICE. */
grng_status grng_get_edges(const grng_index *idx, int32_t layer, int32_t *uv_dev, int64_t capacity,
                           int64_t *num_edges);

/* Counters and device timings of the last calls (host struct). */
grng_status grng_get_stats(const grng_index *idx, grng_stats *out);

/* Release everything the index owns.  NULL is a no-op. */
void grng_destroy(grng_index *idx);

/* ---- Learned witness-domain ranking ---------------------------------------
 * The exhaustive scan (Section 2, Stages V-VI) visits the candidate witness
 * domains of a pair until one holds a witness.  The order never changes an
 * edge (every domain that can hold a witness is still visited until one is
 * found); it changes only how many witness tests are spent.  A small MLP,
 *     h = relu(f W1 + b1),  s = h . w2 + b2,
 * scores each candidate domain from GRNG_MLP_FEATURES scale-free features
 * (distances of x and y to the domain's pivot, their smaller and larger
 * value (the larger is the lune-order key), the domain's covering radius and
 * pivot radius, its Proposition 3 margin and size, all relative to d(x,y)).  Parameters are one float32 device vector of grng_mlp_params()
 * values laid out [W1 (features x hidden, row-major), b1, w2, b2].  The loss
 * is the mean binary cross-entropy with logits against "the domain holds a
 * witness".  Training samples come from the last grng_build_rng. */
#define GRNG_MLP_FEATURES 9
#define GRNG_MLP_HIDDEN 64

/* Number of parameters: F*H + 2H + 1 = 705. */
int32_t grng_mlp_params(void);

/* Loss and its gradient on n samples.  feats_dev: float32 [n][9] (device),
 * labels_dev: uint8 [n] in {0,1} (device), grad_dev: float32 [params]
 * (device, written), *loss: host float.  Blocks of samples are reduced in a
 * fixed order, so the result is deterministic.  stream: hipStream_t or NULL. */
grng_status grng_mlp_grad(const float *theta_dev, const float *feats_dev, const uint8_t *labels_dev, int64_t n,
                          float *grad_dev, float *loss, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same loss and gradient as grng_mlp_grad, bit for bit, but
 * with no allocation.  The per-block partial gradients go to a fixed scratch
 * array in the library's device memory (11.6 MB on each device the library
 * runs on, held until the process ends), so n is limited to
 * GRNG_MLP_NOALLOC_MAX_SAMPLES; larger n returns GRNG_EINVAL.  The loss is
 * written to loss_dev (float32, device) instead of a host float, and the call
 * returns without synchronizing `stream`.  The stream must belong to the
 * current device.  Every call on a device shares that device's scratch:
 * calls whose work overlaps on one device (other host threads, other
 * streams) race and give undefined results; calls queued on one stream are
 * safe.  Nothing in the scratch needs clearing between calls (each call
 * writes every entry it reads).  Errors: EINVAL, EDEVICE. */
#define GRNG_MLP_NOALLOC_MAX_SAMPLES (1 << 24)
grng_status grng_mlp_grad_noalloc(const float *theta_dev, const float *feats_dev, const uint8_t *labels_dev,
                                  int64_t n, float *grad_dev, float *loss_dev, void *stream);

/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, step size
 * lr) on theta_dev in place; *loss = loss after the last step. */
grng_status grng_mlp_train(float *theta_dev, const float *feats_dev, const uint8_t *labels_dev, int64_t n,
                           int32_t steps, float lr, float *loss, void *stream);

/* Scores of n feature rows with the weights rounded to bf16 (nearest-even)
 * and float32 accumulation: the same arithmetic the scan uses. */
grng_status grng_mlp_score(const float *theta_dev, const float *feats_dev, int64_t n, float *scores_dev,
                           void *stream);

/* Training samples from the last grng_build_rng (which needs a pivot layer):
 * for up to max_pairs pairs spread evenly over the pairs the exhaustive scan
 * handled, one sample per candidate domain of the pair's first point that
 * Proposition 3 does not rule out, labelled by an exact scan of the domain's
 * members.  Writes min(count, capacity) rows of feats_dev (float32 [.][8]) and
 * labels_dev (uint8); *count = samples produced.  GRNG_ECAPACITY when count >
 * capacity (call again with capacity >= *count); GRNG_ESTATE when no guided
 * build is current (after grng_insert_batch, until the next build). */
grng_status grng_log_witness_cells(grng_index *idx, int64_t max_pairs, float *feats_dev, uint8_t *labels_dev,
                                   int64_t capacity, int64_t *count);

/* Install scorer weights (copied and rounded to bf16) for indexes created with
 * witness_order = GRNG_ORDER_LEARNED; grng_build_rng on such an index returns
 * GRNG_ESTATE until a scorer is set.  Queries and insertions use it too. */
grng_status grng_set_scorer(grng_index *idx, const float *theta_dev);

#ifdef __cplusplus
}
#endif

#endif /* GRNG_H */
