// Internal declarations of the gfx950 exact RNG / GRNG library.
// Not part of the public ABI (that is include/grng.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <map>
#include <vector>

#include "grng.h"

namespace grng {

// ---------------------------------------------------------------------------
// Errors: internal code throws Error; the ABI layer turns it into a status.
struct Error : std::runtime_error {
    grng_status status;
    Error(grng_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define GRNG_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::grng::Error(GRNG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GRNG_LAUNCHED() GRNG_HIP(hipGetLastError())

inline void require(bool ok, grng_status s, const std::string &msg) {
    if (!ok) throw Error(s, msg);
}

// ---------------------------------------------------------------------------
// Owning device buffer.
// Per-index cache of device blocks.  Every kernel and copy of an index runs
// on the index's one stream, so a block handed back while work that uses it
// is still queued can be handed out again at once: the next user's work is
// queued behind it.  This keeps hipMalloc / hipFree (which waits for the
// device) out of the middle of a build.  Blocks come in size classes (powers
// of two up to 2 MiB, then eighths of a power of two).
class BlockPool {
public:
    BlockPool() = default;
    BlockPool(const BlockPool &) = delete;
    BlockPool &operator=(const BlockPool &) = delete;
    ~BlockPool();
    void *get(size_t bytes, size_t *cls);   // throws ENOMEM
    void put(void *p, size_t cls);
    void trim(size_t keep);                  // free cached blocks, largest first, down to keep bytes
    size_t cached() const { return cached_; }
private:
    std::multimap<size_t, void *> free_;
    size_t cached_ = 0;
};

// Pool of the index the current C-ABI call works on (null: plain hipMalloc).
extern thread_local BlockPool *g_pool;

// Owning device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    BlockPool *pool = nullptr;            // where the block goes back to (null: hipFree)
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), pool(o.pool) {
        o.p = nullptr;
        o.bytes = 0;
        o.pool = nullptr;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            pool = o.pool;
            o.p = nullptr;
            o.bytes = 0;
            o.pool = nullptr;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (pool)
                pool->put(p, bytes);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        pool = nullptr;
    }
    void alloc(size_t nbytes);            // throws ENOMEM; contents undefined; bytes >= nbytes
    void ensure(size_t nbytes);           // grow (discarding contents) if smaller
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// Sizes and constants.
constexpr int kWave = 64;
inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int pad4(int d) { return (d + 3) & ~3; }

// Pivot layer: pivots, radii, their exact distances and the GRNG.
struct Layer {
    int64_t m = 0;
    int32_t words = 0;         // uint64 words per bitset row: ceil(m / 64)
    std::vector<int32_t> pid_host;
    DevBuf pid;                // int32 [m] point ids
    DevBuf rad;                // double [m] radii (exact grid values)
    DevBuf radi;               // int64 [m] radii in grid units
    DevBuf dpp2;               // double [m*m] exact squared distances
    DevBuf dpp;                // double [m*m] distances (sqrt rounded to nearest)
    DevBuf bits;               // uint64 [m*words] GRNG adjacency (no self bits)
    DevBuf edges;              // int32 [2E] canonical pivot-position pairs
    int64_t nedges = 0;
    DevBuf parent_bits;        // uint64 [m*coarse_words]: coarse relative-domain parents (layer > 0)
};

// A point set prepared against the finest pivot layer, in home order (grouped
// by nearest pivot).  For the indexed set the home cells are also the witness
// groups (grp_off, dvor, gcount, dhome); for a query set only the home order,
// parents and virtual-pivot bits are used.
struct PointState {
    int64_t n = 0;
    int64_t ntiles = 0;
    int64_t nw = 0;                // words of a transposed bit row: ceil(n / 64)
    int64_t orphans = 0;
    std::vector<int32_t> h_perm;   // home-order position -> index in the set (empty after an insertion merge)
    std::vector<int32_t> h_off;    // [m+1] home-order start of each home cell
    DevBuf perm;                   // int32 [n]
    DevBuf inv;                    // int32 [n] index -> home-order position
    DevBuf Xh, nrmh;               // double [n][dp], [n]
    DevBuf Xf;                     // float [n][dp]: the same rows (exact, coordinates are float32 values)
    DevBuf home;                   // int32 [n] home cell (pivot position)
    DevBuf dhome;                  // double [n] upper bound of d(x, p_home)
    DevBuf dhomef;                 // float [n] the same bound rounded up
    DevBuf grp_off;                // int32 [m+1]
    DevBuf dvor;                   // double [m] upper bound of the cell radius
    DevBuf gcount;                 // int32 [m] cell sizes
    DevBuf par_off, par_idx;       // parents CSR (int64 [n+1], int32)
    DevBuf g_rows, v_rows;         // uint64 [n][words] virtual-pivot bits (domains / cells)
    DevBuf g_cols;                 // uint64 [m][nw] transposed g_rows
    DevBuf tiles;                  // int32 [ntiles][3]
    DevBuf tv;                     // uint64 [ntiles][words] OR of v_rows over the tile
    DevBuf gid;                    // int32 [n] global point ids (a batch being inserted), else empty
    DevBuf is_new, tnew;           // uint8 [n], [ntiles]: batch points and tiles (dense insertion only)
    DevBuf dxp;                    // double [n][m] exact d^2 to the pivots, input order
};

// Pivot-side tables of the finest layer used by every pass over points.
struct LayerAux {
    DevBuf Xp, nrmp;               // pivot coordinates and norms
    DevBuf Xpf;                    // float [m][dp] the same coordinates (exact: grid values)
    DevBuf pknn;                   // int32 [m][16] nearest pivots of each pivot
    DevBuf wknn;                   // int32 [m][kw] nearest pivots of each pivot (Proposition 1 witnesses)
    int32_t kw = 0;
    DevBuf bd, bv;                 // float [m][m] shifted pivot distances (virtual-pivot test)
};

// Counters written by kernels (device, uint64 each).
enum Counter {
    C_DIST = 0,       // squared distances computed
    C_WTEST,          // witness predicates evaluated
    C_CAND,           // candidate pairs after Stages I-III
    C_S4,             // survivors of Stage IV
    C_RECHECK,        // exact re-decisions
    C_SURV,           // pairs left for the exhaustive scan (after Stage V)
    C_LUNE,           // witness predicates evaluated by the exhaustive scan
    C_TPV,            // tile pairs that reached Stage V (D(U,U) computed)
    C_TTV,            // D(T,T) computations (not repeated while consecutive tile pairs share T)
    C_UNSORTED,       // rows whose witness-cell list exceeded the sort capacity
    C_UNCERTAIN,      // bf16 pair kernel: survivors with an in-tile witness within the error bound
    C_PD_TU,          // pair kernels: entries of D(T,U) computed
    C_PD_PIV,         // pair kernels: entries of the pivot blocks D(T,P), D(U,P) computed
    C_PD_V,           // pair kernels: entries of the Stage V witness matrices D(U,U), D(T,T) computed
    C_LUNE_KEPT,      // exhaustive scan: witness predicates of pairs that stayed edges
    C_PARTNER_TESTS,  // Stage V with the row's other candidates: witness predicates evaluated
    C_PARTNER_KILLS,  // Stage V with the row's other candidates: pairs proven non-edges
    C_PARTNER_DEEP,   // of those, pairs whose nearest killing partner was in the last quarter of its list
    // 8 work counters for dynamic scheduling (one per XCD), each on its own
    // 128-byte line: atomics on one shared line serialize across the chip.
    C_WORK0 = 32,
    C_WORK_END = C_WORK0 + 8 * 16,
    C_NUM = C_WORK_END
};
constexpr int kWorkStride = 16;   // uint64 slots between two XCDs' work counters

// Learned witness-cell ranking (scan order only).
constexpr int kMlpFeatures = 9;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpFeatures * kMlpHidden + 2 * kMlpHidden + 1;

// Scale-free features of candidate cell c for the pair (x, y): distances of
// x and y to the cell's pivot, cell radius, domain radius, the Proposition 3
// lower bound, log cell size, the pivot's position relative to the lune, all
// divided by d(x, y) (or its square).
__device__ inline void mlp_features(double dx, double dy, double dcell, double rdom, int32_t size, double dxy,
                                    float *f) {
    const double inv = 1.0 / dxy;
    const double v[kMlpFeatures] = {dx * inv,
                                    dy * inv,
                                    dcell * inv,
                                    rdom * inv,
                                    (fmax(dx, dy) - dcell) * inv,
                                    log2(1.0 + (double)size) * 0.1,
                                    (dx * dx + dy * dy) * inv * inv - 1.0,
                                    fmin(dx, dy) * inv,
                                    fmax(dx, dy) * inv};   // the lune-order key
    for (int k = 0; k < kMlpFeatures; ++k) f[k] = (float)fmin(64.0, fmax(-64.0, v[k]));
}

__device__ inline float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Score with bf16 weights [W1, b1, w2, b2] and float32 accumulation.
__device__ inline float mlp_score_bf16(const uint16_t *wb, const float *f) {
    const uint16_t *W1 = wb, *b1 = wb + kMlpFeatures * kMlpHidden, *w2 = b1 + kMlpHidden;
    float s = bf16_bits_to_f32(wb[kMlpParams - 1]);
    for (int j = 0; j < kMlpHidden; ++j) {
        float a = bf16_bits_to_f32(b1[j]);
        for (int k = 0; k < kMlpFeatures; ++k) a = fmaf(f[k], bf16_bits_to_f32(W1[k * kMlpHidden + j]), a);
        s = fmaf(a > 0.f ? a : 0.f, bf16_bits_to_f32(w2[j]), s);
    }
    return s;
}

// k_mlp.hip
void launch_mlp_grad(hipStream_t s, const float *theta, const float *feats, const uint8_t *labels, int64_t n,
                     float *grad, float *loss, DevBuf &work);
// The same gradient with the partials in the library's fixed device scratch
// (no allocation); n <= kNoAllocMaxSamples.
constexpr int64_t kNoAllocMaxSamples = GRNG_MLP_NOALLOC_MAX_SAMPLES;
void launch_mlp_grad_noalloc(hipStream_t s, const float *theta, const float *feats, const uint8_t *labels,
                             int64_t n, float *grad, float *loss_dev);
void launch_adam(hipStream_t s, float *theta, const float *g, float *m, float *v, int t, float lr);
void launch_pack_bf16(hipStream_t s, const float *theta, uint16_t *out);
void launch_mlp_score(hipStream_t s, const uint16_t *wb, const float *feats, int64_t n, float *scores);
// Returns the number of samples; writes them only when it fits in capacity.
int64_t launch_log_cells(hipStream_t s, int64_t nsamp, int64_t npairs, const int32_t *px, const int32_t *py,
                         const double *pd2, int dp, const double *Xh, const double *nrmh, const int32_t *grp_off,
                         const double *dvor, const double *rad, const double *Xp, const double *nrmp,
                         const int64_t *rel_off, const int32_t *rel_grp, const double *rel_d2x,
                         const uint64_t *row_dmax, float *feats, uint8_t *labels, int64_t capacity);

// State of the last build's exhaustive scan, kept for logging training samples.
struct ExhaustiveState {
    bool valid = false;            // set by a guided build_rng
    int64_t np = 0;
    DevBuf x, y, d2;               // pairs sorted by row point
    DevBuf rel_off, rel_grp, rel_d2x;
    DevBuf row_dmax;               // uint64 [n]: the d^2 bound the rows' cell lists were formed for
};

}  // namespace grng

struct grng_index {
    grng::BlockPool pool;      // first member: destroyed after every buffer below
    hipStream_t stream = nullptr;
    grng_options opt{};
    int32_t d = 0, dp = 0, q = 0;
    int64_t n = 0, cap = 0;
    double kmax = 0;           // largest |grid integer| seen so far
    grng::DevBuf X;            // double [cap*dp] exact coordinates, rows zero-padded
    grng::DevBuf nrm;          // double [cap] exact squared norms
    std::vector<grng::Layer> layers;
    grng::PointState ps;       // valid when rng_built (with a layer)
    grng::LayerAux aux;        // valid when rng_built (with a layer)
    bool rng_built = false;
    grng::DevBuf edges;        // int32 [2E] canonical exemplar RNG edges
    int64_t nedges = 0;
    grng::DevBuf counters;     // uint64 [C_NUM]
    grng::ExhaustiveState ex;  // last guided build's exhaustive pairs (for training samples)
    grng::DevBuf scorer;       // uint16 [kMlpParams] bf16 scorer weights (learned order)
    int32_t tuned_kw = 0;      // Proposition 1 witness pivots chosen by the autotuner (0: not tuned)
    int32_t tuned_k4 = 0;      // Stage IV pivot witnesses chosen by the autotuner (0: not tuned)
    int32_t tuned_prec = -1;   // GRNG_PREC_AUTO: the form chosen by the autotuner (-1: not tuned)
    double ms_tune = 0;        // device time the autotuner spent
    grng_stats stats{};
};

namespace grng {

// ---------------------------------------------------------------------------
// Launchers (one per kernel family; defined next to the kernels).

// k_basic.hip
void launch_grid_check(hipStream_t s, const float *x, int64_t count, double scale, uint64_t *kmax_bits,
                       int32_t *bad);
void launch_grid_check_f64(hipStream_t s, const double *x, int64_t count, double scale, uint64_t *kmax_bits,
                           int32_t *bad);
void launch_to_f64(hipStream_t s, const float *src, int64_t n, int d, int dp, double *dst, double *nrm);
void launch_dist2(hipStream_t s, const double *A, const double *nA, int64_t na, const double *B,
                  const double *nB, int64_t nb, int dp, double *out, int64_t ldo, bool use_mfma);
void launch_sqrt(hipStream_t s, const double *in, double *out, int64_t count);
void launch_gather_rows(hipStream_t s, const double *src, const int32_t *idx, int64_t n, int dp, double *dst);
void launch_gather_f64(hipStream_t s, const double *src, const int32_t *idx, int64_t n, double *dst);
void launch_to_f32(hipStream_t s, const double *src, int64_t count, float *dst);
void launch_iota_inverse(hipStream_t s, const int32_t *perm, int64_t n, int32_t *inv);
void launch_scan_i64(hipStream_t s, const int64_t *in, int64_t n, int64_t *out_excl);  // out has n+1
void launch_scan_i32_to_i64(hipStream_t s, const int32_t *in, int64_t n, int64_t *out_excl);
// Insertion merge of per-point state (old rows of each cell, then its batch rows).
void launch_merge_positions(hipStream_t s, int64_t n1, int64_t m, const int32_t *new_off, const int32_t *old_off,
                            const int32_t *bat_off, int32_t *src);
void launch_merge_rows(hipStream_t s, int64_t n1, size_t row_bytes, const int32_t *src, const void *old,
                       const void *bat, uint32_t bias, void *out);
void launch_merge_csr_len(hipStream_t s, int64_t n1, const int32_t *src, const int64_t *old_off,
                          const int64_t *bat_off, int32_t *len);
void launch_merge_csr_copy(hipStream_t s, int64_t n1, const int32_t *src, const int64_t *old_off,
                           const int32_t *old_idx, const int64_t *bat_off, const int32_t *bat_idx,
                           const int64_t *new_off, int32_t *new_idx);
void launch_bits_transpose(hipStream_t s, const uint64_t *rows, int64_t n, int32_t words, int64_t m,
                           uint64_t *cols);
void launch_fill_u64(hipStream_t s, uint64_t *p, int64_t count, uint64_t v);

// k_pivots.hip
// Candidates after adding pivots to a layer: pairs with a new pivot, and old links.
void launch_insert_candidates(hipStream_t s, int64_t m1, int32_t words1, const int32_t *oldpos,
                              const uint64_t *old_bits, int32_t words0, uint64_t *cand);
void launch_grng_layer(hipStream_t s, int64_t m, const double *dpp, const double *dpp2, const double *rad,
                       const int64_t *radi, int32_t q, const uint64_t *cand_bits, int32_t words,
                       const int32_t *witness_first, int64_t nfirst, uint64_t *bits, uint64_t *counters,
                       const uint8_t *isnew = nullptr);
void launch_relative_parents(hipStream_t s, int64_t mc, const int32_t *coarse_pos_in_fine,
                             const double *dpp2_fine, int64_t mf, const double *rad_c, const double *rad_f,
                             uint64_t *parent_bits, int32_t cwords);
void launch_guided_candidates(hipStream_t s, int64_t mf, const uint64_t *parent_bits, int32_t cwords,
                              const uint64_t *coarse_bits, int64_t mc, uint64_t *cand_bits, int32_t fwords);
void launch_point_pass1(hipStream_t s, int64_t n, int64_t m, const double *dxp, const double *rad,
                        int32_t *home, double *d2home, int32_t *npar, int32_t *second);
void launch_group_radius(hipStream_t s, int64_t n, const int32_t *home, const double *d2home,
                         uint64_t *d2vor_bits, int32_t *gcount);
void launch_parents(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp, const double *rad,
                    const int64_t *par_off, int32_t *par_idx);
void launch_shifted_pivot_dists(hipStream_t s, int64_t m, const double *dpp, const double *rad, const double *dvor,
                                float *bd, float *bv);
// Virtual-pivot bit rows of every point (Propositions 1-2).  cols: only the
// cell-radius bits of the listed pivots, OR-ed into v_rows (g_rows untouched).
void launch_vgrng(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp, const float *bd,
                  const float *bv, const double *rad, const double *dvor, const int32_t *gcount, const int64_t *par_off,
                  const int32_t *par_idx, const uint64_t *layer_bits, int32_t words, const int32_t *home,
                  const int32_t *wknn, int32_t kw, uint64_t *g_rows, uint64_t *v_rows, uint64_t *counters,
                  const int32_t *cols = nullptr, int32_t ncols = 0);

// k_rng.hip
struct PairList {
    int32_t *x;       // position of the row point (in its own point set, home order)
    int32_t *y;       // position of the other point (home order of the indexed set)
    double *d2;       // exact squared distance
    uint64_t *count;  // number of pairs requested (may exceed cap)
    int64_t cap;
};

// One side of the tiled pair enumeration (device pointers, home order).
struct PointsView {
    const double *Xh;        // [n][dp] coordinates
    const double *nrmh;      // [n] squared norms
    const int64_t *par_off;  // [n+1] parents CSR
    const int32_t *par_idx;
    const uint64_t *v_rows;  // [n][words] cell bits of the virtual-pivot test
    const uint64_t *g_cols;  // [m][nw] transposed domain bits of the virtual-pivot test
    int64_t nw;
    const int32_t *tiles;    // [ntiles][3]: start, length (<= 64), home cell
    const int32_t *gid;      // [n] global point id (PM_INSERT), else null
    int32_t new_from;        // ids >= new_from belong to the batch being inserted
    const uint8_t *is_new;   // [n] 1 for points of the batch being inserted (PM_NEW_ONLY), else null
};
// PM_SELF: both sides are the indexed set (pairs y > x).
// PM_NEW_ONLY (with PM_SELF): only pairs with at least one point of the batch
//   being inserted (dense batches: the batch points keep their cells' tiles).
// PM_INSERT: the row side is the batch being inserted (sparse batches, tiles
//   packed across cells) and the other side the whole set with the batch in
//   it; a pair of two batch points is kept once (larger id on the indexed
//   side) and a point is not paired with its own copy.
enum PairMode { PM_SELF = 1, PM_INSERT = 2, PM_NEW_ONLY = 4 };

constexpr int kPivWitness = 16;   // pivot witnesses per tile pair in the tiled pair kernel
void launch_pivot_knn(hipStream_t s, int64_t m, const double *dpp2, int32_t K, int32_t *pknn);   // pknn [m][16]
void launch_tile_vmask(hipStream_t s, int64_t ntiles, const int32_t *tiles, const uint64_t *v_rows, int32_t words,
                       uint64_t *tv);
// Tile pairs are listed in cells (row tile T, block of 64 indexed tiles),
// cells ordered by blocks of kTilePairBlockT row tiles (see k_tile_pairs);
// pass 0 (off == null) counts per cell into cnt[tile_pair_cells(ntA, ntB)],
// zeroed beforehand; pass 1 writes the pairs at the scanned cell offsets.
constexpr int kTilePairBlockT = 16;
inline int64_t tile_pair_cells(int64_t ntA, int64_t ntB) {
    return (ntA + kTilePairBlockT - 1) / kTilePairBlockT * kTilePairBlockT * ((ntB + 63) / 64);
}
void launch_tile_pairs(hipStream_t s, int64_t ntA, const int32_t *tilesA, const uint64_t *tvA, const uint8_t *newA,
                       int64_t ntB, const int32_t *tilesB, const uint64_t *tvB, const uint8_t *newB, int32_t words,
                       int mode, const int64_t *off, int32_t *cnt, int32_t *oT, int32_t *oU);
// Tile-pair records for the pair kernel: words per record.
constexpr int kPairRecordWords = 12 + 2 * 64;
void launch_pair_masks(hipStream_t s, int64_t tp0, int64_t n, const int32_t *tpT, const int32_t *tpU,
                       const PointsView &A, const PointsView &B, int mode, int32_t words, const int32_t *pknn,
                       int32_t K, uint64_t *rec);
void launch_pairs_tiled(hipStream_t s, int64_t ntp, const uint64_t *rec, const double *XA, const double *nrmA,
                        const double *XB, const double *nrmB, int mode, int dp, int32_t K,
                        const double *Xp, const double *nrmp, PairList out, uint64_t *dmax_bits, uint64_t *work,
                        uint64_t *counters);
// bf16 tiles; survivors are written with d2 = -1: launch_pairs_exact_d2 fills
// in their exact squared distances (and the per-row maxima) afterwards.
void launch_pairs_bf16(hipStream_t s, int64_t ntp, const uint64_t *rec, const float *XAf, const float *XBf, int mode,
                       int dp, int32_t K, const float *Xpf, PairList out, uint64_t *work, uint64_t *counters);
void launch_pairs_exact_d2(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, int dp, const double *XA,
                           const double *XB, double *d2, uint64_t *dmax_bits);
// Exhaustive path: every pair with its distance key (squared Euclidean, L1
// or L-infinity distance: GRNG_METRIC_*), then every pair against every point
// for the graph's empty region (GRNG_GRAPH_*).
void launch_pairs_all(hipStream_t s, int64_t nA, const double *XA, const double *nrmA, int64_t nB, const double *XB,
                      const double *nrmB, int dp, bool self, int metric, PairList out, uint64_t *counters);
void launch_relevant_groups(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp,
                            const double *dvor, const int32_t *gcount, const uint64_t *dmax_bits,
                            const int64_t *rel_off, int32_t *rel_cnt, int32_t *rel_grp, double *rel_d2x,
                            uint64_t *counters, bool sort = true);
void launch_pairs_sort_rows(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, const double *pd2,
                            int64_t n, int32_t *cnt, int64_t *off, int32_t *ox, int32_t *oy, double *od2);
void launch_lune_guided(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const double *pd2,
                        int dp, const double *Xx, const double *nrmx, const double *Xh, const double *nrmh,
                        int64_t nh, const double *dhome, const float *Xxf, const float *Xhf, const float *dhomef,
                        const int32_t *zstart, const int32_t *grp_off, const double *dvor,
                        const double *Xp, const double *nrmp, const int64_t *rel_off, const int32_t *rel_grp,
                        const double *rel_d2x, const double *rad, const uint16_t *scorer, bool lune_order,
                        bool prekilled, uint8_t *alive,
                        uint64_t *work, uint64_t *counters);
constexpr int kPartnerWitnesses = 64;   // partners per row point in one list
constexpr int kPartnerLists = 2;        // lists: the 64 nearest partners, then the next 64
constexpr double kPartnerDeepShare = 0.01;   // the next list is used while this share of kills came from deep partners
// Stage V with the row's other candidates as witnesses: each row point's 64
// nearest partners in a row-sorted pair list (off: row offsets) and, when
// off2 is given, in the same pairs sorted by their second point (with a
// nearer lists pid / pd2p: the next 64); then a proven-kill pass writing
// alive[p] (0: proven non-edge, 1: left to the scan; again: pairs decided
// with a nearer list are skipped).
void launch_partner_top(hipStream_t s, int64_t nrows, const int64_t *off, const int32_t *py, const double *pd2,
                        const int64_t *off2, const int32_t *py2, const double *pd22, const int32_t *pid,
                        const float *pd2p, int32_t *wid, float *wd2);
void launch_partner_witness(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, const double *pd2,
                            int dp, const float *Xf, const double *Xd, const int32_t *wid, const float *wd2,
                            bool both, bool again, uint8_t *alive, uint64_t *counters);
// Per row of a row-sorted pair list, the largest d^2 of its pairs with
// alive[p] != 0 (0 when there is none), as float64 bits.
void launch_live_dmax(hipStream_t s, int64_t nrows, const int64_t *off, const double *pd2, const uint8_t *alive,
                      uint64_t *dmax_bits);
void launch_lune_all(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const double *pd2,
                     int64_t n, int dp, const double *Xx, const double *nrmx, const double *X, const double *nrm,
                     int64_t z_from, int metric, int graph, int beta_q, int grid_exp, uint8_t *alive,
                     uint64_t *counters);
void launch_pair_d2(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, int dp, const double *Xh,
                    const double *nrmh, double *d2, uint64_t *dmax_bits);
void launch_query_csr(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                      const int32_t *qperm, const int32_t *perm, int64_t nq, int32_t *deg, const int64_t *off,
                      int32_t *fill, int32_t *nbr, int pass);
void launch_pairs_to_ids(hipStream_t s, int64_t np, int32_t *px, int32_t *py, const int32_t *mx, const int32_t *my);
void launch_sort_segments(hipStream_t s, int64_t nseg, const int64_t *off, int32_t *vals);
void launch_map_ids(hipStream_t s, int64_t count, int32_t *v, const int32_t *map);
void launch_edges_to_pairs(hipStream_t s, int64_t ne, const int32_t *uv, const int32_t *inv, int32_t *px, int32_t *py);

// k_edges.hip
void launch_edges_count(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py,
                        const uint8_t *alive, const int32_t *perm, int32_t *deg);
void launch_edges_fill(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                       const int32_t *perm, const int64_t *off, int32_t *fillpos, int32_t *nbr);
void launch_edges_emit(hipStream_t s, int64_t n, const int64_t *off, int32_t *nbr, int32_t *uv);
void launch_bits_to_edges_count(hipStream_t s, int64_t m, const uint64_t *bits, int32_t words, int32_t *deg);
void launch_bits_to_edges_emit(hipStream_t s, int64_t m, const uint64_t *bits, int32_t words, const int64_t *off,
                               int32_t *uv);

}  // namespace grng
