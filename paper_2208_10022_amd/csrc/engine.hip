// Host engine and C ABI of the gfx950 exact RNG / GRNG library (see include/grng.h).
//
// Every step of the build runs in the library's own kernels on the caller's
// stream; the host only validates arguments, sizes buffers, performs the
// counting sort that orders points by home cell, and moves small arrays.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "common.h"

namespace grng {

namespace {

thread_local std::string g_last_error;

// Failure injection for tests of the error paths: with GRNG_FAIL_ALLOC_AT=k
// in the environment, the k-th device allocation of each C-ABI call fails
// with GRNG_ENOMEM (the variable is read at the start of every call).
thread_local int64_t g_alloc_calls = 0;
thread_local int64_t g_fail_at = -1;   // -1: disabled

void arm_failure_injection() {
    const char *e = std::getenv("GRNG_FAIL_ALLOC_AT");
    g_fail_at = (e && *e) ? std::atoll(e) : -1;
    g_alloc_calls = 0;
}

int64_t fail_at() { return g_fail_at; }

constexpr int kDefaultK = kPivWitness;
constexpr int kDefaultVgrngPivots = 256;

// Witness-pivot counts in effect: the autotuner's choice, else the option,
// else the default.
int32_t vgrng_pivots(const grng_index *idx, int64_t m) {
    const int32_t k = idx->tuned_kw > 0 ? idx->tuned_kw
                                        : (idx->opt.vgrng_pivots > 0 ? idx->opt.vgrng_pivots : kDefaultVgrngPivots);
    return (int32_t)std::min<int64_t>(m, k);
}

int32_t stage4_pivots(const grng_index *idx) {
    return idx->tuned_k4 > 0 ? idx->tuned_k4 : (idx->opt.stage4_pivots > 0 ? idx->opt.stage4_pivots : kDefaultK);
}

// Arithmetic form in effect: the option, or under GRNG_PREC_AUTO the
// autotuner's choice of the pair kernel's tiles, else bf16 tiles from a
// padded dimension of 32 (one bf16 MFMA step deep).
int32_t precision(const grng_index *idx) {
    if (idx->opt.precision != GRNG_PREC_AUTO) return idx->opt.precision;
    if (idx->tuned_prec >= 0) return idx->tuned_prec;
    return idx->dp >= 32 ? GRNG_PREC_BF16 : GRNG_PREC_FP32;
}

struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit EventTimer(hipStream_t st) : s(st) {
        GRNG_HIP(hipEventCreate(&a));
        GRNG_HIP(hipEventCreate(&b));
        GRNG_HIP(hipEventRecord(a, s));
    }
    double stop() {
        GRNG_HIP(hipEventRecord(b, s));
        GRNG_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        GRNG_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~EventTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

template <class T>
void d2h(std::vector<T> &dst, const void *src, size_t count, hipStream_t s) {
    dst.resize(count);
    if (count) GRNG_HIP(hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s));
    GRNG_HIP(hipStreamSynchronize(s));
}

template <class T>
void h2d(DevBuf &dst, const std::vector<T> &src, hipStream_t s) {
    dst.alloc(src.size() * sizeof(T));
    if (!src.empty()) GRNG_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    GRNG_HIP(hipStreamSynchronize(s));   // the host vector may go away after return
}

void zero(DevBuf &b, hipStream_t s) { launch_fill_u64(s, b.as<uint64_t>(), (int64_t)(b.bytes / 8), 0ull); }

void check_opts(const grng_options *o) {
    require(o != nullptr, GRNG_EINVAL, "options pointer is NULL");
    require(o->grid_exp >= 0 && o->grid_exp <= 60, GRNG_EINVAL, "grid_exp must be in [0, 60]");
    require(o->precision >= GRNG_PREC_FP64 && o->precision <= GRNG_PREC_AUTO, GRNG_EINVAL, "unknown precision");
    require(o->witness_order == GRNG_ORDER_DISTANCE || o->witness_order == GRNG_ORDER_LEARNED ||
                o->witness_order == GRNG_ORDER_LUNE, GRNG_EINVAL,
            "unknown witness order");
    require(o->use_graph == 0, GRNG_EINVAL, "use_graph must be 0 (graph capture is not implemented)");
    require(o->autotune == 0 || o->autotune == 1, GRNG_EINVAL, "autotune must be 0 or 1");
    require(o->stage4_pivots >= 0 && o->stage4_pivots <= kPivWitness, GRNG_EINVAL, "stage4_pivots must be in [0, 16]");
    require(o->vgrng_pivots >= 0, GRNG_EINVAL, "vgrng_pivots must be >= 0");
    require(o->metric >= GRNG_METRIC_L2 && o->metric <= GRNG_METRIC_LINF, GRNG_EINVAL, "unknown metric");
    require(o->graph >= GRNG_GRAPH_RNG && o->graph <= GRNG_GRAPH_BETA, GRNG_EINVAL, "unknown graph");
    require(o->graph == GRNG_GRAPH_RNG || o->metric == GRNG_METRIC_L2, GRNG_EINVAL,
            "the Gabriel graph and the beta-skeleton are defined for the Euclidean metric only");
    if (o->graph == GRNG_GRAPH_BETA)
        require(o->beta_quarters >= 4 && o->beta_quarters <= 64, GRNG_EINVAL, "beta_quarters must be in [4, 64]");
    else
        require(o->beta_quarters == 0, GRNG_EINVAL, "beta_quarters must be 0 unless graph is GRNG_GRAPH_BETA");
    for (int t = 0; t < 3; ++t) require(o->reserved[t] == 0, GRNG_EINVAL, "reserved option fields must be 0");
}

// Validate float32 values on the device: finite, on the 2^-q grid, |k| < 2^24.
// Returns the largest |k|.
double grid_validate(grng_index *idx, const float *v, int64_t count, const char *what) {
    DevBuf tmp;
    tmp.alloc(16);
    zero(tmp, idx->stream);
    uint64_t *kmax = tmp.as<uint64_t>();
    int32_t *bad = reinterpret_cast<int32_t *>(kmax + 1);
    launch_grid_check(idx->stream, v, count, std::ldexp(1.0, idx->q), kmax, bad);
    std::vector<uint64_t> h;
    d2h(h, tmp.p, 2, idx->stream);
    double km;
    std::memcpy(&km, &h[0], 8);
    require((h[1] & 0xffffffffu) == 0, GRNG_ENOTGRID,
            std::string(what) + ": values must be finite multiples of 2^-grid_exp with |value * 2^grid_exp| < 2^24");
    return km;
}

void check_magnitude(const grng_index *idx, double kmax) {
    // d * kmax^2 < 2^51 keeps every float64 partial sum of a squared distance exact.
    require((double)idx->d * kmax * kmax < std::ldexp(1.0, 51), GRNG_ENOTGRID,
            "coordinates too large for exact float64 squared distances: need d * kmax^2 < 2^51");
}

int32_t words_of(int64_t m) { return (int32_t)div_up(m, 64); }

// Sorted canonical edge list from a symmetric bitset.
void bits_to_edges(hipStream_t s, int64_t m, const DevBuf &bits, int32_t words, DevBuf &edges, int64_t &ne) {
    DevBuf deg, off;
    deg.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
    off.alloc(sizeof(int64_t) * (size_t)(m + 1));
    launch_bits_to_edges_count(s, m, bits.as<uint64_t>(), words, deg.as<int32_t>());
    launch_scan_i32_to_i64(s, deg.as<int32_t>(), m, off.as<int64_t>());
    std::vector<int64_t> tot;
    d2h(tot, off.as<int64_t>() + m, 1, s);
    ne = tot[0];
    edges.alloc(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(ne, 1));
    launch_bits_to_edges_emit(s, m, bits.as<uint64_t>(), words, off.as<int64_t>(), edges.as<int32_t>());
}

// Sorted canonical edge list (point ids) from surviving pairs.
void pairs_to_edges(hipStream_t s, int64_t n, int64_t npairs, const int32_t *px, const int32_t *py,
                    const uint8_t *alive, const int32_t *perm, DevBuf &edges, int64_t &ne) {
    DevBuf deg, fill, off, nbr;
    deg.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 2));
    fill.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 2));
    zero(deg, s);
    zero(fill, s);
    off.alloc(sizeof(int64_t) * (size_t)(n + 1));
    launch_edges_count(s, npairs, px, py, alive, perm, deg.as<int32_t>());
    launch_scan_i32_to_i64(s, deg.as<int32_t>(), n, off.as<int64_t>());
    std::vector<int64_t> tot;
    d2h(tot, off.as<int64_t>() + n, 1, s);
    ne = tot[0];
    nbr.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(ne, 1));
    edges.alloc(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(ne, 1));
    launch_edges_fill(s, npairs, px, py, alive, perm, off.as<int64_t>(), fill.as<int32_t>(), nbr.as<int32_t>());
    launch_edges_emit(s, n, off.as<int64_t>(), nbr.as<int32_t>(), edges.as<int32_t>());
}

struct Pairs {
    DevBuf x, y, d2, count;
    int64_t cap = 0;
    void reserve(int64_t c) {
        cap = std::max<int64_t>(c, 1);
        x.alloc(sizeof(int32_t) * (size_t)cap);
        y.alloc(sizeof(int32_t) * (size_t)cap);
        d2.alloc(sizeof(double) * (size_t)cap);
        if (!count.p) count.alloc(8);
    }
    PairList view() { return PairList{x.as<int32_t>(), y.as<int32_t>(), d2.as<double>(), count.as<uint64_t>(), cap}; }
};

void read_counters(grng_index *idx, uint64_t out[C_NUM]) {
    std::vector<uint64_t> h;
    d2h(h, idx->counters.p, C_NUM, idx->stream);
    for (int t = 0; t < C_NUM; ++t) out[t] = h[t];
}

void reset_counters(grng_index *idx) { zero(idx->counters, idx->stream); }

// ---------------------------------------------------------------------------

void do_create(grng_index **out, const float *pts, int64_t n, int32_t d, void *stream, const grng_options *opt) {
    require(out != nullptr, GRNG_EINVAL, "out pointer is NULL");
    *out = nullptr;
    require(pts != nullptr, GRNG_EINVAL, "points pointer is NULL");
    require(n >= 1 && n <= (int64_t)INT32_MAX - 1, GRNG_EINVAL, "n must be in [1, 2^31 - 2]");
    require(d >= 1 && d <= 1024, GRNG_EINVAL, "d must be in [1, 1024]");
    check_opts(opt);
    auto *idx = new grng_index();
    try {
        idx->stream = static_cast<hipStream_t>(stream);
        idx->opt = *opt;
        idx->d = d;
        idx->dp = pad4(d);
        idx->q = opt->grid_exp;
        idx->counters.alloc(8 * C_NUM);
        reset_counters(idx);
        const double km = grid_validate(idx, pts, n * (int64_t)d, "points");
        check_magnitude(idx, km);
        idx->kmax = km;
        idx->n = n;
        idx->cap = n;
        idx->X.alloc(sizeof(double) * (size_t)(n * idx->dp));
        idx->nrm.alloc(sizeof(double) * (size_t)n);
        launch_to_f64(idx->stream, pts, n, d, idx->dp, idx->X.as<double>(), idx->nrm.as<double>());
        GRNG_HIP(hipStreamSynchronize(idx->stream));
        idx->stats.n_points = n;
    } catch (...) {
        delete idx;
        throw;
    }
    *out = idx;
}

void do_build_layer(grng_index *idx, int32_t layer, const int32_t *pid_dev, const float *rad_dev, int64_t m) {
    require(idx != nullptr, GRNG_EINVAL, "index is NULL");
    require(pid_dev != nullptr && rad_dev != nullptr, GRNG_EINVAL, "pivot or radius pointer is NULL");
    require(layer >= 0, GRNG_EINVAL, "layer must be >= 0");
    require(layer <= (int32_t)idx->layers.size(), GRNG_ESTATE, "layers must be built in order 0, 1, ...");
    require(m >= 1 && m <= idx->n, GRNG_EINVAL, "m must be in [1, n]");
    require(idx->opt.metric == GRNG_METRIC_L2 && idx->opt.graph == GRNG_GRAPH_RNG, GRNG_EINVAL,
            "pivot layers guide the Euclidean RNG only; other metrics and graphs are built exhaustively");
    hipStream_t s = idx->stream;
    EventTimer timer(s);
    reset_counters(idx);
    Layer L;
    L.m = m;
    L.words = words_of(m);
    // Validate pivot ids on the host (distinct, ascending, in range).
    d2h(L.pid_host, pid_dev, (size_t)m, s);
    for (int64_t t = 0; t < m; ++t) {
        require(L.pid_host[t] >= 0 && L.pid_host[t] < idx->n, GRNG_EINVAL, "pivot id out of range");
        require(t == 0 || L.pid_host[t] > L.pid_host[t - 1], GRNG_EINVAL, "pivot ids must be strictly ascending");
    }
    const double rkmax = grid_validate(idx, rad_dev, m, "radii");
    (void)rkmax;
    std::vector<float> rad_f;
    d2h(rad_f, rad_dev, (size_t)m, s);
    std::vector<double> rad_d((size_t)m);
    std::vector<int64_t> rad_i((size_t)m);
    for (int64_t t = 0; t < m; ++t) {
        require(rad_f[t] >= 0.0f, GRNG_ENOTGRID, "radii must be >= 0");
        rad_d[t] = (double)rad_f[t];
        rad_i[t] = (int64_t)std::ldexp(rad_d[t], idx->q);
    }
    // Nested layers (Theorem 2): every coarser pivot is a pivot here.
    std::vector<int32_t> coarse_pos;
    if (layer > 0) {
        const Layer &C = idx->layers[layer - 1];
        coarse_pos.resize((size_t)C.m);
        for (int64_t t = 0; t < C.m; ++t) {
            auto it = std::lower_bound(L.pid_host.begin(), L.pid_host.end(), C.pid_host[t]);
            require(it != L.pid_host.end() && *it == C.pid_host[t], GRNG_EINVAL,
                    "pivots of layer l-1 must be a subset of the pivots of layer l");
            coarse_pos[t] = (int32_t)(it - L.pid_host.begin());
        }
    }
    L.pid.alloc(sizeof(int32_t) * (size_t)m);
    GRNG_HIP(hipMemcpyAsync(L.pid.p, pid_dev, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, s));
    h2d(L.rad, rad_d, s);
    h2d(L.radi, rad_i, s);
    // Pivot coordinates and exact pivot-pivot distances (MFMA f64 tiles).
    DevBuf Xp, nrmp;
    Xp.alloc(sizeof(double) * (size_t)(m * idx->dp));
    nrmp.alloc(sizeof(double) * (size_t)m);
    launch_gather_rows(s, idx->X.as<double>(), L.pid.as<int32_t>(), m, idx->dp, Xp.as<double>());
    launch_gather_f64(s, idx->nrm.as<double>(), L.pid.as<int32_t>(), m, nrmp.as<double>());
    L.dpp2.alloc(sizeof(double) * (size_t)(m * m));
    L.dpp.alloc(sizeof(double) * (size_t)(m * m));
    launch_dist2(s, Xp.as<double>(), nrmp.as<double>(), m, Xp.as<double>(), nrmp.as<double>(), m, idx->dp,
                 L.dpp2.as<double>(), m, true);
    launch_sqrt(s, L.dpp2.as<double>(), L.dpp.as<double>(), m * m);
    L.bits.alloc(sizeof(uint64_t) * (size_t)(m * L.words));
    DevBuf cand, wfirst;
    const uint64_t *cand_ptr = nullptr;
    const int32_t *wfirst_ptr = nullptr;
    int64_t nfirst = 0;
    if (layer > 0) {
        const Layer &C = idx->layers[layer - 1];
        const int32_t cw = C.words;
        DevBuf cpos;
        h2d(cpos, coarse_pos, s);
        L.parent_bits.alloc(sizeof(uint64_t) * (size_t)(m * cw));
        launch_relative_parents(s, C.m, cpos.as<int32_t>(), L.dpp2.as<double>(), m, C.rad.as<double>(),
                                L.rad.as<double>(), L.parent_bits.as<uint64_t>(), cw);
        cand.alloc(sizeof(uint64_t) * (size_t)(m * L.words));
        launch_guided_candidates(s, m, L.parent_bits.as<uint64_t>(), cw, C.bits.as<uint64_t>(), C.m,
                                 cand.as<uint64_t>(), L.words);
        cand_ptr = cand.as<uint64_t>();
        wfirst = std::move(cpos);
        wfirst_ptr = wfirst.as<int32_t>();
        nfirst = C.m;
    }
    launch_grng_layer(s, m, L.dpp.as<double>(), L.dpp2.as<double>(), L.rad.as<double>(), L.radi.as<int64_t>(),
                      idx->q, cand_ptr, L.words, wfirst_ptr, nfirst, L.bits.as<uint64_t>(),
                      idx->counters.as<uint64_t>());
    bits_to_edges(s, m, L.bits, L.words, L.edges, L.nedges);
    const double ms = timer.stop();
    uint64_t c[C_NUM];
    read_counters(idx, c);
    // Commit: discard finer layers and the RNG built on them.
    idx->layers.resize((size_t)layer);
    idx->layers.push_back(std::move(L));
    idx->rng_built = false;
    idx->ps = PointState();
    idx->ex = ExhaustiveState();
    idx->edges.release();
    idx->nedges = 0;
    idx->stats.n_layers = (int64_t)idx->layers.size();
    idx->stats.ms_layers = ms;
    idx->stats.witness_tests = (double)c[C_WTEST];
    idx->stats.rechecks = (double)c[C_RECHECK];
    idx->stats.distance_computations = (double)(m * (m - 1) / 2);
}

// Exact RNG without a pivot layer: every pair against every point.
void build_rng_brute(grng_index *idx, DevBuf &edges, int64_t &ne, double &ms_lune) {
    hipStream_t s = idx->stream;
    const int64_t n = idx->n;
    Pairs P;
    P.reserve(n * (n - 1) / 2);
    zero(P.count, s);
    launch_pairs_all(s, n, idx->X.as<double>(), idx->nrm.as<double>(), n, idx->X.as<double>(), idx->nrm.as<double>(),
                     idx->dp, true, idx->opt.metric, P.view(), idx->counters.as<uint64_t>());
    const int64_t np = n * (n - 1) / 2;
    DevBuf alive;
    alive.alloc((size_t)std::max<int64_t>(np, 8));
    EventTimer lt(s);
    launch_lune_all(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), n, idx->dp, idx->X.as<double>(),
                    idx->nrm.as<double>(), idx->X.as<double>(), idx->nrm.as<double>(), 0, idx->opt.metric,
                    idx->opt.graph, idx->opt.beta_quarters, idx->opt.grid_exp, alive.as<uint8_t>(),
                    idx->counters.as<uint64_t>());
    ms_lune = lt.stop();
    pairs_to_edges(s, n, np, P.x.as<int32_t>(), P.y.as<int32_t>(), alive.as<uint8_t>(), nullptr, edges, ne);
}

// Stage trace on stderr when the environment sets GRNG_TRACE (diagnostics of
// long builds: each line is printed when its stage has finished on the device).
bool trace_on() {
    static const bool on = std::getenv("GRNG_TRACE") != nullptr;
    return on;
}

void trace(const char *stage, double ms, int64_t count) {
    if (trace_on()) std::fprintf(stderr, "[grng] %s done: %.1f ms (%lld)\n", stage, ms, (long long)count);
}

struct BuildTimes {
    double vgrng = 0, masks = 0, pairs = 0, lune = 0, partner = 0;
    int64_t tile_pairs = 0;
    double host_dist = 0;   // squared distances of whole tables (point-pivot D_XP) computed on the way
};

// Pivot-side tables of the finest layer (coordinates, nearest pivots).
void prepare_aux(grng_index *idx, const Layer &L, LayerAux &aux) {
    hipStream_t s = idx->stream;
    const int64_t m = L.m;
    const int dp = idx->dp;
    aux.Xp.alloc(sizeof(double) * (size_t)(m * dp));
    aux.nrmp.alloc(sizeof(double) * (size_t)m);
    launch_gather_rows(s, idx->X.as<double>(), L.pid.as<int32_t>(), m, dp, aux.Xp.as<double>());
    launch_gather_f64(s, idx->nrm.as<double>(), L.pid.as<int32_t>(), m, aux.nrmp.as<double>());
    aux.Xpf.alloc(sizeof(float) * (size_t)(m * dp));
    launch_to_f32(s, aux.Xp.as<double>(), m * dp, aux.Xpf.as<float>());
    aux.pknn.alloc(4 * (size_t)(m * kPivWitness));
    launch_pivot_knn(s, m, L.dpp2.as<double>(), kPivWitness, aux.pknn.as<int32_t>());
    // Proposition 1 witnesses per point block: the pivots nearest its home cell.
    aux.kw = vgrng_pivots(idx, m);
    if (aux.kw < m) {
        aux.wknn.alloc(4 * (size_t)(m * aux.kw));
        launch_pivot_knn(s, m, L.dpp2.as<double>(), aux.kw, aux.wknn.as<int32_t>());
    } else {
        aux.wknn.release();
    }
    aux.bd.alloc(4 * (size_t)(m * m));
    aux.bv.alloc(4 * (size_t)(m * m));
}

// Prepare a point set against the finest layer L.
//   cells == nullptr: P is the indexed set; its home cells become the witness
//     groups (cell radii, sizes) and the shifted pivot tables in aux are filled.
//   cells != nullptr: P is a query set; cell radii and sizes come from `cells`.
// is_new (host, optional): per input index, 1 for points inserted in this batch.
// locality: inside a home cell, group the points by their second-nearest
// pivot (a full build only: insertion needs each cell's old points first).
// dxp_ready: P.dxp already holds the point-pivot distances.
void prepare_points(grng_index *idx, const Layer &L, LayerAux &aux, const double *X, const double *nrm, int64_t n,
                    const PointState *cells, const std::vector<uint8_t> *is_new, PointState &P, BuildTimes &bt,
                    bool locality = false, bool dxp_ready = false) {
    hipStream_t s = idx->stream;
    const int64_t m = L.m;
    const int dp = idx->dp;
    const int32_t words = L.words;
    uint64_t *ctr = idx->counters.as<uint64_t>();
    const bool indexed = cells == nullptr;
    P.n = n;
    // A1: exact point-pivot distances (MFMA f64 tiles), input order [n][m].
    if (!dxp_ready) {
        P.dxp.alloc(sizeof(double) * (size_t)(n * m));
        launch_dist2(s, X, nrm, n, aux.Xp.as<double>(), aux.nrmp.as<double>(), m, dp, P.dxp.as<double>(), m, true);
        bt.host_dist += (double)n * (double)m;
    }
    // A2: parent counts, home cell, cell radius.
    DevBuf home, d2home, npar, d2vor, gcount, second;
    home.alloc(4 * (size_t)n);
    d2home.alloc(8 * (size_t)n);
    npar.alloc(4 * (size_t)n);
    if (locality) second.alloc(4 * (size_t)n);
    launch_point_pass1(s, n, m, P.dxp.as<double>(), L.rad.as<double>(), home.as<int32_t>(), d2home.as<double>(),
                       npar.as<int32_t>(), locality ? second.as<int32_t>() : nullptr);
    std::vector<int32_t> h_home, h_npar, h_gcount((size_t)m, 0);
    std::vector<double> h_d2home, h_d2vor((size_t)m, 0.0);
    d2h(h_home, home.p, (size_t)n, s);
    trace("pivot distances and home cells", 0.0, n * m);
    d2h(h_npar, npar.p, (size_t)n, s);
    if (indexed) d2h(h_d2home, d2home.p, (size_t)n, s);
    // Home order: stable counting sort by home cell (host, O(n)), after one by
    // the second-nearest pivot when asked, so that a 64-point tile of a cell
    // faces fewer neighbouring cells.
    std::vector<int32_t> order((size_t)n);
    if (locality) {
        std::vector<int32_t> h_second;
        d2h(h_second, second.p, (size_t)n, s);
        std::vector<int64_t> at((size_t)m + 1, 0);
        for (int64_t x = 0; x < n; ++x) ++at[(size_t)h_second[x] + 1];
        for (int64_t c = 0; c < m; ++c) at[c + 1] += at[c];
        for (int64_t x = 0; x < n; ++x) order[at[h_second[x]]++] = (int32_t)x;
    } else {
        for (int64_t x = 0; x < n; ++x) order[x] = (int32_t)x;
    }
    for (int64_t x = 0; x < n; ++x) ++h_gcount[h_home[x]];
    P.h_off.assign((size_t)m + 1, 0);
    for (int64_t c = 0; c < m; ++c) P.h_off[c + 1] = P.h_off[c] + h_gcount[c];
    P.h_perm.resize((size_t)n);
    {
        std::vector<int32_t> pos(P.h_off.begin(), P.h_off.end() - 1);
        for (int64_t t = 0; t < n; ++t) {
            const int32_t x = order[t];
            P.h_perm[pos[h_home[x]]++] = x;
        }
    }
    std::vector<int32_t> home_h((size_t)n);
    std::vector<int64_t> par_off((size_t)n + 1, 0);
    std::vector<double> dhome;
    P.orphans = 0;
    if (indexed) dhome.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t x = P.h_perm[i];
        home_h[i] = h_home[x];
        par_off[i + 1] = par_off[i] + h_npar[x];
        P.orphans += h_npar[x] == 0;
        if (indexed) {
            dhome[i] = std::sqrt(h_d2home[x]) * (1.0 + 1e-15);   // upper bound of d(x, p_home)
            h_d2vor[h_home[x]] = std::max(h_d2vor[h_home[x]], h_d2home[x]);
        }
    }
    h2d(P.perm, P.h_perm, s);
    h2d(P.home, home_h, s);
    h2d(P.par_off, par_off, s);
    if (indexed) {
        std::vector<double> dvor((size_t)m);
        for (int64_t c = 0; c < m; ++c) dvor[c] = std::sqrt(h_d2vor[c]) * (1.0 + 1e-15);   // upper bound of the cell radius
        h2d(P.grp_off, P.h_off, s);
        h2d(P.dhome, dhome, s);
        std::vector<float> dhomef((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            float f = (float)dhome[i];
            if ((double)f < dhome[i]) f = std::nextafter(f, INFINITY);
            dhomef[i] = f;
        }
        h2d(P.dhomef, dhomef, s);
        h2d(P.dvor, dvor, s);
        h2d(P.gcount, h_gcount, s);
        launch_shifted_pivot_dists(s, m, L.dpp.as<double>(), L.rad.as<double>(), P.dvor.as<double>(),
                                   aux.bd.as<float>(), aux.bv.as<float>());
    }
    const PointState &C = indexed ? P : *cells;
    P.inv.alloc(4 * (size_t)n);
    launch_iota_inverse(s, P.perm.as<int32_t>(), n, P.inv.as<int32_t>());
    P.Xh.alloc(sizeof(double) * (size_t)(n * dp));
    P.nrmh.alloc(sizeof(double) * (size_t)n);
    launch_gather_rows(s, X, P.perm.as<int32_t>(), n, dp, P.Xh.as<double>());
    launch_gather_f64(s, nrm, P.perm.as<int32_t>(), n, P.nrmh.as<double>());
    P.Xf.alloc(sizeof(float) * (size_t)(n * dp));
    launch_to_f32(s, P.Xh.as<double>(), n * dp, P.Xf.as<float>());
    // Parents and virtual-pivot bitsets (Propositions 1-2) as a tiled (min, max) product.
    P.par_idx.alloc(4 * (size_t)std::max<int64_t>(par_off[n], 1));
    launch_parents(s, n, m, P.perm.as<int32_t>(), P.dxp.as<double>(), L.rad.as<double>(), P.par_off.as<int64_t>(),
                   P.par_idx.as<int32_t>());
    P.g_rows.alloc(8 * (size_t)(n * words));
    P.v_rows.alloc(8 * (size_t)(n * words));
    {
        EventTimer vt(s);
        launch_vgrng(s, n, m, P.perm.as<int32_t>(), P.dxp.as<double>(), aux.bd.as<float>(), aux.bv.as<float>(),
                     L.rad.as<double>(), C.dvor.as<double>(), C.gcount.as<int32_t>(), P.par_off.as<int64_t>(),
                     P.par_idx.as<int32_t>(), L.bits.as<uint64_t>(), words, P.home.as<int32_t>(),
                     aux.wknn.as<int32_t>(), aux.kw, P.g_rows.as<uint64_t>(),
                     P.v_rows.as<uint64_t>(), ctr);
        const double ms = vt.stop();
        bt.vgrng += ms;
        trace("virtual-pivot bitsets", ms, n);
    }
    P.nw = div_up(n, 64);
    P.g_cols.alloc(8 * (size_t)(m * P.nw));
    launch_bits_transpose(s, P.g_rows.as<uint64_t>(), n, words, m, P.g_cols.as<uint64_t>());
    // Tiles.  Indexed points: chunks of <= 64 home-order points of one home
    // cell (the cell ball of a tile is then its cell's).  Queries and batches
    // being inserted: cells with few of them share packed tiles of up to 64
    // consecutive home-order points; the tile's cell (its first point's) only
    // chooses the Stage IV pivot witnesses there, which any pivots may be.
    std::vector<int32_t> tiles;
    std::vector<uint8_t> tnew, newh;
    if (indexed) {
        // With a dense batch being inserted (is_new), the batch points follow
        // the old ones inside each cell (stable order) and tiles are cut at
        // that boundary too: a tile is all old or all new.
        if (is_new) {
            newh.resize((size_t)n);
            for (int64_t r = 0; r < n; ++r) newh[r] = (*is_new)[P.h_perm[r]];
        }
        auto add_tiles = [&](int32_t b, int32_t e, int64_t c, uint8_t fresh) {
            for (int32_t st = b; st < e; st += 64) {
                tiles.push_back(st);
                tiles.push_back(std::min<int32_t>(64, e - st));
                tiles.push_back((int32_t)c);
                if (is_new) tnew.push_back(fresh);
            }
        };
        for (int64_t c = 0; c < m; ++c) {
            int32_t split = P.h_off[c + 1];
            if (is_new)
                for (int32_t r = P.h_off[c]; r < P.h_off[c + 1]; ++r)
                    if (newh[r]) { split = r; break; }
            add_tiles(P.h_off[c], split, c, 0);
            add_tiles(split, P.h_off[c + 1], c, 1);
        }
    } else {
        // A cell with at least kOwnTile points keeps tiles of its own (their
        // pivot witnesses and tile-pair filter stay specific); runs of
        // consecutive smaller cells share packed tiles.
        constexpr int32_t kOwnTile = 16;
        int32_t open = -1;   // start of the packed tile being filled
        auto close_packed = [&](int32_t end) {
            if (open >= 0 && end > open) {
                tiles.push_back(open);
                tiles.push_back(end - open);
                tiles.push_back(home_h[open]);
            }
            open = -1;
        };
        for (int64_t c = 0; c < m; ++c) {
            const int32_t b = P.h_off[c], e = P.h_off[c + 1];
            if (e == b) continue;
            if (e - b >= kOwnTile) {
                close_packed(b);
                for (int32_t st = b; st < e; st += 64) {
                    tiles.push_back(st);
                    tiles.push_back(std::min<int32_t>(64, e - st));
                    tiles.push_back((int32_t)c);
                }
                continue;
            }
            if (open >= 0 && e - open > 64) close_packed(b);
            if (open < 0) open = b;
        }
        close_packed((int32_t)n);
    }
    P.ntiles = (int64_t)tiles.size() / 3;
    h2d(P.tiles, tiles, s);
    P.tv.alloc(8 * (size_t)std::max<int64_t>(P.ntiles * words, 1));
    launch_tile_vmask(s, P.ntiles, P.tiles.as<int32_t>(), P.v_rows.as<uint64_t>(), words, P.tv.as<uint64_t>());
    if (is_new) {
        h2d(P.is_new, newh, s);
        h2d(P.tnew, tnew, s);
    }
}

// Insertion state (Section 2, Stage VII; Proposition 5).  The indexed points
// S keep their point-pivot distances, home cells, parents and bit rows from
// one insertion to the next.  The batch is prepared on its own against the
// cells as they are after the insertion (B: also the row side of a sparse
// insertion) and merged into each home cell after the cell's old points (N).
// An old point's bit rows depend on the cells only through their radius
// bounds and sizes, so they stay valid except in the 64-cell words of cells
// whose bound grew or that were empty: those words are recomputed for every
// point.  The batch's distance rows are appended to S.dxp when it has room
// (rows past S.n are unused, so S stays valid) and N then takes the buffer
// over (dxp_moved: the caller gives it back if the insertion fails); else N
// gets a larger copy.  bd_new, bv_new: the shifted pivot tables for the new
// cell bounds, swapped into aux on success.  newrad: radius bound of each
// cell's batch points (0 where there are none).
void merge_batch(grng_index *idx, const Layer &L, LayerAux &aux, PointState &S, const double *Xb, const double *nrmb,
                 int64_t nb, bool dense, PointState &N, PointState &B, DevBuf &bd_new, DevBuf &bv_new,
                 std::vector<double> &newrad, bool &dxp_moved, BuildTimes &bt) {
    hipStream_t s = idx->stream;
    const int64_t m = L.m, n0 = S.n, n1 = n0 + nb;
    const int dp = idx->dp;
    const int32_t words = L.words;
    uint64_t *ctr = idx->counters.as<uint64_t>();
    require(S.dxp.p != nullptr && S.dxp.bytes >= sizeof(double) * (size_t)(n0 * m), GRNG_ESTATE,
            "point-pivot distances of the indexed points are missing");
    EventTimer timer(s);
    // Batch home cells and their squared distances.
    B.dxp.alloc(sizeof(double) * (size_t)(nb * m));
    launch_dist2(s, Xb, nrmb, nb, aux.Xp.as<double>(), aux.nrmp.as<double>(), m, dp, B.dxp.as<double>(), m, true);
    bt.host_dist += (double)nb * (double)m;
    DevBuf hb, d2b, npb;
    hb.alloc(4 * (size_t)nb);
    d2b.alloc(8 * (size_t)nb);
    npb.alloc(4 * (size_t)nb);
    launch_point_pass1(s, nb, m, B.dxp.as<double>(), L.rad.as<double>(), hb.as<int32_t>(), d2b.as<double>(),
                       npb.as<int32_t>(), nullptr);
    std::vector<int32_t> h_hb;
    std::vector<double> h_d2b, dv_old;
    d2h(h_hb, hb.p, (size_t)nb, s);
    d2h(h_d2b, d2b.p, (size_t)nb, s);
    d2h(dv_old, S.dvor.p, (size_t)m, s);
    // Cells after the insertion: sizes, radius bounds (the same values a
    // rebuild computes: the bound is monotone in the squared radius), offsets.
    std::vector<int32_t> bcnt((size_t)m, 0), gcount((size_t)m);
    std::vector<double> dvor(dv_old);
    newrad.assign((size_t)m, 0.0);
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t c = h_hb[b];
        ++bcnt[c];
        newrad[c] = std::max(newrad[c], std::sqrt(h_d2b[b]) * (1.0 + 1e-15));
        dvor[c] = std::max(dvor[c], newrad[c]);
    }
    std::vector<int32_t> grown;   // cells whose bound grew or that were empty
    N.n = n1;
    N.h_off.assign((size_t)m + 1, 0);
    for (int64_t c = 0; c < m; ++c) {
        const int32_t old = S.h_off[c + 1] - S.h_off[c];
        gcount[c] = old + bcnt[c];
        N.h_off[c + 1] = N.h_off[c] + gcount[c];
        if (bcnt[c] > 0 && (old == 0 || dvor[c] > dv_old[c])) grown.push_back((int32_t)c);
    }
    h2d(N.grp_off, N.h_off, s);
    h2d(N.dvor, dvor, s);
    h2d(N.gcount, gcount, s);
    bd_new.alloc(4 * (size_t)(m * m));
    bv_new.alloc(4 * (size_t)(m * m));
    launch_shifted_pivot_dists(s, m, L.dpp.as<double>(), L.rad.as<double>(), N.dvor.as<double>(),
                               bd_new.as<float>(), bv_new.as<float>());
    // The new tables stand in aux while the bit rows are computed.
    struct TablesIn {
        LayerAux &a;
        DevBuf &bd, &bv;
        TablesIn(LayerAux &a_, DevBuf &bd_, DevBuf &bv_) : a(a_), bd(bd_), bv(bv_) { swap(); }
        ~TablesIn() { swap(); }
        void swap() {
            std::swap(a.bd, bd);
            std::swap(a.bv, bv);
        }
    };
    {
        TablesIn in(aux, bd_new, bv_new);
        prepare_points(idx, L, aux, Xb, nrmb, nb, &N, nullptr, B, bt, false, true);
    }
    {
        std::vector<double> dh((size_t)nb);
        std::vector<float> dhf((size_t)nb);
        for (int64_t r = 0; r < nb; ++r) {
            dh[r] = std::sqrt(h_d2b[B.h_perm[r]]) * (1.0 + 1e-15);   // upper bound of d(x, p_home)
            float f = (float)dh[r];
            if ((double)f < dh[r]) f = std::nextafter(f, INFINITY);
            dhf[r] = f;
        }
        h2d(B.dhome, dh, s);
        h2d(B.dhomef, dhf, s);
    }
    // Merged home order and per-point rows.
    DevBuf src, boff;
    src.alloc(4 * (size_t)n1);
    h2d(boff, B.h_off, s);
    launch_merge_positions(s, n1, m, N.grp_off.as<int32_t>(), S.grp_off.as<int32_t>(), boff.as<int32_t>(),
                           src.as<int32_t>());
    auto merge = [&](DevBuf &dst, const DevBuf &a, const DevBuf &b, size_t row_bytes, uint32_t bias) {
        dst.alloc(row_bytes * (size_t)std::max<int64_t>(n1, 1));
        launch_merge_rows(s, n1, row_bytes, src.as<int32_t>(), a.p, b.p, bias, dst.p);
    };
    merge(N.perm, S.perm, B.perm, 4, (uint32_t)n0);
    merge(N.home, S.home, B.home, 4, 0);
    merge(N.Xh, S.Xh, B.Xh, 8 * (size_t)dp, 0);
    merge(N.nrmh, S.nrmh, B.nrmh, 8, 0);
    merge(N.Xf, S.Xf, B.Xf, 4 * (size_t)dp, 0);
    merge(N.dhome, S.dhome, B.dhome, 8, 0);
    merge(N.dhomef, S.dhomef, B.dhomef, 4, 0);
    merge(N.g_rows, S.g_rows, B.g_rows, 8 * (size_t)words, 0);
    merge(N.v_rows, S.v_rows, B.v_rows, 8 * (size_t)words, 0);
    {
        DevBuf plen;
        plen.alloc(4 * (size_t)n1);
        N.par_off.alloc(8 * (size_t)(n1 + 1));
        launch_merge_csr_len(s, n1, src.as<int32_t>(), S.par_off.as<int64_t>(), B.par_off.as<int64_t>(),
                             plen.as<int32_t>());
        launch_scan_i32_to_i64(s, plen.as<int32_t>(), n1, N.par_off.as<int64_t>());
        std::vector<int64_t> tot;
        d2h(tot, N.par_off.as<int64_t>() + n1, 1, s);
        N.par_idx.alloc(4 * (size_t)std::max<int64_t>(tot[0], 1));
        launch_merge_csr_copy(s, n1, src.as<int32_t>(), S.par_off.as<int64_t>(), S.par_idx.as<int32_t>(),
                              B.par_off.as<int64_t>(), B.par_idx.as<int32_t>(), N.par_off.as<int64_t>(),
                              N.par_idx.as<int32_t>());
    }
    N.orphans = S.orphans + B.orphans;
    N.inv.alloc(4 * (size_t)n1);
    launch_iota_inverse(s, N.perm.as<int32_t>(), n1, N.inv.as<int32_t>());
    // Point-pivot distances, input order: the batch rows follow the old ones.
    const size_t row = sizeof(double) * (size_t)m;
    if (S.dxp.bytes >= row * (size_t)n1) {
        N.dxp = std::move(S.dxp);
        dxp_moved = true;
    } else {
        N.dxp.alloc(row * (size_t)(n1 + n1 / 4));   // room for later batches
        GRNG_HIP(hipMemcpyAsync(N.dxp.p, S.dxp.p, row * (size_t)n0, hipMemcpyDeviceToDevice, s));
    }
    GRNG_HIP(hipMemcpyAsync(N.dxp.as<double>() + n0 * m, B.dxp.p, row * (size_t)nb, hipMemcpyDeviceToDevice, s));
    const double ms_merge = timer.stop();
    trace("insertion merge", ms_merge, n1);
    // Cell-radius bits of the grown cells, for every point.
    if (!grown.empty()) {
        DevBuf dcols;
        h2d(dcols, grown, s);
        TablesIn in(aux, bd_new, bv_new);
        EventTimer vt(s);
        launch_vgrng(s, n1, m, N.perm.as<int32_t>(), N.dxp.as<double>(), aux.bd.as<float>(), aux.bv.as<float>(),
                     L.rad.as<double>(), N.dvor.as<double>(), N.gcount.as<int32_t>(), N.par_off.as<int64_t>(),
                     N.par_idx.as<int32_t>(), L.bits.as<uint64_t>(), words, N.home.as<int32_t>(),
                     aux.wknn.as<int32_t>(), aux.kw, N.g_rows.as<uint64_t>(), N.v_rows.as<uint64_t>(), ctr,
                     dcols.as<int32_t>(), (int32_t)grown.size());
        const double ms = vt.stop();
        bt.vgrng += ms;
        trace("cell-radius bits of grown cells", ms, (int64_t)grown.size());
    }
    N.nw = div_up(n1, 64);
    N.g_cols.alloc(8 * (size_t)(m * N.nw));
    launch_bits_transpose(s, N.g_rows.as<uint64_t>(), n1, words, m, N.g_cols.as<uint64_t>());
    // Tiles: chunks of <= 64 points of one cell; with a dense batch, a cell's
    // old and batch points get tiles of their own.
    std::vector<int32_t> tiles;
    std::vector<uint8_t> tnew, newh;
    if (dense) newh.assign((size_t)n1, 0);
    auto add_tiles = [&](int32_t b, int32_t e, int64_t c, uint8_t fresh) {
        for (int32_t st = b; st < e; st += 64) {
            tiles.push_back(st);
            tiles.push_back(std::min<int32_t>(64, e - st));
            tiles.push_back((int32_t)c);
            if (dense) tnew.push_back(fresh);
        }
    };
    for (int64_t c = 0; c < m; ++c) {
        const int32_t b = N.h_off[c], e = N.h_off[c + 1];
        if (!dense) {
            add_tiles(b, e, c, 0);
            continue;
        }
        const int32_t split = b + (S.h_off[c + 1] - S.h_off[c]);
        add_tiles(b, split, c, 0);
        add_tiles(split, e, c, 1);
        for (int32_t r = split; r < e; ++r) newh[r] = 1;
    }
    N.ntiles = (int64_t)tiles.size() / 3;
    h2d(N.tiles, tiles, s);
    N.tv.alloc(8 * (size_t)std::max<int64_t>(N.ntiles * words, 1));
    launch_tile_vmask(s, N.ntiles, N.tiles.as<int32_t>(), N.v_rows.as<uint64_t>(), words, N.tv.as<uint64_t>());
    if (dense) {
        h2d(N.is_new, newh, s);
        h2d(N.tnew, tnew, s);
    }
}

// gid: global point ids of the set (PM_INSERT), or null; new_from: first id
// of the batch being inserted; with_new: pass the batch flags (PM_NEW_ONLY).
PointsView view_of(const PointState &P, const int32_t *gid, int32_t new_from, bool with_new) {
    return PointsView{P.Xh.as<double>(),      P.nrmh.as<double>(),     P.par_off.as<int64_t>(),
                      P.par_idx.as<int32_t>(), P.v_rows.as<uint64_t>(), P.g_cols.as<uint64_t>(),
                      P.nw,                    P.tiles.as<int32_t>(),   gid,
                      new_from,                with_new ? P.is_new.as<uint8_t>() : nullptr};
}

// Stages I-V over candidate tile pairs of A (row side) x B (indexed side).
void run_pairs(grng_index *idx, const Layer &L, const LayerAux &aux, const PointState &A, const PointState &B,
               int mode, Pairs &P, DevBuf &dmax, int64_t &np, BuildTimes &bt) {
    hipStream_t s = idx->stream;
    const int32_t words = L.words;
    const int32_t K = stage4_pivots(idx);
    uint64_t *ctr = idx->counters.as<uint64_t>();
    DevBuf tcnt, toff, tpT, tpU;
    const int64_t ncell = tile_pair_cells(A.ntiles, B.ntiles);
    tcnt.alloc(4 * (size_t)std::max<int64_t>(ncell, 2));
    zero(tcnt, s);
    toff.alloc(8 * (size_t)(ncell + 1));
    const bool with_new = (mode & PM_NEW_ONLY) != 0;
    const uint8_t *na = with_new ? A.tnew.as<uint8_t>() : nullptr, *nb = with_new ? B.tnew.as<uint8_t>() : nullptr;
    launch_tile_pairs(s, A.ntiles, A.tiles.as<int32_t>(), A.tv.as<uint64_t>(), na, B.ntiles, B.tiles.as<int32_t>(),
                      B.tv.as<uint64_t>(), nb, words, mode, nullptr, tcnt.as<int32_t>(), nullptr, nullptr);
    launch_scan_i32_to_i64(s, tcnt.as<int32_t>(), ncell, toff.as<int64_t>());
    std::vector<int64_t> ntp_h;
    d2h(ntp_h, toff.as<int64_t>() + ncell, 1, s);
    const int64_t ntp = ntp_h[0];
    tpT.alloc(4 * (size_t)std::max<int64_t>(ntp, 1));
    tpU.alloc(4 * (size_t)std::max<int64_t>(ntp, 1));
    launch_tile_pairs(s, A.ntiles, A.tiles.as<int32_t>(), A.tv.as<uint64_t>(), na, B.ntiles, B.tiles.as<int32_t>(),
                      B.tv.as<uint64_t>(), nb, words, mode, toff.as<int64_t>(), tcnt.as<int32_t>(), tpT.as<int32_t>(),
                      tpU.as<int32_t>());
    dmax.alloc(8 * (size_t)std::max<int64_t>(A.n, 1));
    // Survivor capacity: 64 per point, and up to 8,192 per point for small
    // row sets (an insertion batch: few rows, each facing the whole index),
    // at most 2^25 pairs.  A pass that overflows is run again with the exact
    // size; at a million points a pass takes tens of seconds where pruning
    // is weak, so there the first capacity is 256 per point when a quarter
    // of the free device memory holds it.
    int64_t cap = std::max<int64_t>(1 << 22, 64 * A.n);
    cap = std::max<int64_t>(cap, std::min<int64_t>(8192 * A.n, 1 << 25));
    if (A.n >= 500000) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess)
            cap = std::max<int64_t>(cap, std::min<int64_t>(256 * A.n, (int64_t)(fr / 4 / 17)));
    }
    std::vector<uint64_t> snapshot;
    d2h(snapshot, idx->counters.p, C_NUM, s);
    const bool ins = (mode & PM_INSERT) != 0;
    const PointsView va = view_of(A, ins ? A.gid.as<int32_t>() : nullptr, 0, with_new),
                     vb = view_of(B, ins ? B.perm.as<int32_t>() : nullptr, ins ? (int32_t)(B.n - A.n) : 0, with_new);
    // Tile-pair records (bounds, pivot ids and candidate masks), written by
    // the mask pass and streamed by the pair kernel, in chunks of at most
    // 2^21 tile pairs (2.3 GB).  Chunks that fit the last-level cache run
    // slower (the pair kernel's workgroups drain unevenly at the end of each
    // launch); 4x larger ones gain under 1% in a build but cost insertions
    // a fresh multi-GB allocation whenever their tile-pair count changes.
    const bool bf16 = precision(idx) == GRNG_PREC_BF16;
    const int64_t chunk = std::min<int64_t>(ntp, (int64_t)1 << 21);
    DevBuf rec;
    rec.alloc(8 * (size_t)kPairRecordWords * (size_t)std::max<int64_t>(chunk, 1));
    for (int attempt = 0; attempt < 3; ++attempt) {
        P.reserve(cap);
        zero(P.count, s);
        zero(dmax, s);
        double ms_m = 0.0, ms = 0.0;
        for (int64_t c0 = 0; c0 < ntp; c0 += chunk) {
            const int64_t nc = std::min<int64_t>(chunk, ntp - c0);
            EventTimer mt(s);
            launch_pair_masks(s, c0, nc, tpT.as<int32_t>(), tpU.as<int32_t>(), va, vb, mode, words,
                              aux.pknn.as<int32_t>(), K, rec.as<uint64_t>());
            ms_m += mt.stop();
            EventTimer pt(s);
            if (bf16)
                launch_pairs_bf16(s, nc, rec.as<uint64_t>(), A.Xf.as<float>(), B.Xf.as<float>(), mode, idx->dp, K,
                                  aux.Xpf.as<float>(), P.view(), ctr + C_WORK0, ctr);
            else
                launch_pairs_tiled(s, nc, rec.as<uint64_t>(), A.Xh.as<double>(), A.nrmh.as<double>(),
                                   B.Xh.as<double>(), B.nrmh.as<double>(), mode, idx->dp, K, aux.Xp.as<double>(),
                                   aux.nrmp.as<double>(), P.view(), dmax.as<uint64_t>(), ctr + C_WORK0, ctr);
            ms += pt.stop();
        }
        bt.masks += ms_m;
        bt.pairs += ms;
        trace("tile-pair masks (Stages I-III)", ms_m, ntp);
        trace("tile pairs (Stages IV-V)", ms, ntp);
        std::vector<uint64_t> h;
        d2h(h, P.count.p, 1, s);
        np = (int64_t)h[0];
        if (np <= cap) {
            if (bf16) {   // exact squared distances of the survivors, and each row's largest
                EventTimer dt(s);
                launch_pairs_exact_d2(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), idx->dp, A.Xh.as<double>(),
                                      B.Xh.as<double>(), P.d2.as<double>(), dmax.as<uint64_t>());
                bt.pairs += dt.stop();
            }
            break;
        }
        require(attempt < 2, GRNG_EDEVICE, "survivor count changed between identical passes");
        cap = np;   // rerun with room for every survivor, from the counters as they were
        GRNG_HIP(hipMemcpyAsync(idx->counters.p, snapshot.data(), 8 * C_NUM, hipMemcpyHostToDevice, s));
        GRNG_HIP(hipStreamSynchronize(s));
    }
    bt.tile_pairs += ntp;
}

// Stages IV-VI: sort pairs by row point, list the witness cells of each row
// point (Proposition 3, x side), then the exhaustive lune scan.
//   X: row side (indexed set or query set), S: indexed set (witnesses).
//   cell_filter: cells that may hold witnesses (S.gcount, or new-point counts).
//   zstart: first witness position per cell (Stage VII: the inserted points), or null.
//   cell_rad: radius bound of each cell's witnesses (S.dvor when null; Stage
//     VII passes the bound of the inserted points alone).
void run_exhaustive(grng_index *idx, const Layer &L, const LayerAux &aux, const PointState &X, const PointState &S,
                    Pairs &P, int64_t np, const DevBuf &dmax, const int32_t *cell_filter, const int32_t *zstart,
                    DevBuf &alive, BuildTimes &bt, ExhaustiveState *keep = nullptr,
                    const double *cell_rad = nullptr) {
    const double *crad = cell_rad ? cell_rad : S.dvor.as<double>();
    hipStream_t s = idx->stream;
    const int64_t n = X.n, m = L.m;
    uint64_t *ctr = idx->counters.as<uint64_t>();
    DevBuf roff;
    {
        DevBuf cnt, sx, sy, sd2;
        cnt.alloc(4 * (size_t)std::max<int64_t>(n + 1, 2));
        zero(cnt, s);
        roff.alloc(8 * (size_t)(n + 1));
        sx.alloc(4 * (size_t)std::max<int64_t>(np, 1));
        sy.alloc(4 * (size_t)std::max<int64_t>(np, 1));
        sd2.alloc(8 * (size_t)std::max<int64_t>(np, 1));
        launch_pairs_sort_rows(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), n, cnt.as<int32_t>(),
                               roff.as<int64_t>(), sx.as<int32_t>(), sy.as<int32_t>(), sd2.as<double>());
        P.x = std::move(sx);
        P.y = std::move(sy);
        P.d2 = std::move(sd2);
    }
    const bool f32 = precision(idx) != GRNG_PREC_FP64;
    alive.alloc((size_t)std::max<int64_t>(np, 8));
    // Stage V with the row's other candidates as witnesses: each pair against
    // the nearest partners of its ends in this list (both ends when they are
    // points of one set; a query's or batch point's partners otherwise).  Not
    // in Stage VII, whose pairs are edges no old point can invalidate.
    const bool prekilled = zstart == nullptr && np > 0;
    if (prekilled) {
        DevBuf wid[2], wd2[2];
        const bool self = X.Xh.p == S.Xh.p;
        EventTimer pt(s);
        // One set: a point's partners are in its row and in its column.
        DevBuf ccnt, coff, cx, cy, cd2;
        if (self) {
            ccnt.alloc(4 * (size_t)std::max<int64_t>(n + 1, 2));
            zero(ccnt, s);
            coff.alloc(8 * (size_t)(n + 1));
            cx.alloc(4 * (size_t)np);
            cy.alloc(4 * (size_t)np);
            cd2.alloc(8 * (size_t)np);
            launch_pairs_sort_rows(s, np, P.y.as<int32_t>(), P.x.as<int32_t>(), P.d2.as<double>(), n,
                                   ccnt.as<int32_t>(), coff.as<int64_t>(), cx.as<int32_t>(), cy.as<int32_t>(),
                                   cd2.as<double>());
        }
        // List 0: the 64 nearest partners.  The next 64 only while the last
        // quarter of a list still kills a share of the pairs (their killers
        // then lie deeper: high dimension, large cells).
        uint64_t k0 = 0, d0 = 0;
        for (int depth = 0; depth < kPartnerLists; ++depth) {
            if (depth > 0) {
                uint64_t c[C_NUM];
                read_counters(idx, c);
                const uint64_t kills = c[C_PARTNER_KILLS] - k0, deep = c[C_PARTNER_DEEP] - d0;
                if (trace_on())
                    std::fprintf(stderr, "[grng] partner list %d: %llu kills, %llu by its last quarter\n", depth - 1,
                                 (unsigned long long)kills, (unsigned long long)deep);
                if ((double)deep < kPartnerDeepShare * (double)kills) break;
                k0 = c[C_PARTNER_KILLS];
                d0 = c[C_PARTNER_DEEP];
            } else {
                uint64_t c[C_NUM];
                read_counters(idx, c);
                k0 = c[C_PARTNER_KILLS];
                d0 = c[C_PARTNER_DEEP];
            }
            DevBuf &wi = wid[depth & 1], &wd = wd2[depth & 1];
            const DevBuf &pi = wid[(depth & 1) ^ 1], &pd = wd2[(depth & 1) ^ 1];
            wi.alloc(4 * (size_t)kPartnerWitnesses * (size_t)n);
            wd.alloc(4 * (size_t)kPartnerWitnesses * (size_t)n);
            launch_partner_top(s, n, roff.as<int64_t>(), P.y.as<int32_t>(), P.d2.as<double>(),
                               self ? coff.as<int64_t>() : nullptr, self ? cy.as<int32_t>() : nullptr,
                               self ? cd2.as<double>() : nullptr, depth ? pi.as<int32_t>() : nullptr,
                               depth ? pd.as<float>() : nullptr, wi.as<int32_t>(), wd.as<float>());
            launch_partner_witness(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), idx->dp,
                                   f32 ? S.Xf.as<float>() : nullptr, S.Xh.as<double>(), wi.as<int32_t>(),
                                   wd.as<float>(), self, depth > 0, alive.as<uint8_t>(), ctr);
        }
        const double ms = pt.stop();
        bt.partner += ms;
        trace("Stage V on partner witnesses", ms, np);
    }
    // The rows' witness cells are those of their live pairs.
    DevBuf ldmax;
    const uint64_t *row_dmax = dmax.as<uint64_t>();
    if (prekilled) {
        ldmax.alloc(8 * (size_t)std::max<int64_t>(n, 1));
        launch_live_dmax(s, n, roff.as<int64_t>(), P.d2.as<double>(), alive.as<uint8_t>(), ldmax.as<uint64_t>());
        row_dmax = ldmax.as<uint64_t>();
    }
    DevBuf rel_cnt, rel_off, rel_grp, rel_d2x;
    rel_cnt.alloc(4 * (size_t)n);
    rel_off.alloc(8 * (size_t)(n + 1));
    // Nearest witness cells first, except in Stage VII, whose cells hold only
    // the inserted points (a few each): there the order is pivot order.
    const bool sort = zstart == nullptr;
    launch_relevant_groups(s, n, m, X.perm.as<int32_t>(), X.dxp.as<double>(), crad, cell_filter, row_dmax,
                           nullptr, rel_cnt.as<int32_t>(), nullptr, nullptr, ctr, sort);
    launch_scan_i32_to_i64(s, rel_cnt.as<int32_t>(), n, rel_off.as<int64_t>());
    std::vector<int64_t> tot;
    d2h(tot, rel_off.as<int64_t>() + n, 1, s);
    rel_grp.alloc(4 * (size_t)std::max<int64_t>(tot[0], 1));
    rel_d2x.alloc(8 * (size_t)std::max<int64_t>(tot[0], 1));
    launch_relevant_groups(s, n, m, X.perm.as<int32_t>(), X.dxp.as<double>(), crad, cell_filter, row_dmax,
                           rel_off.as<int64_t>(), rel_cnt.as<int32_t>(), rel_grp.as<int32_t>(), rel_d2x.as<double>(),
                           ctr, sort);
    EventTimer lt(s);
    launch_lune_guided(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), idx->dp, X.Xh.as<double>(),
                       X.nrmh.as<double>(), S.Xh.as<double>(), S.nrmh.as<double>(), S.n, S.dhome.as<double>(),
                       f32 ? X.Xf.as<float>() : nullptr, f32 ? S.Xf.as<float>() : nullptr,
                       f32 ? S.dhomef.as<float>() : nullptr, zstart,
                       S.grp_off.as<int32_t>(), crad, aux.Xp.as<double>(), aux.nrmp.as<double>(),
                       rel_off.as<int64_t>(), rel_grp.as<int32_t>(), rel_d2x.as<double>(), L.rad.as<double>(),
                       idx->opt.witness_order == GRNG_ORDER_LEARNED ? idx->scorer.as<uint16_t>() : nullptr,
                       idx->opt.witness_order == GRNG_ORDER_LUNE, prekilled,
                       alive.as<uint8_t>(), ctr + C_WORK0, ctr);
    const double lms = lt.stop();
    bt.lune += lms;
    trace("exhaustive lune scan", lms, np);
    if (keep) {
        keep->valid = true;
        keep->np = np;
        keep->x = std::move(P.x);
        keep->y = std::move(P.y);
        keep->d2 = std::move(P.d2);
        keep->rel_off = std::move(rel_off);
        keep->rel_grp = std::move(rel_grp);
        keep->rel_d2x = std::move(rel_d2x);
        if (prekilled) {
            keep->row_dmax = std::move(ldmax);
        } else {
            keep->row_dmax.alloc(8 * (size_t)std::max<int64_t>(n, 1));
            GRNG_HIP(hipMemcpyAsync(keep->row_dmax.p, dmax.p, 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
        }
    }
}

void build_rng_guided(grng_index *idx, PointState &ps, LayerAux &aux, DevBuf &edges, int64_t &ne, BuildTimes &bt,
                      ExhaustiveState &ex) {
    const Layer &L = idx->layers.back();
    prepare_aux(idx, L, aux);
    prepare_points(idx, L, aux, idx->X.as<double>(), idx->nrm.as<double>(), idx->n, nullptr, nullptr, ps, bt, true);
    Pairs P;
    DevBuf dmax, alive;
    int64_t np = 0;
    run_pairs(idx, L, aux, ps, ps, PM_SELF, P, dmax, np, bt);
    // The scan is read twice: for the edges now, and later for training samples.
    run_exhaustive(idx, L, aux, ps, ps, P, np, dmax, ps.gcount.as<int32_t>(), nullptr, alive, bt, &ex);
    pairs_to_edges(idx->stream, idx->n, np, ex.x.as<int32_t>(), ex.y.as<int32_t>(), alive.as<uint8_t>(),
                   ps.perm.as<int32_t>(), edges, ne);
}

void fill_build_stats(grng_index *idx, const BuildTimes &bt) {
    uint64_t c[C_NUM];
    read_counters(idx, c);
    idx->stats.ms_vgrng = bt.vgrng;
    idx->stats.ms_pairs = bt.pairs;
    idx->stats.ms_pair_masks = bt.masks;
    idx->stats.ms_lune = bt.lune;
    idx->stats.tile_pairs = bt.tile_pairs;
    idx->stats.unsorted_cell_rows = (int64_t)c[C_UNSORTED];
    idx->stats.vgrng_pivots = idx->layers.empty() ? 0 : vgrng_pivots(idx, idx->layers.back().m);
    idx->stats.stage4_pivots = idx->layers.empty() ? 0 : stage4_pivots(idx);
    idx->stats.ms_autotune = idx->ms_tune;
    idx->stats.distance_computations = (double)c[C_DIST] + bt.host_dist;
    idx->stats.witness_tests = (double)c[C_WTEST];
    idx->stats.candidate_pairs = (double)c[C_CAND];
    idx->stats.stage4_survivors = (double)c[C_S4];
    idx->stats.rechecks = (double)c[C_RECHECK];
    idx->stats.exhaustive_pairs = (double)c[C_SURV];
    idx->stats.lune_tests = (double)c[C_LUNE];
    idx->stats.screen_uncertain = (double)c[C_UNCERTAIN];
    idx->stats.pair_tile_entries = (double)(c[C_PD_TU] + c[C_PD_PIV] + c[C_PD_V]);
    idx->stats.pair_method_distances = (double)(c[C_CAND] + c[C_PD_PIV] + c[C_PD_V]);
    idx->stats.lune_tests_kept = (double)c[C_LUNE_KEPT];
    idx->stats.partner_tests = (double)c[C_PARTNER_TESTS];
    idx->stats.partner_kills = (double)c[C_PARTNER_KILLS];
    idx->stats.ms_partner = bt.partner;
    // Bytes a witness test reads: the witness row and its cell-distance
    // bound (float32 with the float32 screen, float64 otherwise); a test
    // that ends early on a partial sum reads less.
    idx->stats.precision_used = precision(idx);
    idx->stats.lune_bytes = (double)c[C_LUNE] * (precision(idx) == GRNG_PREC_FP64 ? 8.0 * idx->dp + 8.0
                                                                                     : 4.0 * idx->dp + 4.0);
    const double m = idx->layers.empty() ? 0.0 : (double)idx->layers.back().m;
    idx->stats.vgrng_ops = 2.0 * (double)idx->n * m * (double)idx->aux.kw;
    // MFMA flops of the pair kernel: D(T,U) and the two pivot blocks for every
    // tile pair, D(U,U) for those that reach Stage V, D(T,T) each time it is
    // computed (it is kept while consecutive tile pairs share T).
    idx->stats.pairs_flops = 2.0 * idx->dp * ((64.0 * 64.0 + 2.0 * 64.0 * 16.0) * (double)bt.tile_pairs +
                                              64.0 * 64.0 * (double)(c[C_TPV] + c[C_TTV]));
    {
        const int K = stage4_pivots(idx);
        idx->stats.stage4_ops = 2.0 * 64.0 * 64.0 * (double)((K + 3) / 4 * 4) * (double)bt.tile_pairs;
    }
}

// Autotuner: complete guided builds (results discarded), coordinate-wise:
// under GRNG_PREC_AUTO the pair kernel's tile shape (float64 16x16x4 or
// split bf16 16x16x32 MFMA tiles) first, then Proposition 1 witnesses per
// block, then Stage IV pivots; the fastest device time wins.  Every
// candidate gives the same edges, so only speed is compared.
void autotune(grng_index *idx) {
    const int64_t m = idx->layers.back().m;
    auto trial = [&]() {
        EventTimer t(idx->stream);
        PointState ps;
        LayerAux aux;
        ExhaustiveState ex;
        DevBuf edges;
        int64_t ne = 0;
        BuildTimes bt;
        build_rng_guided(idx, ps, aux, edges, ne, bt, ex);
        return t.stop();
    };
    std::vector<int32_t> kws;
    for (int64_t k = 64; k < m && k <= 1024; k *= 2) kws.push_back((int32_t)k);
    if (m <= 2048) kws.push_back((int32_t)m);
    double best = INFINITY, spent = 0;
    if (idx->opt.precision == GRNG_PREC_AUTO) {
        int32_t best_p = GRNG_PREC_FP32;
        for (int32_t p : {GRNG_PREC_FP32, GRNG_PREC_BF16}) {
            idx->tuned_prec = p;
            const double ms = trial();
            spent += ms;
            trace("autotune tile shape", ms, p);
            if (ms < best) { best = ms; best_p = p; }
        }
        idx->tuned_prec = best_p;
    }
    int32_t best_kw = vgrng_pivots(idx, m);
    idx->tuned_k4 = stage4_pivots(idx);
    for (int32_t kw : kws) {
        idx->tuned_kw = kw;
        const double ms = trial();
        spent += ms;
        trace("autotune vgrng_pivots", ms, kw);
        if (ms < best) { best = ms; best_kw = kw; }
    }
    idx->tuned_kw = best_kw;
    int32_t best_k4 = idx->tuned_k4;
    for (int32_t k4 : {8, 12}) {
        idx->tuned_k4 = k4;
        const double ms = trial();
        spent += ms;
        trace("autotune stage4_pivots", ms, k4);
        if (ms < best) { best = ms; best_k4 = k4; }
    }
    idx->tuned_k4 = best_k4;
    idx->ms_tune = spent;
}

void do_build_rng(grng_index *idx) {
    require(idx != nullptr, GRNG_EINVAL, "index is NULL");
    require(idx->opt.witness_order != GRNG_ORDER_LEARNED || idx->scorer.p != nullptr, GRNG_ESTATE,
            "the learned witness order needs grng_set_scorer first");
    if (idx->opt.autotune && idx->tuned_kw == 0 && !idx->layers.empty()) autotune(idx);
    hipStream_t s = idx->stream;
    EventTimer timer(s);
    reset_counters(idx);
    DevBuf edges;
    int64_t ne = 0;
    BuildTimes bt;
    PointState ps;
    LayerAux aux;
    ExhaustiveState ex;
    if (idx->layers.empty()) {
        require(idx->n <= 65535, GRNG_EINVAL, "without a pivot layer build_rng is limited to 65535 points");
        build_rng_brute(idx, edges, ne, bt.lune);
    } else {
        build_rng_guided(idx, ps, aux, edges, ne, bt, ex);
    }
    idx->ex = std::move(ex);
    const double ms = timer.stop();
    idx->edges = std::move(edges);
    idx->nedges = ne;
    idx->ps = std::move(ps);
    idx->aux = std::move(aux);
    idx->rng_built = true;
    idx->stats.n_edges = ne;
    idx->stats.orphans = idx->ps.orphans;
    idx->stats.ms_rng = ms;
    fill_build_stats(idx, bt);
}

// Convert and validate a float32 point batch into exact float64 rows.
double upload_points(grng_index *idx, const float *pts, int64_t count, DevBuf &X, DevBuf &nrm, const char *what) {
    require(pts != nullptr, GRNG_EINVAL, std::string(what) + " pointer is NULL");
    const double km = std::max(grid_validate(idx, pts, count * (int64_t)idx->d, what), idx->kmax);
    check_magnitude(idx, km);
    X.alloc(sizeof(double) * (size_t)(count * idx->dp));
    nrm.alloc(sizeof(double) * (size_t)count);
    launch_to_f64(idx->stream, pts, count, idx->d, idx->dp, X.as<double>(), nrm.as<double>());
    return km;
}

void do_query(grng_index *idx, const float *q, int64_t nq, int64_t *offsets, int32_t *nbrs, int64_t capacity,
              int64_t *needed) {
    require(idx != nullptr && offsets != nullptr && needed != nullptr, GRNG_EINVAL, "NULL argument");
    require(nq >= 1 && nq <= (int64_t)INT32_MAX - 1, GRNG_EINVAL, "nq must be >= 1");
    require(capacity >= 0, GRNG_EINVAL, "capacity must be >= 0");
    require(idx->rng_built, GRNG_ESTATE, "build_rng must run before query_neighbors");
    hipStream_t s = idx->stream;
    EventTimer timer(s);
    reset_counters(idx);
    DevBuf Xq, nq2;
    upload_points(idx, q, nq, Xq, nq2, "queries");
    Pairs P;
    DevBuf alive;
    int64_t np = 0;
    const int32_t *qperm = nullptr, *sperm = nullptr;
    PointState Q;
    BuildTimes bt;
    if (idx->layers.empty()) {
        require(nq <= 65535, GRNG_EINVAL, "without a pivot layer query_neighbors takes at most 65535 queries");
        np = nq * idx->n;
        P.reserve(np);
        zero(P.count, s);
        launch_pairs_all(s, nq, Xq.as<double>(), nq2.as<double>(), idx->n, idx->X.as<double>(), idx->nrm.as<double>(),
                         idx->dp, false, idx->opt.metric, P.view(), idx->counters.as<uint64_t>());
        alive.alloc((size_t)std::max<int64_t>(np, 8));
        EventTimer lt(s);
        launch_lune_all(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), idx->n, idx->dp,
                        Xq.as<double>(), nq2.as<double>(), idx->X.as<double>(), idx->nrm.as<double>(), 0,
                        idx->opt.metric, idx->opt.graph, idx->opt.beta_quarters, idx->opt.grid_exp,
                        alive.as<uint8_t>(), idx->counters.as<uint64_t>());
        bt.lune = lt.stop();
    } else {
        const Layer &L = idx->layers.back();
        PointState &S = idx->ps;
        prepare_points(idx, L, idx->aux, Xq.as<double>(), nq2.as<double>(), nq, &S, nullptr, Q, bt);
        DevBuf dmax;
        run_pairs(idx, L, idx->aux, Q, S, 0, P, dmax, np, bt);
        run_exhaustive(idx, L, idx->aux, Q, S, P, np, dmax, S.gcount.as<int32_t>(), nullptr, alive, bt);
        qperm = Q.perm.as<int32_t>();
        sperm = S.perm.as<int32_t>();
    }
    // CSR per query, neighbours ascending.
    DevBuf deg, fill;
    deg.alloc(4 * (size_t)std::max<int64_t>(nq, 2));
    fill.alloc(4 * (size_t)std::max<int64_t>(nq, 2));
    zero(deg, s);
    zero(fill, s);
    launch_query_csr(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), alive.as<uint8_t>(), qperm, sperm, nq,
                     deg.as<int32_t>(), nullptr, nullptr, nullptr, 0);
    launch_scan_i32_to_i64(s, deg.as<int32_t>(), nq, offsets);
    std::vector<int64_t> tot;
    d2h(tot, offsets + nq, 1, s);
    *needed = tot[0];
    if (tot[0] > capacity) throw Error(GRNG_ECAPACITY, "neighbour buffer too small");
    if (tot[0] > 0) {
        require(nbrs != nullptr, GRNG_EINVAL, "neighbour pointer is NULL");
        launch_query_csr(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), alive.as<uint8_t>(), qperm, sperm, nq,
                         deg.as<int32_t>(), offsets, fill.as<int32_t>(), nbrs, 1);
        launch_sort_segments(s, nq, offsets, nbrs);
    }
    idx->stats.ms_query = timer.stop();
    uint64_t c[C_NUM];
    read_counters(idx, c);
    idx->stats.witness_tests = (double)c[C_WTEST];
    idx->stats.lune_tests = (double)c[C_LUNE];
}

void do_insert(grng_index *idx, const float *pts, int64_t nb) {
    require(idx != nullptr, GRNG_EINVAL, "index is NULL");
    require(nb >= 1, GRNG_EINVAL, "nb must be >= 1");
    require(idx->n + nb <= (int64_t)INT32_MAX - 1, GRNG_EINVAL, "too many points");
    require(idx->rng_built, GRNG_ESTATE, "build_rng must run before insert_batch");
    hipStream_t s = idx->stream;
    EventTimer timer(s);
    reset_counters(idx);
    DevBuf Xb, nrmb;
    const double kmax_new = upload_points(idx, pts, nb, Xb, nrmb, "points");
    const int64_t n0 = idx->n, n1 = n0 + nb;
    const int dp = idx->dp;
    // New point arena: old rows then the batch (ids n0 .. n1-1).
    DevBuf X1, nrm1;
    X1.alloc(sizeof(double) * (size_t)(n1 * dp));
    nrm1.alloc(sizeof(double) * (size_t)n1);
    GRNG_HIP(hipMemcpyAsync(X1.p, idx->X.p, sizeof(double) * (size_t)(n0 * dp), hipMemcpyDeviceToDevice, s));
    GRNG_HIP(hipMemcpyAsync(X1.as<double>() + n0 * dp, Xb.p, sizeof(double) * (size_t)(nb * dp),
                            hipMemcpyDeviceToDevice, s));
    GRNG_HIP(hipMemcpyAsync(nrm1.p, idx->nrm.p, sizeof(double) * (size_t)n0, hipMemcpyDeviceToDevice, s));
    GRNG_HIP(hipMemcpyAsync(nrm1.as<double>() + n0, nrmb.p, sizeof(double) * (size_t)nb, hipMemcpyDeviceToDevice, s));
    DevBuf edges;
    int64_t ne = 0;
    BuildTimes bt;
    PointState ps;
    if (idx->layers.empty()) {
        // Without a pivot layer the insertion is a plain exhaustive rebuild.
        require(n1 <= 65535, GRNG_EINVAL, "without a pivot layer the index is limited to 65535 points");
        std::swap(idx->X, X1);
        std::swap(idx->nrm, nrm1);
        const int64_t n_save = idx->n;
        idx->n = n1;
        try {
            build_rng_brute(idx, edges, ne, bt.lune);
        } catch (...) {
            std::swap(idx->X, X1);
            std::swap(idx->nrm, nrm1);
            idx->n = n_save;
            throw;
        }
    } else {
        const Layer &L = idx->layers.back();
        LayerAux &aux = idx->aux;
        PointState &S = idx->ps;
        const int64_t m = L.m;
        // Localization of the new points (Stages I-VI) against S u B.  A dense
        // batch (at least kDenseBatch points per pivot cell on average) keeps
        // the batch points in their cells' tiles and scans the tile pairs with
        // a batch tile; a sparse one is the row side of its own, with tiles
        // packed across cells.
        constexpr int64_t kDenseBatch = 8;
        const bool dense = nb >= kDenseBatch * m;
        PointState qs;
        DevBuf bd_new, bv_new;
        std::vector<double> newrad;
        bool dxp_moved = false;
        try {
            merge_batch(idx, L, aux, S, Xb.as<double>(), nrmb.as<double>(), nb, dense, ps, qs, bd_new, bv_new,
                        newrad, dxp_moved, bt);
            Pairs Pn;
            DevBuf dmax_n, alive_n;
            int64_t np_n = 0;
            if (dense) {
                run_pairs(idx, L, aux, ps, ps, PM_SELF | PM_NEW_ONLY, Pn, dmax_n, np_n, bt);
                run_exhaustive(idx, L, aux, ps, ps, Pn, np_n, dmax_n, ps.gcount.as<int32_t>(), nullptr, alive_n,
                               bt);
                launch_pairs_to_ids(s, np_n, Pn.x.as<int32_t>(), Pn.y.as<int32_t>(), ps.perm.as<int32_t>(),
                                    ps.perm.as<int32_t>());
            } else {
                std::vector<int32_t> g(qs.h_perm.size());
                for (size_t r = 0; r < g.size(); ++r) g[r] = (int32_t)(n0 + qs.h_perm[r]);
                h2d(qs.gid, g, s);
                run_pairs(idx, L, aux, qs, ps, PM_INSERT, Pn, dmax_n, np_n, bt);
                run_exhaustive(idx, L, aux, qs, ps, Pn, np_n, dmax_n, ps.gcount.as<int32_t>(), nullptr, alive_n,
                               bt);
                launch_pairs_to_ids(s, np_n, Pn.x.as<int32_t>(), Pn.y.as<int32_t>(), qs.gid.as<int32_t>(),
                                    ps.perm.as<int32_t>());
            }
            // Stage VII (Proposition 5): an existing edge survives iff no
            // inserted point lies in its lune; only the inserted points are
            // witnesses (each cell's batch points follow its old ones), so a
            // cell's witness ball is that of its inserted points.
            EventTimer t7(s);
            std::vector<int32_t> newcount((size_t)m), zst((size_t)m);
            for (int64_t c = 0; c < m; ++c) {
                zst[c] = ps.h_off[c] + (S.h_off[c + 1] - S.h_off[c]);
                newcount[c] = ps.h_off[c + 1] - zst[c];
            }
            DevBuf d_newcount, d_zst, d_newrad;
            h2d(d_newcount, newcount, s);
            h2d(d_zst, zst, s);
            h2d(d_newrad, newrad, s);
            const int64_t ne0 = idx->nedges;
            Pairs Po;
            Po.reserve(ne0);
            DevBuf dmax_o, alive_o;
            dmax_o.alloc(8 * (size_t)n1);
            zero(dmax_o, s);
            launch_edges_to_pairs(s, ne0, idx->edges.as<int32_t>(), ps.inv.as<int32_t>(), Po.x.as<int32_t>(),
                                  Po.y.as<int32_t>());
            launch_pair_d2(s, ne0, Po.x.as<int32_t>(), Po.y.as<int32_t>(), dp, ps.Xh.as<double>(),
                           ps.nrmh.as<double>(), Po.d2.as<double>(), dmax_o.as<uint64_t>());
            run_exhaustive(idx, L, aux, ps, ps, Po, ne0, dmax_o, d_newcount.as<int32_t>(), d_zst.as<int32_t>(),
                           alive_o, bt, nullptr, d_newrad.as<double>());
            trace("Stage VII on the old edges", t7.stop(), ne0);
            // Merge: surviving old edges and new edges.
            EventTimer te(s);
            Pairs Pm;
            Pm.reserve(ne0 + np_n);
            DevBuf alive_m;
            alive_m.alloc((size_t)std::max<int64_t>(ne0 + np_n, 8));
            auto cat = [&](DevBuf &dst, const DevBuf &a, const DevBuf &b, size_t el, int64_t na, int64_t nb2) {
                if (na) GRNG_HIP(hipMemcpyAsync(dst.p, a.p, el * (size_t)na, hipMemcpyDeviceToDevice, s));
                if (nb2)
                    GRNG_HIP(hipMemcpyAsync(static_cast<char *>(dst.p) + el * (size_t)na, b.p, el * (size_t)nb2,
                                            hipMemcpyDeviceToDevice, s));
            };
            launch_pairs_to_ids(s, ne0, Po.x.as<int32_t>(), Po.y.as<int32_t>(), ps.perm.as<int32_t>(),
                                ps.perm.as<int32_t>());
            cat(Pm.x, Po.x, Pn.x, 4, ne0, np_n);
            cat(Pm.y, Po.y, Pn.y, 4, ne0, np_n);
            cat(alive_m, alive_o, alive_n, 1, ne0, np_n);
            pairs_to_edges(s, n1, ne0 + np_n, Pm.x.as<int32_t>(), Pm.y.as<int32_t>(), alive_m.as<uint8_t>(),
                           nullptr, edges, ne);
            trace("edge list of the union", te.stop(), ne);
        } catch (...) {
            if (dxp_moved) S.dxp = std::move(ps.dxp);   // its first n0 rows are as they were
            throw;
        }
        idx->ps = std::move(ps);
        std::swap(aux.bd, bd_new);
        std::swap(aux.bv, bv_new);
        idx->ex = ExhaustiveState();   // training samples come from full builds only
        std::swap(idx->X, X1);
        std::swap(idx->nrm, nrm1);
        idx->n = n1;
    }
    const double ms = timer.stop();
    idx->cap = idx->n;
    idx->kmax = kmax_new;
    idx->edges = std::move(edges);
    idx->nedges = ne;
    idx->stats.n_points = idx->n;
    idx->stats.n_edges = ne;
    idx->stats.orphans = idx->ps.orphans;
    idx->stats.ms_insert = ms;
    fill_build_stats(idx, bt);
}

// Pivots added to a built layer: the dynamic pivot layers of the paper
// (Section 2, Stage I promotes a point without parents to a pivot; Section 3
// inserts pivots into a GRNG layer with Stages I-VI and unlinks pivots with
// Stage VII).  The layer's GRNG becomes GRNG(P u B) exactly.  Adding pivots
// can only unlink a pair of old pivots (a new pivot may lie in its
// generalized lune), so the candidates are the old links, tested against the
// new pivots only, and every pair with a new pivot, tested against all.
// Layers stay nested: a pivot added to layer l must already be a pivot of
// every finer layer.  The exemplar RNG does not depend on the pivots; when
// the finest layer changes, the kept per-point state is rebuilt against it.
void do_insert_pivots(grng_index *idx, int32_t layer, const int32_t *pid_dev, const float *rad_dev, int64_t nb) {
    require(idx != nullptr, GRNG_EINVAL, "index is NULL");
    require(pid_dev != nullptr && rad_dev != nullptr, GRNG_EINVAL, "pivot or radius pointer is NULL");
    require(layer >= 0 && layer < (int32_t)idx->layers.size(), GRNG_ESTATE, "no such layer");
    require(nb >= 1, GRNG_EINVAL, "nb must be >= 1");
    hipStream_t s = idx->stream;
    EventTimer timer(s);
    reset_counters(idx);
    const Layer &O = idx->layers[layer];
    const int64_t m0 = O.m, m1 = m0 + nb;
    require(m1 <= idx->n, GRNG_EINVAL, "more pivots than points");
    std::vector<int32_t> nid;
    d2h(nid, pid_dev, (size_t)nb, s);
    for (int64_t t = 0; t < nb; ++t) {
        require(nid[t] >= 0 && nid[t] < idx->n, GRNG_EINVAL, "pivot id out of range");
        require(t == 0 || nid[t] > nid[t - 1], GRNG_EINVAL, "new pivot ids must be strictly ascending");
        require(!std::binary_search(O.pid_host.begin(), O.pid_host.end(), nid[t]), GRNG_EINVAL,
                "a new pivot is already a pivot of this layer");
        for (size_t l = (size_t)layer + 1; l < idx->layers.size(); ++l)
            require(std::binary_search(idx->layers[l].pid_host.begin(), idx->layers[l].pid_host.end(), nid[t]),
                    GRNG_EINVAL, "a pivot added to layer l must be a pivot of every finer layer");
    }
    (void)grid_validate(idx, rad_dev, nb, "radii");
    std::vector<float> nrad;
    d2h(nrad, rad_dev, (size_t)nb, s);
    std::vector<double> orad;
    std::vector<int64_t> oradi;
    d2h(orad, O.rad.p, (size_t)m0, s);
    d2h(oradi, O.radi.p, (size_t)m0, s);
    // Merged pivot list, ascending ids: old position of each (-1: new).
    Layer L;
    L.m = m1;
    L.words = words_of(m1);
    L.pid_host.resize((size_t)m1);
    std::vector<int32_t> oldpos((size_t)m1), newpos;
    std::vector<uint8_t> isnew((size_t)m1, 0);
    std::vector<double> rad_d((size_t)m1);
    std::vector<int64_t> rad_i((size_t)m1);
    for (int64_t a = 0, b = 0, t = 0; t < m1; ++t) {
        if (b >= nb || (a < m0 && O.pid_host[a] < nid[b])) {
            L.pid_host[t] = O.pid_host[a];
            oldpos[t] = (int32_t)a;
            rad_d[t] = orad[a];
            rad_i[t] = oradi[a];
            ++a;
        } else {
            require(nrad[b] >= 0.0f, GRNG_ENOTGRID, "radii must be >= 0");
            L.pid_host[t] = nid[b];
            oldpos[t] = -1;
            isnew[t] = 1;
            newpos.push_back((int32_t)t);
            rad_d[t] = (double)nrad[b];
            rad_i[t] = (int64_t)std::ldexp(rad_d[t], idx->q);
            ++b;
        }
    }
    h2d(L.pid, L.pid_host, s);
    h2d(L.rad, rad_d, s);
    h2d(L.radi, rad_i, s);
    DevBuf Xp, nrmp;
    Xp.alloc(sizeof(double) * (size_t)(m1 * idx->dp));
    nrmp.alloc(sizeof(double) * (size_t)m1);
    launch_gather_rows(s, idx->X.as<double>(), L.pid.as<int32_t>(), m1, idx->dp, Xp.as<double>());
    launch_gather_f64(s, idx->nrm.as<double>(), L.pid.as<int32_t>(), m1, nrmp.as<double>());
    L.dpp2.alloc(sizeof(double) * (size_t)(m1 * m1));
    L.dpp.alloc(sizeof(double) * (size_t)(m1 * m1));
    launch_dist2(s, Xp.as<double>(), nrmp.as<double>(), m1, Xp.as<double>(), nrmp.as<double>(), m1, idx->dp,
                 L.dpp2.as<double>(), m1, true);
    launch_sqrt(s, L.dpp2.as<double>(), L.dpp.as<double>(), m1 * m1);
    // Candidates (old links and pairs with a new pivot); new pivots are the
    // first witnesses, the only ones for old links.
    DevBuf d_oldpos, d_isnew, d_new, cand;
    h2d(d_oldpos, oldpos, s);
    h2d(d_isnew, isnew, s);
    h2d(d_new, newpos, s);
    cand.alloc(sizeof(uint64_t) * (size_t)(m1 * L.words));
    launch_insert_candidates(s, m1, L.words, d_oldpos.as<int32_t>(), O.bits.as<uint64_t>(), O.words,
                             cand.as<uint64_t>());
    L.bits.alloc(sizeof(uint64_t) * (size_t)(m1 * L.words));
    launch_grng_layer(s, m1, L.dpp.as<double>(), L.dpp2.as<double>(), L.rad.as<double>(), L.radi.as<int64_t>(),
                      idx->q, cand.as<uint64_t>(), L.words, d_new.as<int32_t>(), nb, L.bits.as<uint64_t>(),
                      idx->counters.as<uint64_t>(), d_isnew.as<uint8_t>());
    bits_to_edges(s, m1, L.bits, L.words, L.edges, L.nedges);
    // Relative-domain parents (Theorem 2) of this layer and of the next finer one.
    auto parents_of = [&](const Layer &C, const Layer &F, DevBuf &out) {
        std::vector<int32_t> cpos((size_t)C.m);
        for (int64_t t = 0; t < C.m; ++t)
            cpos[t] = (int32_t)(std::lower_bound(F.pid_host.begin(), F.pid_host.end(), C.pid_host[t]) -
                                F.pid_host.begin());
        DevBuf d_cpos;
        h2d(d_cpos, cpos, s);
        out.alloc(sizeof(uint64_t) * (size_t)(F.m * C.words));
        launch_relative_parents(s, C.m, d_cpos.as<int32_t>(), F.dpp2.as<double>(), F.m, C.rad.as<double>(),
                                F.rad.as<double>(), out.as<uint64_t>(), C.words);
    };
    if (layer > 0) parents_of(idx->layers[layer - 1], L, L.parent_bits);
    DevBuf next_parents;
    const bool has_finer = layer + 1 < (int32_t)idx->layers.size();
    if (has_finer) parents_of(L, idx->layers[layer + 1], next_parents);
    // The finest layer changed: per-point state against it.
    const bool finest = !has_finer;
    PointState ps;
    LayerAux aux;
    BuildTimes bt;
    if (finest && idx->rng_built) {
        prepare_aux(idx, L, aux);
        prepare_points(idx, L, aux, idx->X.as<double>(), idx->nrm.as<double>(), idx->n, nullptr, nullptr, ps, bt,
                       true);
    }
    const double ms = timer.stop();
    uint64_t c[C_NUM];
    read_counters(idx, c);
    // Commit.
    idx->layers[layer] = std::move(L);
    if (has_finer) idx->layers[layer + 1].parent_bits = std::move(next_parents);
    if (finest && idx->rng_built) {
        idx->ps = std::move(ps);
        idx->aux = std::move(aux);
        idx->ex = ExhaustiveState();
        idx->stats.orphans = idx->ps.orphans;
    }
    idx->stats.n_layers = (int64_t)idx->layers.size();
    idx->stats.ms_layers = ms;
    idx->stats.witness_tests = (double)c[C_WTEST];
    idx->stats.rechecks = (double)c[C_RECHECK];
}

// Ids of the points without a parent in the finest layer (orphans), ascending.
void do_get_orphans(grng_index *idx, int32_t *ids_dev, int64_t capacity, int64_t *count) {
    require(idx != nullptr && count != nullptr, GRNG_EINVAL, "NULL argument");
    require(capacity >= 0, GRNG_EINVAL, "capacity must be >= 0");
    require(idx->rng_built && !idx->layers.empty(), GRNG_ESTATE, "needs a pivot layer and a built RNG");
    hipStream_t s = idx->stream;
    const PointState &P = idx->ps;
    std::vector<int64_t> off;
    std::vector<int32_t> perm;
    d2h(off, P.par_off.p, (size_t)(P.n + 1), s);
    d2h(perm, P.perm.p, (size_t)P.n, s);
    std::vector<int32_t> ids;
    for (int64_t i = 0; i < P.n; ++i)
        if (off[i + 1] == off[i]) ids.push_back(perm[i]);
    std::sort(ids.begin(), ids.end());
    *count = (int64_t)ids.size();
    if ((int64_t)ids.size() > capacity) throw Error(GRNG_ECAPACITY, "id buffer too small");
    if (!ids.empty()) {
        require(ids_dev != nullptr, GRNG_EINVAL, "id pointer is NULL");
        GRNG_HIP(hipMemcpyAsync(ids_dev, ids.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice, s));
        GRNG_HIP(hipStreamSynchronize(s));
    }
}

void do_get_edges(const grng_index *idx, int32_t layer, int32_t *uv, int64_t capacity, int64_t *num) {
    require(idx != nullptr, GRNG_EINVAL, "index is NULL");
    require(num != nullptr, GRNG_EINVAL, "num_edges pointer is NULL");
    require(capacity >= 0, GRNG_EINVAL, "capacity must be >= 0");
    const DevBuf *src;
    int64_t ne;
    if (layer == -1) {
        require(idx->rng_built, GRNG_ESTATE, "the RNG has not been built");
        src = &idx->edges;
        ne = idx->nedges;
    } else {
        require(layer >= 0 && layer < (int32_t)idx->layers.size(), GRNG_ESTATE, "no such layer");
        src = &idx->layers[layer].edges;
        ne = idx->layers[layer].nedges;
    }
    *num = ne;
    if (ne > capacity) throw Error(GRNG_ECAPACITY, "edge buffer too small");
    if (ne == 0) return;
    require(uv != nullptr, GRNG_EINVAL, "uv pointer is NULL");
    GRNG_HIP(hipMemcpyAsync(uv, src->p, sizeof(int32_t) * 2 * (size_t)ne, hipMemcpyDeviceToDevice, idx->stream));
    // A layer's edges are kept as positions in its pivot list; the caller gets
    // point ids.  Pivot ids ascend, so the mapping keeps the canonical order.
    if (layer >= 0) launch_map_ids(idx->stream, 2 * ne, uv, idx->layers[layer].pid.as<int32_t>());
    GRNG_HIP(hipStreamSynchronize(idx->stream));
}

// ---------------------------------------------------------------------------
// Learned witness-cell ranking.

void do_mlp_grad(const float *theta, const float *feats, const uint8_t *labels, int64_t n, float *grad,
                 float *loss_host, void *stream) {
    require(theta && feats && labels && grad && loss_host, GRNG_EINVAL, "NULL argument");
    require(n >= 1, GRNG_EINVAL, "n must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf scratch, lbuf;
    lbuf.alloc(8);
    launch_mlp_grad(s, theta, feats, labels, n, grad, lbuf.as<float>(), scratch);
    std::vector<float> h;
    d2h(h, lbuf.p, 1, s);
    *loss_host = h[0];
}

void do_mlp_train(float *theta, const float *feats, const uint8_t *labels, int64_t n, int32_t steps, float lr,
                  float *loss_host, void *stream) {
    require(theta && feats && labels && loss_host, GRNG_EINVAL, "NULL argument");
    require(n >= 1 && steps >= 1 && lr > 0.f, GRNG_EINVAL, "n, steps and lr must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf scratch, g, m, v, lbuf;
    g.alloc(4 * kMlpParams);
    m.alloc(4 * kMlpParams);
    v.alloc(4 * kMlpParams);
    lbuf.alloc(8);
    zero(m, s);
    zero(v, s);
    for (int32_t t = 1; t <= steps; ++t) {
        launch_mlp_grad(s, theta, feats, labels, n, g.as<float>(), lbuf.as<float>(), scratch);
        launch_adam(s, theta, g.as<float>(), m.as<float>(), v.as<float>(), t, lr);
    }
    launch_mlp_grad(s, theta, feats, labels, n, g.as<float>(), lbuf.as<float>(), scratch);
    std::vector<float> h;
    d2h(h, lbuf.p, 1, s);
    *loss_host = h[0];
}

void do_mlp_score(const float *theta, const float *feats, int64_t n, float *scores, void *stream) {
    require(theta != nullptr, GRNG_EINVAL, "NULL argument");
    require(n >= 0, GRNG_EINVAL, "n must be >= 0");
    require(n == 0 || (feats && scores), GRNG_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf wb;
    wb.alloc(2 * kMlpParams);
    launch_pack_bf16(s, theta, wb.as<uint16_t>());
    launch_mlp_score(s, wb.as<uint16_t>(), feats, n, scores);
    GRNG_HIP(hipStreamSynchronize(s));
}

void do_log_cells(grng_index *idx, int64_t max_pairs, float *feats, uint8_t *labels, int64_t capacity,
                  int64_t *count) {
    require(idx && count, GRNG_EINVAL, "NULL argument");
    require(max_pairs >= 0 && capacity >= 0, GRNG_EINVAL, "sizes must be >= 0");
    require(idx->rng_built && !idx->layers.empty() && idx->ex.valid, GRNG_ESTATE,
            "needs a build_rng with a pivot layer");
    hipStream_t s = idx->stream;
    const ExhaustiveState &ex = idx->ex;
    const PointState &ps = idx->ps;
    const int64_t nsamp = std::min(max_pairs, ex.np);
    if (capacity > 0) require(feats && labels, GRNG_EINVAL, "NULL sample buffers");
    *count = launch_log_cells(s, nsamp, ex.np, ex.x.as<int32_t>(), ex.y.as<int32_t>(), ex.d2.as<double>(), idx->dp,
                              ps.Xh.as<double>(), ps.nrmh.as<double>(), ps.grp_off.as<int32_t>(),
                              ps.dvor.as<double>(), idx->layers.back().rad.as<double>(), idx->aux.Xp.as<double>(),
                              idx->aux.nrmp.as<double>(), ex.rel_off.as<int64_t>(), ex.rel_grp.as<int32_t>(),
                              ex.rel_d2x.as<double>(), ex.row_dmax.as<uint64_t>(), feats, labels, capacity);
    if (*count > capacity) throw Error(GRNG_ECAPACITY, "sample buffer too small");
}

void do_set_scorer(grng_index *idx, const float *theta) {
    require(idx && theta, GRNG_EINVAL, "NULL argument");
    DevBuf wb;
    wb.alloc(2 * kMlpParams);
    launch_pack_bf16(idx->stream, theta, wb.as<uint16_t>());
    GRNG_HIP(hipStreamSynchronize(idx->stream));
    idx->scorer = std::move(wb);
}

// Device blocks an index keeps cached between calls.
constexpr size_t kPoolKeep = size_t(8) << 30;

// Makes the index's block pool the current one for the duration of a call
// and trims its cache when the call ends.
struct PoolScope {
    grng_index *idx;
    BlockPool *saved;
    explicit PoolScope(grng_index *i) : idx(i), saved(g_pool) { g_pool = i ? &i->pool : nullptr; }
    ~PoolScope() {
        if (idx) idx->pool.trim(kPoolKeep);
        g_pool = saved;
    }
};

template <class F>
grng_status guarded(F &&f) {
    try {
        arm_failure_injection();
        f();
        return GRNG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GRNG_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GRNG_EDEVICE;
    } catch (...) {
        g_last_error = "unknown failure";
        return GRNG_EDEVICE;
    }
}

}  // namespace

thread_local BlockPool *g_pool = nullptr;

namespace {

size_t size_class(size_t n) {
    size_t c = n < 256 ? 256 : n;
    size_t pw = 256;
    while (pw < c) pw <<= 1;
    if (pw <= (size_t(2) << 20)) return pw;
    const size_t g = pw >> 3;   // eighths of the power of two: at most 12.5% slack
    return (c + g - 1) / g * g;
}

void *device_malloc(size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

}  // namespace

BlockPool::~BlockPool() { trim(0); }

void *BlockPool::get(size_t bytes, size_t *cls) {
    *cls = size_class(bytes);
    auto it = free_.find(*cls);
    if (it != free_.end()) {
        void *p = it->second;
        free_.erase(it);
        cached_ -= *cls;
        return p;
    }
    void *p = device_malloc(*cls);
    if (!p && cached_) {   // give the cache back and try once more
        trim(0);
        p = device_malloc(*cls);
    }
    if (!p) throw Error(GRNG_ENOMEM, "device allocation of " + std::to_string(*cls) + " bytes failed");
    return p;
}

void BlockPool::put(void *p, size_t cls) {
    free_.emplace(cls, p);
    cached_ += cls;
}

void BlockPool::trim(size_t keep) {
    while (cached_ > keep && !free_.empty()) {
        auto it = std::prev(free_.end());
        (void)hipFree(it->second);
        cached_ -= it->first;
        free_.erase(it);
    }
}

void DevBuf::alloc(size_t nbytes) {
    release();
    nbytes = (nbytes + 7) & ~size_t(7);
    if (nbytes == 0) nbytes = 8;
    ++g_alloc_calls;
    if (fail_at() > 0 && g_alloc_calls == fail_at())
        throw Error(GRNG_ENOMEM, "device allocation failed (injected by GRNG_FAIL_ALLOC_AT)");
    if (g_pool) {
        size_t cls = 0;
        p = g_pool->get(nbytes, &cls);
        bytes = cls;
        pool = g_pool;
        return;
    }
    p = device_malloc(nbytes);
    if (!p) throw Error(GRNG_ENOMEM, "device allocation of " + std::to_string(nbytes) + " bytes failed");
    bytes = nbytes;
}

void DevBuf::ensure(size_t nbytes) {
    if (bytes < nbytes) alloc(nbytes);
}

}  // namespace grng

using namespace grng;

extern "C" {

int32_t grng_abi_version(void) { return GRNG_ABI_VERSION; }

const char *grng_last_error(void) { return g_last_error.c_str(); }

grng_status grng_create(grng_index **out, const float *points_dev, int64_t n, int32_t d, void *stream,
                        const grng_options *opt) {
    return guarded([&] { do_create(out, points_dev, n, d, stream, opt); });
}

grng_status grng_build_grng_layer(grng_index *idx, int32_t layer, const int32_t *pivot_ids_dev,
                                  const float *radii_dev, int64_t m) {
    return guarded([&] {
        PoolScope ps(idx);
        do_build_layer(idx, layer, pivot_ids_dev, radii_dev, m);
    });
}

grng_status grng_build_rng(grng_index *idx) {
    return guarded([&] {
        PoolScope ps(idx);
        do_build_rng(idx);
    });
}

grng_status grng_insert_batch(grng_index *idx, const float *points_dev, int64_t nb) {
    return guarded([&] {
        PoolScope ps(idx);
        do_insert(idx, points_dev, nb);
    });
}

grng_status grng_insert_pivots(grng_index *idx, int32_t layer, const int32_t *pivot_ids_dev, const float *radii_dev,
                               int64_t nb) {
    return guarded([&] {
        PoolScope ps(idx);
        do_insert_pivots(idx, layer, pivot_ids_dev, radii_dev, nb);
    });
}

grng_status grng_get_orphans(grng_index *idx, int32_t *ids_dev, int64_t capacity, int64_t *count) {
    return guarded([&] {
        PoolScope ps(idx);
        do_get_orphans(idx, ids_dev, capacity, count);
    });
}

grng_status grng_query_neighbors(grng_index *idx, const float *q_dev, int64_t nq, int64_t *offsets_dev,
                                 int32_t *nbrs_dev, int64_t capacity, int64_t *needed) {
    return guarded([&] {
        PoolScope ps(idx);
        do_query(idx, q_dev, nq, offsets_dev, nbrs_dev, capacity, needed);
    });
}

int32_t grng_mlp_params(void) { return kMlpParams; }

grng_status grng_mlp_grad(const float *theta_dev, const float *feats_dev, const uint8_t *labels_dev, int64_t n,
                          float *grad_dev, float *loss, void *stream) {
    return guarded([&] { do_mlp_grad(theta_dev, feats_dev, labels_dev, n, grad_dev, loss, stream); });
}

grng_status grng_mlp_grad_noalloc(const float *theta_dev, const float *feats_dev, const uint8_t *labels_dev,
                                  int64_t n, float *grad_dev, float *loss_dev, void *stream) {
    return guarded([&] {
        require(theta_dev && feats_dev && labels_dev && grad_dev && loss_dev, GRNG_EINVAL, "NULL argument");
        launch_mlp_grad_noalloc(static_cast<hipStream_t>(stream), theta_dev, feats_dev, labels_dev, n, grad_dev,
                                loss_dev);
    });
}

grng_status grng_mlp_train(float *theta_dev, const float *feats_dev, const uint8_t *labels_dev, int64_t n,
                           int32_t steps, float lr, float *loss, void *stream) {
    return guarded([&] { do_mlp_train(theta_dev, feats_dev, labels_dev, n, steps, lr, loss, stream); });
}

grng_status grng_mlp_score(const float *theta_dev, const float *feats_dev, int64_t n, float *scores_dev,
                           void *stream) {
    return guarded([&] { do_mlp_score(theta_dev, feats_dev, n, scores_dev, stream); });
}

grng_status grng_log_witness_cells(grng_index *idx, int64_t max_pairs, float *feats_dev, uint8_t *labels_dev,
                                   int64_t capacity, int64_t *count) {
    return guarded([&] {
        PoolScope ps(idx);
        do_log_cells(idx, max_pairs, feats_dev, labels_dev, capacity, count);
    });
}

grng_status grng_set_scorer(grng_index *idx, const float *theta_dev) {
    return guarded([&] {
        PoolScope ps(idx);
        do_set_scorer(idx, theta_dev);
    });
}

grng_status grng_get_edges(const grng_index *idx, int32_t layer, int32_t *uv_dev, int64_t capacity,
                           int64_t *num_edges) {
    return guarded([&] { do_get_edges(idx, layer, uv_dev, capacity, num_edges); });
}

grng_status grng_get_stats(const grng_index *idx, grng_stats *out) {
    return guarded([&] {
        require(idx != nullptr && out != nullptr, GRNG_EINVAL, "NULL argument");
        *out = idx->stats;
    });
}

void grng_destroy(grng_index *idx) {
    if (!idx) return;
    if (idx->stream) (void)hipStreamSynchronize(idx->stream);
    delete idx;
}

}  // extern "C"
