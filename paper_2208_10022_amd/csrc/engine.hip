// Host engine and C ABI of the gfx950 exact RNG / GRNG library (see include/grng.h).
//
// Every step of the build runs in the library's own kernels on the caller's
// stream; the host only validates arguments, sizes buffers, performs the
// counting sort that orders points by home cell, and moves small arrays.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "common.h"

namespace grng {

namespace {

thread_local std::string g_last_error;
int64_t g_alloc_calls = 0;
int64_t g_fail_at = -2;   // -2: not read yet; -1: disabled

int64_t fail_at() {
    if (g_fail_at == -2) {
        const char *e = std::getenv("GRNG_FAIL_ALLOC_AT");
        g_fail_at = e ? std::atoll(e) : -1;
    }
    return g_fail_at;
}

constexpr int kDefaultK = kPivWitness;

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
    require(o->precision >= GRNG_PREC_FP64 && o->precision <= GRNG_PREC_BF16, GRNG_EINVAL, "unknown precision");
    require(o->witness_order == GRNG_ORDER_DISTANCE || o->witness_order == GRNG_ORDER_LEARNED, GRNG_EINVAL,
            "unknown witness order");
    require(o->stage4_pivots >= 0 && o->stage4_pivots <= kPivWitness, GRNG_EINVAL, "stage4_pivots must be in [0, 16]");
    require(o->reserved_i[0] == 0 && o->reserved_i[1] == 0, GRNG_EINVAL, "reserved option fields must be 0");
    for (int t = 0; t < 4; ++t) require(o->reserved[t] == 0, GRNG_EINVAL, "reserved option fields must be 0");
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
    DevBuf dmax;
    dmax.alloc(8 * (size_t)n);
    launch_pairs_all(s, n, idx->dp, idx->X.as<double>(), idx->nrm.as<double>(), P.view(), dmax.as<uint64_t>(),
                     idx->counters.as<uint64_t>());
    const int64_t np = n * (n - 1) / 2;
    DevBuf alive;
    alive.alloc((size_t)std::max<int64_t>(np, 8));
    EventTimer lt(s);
    launch_lune_all(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), n, idx->dp,
                    idx->X.as<double>(), idx->nrm.as<double>(), alive.as<uint8_t>(), idx->counters.as<uint64_t>());
    ms_lune = lt.stop();
    pairs_to_edges(s, n, np, P.x.as<int32_t>(), P.y.as<int32_t>(), alive.as<uint8_t>(), nullptr, edges, ne);
}

struct BuildTimes {
    double vgrng = 0, pairs = 0, lune = 0;
    int64_t tile_pairs = 0;
};

void build_rng_guided(grng_index *idx, PointState &ps, DevBuf &edges, int64_t &ne, BuildTimes &bt) {
    hipStream_t s = idx->stream;
    const Layer &L = idx->layers.back();
    const int64_t n = idx->n, m = L.m;
    const int dp = idx->dp;
    const int32_t words = L.words;
    const int32_t K = idx->opt.stage4_pivots > 0 ? idx->opt.stage4_pivots : kDefaultK;
    uint64_t *ctr = idx->counters.as<uint64_t>();
    // A1: exact point-pivot distances (MFMA f64 tiles), original order [n][m].
    DevBuf Xp, nrmp, dxp;
    Xp.alloc(sizeof(double) * (size_t)(m * dp));
    nrmp.alloc(sizeof(double) * (size_t)m);
    launch_gather_rows(s, idx->X.as<double>(), L.pid.as<int32_t>(), m, dp, Xp.as<double>());
    launch_gather_f64(s, idx->nrm.as<double>(), L.pid.as<int32_t>(), m, nrmp.as<double>());
    dxp.alloc(sizeof(double) * (size_t)(n * m));
    launch_dist2(s, idx->X.as<double>(), idx->nrm.as<double>(), n, Xp.as<double>(), nrmp.as<double>(), m, dp,
                 dxp.as<double>(), m, true);
    // A2: parents count, home cell, cell radius.
    DevBuf home, d2home, npar, d2vor, gcount;
    home.alloc(4 * (size_t)n);
    d2home.alloc(8 * (size_t)n);
    npar.alloc(4 * (size_t)n);
    d2vor.alloc(8 * (size_t)m);
    gcount.alloc(4 * (size_t)m);
    zero(d2vor, s);
    zero(gcount, s);
    launch_point_pass1(s, n, m, dxp.as<double>(), L.rad.as<double>(), home.as<int32_t>(), d2home.as<double>(),
                       npar.as<int32_t>());
    launch_group_radius(s, n, home.as<int32_t>(), d2home.as<double>(), d2vor.as<uint64_t>(), gcount.as<int32_t>());
    // Home order: stable counting sort by home cell (host; O(n)).
    std::vector<int32_t> h_home, h_npar, h_gcount;
    std::vector<double> h_d2home, h_d2vor;
    d2h(h_home, home.p, (size_t)n, s);
    d2h(h_npar, npar.p, (size_t)n, s);
    d2h(h_d2home, d2home.p, (size_t)n, s);
    d2h(h_gcount, gcount.p, (size_t)m, s);
    d2h(h_d2vor, d2vor.p, (size_t)m, s);
    std::vector<int32_t> off((size_t)m + 1, 0), perm((size_t)n), home_h((size_t)n);
    for (int64_t c = 0; c < m; ++c) off[c + 1] = off[c] + h_gcount[c];
    {
        std::vector<int32_t> pos(off.begin(), off.end() - 1);
        for (int64_t x = 0; x < n; ++x) perm[pos[h_home[x]]++] = (int32_t)x;
    }
    std::vector<int64_t> par_off((size_t)n + 1, 0);
    std::vector<double> dhome((size_t)n), dvor((size_t)m);
    int64_t orphans = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t x = perm[i];
        home_h[i] = h_home[x];
        par_off[i + 1] = par_off[i] + h_npar[x];
        dhome[i] = std::sqrt(h_d2home[x]) * (1.0 + 1e-15);   // upper bound of d(x, p_home)
        orphans += h_npar[x] == 0;
    }
    for (int64_t c = 0; c < m; ++c) dvor[c] = std::sqrt(h_d2vor[c]) * (1.0 + 1e-15);
    ps.n = n;
    ps.orphans = orphans;
    h2d(ps.perm, perm, s);
    h2d(ps.home, home_h, s);
    h2d(ps.grp_off, off, s);
    h2d(ps.par_off, par_off, s);
    h2d(ps.dhome, dhome, s);
    h2d(ps.dvor, dvor, s);
    ps.inv.alloc(4 * (size_t)n);
    launch_iota_inverse(s, ps.perm.as<int32_t>(), n, ps.inv.as<int32_t>());
    ps.Xh.alloc(sizeof(double) * (size_t)(n * dp));
    ps.nrmh.alloc(sizeof(double) * (size_t)n);
    launch_gather_rows(s, idx->X.as<double>(), ps.perm.as<int32_t>(), n, dp, ps.Xh.as<double>());
    launch_gather_f64(s, idx->nrm.as<double>(), ps.perm.as<int32_t>(), n, ps.nrmh.as<double>());
    // Parents and virtual-pivot GRNG bitsets (Propositions 1-2) as a tiled
    // (min, max) product of point-pivot and shifted pivot-pivot distances.
    DevBuf bd, bv;
    bd.alloc(4 * (size_t)(m * m));
    bv.alloc(4 * (size_t)(m * m));
    ps.par_idx.alloc(4 * (size_t)std::max<int64_t>(par_off[n], 1));
    ps.g_rows.alloc(8 * (size_t)(n * words));
    ps.v_rows.alloc(8 * (size_t)(n * words));
    {
        EventTimer vt(s);
        launch_point_pass2(s, n, m, ps.perm.as<int32_t>(), dxp.as<double>(), L.rad.as<double>(), L.dpp.as<double>(),
                           ps.dvor.as<double>(), gcount.as<int32_t>(), L.bits.as<uint64_t>(), words,
                           ps.par_off.as<int64_t>(), ps.par_idx.as<int32_t>(), bd.as<float>(), bv.as<float>(),
                           ps.g_rows.as<uint64_t>(), ps.v_rows.as<uint64_t>(), ctr);
        bt.vgrng = vt.stop();
    }
    const int64_t nw = div_up(n, 64);
    ps.g_cols.alloc(8 * (size_t)(m * nw));
    ps.v_cols.alloc(8 * (size_t)(m * nw));
    launch_bits_transpose(s, ps.g_rows.as<uint64_t>(), n, words, m, ps.g_cols.as<uint64_t>());
    launch_bits_transpose(s, ps.v_rows.as<uint64_t>(), n, words, m, ps.v_cols.as<uint64_t>());
    // Tiles: chunks of <= 64 home-order points of one cell; tile pairs whose
    // cells survive each other's virtual-pivot test (Stage II with cell radii).
    std::vector<int32_t> tiles;
    for (int64_t c = 0; c < m; ++c)
        for (int32_t st = off[c]; st < off[c + 1]; st += 64) {
            tiles.push_back(st);
            tiles.push_back(std::min<int32_t>(64, off[c + 1] - st));
            tiles.push_back((int32_t)c);
        }
    const int64_t ntiles = (int64_t)tiles.size() / 3;
    DevBuf d_tiles, tv, tcnt, toff, tpT, tpU, pknn;
    h2d(d_tiles, tiles, s);
    tv.alloc(8 * (size_t)(ntiles * words));
    launch_tile_vmask(s, ntiles, d_tiles.as<int32_t>(), ps.v_rows.as<uint64_t>(), words, tv.as<uint64_t>());
    tcnt.alloc(4 * (size_t)ntiles);
    toff.alloc(8 * (size_t)(ntiles + 1));
    launch_tile_pairs(s, ntiles, d_tiles.as<int32_t>(), tv.as<uint64_t>(), words, nullptr, tcnt.as<int32_t>(), nullptr,
                      nullptr);
    launch_scan_i32_to_i64(s, tcnt.as<int32_t>(), ntiles, toff.as<int64_t>());
    std::vector<int64_t> ntp_h;
    d2h(ntp_h, toff.as<int64_t>() + ntiles, 1, s);
    const int64_t ntp = ntp_h[0];
    tpT.alloc(4 * (size_t)std::max<int64_t>(ntp, 1));
    tpU.alloc(4 * (size_t)std::max<int64_t>(ntp, 1));
    launch_tile_pairs(s, ntiles, d_tiles.as<int32_t>(), tv.as<uint64_t>(), words, toff.as<int64_t>(),
                      tcnt.as<int32_t>(), tpT.as<int32_t>(), tpU.as<int32_t>());
    pknn.alloc(4 * (size_t)(m * kPivWitness));
    launch_pivot_knn(s, m, L.dpp2.as<double>(), pknn.as<int32_t>());
    // Stages I-V over the tile pairs -> pairs left for the exhaustive scan.
    Pairs P;
    DevBuf dmax;
    dmax.alloc(8 * (size_t)n);
    int64_t cap = std::max<int64_t>(1 << 22, 64 * n);
    int64_t np = 0;
    std::vector<uint64_t> snapshot;
    d2h(snapshot, idx->counters.p, C_NUM, s);
    for (int attempt = 0; attempt < 3; ++attempt) {
        P.reserve(cap);
        zero(P.count, s);
        zero(dmax, s);
        EventTimer pt(s);
        launch_pairs_tiled(s, ntp, tpT.as<int32_t>(), tpU.as<int32_t>(), d_tiles.as<int32_t>(), dp, ps.Xh.as<double>(),
                           ps.nrmh.as<double>(), ps.par_off.as<int64_t>(), ps.par_idx.as<int32_t>(),
                           ps.v_rows.as<uint64_t>(), ps.g_cols.as<uint64_t>(), words, nw, pknn.as<int32_t>(), K,
                           Xp.as<double>(), nrmp.as<double>(), P.view(), dmax.as<uint64_t>(), ctr + C_WORK0, ctr);
        bt.pairs = pt.stop();
        bt.tile_pairs = ntp;
        std::vector<uint64_t> h;
        d2h(h, P.count.p, 1, s);
        np = (int64_t)h[0];
        if (np <= cap) break;
        require(attempt < 2, GRNG_EDEVICE, "survivor count changed between identical passes");
        // Rerun with room for every survivor, from the counters as they were.
        cap = np;
        GRNG_HIP(hipMemcpyAsync(idx->counters.p, snapshot.data(), 8 * C_NUM, hipMemcpyHostToDevice, s));
        GRNG_HIP(hipStreamSynchronize(s));
    }
    // Witness cells per row point (Proposition 3, x side), sorted by distance.
    DevBuf rel_cnt, rel_off, rel_grp, rel_d2x;
    rel_cnt.alloc(4 * (size_t)n);
    rel_off.alloc(8 * (size_t)(n + 1));
    launch_relevant_groups(s, n, m, ps.perm.as<int32_t>(), dxp.as<double>(), ps.dvor.as<double>(),
                           gcount.as<int32_t>(), dmax.as<uint64_t>(), nullptr, rel_cnt.as<int32_t>(), nullptr,
                           nullptr);
    launch_scan_i32_to_i64(s, rel_cnt.as<int32_t>(), n, rel_off.as<int64_t>());
    std::vector<int64_t> tot;
    d2h(tot, rel_off.as<int64_t>() + n, 1, s);
    rel_grp.alloc(4 * (size_t)std::max<int64_t>(tot[0], 1));
    rel_d2x.alloc(8 * (size_t)std::max<int64_t>(tot[0], 1));
    launch_relevant_groups(s, n, m, ps.perm.as<int32_t>(), dxp.as<double>(), ps.dvor.as<double>(),
                           gcount.as<int32_t>(), dmax.as<uint64_t>(), rel_off.as<int64_t>(), rel_cnt.as<int32_t>(),
                           rel_grp.as<int32_t>(), rel_d2x.as<double>());
    // Order the survivors by row point: neighbouring pairs then share their
    // witness cells, which the lune kernel keeps in one XCD's L2.
    {
        DevBuf cnt, roff, sx, sy, sd2;
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
    // Stages IV-VI: exhaustive lune test of the survivors.
    DevBuf alive;
    alive.alloc((size_t)std::max<int64_t>(np, 8));
    EventTimer lt(s);
    launch_lune_guided(s, np, P.x.as<int32_t>(), P.y.as<int32_t>(), P.d2.as<double>(), dp, ps.Xh.as<double>(),
                       ps.nrmh.as<double>(), ps.dhome.as<double>(), ps.grp_off.as<int32_t>(), ps.dvor.as<double>(),
                       Xp.as<double>(), nrmp.as<double>(), rel_off.as<int64_t>(), rel_grp.as<int32_t>(),
                       rel_d2x.as<double>(), alive.as<uint8_t>(), ctr + C_WORK0, ctr);
    bt.lune = lt.stop();
    pairs_to_edges(s, n, np, P.x.as<int32_t>(), P.y.as<int32_t>(), alive.as<uint8_t>(), ps.perm.as<int32_t>(), edges,
                   ne);
}

void do_build_rng(grng_index *idx) {
    require(idx != nullptr, GRNG_EINVAL, "index is NULL");
    hipStream_t s = idx->stream;
    EventTimer timer(s);
    reset_counters(idx);
    DevBuf edges;
    int64_t ne = 0;
    BuildTimes bt;
    PointState ps;
    if (idx->layers.empty()) {
        require(idx->n <= 65535, GRNG_EINVAL, "without a pivot layer build_rng is limited to 65535 points");
        build_rng_brute(idx, edges, ne, bt.lune);
    } else {
        build_rng_guided(idx, ps, edges, ne, bt);
    }
    const double ms = timer.stop();
    uint64_t c[C_NUM];
    read_counters(idx, c);
    idx->edges = std::move(edges);
    idx->nedges = ne;
    idx->ps = std::move(ps);
    idx->rng_built = true;
    idx->stats.n_edges = ne;
    idx->stats.orphans = idx->ps.orphans;
    idx->stats.ms_rng = ms;
    idx->stats.ms_vgrng = bt.vgrng;
    idx->stats.ms_pairs = bt.pairs;
    idx->stats.ms_lune = bt.lune;
    idx->stats.tile_pairs = bt.tile_pairs;
    {
        const double m = idx->layers.empty() ? 0.0 : (double)idx->layers.back().m;
        idx->stats.vgrng_ops = 2.0 * (double)idx->n * m * m;
        idx->stats.pairs_flops = 2.0 * idx->dp * (64.0 * 64.0 + 2.0 * 64.0 * 16.0) * (double)bt.tile_pairs;
    }
    idx->stats.distance_computations = (double)c[C_DIST];
    idx->stats.witness_tests = (double)c[C_WTEST];
    idx->stats.candidate_pairs = (double)c[C_CAND];
    idx->stats.stage4_survivors = (double)c[C_S4];
    idx->stats.rechecks = (double)c[C_RECHECK];
    idx->stats.exhaustive_pairs = (double)c[C_SURV];
    idx->stats.lune_tests = (double)c[C_LUNE];
    idx->stats.lune_bytes = (double)c[C_LUNE] * (8.0 * idx->dp + 16.0);
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
    GRNG_HIP(hipStreamSynchronize(idx->stream));
}

template <class F>
grng_status guarded(F &&f) {
    try {
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

void DevBuf::alloc(size_t nbytes) {
    release();
    nbytes = (nbytes + 7) & ~size_t(7);
    if (nbytes == 0) nbytes = 8;
    ++g_alloc_calls;
    if (fail_at() >= 0 && g_alloc_calls == fail_at())
        throw Error(GRNG_ENOMEM, "device allocation failed (injected by GRNG_FAIL_ALLOC_AT)");
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Error(GRNG_ENOMEM, "device allocation of " + std::to_string(nbytes) + " bytes failed");
    }
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
    return guarded([&] { do_build_layer(idx, layer, pivot_ids_dev, radii_dev, m); });
}

grng_status grng_build_rng(grng_index *idx) {
    return guarded([&] { do_build_rng(idx); });
}

grng_status grng_insert_batch(grng_index *idx, const float *points_dev, int64_t nb) {
    return guarded([&] {
        require(idx != nullptr && points_dev != nullptr, GRNG_EINVAL, "NULL argument");
        require(nb >= 1, GRNG_EINVAL, "nb must be >= 1");
        throw Error(GRNG_ESTATE, "insert_batch is not available in this build");
    });
}

grng_status grng_query_neighbors(grng_index *idx, const float *q_dev, int64_t nq, int64_t *offsets_dev,
                                 int32_t *nbrs_dev, int64_t capacity, int64_t *needed) {
    return guarded([&] {
        require(idx != nullptr && q_dev != nullptr && offsets_dev != nullptr && needed != nullptr, GRNG_EINVAL,
                "NULL argument");
        (void)nq;
        (void)nbrs_dev;
        (void)capacity;
        throw Error(GRNG_ESTATE, "query_neighbors is not available in this build");
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
