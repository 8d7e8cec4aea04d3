// Exemplar-RNG kernels: candidate pairs and the lune-emptiness test.
//
// Pair (x, y) is an RNG edge iff no point z has max(d(x,z), d(y,z)) < d(x,y)
// (Section 1, RNG definition; ties keep the edge).  Squared distances are
// exact float64 values (grid contract), so each lune predicate below is the
// exact decision.  Pruning follows Section 2:
//   Stages I-III  pair kept only if every domain parent of y is in the
//                 virtual-pivot GRNG of x and vice versa (Theorem 1 and
//                 Propositions 1-2), and if the home cells of x and y survive
//                 the same virtual-pivot test with cell radii;
//   Stage IV      pivots as witnesses;
//   Stage V       the points of the pair's two tiles as witnesses, then the
//                 nearest other candidates of each end (partner pass);
//   Stage VI      exhaustive scan over points grouped by home cell, skipping a
//                 whole cell when max(d(x,p), d(y,p)) - radius(p) >= d(x,y)
//                 (Proposition 3) and a single point z of the cell when
//                 max(d(x,p), d(y,p)) - d(z,p) >= d(x,y) or d(z,p) -
//                 min(d(x,p), d(y,p)) >= d(x,y) (Proposition 4, both sides of
//                 the triangle inequality).  These skips use square roots, so
//                 they are taken only with a safety margin (pruning less only
//                 costs work).
//
// Layout: points in home order (grouped by nearest pivot), coordinates as
// zero-padded float64 rows of dp values and their exact float32 copies.
// Stages I-III run in k_pair_masks (one wave per 64 x 64 tile pair, writing
// a record); Stages IV-V in k_pairs_tiled (one workgroup per tile pair at a
// time, tiles in LDS), the partner pass in k_partner_top / k_partner_witness
// (64 partner witnesses per wave); Stage VI in k_lune_guided (one wave per
// surviving pair, 64 lanes streaming witnesses, a wave ballot ends the scan
// at the first witness).
#include <algorithm>

#include "common.h"
#include "dev_util.h"

namespace grng {

namespace {

constexpr int kMaxDp = 128;      // largest padded dimension kept in LDS per wave

__device__ inline double dot_lds(const double *__restrict__ a_lds, const double *__restrict__ b, int dp) {
    double acc = 0.0;
    for (int t = 0; t < dp; t += 2) {
        const double2 bv = *reinterpret_cast<const double2 *>(b + t);
        acc = fma(a_lds[t], bv.x, acc);
        acc = fma(a_lds[t + 1], bv.y, acc);
    }
    return acc;
}

__device__ inline double sqrt_lo(double v) { return sqrt(v) * (1.0 - 1e-15); }
__device__ inline double sqrt_hi(double v) { return sqrt(v) * (1.0 + 1e-15); }

// "a - b >= c" certainly, for non-negative a, b, c given as bounds.
__device__ inline bool surely_ge(double a_lo, double b_hi, double c_hi) {
    return a_lo - b_hi >= c_hi + 1e-13 * (a_lo + b_hi + c_hi);
}

__device__ inline void wave_append(PairList out, bool keep, int32_t x, int32_t y, double d2) {
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(keep);
    if (!m) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long *)out.count, (unsigned long long)__popcll(m));
    base = __shfl(base, 0, kWave);
    if (keep) {
        const uint64_t slot = base + __popcll(m & ((1ull << lane) - 1ull));
        if ((int64_t)slot < out.cap) {
            out.x[slot] = x;
            out.y[slot] = y;
            out.d2[slot] = d2;
        }
    }
}

// ---------------------------------------------------------------------------
// Candidate pairs guided by the pivot layer (Stages I-V), tiled.
//
// Points are split into tiles: chunks of at most 64 consecutive home-order
// points of one home cell.  Tile pairs (T, U), T <= U, whose cells survive
// each other's virtual-pivot test are listed; for the 64 x 64 pairs
// (x in T, y in U):
//   * Stages I-III as bit masks (k_pair_masks): P(x) within GRNG(y) and P(y)
//     within GRNG(x) from the transposed virtual-pivot bitsets, and the cell
//     bits of both;
//   * exact d^2(x, y) from an f64 MFMA tile (16x16x4 blocks, operands in LDS);
//   * Stage IV: the pivots nearest to the two cells as witnesses, with exact
//     d^2 to the pivots from two more MFMA tiles;
//   * Stage V: the 128 points of T and U as witnesses.  The in-tile distance
//     matrices D(T,U), D(T,T), D(U,U) are exact f64 MFMA results rounded to
//     nearest float32 and kept in LDS.  With u = 2^-24 each stored value is
//     within a factor (1 +- u) of the exact one, and max/min of rounded
//     values are the rounded max/min, so fl(max(d^2(x,z), d^2(y,z))) <
//     fl(d^2(x,y)) * (1 - 2^-21) (itself rounded) proves the exact strict
//     inequality: (1+u)^3 (1 - 8u) < 1.  The same certificate ends a pair in
//     Stage IV.  A pair whose only witnesses are too close to call survives
//     to the exact scan, so no edge depends on rounding.
// Survivors go to the global pair list for the exhaustive scan.
__device__ inline uint64_t bits_at(const uint64_t *row, int64_t start, int len) {
    // 64 bits of a bit row starting at bit `start` (bits past len are don't-care)
    const int64_t w = start >> 6;
    const int sh = (int)(start & 63);
    uint64_t v = row[w] >> sh;
    if (sh && ((start + len - 1) >> 6) > w) v |= row[w + 1] << (64 - sh);
    return v;
}

// Proposition 2 for one point x against a 64-point range of the other set:
// bit k is set iff every parent p of x has bit start + k set in its column
// g_cols[p] (p in GRNG(y)).  Parents are taken four at a time, so their ids
// and then their words are all in flight together.
__device__ inline uint64_t parents_mask(const int64_t *__restrict__ par_off, const int32_t *__restrict__ par_idx,
                                        const uint64_t *__restrict__ g_cols, int32_t nw, int64_t x, int64_t start,
                                        int len) {
    uint64_t mk = ~0ull;
    const int64_t q1 = par_off[x + 1];
    for (int64_t q = par_off[x]; q < q1 && mk; q += 4) {
        int32_t p[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = q + k < q1 ? par_idx[q + k] : -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (p[k] >= 0) mk &= bits_at(g_cols + (int64_t)p[k] * nw, start, len);
    }
    return mk;
}

// LDS of k_pairs_tiled for padded dimension dp.  After Stage IV the pivot
// rows and pivot distances are dead, and D(U,U) reuses them.  D(T,T) has
// bytes of its own when they fit, so that it is kept while consecutive tile
// pairs share T (the list is sorted by T); otherwise it reuses them too.
// The Stage V witness matrices D(T,T) and D(U,U) hold float32 entries, or
// 16-bit upper bounds (h16) where that halves their bytes enough for two
// workgroups per CU.
constexpr int kDh = kTile + 2;   // row stride (16-bit entries) of the 16-bit witness matrices
__host__ __device__ inline size_t pairs_wmat_bytes(bool h16) {
    return h16 ? 2 * (size_t)kTile * kDh : 4 * (size_t)kTile * kDl;
}
__host__ __device__ inline size_t pairs_lds_phase_a(int dp) {
    return 8 * (size_t)kPiv * (dp + 1) + 4 * 2 * (size_t)kTile * kXs;
}
__host__ __device__ inline size_t pairs_lds_fixed(int dp) {
    const size_t ld = (size_t)dp + 1;
    return 8 * (2 * kTile * ld + 2 * kTile + kPiv + 3 * kTile) + 4 * (size_t)kTile * kDl;
}
__host__ __device__ inline bool pairs_keep_tt(int dp, bool h16) {
    const size_t dmat = pairs_wmat_bytes(h16), pa = pairs_lds_phase_a(dp);
    return pairs_lds_fixed(dp) + dmat + (pa > dmat ? pa : dmat) <= 160 * 1024 - 256;
}
__host__ __device__ inline size_t pairs_lds_bytes(int dp, bool h16) {
    const size_t dmat = pairs_wmat_bytes(h16), pa = pairs_lds_phase_a(dp);
    return pairs_lds_fixed(dp) +
           (pairs_keep_tt(dp, h16) ? dmat + (pa > dmat ? pa : dmat) : (pa > 2 * dmat ? pa : 2 * dmat));
}
// Two 8-wave workgroups per CU need each at most half of the 160 KiB of LDS
// (allocated in 512-byte granules, with the kernel's static bytes).
inline bool pairs_two_per_cu(size_t lds) { return 2 * ((lds + 64 + 511) / 512 * 512) <= 160 * 1024; }

// Witness-matrix entries: float32, or the upper 16 bits of the float32 bit
// pattern rounded up (an upper bound with 8 significant bits; non-negative
// values only, whose bit patterns order as unsigned integers).
__device__ inline void put_wmat(float *p, double v) { *p = (float)v; }
__device__ inline void put_wmat(uint16_t *p, double v) {
    const uint32_t b = __float_as_uint(__double2float_ru(v));
    *p = (uint16_t)((b + 0xffffu) >> 16);
}
__device__ inline float get_wmat(const float *p) { return *p; }
__device__ inline float get_wmat(const uint16_t *p) { return __uint_as_float((uint32_t)*p << 16); }

// Rows [0, rows) of a tile into LDS (row stride ld doubles), zero rows past
// len; spread over nthr threads (t = this thread's index among them), four
// threads per row, 16-byte loads.
__device__ inline void load_rows(double *dst, const double *__restrict__ src, int len, int rows, int dp, int ld,
                                 int t, int nthr) {
    for (int r = t >> 2; r < rows; r += nthr >> 2) {
        for (int c = 2 * (t & 3); c < dp; c += 8) {
            double2 v = {0.0, 0.0};
            if (r < len) v = *reinterpret_cast<const double2 *>(src + (int64_t)r * dp + c);
            dst[r * ld + c] = v.x;
            dst[r * ld + c + 1] = v.y;
        }
    }
}

constexpr int kPairThreads = 512;   // 8 waves per tile pair
constexpr int kPairWaves = kPairThreads / 64;

// One wave, NB independent 16x16 blocks of |a_i - b_j|^2 at once: exact f64
// MFMA results rounded to nearest float32 (the MFMA chains interleave, so the
// matrix unit is not idle on dependences).
template <int NB, typename OT>
__device__ inline void dist_blocks(const double *const sa[NB], const double *const na[NB], const double *const sb[NB],
                                   const double *const nb[NB], const int r0[NB], const int c0[NB], int dp, int ld,
                                   OT *const D[NB], const int dld[NB]) {
    const int lane = threadIdx.x & 63, il = lane & 15, kl = lane >> 4;
    v4d acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < dp; kk += 4) {
        double av[NB], bv[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            av[q] = sa[q][(r0[q] + il) * ld + kk + kl];
            bv[q] = sb[q][(c0[q] + il) * ld + kk + kl];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc[q], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
        for (int r = 0; r < 4; ++r) {
            const int i = r0[q] + 4 * r + kl, j = c0[q] + il;
            put_wmat(&D[q][i * dld[q] + j], na[q][i] + nb[q][j] - 2.0 * acc[q][r]);
        }
}

// Stages I-III for the tile pairs [tp0, tp0 + n): one wave per tile pair
// writes its record (kPairRecWords words): the tiles' start, length and home
// cell, the Stage IV pivot witnesses, then the candidate masks of the rows
// of T (bit j: y = U[j] passes Theorem 1 and Propositions 1-2 from x's side)
// and of the rows of U (bit i: the same from y's side).  A pair (i, j) is a
// candidate when both bits are set.  Only dependent gathers here; the pair
// kernel then starts each tile pair from one streamed record.
__global__ __launch_bounds__(256) void k_pair_masks(int64_t tp0, int64_t n, const int32_t *__restrict__ tpT,
                                                    const int32_t *__restrict__ tpU, PointsView A, PointsView B,
                                                    int mode, int32_t words, const int32_t *__restrict__ pknn,
                                                    int32_t K, uint64_t *__restrict__ rec) {
    const int lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n) return;   // the whole wave
    const bool self = (mode & PM_SELF) != 0;
    const int32_t T = tpT[tp0 + k], U = tpU[tp0 + k];
    const int32_t sT = A.tiles[3 * T], lT = A.tiles[3 * T + 1], a = A.tiles[3 * T + 2];
    const int32_t sU = B.tiles[3 * U], lU = B.tiles[3 * U + 1], b = B.tiles[3 * U + 2];
    uint64_t *r = rec + k * kPairRecWords;
    const int i = lane;
    // rows of T.  Pairs need P(x) within GRNG(y) (bits of the y side).
    // Insertion: drop y = the row point's own copy, and a batch point y
    // paired with a batch row point of larger or equal id (that pair is
    // produced once, from the other side).
    uint64_t ins = 0, newU = ~0ull;
    if (mode & PM_NEW_ONLY) newU = __ballot(i < lU && B.is_new[sU + i]);
    if (mode & PM_INSERT) {
        const int32_t gy = i < lU ? B.gid[sU + i] : -1;
        const int32_t gx = i < lT ? A.gid[sT + i] : -1;
        for (int t = 0; t < 64; ++t) {
            const int32_t gxt = __shfl(gx, t, kWave);   // every lane takes part in the shuffle
            const uint64_t m = __ballot(gy >= B.new_from && gy <= gxt);
            if (i == t) ins = m;
        }
    }
    uint64_t mx = 0, my = 0;
    if (i < lT) {
        const int64_t x = sT + i;
        mx = parents_mask(A.par_off, A.par_idx, B.g_cols, B.nw, x, sU, lU);
        mx &= ((A.v_rows[x * words + (b >> 6)] >> (b & 63)) & 1ull) ? ~0ull : 0ull;
        if (self && T == U) mx &= i == 63 ? 0ull : (~0ull << (i + 1));   // y > x inside one tile
        mx &= ~ins;
        if ((mode & PM_NEW_ONLY) && !A.is_new[x]) mx &= newU;   // a batch point on one side
        mx &= lU == 64 ? ~0ull : ((1ull << lU) - 1ull);
    }
    if (i < lU) {
        const int64_t y = sU + i;
        // The cell test needs the row points inside the cell ball of a:
        // true for indexed points, not for queries.
        my = parents_mask(B.par_off, B.par_idx, A.g_cols, A.nw, y, sT, lT);
        if (self) my &= ((B.v_rows[y * words + (a >> 6)] >> (a & 63)) & 1ull) ? ~0ull : 0ull;
    }
    r[kPairRecMeta + i] = mx;
    r[kPairRecMeta + kTile + i] = my;
    if (lane < 3) {
        const int32_t lo = lane == 0 ? sT : lane == 1 ? a : sU, hi = lane == 0 ? lT : lane == 1 ? lU : b;
        r[lane] = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    } else if (lane < 3 + kPiv / 2) {
        // Stage IV pivot witnesses: the K nearest pivots of cell a (a == b),
        // else about half from each cell; slots past K repeat a's first
        const int ka = (a == b) ? K : (K + 1) / 2;
        int32_t pv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = 2 * (lane - 3) + h;
            pv[h] = t < ka ? pknn[a * kPiv + t] : (t < K ? pknn[b * kPiv + (t - ka)] : pknn[a * kPiv]);
        }
        r[lane] = ((uint64_t)(uint32_t)pv[1] << 32) | (uint32_t)pv[0];
    }
}

template <typename WT>   // witness-matrix entry: float, or uint16_t upper bounds
__global__ __launch_bounds__(kPairThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs_tiled(
    int64_t ntp, const uint64_t *__restrict__ rec, const double *__restrict__ XA, const double *__restrict__ nrmA,
    const double *__restrict__ XB, const double *__restrict__ nrmB, int mode, int dp, int32_t K,
    const double *__restrict__ Xp, const double *__restrict__ nrmp, PairList out,
    unsigned long long *dmax_bits, unsigned long long *work, unsigned long long *counters) {
    // LDS: rows of T and U (ld = dp + 1 doubles per row), norms, candidate
    // masks, the 64 x 64 bit mask of Stage IV survivors, D(T,U), D(T,T); then
    // either the pivot rows and pivot distances (Stages I-IV) or D(U,U)
    // (Stage V) in the same bytes (for dp > 96 D(T,T) shares them too).
    extern __shared__ __align__(16) double lds[];   // 16-byte loads of rows and distance tiles
    const int ld = dp + 1;
    double *sX = lds, *sY = sX + kTile * ld;
    double *nX = sY + kTile * ld, *nY = nX + kTile, *nP = nY + kTile;
    uint64_t *mX = (uint64_t *)(nP + kPiv), *mY = mX + kTile, *surv = mY + kTile;
    float *DTU = (float *)(surv + kTile);
    constexpr bool h16 = sizeof(WT) == 2;
    constexpr int wld = h16 ? kDh : kDl;   // row stride of D(T,T) and D(U,U)
    const size_t wbytes = pairs_wmat_bytes(h16);
    unsigned char *region = (unsigned char *)(DTU + kTile * kDl);
    const bool keep_tt = pairs_keep_tt(dp, h16);
    WT *DTT = (WT *)region;
    unsigned char *region2 = keep_tt ? region + wbytes : region;
    double *sP = (double *)region2;
    float *XP = (float *)(sP + kPiv * ld), *YP = XP + kTile * kXs;
    WT *DUU = (WT *)(keep_tt ? region2 : region + wbytes);
    int32_t tt_start = -1, sx_start = -1;   // tiles whose D(T,T) / rows are in LDS (block-uniform)
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const bool self = (mode & PM_SELF) != 0;
    uint32_t ncand = 0, ns4 = 0, nsurv = 0, ntpv = 0, nttv = 0;
    uint64_t ndist = 0, dtu = 0, dpv = 0, dv = 0;   // tile entries computed (thread 0)
    WaveOut wo;
    // Claims alternate between two sets of slots (iteration parity): thread
    // 0 claims the next tile pair during Stage IV of the current one, so the
    // loop needs no barrier of its own.  The record words before the masks
    // (tiles' start, length and cell, pivot ids) are fetched one tile pair
    // ahead, so that no wave waits on the record before loading rows.
    __shared__ int64_t s_tp[2], s_nx;
    __shared__ uint64_t s_cm[2][kPairRecMeta], s_nm[kPairRecMeta];
    __shared__ int s_any[2];
    const int xcd0 = blockIdx.x % kXcds;
    int xr = 0;
    int64_t cur = 0, cend = 0, nxt = -2;   // thread 0: the claimed chunk; the tile pair after the current one
    auto next_tp = [&]() -> int64_t {
        if (cur >= cend && !claim_chunk(ntp, kPairChunk, xcd0, xr, work, &cur, &cend)) {
            cur = cend = -1;
            return -1;
        }
        return cur++;
    };
    uint64_t nmeta = 0;   // lanes 0-11 of wave 0: a word of the next tile pair's record
    // Thread 0: the tile pair of parity q is the one claimed ahead (nxt),
    // whose record words are in s_nm; claim the one after it.
    auto claim = [&](int q) {
        s_tp[q] = nxt;
        if (nxt >= 0)
            for (int k = 0; k < kPairRecMeta; ++k) s_cm[q][k] = s_nm[k];
        nxt = nxt >= 0 ? next_tp() : -1;
        s_nx = nxt;
        s_any[q] = 0;
    };
    if (tid == 0) {
        nxt = next_tp();
        if (nxt >= 0)
            for (int k = 0; k < kPairRecMeta; ++k) s_nm[k] = rec[nxt * kPairRecWords + k];
        claim(0);
    }
    __syncthreads();
    for (int par = 0;; par ^= 1) {
        const int64_t tp = uniform_i64(s_tp[par]);
        if (tp < 0) break;
        const uint64_t *rc = rec + tp * kPairRecWords;
        const uint64_t m0 = s_cm[par][0], m1 = s_cm[par][1], m2 = s_cm[par][2];
        // (the two home cells, in the low half of m1 and the high half of m2,
        // are not needed here)
        const int32_t sT = (int32_t)m0, lT = (int32_t)(m0 >> 32);
        const int32_t lU = (int32_t)(m1 >> 32), sU = (int32_t)m2;
        // 1. candidate masks and norms (waves 6, 7), rows of T (threads
        // 0-255) and U (256-511), pivot rows (wave 5).
        if (w == 6) {
            nX[lane] = lane < lT ? nrmA[sT + lane] : 0.0;
            mX[lane] = rc[kPairRecMeta + lane];
            surv[lane] = 0;
        } else if (w == 7) {
            nY[lane] = lane < lU ? nrmB[sU + lane] : 0.0;
            mY[lane] = rc[kPairRecMeta + kTile + lane];
        } else if (w == 5) {
            const int t = lane >> 2;
            const int32_t pv = (int32_t)(s_cm[par][3 + (t >> 1)] >> (32 * (t & 1)));
            for (int c = 2 * (lane & 3); c < dp; c += 8) {
                const double2 v = *reinterpret_cast<const double2 *>(Xp + (int64_t)pv * dp + c);
                sP[t * ld + c] = v.x;
                sP[t * ld + c + 1] = v.y;
            }
            if ((lane & 3) == 0) nP[t] = nrmp[pv];
        }
        const bool newT = sT != sx_start;   // T's rows stay in LDS while T repeats
        sx_start = sT;
        if (tid < 256) {
            if (newT) load_rows(sX, XA + (int64_t)sT * dp, lT, kTile, dp, ld, tid, 256);
        } else {
            load_rows(sY, XB + (int64_t)sU * dp, lU, kTile, dp, ld, tid - 256, 256);
        }
        __syncthreads();
        // The next tile pair's record words, in flight until Stage IV ends.
        if (tid < kPairRecMeta) {
            const int64_t nx = s_nx;
            if (nx >= 0) nmeta = rec[nx * kPairRecWords + tid];
        }
        // 2a. Per wave: one 16-row block of d^2 to the pivot witnesses (rows
        // of T for waves 0-3, of U for 4-7; +inf past K) and two 16x16 blocks
        // of D(T,U); three interleaved MFMA f64 chains, float32 results.
        {
            const bool ys = w >= 4;
            const int pr = (w & 3) * 16;
            const int id0 = 2 * w, id1 = 2 * w + 1;
            const double *sa[3] = {ys ? sY : sX, sX, sX};
            const double *na[3] = {ys ? nY : nX, nX, nX};
            const double *sb[3] = {sP, sY, sY};
            const double *nb[3] = {nP, nY, nY};
            const int r0[3] = {pr, (id0 >> 2) * 16, (id1 >> 2) * 16};
            const int c0[3] = {0, (id0 & 3) * 16, (id1 & 3) * 16};
            float *D[3] = {ys ? YP : XP, DTU, DTU};
            const int dld[3] = {kXs, kDl, kDl};
            dist_blocks<3, float>(sa, na, sb, nb, r0, c0, dp, ld, D, dld);
            if ((lane & 15) >= K) {   // unused pivot slots never witness
                float *Pd = ys ? YP : XP;
                for (int r = 0; r < 4; ++r) Pd[(pr + 4 * r + (lane >> 4)) * kXs + (lane & 15)] = INFINITY;
            }
        }
        __syncthreads();
        // 2b. Stages I-IV for all 64 x 64 pairs: thread = rows ty + 16k
        // (k < 4) x columns tx, tx + 32.  C = min over pivots of max(d^2(x,p),
        // d^2(y,p)) as a (min,max) product over LDS rows; a candidate dies
        // when C < d^2(x,y) * (1 - 2^-21) in float32, which proves a pivot
        // witness.
        {
            // All operands are non-negative float32 values or +inf, whose bit
            // patterns order as unsigned integers: integer min/max (three-input
            // min) need no NaN handling.
            const int tx = tid & 31, ty = tid >> 5;
            uint32_t c[4][2];
#pragma unroll
            for (int r = 0; r < 4; ++r) c[r][0] = c[r][1] = kInfBits;
#pragma unroll
            for (int t0 = 0; t0 < kPiv; t0 += 4) {
                if (t0 >= K) break;
                uint4 xv[4], yv[2];
#pragma unroll
                for (int r = 0; r < 4; ++r) xv[r] = *reinterpret_cast<const uint4 *>(XP + (ty + 16 * r) * kXs + t0);
#pragma unroll
                for (int q = 0; q < 2; ++q) yv[q] = *reinterpret_cast<const uint4 *>(YP + (tx + 32 * q) * kXs + t0);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        c[r][q] = umin3(c[r][q], umax2(xv[r].x, yv[q].x), umax2(xv[r].y, yv[q].y));
                        c[r][q] = umin3(c[r][q], umax2(xv[r].z, yv[q].z), umax2(xv[r].w, yv[q].w));
                    }
            }
            const uint64_t my0 = mY[tx], my1 = mY[tx + 32];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ty + 16 * r;
                const uint64_t mxi = mX[i];
                uint64_t bits = 0;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int j = tx + 32 * q;
                    const bool cand = ((mxi >> j) & 1ull) && (((q ? my1 : my0) >> i) & 1ull);
                    ncand += cand;
                    if (cand && !(c[r][q] < __float_as_uint(DTU[i * kDl + j] * kCertain))) bits |= 1ull << j;
                }
                if (bits) {
                    ns4 += __popcll(bits);
                    atomicOr((unsigned long long *)&surv[i], (unsigned long long)bits);
                    s_any[par] = 1;
                }
            }
        }
        // The next tile pair's record words, then its claim (thread 0, same
        // wave, in program order), before the barrier that ends Stage IV.
        if (tid < kPairRecMeta) s_nm[tid] = nmeta;
        if (tid == 0) claim(par ^ 1);
        __syncthreads();
        if (tid == 0) {
            dtu += (uint64_t)lT * (uint64_t)lU;
            dpv += (uint64_t)(lT + lU) * (uint64_t)K;
        }
        if (!s_any[par]) continue;   // uniform: no Stage IV survivor in this tile pair
        ntpv += tid == 0;
        // 2c. D(U,U), written over the pivot data, which is dead now, and
        // D(T,T) when T's points may witness and it is not in LDS already:
        // then waves 0-3 take D(T,T) and waves 4-7 D(U,U), four interleaved
        // blocks each; else all eight waves take D(U,U), two blocks each.
        {
            const bool need_tt = self && sT != tt_start;
            if (need_tt && keep_tt) tt_start = sT;
            nttv += need_tt && tid == 0;
            if (tid == 0) dv += (uint64_t)lU * lU + (need_tt ? (uint64_t)lT * lT : 0);
            const bool us = !need_tt || w >= 4;
            const int nh = need_tt ? 2 : 1;
            const double *sa[2], *na[2];
            int r0[2], c0[2], dld[2] = {wld, wld};
            WT *D[2];
            for (int h = 0; h < nh; ++h) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int id = need_tt ? 4 * (w & 3) + 2 * h + q : 2 * w + q;
                    sa[q] = us ? sY : sX;
                    na[q] = us ? nY : nX;
                    r0[q] = (id >> 2) * 16;
                    c0[q] = (id & 3) * 16;
                    D[q] = us ? DUU : DTT;
                }
                dist_blocks<2, WT>(sa, na, sa, na, r0, c0, dp, ld, D, dld);
            }
        }
        __syncthreads();
        // 3. Stage V: each wave walks rows w, w+8, ...; every Stage IV survivor
        // (i, j) is tested against the points of T and U, one lane per witness
        // z, with the float32 certificate above (16-bit witness-matrix entries
        // are upper bounds of the exact values, so a kill stays a proof).
        for (int i = w; i < lT; i += kPairWaves) {
            uint64_t row = surv[i];
            if (!row) continue;
            // the x side of every test of this row, once per row
            const float ax = (self && lane < lT) ? get_wmat(&DTT[i * wld + lane]) : INFINITY;
            const float au = lane < lU ? DTU[i * kDl + lane] : INFINITY;
            double rmax = -1.0;
            while (row) {
                const int j = __ffsll((long long)row) - 1;
                row &= row - 1;
                const float t = DTU[i * kDl + j] * kCertain;
                const float by = (self && lane < lT) ? DTU[lane * kDl + j] : INFINITY;
                const float bu = lane < lU ? get_wmat(&DUU[j * wld + lane]) : INFINITY;
                if (__ballot((ax < t && by < t) || (au < t && bu < t))) continue;   // max(., .) < t
                // survivor: exact d^2, the dot product spread over the lanes
                // (every partial sum is exact, so the order does not matter)
                double part = 0.0;
                for (int c = lane; c < dp; c += 64) part = fma(sX[i * ld + c], sY[j * ld + c], part);
                for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
                const double dd = nX[i] + nY[j] - 2.0 * part;
                if (lane == wo.cnt) {
                    wo.x = sT + i;
                    wo.y = sU + j;
                    wo.d2 = dd;
                }
                rmax = fmax(rmax, dd);
                ++nsurv;
                if (++wo.cnt == 64) wo.flush(out);
            }
            if (rmax >= 0.0 && lane == 0)
                atomicMax(&dmax_bits[sT + i], (unsigned long long)__double_as_longlong(rmax));
        }
        __syncthreads();
    }
    wo.flush(out);
    ncand = wave_sum(ncand);
    ns4 = wave_sum(ns4);
    if (lane == 0) {
        // witness tests: K pivot tests per candidate (Stage IV), 64 or 128
        // in-tile tests per Stage IV survivor (Stage V)
        const uint64_t tests = (uint64_t)ncand * (uint64_t)K + (uint64_t)ns4 * (self ? 128u : 64u);
        atomicAdd(&counters[C_CAND], (unsigned long long)ncand);
        atomicAdd(&counters[C_S4], (unsigned long long)ns4);
        atomicAdd(&counters[C_WTEST], (unsigned long long)tests);
        atomicAdd(&counters[C_SURV], (unsigned long long)nsurv);
        if (ntpv) atomicAdd(&counters[C_TPV], (unsigned long long)ntpv);
        if (nttv) atomicAdd(&counters[C_TTV], (unsigned long long)nttv);
        if (w == 0) {
            ndist = dtu + dpv + dv;
            atomicAdd(&counters[C_DIST], (unsigned long long)ndist);
            atomicAdd(&counters[C_PD_TU], (unsigned long long)dtu);
            atomicAdd(&counters[C_PD_PIV], (unsigned long long)dpv);
            atomicAdd(&counters[C_PD_V], (unsigned long long)dv);
        }
    }
}

// Counting sort of the pair list by row point (stable within a row is not
// needed: the lune verdict of a pair does not depend on its position).
// Pairs arrive in runs of equal row point (a tile pair's survivors row by
// row): each run of lanes with one row point takes its slots with a single
// atomic, so that a row with thousands of pairs is not one contended counter.
// run_start: bit l set iff lane l starts a run (its row differs from lane l-1's).
__device__ inline uint64_t run_starts(int32_t x) {
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(x, 1, 64);
    return __ballot(lane == 0 || prev != x);
}

__global__ void k_pairs_count_rows(int64_t np, const int32_t *px, int32_t *cnt) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int32_t x = p < np ? px[p] : -1;
    const uint64_t st = run_starts(x);
    if (x < 0 || !((st >> lane) & 1ull)) return;
    const uint64_t later = lane == 63 ? 0ull : st & (~0ull << (lane + 1));
    const int end = later ? __ffsll((long long)later) - 1 : 64;
    atomicAdd(&cnt[x], end - lane);
}

__global__ void k_pairs_scatter_rows(int64_t np, const int32_t *px, const int32_t *py, const double *pd2,
                                     const int64_t *off, int32_t *fill, int32_t *ox, int32_t *oy, double *od2) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int32_t x = p < np ? px[p] : -1;
    const uint64_t st = run_starts(x);
    const uint64_t later = lane == 63 ? 0ull : st & (~0ull << (lane + 1));
    const int end = later ? __ffsll((long long)later) - 1 : 64;
    int32_t base = 0;
    if (x >= 0 && ((st >> lane) & 1ull)) base = atomicAdd(&fill[x], end - lane);
    const uint64_t upto = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
    const int first = 63 - __clzll((long long)(st & upto));   // the lane that starts this lane's run
    base = __shfl(base, first, 64);
    if (x < 0) return;
    const int64_t s = off[x] + base + (lane - first);
    ox[s] = x;
    oy[s] = py[p];
    od2[s] = pd2[p];
}

// Few rows (an insertion batch or a query set): each workgroup counts its
// chunk of pairs in an LDS histogram and takes its slots in every row with
// one global atomic per row.
constexpr int kRowsLdsMax = 8192;    // rows of the LDS histogram (32 KB)
constexpr int kSortPer = 16;         // pairs per thread
__global__ __launch_bounds__(1024) void k_pairs_count_rows_lds(int64_t np, const int32_t *px, int64_t n,
                                                               int32_t *cnt) {
    extern __shared__ int32_t hist[];
    const int tid = threadIdx.x;
    for (int64_t r = tid; r < n; r += 1024) hist[r] = 0;
    __syncthreads();
    const int64_t lo = blockIdx.x * (int64_t)(1024 * kSortPer);
    for (int u = 0; u < kSortPer; ++u) {
        const int64_t p = lo + (int64_t)u * 1024 + tid;
        if (p < np) atomicAdd(&hist[px[p]], 1);
    }
    __syncthreads();
    for (int64_t r = tid; r < n; r += 1024)
        if (hist[r]) atomicAdd(&cnt[r], hist[r]);
}

__global__ __launch_bounds__(1024) void k_pairs_scatter_rows_lds(int64_t np, const int32_t *px, const int32_t *py,
                                                                 const double *pd2, int64_t n, const int64_t *off,
                                                                 int32_t *fill, int32_t *ox, int32_t *oy,
                                                                 double *od2) {
    extern __shared__ int32_t hist[];
    const int tid = threadIdx.x;
    for (int64_t r = tid; r < n; r += 1024) hist[r] = 0;
    __syncthreads();
    const int64_t lo = blockIdx.x * (int64_t)(1024 * kSortPer);
    int32_t slot[kSortPer];
#pragma unroll
    for (int u = 0; u < kSortPer; ++u) {
        const int64_t p = lo + (int64_t)u * 1024 + tid;
        slot[u] = p < np ? atomicAdd(&hist[px[p]], 1) : 0;
    }
    __syncthreads();
    for (int64_t r = tid; r < n; r += 1024)
        if (hist[r]) hist[r] = atomicAdd(&fill[r], hist[r]);   // the chunk's first slot in row r
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSortPer; ++u) {
        const int64_t p = lo + (int64_t)u * 1024 + tid;
        if (p >= np) continue;
        const int32_t x = px[p];
        const int64_t s = off[x] + hist[x] + slot[u];
        ox[s] = x;
        oy[s] = py[p];
        od2[s] = pd2[p];
    }
}

// Tile bookkeeping: OR of the cell bits of a tile's points; tile pairs whose
// cells survive each other's virtual-pivot test; nearest pivots of each pivot.
__global__ void k_tile_vmask(int64_t ntiles, const int32_t *tiles, const uint64_t *v_rows, int32_t words,
                             uint64_t *tv) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= ntiles * words) return;
    const int64_t t = e / words;
    const int32_t wd = (int32_t)(e % words);
    const int32_t s = tiles[3 * t], l = tiles[3 * t + 1];
    uint64_t acc = 0;
    for (int r = 0; r < l; ++r) acc |= v_rows[(int64_t)(s + r) * words + wd];
    tv[e] = acc;
}

// Tile pairs in blocked order.  Cell (T, Ub) holds the pairs of row tile T
// with the indexed tiles of the 64-wide block Ub; cells are ordered by blocks
// of kTilePairBlockT consecutive row tiles, then Ub, then T:
//     cell index ((T / kTilePairBlockT) * nUb + Ub) * kTilePairBlockT + T % kTilePairBlockT.
// The pair kernel's workgroups claim consecutive chunks of this list, so
// those running together on one XCD work on the same 64 indexed tiles, whose
// rows are then read from that XCD's L2 instead of memory (row-major order
// would spread them over a thousand different indexed tiles), while each
// workgroup still keeps its row tile in LDS over a cell's pairs.
// Pass 0 (off == null) writes each cell's pair count (cells never visited
// must be zero beforehand); pass 1 writes the pairs at the scanned offsets.
__global__ __launch_bounds__(64) void k_tile_pairs(int64_t ntA, const int32_t *tilesA, const uint64_t *tvA,
                                                   const uint8_t *newA, int64_t ntB, const int32_t *tilesB,
                                                   const uint64_t *tvB, const uint8_t *newB, int32_t words, int mode,
                                                   int64_t nUb, const int64_t *off, int32_t *cnt, int32_t *oT,
                                                   int32_t *oU) {
    const int lane = threadIdx.x;
    const int64_t T = blockIdx.x;
    const int32_t a = tilesA[3 * T + 2];
    const bool tnew = newA ? newA[T] != 0 : false;
    const bool self = (mode & PM_SELF) != 0;
    const int64_t cbase = (T / kTilePairBlockT) * nUb * kTilePairBlockT + T % kTilePairBlockT;
    for (int64_t ub = self ? T / 64 : 0; ub < nUb; ++ub) {
        const int64_t U = ub * 64 + lane;
        bool keep = false;
        if (U < ntB && (!self || U >= T)) {
            const int32_t b = tilesB[3 * U + 2];
            // Cell b must survive the virtual-pivot test of some point of T; when
            // the row points are indexed points (their cell balls contain them),
            // cell a must also survive the test of some point of U.
            keep = (tvA[T * words + (b >> 6)] >> (b & 63)) & 1ull;
            if (keep && self) keep = (tvB[U * words + (a >> 6)] >> (a & 63)) & 1ull;
            if ((mode & PM_NEW_ONLY) && !tnew && !newB[U]) keep = false;
        }
        const uint64_t m = __ballot(keep);
        const int64_t c = cbase + ub * kTilePairBlockT;
        if (!off) {
            if (lane == 0) cnt[c] = __popcll(m);
        } else if (keep) {
            const int64_t slot = off[c] + __popcll(m & ((1ull << lane) - 1ull));
            oT[slot] = (int32_t)T;
            oU[slot] = (int32_t)U;
        }
    }
}

// The K nearest pivots of each pivot (itself first), ties by index; K > m
// repeats the pivot itself past the m-th.
__global__ __launch_bounds__(64) void k_pivot_knn(int64_t m, const double *dpp2, int32_t K, int32_t *pknn) {
    const int lane = threadIdx.x;
    const int64_t a = blockIdx.x;
    double last = -1.0;
    int64_t lastk = -1;
    for (int t = 0; t < K; ++t) {
        double best = INFINITY;
        int64_t bk = m;
        for (int64_t k = lane; k < m; k += 64) {
            const double v = dpp2[a * m + k];
            const bool after = v > last || (v == last && k > lastk);
            if (after && (v < best || (v == best && k < bk))) { best = v; bk = k; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, kWave);
            const int64_t ok = __shfl_xor(bk, o, kWave);
            if (ob < best || (ob == best && ok < bk)) { best = ob; bk = ok; }
        }
        if (bk >= m) bk = a;    // fewer than K pivots: repeat the pivot itself
        else { last = best; lastk = bk; }
        if (lane == 0) pknn[a * K + t] = (int32_t)bk;
    }
}

// The same list for layers of at most kKnnSortMax pivots: one workgroup
// sorts pivot a's row of squared distances in LDS (bitonic, by distance,
// then index) and keeps the first K.  Equal to the selection above.
constexpr int kKnnSortMax = 4096;
__global__ __launch_bounds__(256) void k_pivot_knn_sorted(int64_t m, int32_t cap, const double *dpp2, int32_t K,
                                                          int32_t *pknn) {
    extern __shared__ __align__(16) unsigned char knn_smem[];
    double *key = (double *)knn_smem;
    int32_t *kid = (int32_t *)(key + cap);
    const int64_t a = blockIdx.x;
    for (int e = threadIdx.x; e < cap; e += blockDim.x) {
        key[e] = e < m ? dpp2[a * m + e] : INFINITY;
        kid[e] = e;   // padding sorts after every pivot (index >= m)
    }
    __syncthreads();
    for (int size = 2; size <= cap; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = threadIdx.x; e < cap; e += blockDim.x) {
                const int f = e ^ stride;
                if (f > e) {
                    const bool up = (e & size) == 0;
                    const bool gt = key[e] > key[f] || (key[e] == key[f] && kid[e] > kid[f]);
                    if (gt == up) {
                        const double tk = key[e];
                        key[e] = key[f];
                        key[f] = tk;
                        const int32_t ti = kid[e];
                        kid[e] = kid[f];
                        kid[f] = ti;
                    }
                }
            }
            __syncthreads();
        }
    for (int t = threadIdx.x; t < K; t += blockDim.x) pknn[a * K + t] = t < m ? kid[t] : (int32_t)a;
}

// Distance key of two rows under a metric (GRNG_METRIC_*): the squared
// Euclidean distance, the L1 or the L-infinity distance, all exact in float64
// on the grid (every difference, square and partial sum is an integer number
// of grid units below 2^53).
__device__ inline double metric_key(const double *__restrict__ a, const double *__restrict__ b, int dp, int metric) {
    double acc = 0.0;
    for (int t = 0; t < dp; ++t) {
        const double e = a[t] - b[t];
        if (metric == GRNG_METRIC_L2)
            acc = fma(e, e, acc);
        else if (metric == GRNG_METRIC_L1)
            acc += fabs(e);
        else
            acc = fmax(acc, fabs(e));
    }
    return acc;
}

// All pairs (no pivot layer): i < j within one set, or every (i, j) across
// two sets, with their distance keys.  Thread per pair, one block row per i.
__global__ void k_pairs_all(int64_t nA, const double *__restrict__ XA, const double *__restrict__ nrmA, int64_t nB,
                            const double *__restrict__ XB, const double *__restrict__ nrmB, int dp, int self,
                            int metric, PairList out, unsigned long long *counters) {
    const int64_t i = blockIdx.y;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool keep = j < nB && (!self || j > i);
    double d2 = 0.0;
    if (keep) {
        if (metric == GRNG_METRIC_L2) {
            double acc = 0.0;
            for (int t = 0; t < dp; ++t) acc = fma(XA[i * dp + t], XB[j * dp + t], acc);
            d2 = nrmA[i] + nrmB[j] - 2.0 * acc;
        } else {
            d2 = metric_key(XA + i * dp, XB + j * dp, dp, metric);
        }
    }
    wave_append(out, keep, (int32_t)i, (int32_t)j, d2);
    const uint32_t c = wave_sum(keep ? 1u : 0u);
    if ((threadIdx.x & 63) == 0 && c) {
        atomicAdd(&counters[C_DIST], (unsigned long long)c);
        atomicAdd(&counters[C_CAND], (unsigned long long)c);
    }
}

// ---------------------------------------------------------------------------
// Witness cells relevant to a row point x: cell c may hold a witness of some
// pair (x, y) of x only if d(x, p_c) - radius(c) < max_y d(x, y)
// (Proposition 3 with the x-side distance alone).  pass 0 counts, pass 1
// fills the cells sorted by d(x, p_c) ascending with their exact d^2(x, p_c).
constexpr int kRelSortMax = 4096;   // kept cells sorted in LDS per row (8-byte keys)
constexpr int kRelThreads = 256;    // threads per row in the writing pass (they share the sort)

__global__ __launch_bounds__(kRelThreads) void k_relevant_groups(int64_t n, int64_t m, const int32_t *perm,
                                                                 const double *dxp, const double *dvor,
                                                                 const int32_t *gcount, const uint64_t *dmax_bits,
                                                                 const int64_t *rel_off, int32_t *rel_cnt,
                                                                 int32_t *rel_grp, double *rel_d2x, int32_t cap,
                                                                 int pass, unsigned long long *counters) {
    // Pass 0 (one wave per row) counts the cells of row point i that may hold
    // a witness of any of its pairs (Proposition 3 with the row's largest pair
    // distance); pass 1 writes them, nearest pivot first (a bitonic sort in
    // LDS of at most cap entries, a power of two, by the whole workgroup), or
    // in pivot order when there are more than cap of them or cap is 0 (the
    // order only steers the scan, it never changes a verdict).  Sort key: the float32
    // bits of d^2 (monotone in d^2 for non-negative values) above the cell id.
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *key = (uint64_t *)smem;
    const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
    // Rows in a grid-stride loop: most rows of an insertion's Stage VII have
    // nothing to write, and a workgroup per row would be launch-bound.
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        __syncthreads();   // the previous row's keys are read out
        const double dmax2 = __longlong_as_double((long long)dmax_bits[i]);
        if (!(dmax2 > 0.0)) {
            if (pass == 0 && tid == 0) rel_cnt[i] = 0;
            continue;
        }
        int64_t o = 0, cnt = 0;
        if (pass == 1) {
            o = rel_off[i];
            cnt = rel_off[i + 1] - o;
            if (cnt == 0) continue;
        }
        const bool sorted = cnt <= cap;
        if (pass == 1 && !sorted && cap > 0 && tid == 0) atomicAdd(&counters[C_UNSORTED], 1ull);
        const double dmax_hi = sqrt_hi(dmax2);
        const double *row = dxp + (int64_t)perm[i] * m;
        if (tid < 64) {
            int64_t pos = 0;
            for (int64_t k0 = 0; k0 < m; k0 += 256) {
                // four groups of 64 cells per pass, their loads in flight together
                double d2[4], dv[4];
                int32_t gc[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t k = k0 + 64 * u + lane;
                    const bool in = k < m;
                    d2[u] = in ? row[k] : INFINITY;
                    dv[u] = in ? dvor[k] : 0.0;
                    gc[u] = in ? gcount[k] : 0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t k = k0 + 64 * u + lane;
                    // skip when d(x, p_k) - radius_k >= the row's largest pair
                    // distance, tested on squares (d2 is exact; the margin covers
                    // the rounding of the right side)
                    const double r = dv[u] + dmax_hi;
                    const bool keep = gc[u] > 0 && !(d2[u] >= r * r * (1.0 + 1e-12));
                    const uint64_t bal = __ballot(keep);
                    if (pass == 1 && keep) {
                        const int64_t t = pos + __popcll(bal & ((1ull << lane) - 1ull));
                        if (sorted) {
                            key[t] = ((uint64_t)__float_as_uint((float)d2[u]) << 32) | (uint64_t)(uint32_t)k;
                        } else {
                            rel_grp[o + t] = (int32_t)k;
                            rel_d2x[o + t] = d2[u];
                        }
                    }
                    pos += __popcll(bal);
                }
            }
            if (pass == 0 && lane == 0) rel_cnt[i] = (int32_t)pos;
        }
        if (pass == 0 || !sorted) continue;   // uniform over the workgroup
        int32_t P = 64;
        while (P < cnt) P <<= 1;
        for (int64_t t = cnt + tid; t < P; t += nt) key[t] = ~0ull;
        __syncthreads();
        for (int32_t size = 2; size <= P; size <<= 1) {
            for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (int32_t t = tid; t < (P >> 1); t += nt) {
                    const int32_t lo = 2 * t - (t & (stride - 1));
                    const int32_t hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t ka = key[lo], kb = key[hi];
                    if ((ka > kb) == up) {
                        key[lo] = kb;
                        key[hi] = ka;
                    }
                }
                __syncthreads();
            }
        }
        for (int64_t t = tid; t < cnt; t += nt) {
            const int32_t k = (int32_t)(uint32_t)key[t];
            rel_grp[o + t] = k;
            rel_d2x[o + t] = row[k];   // the exact value, not the float32 key
        }
    }
}

// ---------------------------------------------------------------------------
// Stage V with the row's other candidates as witnesses (Algorithm 1, Stage 5:
// a candidate x_k of Q invalidates link (Q, x_j) when it lies in their lune).
// Here a row point's candidates are its partners in the exhaustive pair list
// (the pairs Stages I-V left), and each pair (x, y) is tested against the 64
// partners of x nearest to x and, when y is a point of the same set, the 64
// partners of y nearest to y.  Only proven kills count (anything uncertain is
// left to the exhaustive scan), so the witness choice affects work only.

static_assert(kPartnerWitnesses == kWave, "one partner witness per lane");

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = __shfl_xor((uint32_t)v, m, kWave), hi = __shfl_xor((uint32_t)(v >> 32), m, kWave);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = __shfl((uint32_t)v, src, kWave), hi = __shfl((uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}
// Ascending bitonic sort of one value per lane across the wave.
__device__ inline uint64_t wave_sort_u64(uint64_t k) {
    const int lane = threadIdx.x & 63;
    for (int size = 2; size <= 64; size <<= 1)
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint64_t o = shfl_xor_u64(k, j);
            const bool keep_min = ((lane & j) == 0) == ((lane & size) == 0 || size == 64);
            k = keep_min ? (o < k ? o : k) : (o > k ? o : k);
        }
    return k;
}
// Ascending order of a bitonic sequence held one value per lane.
__device__ inline uint64_t wave_merge_u64(uint64_t k) {
    const int lane = threadIdx.x & 63;
    for (int j = 32; j > 0; j >>= 1) {
        const uint64_t o = shfl_xor_u64(k, j);
        k = (lane & j) == 0 ? (o < k ? o : k) : (o > k ? o : k);
    }
    return k;
}

// The kPartnerWitnesses (64) nearest partners of each row point: in the list
// sorted by row point (row r at [off[r], off[r+1])) and, when given, in the
// same pairs sorted by their other point (off2, py2, pd22: the pairs where r
// is the second point).  Key = float32 d^2 rounded up (an upper bound; bit
// patterns of non-negative floats order as integers), then the partner's
// index.  One wave per row, 64 entries per step merged into the running best
// 64.  Unused slots: id -1, d^2 +inf.  With the nearer lists before them
// (pid, pd2p), only keys after the row's last one there count: the next 64.
__global__ __launch_bounds__(256) void k_partner_top(int64_t nrows, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ py, const double *__restrict__ pd2,
                                                     const int64_t *__restrict__ off2,
                                                     const int32_t *__restrict__ py2,
                                                     const double *__restrict__ pd22,
                                                     const int32_t *__restrict__ pid,
                                                     const float *__restrict__ pd2p, int32_t *__restrict__ wid,
                                                     float *__restrict__ wd2) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < nrows; r += nw) {
        uint64_t best = ~0ull;
        bool first = true;
        uint64_t after = 0;   // keys up to this one are in the nearer list
        bool any = true;
        if (pid) {
            const int32_t last = pid[r * kPartnerWitnesses + kPartnerWitnesses - 1];
            any = last >= 0;   // a nearer list with fewer than 64 holds them all
            if (any)
                after = ((uint64_t)__float_as_uint(pd2p[r * kPartnerWitnesses + kPartnerWitnesses - 1]) << 32) |
                        (uint32_t)last;
        }
        for (int src = 0; src < (off2 ? 2 : 1); ++src) {
            const int64_t *o = src ? off2 : off;
            const int32_t *ids = src ? py2 : py;
            const double *dd = src ? pd22 : pd2;
            const int64_t b = o[r], e = any ? o[r + 1] : b;
            for (int64_t c0 = b; c0 < e; c0 += 64) {
                const int64_t i = c0 + lane;
                uint64_t k = ~0ull;
                if (i < e) k = ((uint64_t)__float_as_uint(__double2float_ru(dd[i])) << 32) | (uint32_t)ids[i];
                if (pid && k <= after) k = ~0ull;
                k = wave_sort_u64(k);
                if (first) {
                    best = k;
                    first = false;
                    continue;
                }
                // best and k ascending: the lane-wise min of best and k reversed
                // holds the 64 smallest of both, as a bitonic sequence
                const uint64_t rk = shfl_u64(k, 63 - lane);
                best = wave_merge_u64(rk < best ? rk : best);
            }
        }
        const bool none = best == ~0ull;
        wid[r * kPartnerWitnesses + lane] = none ? -1 : (int32_t)(uint32_t)best;
        wd2[r * kPartnerWitnesses + lane] = none ? INFINITY : __uint_as_float((uint32_t)(best >> 32));
    }
}

// Largest d^2 of each row's pairs that the partner pass left (0 for none):
// the witness cells a row needs shrink to those of its live pairs.
__global__ __launch_bounds__(256) void k_live_dmax(int64_t nrows, const int64_t *__restrict__ off,
                                                   const double *__restrict__ pd2, const uint8_t *__restrict__ alive,
                                                   uint64_t *__restrict__ dmax_bits) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6); r < nrows; r += nw) {
        double mx = 0.0;
        for (int64_t i = off[r] + lane; i < off[r + 1]; i += 64)
            if (alive[i]) mx = fmax(mx, pd2[i]);
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
        if (lane == 0) dmax_bits[r] = (uint64_t)__double_as_longlong(mx);
    }
}

// d^2(a, b) < t proven on rows of dp values (early exit once a partial sum
// reaches t: partial sums only grow).  Float32 rows: the direct-form sum's
// relative error is below (dp+2) 2^-24, so t is the pair's d^2 lowered by
// (dp+8) 2^-24 and rounded down; float64 rows: exact sums, t = d^2.
template <typename T>
__device__ inline bool below(const T *__restrict__ a, const T *__restrict__ b, int dp, T t) {
    T s = 0;
    for (int c = 0; c < dp; c += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T e = a[c + u] - b[c + u];
            s = fma(e, e, s);
        }
        if (!(s < t)) return false;
    }
    return true;
}

// The proven-kill pass.  The list is sorted by row point, and each wave
// takes chunks of kPartnerChunk consecutive pairs, so most of a chunk shares
// its row point x: the 64 partners of x (one per lane) are loaded once per
// row point with the first KR coordinates of their rows in registers, and a
// pair (x, y) then tests them against y's row, which is the same for the
// whole wave.  A pair that survives is tested against the partners of y
// (their rows gathered) with x's row.
constexpr int kPartnerChunk = 64;

template <typename T, int KR>
__global__ __launch_bounds__(256) void k_partner_witness(int64_t np, const int32_t *__restrict__ px,
                                                         const int32_t *__restrict__ py,
                                                         const double *__restrict__ pd2, int dp,
                                                         const T *__restrict__ X, const int32_t *__restrict__ wid,
                                                         const float *__restrict__ wd2, bool both,
                                                         bool again, uint8_t *__restrict__ alive,
                                                         unsigned long long *counters) {
    constexpr bool F32 = sizeof(T) == 4;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const double g32 = (double)(dp + 8) * 0x1p-24;
    const int64_t nchunks = (np + kPartnerChunk - 1) / kPartnerChunk;
    uint32_t ntests = 0, nkill = 0, ndeep = 0;
    for (int64_t ch = blockIdx.x * 4 + (threadIdx.x >> 6); ch < nchunks; ch += nw) {
        const int64_t p0 = ch * kPartnerChunk, p1 = p0 + kPartnerChunk < np ? p0 + kPartnerChunk : np;
        int32_t cx = -1, z0 = -1;
        float w0 = INFINITY;
        T zr[KR];
        for (int64_t p = p0; p < p1; ++p) {
            if (again && alive[p] == 0) continue;   // decided with a nearer list (uniform)
            const int32_t x = __builtin_amdgcn_readfirstlane(px[p]);
            const int32_t y = __builtin_amdgcn_readfirstlane(py[p]);
            const double d2 = pd2[p];
            if (x != cx) {   // uniform
                cx = x;
                z0 = wid[(int64_t)x * kPartnerWitnesses + lane];
                w0 = wd2[(int64_t)x * kPartnerWitnesses + lane];
                const T *zrow = X + (int64_t)(z0 < 0 ? 0 : z0) * dp;
#pragma unroll
                for (int c = 0; c < KR; ++c) zr[c] = c < dp ? zrow[c] : T(0);
            }
            const T t = F32 ? (T)__double2float_rd(d2 - d2 * g32) : (T)d2;
            // x's partners against y
            bool kill = false;
            if (z0 >= 0 && z0 != y && (double)w0 < d2) {
                ++ntests;
                const T *yr = X + (int64_t)y * dp;
                T acc = 0;
                bool out = false;
#pragma unroll
                for (int c = 0; c < KR; c += 4) {
                    if (c < dp && !out) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const T e = yr[c + u] - zr[c + u];
                            acc = fma(e, e, acc);
                        }
                        if ((c & 4) && !(acc < t)) out = true;
                    }
                }
                const T *zrow = X + (int64_t)z0 * dp;
                for (int c = KR; c < dp && !out; c += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const T e = yr[c + u] - zrow[c + u];
                        acc = fma(e, e, acc);
                    }
                    if (!(acc < t)) out = true;
                }
                kill = !out && acc < t;
            }
            uint64_t km = __ballot(kill);   // lanes hold the partners nearest first
            bool dead = km != 0;
            if (!dead && both) {
                // y's partners against x
                const int32_t z1 = wid[(int64_t)y * kPartnerWitnesses + lane];
                const float w1 = wd2[(int64_t)y * kPartnerWitnesses + lane];
                bool kill1 = false;
                if (z1 >= 0 && z1 != x && (double)w1 < d2) {
                    ++ntests;
                    kill1 = below(X + (int64_t)x * dp, X + (int64_t)z1 * dp, dp, t);
                }
                km = __ballot(kill1);
                dead = km != 0;
            }
            if (lane == 0) {
                alive[p] = dead ? 0 : 1;
                nkill += dead;
                ndeep += dead && __ffsll((long long)km) - 1 >= kPartnerWitnesses - kPartnerWitnesses / 4;
            }
        }
    }
    ntests = wave_sum(ntests);
    if (lane == 0) {
        atomicAdd(&counters[C_WTEST], (unsigned long long)ntests);
        atomicAdd(&counters[C_DIST], (unsigned long long)ntests);
        atomicAdd(&counters[C_PARTNER_TESTS], (unsigned long long)ntests);
        if (nkill) atomicAdd(&counters[C_PARTNER_KILLS], (unsigned long long)nkill);
        if (ndeep) atomicAdd(&counters[C_PARTNER_DEEP], (unsigned long long)ndeep);
    }
}

// ---------------------------------------------------------------------------
// Exhaustive lune test of surviving pairs (Stages IV-VI).  One wave per pair.
//
// The row point's relevant cells are taken 64 at a time (one per lane):
// distance of y to the cell's pivot, the pivot itself as a witness, and the
// Proposition 3 skip.  The members of the cells still to scan are then laid
// end to end in visit order (a wave prefix sum of member counts) and
// streamed 256 per step across cell boundaries, each lane keeping a cursor
// into the per-wave cell table in LDS; a ballot after each step ends the
// pair at the first witness.  Streaming across cells keeps many loads in
// flight per step where a cell-at-a-time scan would pay the memory latency
// once per (small) cell.
constexpr int kLuneWaves = 4;

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// The first 8 coordinates of each float32 row, packed (dp > 8).
__global__ void k_row_prefix(const float *__restrict__ X, int64_t n, int dp, float *__restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * 8) return;
    out[e] = X[(e >> 3) * dp + (e & 7)];
}

template <bool F32>
__global__ __launch_bounds__(256) void k_lune_guided(
    int64_t npairs, const int32_t *__restrict__ px, const int32_t *__restrict__ py, const double *__restrict__ pd2,
    int dp, const double *__restrict__ Xx, const double *__restrict__ nrmx, const double *__restrict__ Xh,
    const double *__restrict__ nrmh, const double *__restrict__ dhome, const float *__restrict__ Xxf,
    const float *__restrict__ Xhf, const float *__restrict__ Xpre, int pst, const float *__restrict__ dhomef,
    const int32_t *__restrict__ zstart, const int32_t *__restrict__ grp_off, const double *__restrict__ dvor,
    const double *__restrict__ Xp, const double *__restrict__ nrmp, const int64_t *__restrict__ rel_off,
    const int32_t *__restrict__ rel_grp, const double *__restrict__ rel_d2x, const double *__restrict__ rad,
    const uint16_t *__restrict__ scorer, bool lune_order, bool prekilled,
    uint8_t *__restrict__ alive, unsigned long long *work, unsigned long long *counters) {
    // Per-wave cell table in visit order: first member, exclusive member
    // prefix (entry 64 = total) and max(d(x,p), d(y,p)) lower bound.
    __shared__ int32_t t_z0[kLuneWaves][64];
    __shared__ int32_t t_pre[kLuneWaves][65];
    __shared__ double t_gmax[kLuneWaves][64];
    __shared__ double t_gmin[kLuneWaves][64];   // min(d(x,p), d(y,p)) upper bound
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t *z0t = t_z0[wv], *pre = t_pre[wv];
    double *gmt = t_gmax[wv], *gmn = t_gmin[wv];
    // Dynamic, XCD-aware scheduling: workgroups are dealt round-robin to the
    // 8 XCDs, so a wave on XCD c claims pairs from the c-th contiguous eighth
    // of the list (sorted by row point: its witness cells stay in that XCD's
    // L2), then helps the other eighths.  Pair costs vary by orders of
    // magnitude, so static assignment would leave long tails.
    const int xcd0 = blockIdx.x % kXcds;
    int xr = 0;
    uint32_t ntests = 0, ndist = 0, nrecheck = 0;
    unsigned long long nkept = 0;   // tests of pairs that stay edges
    // Float32 screen: the direct-form sum of dp squared float32 differences
    // has relative error below gamma_{dp+2} = (dp+2)u / (1 - (dp+2)u),
    // u = 2^-24 (one rounding per difference, one per fused multiply-add,
    // all terms non-negative).  With g = (dp+8)u > gamma, a float32 value
    // below rd(d2 (1-g)) proves d^2 < d2 and one at or above ru(d2 (1+g))
    // proves d^2 >= d2; anything between is decided again in exact float64.
    const double g32 = (double)(dp + 8) * 0x1p-24;
    const bool xself = Xx == Xh;   // x is a point of the scanned set (not a query)
    int64_t cur = 0, cend = 0;   // the wave's claimed chunk (uniform)
    // The first 64 cells of row point cx, held per lane: consecutive pairs of
    // a wave mostly share their row point (the list is sorted by it).
    int64_t cx = -1;
    int32_t cg = 0;
    double cd2x = 0.0, csx = 0.0, cnp = 0.0, cdv = 0.0;
    for (;;) {
        if (cur >= cend) {
            int64_t b = -1, e = -1;
            if (lane == 0 && !claim_chunk(npairs, kLuneChunk, xcd0, xr, work, &b, &e)) b = e = -1;
            cur = __shfl(b, 0, kWave);
            cend = __shfl(e, 0, kWave);
            xr = __shfl(xr, 0, kWave);
            if (cur < 0) break;
        }
        const int64_t p = cur++;
        if (prekilled && alive[p] == 0) continue;   // a proven kill of the partner pass (uniform)
        const int64_t x = __builtin_amdgcn_readfirstlane(px[p]);
        const int64_t y = __builtin_amdgcn_readfirstlane(py[p]);
        const double d2 = pd2[p];
        const double *xs = Xx + x * dp;
        const double *ys = Xh + y * dp;
        const double nry = nrmh[y];
        const double dxy_hi = sqrt_hi(d2);
        const float *xf = F32 ? Xxf + x * dp : nullptr;
        const float *yf = F32 ? Xhf + y * dp : nullptr;
        const float tlo = __double2float_rd(d2 - d2 * g32), thi = __double2float_ru(d2 + d2 * g32);
        const uint32_t ntests0 = ntests;
        bool dead = false;
        const int64_t r0 = rel_off[x], r1 = rel_off[x + 1];
        for (int64_t c0 = r0; c0 < r1 && !dead; c0 += 64) {
            const int64_t c = c0 + lane;
            bool scan = false;
            double gmax = 0.0, gmin = 0.0;
            int32_t z0 = 0, nmem = 0;
            float key = -INFINITY;
            if (c < r1) {
                const bool hit = c0 == r0 && x == cx;
                const int32_t g = hit ? cg : rel_grp[c];
                const double d2x = hit ? cd2x : rel_d2x[c];
                const double npg = hit ? cnp : nrmp[g];
                const double dvg = hit ? cdv : dvor[g];
                const double sxg = hit ? csx : sqrt(d2x);
                if (c0 == r0 && !hit) {
                    cg = g;
                    cd2x = d2x;
                    cnp = npg;
                    cdv = dvg;
                    csx = sxg;
                }
                const double d2y = nry + npg - 2.0 * dot_lds(ys, Xp + (int64_t)g * dp, dp);
                ++ndist;
                ++ntests;
                // Stage IV: the cell's pivot itself as a witness (exact); not
                // when only part of each cell may witness (zstart given).
                if (!zstart && d2x < d2 && d2y < d2) dead = true;
                const double dxl = sxg * (1.0 - 1e-15), dyl = sqrt_lo(d2y);
                gmax = fmax(dxl, dyl);
                gmin = fmin(sxg * (1.0 + 1e-15), sqrt_hi(d2y));
                // Proposition 3: skip the cell when it lies wholly outside the lune.
                scan = !surely_ge(gmax, dvg, dxy_hi);
                if (lune_order) key = (float)(-gmax);   // nearest to both ends first
                if (scan) {
                    z0 = zstart ? zstart[g] : grp_off[g];
                    nmem = grp_off[g + 1] - z0;
                    if (scorer) {
                        float f[kMlpFeatures];
                        mlp_features(sqrt(d2x), sqrt(d2y), dvor[g], rad[g], grp_off[g + 1] - grp_off[g], sqrt(d2),
                                     f);
                        key = mlp_score_bf16(scorer, f);
                        if (!(key == key)) key = -INFINITY;   // keep (key, lane) a strict total order
                    }
                }
            }
            if (c0 == r0) cx = x;
            if (__ballot(dead)) { dead = true; break; }
            if (!__ballot(scan && nmem > 0)) continue;
            // Visit order: chunk order (cells sorted by distance to x), or by
            // descending key, the learned score or -max(d(x,p), d(y,p)) (wave
            // bitonic sort of (key, lane)).
            int src = lane;
            if (scorer || lune_order) {
                float k = scan ? key : -INFINITY;
                for (int sz = 2; sz <= 64; sz <<= 1)
                    for (int j = sz >> 1; j > 0; j >>= 1) {
                        const float ok = __shfl_xor(k, j, kWave);
                        const int oi = __shfl_xor(src, j, kWave);
                        const bool desc = (lane & sz) == 0;
                        const bool lower = (lane & j) == 0;
                        const bool other_first = ok > k || (ok == k && oi < src);
                        if (lower == desc ? other_first : !other_first) {
                            k = ok;
                            src = oi;
                        }
                    }
            }
            // Cell table in visit order (position = lane after the sort).
            const int n_at = __shfl(scan ? nmem : 0, src, kWave);
            const int incl = wave_incl_scan(n_at);
            z0t[lane] = __shfl(z0, src, kWave);
            gmt[lane] = __shfl(gmax, src, kWave);
            gmn[lane] = __shfl(gmin, src, kWave);
            pre[lane] = incl - n_at;
            if (lane == 63) pre[64] = incl;
            const int total = __shfl(incl, 63, kWave);
            __builtin_amdgcn_wave_barrier();
            int kc[4] = {0, 0, 0, 0};   // per-slot cursors into the table (monotone)
            for (int base = 0; base < total; base += 256) {
                bool wit = false;
                // A step runs in phases so that the loads of its four slots
                // are in flight together: slot -> witness id and cell entry,
                // then d(z, p), then Proposition 4, then the first 8
                // coordinates of the rows that pass it.
                int32_t zz[4], ce[4];
                bool ok[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int sl = base + 64 * u + lane;
                    ok[u] = sl < total;
                    zz[u] = 0;
                    ce[u] = 0;
                    if (ok[u]) {
                        while (pre[kc[u] + 1] <= sl) ++kc[u];
                        ce[u] = kc[u];
                        zz[u] = z0t[kc[u]] + (sl - pre[kc[u]]);
                        // The pair's own points are never witnesses (max = d(x,y)).
                        ok[u] = !(zz[u] == y || (xself && zz[u] == x));
                    }
                }
                double dzv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) dzv[u] = ok[u] ? (F32 ? (double)dhomef[zz[u]] : dhome[zz[u]]) : 0.0;
                // Proposition 4: skip z when max(d(x,p), d(y,p)) - d(z,p) >= d(x,y);
                // by the same triangle inequality also when d(z,p) -
                // min(d(x,p), d(y,p)) >= d(x,y).  The stored d(z,p) is an
                // upper bound; 1 - 2^-21 of it is a lower bound.
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    ok[u] = ok[u] && !surely_ge(gmt[ce[u]], dzv[u], dxy_hi) &&
                            !surely_ge(dzv[u] * (1.0 - 0x1p-21), gmn[ce[u]], dxy_hi);
                // Exact test: on the grid every difference, square and partial
                // sum is an integer multiple of 2^-2q below 2^53.  The partial
                // sums are exact lower bounds, so the early out below applies.
                auto exact_witness = [&](int64_t z) {
                    const double *zr = Xh + z * dp;
                    double sx = 0.0, sy = 0.0;
                    for (int cc = 0; cc < dp; cc += 2) {
                        if (cc >= 8 && (cc & 7) == 0 && !(sx < d2 && sy < d2)) break;
                        const double2 zv = *reinterpret_cast<const double2 *>(zr + cc);
                        double e = xs[cc] - zv.x;
                        sx = fma(e, e, sx);
                        e = xs[cc + 1] - zv.y;
                        sx = fma(e, e, sx);
                        e = ys[cc] - zv.x;
                        sy = fma(e, e, sy);
                        e = ys[cc + 1] - zv.y;
                        sy = fma(e, e, sy);
                    }
                    return sx < d2 && sy < d2;
                };
                if (F32) {
                    float4 r0[4], r1[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        r0[u] = r1[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (ok[u]) {
                            // the first 8 coordinates from the packed prefix rows
                            const float *zr = Xpre + (int64_t)zz[u] * pst;
                            r0[u] = *reinterpret_cast<const float4 *>(zr);
                            if (dp > 4) r1[u] = *reinterpret_cast<const float4 *>(zr + 4);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (!ok[u]) continue;
                        // Direct-form float32 sums, coordinates 0-7 from the
                        // registers (zero past dp), the rest from the row.
                        float sx = 0.f, sy = 0.f, e;
                        e = xf[0] - r0[u].x; sx = fmaf(e, e, sx);
                        e = xf[1] - r0[u].y; sx = fmaf(e, e, sx);
                        e = xf[2] - r0[u].z; sx = fmaf(e, e, sx);
                        e = xf[3] - r0[u].w; sx = fmaf(e, e, sx);
                        e = yf[0] - r0[u].x; sy = fmaf(e, e, sy);
                        e = yf[1] - r0[u].y; sy = fmaf(e, e, sy);
                        e = yf[2] - r0[u].z; sy = fmaf(e, e, sy);
                        e = yf[3] - r0[u].w; sy = fmaf(e, e, sy);
                        if (dp > 4) {
                            e = xf[4] - r1[u].x; sx = fmaf(e, e, sx);
                            e = xf[5] - r1[u].y; sx = fmaf(e, e, sx);
                            e = xf[6] - r1[u].z; sx = fmaf(e, e, sx);
                            e = xf[7] - r1[u].w; sx = fmaf(e, e, sx);
                            e = yf[4] - r1[u].x; sy = fmaf(e, e, sy);
                            e = yf[5] - r1[u].y; sy = fmaf(e, e, sy);
                            e = yf[6] - r1[u].z; sy = fmaf(e, e, sy);
                            e = yf[7] - r1[u].w; sy = fmaf(e, e, sy);
                        }
                        const float *zr = Xhf + (int64_t)zz[u] * dp;
                        for (int cc = 8; cc < dp; cc += 4) {
                            // Early out every 8 coordinates: adding non-negative
                            // terms never lowers a rounded sum, so a partial sum
                            // at or above thi proves the full one is too, and z
                            // is no witness.  Most candidates end at the first
                            // check, reading half a 16-D row.
                            if ((cc & 7) == 0 && !(sx < thi && sy < thi)) break;
                            const float4 zv = *reinterpret_cast<const float4 *>(zr + cc);
                            e = xf[cc] - zv.x; sx = fmaf(e, e, sx);
                            e = xf[cc + 1] - zv.y; sx = fmaf(e, e, sx);
                            e = xf[cc + 2] - zv.z; sx = fmaf(e, e, sx);
                            e = xf[cc + 3] - zv.w; sx = fmaf(e, e, sx);
                            e = yf[cc] - zv.x; sy = fmaf(e, e, sy);
                            e = yf[cc + 1] - zv.y; sy = fmaf(e, e, sy);
                            e = yf[cc + 2] - zv.z; sy = fmaf(e, e, sy);
                            e = yf[cc + 3] - zv.w; sy = fmaf(e, e, sy);
                        }
                        if (sx < tlo && sy < tlo) {
                            wit = true;
                        } else if (!(sx >= thi || sy >= thi)) {
                            ++nrecheck;   // too close to call in float32
                            wit = wit || exact_witness(zz[u]);
                        }
                        ndist += 2;
                        ++ntests;
                    }
                } else {
                    // float64 rows: the first 4 coordinates of every slot that
                    // passed Proposition 4 are fetched together (dp >= 4).
                    double2 q0[4], q1[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        q0[u] = q1[u] = make_double2(0.0, 0.0);
                        if (ok[u]) {
                            const double *zr = Xh + (int64_t)zz[u] * dp;
                            q0[u] = *reinterpret_cast<const double2 *>(zr);
                            q1[u] = *reinterpret_cast<const double2 *>(zr + 2);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (!ok[u]) continue;
                        double sx = 0.0, sy = 0.0, e;
                        e = xs[0] - q0[u].x; sx = fma(e, e, sx);
                        e = xs[1] - q0[u].y; sx = fma(e, e, sx);
                        e = xs[2] - q1[u].x; sx = fma(e, e, sx);
                        e = xs[3] - q1[u].y; sx = fma(e, e, sx);
                        e = ys[0] - q0[u].x; sy = fma(e, e, sy);
                        e = ys[1] - q0[u].y; sy = fma(e, e, sy);
                        e = ys[2] - q1[u].x; sy = fma(e, e, sy);
                        e = ys[3] - q1[u].y; sy = fma(e, e, sy);
                        const double *zr = Xh + (int64_t)zz[u] * dp;
                        for (int cc = 4; cc < dp; cc += 2) {
                            if ((cc & 7) == 0 && !(sx < d2 && sy < d2)) break;
                            const double2 zv = *reinterpret_cast<const double2 *>(zr + cc);
                            e = xs[cc] - zv.x; sx = fma(e, e, sx);
                            e = xs[cc + 1] - zv.y; sx = fma(e, e, sx);
                            e = ys[cc] - zv.x; sy = fma(e, e, sy);
                            e = ys[cc + 1] - zv.y; sy = fma(e, e, sy);
                        }
                        wit = wit || (sx < d2 && sy < d2);
                        ndist += 2;
                        ++ntests;
                    }
                }
                if (__ballot(wit)) { dead = true; break; }
            }
            __builtin_amdgcn_wave_barrier();   // the table is rewritten by the next chunk
        }
        if (lane == 0) alive[p] = dead ? 0 : 1;
        if (!dead) nkept += ntests - ntests0;
    }
    ntests = wave_sum(ntests);
    ndist = wave_sum(ndist);
    nrecheck = wave_sum(nrecheck);
    for (int o = 32; o > 0; o >>= 1) nkept += __shfl_xor(nkept, o, kWave);
    if (lane == 0) {
        atomicAdd(&counters[C_WTEST], (unsigned long long)ntests);
        atomicAdd(&counters[C_LUNE], (unsigned long long)ntests);
        atomicAdd(&counters[C_DIST], (unsigned long long)ndist);
        if (nrecheck) atomicAdd(&counters[C_RECHECK], (unsigned long long)nrecheck);
        if (nkept) atomicAdd(&counters[C_LUNE_KEPT], nkept);
    }
}

// Unsigned 128-bit sums of squares for the exact beta-skeleton test.
struct U128 {
    uint64_t lo, hi;
};
__device__ inline void add_square(U128 &acc, int64_t e) {
    const uint64_t u = (uint64_t)(e < 0 ? -e : e);
    const uint64_t lo = u * u;
    acc.lo += lo;
    acc.hi += __umul64hi(u, u) + (acc.lo < lo);
}
__device__ inline bool lt_u128(const U128 &a, const U128 &b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// Empty-region test against every point (no pivot layer).  One wave per
// pair, 64 witnesses per step, a ballot ends the pair at the first point in
// its region:
//   RNG      max(d(x,z), d(y,z)) < d(x,y) under the index's metric (distance
//            keys: squared Euclidean, L1, L-infinity);
//   Gabriel  d^2(x,z) + d^2(y,z) < d^2(x,y), tested as d^2(x,z) < d^2(x,y) -
//            d^2(y,z) (exact: a difference of integers below 2^53);
//   beta     (lune-based beta-skeleton, beta = a/4 >= 1) z in both open balls
//            of radius beta d(x,y)/2 centred at (1 - beta/2) x + (beta/2) y
//            and (beta/2) x + (1 - beta/2) y; times 16 these are
//            |8(z - x) + a(x - y)|^2 < a^2 d^2(x,y) and the same with x and y
//            swapped.  On the grid each term 8(z - x) + a(x - y) is an integer
//            of at most 32 bits in units of 2^-q, formed exactly in float64;
//            its square and the sums are taken in 128-bit integers.
// Partial sums (or maxima) of non-negative terms only grow, so a partial key
// at or above the threshold ends a test early.
__global__ __launch_bounds__(256) void k_lune_all(int64_t npairs, const int32_t *__restrict__ px,
                                                  const int32_t *__restrict__ py, const double *__restrict__ pd2,
                                                  int64_t n, int dp, const double *__restrict__ Xx,
                                                  const double *__restrict__ nrmx, const double *__restrict__ X,
                                                  const double *__restrict__ nrm, int64_t z_from, int metric,
                                                  int graph, int beta_q, double gscale, uint8_t *__restrict__ alive,
                                                  unsigned long long *counters) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const bool gabriel = graph == GRNG_GRAPH_GABRIEL;
    const bool beta = graph == GRNG_GRAPH_BETA;
    const double a = (double)beta_q;
    uint32_t ntests = 0;
    for (int64_t p = wave0; p < npairs; p += nwaves) {
        const int64_t x = __builtin_amdgcn_readfirstlane(px[p]);
        const int64_t y = __builtin_amdgcn_readfirstlane(py[p]);
        const double d2 = pd2[p];
        const double *xs = Xx + x * dp;
        const double *ys = X + y * dp;
        U128 rhs = {0, 0};   // beta: a^2 d^2(x,y) in grid units
        if (beta) {
            uint64_t s = 0;   // d^2(x,y) < 2^53 grid units under the grid contract
            for (int c = 0; c < dp; ++c) {
                const int64_t e = (int64_t)((xs[c] - ys[c]) * gscale);
                s += (uint64_t)(e * e);
            }
            const uint64_t a2 = (uint64_t)beta_q * (uint64_t)beta_q;
            rhs.lo = a2 * s;
            rhs.hi = __umul64hi(a2, s);
        }
        bool dead = false;
        for (int64_t zb = z_from; zb < n; zb += 64) {
            const int64_t z = zb + lane;
            bool wit = false;
            if (z < n && beta) {
                const double *zr = X + z * dp;
                U128 s1 = {0, 0}, s2 = {0, 0};
                for (int c = 0; c < dp; ++c) {
                    if (c >= 8 && (c & 7) == 0 && !(lt_u128(s1, rhs) && lt_u128(s2, rhs))) break;
                    const double xy = xs[c] - ys[c];
                    add_square(s1, (int64_t)((8.0 * (zr[c] - xs[c]) + a * xy) * gscale));
                    add_square(s2, (int64_t)((8.0 * (zr[c] - ys[c]) - a * xy) * gscale));
                }
                wit = lt_u128(s1, rhs) && lt_u128(s2, rhs);
                ++ntests;
            } else if (z < n) {
                const double *zr = X + z * dp;
                double sx = 0.0, sy = 0.0;
                for (int c = 0; c < dp; ++c) {
                    if (c >= 8 && (c & 7) == 0) {
                        if (gabriel ? !(sx + sy < d2) : !(sx < d2 && sy < d2)) break;
                    }
                    const double ex = xs[c] - zr[c], ey = ys[c] - zr[c];
                    if (metric == GRNG_METRIC_L2) {
                        sx = fma(ex, ex, sx);
                        sy = fma(ey, ey, sy);
                    } else if (metric == GRNG_METRIC_L1) {
                        sx += fabs(ex);
                        sy += fabs(ey);
                    } else {
                        sx = fmax(sx, fabs(ex));
                        sy = fmax(sy, fabs(ey));
                    }
                }
                wit = gabriel ? (sx < d2 - sy) : (sx < d2 && sy < d2);
                ++ntests;
            }
            if (__ballot(wit)) { dead = true; break; }
        }
        if (lane == 0) alive[p] = dead ? 0 : 1;
    }
    ntests = wave_sum(ntests);
    if (lane == 0) {
        atomicAdd(&counters[C_WTEST], (unsigned long long)ntests);
        atomicAdd(&counters[C_LUNE], (unsigned long long)ntests);
        atomicAdd(&counters[C_DIST], 2ull * ntests);
    }
}

}  // namespace

void launch_pivot_knn(hipStream_t s, int64_t m, const double *dpp2, int32_t K, int32_t *pknn) {
    if (m == 0) return;
    if (m <= kKnnSortMax && K > 16) {
        int32_t cap = 2;
        while (cap < m) cap <<= 1;
        k_pivot_knn_sorted<<<(unsigned)m, 256, (size_t)cap * 12, s>>>(m, cap, dpp2, K, pknn);
    } else {
        k_pivot_knn<<<(unsigned)m, 64, 0, s>>>(m, dpp2, K, pknn);
    }
    GRNG_LAUNCHED();
}

void launch_tile_vmask(hipStream_t s, int64_t ntiles, const int32_t *tiles, const uint64_t *v_rows, int32_t words,
                       uint64_t *tv) {
    if (ntiles == 0) return;
    k_tile_vmask<<<(unsigned)div_up(ntiles * words, 256), 256, 0, s>>>(ntiles, tiles, v_rows, words, tv);
    GRNG_LAUNCHED();
}

void launch_tile_pairs(hipStream_t s, int64_t ntA, const int32_t *tilesA, const uint64_t *tvA, const uint8_t *newA,
                       int64_t ntB, const int32_t *tilesB, const uint64_t *tvB, const uint8_t *newB, int32_t words,
                       int mode, const int64_t *off, int32_t *cnt, int32_t *oT, int32_t *oU) {
    if (ntA == 0) return;
    const int64_t nUb = div_up(ntB, 64);
    k_tile_pairs<<<(unsigned)ntA, 64, 0, s>>>(ntA, tilesA, tvA, newA, ntB, tilesB, tvB, newB, words, mode, nUb, off,
                                              cnt, oT, oU);
    GRNG_LAUNCHED();
}

void launch_pair_masks(hipStream_t s, int64_t tp0, int64_t n, const int32_t *tpT, const int32_t *tpU,
                       const PointsView &A, const PointsView &B, int mode, int32_t words, const int32_t *pknn,
                       int32_t K, uint64_t *rec) {
    if (n == 0) return;
    require(K >= 1 && K <= kPiv, GRNG_EINVAL, "Stage IV pivot count out of range");
    k_pair_masks<<<(unsigned)div_up(n, 4), 256, 0, s>>>(tp0, n, tpT, tpU, A, B, mode, words, pknn, K, rec);
    GRNG_LAUNCHED();
}

void launch_pairs_tiled(hipStream_t s, int64_t ntp, const uint64_t *rec, const double *XA, const double *nrmA,
                        const double *XB, const double *nrmB, int mode, int dp, int32_t K,
                        const double *Xp, const double *nrmp, PairList out, uint64_t *dmax_bits, uint64_t *work,
                        uint64_t *counters) {
    if (ntp == 0) return;
    require(dp <= kMaxDp, GRNG_EINVAL, "dimension too large for the pair kernel");
    require(K >= 1 && K <= kPiv, GRNG_EINVAL, "Stage IV pivot count out of range");
    launch_fill_u64(s, work, kXcds * kWorkStride, 0ull);
    // 16-bit witness matrices only where they make room for a second
    // workgroup per CU (32-D rows, for instance): they cost some Stage V
    // kills (8 significant bits), which then go to the exhaustive scan.
    const bool h16 = !pairs_two_per_cu(pairs_lds_bytes(dp, false)) && pairs_two_per_cu(pairs_lds_bytes(dp, true));
    const size_t lds = pairs_lds_bytes(dp, h16);
    require(lds <= 160 * 1024, GRNG_EINVAL, "dimension too large for the pair kernel's LDS tiles");
    const void *fn = h16 ? (const void *)k_pairs_tiled<uint16_t> : (const void *)k_pairs_tiled<float>;
    if (lds > 64 * 1024) GRNG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int64_t grid = std::max<int64_t>(kXcds, std::min<int64_t>(div_up(ntp, kPairChunk), 256 * 4));
    if (h16)
        k_pairs_tiled<uint16_t><<<(unsigned)grid, kPairThreads, lds, s>>>(
            ntp, rec, XA, nrmA, XB, nrmB, mode, dp, K, Xp, nrmp, out, (unsigned long long *)dmax_bits,
            (unsigned long long *)work, (unsigned long long *)counters);
    else
        k_pairs_tiled<float><<<(unsigned)grid, kPairThreads, lds, s>>>(
            ntp, rec, XA, nrmA, XB, nrmB, mode, dp, K, Xp, nrmp, out, (unsigned long long *)dmax_bits,
            (unsigned long long *)work, (unsigned long long *)counters);
    GRNG_LAUNCHED();
}

void launch_pairs_all(hipStream_t s, int64_t nA, const double *XA, const double *nrmA, int64_t nB, const double *XB,
                      const double *nrmB, int dp, bool self, int metric, PairList out, uint64_t *counters) {
    if (nA == 0 || nB == 0) return;
    require(nA <= 65535, GRNG_EINVAL, "brute-force pair enumeration limited to 65535 row points");
    dim3 g((unsigned)div_up(nB, 256), (unsigned)nA);
    k_pairs_all<<<g, 256, 0, s>>>(nA, XA, nrmA, nB, XB, nrmB, dp, self ? 1 : 0, metric, out,
                                  (unsigned long long *)counters);
    GRNG_LAUNCHED();
}

void launch_relevant_groups(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp,
                            const double *dvor, const int32_t *gcount, const uint64_t *dmax_bits,
                            const int64_t *rel_off, int32_t *rel_cnt, int32_t *rel_grp, double *rel_d2x,
                            uint64_t *counters, bool sort) {
    if (n == 0) return;
    require(n <= 0x7fffffffLL, GRNG_EINVAL, "too many points for the witness-cell pass");
    int32_t cap = 64;   // sort capacity: the layer size rounded up to a power of two, at most kRelSortMax
    while (cap < m && cap < kRelSortMax) cap <<= 1;
    if (!sort) cap = 0;   // pivot order for every row
    const size_t lds = (size_t)cap * sizeof(uint64_t);
    if (rel_off == nullptr) {
        k_relevant_groups<<<(unsigned)std::min<int64_t>(n, 65536), 64, 0, s>>>(
            n, m, perm, dxp, dvor, gcount, dmax_bits, nullptr, rel_cnt, nullptr, nullptr, cap, 0,
            (unsigned long long *)counters);
    } else {
        // unsorted rows are written by one wave: a single-wave workgroup
        k_relevant_groups<<<(unsigned)std::min<int64_t>(n, 65536), sort ? kRelThreads : 64, lds, s>>>(
            n, m, perm, dxp, dvor, gcount, dmax_bits, rel_off, rel_cnt, rel_grp, rel_d2x, cap, 1,
            (unsigned long long *)counters);
    }
    GRNG_LAUNCHED();
}

void launch_pairs_sort_rows(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, const double *pd2,
                            int64_t n, int32_t *cnt, int64_t *off, int32_t *ox, int32_t *oy, double *od2) {
    if (np == 0) return;
    const bool lds = n <= kRowsLdsMax;
    const unsigned gl = (unsigned)div_up(np, 1024 * kSortPer);
    const size_t hb = sizeof(int32_t) * (size_t)n;
    if (lds)
        k_pairs_count_rows_lds<<<gl, 1024, hb, s>>>(np, px, n, cnt);
    else
        k_pairs_count_rows<<<(unsigned)div_up(np, 256), 256, 0, s>>>(np, px, cnt);
    GRNG_LAUNCHED();
    launch_scan_i32_to_i64(s, cnt, n, off);
    launch_fill_u64(s, (uint64_t *)cnt, div_up(n, 2), 0ull);
    if (lds)
        k_pairs_scatter_rows_lds<<<gl, 1024, hb, s>>>(np, px, py, pd2, n, off, cnt, ox, oy, od2);
    else
        k_pairs_scatter_rows<<<(unsigned)div_up(np, 256), 256, 0, s>>>(np, px, py, pd2, off, cnt, ox, oy, od2);
    GRNG_LAUNCHED();
}

void launch_lune_guided(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const double *pd2,
                        int dp, const double *Xx, const double *nrmx, const double *Xh, const double *nrmh,
                        int64_t nh, const double *dhome, const float *Xxf, const float *Xhf, const float *dhomef,
                        const int32_t *zstart, const int32_t *grp_off,
                        const double *dvor, const double *Xp, const double *nrmp, const int64_t *rel_off,
                        const int32_t *rel_grp, const double *rel_d2x, const double *rad, const uint16_t *scorer,
                        bool lune_order, bool prekilled,
                        uint8_t *alive, uint64_t *work, uint64_t *counters) {
    if (npairs == 0) return;
    require(dp <= kMaxDp, GRNG_EINVAL, "dimension too large for the lune kernel");
    launch_fill_u64(s, work, kXcds * kWorkStride, 0ull);
    // The waves claim pairs dynamically, so the grid only sets how many scan
    // at once.  While the float32 witness rows fit in the 256 MiB last-level
    // cache, the scan waits on their load latency, and four workgroups (16
    // waves) per CU, as many as its registers allow, hide more of it than
    // three (15% faster on the 100k x 16-D build).  Rows streamed from HBM
    // (1M x 96-D: 384 MB) and the float64 scan (twice the bytes per row) run
    // faster with three (by 10% and 4%).
    const bool f32 = Xxf && Xhf && dhomef;
    const bool cached = f32 && nh * (int64_t)dp * 4 <= (int64_t)256 << 20;
    const int64_t grid = std::max<int64_t>(kXcds, std::min<int64_t>(div_up(npairs, 4), 256 * (cached ? 4 : 3)));
    // Most float32 witness tests end after the first 8 coordinates (their
    // partial sums already exceed the pair's distance); a packed copy of
    // those 8 coordinates per row lets a scan step read them from a quarter
    // of the cache lines (rows of more than 8 coordinates).
    DevBuf pre;
    const float *Xpre = Xhf;
    int pst = dp;
    if (f32 && dp > 8) {
        pre.alloc(sizeof(float) * 8 * (size_t)std::max<int64_t>(nh, 1));
        k_row_prefix<<<(unsigned)div_up(nh * 8, 256), 256, 0, s>>>(Xhf, nh, dp, pre.as<float>());
        GRNG_LAUNCHED();
        Xpre = pre.as<float>();
        pst = 8;
    }
    if (f32)
        k_lune_guided<true><<<(unsigned)grid, 256, 0, s>>>(
            npairs, px, py, pd2, dp, Xx, nrmx, Xh, nrmh, dhome, Xxf, Xhf, Xpre, pst, dhomef, zstart, grp_off, dvor,
            Xp, nrmp, rel_off, rel_grp, rel_d2x, rad, scorer, lune_order, prekilled, alive, (unsigned long long *)work,
            (unsigned long long *)counters);
    else
        k_lune_guided<false><<<(unsigned)grid, 256, 0, s>>>(
            npairs, px, py, pd2, dp, Xx, nrmx, Xh, nrmh, dhome, Xxf, Xhf, Xpre, pst, dhomef, zstart, grp_off, dvor,
            Xp, nrmp, rel_off, rel_grp, rel_d2x, rad, scorer, lune_order, prekilled, alive, (unsigned long long *)work,
            (unsigned long long *)counters);
    GRNG_LAUNCHED();
}

void launch_partner_top(hipStream_t s, int64_t nrows, const int64_t *off, const int32_t *py, const double *pd2,
                        const int64_t *off2, const int32_t *py2, const double *pd22, const int32_t *pid,
                        const float *pd2p, int32_t *wid, float *wd2) {
    if (nrows == 0) return;
    const int64_t grid = std::min<int64_t>(div_up(nrows, 4), 1 << 16);
    k_partner_top<<<(unsigned)grid, 256, 0, s>>>(nrows, off, py, pd2, off2, py2, pd22, pid, pd2p, wid, wd2);
    GRNG_LAUNCHED();
}

void launch_partner_witness(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, const double *pd2,
                            int dp, const float *Xf, const double *Xd, const int32_t *wid, const float *wd2,
                            bool both, bool again, uint8_t *alive, uint64_t *counters) {
    if (np == 0) return;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(div_up(div_up(np, kPartnerChunk), 4), 4096));
    unsigned long long *ctr = (unsigned long long *)counters;
    if (Xf && dp <= 16)
        k_partner_witness<float, 16><<<(unsigned)grid, 256, 0, s>>>(np, px, py, pd2, dp, Xf, wid, wd2, both, again,
                                                                   alive, ctr);
    else if (Xf)
        k_partner_witness<float, 32><<<(unsigned)grid, 256, 0, s>>>(np, px, py, pd2, dp, Xf, wid, wd2, both, again,
                                                                   alive, ctr);
    else
        k_partner_witness<double, 16><<<(unsigned)grid, 256, 0, s>>>(np, px, py, pd2, dp, Xd, wid, wd2, both, again,
                                                                    alive, ctr);
    GRNG_LAUNCHED();
}

void launch_live_dmax(hipStream_t s, int64_t nrows, const int64_t *off, const double *pd2, const uint8_t *alive,
                      uint64_t *dmax_bits) {
    if (nrows == 0) return;
    k_live_dmax<<<(unsigned)std::min<int64_t>(div_up(nrows, 4), 1 << 16), 256, 0, s>>>(nrows, off, pd2, alive,
                                                                                        dmax_bits);
    GRNG_LAUNCHED();
}

void launch_lune_all(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const double *pd2,
                     int64_t n, int dp, const double *Xx, const double *nrmx, const double *X, const double *nrm,
                     int64_t z_from, int metric, int graph, int beta_q, int grid_exp, uint8_t *alive,
                     uint64_t *counters) {
    if (npairs == 0) return;
    require(dp <= kMaxDp, GRNG_EINVAL, "dimension too large for the lune kernel");
    const int64_t grid = std::min<int64_t>(div_up(npairs, 4), 1 << 16);
    k_lune_all<<<(unsigned)grid, 256, 0, s>>>(npairs, px, py, pd2, n, dp, Xx, nrmx, X, nrm, z_from, metric, graph,
                                              beta_q, std::ldexp(1.0, grid_exp),
                                              alive, (unsigned long long *)counters);
    GRNG_LAUNCHED();
}

}  // namespace grng
