// Pivot-layer kernels.
//
//  * GRNG of a pivot layer (Section 2, Definition 1), brute force over pivot
//    triples, optionally restricted to candidate pairs allowed by a coarser
//    layer (Section 3, Theorem 2) with coarse pivots tried first as witnesses
//    (Section 3, Stage IV).  Each generalized-lune side test
//        d(k,i) + c < d(i,j)
//    is screened in float64 from correctly rounded square roots of exact
//    squared distances and re-decided exactly with 128-bit integers when the
//    screen cannot separate the two sides (the only inexact step is sqrt).
//  * Per-point passes for the exemplar RNG: domain parents (Section 1, pivot
//    domain equation, exact), nearest pivot ("home" cell used to group
//    witnesses), and two virtual-pivot GRNG
//    bitsets of each point (Section 2, Proposition 1 with the point as a zero
//    radius pivot): one over the pivot domains (radii r) and one over the
//    home cells (radius = cell radius, which covers every point, orphans
//    included).  These bitsets only prune, so they are computed
//    conservatively: a pivot is dropped only when the test holds with margin.
#include "common.h"

namespace grng {

namespace {

// Exact truth of sqrt(a) + c < sqrt(b) for grid integers a, b < 2^53 and
// 0 <= c < 2^27: needs c^2 < b, T = b + c^2 - a > 0 and 4 c^2 b < T^2.
__device__ inline bool exact_sqrt_plus_lt(uint64_t a, uint64_t c, uint64_t b) {
    const uint64_t cc = c * c;
    if (cc >= b) return false;
    const int64_t t = (int64_t)(b + cc) - (int64_t)a;
    if (t <= 0) return false;
    const uint64_t ut = (uint64_t)t;
    const uint64_t thi = __umul64hi(ut, ut), tlo = ut * ut;          // T^2
    const uint64_t phi0 = __umul64hi(cc, b), plo0 = cc * b;         // c^2 b
    const uint64_t phi = (phi0 << 2) | (plo0 >> 62), plo = plo0 << 2;  // 4 c^2 b (< 2^110)
    return phi < thi || (phi == thi && plo < tlo);
}

__device__ inline uint64_t grid_int(double v, double scale2) { return (uint64_t)(v * scale2); }

// Side test "dk + c < dij" with a float64 screen and exact fallback.
__device__ inline bool side_lt(double dk, double c, double dij, double d2k, int64_t ci, double d2ij, double s2,
                               uint32_t &rechecks) {
    const double diff = (dk + c) - dij;
    const double tol = 1e-12 * (dk + c + dij);
    if (diff < -tol) return true;
    if (diff > tol) return false;
    ++rechecks;
    return exact_sqrt_plus_lt(grid_int(d2k, s2), (uint64_t)ci, grid_int(d2ij, s2));
}

// One wave per (row i, 64 consecutive columns j); only j > i is tested.
// isnew (pivots added to a built layer, or null): a pair of two old pivots was
// linked before the addition, so only the new pivots (listed first in
// wfirst) can block it (the pivot-level Stage VII); other pairs test every
// witness.
__global__ __launch_bounds__(256) void k_grng_layer(int64_t m, const double *dpp, const double *dpp2,
                                                    const double *rad, const int64_t *radi, double s2,
                                                    const uint64_t *cand_bits, int32_t words,
                                                    const int32_t *wfirst, int64_t nfirst, const uint8_t *isnew,
                                                    uint64_t *bits, unsigned long long *counters) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t i = wave / words;
    const int32_t wj = (int32_t)(wave % words);
    if (i >= m) return;
    const int64_t j = (int64_t)wj * 64 + lane;
    bool active = j > i && j < m;
    if (active && cand_bits) active = (cand_bits[i * words + wj] >> lane) & 1ull;
    const double ri = active ? rad[i] : 0.0, rj = active ? rad[j] : 0.0;
    const int64_t rii = active ? radi[i] : 0, rji = active ? radi[j] : 0;
    const double dij = active ? dpp[i * m + j] : 0.0, d2ij = active ? dpp2[i * m + j] : 0.0;
    const double c1 = 2.0 * ri + rj, c2 = ri + 2.0 * rj;
    const int64_t c1i = 2 * rii + rji, c2i = rii + 2 * rji;
    const bool oldpair = isnew && active && !isnew[i] && !isnew[j];
    bool linked = active, live = active;   // live: still testing witnesses
    uint32_t tests = 0, rechecks = 0;
    const int64_t total = nfirst + m;
    for (int64_t s = 0; s < total; ++s) {
        if (s == nfirst && oldpair) live = false;
        if (!__ballot(live)) break;
        const int64_t k = s < nfirst ? wfirst[s] : s - nfirst;
        if (!live || k == i || k == j) continue;
        ++tests;
        // Cheap exact pre-test on squared distances: dk + c < dij needs dk^2 < dij^2.
        const double d2ki = dpp2[k * m + i], d2kj = dpp2[k * m + j];
        if (d2ki >= d2ij || d2kj >= d2ij) continue;
        if (side_lt(dpp[k * m + i], c1, dij, d2ki, c1i, d2ij, s2, rechecks) &&
            side_lt(dpp[k * m + j], c2, dij, d2kj, c2i, d2ij, s2, rechecks))
            linked = live = false;
    }
    const uint64_t word = __ballot(linked);
    if (lane == 0) bits[i * words + wj] = word;
    for (int o = 32; o > 0; o >>= 1) {
        tests += __shfl_xor(tests, o, kWave);
        rechecks += __shfl_xor(rechecks, o, kWave);
    }
    if (lane == 0) {
        atomicAdd(&counters[C_WTEST], (unsigned long long)tests);
        atomicAdd(&counters[C_RECHECK], (unsigned long long)rechecks);
    }
}

// Candidate pairs after pivots were added to a layer (m1 pivots, positions
// of the merged ascending id list): every pair with a new pivot, and the
// pairs of old pivots that were linked (adding witnesses can only unlink).
// oldpos[i]: the old position of pivot i, or -1 for a new one.
__global__ void k_insert_candidates(int64_t m1, int32_t words1, const int32_t *oldpos, const uint64_t *old_bits,
                                    int32_t words0, uint64_t *cand) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= m1 * (int64_t)words1) return;
    const int64_t i = e / words1;
    const int32_t w = (int32_t)(e % words1);
    const int32_t oi = oldpos[i];
    uint64_t acc = 0;
    for (int b = 0; b < 64; ++b) {
        const int64_t j = (int64_t)w * 64 + b;
        if (j >= m1) break;
        if (j == i) continue;
        const int32_t oj = oldpos[j];
        const bool c = oi < 0 || oj < 0 || ((old_bits[(int64_t)oi * words0 + (oj >> 6)] >> (oj & 63)) & 1ull);
        acc |= (uint64_t)c << b;
    }
    cand[e] = acc;
}

// Mirror the upper triangle: bit (j, i) = bit (i, j) for i < j.
__global__ void k_symmetrize(int64_t m, int32_t words, uint64_t *bits) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= m * (int64_t)words) return;
    const int64_t j = e / words;
    const int32_t wi = (int32_t)(e % words);
    uint64_t acc = 0;
    for (int b = 0; b < 64; ++b) {
        const int64_t i = (int64_t)wi * 64 + b;
        if (i >= j) break;
        acc |= ((bits[i * words + (j >> 6)] >> (j & 63)) & 1ull) << b;
    }
    // Words entirely below the diagonal take only the mirrored bits; the word
    // holding the diagonal keeps its upper part.
    const int64_t lo = (int64_t)wi * 64;
    if (lo + 63 < j) {
        bits[e] = acc;
    } else if (lo <= j) {
        const int sh = (int)(j - lo);
        const uint64_t keep = sh == 63 ? 0ull : (~0ull << (sh + 1));
        bits[e] = (bits[e] & keep) | acc;
    }
}

// Relative pivot domain (Section 3): fine pivot f is a child of coarse pivot c
// iff r_c - r_f >= 0 and d(c, f) <= r_c - r_f, i.e. d^2 <= (r_c - r_f)^2 exactly.
__global__ void k_relative_parents(int64_t mc, const int32_t *cpos, const double *dpp2f, int64_t mf,
                                   const double *radc, const double *radf, uint64_t *pbits, int32_t cwords) {
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= mf) return;
    for (int32_t w = 0; w < cwords; ++w) {
        uint64_t acc = 0;
        for (int b = 0; b < 64; ++b) {
            const int64_t c = (int64_t)w * 64 + b;
            if (c >= mc) break;
            const double slack = radc[c] - radf[f];   // exact: both on the grid, < 2^25 units
            if (slack >= 0.0 && dpp2f[(int64_t)cpos[c] * mf + f] <= slack * slack) acc |= 1ull << b;
        }
        pbits[f * cwords + w] = acc;
    }
}

// Fine pair (i, j) stays a candidate iff every coarse parent a of i and b of j
// has a == b or a GRNG link (Section 3, Theorem 2).
__global__ void k_guided_candidates(int64_t mf, const uint64_t *pbits, int32_t cwords, const uint64_t *cbits,
                                    int64_t mc, uint64_t *cand, int32_t fwords) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t i = wave / fwords;
    const int32_t wj = (int32_t)(wave % fwords);
    if (i >= mf) return;
    const int64_t j = (int64_t)wj * 64 + lane;
    bool ok = j < mf && j != i;
    if (ok) {
        for (int32_t w = 0; w < cwords && ok; ++w) {
            uint64_t allowed = ~0ull;   // coarse pivots b allowed for the parents of j
            // allowed_w = AND over parents a of i of (G_c[a] | {a}) restricted to word w
            for (int32_t wa = 0; wa < cwords; ++wa) {
                uint64_t pw = pbits[i * cwords + wa];
                while (pw) {
                    const int b = __ffsll((long long)pw) - 1;
                    pw &= pw - 1;
                    const int64_t a = (int64_t)wa * 64 + b;
                    uint64_t row = cbits[a * cwords + w];
                    if ((a >> 6) == w) row |= 1ull << (a & 63);
                    allowed &= row;
                }
            }
            if (pbits[j * cwords + w] & ~allowed) ok = false;
        }
    }
    const uint64_t word = __ballot(ok);
    if (lane == 0) cand[i * fwords + wj] = word;
}

// Wave per point (original order): parent count, nearest pivot, its distance^2.
__global__ __launch_bounds__(256) void k_point_pass1(int64_t n, int64_t m, const double *dxp, const double *rad,
                                                     int32_t *home, double *d2home, int32_t *npar, int32_t *second) {
    const int lane = threadIdx.x & 63;
    const int64_t x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= n) return;
    int cnt = 0;
    double best = INFINITY, best2 = INFINITY;   // nearest and second-nearest pivot
    int64_t bk = m, bk2 = m;
    for (int64_t k = lane; k < m; k += 64) {
        const double d2 = dxp[x * m + k];
        const double r = rad[k];
        if (d2 <= r * r) ++cnt;   // exact: r*r is exact on the grid
        if (d2 < best) {
            best2 = best; bk2 = bk;
            best = d2; bk = k;
        } else if (d2 < best2) {
            best2 = d2; bk2 = k;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, kWave);
        const double ob = __shfl_xor(best, o, kWave), ob2 = __shfl_xor(best2, o, kWave);
        const int64_t ok = __shfl_xor(bk, o, kWave), ok2 = __shfl_xor(bk2, o, kWave);
        // merge two (best, second) lists, ties by pivot index
        const bool mine = best < ob || (best == ob && bk < ok);
        const double w1 = mine ? best : ob, l1 = mine ? ob : best, s1 = mine ? best2 : ob2;
        const int64_t wk = mine ? bk : ok, lk = mine ? ok : bk, sk = mine ? bk2 : ok2;
        const bool lose = l1 < s1 || (l1 == s1 && lk < sk);
        best = w1; bk = wk;
        best2 = lose ? l1 : s1; bk2 = lose ? lk : sk;
    }
    if (lane == 0) {
        home[x] = (int32_t)bk;
        d2home[x] = best;
        npar[x] = cnt;
        if (second) second[x] = bk2 < m ? (int32_t)bk2 : (int32_t)bk;
    }
}

__global__ void k_group_radius(int64_t n, const int32_t *home, const double *d2home, unsigned long long *d2vor,
                               int32_t *gcount) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x >= n) return;
    atomicMax(&d2vor[home[x]], (unsigned long long)__double_as_longlong(d2home[x]));
    atomicAdd(&gcount[home[x]], 1);
}

// Exact domain parents of each point (Section 1, pivot domain equation), in
// pivot order; one wave per point in home order.
__global__ __launch_bounds__(256) void k_parents(int64_t n, int64_t m, const int32_t *__restrict__ perm,
                                                 const double *__restrict__ dxp, const double *__restrict__ rad,
                                                 const int64_t *__restrict__ par_off, int32_t *__restrict__ par_idx) {
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double *row = dxp + (int64_t)perm[i] * m;
    int64_t pw = par_off[i];
    for (int64_t k0 = 0; k0 < m; k0 += 64) {
        const int64_t k = k0 + lane;
        bool par = false;
        if (k < m) {
            const double r = rad[k];
            par = row[k] <= r * r;   // exact: r*r is exact on the grid
        }
        const uint64_t pm = __ballot(par);
        if (par) par_idx[pw + __popcll(pm & ((1ull << lane) - 1ull))] = (int32_t)k;
        pw += __popcll(pm);
    }
}

// Shifted pivot distances for the virtual-pivot test, rounded up:
// bd[k][j] = d(p_j, p_k) + r_j and bv[k][j] = d(p_j, p_k) + cellradius_j.
__global__ void k_shifted_pivot_dists(int64_t m, const double *dpp, const double *rad, const double *dvor,
                                      float *bd, float *bv) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= m * m) return;
    const int64_t j = e % m;
    const double d = dpp[e] * (1.0 + 1e-15);
    bd[e] = __double2float_ru(d + rad[j]);
    bv[e] = __double2float_ru(d + dvor[j]);
}

// Virtual-pivot GRNG bitsets of every point as a (min, max) matrix product.
// For point x and pivot j with radius rad_j (Section 2, Proposition 1 with x
// as a zero-radius pivot), j is dropped iff some pivot k has
//     d(x,p_k) + rad_j < d(x,p_j)  and  d(p_j,p_k) + 2 rad_j < d(x,p_j),
// i.e. iff  C[x][j] + rad_j < d(x,p_j)  with
//     C[x][j] = min_k max(d(x,p_k), d(p_j,p_k) + rad_j).
// Each workgroup computes a 64-point x 64-pivot tile of C for both radius
// choices (domain radius and home-cell radius), 4 x 4 entries per thread,
// with 32-pivot slices of both operands staged in LDS.  Operands are float32
// rounded up, so C is an upper bound and dropping j stays sound (a dropped
// pivot is dropped by the exact test too).
constexpr int kVT_X = 64, kVT_J = 64, kVT_K = 32;
__device__ inline uint32_t vt_max(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ inline uint32_t vt_min3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t m = a < b ? a : b;
    return m < c ? m : c;
}

// d(x, p_k) for the witness pivots of x's 64-point block (the kw pivots
// nearest to the home cell of the block's first point, or all pivots when
// kw == m), float32 rounded up, [n][kw]: gathered once per build so that the
// tile kernel streams contiguous rows instead of gathering scattered entries
// of D_XP for every pivot tile.
// Rows x0 .. x0 + rows - 1 (x0 a multiple of 64) into ax[0 .. rows * kw).
__global__ __launch_bounds__(256) void k_witness_dists(int64_t x0, int64_t rows, int64_t m,
                                                       const int32_t *__restrict__ perm, const double *__restrict__ dxp,
                                                       const int32_t *__restrict__ home,
                                                       const int32_t *__restrict__ wknn, int32_t kw,
                                                       float *__restrict__ ax) {
    const int64_t e = blockIdx.x * 256ll + threadIdx.x;
    if (e >= rows * kw) return;
    const int64_t i = x0 + e / kw;
    const int32_t k = (int32_t)(e % kw);
    const int32_t p = kw < m ? wknn[(int64_t)home[i / kVT_X * kVT_X] * kw + k] : k;
    ax[e] = __double2float_ru(sqrt(dxp[(int64_t)perm[i] * m + p]) * (1.0 + 1e-15));
}

// kCols: the cell-radius bits of listed pivots only (cols[0 .. ncols), any
// order, 64 per workgroup column), OR-ed into v_rows: an insertion that grew
// those cells' radius bounds.  A bit that was set stays set (sound: each
// computation only drops pivots that are provably not needed).
template <bool kCols>
__global__ __launch_bounds__(256) void k_vgrng_tiles(
    int64_t n, int64_t m, const int32_t *__restrict__ perm, const double *__restrict__ dxp,
    const float *__restrict__ bd, const float *__restrict__ bv, const double *__restrict__ rad,
    const double *__restrict__ dvor, const int32_t *__restrict__ gcount, const int64_t *__restrict__ par_off,
    const int32_t *__restrict__ par_idx, const uint64_t *__restrict__ layer_bits, int32_t words,
    const int32_t *__restrict__ home, const int32_t *__restrict__ wknn, int32_t kw, int64_t xbase,
    const float *__restrict__ ax, const int32_t *__restrict__ cols, int32_t ncols, uint64_t *__restrict__ g_rows,
    uint64_t *__restrict__ v_rows, unsigned long long *counters) {
    __shared__ __align__(16) float sA[kVT_X][kVT_K + 2];   // rows 8-byte aligned: pairs of k in one load
    __shared__ __align__(16) float sD[kCols ? 1 : kVT_K][kVT_J];
    __shared__ __align__(16) float sV[kVT_K][kVT_J];
    __shared__ int32_t sK[kVT_K];
    __shared__ int32_t sJ[kVT_J];
    __shared__ uint64_t sCand[kVT_X];
    __shared__ unsigned long long sG[kVT_X], sVb[kVT_X];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t x0 = xbase + blockIdx.x * (int64_t)kVT_X;   // ax holds rows from xbase on
    // pivot block: one 64-bit word of the bit rows, or 64 listed pivots
    const int32_t wj = kCols ? 0 : (int32_t)blockIdx.y;
    const int64_t j0 = (int64_t)wj * kVT_J;
    if (tid < kVT_J) {
        const int64_t c = (int64_t)blockIdx.y * kVT_J + tid;
        sJ[tid] = kCols ? (c < ncols ? cols[c] : -1) : (j0 + tid < m ? (int32_t)(j0 + tid) : -1);
    }
    if (!kCols && tid < kVT_X) {
        // Theorem 1 candidates: pivots linked to (or equal to) every parent of x.
        const int64_t i = x0 + tid;
        uint64_t c = 0;
        if (i < n) {
            c = ~0ull;
            for (int64_t t = par_off[i]; t < par_off[i + 1]; ++t) {
                const int32_t p = par_idx[t];
                uint64_t row = layer_bits[(int64_t)p * words + wj];
                if ((p >> 6) == wj) row |= 1ull << (p & 63);
                c &= row;
            }
        }
        sCand[tid] = c;
        sG[tid] = 0;
        sVb[tid] = 0;
    }
    // Operands are non-negative float32 values or +inf, whose bit patterns
    // order as unsigned integers: integer max and three-input min, no NaN
    // handling.
    uint32_t cD[4][4], cV[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) cD[r][c] = cV[r][c] = 0x7f800000u;
    // Witness pivots: the kw pivots nearest to the home cell of the block's
    // first point (in that order), or all of them when kw == m.  Any subset
    // of pivots gives a valid witness set: fewer witnesses only prune less.
    const int32_t *wk = kw < m ? wknn + (int64_t)home[x0] * kw : nullptr;
    for (int64_t k0 = 0; k0 < kw; k0 += kVT_K) {
        __syncthreads();
        if (tid < kVT_K) sK[tid] = k0 + tid < kw ? (wk ? wk[k0 + tid] : (int32_t)(k0 + tid)) : -1;
        __syncthreads();
        for (int e = tid; e < kVT_X * kVT_K; e += 256) {
            const int r = e / kVT_K, kk = e % kVT_K;
            const int64_t i = x0 + r;
            sA[r][kk] = (i < n && k0 + kk < kw) ? ax[(i - xbase) * kw + k0 + kk] : INFINITY;
        }
        for (int e = tid; e < kVT_K * kVT_J; e += 256) {
            const int kk = e / kVT_J, jj = e % kVT_J;
            const int32_t k = sK[kk], j = sJ[jj];
            const bool ok = k >= 0 && j >= 0;
            if (!kCols) sD[kk][jj] = ok ? bd[(int64_t)k * m + j] : INFINITY;
            sV[kk][jj] = ok ? bv[(int64_t)k * m + j] : INFINITY;
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < kVT_K; kk += 2) {
            // a thread's four columns are adjacent: one 16-byte load per row of
            // D and V, one 8-byte load per point row for two witnesses
            uint32_t a[2][4], d[2][4], v[2][4];
            for (int r = 0; r < 4; ++r) {
                const uint2 t = *reinterpret_cast<const uint2 *>(&sA[ty + 16 * r][kk]);
                a[0][r] = t.x;
                a[1][r] = t.y;
            }
            for (int h = 0; h < 2; ++h) {
                const uint4 tv = *reinterpret_cast<const uint4 *>(&sV[kk + h][4 * tx]);
                v[h][0] = tv.x; v[h][1] = tv.y; v[h][2] = tv.z; v[h][3] = tv.w;
                if (!kCols) {
                    const uint4 td = *reinterpret_cast<const uint4 *>(&sD[kk + h][4 * tx]);
                    d[h][0] = td.x; d[h][1] = td.y; d[h][2] = td.z; d[h][3] = td.w;
                }
            }
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    if (!kCols)
                        cD[r][c] = vt_min3(cD[r][c], vt_max(a[0][r], d[0][c]), vt_max(a[1][r], d[1][c]));
                    cV[r][c] = vt_min3(cV[r][c], vt_max(a[0][r], v[0][c]), vt_max(a[1][r], v[1][c]));
                }
        }
    }
    // Epilogue: keep bits.
    for (int r = 0; r < 4; ++r) {
        const int xr = ty + 16 * r;
        const int64_t i = x0 + xr;
        if (i >= n) continue;
        const double *row = dxp + (int64_t)perm[i] * m;
        for (int c = 0; c < 4; ++c) {
            const int jc = 4 * tx + c;
            const int32_t j = sJ[jc];
            if (j < 0) continue;
            const double dj = sqrt(row[j]) * (1.0 - 1e-15);
            const double rj = rad[j], vj = dvor[j];
            const double mj = 1e-6 * (dj + 3.0 * fmax(rj, vj)) + 1e-300;
            const bool candV = gcount[j] > 0;
            const bool keepV = candV && !((double)__uint_as_float(cV[r][c]) + vj < dj - mj);
            if (kCols) {
                if (keepV) atomicOr((unsigned long long *)&v_rows[i * words + (j >> 6)], 1ull << (j & 63));
                continue;
            }
            const bool candD = (sCand[xr] >> jc) & 1ull;
            const bool keepD = candD && !((double)__uint_as_float(cD[r][c]) + rj < dj - mj);
            if (keepD) atomicOr(&sG[xr], 1ull << jc);
            if (keepV) atomicOr(&sVb[xr], 1ull << jc);
        }
    }
    if (kCols) return;
    __syncthreads();
    if (tid < kVT_X && x0 + tid < n) {
        g_rows[(x0 + tid) * words + wj] = sG[tid];
        v_rows[(x0 + tid) * words + wj] = sVb[tid];
    }
    if (tid == 0) {
        const int64_t rows = (n - x0) < kVT_X ? (n - x0) : kVT_X;
        const int64_t ncol = (m - j0) < kVT_J ? (m - j0) : kVT_J;
        atomicAdd(&counters[C_WTEST], (unsigned long long)(2 * rows * ncol * kw));
    }
}

}  // namespace

void launch_grng_layer(hipStream_t s, int64_t m, const double *dpp, const double *dpp2, const double *rad,
                       const int64_t *radi, int32_t q, const uint64_t *cand_bits, int32_t words,
                       const int32_t *witness_first, int64_t nfirst, uint64_t *bits, uint64_t *counters,
                       const uint8_t *isnew) {
    if (m == 0) return;
    const double s2 = ldexp(1.0, 2 * q);
    const int64_t waves = m * words;
    k_grng_layer<<<(unsigned)div_up(waves, 4), 256, 0, s>>>(m, dpp, dpp2, rad, radi, s2, cand_bits, words,
                                                            witness_first, nfirst, isnew, bits,
                                                            (unsigned long long *)counters);
    GRNG_LAUNCHED();
    const int64_t e = m * words;
    k_symmetrize<<<(unsigned)div_up(e, 256), 256, 0, s>>>(m, words, bits);
    GRNG_LAUNCHED();
}

void launch_insert_candidates(hipStream_t s, int64_t m1, int32_t words1, const int32_t *oldpos,
                              const uint64_t *old_bits, int32_t words0, uint64_t *cand) {
    if (m1 == 0) return;
    k_insert_candidates<<<(unsigned)div_up(m1 * words1, 256), 256, 0, s>>>(m1, words1, oldpos, old_bits, words0,
                                                                          cand);
    GRNG_LAUNCHED();
}

void launch_relative_parents(hipStream_t s, int64_t mc, const int32_t *coarse_pos_in_fine, const double *dpp2_fine,
                             int64_t mf, const double *rad_c, const double *rad_f, uint64_t *parent_bits,
                             int32_t cwords) {
    if (mf == 0) return;
    k_relative_parents<<<(unsigned)div_up(mf, 128), 128, 0, s>>>(mc, coarse_pos_in_fine, dpp2_fine, mf, rad_c, rad_f,
                                                                 parent_bits, cwords);
    GRNG_LAUNCHED();
}

void launch_guided_candidates(hipStream_t s, int64_t mf, const uint64_t *parent_bits, int32_t cwords,
                              const uint64_t *coarse_bits, int64_t mc, uint64_t *cand_bits, int32_t fwords) {
    if (mf == 0) return;
    const int64_t waves = mf * fwords;
    k_guided_candidates<<<(unsigned)div_up(waves, 4), 256, 0, s>>>(mf, parent_bits, cwords, coarse_bits, mc,
                                                                   cand_bits, fwords);
    GRNG_LAUNCHED();
}

void launch_point_pass1(hipStream_t s, int64_t n, int64_t m, const double *dxp, const double *rad,
                        int32_t *home, double *d2home, int32_t *npar, int32_t *second) {
    if (n == 0) return;
    k_point_pass1<<<(unsigned)div_up(n, 4), 256, 0, s>>>(n, m, dxp, rad, home, d2home, npar, second);
    GRNG_LAUNCHED();
}

void launch_group_radius(hipStream_t s, int64_t n, const int32_t *home, const double *d2home, uint64_t *d2vor_bits,
                         int32_t *gcount) {
    if (n == 0) return;
    k_group_radius<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, home, d2home, (unsigned long long *)d2vor_bits,
                                                            gcount);
    GRNG_LAUNCHED();
}

void launch_parents(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp, const double *rad,
                    const int64_t *par_off, int32_t *par_idx) {
    if (n == 0) return;
    k_parents<<<(unsigned)div_up(n, 4), 256, 0, s>>>(n, m, perm, dxp, rad, par_off, par_idx);
    GRNG_LAUNCHED();
}

void launch_shifted_pivot_dists(hipStream_t s, int64_t m, const double *dpp, const double *rad, const double *dvor,
                                float *bd, float *bv) {
    if (m == 0) return;
    k_shifted_pivot_dists<<<(unsigned)div_up(m * m, 256), 256, 0, s>>>(m, dpp, rad, dvor, bd, bv);
    GRNG_LAUNCHED();
}

void launch_vgrng(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp, const float *bd,
                  const float *bv, const double *rad, const double *dvor, const int32_t *gcount, const int64_t *par_off,
                  const int32_t *par_idx, const uint64_t *layer_bits, int32_t words, const int32_t *home,
                  const int32_t *wknn, int32_t kw, uint64_t *g_rows, uint64_t *v_rows, uint64_t *counters,
                  const int32_t *cols, int32_t ncols) {
    if (n == 0 || (cols && ncols == 0)) return;
    require(kw >= 1 && kw <= m, GRNG_EINVAL, "witness pivot count out of range");
    require(div_up(m, kVT_J) <= 65535, GRNG_EINVAL, "pivot layer too large for the virtual-pivot kernel");
    // point rows per pass: at most 2^19, whose witness distances take at most 4 GiB
    const int64_t chunk = std::min<int64_t>(
        std::min<int64_t>(div_up(n, kVT_X) * kVT_X, (int64_t)1 << 19),
        std::max<int64_t>(kVT_X, (((int64_t)1 << 30) / kw) / kVT_X * kVT_X));
    DevBuf ax;
    ax.alloc(4 * (size_t)chunk * (size_t)kw);
    for (int64_t x0 = 0; x0 < n; x0 += chunk) {
        const int64_t rows = std::min<int64_t>(chunk, n - x0);
        k_witness_dists<<<(unsigned)div_up(rows * kw, 256), 256, 0, s>>>(x0, rows, m, perm, dxp, home, wknn, kw,
                                                                         ax.as<float>());
        GRNG_LAUNCHED();
        dim3 g((unsigned)div_up(rows, kVT_X), (unsigned)div_up(cols ? ncols : m, kVT_J));
        if (cols)
            k_vgrng_tiles<true><<<g, 256, 0, s>>>(n, m, perm, dxp, bd, bv, rad, dvor, gcount, par_off, par_idx,
                                                  layer_bits, words, home, wknn, kw, x0, ax.as<float>(), cols, ncols,
                                                  g_rows, v_rows, (unsigned long long *)counters);
        else
            k_vgrng_tiles<false><<<g, 256, 0, s>>>(n, m, perm, dxp, bd, bv, rad, dvor, gcount, par_off, par_idx,
                                                   layer_bits, words, home, wknn, kw, x0, ax.as<float>(), nullptr, 0,
                                                   g_rows, v_rows, (unsigned long long *)counters);
        GRNG_LAUNCHED();
    }
}

}  // namespace grng
