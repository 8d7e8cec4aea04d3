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
//    witnesses), nearest pivots for Stage IV, and two virtual-pivot GRNG
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
__global__ __launch_bounds__(256) void k_grng_layer(int64_t m, const double *dpp, const double *dpp2,
                                                    const double *rad, const int64_t *radi, double s2,
                                                    const uint64_t *cand_bits, int32_t words,
                                                    const int32_t *wfirst, int64_t nfirst, uint64_t *bits,
                                                    unsigned long long *counters) {
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
    bool linked = active;
    uint32_t tests = 0, rechecks = 0;
    const int64_t total = nfirst + m;
    for (int64_t s = 0; s < total; ++s) {
        if (!__ballot(linked)) break;
        const int64_t k = s < nfirst ? wfirst[s] : s - nfirst;
        if (!linked || k == i || k == j) continue;
        ++tests;
        const double dki = dpp[k * m + i];
        const double dkj = dpp[k * m + j];
        // Cheap exact pre-test: dk + c < dij needs dk < dij.
        if (dki >= dij || dkj >= dij) continue;
        if (side_lt(dki, c1, dij, dpp2[k * m + i], c1i, d2ij, s2, rechecks) &&
            side_lt(dkj, c2, dij, dpp2[k * m + j], c2i, d2ij, s2, rechecks))
            linked = false;
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
            uint64_t pi = pbits[i * cwords + 0];
            (void)pi;
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
                                                     int32_t *home, double *d2home, int32_t *npar) {
    const int lane = threadIdx.x & 63;
    const int64_t x = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= n) return;
    int cnt = 0;
    double best = INFINITY;
    int64_t bk = m;
    for (int64_t k = lane; k < m; k += 64) {
        const double d2 = dxp[x * m + k];
        const double r = rad[k];
        if (d2 <= r * r) ++cnt;   // exact: r*r is exact on the grid
        if (d2 < best) { best = d2; bk = k; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, kWave);
        const double ob = __shfl_xor(best, o, kWave);
        const int64_t ok = __shfl_xor(bk, o, kWave);
        if (ob < best || (ob == best && ok < bk)) { best = ob; bk = ok; }
    }
    if (lane == 0) {
        home[x] = (int32_t)bk;
        d2home[x] = best;
        npar[x] = cnt;
    }
}

__global__ void k_group_radius(int64_t n, const int32_t *home, const double *d2home, unsigned long long *d2vor,
                               int32_t *gcount) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x >= n) return;
    atomicMax(&d2vor[home[x]], (unsigned long long)__double_as_longlong(d2home[x]));
    atomicAdd(&gcount[home[x]], 1);
}

// Upper bound of sqrt for conservative pruning bounds.
__device__ inline double sqrt_up(double v) { return sqrt(v) * (1.0 + 1e-15); }

// Wave per point in home order.  LDS: sorted distances to pivots and indices.
__global__ __launch_bounds__(64) void k_point_pass2(int64_t n, int64_t m, int32_t mpow2, const int32_t *perm,
                                                    const double *dxp, const double *rad, const double *dpp,
                                                    const uint64_t *layer_bits, int32_t words,
                                                    const double *dvor, const int32_t *gcount,
                                                    const int64_t *par_off, int32_t *par_idx, int32_t K,
                                                    int32_t *knn, uint64_t *g_rows, uint64_t *v_rows,
                                                    unsigned long long *counters) {
    extern __shared__ unsigned char smem[];
    double *key = (double *)smem;
    int32_t *kid = (int32_t *)(key + mpow2);
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const int64_t x = perm[i];
    const double *row = dxp + x * m;
    // Parents (exact) in pivot order, and the distance table.
    int64_t pw = par_off[i];
    for (int64_t k0 = 0; k0 < mpow2; k0 += 64) {
        const int64_t k = k0 + lane;
        bool par = false;
        if (k < m) {
            const double d2 = row[k];
            const double r = rad[k];
            par = d2 <= r * r;
            key[k] = sqrt(d2);
            kid[k] = (int32_t)k;
        } else if (k < mpow2) {
            key[k] = INFINITY;
            kid[k] = (int32_t)k;
        }
        const uint64_t pm = __ballot(par);
        if (par) par_idx[pw + __popcll(pm & ((1ull << lane) - 1ull))] = (int32_t)k;
        pw += __popcll(pm);
    }
    __syncthreads();
    // Bitonic sort of (distance, index) ascending.
    for (int32_t size = 2; size <= mpow2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t t = lane; t < (mpow2 >> 1); t += 64) {
                const int32_t lo = 2 * t - (t & (stride - 1));
                const int32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double a = key[lo], b = key[hi];
                const int32_t ia = kid[lo], ib = kid[hi];
                const bool gt = a > b || (a == b && ia > ib);
                if (gt == up) {
                    key[lo] = b; key[hi] = a;
                    kid[lo] = ib; kid[hi] = ia;
                }
            }
            __syncthreads();
        }
    }
    for (int32_t t = lane; t < K; t += 64) knn[i * K + t] = t < m ? kid[t] : kid[0];
    const int64_t p0 = par_off[i], p1 = par_off[i + 1];
    uint32_t tests = 0;
    for (int32_t w = 0; w < words; ++w) {
        const int64_t j = (int64_t)w * 64 + lane;
        const bool valid = j < m;
        // Candidates for GRNG(x) (Theorem 1): linked to, or equal to, every parent.
        bool candD = valid;
        for (int64_t t = p0; t < p1 && candD; ++t) {
            const int32_t p = par_idx[t];
            candD = (p == j) || ((layer_bits[(int64_t)p * words + w] >> lane) & 1ull);
        }
        bool candV = valid && gcount[j] > 0;
        const double dj = valid ? sqrt(row[j]) : 0.0;
        const double rj = valid ? rad[j] : 0.0;
        const double vj = valid ? dvor[j] : 0.0;
        const double mj = 1e-12 * (dj + 3.0 * fmax(rj, vj)) + 1e-300;
        // Prune when some pivot k lies in the G-lune of (x, 0) and (p_j, radius):
        //   d(x,k) + rad < d(x,j)  and  d(j,k) + 2 rad < d(x,j), with margin.
        const double tD = dj - rj - mj, tV = dj - vj - mj;
        bool liveD = candD && tD > 0.0, liveV = candV && tV > 0.0;
        bool keepD = candD, keepV = candV;
        for (int32_t s = 0; s < m; ++s) {
            const double dk = key[s];
            liveD = liveD && keepD && dk < tD;
            liveV = liveV && keepV && dk < tV;
            if (!__ballot(liveD || liveV)) break;
            if (!(liveD || liveV)) continue;
            const int32_t k = kid[s];
            const double djk = dpp[(int64_t)k * m + j];
            ++tests;
            if (liveD && djk + 2.0 * rj < dj - mj) keepD = false;
            if (liveV && djk + 2.0 * vj < dj - mj) keepV = false;
        }
        const uint64_t gd = __ballot(keepD), gv = __ballot(keepV);
        if (lane == 0) {
            g_rows[i * words + w] = gd;
            v_rows[i * words + w] = gv;
        }
    }
    for (int o = 32; o > 0; o >>= 1) tests += __shfl_xor(tests, o, kWave);
    if (lane == 0) atomicAdd(&counters[C_WTEST], (unsigned long long)tests);
}

}  // namespace

void launch_grng_layer(hipStream_t s, int64_t m, const double *dpp, const double *dpp2, const double *rad,
                       const int64_t *radi, int32_t q, const uint64_t *cand_bits, int32_t words,
                       const int32_t *witness_first, int64_t nfirst, uint64_t *bits, uint64_t *counters) {
    if (m == 0) return;
    const double s2 = ldexp(1.0, 2 * q);
    const int64_t waves = m * words;
    k_grng_layer<<<(unsigned)div_up(waves, 4), 256, 0, s>>>(m, dpp, dpp2, rad, radi, s2, cand_bits, words,
                                                            witness_first, nfirst, bits,
                                                            (unsigned long long *)counters);
    GRNG_LAUNCHED();
    const int64_t e = m * words;
    k_symmetrize<<<(unsigned)div_up(e, 256), 256, 0, s>>>(m, words, bits);
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
                        int32_t *home, double *d2home, int32_t *npar) {
    if (n == 0) return;
    k_point_pass1<<<(unsigned)div_up(n, 4), 256, 0, s>>>(n, m, dxp, rad, home, d2home, npar);
    GRNG_LAUNCHED();
}

void launch_group_radius(hipStream_t s, int64_t n, const int32_t *home, const double *d2home, uint64_t *d2vor_bits,
                         int32_t *gcount) {
    if (n == 0) return;
    k_group_radius<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, home, d2home, (unsigned long long *)d2vor_bits,
                                                            gcount);
    GRNG_LAUNCHED();
}

void launch_point_pass2(hipStream_t s, int64_t n, int64_t m, const int32_t *perm, const double *dxp,
                        const double *rad, const double *dpp, const uint64_t *layer_bits, int32_t words,
                        const double *dvor, const int32_t *gcount, const int64_t *par_off, int32_t *par_idx,
                        int32_t K, int32_t *knn, uint64_t *g_rows, uint64_t *v_rows, uint64_t *counters) {
    if (n == 0) return;
    int32_t mp = 64;
    while (mp < m) mp <<= 1;
    const size_t lds = (size_t)mp * (sizeof(double) + sizeof(int32_t));
    require(lds <= 160 * 1024, GRNG_EINVAL, "pivot layer too large for the per-point pass");
    k_point_pass2<<<(unsigned)n, 64, lds, s>>>(n, m, mp, perm, dxp, rad, dpp, layer_bits, words, dvor, gcount,
                                               par_off, par_idx, K, knn, g_rows, v_rows,
                                               (unsigned long long *)counters);
    GRNG_LAUNCHED();
}

}  // namespace grng
