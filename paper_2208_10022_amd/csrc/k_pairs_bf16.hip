// Candidate pairs guided by the pivot layer (Section 2, Stages IV-V) with
// bf16 matrix-core distance tiles and a per-tile error bound.
//
// Same work as k_pairs_tiled (one 8-wave workgroup per 64 x 64 tile pair, the
// tile-pair records of k_pair_masks, survivors to the exhaustive scan), but
// the distance tiles D(T,U), D(T,P), D(U,P), D(T,T), D(U,U) come from
// v_mfma_f32_16x16x32_bf16 with float32 accumulation instead of float64
// MFMA, and every certificate carries an explicit error bound.
//
// Centring.  Tile T (home cell a) is centred at its cell pivot p_a, tile U
// (home cell b) at p_b; the pivot witnesses are centred twice, at p_a (for
// D(T,P)) and at p_b (for D(U,P)).  With a = x - p_a, b = y - p_b:
//     d^2(x,y) = |x - p_b|^2 + |y - p_a|^2 - |p_a - p_b|^2 - 2 a.b,
// so the one inexact term, a.b, has operands no longer than the cell radii.
// The three squared distances are exact in float64 (grid contract): |y -
// p_a|^2 from U's float32 rows at load time, |x - p_b|^2 from T's centred
// rows (stored exactly as three bf16 parts) whenever b changes, |p_a - p_b|^2
// from the two pivots' rows.
//
// Split.  A centred value v = fl32(x - c) is stored as bf16 parts hi =
// bf16(v), lo = bf16(v - hi) (v - hi is exact in float32) and, for T, lo2 =
// bf16(v - hi - lo), which makes hi + lo + lo2 = v exactly.  hi + lo is within
// 2^-16 (1 + 2^-7) |v| of v, and v within 2^-24 |x - c| of x - c.
//
// Error bound.  A dot product a.b is the sum of three MFMA products hi.hi +
// hi.lo + lo.hi (bf16 x bf16 products are exact in float32), with error at
// most eps |a| |b|, eps = 3.1 * 2^-16 + 1.02 * gamma(3 kp), gamma(n) = n u /
// (1 - n u), u = 2^-24: twice the split error, the dropped lo.lo term, and
// float32 rounding at every accumulation step; eps < 7.2e-5 for kp <= 128.
// The squared distance is formed in float32 from float32 roundings of the
// exact terms; each rounding and operation adds at most u times the
// magnitude of its operands.  So an entry's error is at most
//     2 eps R_X R_Y + 6 u S,
// R_X the largest |x - c| of the block's rows (rounded up) and S the largest
// sum of the magnitudes of an entry's exact terms; bounds are computed per
// tile pair and block of entries.
//
// Certificates (a witness z kills (x, y) when max(d(x,z), d(y,z)) < d(x,y)):
//   Stage IV  min over pivots of max(d2_est(x,p), d2_est(y,p)) < d2_est(x,y) - tau4,
//             tau4 = E_TU + max(E_TP, E_UP);
//   Stage V   max(d2_est(x,z), d2_est(y,z)) < d2_est(x,y) - tau5 for z in T or U,
//             tau5 = E_TU + max(E_TT, E_TU, E_UU).
// Each threshold is rounded down, so a kill is a proof.  Every other pair
// survives, among them those whose best witness lies within the bound of a
// tie (counted as uncertain): the exhaustive scan re-decides all survivors
// exactly (float32 screen, float64 re-decision), so no verdict depends on
// rounding.  Survivors leave this kernel without their squared distance;
// k_pairs_exact_d2 computes it exactly in float64 afterwards.
#include "common.h"
#include "dev_util.h"

namespace grng {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBThreads = 512;            // 8 waves per tile pair
constexpr int kBWaves = kBThreads / 64;
constexpr int kKb = 32;                   // K of one v_mfma_f32_16x16x32_bf16
constexpr int kMaxKp = 128;               // largest padded dimension (LDS rows)
constexpr float kEps = 7.2e-5f;           // dot-product error factor eps (kp <= 128, see above)
constexpr float kU6 = 6.0f * 0x1p-24f;    // six float32 roundings per entry

// bf16 row stride for kp padded coordinates: 16 spare bytes, so that the 16
// rows one MFMA operand load touches start in different LDS banks.
__host__ __device__ inline int bstride(int kp) { return kp + 8; }

// LDS layout (bytes): T rows (hi, lo, lo2), U rows (hi, lo), masks, Stage
// IV survivor bits (two sets, by iteration parity), per-row terms, D(T,U)
// (float32), D(T,T) (16-bit upper bounds, kept while consecutive tile pairs
// share T), D(U,U) (16-bit upper bounds), then the pivot rows (twice
// centred) and pivot distances of Stages I-IV.  A Stage V witness entry
// only needs to bound the estimate from above: the kill test stays a proof.
// Nothing Stage V reads is written before the next tile pair's second
// barrier, so no barrier ends Stage V.
struct BLayout {
    int kp, ks;
    size_t rows, fixed, dmat, dtt, phase_a, region, total;
};

constexpr int kTerms = 4 * kTile + 2 * kPiv + 16;   // floats of per-row terms and tile radii

__host__ __device__ inline BLayout blayout(int kp) {
    BLayout L;
    L.kp = kp;
    L.ks = bstride(kp);
    L.rows = 5 * (size_t)kTile * L.ks * 2;                          // hT, lT, l2T, hU, lU
    L.fixed = L.rows + 8 * 4 * (size_t)kTile + 4 * (size_t)kTerms;  // masks, survivor bits, terms
    L.dmat = 4 * (size_t)kTile * kDl;
    L.dtt = 2 * (size_t)kTile * kDl;
    L.phase_a = 4 * (size_t)kPiv * L.ks * 2 + 4 * 2 * (size_t)kTile * kXs;   // pivot rows x2, XP, YP
    L.region = L.phase_a;
    L.total = L.fixed + L.dmat + 2 * L.dtt + L.region;   // D(T,T) and D(U,U) take dtt bytes each
    return L;
}

// Directed rounding for non-negative float32 operands: the round-to-nearest
// result moved one unit in the last place up (an upper bound of the exact
// value) or down (a lower bound; results <= 0 are left as they are, and a
// threshold <= 0 never certifies anything).
__device__ inline float up_ulp(float v) { return v > 0.f ? __uint_as_float(__float_as_uint(v) + 1u) : 0x1p-149f; }
__device__ inline float add_up(float a, float b) { return up_ulp(a + b); }
__device__ inline float mul_up(float a, float b) { return up_ulp(a * b); }
__device__ inline float sub_dn(float a, float b) {
    const float r = a - b;
    return r > 0.f ? __uint_as_float(__float_as_uint(r) - 1u) : r;
}

// Centre, split and store rows [0, nrows) of a float32 point set (row r at
// src + r * dp; zero rows past len) into bf16 parts hi, lo and optionally
// lo2 (null: not stored).  Per row: nrm[r] = fl32(|x - cen|^2) and, when far
// is given, far[r] = fl32(|x - cen2|^2), both exact in float64 first; the
// largest |x - cen| (rounded up) goes to *rmax and the largest far[r]
// (rounded up) to *fmax.  Four adjacent threads per row, each taking 8
// consecutive coordinates of every 32; t in [0, nthr), nthr a multiple of 4.
__device__ inline void load_split(__bf16 *hi, __bf16 *lo, __bf16 *lo2, float *nrm, float *far,
                                  unsigned int *rmax, unsigned int *fmax, const float *__restrict__ src, int len,
                                  int nrows, int dp, int kp, int ks, const float *__restrict__ cen,
                                  const float *__restrict__ cen2, int t, int nthr) {
    for (int r = t >> 2; r < nrows; r += nthr >> 2) {
        double acc = 0.0, acc2 = 0.0;
        for (int c0 = 8 * (t & 3); c0 < kp; c0 += kKb) {
            bf16x8 h, l, l2;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int c = c0 + 4 * q;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f), w = v, w2 = v;
                if (r < len && c < dp) {
                    v = *reinterpret_cast<const float4 *>(src + (int64_t)r * dp + c);
                    w = *reinterpret_cast<const float4 *>(cen + c);
                    if (far) w2 = *reinterpret_cast<const float4 *>(cen2 + c);
                }
                const float xv[4] = {v.x, v.y, v.z, v.w}, cv[4] = {w.x, w.y, w.z, w.w},
                            c2[4] = {w2.x, w2.y, w2.z, w2.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float e = xv[k] - cv[k];
                    const __bf16 hb = (__bf16)e;
                    const float r1 = e - (float)hb;
                    const __bf16 lb = (__bf16)r1;
                    h[4 * q + k] = hb;
                    l[4 * q + k] = lb;
                    l2[4 * q + k] = (__bf16)(r1 - (float)lb);
                    const double f = (double)xv[k] - (double)cv[k];   // exact: grid values
                    acc = fma(f, f, acc);                             // exact: d (2 kmax)^2 < 2^53
                    const double g = (double)xv[k] - (double)c2[k];
                    acc2 = fma(g, g, acc2);
                }
            }
            *reinterpret_cast<bf16x8 *>(hi + r * ks + c0) = h;
            *reinterpret_cast<bf16x8 *>(lo + r * ks + c0) = l;
            if (lo2) *reinterpret_cast<bf16x8 *>(lo2 + r * ks + c0) = l2;
        }
        acc += __shfl_xor(acc, 1, kWave);   // the row's four threads are adjacent lanes
        acc += __shfl_xor(acc, 2, kWave);
        acc2 += __shfl_xor(acc2, 1, kWave);
        acc2 += __shfl_xor(acc2, 2, kWave);
        if ((t & 3) == 0) {
            nrm[r] = (float)acc;
            if (far) far[r] = (float)acc2;
            if (r < len) {
                atomicMax(rmax, __float_as_uint(__double2float_ru(sqrt(acc) * (1.0 + 0x1p-50))));
                if (far) atomicMax(fmax, __float_as_uint(__double2float_ru(acc2)));
            }
        }
    }
}

// |x - p_b|^2 for the rows of T from their exact centred parts (hi + lo +
// lo2 = fl32(x - p_a)) and p_a - p_b: float64, four threads per row; t in
// [0, nthr).  Where fl32(x - p_a) was rounded (|x - p_a| beyond 2^24 grid
// units), the value is within a few units of 2^-24 of the exact one, far
// inside the bound.  The largest value (rounded up) goes to *fmax.
__device__ inline void cross_terms(const __bf16 *hi, const __bf16 *lo, const __bf16 *lo2, const float *__restrict__ pa,
                                   const float *__restrict__ pb, int len, int dp, int ks, float *far,
                                   unsigned int *fmax, int t, int nthr) {
    for (int r = t >> 2; r < kTile; r += nthr >> 2) {
        double acc = 0.0;
        for (int c = t & 3; c < dp; c += 4) {
            const double v = (double)(float)hi[r * ks + c] + (double)(float)lo[r * ks + c] +
                             (double)(float)lo2[r * ks + c];
            const double e = v + ((double)pa[c] - (double)pb[c]);
            acc = fma(e, e, acc);
        }
        acc += __shfl_xor(acc, 1, kWave);
        acc += __shfl_xor(acc, 2, kWave);
        if ((t & 3) == 0) {
            far[r] = (float)acc;
            if (r < len) atomicMax(fmax, __float_as_uint(__double2float_ru(acc)));
        }
    }
}

// Entries of the distance blocks: float32, or the upper 16 bits of the
// float32 value rounded up (an upper bound with 8 significant bits; the
// values are non-negative or +inf, so the bit patterns order like the values).
__device__ inline void put_d(float *p, float v) { *p = v; }
__device__ inline void put_d(uint16_t *p, float v) { *p = (uint16_t)((__float_as_uint(v) + 0xffffu) >> 16); }
__device__ inline float get_d16(const uint16_t *p) { return __uint_as_float((uint32_t)*p << 16); }

// One wave: a 16 x 16 block of estimated squared distances,
//     D[i][j] = max(0, ta[i] + (tb[j] - off) - 2 (hi.hi + hi.lo + lo.hi)),
// rows r0.. of A against rows c0.. of B.
template <typename DT>
__device__ inline void bf16_block(const __bf16 *ah, const __bf16 *al, const float *ta, const __bf16 *bh,
                                  const __bf16 *bl, const float *tb, float off, int r0, int c0, int kp, int ks,
                                  DT *D, int dld) {
    const int lane = threadIdx.x & 63, il = lane & 15, kl = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < kp; kk += kKb) {
        const int ko = kk + 8 * kl;
        const bf16x8 xh = *reinterpret_cast<const bf16x8 *>(ah + (r0 + il) * ks + ko);
        const bf16x8 yh = *reinterpret_cast<const bf16x8 *>(bh + (c0 + il) * ks + ko);
        const bf16x8 yl = *reinterpret_cast<const bf16x8 *>(bl + (c0 + il) * ks + ko);
        const bf16x8 xl = *reinterpret_cast<const bf16x8 *>(al + (r0 + il) * ks + ko);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0);
    }
    const int j = c0 + il;
    const float tbj = tb[j] - off;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = r0 + 4 * kl + r;
        put_d(&D[i * dld + j], fmaxf(0.f, fmaf(-2.f, acc[r], ta[i] + tbj)));
    }
}

// Error bound of a block of estimated entries (an upper bound): 2 eps R_X
// R_Y + 6 u S, S the largest sum of magnitudes of an entry's exact terms.
__device__ inline float ebound(float rx, float ry, float s) {
    return add_up(mul_up(2.f * kEps, mul_up(rx, ry)), mul_up(kU6, s));
}

__global__ __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs_bf16(
    int64_t ntp, const uint64_t *__restrict__ rec, const float *__restrict__ XAf, const float *__restrict__ XBf,
    int mode, int dp, int kp, int32_t K, const float *__restrict__ Xpf, PairList out, unsigned long long *work,
    unsigned long long *counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BLayout LY = blayout(kp);
    const int ks = LY.ks;
    __bf16 *hT = (__bf16 *)smem, *lT = hT + kTile * ks, *l2T = lT + kTile * ks;
    __bf16 *hU = l2T + kTile * ks, *lU = hU + kTile * ks;
    uint64_t *mX = (uint64_t *)(smem + LY.rows), *mY = mX + kTile, *survb = mY + kTile;   // survb: 2 x 64
    // per-row terms: |x - p_a|^2, |x - p_b|^2 (T); |y - p_b|^2, |y - p_a|^2 (U);
    // |p - p_a|^2, |p - p_b|^2 (pivots); then the tile radii and maxima
    float *nT = (float *)(survb + 2 * kTile), *fT = nT + kTile, *nU = fT + kTile, *fU = nU + kTile;
    float *nPa = fU + kTile, *nPb = nPa + kPiv;
    // rad (float bits): [0] R_T, [1] R_U, [2] R_Pa, [3] R_Pb, [4] max |x - p_b|^2,
    // [5] max |y - p_a|^2, [6] |p_a - p_b|^2
    unsigned int *rad = (unsigned int *)(nPb + kPiv);
    float *DTU = (float *)(smem + LY.fixed);
    uint16_t *DTT = (uint16_t *)(smem + LY.fixed + LY.dmat);
    uint16_t *DUU = (uint16_t *)(smem + LY.fixed + LY.dmat + LY.dtt);
    unsigned char *region = smem + LY.fixed + LY.dmat + 2 * LY.dtt;
    __bf16 *hPa = (__bf16 *)region, *lPa = hPa + kPiv * ks, *hPb = lPa + kPiv * ks, *lPb = hPb + kPiv * ks;
    float *XP = (float *)(lPb + kPiv * ks), *YP = XP + kTile * kXs;
    // Claims alternate between two sets of slots (iteration parity): thread
    // 0 claims the next tile pair during Stage IV of the current one, so no
    // barrier is needed between two tile pairs' work.
    __shared__ int64_t s_tp[2], s_nx;
    // record words before the masks (tiles' start, length and cell, pivot
    // ids): the current tile pair's, and the next one's, fetched one tile
    // pair ahead so that no wave waits on the record before loading rows
    __shared__ uint64_t s_cm[2][kPairRecMeta], s_nm[kPairRecMeta];
    __shared__ int s_any[2], s_newT[2], s_newB[2];
    __shared__ int32_t s_sx, s_b;   // T tile whose rows are in LDS; the cell its cross terms are for
    __shared__ int32_t s_dtt;       // T tile whose D(T,T) is in LDS
    __shared__ float s_tau4, s_tau5;
    const bool self = (mode & PM_SELF) != 0;
    uint32_t ncand = 0, ns4 = 0, nsurv = 0, ntpv = 0, nttv = 0, nunc = 0;
    uint64_t dtu = 0, dpv = 0, dv = 0;   // tile entries computed (thread 0)
    WaveOut wo;
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
        // T's rows stay in LDS while consecutive tile pairs share T, and
        // its cross terms while they also share U's cell
        int32_t st = -1, sb = -1;
        if (s_tp[q] >= 0) {
            st = (int32_t)s_cm[q][0];
            sb = (int32_t)(s_cm[q][2] >> 32);
        }
        s_newT[q] = st != s_sx;
        s_newB[q] = s_newT[q] || sb != s_b;
        s_sx = st;
        s_b = sb;
        if (s_newT[q]) rad[0] = 0u;
        if (s_newB[q]) rad[4] = 0u;
        rad[1] = rad[2] = rad[3] = rad[5] = 0u;
    };
    if (threadIdx.x == 0) {
        s_sx = -1;
        s_b = -1;
        s_dtt = -1;
        nxt = next_tp();
        if (nxt >= 0)
            for (int k = 0; k < kPairRecMeta; ++k) s_nm[k] = rec[nxt * kPairRecWords + k];
        claim(0);
    }
    __syncthreads();
    for (int par = 0;; par ^= 1) {
        const int64_t tp = uniform_i64(s_tp[par]);
        if (tp < 0) break;
        // Per-thread LDS addresses are recomputed in every iteration rather
        // than held across it (held, they exceed the register budget).
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, w = tid >> 6;
        const bool newT = s_newT[par] != 0, newB = s_newB[par] != 0;
        const uint64_t *rc = rec + tp * kPairRecWords;
        const uint64_t m0 = s_cm[par][0], m1 = s_cm[par][1], m2 = s_cm[par][2];
        const int32_t sT = (int32_t)m0, lTn = (int32_t)(m0 >> 32);
        const int32_t a = (int32_t)m1, lUn = (int32_t)(m1 >> 32), sU = (int32_t)m2, b = (int32_t)(m2 >> 32);
        const float *pa = Xpf + (int64_t)a * dp, *pb = Xpf + (int64_t)b * dp;
        // 1. masks; centred split rows of T (when new), of U and of the pivots.
        if (w == 6) {
            mX[lane] = rc[kPairRecMeta + lane];
            survb[par * kTile + lane] = 0;
        } else if (w == 7) {
            mY[lane] = rc[kPairRecMeta + kTile + lane];
        } else if (w == 5) {
            // 16 pivot rows, each centred at p_a and at p_b, four lanes per row;
            // slots past K repeat a valid pivot (their distances become +inf)
            // (each row read once and split for both centres)
            const int t = lane >> 2, q4 = lane & 3;
            const int32_t pv = (int32_t)(s_cm[par][3 + (t >> 1)] >> (32 * (t & 1)));
            const float *src = Xpf + (int64_t)pv * dp;
            double acca = 0.0, accb = 0.0;
            for (int c0 = 8 * q4; c0 < kp; c0 += kKb) {
                float4 v[2], ca[2], cb[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int c = c0 + 4 * q;
                    v[q] = ca[q] = cb[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (c < dp) {
                        v[q] = *reinterpret_cast<const float4 *>(src + c);
                        ca[q] = *reinterpret_cast<const float4 *>(pa + c);
                        cb[q] = *reinterpret_cast<const float4 *>(pb + c);
                    }
                }
                bf16x8 ha, la, hb, lb;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float xv[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
                    const float av[4] = {ca[q].x, ca[q].y, ca[q].z, ca[q].w};
                    const float bv[4] = {cb[q].x, cb[q].y, cb[q].z, cb[q].w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float ea = xv[k] - av[k], eb = xv[k] - bv[k];
                        const __bf16 h1 = (__bf16)ea, h2 = (__bf16)eb;
                        ha[4 * q + k] = h1;
                        la[4 * q + k] = (__bf16)(ea - (float)h1);
                        hb[4 * q + k] = h2;
                        lb[4 * q + k] = (__bf16)(eb - (float)h2);
                        const double fa = (double)xv[k] - (double)av[k], fb = (double)xv[k] - (double)bv[k];
                        acca = fma(fa, fa, acca);   // exact (grid values)
                        accb = fma(fb, fb, accb);
                    }
                }
                *reinterpret_cast<bf16x8 *>(hPa + t * ks + c0) = ha;
                *reinterpret_cast<bf16x8 *>(lPa + t * ks + c0) = la;
                *reinterpret_cast<bf16x8 *>(hPb + t * ks + c0) = hb;
                *reinterpret_cast<bf16x8 *>(lPb + t * ks + c0) = lb;
            }
            acca += __shfl_xor(acca, 1, kWave);
            acca += __shfl_xor(acca, 2, kWave);
            accb += __shfl_xor(accb, 1, kWave);
            accb += __shfl_xor(accb, 2, kWave);
            if (q4 == 0) {
                nPa[t] = (float)acca;
                nPb[t] = (float)accb;
                atomicMax(&rad[2], __float_as_uint(__double2float_ru(sqrt(acca) * (1.0 + 0x1p-50))));
                atomicMax(&rad[3], __float_as_uint(__double2float_ru(sqrt(accb) * (1.0 + 0x1p-50))));
            }
            // |p_a - p_b|^2, exact in float64 (partial sums over the lanes)
            double acc = 0.0;
            for (int c = lane; c < dp; c += 64) {
                const double e = (double)pa[c] - (double)pb[c];
                acc = fma(e, e, acc);
            }
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
            if (lane == 0) rad[6] = __float_as_uint((float)acc);
        }
        if (newT) {
            if (tid < 256)
                load_split(hT, lT, l2T, nT, nullptr, &rad[0], nullptr, XAf + (int64_t)sT * dp, lTn, kTile, dp, kp, ks,
                           pa, nullptr, tid, 256);
            else
                load_split(hU, lU, nullptr, nU, fU, &rad[1], &rad[5], XBf + (int64_t)sU * dp, lUn, kTile, dp, kp, ks,
                           pb, pa, tid - 256, 256);
        } else if (tid < 256) {
            load_split(hU, lU, nullptr, nU, fU, &rad[1], &rad[5], XBf + (int64_t)sU * dp, lUn, kTile, dp, kp, ks, pb,
                       pa, tid, 256);
        } else if (newB && w != 5) {
            // T's rows are in LDS already: its cross terms for U's new cell,
            // by waves 4, 6 and 7 (the last two after their mask loads)
            const int t = w == 4 ? lane : (w == 6 ? 64 + lane : 128 + lane);
            cross_terms(hT, lT, l2T, pa, pb, lTn, dp, ks, fT, &rad[4], t, 192);
        }
        __syncthreads();
        if (newB && newT) {   // T's rows arrived in this phase
            cross_terms(hT, lT, l2T, pa, pb, lTn, dp, ks, fT, &rad[4], tid, kBThreads);
            __syncthreads();
        }
        // The next tile pair's record words, in flight until Stage IV ends.
        if (tid < kPairRecMeta) {
            const int64_t nx = s_nx;
            if (nx >= 0) nmeta = rec[nx * kPairRecWords + tid];
        }
        // 2a. D(T,U) (two blocks per wave) and one block of pivot distances
        // (rows of T for waves 0-3, of U for 4-7).
        {
            const bool ys = w >= 4;
            const int pr = (w & 3) * 16;
            const int id0 = 2 * w, id1 = 2 * w + 1;
            const float dab = __uint_as_float(rad[6]);
            bf16_block(hT, lT, fT, hU, lU, fU, dab, (id0 >> 2) * 16, (id0 & 3) * 16, kp, ks, DTU, kDl);
            bf16_block(hT, lT, fT, hU, lU, fU, dab, (id1 >> 2) * 16, (id1 & 3) * 16, kp, ks, DTU, kDl);
            if (ys)
                bf16_block(hU, lU, nU, hPb, lPb, nPb, 0.f, pr, 0, kp, ks, YP, kXs);
            else
                bf16_block(hT, lT, nT, hPa, lPa, nPa, 0.f, pr, 0, kp, ks, XP, kXs);
            if ((lane & 15) >= K) {   // unused pivot slots never witness
                float *Pd = ys ? YP : XP;
                for (int r = 0; r < 4; ++r) Pd[(pr + 4 * r + (lane >> 4)) * kXs + (lane & 15)] = INFINITY;
            }
            if (tid == 0) {
                const float rT = __uint_as_float(rad[0]), rU = __uint_as_float(rad[1]);
                const float rPa = __uint_as_float(rad[2]), rPb = __uint_as_float(rad[3]);
                const float fTm = __uint_as_float(rad[4]), fUm = __uint_as_float(rad[5]);
                // magnitudes of an entry's exact terms: D(T,U): |x-p_b|^2 +
                // |y-p_a|^2 + |p_a-p_b|^2 + 2|a||b|; D(T,P): |a|^2 + |p-p_a|^2 +
                // 2|a||p-p_a| = (|a| + |p-p_a|)^2; likewise for U and for T, U alone
                const float sTU = add_up(add_up(fTm, fUm), add_up(up_ulp(dab), mul_up(2.f, mul_up(rT, rU))));
                const float sTP = mul_up(add_up(rT, rPa), add_up(rT, rPa));
                const float sUP = mul_up(add_up(rU, rPb), add_up(rU, rPb));
                const float eTU = ebound(rT, rU, sTU);
                const float eP = fmaxf(ebound(rT, rPa, sTP), ebound(rU, rPb, sUP));
                const float eTT = ebound(rT, rT, mul_up(4.f, mul_up(rT, rT)));
                const float eUU = ebound(rU, rU, mul_up(4.f, mul_up(rU, rU)));
                s_tau4 = add_up(eTU, eP);
                s_tau5 = add_up(eTU, fmaxf(eTU, fmaxf(eTT, eUU)));
            }
        }
        __syncthreads();
        const float tau4 = s_tau4, tau5 = s_tau5;
        // 2b. Stage IV: C = min over pivots of max(d2(x,p), d2(y,p)) as a
        // (min,max) product on float bit patterns (non-negative or +inf);
        // a candidate dies when C < d2(x,y) - tau4 (rounded down).
        {
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
                    const float thr = sub_dn(DTU[i * kDl + j], tau4);
                    const uint32_t tb = thr > 0.f ? __float_as_uint(thr) : 0u;
                    if (cand && !(c[r][q] < tb)) bits |= 1ull << j;
                }
                if (bits) {
                    ns4 += __popcll(bits);
                    atomicOr((unsigned long long *)&survb[par * kTile + i], (unsigned long long)bits);
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
            dtu += (uint64_t)lTn * (uint64_t)lUn;
            dpv += (uint64_t)(lTn + lUn) * (uint64_t)K;
        }
        if (!s_any[par]) continue;   // uniform
        ntpv += tid == 0;
        // 2c. D(U,U) and, when T's points may witness and T changed since
        // D(T,T) was last formed, D(T,T) (two blocks of each per wave).
        const bool newTT = self && s_dtt != sT;
        if (tid == 0) dv += (uint64_t)lUn * lUn + (newTT ? (uint64_t)lTn * lTn : 0);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int id = 2 * w + q;
            bf16_block(hU, lU, nU, hU, lU, nU, 0.f, (id >> 2) * 16, (id & 3) * 16, kp, ks, DUU, kDl);
            if (newTT) bf16_block(hT, lT, nT, hT, lT, nT, 0.f, (id >> 2) * 16, (id & 3) * 16, kp, ks, DTT, kDl);
        }
        nttv += tid == 0 && newTT;
        __syncthreads();
        if (tid == 0 && newTT) s_dtt = sT;
        // 3. Stage V: each wave walks rows w, w + 8, ...; every Stage IV
        // survivor (i, j) against the 128 points of T and U, one lane per
        // witness z (T[lane] and U[lane]).
        for (int i = w; i < lTn; i += kBWaves) {
            uint64_t row = survb[par * kTile + i];
            if (!row) continue;
            const float ax = (self && lane < lTn) ? get_d16(&DTT[i * kDl + lane]) : INFINITY;
            const float au = lane < lUn ? DTU[i * kDl + lane] : INFINITY;
            while (row) {
                const int j = __ffsll((long long)row) - 1;
                row &= row - 1;
                const float dxy = DTU[i * kDl + j];
                const float t = sub_dn(dxy, tau5), tu = add_up(dxy, tau5);
                const float by = (self && lane < lTn) ? DTU[lane * kDl + j] : INFINITY;
                const float bu = lane < lUn ? get_d16(&DUU[j * kDl + lane]) : INFINITY;
                if (__ballot((ax < t && by < t) || (au < t && bu < t))) continue;   // a certain witness
                // a survivor; uncertain when some witness other than x and y lies
                // within the bound
                const int32_t zt = sT + lane, zu = sU + lane, px_ = sT + i, py_ = sU + j;
                const bool oT = zt != px_ && zt != py_, oU = zu != px_ && zu != py_;
                nunc += (lane == 0) &
                        (__ballot((oT && ax < tu && by < tu) || (oU && au < tu && bu < tu)) != 0);
                if (lane == wo.cnt) {
                    wo.x = sT + i;
                    wo.y = sU + j;
                    wo.d2 = -1.0;   // the exact value comes from k_pairs_exact_d2
                }
                ++nsurv;
                if (++wo.cnt == 64) wo.flush(out);
            }
        }
    }
    wo.flush(out);
    ncand = wave_sum(ncand);
    ns4 = wave_sum(ns4);
    nunc = wave_sum(nunc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        const uint64_t tests = (uint64_t)ncand * (uint64_t)K + (uint64_t)ns4 * (self ? 128u : 64u);
        atomicAdd(&counters[C_CAND], (unsigned long long)ncand);
        atomicAdd(&counters[C_S4], (unsigned long long)ns4);
        atomicAdd(&counters[C_WTEST], (unsigned long long)tests);
        atomicAdd(&counters[C_SURV], (unsigned long long)nsurv);
        if (nunc) atomicAdd(&counters[C_UNCERTAIN], (unsigned long long)nunc);
        if (ntpv) atomicAdd(&counters[C_TPV], (unsigned long long)ntpv);
        if (nttv) atomicAdd(&counters[C_TTV], (unsigned long long)nttv);
        if (w == 0) {
            atomicAdd(&counters[C_DIST], (unsigned long long)(dtu + dpv + dv));
            atomicAdd(&counters[C_PD_TU], (unsigned long long)dtu);
            atomicAdd(&counters[C_PD_PIV], (unsigned long long)dpv);
            atomicAdd(&counters[C_PD_V], (unsigned long long)dv);
        }
    }
}

// Exact float64 squared distances of listed pairs (XA[px] against XB[py];
// direct form, exact on the grid) and each row point's largest one.  Eight
// lanes per pair.
__global__ __launch_bounds__(256) void k_pairs_exact_d2(int64_t np, const int32_t *__restrict__ px,
                                                        const int32_t *__restrict__ py, int dp,
                                                        const double *__restrict__ XA, const double *__restrict__ XB,
                                                        double *__restrict__ d2, unsigned long long *dmax_bits) {
    const int64_t p = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    double acc = 0.0;
    int32_t x = 0;
    if (p < np) {
        x = px[p];
        const double *u = XA + (int64_t)x * dp, *v = XB + (int64_t)py[p] * dp;
        for (int c = 2 * sub; c < dp; c += 16) {
            const double2 s = *reinterpret_cast<const double2 *>(u + c);
            const double2 t = *reinterpret_cast<const double2 *>(v + c);
            const double e0 = s.x - t.x, e1 = s.y - t.y;
            acc = fma(e0, e0, acc);
            acc = fma(e1, e1, acc);
        }
    }
    acc += __shfl_xor(acc, 1, kWave);
    acc += __shfl_xor(acc, 2, kWave);
    acc += __shfl_xor(acc, 4, kWave);
    if (p < np && sub == 0) {
        d2[p] = acc;
        atomicMax(&dmax_bits[x], (unsigned long long)__double_as_longlong(acc));
    }
}

}  // namespace

void launch_pairs_bf16(hipStream_t s, int64_t ntp, const uint64_t *rec, const float *XAf, const float *XBf, int mode,
                       int dp, int32_t K, const float *Xpf, PairList out, uint64_t *work, uint64_t *counters) {
    if (ntp == 0) return;
    require(dp <= kMaxKp, GRNG_EINVAL, "dimension too large for the bf16 pair kernel");
    require(K >= 1 && K <= kPiv, GRNG_EINVAL, "Stage IV pivot count out of range");
    launch_fill_u64(s, work, kXcds * kWorkStride, 0ull);
    const int kp = (dp + kKb - 1) / kKb * kKb;
    const BLayout L = blayout(kp);
    require(L.total <= 160 * 1024, GRNG_EINVAL, "dimension too large for the bf16 pair kernel's LDS tiles");
    if (L.total > 64 * 1024)
        GRNG_HIP(hipFuncSetAttribute((const void *)k_pairs_bf16, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.total));
    const int64_t grid = std::max<int64_t>(kXcds, std::min<int64_t>(div_up(ntp, kPairChunk), 256 * 4));
    k_pairs_bf16<<<(unsigned)grid, kBThreads, L.total, s>>>(ntp, rec, XAf, XBf, mode, dp, kp, K, Xpf, out,
                                                             (unsigned long long *)work,
                                                             (unsigned long long *)counters);
    GRNG_LAUNCHED();
}

void launch_pairs_exact_d2(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, int dp, const double *XA,
                           const double *XB, double *d2, uint64_t *dmax_bits) {
    if (np == 0) return;
    k_pairs_exact_d2<<<(unsigned)div_up(np * 8, 256), 256, 0, s>>>(np, px, py, dp, XA, XB, d2,
                                                                    (unsigned long long *)dmax_bits);
    GRNG_LAUNCHED();
}

}  // namespace grng
