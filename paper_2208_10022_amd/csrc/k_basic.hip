// Basic kernels: input validation, exact float64 distance tiles, scans, gathers.
//
// Exactness: coordinates are k * 2^-q with |k| < 2^24 and d * kmax^2 < 2^51,
// so every product, partial sum and final value of
//     d^2(a, b) = ||a||^2 + ||b||^2 - 2 a.b
// is an integer multiple of 2^-2q below 2^53 in magnitude: float64 holds each
// exactly, whatever the summation order and whether or not FMA is used.  The
// MFMA f64 tile therefore returns the exact squared distance (Section 1: the
// method's cost unit is the distance computation; here each one is exact).
#include "common.h"

namespace grng {

namespace {

__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__global__ void k_grid_check(const float *x, int64_t count, double scale, unsigned long long *kmax_bits,
                             int32_t *bad) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double local = 0.0;
    int b = 0;
    for (; i < count; i += stride) {
        double v = (double)x[i];
        if (!isfinite(v)) { b = 1; continue; }
        double k = v * scale;
        if (k != rint(k) || fabs(k) >= 16777216.0) b = 1;
        local = fmax(local, fabs(k));
    }
    local = wave_max(local);
    uint64_t anybad = __ballot(b);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMax(kmax_bits, (unsigned long long)__double_as_longlong(local));
        if (anybad) atomicOr(bad, 1);
    }
}

__global__ void k_grid_check_f64(const double *x, int64_t count, double scale, unsigned long long *kmax_bits,
                                 int32_t *bad) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double local = 0.0;
    int b = 0;
    for (; i < count; i += stride) {
        double v = x[i];
        if (!isfinite(v)) { b = 1; continue; }
        double k = v * scale;
        if (k != rint(k) || fabs(k) >= 16777216.0 || k < 0.0) b = 1;
        local = fmax(local, fabs(k));
    }
    local = wave_max(local);
    uint64_t anybad = __ballot(b);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMax(kmax_bits, (unsigned long long)__double_as_longlong(local));
        if (anybad) atomicOr(bad, 1);
    }
}

__global__ void k_to_f64(const float *src, int64_t n, int d, int dp, double *dst, double *nrm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < dp; ++t) {
        double v = t < d ? (double)src[i * d + t] : 0.0;
        dst[i * dp + t] = v;
        s = fma(v, v, s);
    }
    nrm[i] = s;
}

// Plain VALU tile: one thread per output entry, rows staged through LDS.
constexpr int kVT = 16;
__global__ void k_dist2_valu(const double *A, const double *nA, int64_t na, const double *B, const double *nB,
                             int64_t nb, int dp, double *out, int64_t ldo) {
    __shared__ double As[kVT][33];
    __shared__ double Bs[kVT][33];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int64_t i = blockIdx.y * (int64_t)kVT + ty;
    const int64_t j = blockIdx.x * (int64_t)kVT + tx;
    double acc = 0.0;
    for (int k0 = 0; k0 < dp; k0 += 32) {
        for (int t = tx; t < 32; t += kVT) {
            int64_t ai = blockIdx.y * (int64_t)kVT + ty;
            int64_t bj = blockIdx.x * (int64_t)kVT + ty;
            As[ty][t] = (ai < na && k0 + t < dp) ? A[ai * dp + k0 + t] : 0.0;
            Bs[ty][t] = (bj < nb && k0 + t < dp) ? B[bj * dp + k0 + t] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < 32; ++t) acc = fma(As[ty][t], Bs[tx][t], acc);
        __syncthreads();
    }
    if (i < na && j < nb) out[i * ldo + j] = nA[i] + nB[j] - 2.0 * acc;
}

// MFMA tile: 64 x 64 outputs per workgroup of 4 waves (2 x 2), each wave a
// 32 x 32 block made of 2 x 2 v_mfma_f64_16x16x4f64 accumulators.  Operand
// rows are staged through LDS in K-chunks of 32.
//   A operand (16x4): lane l holds A[l % 16][l / 16]
//   B operand (4x16): lane l holds B[l / 16][l % 16]   (B = points^T)
//   D (16x16):        lane l, item r holds D[4 * r + l / 16][l % 16]
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMT = 64;
constexpr int kMK = 32;
__global__ __launch_bounds__(256) void k_dist2_mfma(const double *A, const double *nA, int64_t na,
                                                    const double *B, const double *nB, int64_t nb, int dp,
                                                    double *out, int64_t ldo) {
    __shared__ double As[kMT][kMK + 1];
    __shared__ double Bs[kMT][kMK + 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t row0 = blockIdx.y * (int64_t)kMT;
    const int64_t col0 = blockIdx.x * (int64_t)kMT;
    v4d acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < dp; k0 += kMK) {
        for (int e = threadIdx.x; e < kMT * kMK; e += 256) {
            int r = e / kMK, t = e % kMK;
            int64_t ai = row0 + r, bj = col0 + r;
            As[r][t] = (ai < na && k0 + t < dp) ? A[ai * dp + k0 + t] : 0.0;
            Bs[r][t] = (bj < nb && k0 + t < dp) ? B[bj * dp + k0 + t] : 0.0;
        }
        __syncthreads();
        const int kl = lane >> 4, il = lane & 15;
        for (int kk = 0; kk < kMK; kk += 4) {
            double av[2], bv[2];
            for (int a = 0; a < 2; ++a) av[a] = As[wr * 32 + a * 16 + il][kk + kl];
            for (int b = 0; b < 2; ++b) bv[b] = Bs[wc * 32 + b * 16 + il][kk + kl];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    const int jl = lane & 15, ib = lane >> 4;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            int64_t j = col0 + wc * 32 + b * 16 + jl;
            if (j >= nb) continue;
            double nbj = nB[j];
            for (int r = 0; r < 4; ++r) {
                int64_t i = row0 + wr * 32 + a * 16 + 4 * r + ib;
                if (i < na) out[i * ldo + j] = nA[i] + nbj - 2.0 * acc[a][b][r];
            }
        }
}

__global__ void k_sqrt(const double *in, double *out, int64_t count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) out[i] = sqrt(in[i]);
}

__global__ void k_gather_rows(const double *src, const int32_t *idx, int64_t n, int dp, double *dst) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * dp) return;
    int64_t i = e / dp;
    int t = (int)(e % dp);
    dst[e] = src[(int64_t)idx[i] * dp + t];
}

__global__ void k_gather_f64(const double *src, const int32_t *idx, int64_t n, double *dst) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_inverse(const int32_t *perm, int64_t n, int32_t *inv) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) inv[perm[i]] = (int32_t)i;
}

// Single-workgroup exclusive scan in passes of 4096 entries: each thread
// takes 4 consecutive entries (coalesced loads and stores across the wave),
// waves scan their sums with shuffles, and the 16 wave totals carry the
// running offset from pass to pass.
// Workgroup b scans entries [b * chunk, min(n, (b + 1) * chunk)) starting
// from base[b] (0 without base); the last workgroup writes the total out[n].
template <class TI>
__global__ __launch_bounds__(1024) void k_scan(const TI *in, int64_t n, int64_t chunk, const int64_t *base,
                                               int64_t *out) {
    constexpr int kPer = 4;
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    int64_t carry = base ? base[blockIdx.x] : 0;
    for (int64_t b0 = lo; b0 < hi; b0 += 1024 * kPer) {
        const int64_t i0 = b0 + (int64_t)t * kPer;
        int64_t v[kPer], sum = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            v[u] = i0 + u < hi ? (int64_t)in[i0 + u] : 0;
            sum += v[u];
        }
        int64_t inc = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t up = __shfl_up(inc, o, 64);
            if (lane >= o) inc += up;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int64_t before = 0, total = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int64_t x = wsum[j];
            before += j < w ? x : 0;
            total += x;
        }
        int64_t run = carry + before + inc - sum;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (i0 + u < hi) out[i0 + u] = run;
            run += v[u];
        }
        carry += total;
        __syncthreads();   // wsum is rewritten by the next pass
    }
    if (t == 0 && blockIdx.x == gridDim.x - 1) out[n] = carry;
}

// Sum of each workgroup's chunk (the first step of a scan over many workgroups).
template <class TI>
__global__ __launch_bounds__(1024) void k_chunk_sums(const TI *in, int64_t n, int64_t chunk, int64_t *sums) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    int64_t acc = 0;
    for (int64_t i = lo + t; i < hi; i += 1024) acc += (int64_t)in[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (t == 0) {
        int64_t tot = 0;
        for (int j = 0; j < 16; ++j) tot += wsum[j];
        sums[blockIdx.x] = tot;
    }
}

__global__ void k_bits_transpose(const uint64_t *rows, int64_t n, int32_t words, int64_t m, uint64_t *cols,
                                 int64_t nw) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= m * nw) return;
    int64_t w = e / m, j = e % m;   // consecutive threads: consecutive pivots, same point word
    uint64_t acc = 0;
    const int64_t x0 = w * 64;
    for (int b = 0; b < 64; ++b) {
        int64_t x = x0 + b;
        if (x >= n) break;
        uint64_t word = rows[x * words + (j >> 6)];
        acc |= ((word >> (j & 63)) & 1ull) << b;
    }
    cols[j * nw + w] = acc;
}

__global__ void k_fill_u64(uint64_t *p, int64_t count, uint64_t v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

inline unsigned grid1(int64_t work, int block) {
    int64_t g = div_up(work, block);
    return (unsigned)(g < 1 ? 1 : g);
}

// float64 -> float32 (values that are float32 on input stay exact).
__global__ void k_to_f32(const double *src, int64_t count, float *dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (float)src[i];
}


// Insertion merge.  The merged home order keeps each cell's old points first
// and appends the cell's batch points after them.  src[r] >= 0 names the old
// position that position r takes its row from, src[r] < 0 the batch
// position -1 - src[r].  The offsets arrays have m + 1 entries.
__global__ void k_merge_positions(int64_t n1, int64_t m, const int32_t *__restrict__ new_off,
                                  const int32_t *__restrict__ old_off, const int32_t *__restrict__ bat_off,
                                  int32_t *__restrict__ src) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n1) return;
    int64_t lo = 0, hi = m;   // the cell c with new_off[c] <= r < new_off[c + 1]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (new_off[mid] <= r) lo = mid; else hi = mid;
    }
    const int32_t k = (int32_t)r - new_off[lo], old = old_off[lo + 1] - old_off[lo];
    src[r] = k < old ? old_off[lo] + k : -1 - (bat_off[lo] + k - old);
}

// Rows of rw 32-bit words from the old or the batch side; bias is added to
// batch-side words (batch-local point ids becoming global ids), else 0.
__global__ void k_merge_rows32(int64_t n1, int32_t rw, const int32_t *__restrict__ src,
                               const uint32_t *__restrict__ old, const uint32_t *__restrict__ bat, uint32_t bias,
                               uint32_t *__restrict__ out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n1 * rw) return;
    const int64_t r = e / rw;
    const int32_t t = (int32_t)(e - r * rw), sr = src[r];
    out[e] = sr >= 0 ? old[(int64_t)sr * rw + t] : bat[(int64_t)(-1 - sr) * rw + t] + bias;
}

// Ragged rows (CSR): first the length of each merged row, then the copy.
__global__ void k_merge_csr_len(int64_t n1, const int32_t *__restrict__ src, const int64_t *__restrict__ old_off,
                                const int64_t *__restrict__ bat_off, int32_t *__restrict__ len) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n1) return;
    const int32_t sr = src[r];
    len[r] = (int32_t)(sr >= 0 ? old_off[sr + 1] - old_off[sr] : bat_off[-sr] - bat_off[-1 - sr]);
}

__global__ void k_merge_csr_copy(int64_t n1, const int32_t *__restrict__ src, const int64_t *__restrict__ old_off,
                                 const int32_t *__restrict__ old_idx, const int64_t *__restrict__ bat_off,
                                 const int32_t *__restrict__ bat_idx, const int64_t *__restrict__ new_off,
                                 int32_t *__restrict__ out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n1) return;
    const int32_t sr = src[r];
    const int64_t *off = sr >= 0 ? old_off : bat_off;
    const int32_t *idx = sr >= 0 ? old_idx : bat_idx;
    const int64_t b = sr >= 0 ? sr : -1 - sr;
    int64_t o = new_off[r];
    for (int64_t t = off[b]; t < off[b + 1]; ++t) out[o++] = idx[t];
}

}  // namespace

void launch_grid_check(hipStream_t s, const float *x, int64_t count, double scale, uint64_t *kmax_bits,
                       int32_t *bad) {
    int64_t g = div_up(count, 256);
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    k_grid_check<<<(unsigned)g, 256, 0, s>>>(x, count, scale, (unsigned long long *)kmax_bits, bad);
    GRNG_LAUNCHED();
}

void launch_grid_check_f64(hipStream_t s, const double *x, int64_t count, double scale, uint64_t *kmax_bits,
                           int32_t *bad) {
    int64_t g = div_up(count, 256);
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    k_grid_check_f64<<<(unsigned)g, 256, 0, s>>>(x, count, scale, (unsigned long long *)kmax_bits, bad);
    GRNG_LAUNCHED();
}

void launch_to_f64(hipStream_t s, const float *src, int64_t n, int d, int dp, double *dst, double *nrm) {
    k_to_f64<<<grid1(n, 256), 256, 0, s>>>(src, n, d, dp, dst, nrm);
    GRNG_LAUNCHED();
}

void launch_dist2(hipStream_t s, const double *A, const double *nA, int64_t na, const double *B,
                  const double *nB, int64_t nb, int dp, double *out, int64_t ldo, bool use_mfma) {
    if (na == 0 || nb == 0) return;
    if (use_mfma) {
        dim3 g((unsigned)div_up(nb, kMT), (unsigned)div_up(na, kMT));
        require(g.y <= 65535u, GRNG_EINVAL, "distance tile grid too tall");
        k_dist2_mfma<<<g, 256, 0, s>>>(A, nA, na, B, nB, nb, dp, out, ldo);
    } else {
        dim3 g((unsigned)div_up(nb, kVT), (unsigned)div_up(na, kVT));
        require(g.y <= 65535u, GRNG_EINVAL, "distance tile grid too tall");
        k_dist2_valu<<<g, dim3(kVT, kVT), 0, s>>>(A, nA, na, B, nB, nb, dp, out, ldo);
    }
    GRNG_LAUNCHED();
}

void launch_sqrt(hipStream_t s, const double *in, double *out, int64_t count) {
    if (count == 0) return;
    k_sqrt<<<grid1(count, 256), 256, 0, s>>>(in, out, count);
    GRNG_LAUNCHED();
}

void launch_gather_rows(hipStream_t s, const double *src, const int32_t *idx, int64_t n, int dp, double *dst) {
    if (n == 0) return;
    k_gather_rows<<<grid1(n * dp, 256), 256, 0, s>>>(src, idx, n, dp, dst);
    GRNG_LAUNCHED();
}

void launch_to_f32(hipStream_t s, const double *src, int64_t count, float *dst) {
    if (count == 0) return;
    k_to_f32<<<grid1(count, 256), 256, 0, s>>>(src, count, dst);
    GRNG_LAUNCHED();
}

void launch_gather_f64(hipStream_t s, const double *src, const int32_t *idx, int64_t n, double *dst) {
    if (n == 0) return;
    k_gather_f64<<<grid1(n, 256), 256, 0, s>>>(src, idx, n, dst);
    GRNG_LAUNCHED();
}

void launch_iota_inverse(hipStream_t s, const int32_t *perm, int64_t n, int32_t *inv) {
    if (n == 0) return;
    k_inverse<<<grid1(n, 256), 256, 0, s>>>(perm, n, inv);
    GRNG_LAUNCHED();
}

// Exclusive scan with the total in out[n]: one workgroup up to 2^16
// entries, else chunk sums, their scan, and one workgroup per 4,096-entry
// chunk.
template <class TI>
void scan_to_i64(hipStream_t s, const TI *in, int64_t n, int64_t *out) {
    constexpr int64_t kChunk = 4096;
    if (n <= (int64_t)1 << 16) {
        k_scan<TI><<<1, 1024, 0, s>>>(in, n, n > 0 ? n : 1, nullptr, out);
        GRNG_LAUNCHED();
        return;
    }
    const int64_t nc = div_up(n, kChunk);
    DevBuf sums, base;
    sums.alloc(8 * (size_t)nc);
    base.alloc(8 * (size_t)(nc + 1));
    k_chunk_sums<TI><<<(unsigned)nc, 1024, 0, s>>>(in, n, kChunk, sums.as<int64_t>());
    GRNG_LAUNCHED();
    k_scan<int64_t><<<1, 1024, 0, s>>>(sums.as<int64_t>(), nc, nc, nullptr, base.as<int64_t>());
    GRNG_LAUNCHED();
    k_scan<TI><<<(unsigned)nc, 1024, 0, s>>>(in, n, kChunk, base.as<int64_t>(), out);
    GRNG_LAUNCHED();
}

void launch_scan_i64(hipStream_t s, const int64_t *in, int64_t n, int64_t *out_excl) {
    scan_to_i64<int64_t>(s, in, n, out_excl);
}

void launch_scan_i32_to_i64(hipStream_t s, const int32_t *in, int64_t n, int64_t *out_excl) {
    scan_to_i64<int32_t>(s, in, n, out_excl);
}

void launch_bits_transpose(hipStream_t s, const uint64_t *rows, int64_t n, int32_t words, int64_t m,
                           uint64_t *cols) {
    const int64_t nw = div_up(n, 64);
    if (m == 0 || nw == 0) return;
    k_bits_transpose<<<grid1(m * nw, 256), 256, 0, s>>>(rows, n, words, m, cols, nw);
    GRNG_LAUNCHED();
}

void launch_merge_positions(hipStream_t s, int64_t n1, int64_t m, const int32_t *new_off, const int32_t *old_off,
                            const int32_t *bat_off, int32_t *src) {
    if (n1 == 0) return;
    k_merge_positions<<<grid1(n1, 256), 256, 0, s>>>(n1, m, new_off, old_off, bat_off, src);
    GRNG_LAUNCHED();
}

void launch_merge_rows(hipStream_t s, int64_t n1, size_t row_bytes, const int32_t *src, const void *old,
                       const void *bat, uint32_t bias, void *out) {
    require(row_bytes % 4 == 0, GRNG_EINVAL, "merged rows must be whole 32-bit words");
    const int32_t rw = (int32_t)(row_bytes / 4);
    if (n1 == 0 || rw == 0) return;
    k_merge_rows32<<<grid1(n1 * rw, 256), 256, 0, s>>>(n1, rw, src, static_cast<const uint32_t *>(old),
                                                       static_cast<const uint32_t *>(bat), bias,
                                                       static_cast<uint32_t *>(out));
    GRNG_LAUNCHED();
}

void launch_merge_csr_len(hipStream_t s, int64_t n1, const int32_t *src, const int64_t *old_off,
                          const int64_t *bat_off, int32_t *len) {
    if (n1 == 0) return;
    k_merge_csr_len<<<grid1(n1, 256), 256, 0, s>>>(n1, src, old_off, bat_off, len);
    GRNG_LAUNCHED();
}

void launch_merge_csr_copy(hipStream_t s, int64_t n1, const int32_t *src, const int64_t *old_off,
                           const int32_t *old_idx, const int64_t *bat_off, const int32_t *bat_idx,
                           const int64_t *new_off, int32_t *new_idx) {
    if (n1 == 0) return;
    k_merge_csr_copy<<<grid1(n1, 256), 256, 0, s>>>(n1, src, old_off, old_idx, bat_off, bat_idx, new_off, new_idx);
    GRNG_LAUNCHED();
}

void launch_fill_u64(hipStream_t s, uint64_t *p, int64_t count, uint64_t v) {
    if (count == 0) return;
    k_fill_u64<<<grid1(count, 256), 256, 0, s>>>(p, count, v);
    GRNG_LAUNCHED();
}

}  // namespace grng
