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
template <class TI>
__global__ __launch_bounds__(1024) void k_scan(const TI *in, int64_t n, int64_t *out) {
    constexpr int kPer = 4;
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < n; b0 += 1024 * kPer) {
        const int64_t i0 = b0 + (int64_t)t * kPer;
        int64_t v[kPer], sum = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            v[u] = i0 + u < n ? (int64_t)in[i0 + u] : 0;
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
            if (i0 + u < n) out[i0 + u] = run;
            run += v[u];
        }
        carry += total;
        __syncthreads();   // wsum is rewritten by the next pass
    }
    if (t == 0) out[n] = carry;
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

void launch_scan_i64(hipStream_t s, const int64_t *in, int64_t n, int64_t *out_excl) {
    k_scan<int64_t><<<1, 1024, 0, s>>>(in, n, out_excl);
    GRNG_LAUNCHED();
}

void launch_scan_i32_to_i64(hipStream_t s, const int32_t *in, int64_t n, int64_t *out_excl) {
    k_scan<int32_t><<<1, 1024, 0, s>>>(in, n, out_excl);
    GRNG_LAUNCHED();
}

void launch_bits_transpose(hipStream_t s, const uint64_t *rows, int64_t n, int32_t words, int64_t m,
                           uint64_t *cols) {
    const int64_t nw = div_up(n, 64);
    if (m == 0 || nw == 0) return;
    k_bits_transpose<<<grid1(m * nw, 256), 256, 0, s>>>(rows, n, words, m, cols, nw);
    GRNG_LAUNCHED();
}

void launch_fill_u64(hipStream_t s, uint64_t *p, int64_t count, uint64_t v) {
    if (count == 0) return;
    k_fill_u64<<<grid1(count, 256), 256, 0, s>>>(p, count, v);
    GRNG_LAUNCHED();
}

}  // namespace grng
