// Learned witness-cell ranking: a 2-layer MLP that scores the candidate
// witness cells of a pair so the exhaustive scan (Section 2, Stages V-VI)
// visits the cell most likely to hold a witness first.  It only orders the
// scan: every cell is still scanned unless the pair dies, so edges never
// change.
//
//   h = relu(f W1 + b1), s = h . w2 + b2      f: 9 scale-free features
//   loss = mean softplus(s) - label * s       (cross-entropy with logits)
// Parameters: one float vector [W1 (F x H row-major), b1, w2, b2].
//
// Training: fused forward + backward over blocks of 64 samples staged in LDS,
// per-block partial gradients reduced in a fixed order (deterministic), then
// an Adam step.  Scoring in the scan uses the weights rounded to bf16 with
// float32 accumulation.
#include <mutex>

#include "common.h"

namespace grng {

namespace {

constexpr int F = kMlpFeatures, H = kMlpHidden, P = kMlpParams;
static_assert(P <= 3 * 256, "each of 256 threads owns at most three parameters");
constexpr int kB = 64;   // samples per LDS batch

__device__ inline float softplus(float s) { return s > 0.f ? s + log1pf(expf(-s)) : log1pf(expf(s)); }

// One block: samples [b0, b1) in batches of 64; 4 threads per sample compute
// 16 hidden units each.  Thread t owns parameters t, t+256, t+512 and sums
// their gradient over the block's samples in sample order.
__global__ __launch_bounds__(256) void k_mlp_grad_partial(const float *__restrict__ theta,
                                                          const float *__restrict__ feats,
                                                          const uint8_t *__restrict__ labels, int64_t n,
                                                          int64_t per_block, float *__restrict__ partial,
                                                          float *__restrict__ partial_loss) {
    __shared__ float sX[kB][F];
    __shared__ float sH[kB][H + 1];
    __shared__ float sDH[kB][H + 1];
    __shared__ float sDS[kB];
    __shared__ float sL[kB];
    const int t = threadIdx.x;
    const int64_t b0 = blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < n ? b0 + per_block : n;
    const float *W1 = theta, *bb1 = theta + F * H, *w2 = bb1 + H;
    const float b2 = theta[P - 1];
    float acc[3] = {0.f, 0.f, 0.f};
    float lacc = 0.f;
    const float inv_n = 1.0f / (float)n;
    for (int64_t base = b0; base < b1; base += kB) {
        const int i = t >> 2, q = t & 3;
        const int64_t smp = base + i;
        const bool ok = smp < b1;
        if (q == 0)
            for (int f = 0; f < F; ++f) sX[i][f] = ok ? feats[smp * F + f] : 0.f;
        __syncthreads();
        float part = 0.f;
        float pre[16];
        for (int jj = 0; jj < 16; ++jj) {
            const int j = q * 16 + jj;
            float a = bb1[j];
            for (int f = 0; f < F; ++f) a = fmaf(sX[i][f], W1[f * H + j], a);
            pre[jj] = a;
            const float h = a > 0.f ? a : 0.f;
            sH[i][j] = ok ? h : 0.f;
            part = fmaf(h, w2[j], part);
        }
        part += __shfl_xor(part, 1, kWave);
        part += __shfl_xor(part, 2, kWave);
        const float s = part + b2;
        const float y = ok ? (float)labels[smp] : 0.f;
        const float ds = ok ? (1.f / (1.f + expf(-s)) - y) * inv_n : 0.f;
        for (int jj = 0; jj < 16; ++jj) {
            const int j = q * 16 + jj;
            sDH[i][j] = pre[jj] > 0.f ? ds * w2[j] : 0.f;
        }
        if (q == 0) {
            sDS[i] = ds;
            sL[i] = ok ? softplus(s) - y * s : 0.f;
        }
        __syncthreads();
        for (int r = 0; r < 3; ++r) {
            const int p = t + 256 * r;
            if (p >= P) break;
            float a = 0.f;
            if (p < F * H) {
                const int f = p / H, j = p % H;
                for (int k = 0; k < kB; ++k) a = fmaf(sX[k][f], sDH[k][j], a);
            } else if (p < F * H + H) {
                const int j = p - F * H;
                for (int k = 0; k < kB; ++k) a += sDH[k][j];
            } else if (p < F * H + 2 * H) {
                const int j = p - F * H - H;
                for (int k = 0; k < kB; ++k) a = fmaf(sH[k][j], sDS[k], a);
            } else {
                for (int k = 0; k < kB; ++k) a += sDS[k];
            }
            acc[r] += a;
        }
        if (t == 0)
            for (int k = 0; k < kB; ++k) lacc += sL[k];
        __syncthreads();
    }
    for (int r = 0; r < 3; ++r) {
        const int p = t + 256 * r;
        if (p < P) partial[blockIdx.x * (int64_t)P + p] = acc[r];
    }
    if (t == 0) partial_loss[blockIdx.x] = lacc * inv_n;
}

// Fixed-order sum of the per-block partials (deterministic gradient).
__global__ void k_mlp_reduce(const float *partial, const float *partial_loss, int64_t nblocks, float *grad,
                             float *loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) {
        float a = 0.f;
        for (int64_t b = 0; b < nblocks; ++b) a += partial[b * P + p];
        grad[p] = a;
    }
    if (p == 0) {
        float l = 0.f;
        for (int64_t b = 0; b < nblocks; ++b) l += partial_loss[b];
        *loss = l;
    }
}

__global__ void k_adam(float *theta, const float *g, float *m, float *v, int t, float lr) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float mh = mp / (1.f - powf(b1, (float)t));
    const float vh = vp / (1.f - powf(b2, (float)t));
    theta[p] -= lr * mh / (sqrtf(vh) + eps);
}

// Round-to-nearest-even float -> bf16 (kept as uint16 bits).
__device__ inline uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void k_pack_bf16(const float *theta, uint16_t *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) out[p] = to_bf16(theta[p]);
}

__global__ void k_mlp_score(const uint16_t *__restrict__ wb, const float *__restrict__ feats, int64_t n,
                            float *__restrict__ scores) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[F];
    for (int k = 0; k < F; ++k) f[k] = feats[i * F + k];
    scores[i] = mlp_score_bf16(wb, f);
}

// Training samples from the last build's exhaustive-scan pairs: for sampled
// pairs, every candidate cell of the row point that Proposition 3 does not
// skip gives one sample (features, label = the cell holds a witness, decided
// exactly by scanning its members).  One wave per sampled pair.  Pass 0
// counts each pair's samples; pass 1 writes them at the pair's scanned
// offset in cell order, so the sample list is the same on every run.
__global__ __launch_bounds__(256) void k_log_cells(
    int64_t nsamp, int64_t npairs, const int32_t *__restrict__ px, const int32_t *__restrict__ py,
    const double *__restrict__ pd2, int dp, const double *__restrict__ Xh, const double *__restrict__ nrmh,
    const int32_t *__restrict__ grp_off, const double *__restrict__ dvor, const double *__restrict__ rad,
    const double *__restrict__ Xp, const double *__restrict__ nrmp, const int64_t *__restrict__ rel_off,
    const int32_t *__restrict__ rel_grp, const double *__restrict__ rel_d2x, const uint64_t *__restrict__ row_dmax,
    int64_t *__restrict__ cnt, const int64_t *__restrict__ off, float *__restrict__ feats,
    uint8_t *__restrict__ labels, int pass) {
    const int lane = threadIdx.x & 63;
    const int64_t s = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= nsamp) return;
    const int64_t p = (int64_t)((double)s * (double)npairs / (double)nsamp);
    const int64_t x = __builtin_amdgcn_readfirstlane(px[p]);
    const int64_t y = __builtin_amdgcn_readfirstlane(py[p]);
    const double d2 = pd2[p];
    int64_t slot = pass ? off[s] : 0;
    // a pair beyond its row's cell bound (one the partner pass decided)
    // would see only part of its cells: not a sample
    if (d2 <= 0.0 || d2 > __longlong_as_double((long long)row_dmax[x])) {
        if (!pass && lane == 0) cnt[s] = 0;
        return;
    }
    const double dxy = sqrt(d2);
    const double *xs = Xh + x * dp, *ys = Xh + y * dp;
    const double nrx = nrmh[x], nry = nrmh[y];
    for (int64_t c0 = rel_off[x]; c0 < rel_off[x + 1]; c0 += 64) {
        const int64_t c = c0 + lane;
        bool cand = false;
        float f[F];
        int32_t g = 0;
        if (c < rel_off[x + 1]) {
            g = rel_grp[c];
            double accy = 0.0;
            for (int t = 0; t < dp; ++t) accy = fma(ys[t], Xp[(int64_t)g * dp + t], accy);
            const double d2y = nry + nrmp[g] - 2.0 * accy;
            mlp_features(sqrt(rel_d2x[c]), sqrt(d2y), dvor[g], rad[g], grp_off[g + 1] - grp_off[g], dxy, f);
            cand = f[4] < 1.0f;    // Proposition 3 does not skip the cell
        }
        uint64_t todo = __ballot(cand);
        if (!pass) {
            slot += __popcll(todo);
            continue;
        }
        while (todo) {
            const int src = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int32_t gg = __shfl(g, src, kWave);
            bool wit = false;
            for (int64_t z = grp_off[gg] + lane; z < grp_off[gg + 1] && !wit; z += 64) {
                double sx = 0.0, sy = 0.0;
                for (int t = 0; t < dp; ++t) {
                    sx = fma(xs[t], Xh[z * dp + t], sx);
                    sy = fma(ys[t], Xh[z * dp + t], sy);
                }
                wit = (nrx + nrmh[z] - 2.0 * sx) < d2 && (nry + nrmh[z] - 2.0 * sy) < d2;
            }
            const bool any = __ballot(wit) != 0;
            if (lane == src) {
                for (int k = 0; k < F; ++k) feats[slot * F + k] = f[k];
                labels[slot] = any ? 1 : 0;
            }
            ++slot;
        }
    }
    if (!pass && lane == 0) cnt[s] = slot;
}

}  // namespace

namespace {

constexpr int64_t kGradPerBlock = 4096;   // samples per block of the partial-gradient kernel

// Partial gradients of ceil(n / kGradPerBlock) blocks ([nb][P], then [nb]
// losses) in `partial`, reduced in a fixed order into grad and *loss.
void grad_into(hipStream_t s, const float *theta, const float *feats, const uint8_t *labels, int64_t n,
               float *grad, float *loss, float *partial) {
    const int64_t nb = div_up(n, kGradPerBlock);
    float *pl = partial + nb * P;
    k_mlp_grad_partial<<<(unsigned)nb, 256, 0, s>>>(theta, feats, labels, n, kGradPerBlock, partial, pl);
    GRNG_LAUNCHED();
    k_mlp_reduce<<<(unsigned)div_up(P, 256), 256, 0, s>>>(partial, pl, nb, grad, loss);
    GRNG_LAUNCHED();
}

// Fixed device scratch of the allocation-free gradient: room for the
// partials of kNoAllocMaxSamples samples (4,096 blocks x 706 floats, 11.6 MB
// per device, held until the process ends).  Host code never passes the
// array's name to a kernel: on the host it is only a stand-in for the
// symbol; the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
constexpr int64_t kNoAllocBlocks = kNoAllocMaxSamples / kGradPerBlock;
static_assert(kNoAllocBlocks * kGradPerBlock == kNoAllocMaxSamples, "whole blocks");
static __device__ __align__(256) float scratch[kNoAllocBlocks * (P + 1)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};

float *scratch_of_current_device() {
    int dev = 0;
    GRNG_HIP(hipGetDevice(&dev));
    require(dev >= 0 && dev < kMaxDevices, GRNG_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        GRNG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = static_cast<float *>(ptr);
    }
    return g_scratch_dev[dev];
}

}  // namespace

void launch_mlp_grad(hipStream_t s, const float *theta, const float *feats, const uint8_t *labels, int64_t n,
                     float *grad, float *loss, DevBuf &work) {
    require(n >= 1, GRNG_EINVAL, "need at least one sample");
    const int64_t nb = div_up(n, kGradPerBlock);
    work.ensure(sizeof(float) * (size_t)(nb * P + nb));
    grad_into(s, theta, feats, labels, n, grad, loss, work.as<float>());
}

void launch_mlp_grad_noalloc(hipStream_t s, const float *theta, const float *feats, const uint8_t *labels,
                             int64_t n, float *grad, float *loss_dev) {
    require(n >= 1 && n <= kNoAllocMaxSamples, GRNG_EINVAL,
            "grng_mlp_grad_noalloc takes 1 to GRNG_MLP_NOALLOC_MAX_SAMPLES samples");
    grad_into(s, theta, feats, labels, n, grad, loss_dev, scratch_of_current_device());
}

void launch_adam(hipStream_t s, float *theta, const float *g, float *m, float *v, int t, float lr) {
    k_adam<<<(unsigned)div_up(P, 256), 256, 0, s>>>(theta, g, m, v, t, lr);
    GRNG_LAUNCHED();
}

void launch_pack_bf16(hipStream_t s, const float *theta, uint16_t *out) {
    k_pack_bf16<<<(unsigned)div_up(P, 256), 256, 0, s>>>(theta, out);
    GRNG_LAUNCHED();
}

void launch_mlp_score(hipStream_t s, const uint16_t *wb, const float *feats, int64_t n, float *scores) {
    if (n == 0) return;
    k_mlp_score<<<(unsigned)div_up(n, 256), 256, 0, s>>>(wb, feats, n, scores);
    GRNG_LAUNCHED();
}

int64_t launch_log_cells(hipStream_t s, int64_t nsamp, int64_t npairs, const int32_t *px, const int32_t *py,
                         const double *pd2, int dp, const double *Xh, const double *nrmh, const int32_t *grp_off,
                         const double *dvor, const double *rad, const double *Xp, const double *nrmp,
                         const int64_t *rel_off, const int32_t *rel_grp, const double *rel_d2x,
                         const uint64_t *row_dmax, float *feats, uint8_t *labels, int64_t capacity) {
    if (nsamp == 0 || npairs == 0) return 0;
    DevBuf cnt, off;
    cnt.alloc(sizeof(int64_t) * (size_t)nsamp);
    off.alloc(sizeof(int64_t) * (size_t)(nsamp + 1));
    const unsigned grid = (unsigned)div_up(nsamp, 4);
    k_log_cells<<<grid, 256, 0, s>>>(nsamp, npairs, px, py, pd2, dp, Xh, nrmh, grp_off, dvor, rad, Xp, nrmp, rel_off,
                                     rel_grp, rel_d2x, row_dmax, cnt.as<int64_t>(), nullptr, nullptr, nullptr, 0);
    GRNG_LAUNCHED();
    launch_scan_i64(s, cnt.as<int64_t>(), nsamp, off.as<int64_t>());
    int64_t total = 0;
    GRNG_HIP(hipMemcpyAsync(&total, off.as<int64_t>() + nsamp, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GRNG_HIP(hipStreamSynchronize(s));
    if (total > capacity || total == 0) return total;
    k_log_cells<<<grid, 256, 0, s>>>(nsamp, npairs, px, py, pd2, dp, Xh, nrmh, grp_off, dvor, rad, Xp, nrmp, rel_off,
                                     rel_grp, rel_d2x, row_dmax, nullptr, off.as<int64_t>(), feats, labels, 1);
    GRNG_LAUNCHED();
    GRNG_HIP(hipStreamSynchronize(s));
    return total;
}

}  // namespace grng
