// Device helpers shared by the pair and lune kernels (internal header).
#pragma once

#include "common.h"

namespace grng {
namespace {

__device__ inline uint32_t wave_sum(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

constexpr int kXcds = 8;       // XCDs of an MI355X; workgroups are dealt to them round-robin

// Dynamic, XCD-aware scheduling over n items split into 8 contiguous ranges:
// a caller on XCD c claims chunks of its own range first, then helps the
// other ranges (xr counts the ranges it has exhausted).  Returns false when
// every range is used up; otherwise [*b, *e) is the claimed chunk.
__device__ inline bool claim_chunk(int64_t n, int64_t chunk, int xcd0, int &xr, unsigned long long *work,
                                   int64_t *b, int64_t *e) {
    while (xr < kXcds) {
        const int c = (xcd0 + xr) % kXcds;
        const int64_t lo = n * c / kXcds, hi = n * (c + 1) / kXcds;
        const int64_t s = lo + (int64_t)atomicAdd(&work[c * kWorkStride], 1ull) * chunk;
        if (s < hi) {
            *b = s;
            *e = s + chunk < hi ? s + chunk : hi;
            return true;
        }
        ++xr;
    }
    return false;
}

constexpr int kTile = 64;
constexpr int kPiv = 16;        // pivot witnesses per tile pair (one MFMA column block)
constexpr int kDl = kTile + 1;  // row stride (floats) of the in-tile distance matrices
constexpr float kCertain = 1.0f - 0x1p-21f;   // threshold factor of the float32 witness certificate
constexpr int kXs = kPiv + 4;   // row stride (floats) of the pivot distances: 16-byte aligned rows
constexpr int kPairChunk = 32;   // tile pairs claimed per atomic: consecutive ones mostly share T, whose rows and D(T,T) stay in LDS
constexpr int kPairRecMeta = 12;  // record words before the masks: tiles' start, length, home cell; pivot ids
constexpr int kPairRecWords = kPairRecordWords;
static_assert(kPairRecWords == kPairRecMeta + 2 * kTile, "record layout");
constexpr int kLuneChunk = 4;   // pairs claimed per atomic by one wave of the exhaustive scan

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline uint64_t uniform_u64(uint64_t v) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}
__device__ inline int64_t uniform_i64(int64_t v) { return (int64_t)uniform_u64((uint64_t)v); }

constexpr uint32_t kInfBits = 0x7f800000u;   // +inf as float32 bits
__device__ inline uint32_t umax2(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ inline uint32_t umin3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t m = a < b ? a : b;
    return m < c ? m : c;
}

// Up to 64 survivors of one wave, one per lane, appended to the pair list
// with a single atomic.
struct WaveOut {
    int cnt = 0;   // uniform
    int32_t x = 0, y = 0;
    double d2 = 0.0;
    __device__ void flush(PairList out) {
        if (cnt == 0) return;
        const int lane = threadIdx.x & 63;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long *)out.count, (unsigned long long)cnt);
        base = __shfl(base, 0, kWave);
        if (lane < cnt && (int64_t)(base + lane) < out.cap) {
            out.x[base + lane] = x;
            out.y[base + lane] = y;
            out.d2[base + lane] = d2;
        }
        cnt = 0;
    }
};


}  // namespace
}  // namespace grng
