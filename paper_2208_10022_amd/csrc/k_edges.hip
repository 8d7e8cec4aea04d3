// Edge canonicalization: surviving pairs -> sorted (u < v) pairs of point ids.
// Counting pass per smaller endpoint, exclusive scan, scatter, then each
// endpoint's short neighbour list is sorted in place, so the output order is
// canonical (u ascending, then v ascending) whatever the order pairs arrived.
#include "common.h"

namespace grng {

namespace {

__device__ inline void pair_ids(int64_t p, const int32_t *px, const int32_t *py, const int32_t *perm, int32_t &u,
                                int32_t &v) {
    int32_t a = px[p], b = py[p];
    if (perm) {
        a = perm[a];
        b = perm[b];
    }
    u = a < b ? a : b;
    v = a < b ? b : a;
}

__global__ void k_edges_count(int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                              const int32_t *perm, int32_t *deg) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= npairs || !alive[p]) return;
    int32_t u, v;
    pair_ids(p, px, py, perm, u, v);
    atomicAdd(&deg[u], 1);
}

__global__ void k_edges_fill(int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                             const int32_t *perm, const int64_t *off, int32_t *fillpos, int32_t *nbr) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= npairs || !alive[p]) return;
    int32_t u, v;
    pair_ids(p, px, py, perm, u, v);
    const int32_t slot = atomicAdd(&fillpos[u], 1);
    nbr[off[u] + slot] = v;
}

__global__ void k_edges_emit(int64_t n, const int64_t *off, int32_t *nbr, int32_t *uv) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int64_t b = off[u], e = off[u + 1];
    for (int64_t s = b + 1; s < e; ++s) {   // insertion sort: lists are short
        const int32_t v = nbr[s];
        int64_t t = s - 1;
        while (t >= b && nbr[t] > v) {
            nbr[t + 1] = nbr[t];
            --t;
        }
        nbr[t + 1] = v;
    }
    for (int64_t s = b; s < e; ++s) {
        uv[2 * s] = (int32_t)u;
        uv[2 * s + 1] = nbr[s];
    }
}

__global__ void k_bits_count(int64_t m, const uint64_t *bits, int32_t words, int32_t *deg) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t c = 0;
    for (int32_t w = 0; w < words; ++w) {
        uint64_t word = bits[i * words + w];
        const int64_t lo = (int64_t)w * 64;
        if (lo + 63 <= i) continue;
        if (lo <= i) word &= (i - lo == 63) ? 0ull : (~0ull << (i - lo + 1));
        c += __popcll(word);
    }
    deg[i] = c;
}

__global__ void k_bits_emit(int64_t m, const uint64_t *bits, int32_t words, const int64_t *off, int32_t *uv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t s = off[i];
    for (int32_t w = 0; w < words; ++w) {
        uint64_t word = bits[i * words + w];
        const int64_t lo = (int64_t)w * 64;
        if (lo + 63 <= i) continue;
        if (lo <= i) word &= (i - lo == 63) ? 0ull : (~0ull << (i - lo + 1));
        while (word) {
            const int b = __ffsll((long long)word) - 1;
            word &= word - 1;
            uv[2 * s] = (int32_t)i;
            uv[2 * s + 1] = (int32_t)(lo + b);
            ++s;
        }
    }
}

inline unsigned grid1(int64_t work) { return (unsigned)(div_up(work, 256) < 1 ? 1 : div_up(work, 256)); }

}  // namespace

void launch_edges_count(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                        const int32_t *perm, int32_t *deg) {
    if (npairs == 0) return;
    k_edges_count<<<grid1(npairs), 256, 0, s>>>(npairs, px, py, alive, perm, deg);
    GRNG_LAUNCHED();
}

void launch_edges_fill(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                       const int32_t *perm, const int64_t *off, int32_t *fillpos, int32_t *nbr) {
    if (npairs == 0) return;
    k_edges_fill<<<grid1(npairs), 256, 0, s>>>(npairs, px, py, alive, perm, off, fillpos, nbr);
    GRNG_LAUNCHED();
}

void launch_edges_emit(hipStream_t s, int64_t n, const int64_t *off, int32_t *nbr, int32_t *uv) {
    if (n == 0) return;
    k_edges_emit<<<grid1(n), 256, 0, s>>>(n, off, nbr, uv);
    GRNG_LAUNCHED();
}

void launch_bits_to_edges_count(hipStream_t s, int64_t m, const uint64_t *bits, int32_t words, int32_t *deg) {
    if (m == 0) return;
    k_bits_count<<<grid1(m), 256, 0, s>>>(m, bits, words, deg);
    GRNG_LAUNCHED();
}

void launch_bits_to_edges_emit(hipStream_t s, int64_t m, const uint64_t *bits, int32_t words, const int64_t *off,
                               int32_t *uv) {
    if (m == 0) return;
    k_bits_emit<<<grid1(m), 256, 0, s>>>(m, bits, words, off, uv);
    GRNG_LAUNCHED();
}

}  // namespace grng
