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

// Exact d^2 of listed pairs (one set, home order) and the per-row maximum.
__global__ void k_pair_d2(int64_t np, const int32_t *px, const int32_t *py, int dp, const double *Xh,
                          const double *nrmh, double *d2, unsigned long long *dmax_bits) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int64_t x = px[p], y = py[p];
    double acc = 0.0;
    for (int t = 0; t < dp; ++t) acc = fma(Xh[x * dp + t], Xh[y * dp + t], acc);
    const double v = nrmh[x] + nrmh[y] - 2.0 * acc;
    d2[p] = v;
    atomicMax(&dmax_bits[x], (unsigned long long)__double_as_longlong(v));
}

// Query output: pass 0 counts neighbours per query, pass 1 scatters the
// neighbour's point id into the query's CSR segment.
__global__ void k_query_csr(int64_t np, const int32_t *px, const int32_t *py, const uint8_t *alive,
                            const int32_t *qperm, const int32_t *perm, int32_t *deg, const int64_t *off,
                            int32_t *fill, int32_t *nbr, int pass) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= np || !alive[p]) return;
    const int32_t q = qperm ? qperm[px[p]] : px[p];
    const int32_t v = perm ? perm[py[p]] : py[p];
    if (pass == 0) {
        atomicAdd(&deg[q], 1);
    } else {
        nbr[off[q] + atomicAdd(&fill[q], 1)] = v;
    }
}

__global__ void k_sort_segments(int64_t nseg, const int64_t *off, int32_t *vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nseg) return;
    const int64_t b = off[i], e = off[i + 1];
    for (int64_t s = b + 1; s < e; ++s) {
        const int32_t v = vals[s];
        int64_t t = s - 1;
        while (t >= b && vals[t] > v) {
            vals[t + 1] = vals[t];
            --t;
        }
        vals[t + 1] = v;
    }
}

// Existing edges (point ids) -> pairs of home-order positions.
__global__ void k_edges_to_pairs(int64_t ne, const int32_t *uv, const int32_t *inv, int32_t *px, int32_t *py) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= ne) return;
    px[e] = inv[uv[2 * e]];
    py[e] = inv[uv[2 * e + 1]];
}

// Pair endpoints from set positions to point ids: px[p] = mx[px[p]], py[p] = my[py[p]].
__global__ void k_pairs_to_ids(int64_t np, int32_t *px, int32_t *py, const int32_t *mx, const int32_t *my) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= np) return;
    px[p] = mx[px[p]];
    py[p] = my[py[p]];
}

// Values through a table: v[t] = map[v[t]] (pivot-list positions to point ids).
__global__ void k_map_ids(int64_t count, int32_t *v, const int32_t *map) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < count) v[t] = map[v[t]];
}

inline unsigned grid1(int64_t work) { return (unsigned)(div_up(work, 256) < 1 ? 1 : div_up(work, 256)); }

}  // namespace

void launch_pair_d2(hipStream_t s, int64_t np, const int32_t *px, const int32_t *py, int dp, const double *Xh,
                    const double *nrmh, double *d2, uint64_t *dmax_bits) {
    if (np == 0) return;
    k_pair_d2<<<grid1(np), 256, 0, s>>>(np, px, py, dp, Xh, nrmh, d2, (unsigned long long *)dmax_bits);
    GRNG_LAUNCHED();
}

void launch_query_csr(hipStream_t s, int64_t npairs, const int32_t *px, const int32_t *py, const uint8_t *alive,
                      const int32_t *qperm, const int32_t *perm, int64_t nq, int32_t *deg, const int64_t *off,
                      int32_t *fill, int32_t *nbr, int pass) {
    (void)nq;
    if (npairs == 0) return;
    k_query_csr<<<grid1(npairs), 256, 0, s>>>(npairs, px, py, alive, qperm, perm, deg, off, fill, nbr, pass);
    GRNG_LAUNCHED();
}

void launch_edges_to_pairs(hipStream_t s, int64_t ne, const int32_t *uv, const int32_t *inv, int32_t *px, int32_t *py) {
    if (ne == 0) return;
    k_edges_to_pairs<<<grid1(ne), 256, 0, s>>>(ne, uv, inv, px, py);
    GRNG_LAUNCHED();
}

void launch_pairs_to_ids(hipStream_t s, int64_t np, int32_t *px, int32_t *py, const int32_t *mx, const int32_t *my) {
    if (np == 0) return;
    k_pairs_to_ids<<<grid1(np), 256, 0, s>>>(np, px, py, mx, my);
    GRNG_LAUNCHED();
}

void launch_map_ids(hipStream_t s, int64_t count, int32_t *v, const int32_t *map) {
    if (count == 0) return;
    k_map_ids<<<grid1(count), 256, 0, s>>>(count, v, map);
    GRNG_LAUNCHED();
}

void launch_sort_segments(hipStream_t s, int64_t nseg, const int64_t *off, int32_t *vals) {
    if (nseg == 0) return;
    k_sort_segments<<<grid1(nseg), 256, 0, s>>>(nseg, off, vals);
    GRNG_LAUNCHED();
}

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
