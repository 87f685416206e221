// Graph statistics: the 32-bin degree histogram, the tail exponent of the
// degree distribution and a wedge-closure sample, for one graph or for every
// graph of a batch whose edge lists share one vertex space (graph g owns
// vertices [v0, v1)).
//
// The paper characterises its graphs by their degree distributions and fitted
// power-law exponents (Results, Fig. 3; a finite mean degree implies
// gamma > 2).  The exponent here is the discrete maximum-likelihood
// approximation of Clauset, Shalizi & Newman (SIAM Review 2009):
//   gamma = 1 + N_t / sum_{d >= d_min} ln(d / (d_min - 1/2)),
// over vertices of degree >= d_min = 2 ceil(2E / n), computed in binary64.
// The summation order is fixed by the graph's own vertex numbering (chunks of
// 4096 vertices, a fixed tree inside each chunk and across chunks), so a graph
// gets the same bits alone or inside a batch, on every run and device.
// Wedges are sampled on the simple undirected graph (symmetrized, no
// self-loops, no repeats): centre v with probability proportional to
// C(d_v, 2), then two distinct neighbours; the wedge is closed when they are
// adjacent.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "stats.hpp"

namespace sfg {
namespace {

constexpr int kChunk = 4096;  // vertices per statistics chunk
constexpr int kChunkThreads = 256;
constexpr int kPer = kChunk / kChunkThreads;

__device__ __forceinline__ int log2_bin(uint64_t d) {
    if (d == 0) return 0;
    const int b = 64 - __clzll(d);  // floor(log2 d) + 1
    return b > 31 ? 31 : b;
}

// The graph owning statistics chunk c (binary search over chunk0).
__device__ __forceinline__ uint32_t graph_of_chunk(const StatGraph *G, uint32_t count, uint64_t c) {
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (G[mid].chunk0 <= c)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One workgroup per chunk: degree histogram (integer atomics) and the
// exponent's partial sum and count in a fixed order.
// Workgroups walk the chunks (persistent: a grid smaller than the chunk count
// takes chunks blockIdx.x, blockIdx.x + gridDim.x, ...): degree histogram
// (integer atomics) and the exponent's partial sum and count of each chunk in
// a fixed order, so the grid does not change any result.
__global__ __launch_bounds__(kChunkThreads) void stats_chunks(const StatGraph *G, uint32_t count, uint64_t total,
                                                              const uint64_t *raw, uint64_t *hist, double *psum,
                                                              uint64_t *pcnt) {
    __shared__ uint32_t s_h[32];
    __shared__ double s_sum[kChunkThreads];
    __shared__ uint64_t s_cnt[kChunkThreads];
    __shared__ uint32_t s_g;
    for (uint64_t c = blockIdx.x; c < total; c += gridDim.x) {
        if (threadIdx.x == 0) s_g = graph_of_chunk(G, count, c);
        if (threadIdx.x < 32) s_h[threadIdx.x] = 0;
        __syncthreads();
        const StatGraph &g = G[s_g];
        const uint64_t v0 = g.v0 + (c - g.chunk0) * kChunk;
        const double denom = (double)g.dmin - 0.5;
        double sum = 0.0;
        uint64_t cnt = 0;
        for (int j = 0; j < kPer; ++j) {
            const uint64_t v = v0 + (uint64_t)threadIdx.x * kPer + j;
            if (v < g.v1) {
                const uint64_t d = raw[v + 1] - raw[v];
                atomicAdd(&s_h[log2_bin(d)], 1u);
                if (d >= g.dmin && d > 0) {
                    sum += log((double)d / denom);
                    ++cnt;
                }
            }
        }
        s_sum[threadIdx.x] = sum;
        s_cnt[threadIdx.x] = cnt;
        __syncthreads();
        for (int off = kChunkThreads / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
                s_cnt[threadIdx.x] += s_cnt[threadIdx.x + off];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            psum[c] = s_sum[0];
            pcnt[c] = s_cnt[0];
        }
        if (threadIdx.x < 32 && s_h[threadIdx.x])
            atomicAdd((unsigned long long *)&hist[(uint64_t)g.out * 32 + threadIdx.x],
                      (unsigned long long)s_h[threadIdx.x]);
        __syncthreads();  // s_g, s_h and the partial sums are reused by the next chunk
    }
}

// One workgroup per graph: the exponent from its chunks' partials.
__global__ __launch_bounds__(256) void stats_gamma(const StatGraph *G, const double *psum, const uint64_t *pcnt,
                                                   double *gamma) {
    __shared__ double s_sum[256];
    __shared__ uint64_t s_cnt[256];
    const StatGraph &g = G[blockIdx.x];
    const uint64_t nch = (g.v1 - g.v0 + kChunk - 1) / kChunk;
    double sum = 0.0;
    uint64_t cnt = 0;
    for (uint64_t c = threadIdx.x; c < nch; c += 256) {
        sum += psum[g.chunk0 + c];
        cnt += pcnt[g.chunk0 + c];
    }
    s_sum[threadIdx.x] = sum;
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        gamma[g.out] = (s_cnt[0] > 0 && s_sum[0] > 0.0) ? 1.0 + (double)s_cnt[0] / s_sum[0] : (double)NAN;
}

// Inclusive prefix sum of C(d_v, 2) over the simple CSR's degrees, in three
// steps over chunks of kChunk vertices of the whole vertex space.
__device__ __forceinline__ uint64_t pairs_of(const uint64_t *rp, uint64_t v) {
    const uint64_t d = rp[v + 1] - rp[v];
    return d >= 2 ? d * (d - 1) / 2 : 0;
}

__global__ __launch_bounds__(256) void wedge_chunk_sums(const uint64_t *rp, uint64_t n, uint64_t *csum) {
    __shared__ uint64_t s[256];
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    uint64_t acc = 0;
    for (uint64_t v = c0 + threadIdx.x; v < c0 + kChunk && v < n; v += 256) acc += pairs_of(rp, v);
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) csum[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void wedge_chunk_scan(uint64_t *csum, uint64_t nchunks) {
    __shared__ uint64_t s[1024];
    const uint64_t per = (nchunks + 1023) / 1024;
    const uint64_t lo = (uint64_t)threadIdx.x * per, hi = min(lo + per, nchunks);
    uint64_t acc = 0;
    for (uint64_t c = lo; c < hi; ++c) acc += csum[c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t o = threadIdx.x >= (uint32_t)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += o;
        __syncthreads();
    }
    uint64_t run = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
    for (uint64_t c = lo; c < hi; ++c) {
        const uint64_t x = csum[c];
        csum[c] = run;
        run += x;
    }
}

__global__ __launch_bounds__(256) void wedge_chunk_apply(const uint64_t *rp, uint64_t n, const uint64_t *cbase,
                                                         uint64_t *pre) {
    __shared__ uint64_t s[256];
    constexpr int per = kChunk / 256;
    const uint64_t v0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * per;
    uint64_t x[per];
    uint64_t acc = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        x[j] = v0 + j < n ? pairs_of(rp, v0 + j) : 0;
        acc += x[j];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t o = threadIdx.x >= (uint32_t)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += o;
        __syncthreads();
    }
    uint64_t run = cbase[blockIdx.x] + (threadIdx.x > 0 ? s[threadIdx.x - 1] : 0);
#pragma unroll
    for (int j = 0; j < per; ++j) {
        run += x[j];
        if (v0 + j < n) pre[v0 + j] = run;
    }
}

template <typename IdT>
__device__ __forceinline__ bool adjacent(const uint64_t *rp, const IdT *col, uint64_t v, uint64_t w) {
    uint64_t lo = rp[v], hi = rp[v + 1];
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)col[mid] < w)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < rp[v + 1] && (uint64_t)col[lo] == w;
}

struct WedgeArgs {
    const StatGraph *G;
    uint32_t count, samples;
    const uint64_t *rp, *pre;
    const void *col;
    uint32_t key0, key1;
    unsigned long long *closed;  // indexed by StatGraph::out
    uint64_t nv;                 // vertices of the shared space
};

// Sample i of graph g: Philox block (i, 0, 0, WEDGE | gid << 8).
template <typename IdT> __global__ __launch_bounds__(256) void wedge_sample(WedgeArgs a) {
    const uint64_t total_items = (uint64_t)a.count * a.samples;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t it = (uint64_t)blockIdx.x * 256 + threadIdx.x; it < total_items; it += stride) {
        const StatGraph &g = a.G[it / a.samples];
        const uint32_t i = (uint32_t)(it % a.samples);
        if (g.v1 == g.v0) continue;
        const uint64_t base = g.v0 > 0 ? a.pre[g.v0 - 1] : 0;
        const uint64_t total = a.pre[g.v1 - 1] - base;
        if (total == 0) continue;
        const Block4 w = philox(i, 0, 0, TAG_WEDGE | (g.gid << 8), a.key0, a.key1);
        const uint64_t target = base + uidx64(make_u64(w.w0, w.w1), total);
        // centre: first v with pre[v] > target
        uint64_t lo = g.v0, hi = g.v1;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (a.pre[mid] > target)
                hi = mid;
            else
                lo = mid + 1;
        }
        const uint64_t v = lo;
        const IdT *col = static_cast<const IdT *>(a.col);
        const uint32_t d = (uint32_t)(a.rp[v + 1] - a.rp[v]);
        const uint32_t x = uidx32(w.w2, d);
        uint32_t y = uidx32(w.w3, d - 1);
        if (y >= x) ++y;
        const uint64_t na = (uint64_t)col[a.rp[v] + x], nb = (uint64_t)col[a.rp[v] + y];
        // (ids outside the vertex space come only from invalid input; they
        // are never looked up)
        if (na < a.nv && adjacent<IdT>(a.rp, col, na, nb)) atomicAdd(&a.closed[g.out], 1ull);
    }
}

__global__ void stats_clear(const StatGraph *G, uint32_t count, uint64_t *hist, long long *closed) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count * 32) return;
    const StatGraph &g = G[i / 32];
    hist[(uint64_t)g.out * 32 + i % 32] = 0;
    if (i % 32 == 0) closed[g.out] = 0;
}

// closed = -1 for a graph with no wedge at all.
__global__ void wedge_mark_empty(const StatGraph *G, uint32_t count, const uint64_t *pre, long long *closed) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const StatGraph &g = G[i];
    const uint64_t base = g.v0 > 0 ? pre[g.v0 - 1] : 0;
    if (g.v1 == g.v0 || pre[g.v1 - 1] == base) closed[g.out] = -1;
}

}  // namespace

uint64_t stats_chunks_of(uint64_t n) { return (n + kChunk - 1) / kChunk; }

size_t stats_scratch_bytes(uint64_t nv, uint64_t total_chunks) {
    const uint64_t vchunks = (nv + kChunk - 1) / kChunk;
    return align256(std::max<uint64_t>(nv, 1) * 8) + align256(std::max<uint64_t>(vchunks, 1) * 8) +
           align256(std::max<uint64_t>(total_chunks, 1) * 8) * 2;
}

int stats_enqueue(const StatGraph *G_dev, uint32_t count, uint64_t total_chunks, uint64_t nv, const uint64_t *raw,
                  const uint64_t *rp, const void *col, int id_bytes, uint32_t samples, uint64_t seed, uint64_t *hist,
                  double *gamma, int64_t *closed, void *scratch, hipStream_t s, uint32_t grid) {
    char *p = static_cast<char *>(scratch);
    uint64_t *pre = reinterpret_cast<uint64_t *>(p);
    p += align256(std::max<uint64_t>(nv, 1) * 8);
    const uint64_t vchunks = (nv + kChunk - 1) / kChunk;
    uint64_t *csum = reinterpret_cast<uint64_t *>(p);
    p += align256(std::max<uint64_t>(vchunks, 1) * 8);
    double *psum = reinterpret_cast<double *>(p);
    p += align256(std::max<uint64_t>(total_chunks, 1) * 8);
    uint64_t *pcnt = reinterpret_cast<uint64_t *>(p);
    long long *cl = reinterpret_cast<long long *>(closed);
    if (count == 0) return SFG_OK;
    { ProfScope _ps("stats_chunks", s); stats_clear<<<(count * 32 + 255) / 256, 256, 0, s>>>(G_dev, count, hist, cl); }
    if (total_chunks > 0) {
        ProfScope _ps("stats_chunks", s);
        const uint64_t g = grid ? std::min<uint64_t>(grid, total_chunks) : total_chunks;
        stats_chunks<<<(unsigned)g, kChunkThreads, 0, s>>>(G_dev, count, total_chunks, raw, hist, psum, pcnt);
    }
    { ProfScope _ps("stats_gamma", s); stats_gamma<<<count, 256, 0, s>>>(G_dev, psum, pcnt, gamma); }
    if (nv > 0) {
        ProfScope _ps("stats_wedge_scan", s);
        wedge_chunk_sums<<<(unsigned)vchunks, 256, 0, s>>>(rp, nv, csum);
        wedge_chunk_scan<<<1, 1024, 0, s>>>(csum, vchunks);
        wedge_chunk_apply<<<(unsigned)vchunks, 256, 0, s>>>(rp, nv, csum, pre);
    }
    if (samples > 0) {
        WedgeArgs wa{G_dev, count, samples, rp, pre, col, (uint32_t)seed, (uint32_t)(seed >> 32),
                     reinterpret_cast<unsigned long long *>(closed), nv};
        const uint64_t items = (uint64_t)count * samples;
        const unsigned g = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((items + 255) / 256, (uint64_t)device_cu_count() * 16));
        ProfScope _ps("stats_wedge", s);
        if (id_bytes == 4)
            wedge_sample<int32_t><<<g, 256, 0, s>>>(wa);
        else
            wedge_sample<int64_t><<<g, 256, 0, s>>>(wa);
    }
    { ProfScope _ps("stats_wedge", s); wedge_mark_empty<<<(count + 255) / 256, 256, 0, s>>>(G_dev, count, pre, cl); }
    return check_launch("graph statistics");
}

}  // namespace sfg

using namespace sfg;

namespace {
struct GsPlan {
    size_t off_csr, off_rp, off_col, off_table, off_hist, off_scratch, total;
};
GsPlan gs_plan(uint64_t n, uint64_t E, int id_bytes) {
    GsPlan p;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += align256(b);
        return r;
    };
    p.off_csr = take(csr_workspace_bytes(n, E, id_bytes, SFG_CSR_SYMMETRIZE | SFG_CSR_SIMPLE));
    p.off_rp = take((n + 1) * 8);
    p.off_col = take(std::max<uint64_t>(2 * E, 1) * id_bytes);
    p.off_table = take(sizeof(StatGraph));
    p.off_hist = take(0);
    p.off_scratch = take(stats_scratch_bytes(n, stats_chunks_of(n)));
    p.total = o;
    return p;
}
__global__ void set_table(StatGraph *t, StatGraph v) { *t = v; }
}  // namespace

extern "C" size_t graph_stats_workspace_bytes(uint64_t n, uint64_t num_edges, int id_bytes) {
    if (n == 0 || (id_bytes != 4 && id_bytes != 8)) return 0;
    return gs_plan(n, num_edges, id_bytes).total;
}

extern "C" int graph_stats(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes,
                           uint32_t num_samples, uint64_t seed, uint32_t graph_id, uint64_t *degree_hist32,
                           double *gamma, int64_t *closed, void *workspace, size_t workspace_bytes, void *stream) {
    if (n == 0) return fail(SFG_EINVAL, "graph_stats: n must be >= 1");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "graph_stats: id_bytes must be 4 or 8");
    if (!degree_hist32 || !gamma || !closed) return fail(SFG_EINVAL, "graph_stats: NULL output");
    if (num_edges > 0 && (!src || !dst)) return fail(SFG_EINVAL, "graph_stats: NULL edge buffer");
    if (graph_id >= (1u << 24)) return fail(SFG_EINVAL, "graph_stats: graph_id must be < 2^24");
    if (!workspace) return fail(SFG_EINVAL, "graph_stats: workspace is NULL");
    const GsPlan P = gs_plan(n, num_edges, id_bytes);
    if (workspace_bytes < P.total)
        return fail(SFG_ENOSPACE, "graph_stats: workspace has %zu bytes, needs %zu", workspace_bytes, P.total);
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    uint64_t *rp = reinterpret_cast<uint64_t *>(ws + P.off_rp);
    void *col = ws + P.off_col;
    const uint64_t *raw = nullptr;
    // The CSR's own histogram is the multigraph degree histogram.
    int rc = csr_build(n, num_edges, src, dst, id_bytes, SFG_CSR_SYMMETRIZE | SFG_CSR_SIMPLE, rp, col, degree_hist32,
                       nullptr, ws + P.off_csr, P.off_rp - P.off_csr, s, &raw);
    if (rc != SFG_OK) return rc;
    StatGraph g{0, n, 2 * ((2 * num_edges + n - 1) / n), 0, 0, graph_id};
    StatGraph *tab = reinterpret_cast<StatGraph *>(ws + P.off_table);
    { ProfScope _ps("stats_chunks", s); set_table<<<1, 1, 0, s>>>(tab, g); }
    // stats_enqueue recomputes the histogram per graph into degree_hist32.
    return stats_enqueue(tab, 1, stats_chunks_of(n), n, raw, rp, col, id_bytes, num_samples, seed, degree_hist32, gamma,
                         closed, ws + P.off_scratch, s);
}
