// Sampled shortest-path statistics: the average path length and the diameter
// estimate of the paper's Table 2 (Results), both taken over breadth-first
// searches from a sample of source vertices.
//
// Sources are searched 64 at a time, one bit per source in a 64-bit word per
// vertex (bit-parallel multi-source BFS).  Every level is one bottom-up sweep:
// a vertex ORs the frontier words of its neighbours, and the bits it had not
// seen yet are the sources that reach it at this level.  A vertex stops
// reading neighbours as soon as every source of the group has reached it, so
// late levels touch little memory.  Vertices of degree above kHeavy are swept
// by a whole wavefront (lanes split the neighbour list, then OR-reduce), the
// rest by one lane each.  Counts are integers and the OR is order-free, so
// the result does not depend on scheduling.
#include <string.h>

#include <algorithm>

#include "common.hpp"

namespace sfg {
namespace {

constexpr int kPathThreads = 256;
constexpr uint32_t kHeavy = 64;      // degree above which a wavefront sweeps the vertex
constexpr int kGroup = 64;           // sources per bit-parallel search

struct PsPlan {
    size_t off_vis, off_f0, off_f1, off_heavy, off_nheavy, off_cnt, total;
};

PsPlan ps_plan(uint64_t n) {
    PsPlan p;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += align256(b);
        return r;
    };
    p.off_vis = take(n * 8);
    p.off_f0 = take(n * 8);
    p.off_f1 = take(n * 8);
    p.off_heavy = take(n * 8);
    p.off_nheavy = take(8);
    p.off_cnt = take(8);
    p.total = o;
    return p;
}

// Compact list of the heavy vertices (order irrelevant: every use is an OR or
// an integer sum per vertex).
__global__ __launch_bounds__(kPathThreads) void ps_heavy_list(const uint64_t *rp, uint64_t n, uint64_t *heavy,
                                                            unsigned long long *nheavy) {
    const uint64_t stride = (uint64_t)gridDim.x * kPathThreads;
    for (uint64_t v = (uint64_t)blockIdx.x * kPathThreads + threadIdx.x; v < n; v += stride)
        if (rp[v + 1] - rp[v] > kHeavy) heavy[atomicAdd(nheavy, 1ull)] = v;
}

struct Sources {
    int64_t v[kGroup];
    uint32_t count;
};

__global__ void ps_seed(Sources s, uint64_t *vis, uint64_t *front) {
    // One thread: sources may repeat, and their bits then share a word.
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (uint32_t i = 0; i < s.count; ++i) {
            vis[s.v[i]] |= 1ull << i;
            front[s.v[i]] |= 1ull << i;
        }
}

__device__ __forceinline__ void add_count(unsigned long long *cnt, uint64_t x) {
    __shared__ unsigned long long s_acc[kPathThreads / 64];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kPathThreads / 64; ++i) t += s_acc[i];
        if (t) atomicAdd(cnt, t);
    }
}

// Light vertices, one lane each.  next[v] is written for every vertex.
template <typename IdT>
__global__ __launch_bounds__(kPathThreads) void ps_level_light(const uint64_t *rp, const IdT *col, uint64_t n,
                                                              uint64_t all, uint64_t *vis, const uint64_t *front,
                                                              uint64_t *next, unsigned long long *cnt) {
    uint64_t found = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kPathThreads;
    for (uint64_t v = (uint64_t)blockIdx.x * kPathThreads + threadIdx.x; v < n; v += stride) {
        const uint64_t e0 = rp[v], e1 = rp[v + 1];
        if (e1 - e0 > kHeavy) continue;  // swept by ps_level_heavy
        const uint64_t seen = vis[v];
        uint64_t acc = 0;
        if (seen != all)
            for (uint64_t e = e0; e < e1; ++e) {
                const uint64_t x = (uint64_t)col[e];
                if (x < n) acc |= front[x];  // ids at or above n are not vertices
                if ((acc | seen) == all) break;
            }
        const uint64_t fresh = acc & ~seen;
        next[v] = fresh;
        if (fresh) {
            vis[v] = seen | fresh;
            found += (uint64_t)__popcll(fresh);
        }
    }
    add_count(cnt, found);
}

// Heavy vertices, one wavefront each.
template <typename IdT>
__global__ __launch_bounds__(kPathThreads) void ps_level_heavy(const uint64_t *rp, const IdT *col, uint64_t n,
                                                              const uint64_t *heavy, const unsigned long long *nheavy,
                                                              uint64_t all, uint64_t *vis, const uint64_t *front,
                                                              uint64_t *next, unsigned long long *cnt) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nh = *nheavy;
    const uint64_t waves = (uint64_t)gridDim.x * (kPathThreads / 64);
    uint64_t found = 0;
    for (uint64_t h = (uint64_t)blockIdx.x * (kPathThreads / 64) + (threadIdx.x >> 6); h < nh; h += waves) {
        const uint64_t v = heavy[h];
        const uint64_t e0 = rp[v], e1 = rp[v + 1];
        const uint64_t seen = vis[v];
        uint64_t acc = 0;
        if (seen != all)
            for (uint64_t base = e0; base < e1; base += 64) {
                const uint64_t e = base + lane;
                if (e < e1) {
                    const uint64_t x = (uint64_t)col[e];
                    if (x < n) acc |= front[x];
                }
                // OR over the wave; the whole wave stops once the group is
                // complete for v.
                for (int off = 32; off > 0; off >>= 1) acc |= __shfl_xor(acc, off, 64);
                if ((acc | seen) == all) break;
            }
        const uint64_t fresh = acc & ~seen;
        if (lane == 0) {
            next[v] = fresh;
            if (fresh) {
                vis[v] = seen | fresh;
                found += (uint64_t)__popcll(fresh);
            }
        }
    }
    add_count(cnt, found);
}

__global__ void ps_accumulate(const unsigned long long *cnt, uint64_t level, uint64_t *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *cnt) {
        out[0] += level * (uint64_t)*cnt;
        out[1] += (uint64_t)*cnt;
        out[2] = out[2] > level ? out[2] : level;
    }
}

int grid_of(uint64_t items) {
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((items + kPathThreads - 1) / kPathThreads,
                                                         (uint64_t)device_cu_count() * 8));
}

template <typename T> __global__ void ps_fill(T *p, uint64_t n, T v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename IdT>
int run_paths(uint64_t n, const uint64_t *rp, const IdT *col, const int64_t *sources, uint32_t num_sources,
              uint64_t *out, char *ws, const PsPlan &P, hipStream_t s) {
    uint64_t *vis = reinterpret_cast<uint64_t *>(ws + P.off_vis);
    uint64_t *fa = reinterpret_cast<uint64_t *>(ws + P.off_f0);
    uint64_t *fb = reinterpret_cast<uint64_t *>(ws + P.off_f1);
    uint64_t *heavy = reinterpret_cast<uint64_t *>(ws + P.off_heavy);
    auto *nheavy = reinterpret_cast<unsigned long long *>(ws + P.off_nheavy);
    auto *cnt = reinterpret_cast<unsigned long long *>(ws + P.off_cnt);
    const int g = grid_of(n);
    ps_fill<uint64_t><<<1, 64, 0, s>>>(out, 3, 0);
    ps_fill<unsigned long long><<<1, 64, 0, s>>>(nheavy, 1, 0);
    { ProfScope _ps("path_level", s); ps_heavy_list<<<g, kPathThreads, 0, s>>>(rp, n, heavy, nheavy); }
    for (uint32_t g0 = 0; g0 < num_sources; g0 += kGroup) {
        Sources src;
        memset(&src, 0, sizeof(src));
        src.count = std::min<uint32_t>(kGroup, num_sources - g0);
        for (uint32_t i = 0; i < src.count; ++i) src.v[i] = sources[g0 + i];
        const uint64_t all = src.count == 64 ? ~0ull : ((1ull << src.count) - 1);
        ps_fill<uint64_t><<<g, kPathThreads, 0, s>>>(vis, n, 0);
        ps_fill<uint64_t><<<g, kPathThreads, 0, s>>>(fa, n, 0);
        ps_seed<<<1, 64, 0, s>>>(src, vis, fa);
        // A level finds at least one new (source, vertex) pair or ends the
        // search, so at most n levels run.
        for (uint64_t level = 1; level <= n; ++level) {
            ps_fill<unsigned long long><<<1, 64, 0, s>>>(cnt, 1, 0);
            { ProfScope _ps("path_level", s); ps_level_light<IdT><<<g, kPathThreads, 0, s>>>(rp, col, n, all, vis, fa, fb, cnt); }
            { ProfScope _ps("path_level", s); ps_level_heavy<IdT><<<g, kPathThreads, 0, s>>>(rp, col, n, heavy, nheavy, all, vis, fa, fb, cnt); }
            ps_accumulate<<<1, 1, 0, s>>>(cnt, level, out);
            unsigned long long found = 0;
            if (hipMemcpyAsync(&found, cnt, sizeof(found), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(SFG_EDEVICE, "path_stats: %s", hipGetErrorString(hipGetLastError()));
            if (found == 0) break;
            std::swap(fa, fb);
        }
    }
    return check_launch("path_stats");
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t path_stats_workspace_bytes(uint64_t n) { return n ? ps_plan(n).total : 0; }

extern "C" int path_stats(uint64_t n, const uint64_t *row_ptr, const void *col, int id_bytes, const int64_t *sources,
                          uint32_t num_sources, uint64_t *out, void *workspace, size_t workspace_bytes, void *stream) {
    if (n == 0) return fail(SFG_EINVAL, "path_stats: n must be >= 1");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "path_stats: id_bytes must be 4 or 8");
    if (!row_ptr || !col || !out) return fail(SFG_EINVAL, "path_stats: NULL buffer");
    if (num_sources > 0 && !sources) return fail(SFG_EINVAL, "path_stats: NULL sources");
    for (uint32_t i = 0; i < num_sources; ++i)
        if (sources[i] < 0 || (uint64_t)sources[i] >= n)
            return fail(SFG_EINVAL, "path_stats: source %u = %lld is not a vertex", i, (long long)sources[i]);
    const PsPlan P = ps_plan(n);
    if (!workspace) return fail(SFG_EINVAL, "path_stats: workspace is NULL");
    if (workspace_bytes < P.total)
        return fail(SFG_ENOSPACE, "path_stats: workspace has %zu bytes, needs %zu", workspace_bytes, P.total);
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    if (id_bytes == 4)
        return run_paths<int32_t>(n, row_ptr, static_cast<const int32_t *>(col), sources, num_sources, out, ws, P, s);
    return run_paths<int64_t>(n, row_ptr, static_cast<const int64_t *>(col), sources, num_sources, out, ws, P, s);
}
