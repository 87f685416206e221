// Randomized PK by temporary seed modification (PK section, randomization):
// at every expansion a meta-edge is replaced by the edges of its own
// perturbed copy of the seed (absent cells added with probability p_add,
// present cells deleted with probability p_del; draws keyed by the
// meta-edge's iteration and coordinates).
//
// The paper's processors expand meta-edges depth first.  Here the expansion
// is level-synchronous: per iteration every meta-edge computes its perturbed
// cell mask and fan-out, an exclusive scan of the fan-outs gives each its
// output range, and a second sweep writes the children in cell order.  That
// order is the depth-first order of the paper's stack, so the edge list is
// the same, entry for entry.  The fan-out varies per meta-edge, which is why
// the scan is needed; the host reads the level total to size the next level.
#include <string.h>

#include <algorithm>

#include "common.hpp"

namespace sfg {
namespace {

constexpr uint32_t TAG_PERTURB = 7;
constexpr int kPtThreads = 256;
constexpr int kScanPer = 16;                            // fan-outs per thread in the scan
constexpr uint64_t kScanBlock = kPtThreads * kScanPer;  // fan-outs per scan workgroup

struct PtArgs {
    uint64_t adj;            // seed cells as bits (n0 <= 8)
    uint32_t n0, cells;
    uint32_t key0, key1, tagword;
    uint64_t thr_add, thr_del;
};

// The perturbed cell mask of meta-edge (iteration it, row, col).
__device__ __forceinline__ uint64_t perturbed_mask(const PtArgs &a, uint32_t it, uint32_t row, uint32_t col) {
    uint64_t m = 0;
    for (uint32_t b = 0; b * 4 < a.cells; ++b) {
        const Block4 r = philox(row, col, it | (b << 8), a.tagword, a.key0, a.key1);
        const uint32_t w[4] = {r.w0, r.w1, r.w2, r.w3};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t c = b * 4 + i;
            if (c < a.cells) {
                const bool present = (a.adj >> c) & 1u;
                const bool on = present ? !((uint64_t)w[i] < a.thr_del) : ((uint64_t)w[i] < a.thr_add);
                m |= (uint64_t)on << c;
            }
        }
    }
    return m;
}

__global__ __launch_bounds__(kPtThreads) void pt_fanout(PtArgs a, uint32_t it, uint64_t count, const uint32_t *row,
                                                        const uint32_t *col, uint32_t *fan) {
    const uint64_t stride = (uint64_t)gridDim.x * kPtThreads;
    for (uint64_t j = (uint64_t)blockIdx.x * kPtThreads + threadIdx.x; j < count; j += stride)
        fan[j] = (uint32_t)__popcll(perturbed_mask(a, it, row[j], col[j]));
}

// Exclusive scan of fan-outs: per-block sums, a single-block scan of those,
// then the blocks again.
__global__ __launch_bounds__(kPtThreads) void pt_scan_sums(const uint32_t *fan, uint64_t count, uint64_t *bsum) {
    __shared__ uint64_t s[kPtThreads];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanBlock;
    uint64_t x = 0;
    for (uint64_t i = b0 + threadIdx.x; i < b0 + kScanBlock && i < count; i += kPtThreads) x += fan[i];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = kPtThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void pt_scan_blocks(uint64_t *bsum, uint64_t nb, uint64_t *total) {
    __shared__ uint64_t s[1024];
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t lo = std::min<uint64_t>((uint64_t)threadIdx.x * per, nb), hi = std::min<uint64_t>(lo + per, nb);
    uint64_t x = 0;
    for (uint64_t i = lo; i < hi; ++i) x += bsum[i];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = s[threadIdx.x] - x;  // exclusive prefix of this thread's range
    for (uint64_t i = lo; i < hi; ++i) {
        const uint64_t v = bsum[i];
        bsum[i] = run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = s[1023];
}

__global__ __launch_bounds__(kPtThreads) void pt_scan_apply(const uint32_t *fan, uint64_t count, const uint64_t *bsum,
                                                            uint64_t *off) {
    __shared__ uint64_t s[kPtThreads];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanBlock;
    const uint64_t t0 = b0 + (uint64_t)threadIdx.x * kScanPer;
    uint64_t x = 0;
    for (int j = 0; j < kScanPer; ++j)
        if (t0 + j < count) x += fan[t0 + j];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < kPtThreads; o <<= 1) {
        const uint64_t y = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = bsum[blockIdx.x] + s[threadIdx.x] - x;
    for (int j = 0; j < kScanPer; ++j)
        if (t0 + j < count) {
            off[t0 + j] = run;
            run += fan[t0 + j];
        }
}

// Children of every meta-edge, in cell order, at its scanned offset.  A
// workgroup takes kPtThreads consecutive meta-edges, whose children form one
// contiguous output range [off[first], end); when that range fits kExpStage
// entries the children are gathered in LDS and the range is written
// coalesced, else every thread writes its own children.  total: the number of
// children of the whole level (the end of the last range).
constexpr int kExpStage = 4096;

template <typename OutT>
__global__ __launch_bounds__(kPtThreads) void pt_expand(PtArgs a, uint32_t it, uint64_t count, const uint32_t *row,
                                                        const uint32_t *col, const uint64_t *off, uint64_t total,
                                                        OutT *nrow, OutT *ncol) {
    __shared__ OutT s_r[kExpStage], s_c[kExpStage];
    const uint64_t stride = (uint64_t)gridDim.x * kPtThreads;
    for (uint64_t base = (uint64_t)blockIdx.x * kPtThreads; base < count; base += stride) {
        const uint64_t j = base + threadIdx.x;
        const uint64_t last = min(base + kPtThreads, count);  // one past the block's meta-edges
        const uint64_t o0 = off[base], o_end = last < count ? off[last] : total;
        const bool stage = o_end - o0 <= (uint64_t)kExpStage;
        if (j < count) {
            const uint32_t r = row[j], c = col[j];
            uint64_t m = perturbed_mask(a, it, r, c);
            uint64_t o = off[j];
            while (m) {
                const uint32_t cell = (uint32_t)__builtin_ctzll(m);
                m &= m - 1;
                const OutT vr = (OutT)((uint64_t)r * a.n0 + cell / a.n0);
                const OutT vc = (OutT)((uint64_t)c * a.n0 + cell % a.n0);
                if (stage) {
                    s_r[o - o0] = vr;
                    s_c[o - o0] = vc;
                } else {
                    nrow[o] = vr;
                    ncol[o] = vc;
                }
                ++o;
            }
        }
        if (stage) {
            __syncthreads();
            for (uint64_t i = threadIdx.x; i < o_end - o0; i += kPtThreads) {
                nrow[o0 + i] = s_r[i];
                ncol[o0 + i] = s_c[i];
            }
            __syncthreads();
        }
    }
}

int grid_of(uint64_t items) {
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((items + kPtThreads - 1) / kPtThreads,
                                                         (uint64_t)device_cu_count() * 16));
}

struct PtPlan {
    size_t off_r0, off_c0, off_r1, off_c1, off_fan, off_off, off_bsum, off_total, total;
};

PtPlan pt_plan(uint64_t capacity) {
    PtPlan p;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += align256(b);
        return r;
    };
    p.off_r0 = take(capacity * 4);
    p.off_c0 = take(capacity * 4);
    p.off_r1 = take(capacity * 4);
    p.off_c1 = take(capacity * 4);
    p.off_fan = take(capacity * 4);
    p.off_off = take(capacity * 8);
    p.off_bsum = take(((capacity + kScanBlock - 1) / kScanBlock + 1) * 8);
    p.off_total = take(8);
    p.total = o;
    return p;
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t kron_perturbed_workspace_bytes(uint64_t capacity) { return pt_plan(std::max<uint64_t>(capacity, 1)).total; }

extern "C" int kron_perturbed(uint32_t n0, const float *seed_matrix, uint32_t k, double p_add, double p_del,
                              uint64_t seed, uint32_t graph_id, int id_bytes, uint64_t capacity, void *src, void *dst,
                              uint64_t *num_edges, void *workspace, size_t workspace_bytes, void *stream) {
    if (n0 < 2 || n0 > 8) return fail(SFG_EINVAL, "kron_perturbed: n0 must be in [2, 8]");
    if (k == 0) return fail(SFG_EINVAL, "kron_perturbed: k must be >= 1");
    if (!seed_matrix) return fail(SFG_EINVAL, "kron_perturbed: NULL seed matrix");
    if (!(p_add >= 0.0 && p_add <= 1.0) || !(p_del >= 0.0 && p_del <= 1.0))
        return fail(SFG_EINVAL, "kron_perturbed: probabilities must be in [0, 1]");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "kron_perturbed: id_bytes must be 4 or 8");
    if (graph_id >= (1u << 24)) return fail(SFG_EINVAL, "kron_perturbed: graph_id must be < 2^24");
    if (k > 255) return fail(SFG_ERANGE, "kron_perturbed: k above 255");
    uint64_t n = 1;
    for (uint32_t l = 0; l < k; ++l) {
        if (n > (1ull << 32) / n0) return fail(SFG_ERANGE, "kron_perturbed: n0^k above 2^32");
        n *= n0;
    }
    if (id_bytes == 4 && n - 1 > 0x7FFFFFFFull) return fail(SFG_ERANGE, "kron_perturbed: ids do not fit int32");
    PtArgs a;
    memset(&a, 0, sizeof(a));
    a.n0 = n0;
    a.cells = n0 * n0;
    uint32_t e0 = 0;
    for (uint32_t c = 0; c < a.cells; ++c) {
        if (!(seed_matrix[c] >= 0.0f) || seed_matrix[c] > 3.0e38f)
            return fail(SFG_EINVAL, "kron_perturbed: bad seed entry %u", c);
        if (seed_matrix[c] != 0.0f) {
            a.adj |= 1ull << c;
            ++e0;
        }
    }
    if (e0 == 0) return fail(SFG_EINVAL, "kron_perturbed: the seed graph has no edge");
    if (!num_edges || (capacity > 0 && (!src || !dst))) return fail(SFG_EINVAL, "kron_perturbed: NULL output");
    const PtPlan P = pt_plan(std::max<uint64_t>(capacity, 1));
    if (!workspace) return fail(SFG_EINVAL, "kron_perturbed: workspace is NULL");
    if (workspace_bytes < P.total)
        return fail(SFG_ENOSPACE, "kron_perturbed: workspace has %zu bytes, needs %zu", workspace_bytes, P.total);
    if (capacity < e0) return fail(SFG_ENOSPACE, "kron_perturbed: capacity below the %u seed edges", e0);
    // floor(p 2^32) in binary64, compared as u64 with a 32-bit word.
    a.thr_add = (uint64_t)(p_add * 4294967296.0);
    a.thr_del = (uint64_t)(p_del * 4294967296.0);
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.tagword = TAG_PERTURB | (graph_id << 8);
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    uint32_t *r0 = reinterpret_cast<uint32_t *>(ws + P.off_r0), *c0 = reinterpret_cast<uint32_t *>(ws + P.off_c0);
    uint32_t *r1 = reinterpret_cast<uint32_t *>(ws + P.off_r1), *c1 = reinterpret_cast<uint32_t *>(ws + P.off_c1);
    uint32_t *fan = reinterpret_cast<uint32_t *>(ws + P.off_fan);
    uint64_t *off = reinterpret_cast<uint64_t *>(ws + P.off_off);
    uint64_t *bsum = reinterpret_cast<uint64_t *>(ws + P.off_bsum);
    uint64_t *total = reinterpret_cast<uint64_t *>(ws + P.off_total);

    // Iteration 1: the seed's own edges, row-major (the stack's order).
    uint32_t hr[64], hc[64];
    uint64_t count = 0;
    for (uint32_t c = 0; c < a.cells; ++c)
        if ((a.adj >> c) & 1u) {
            hr[count] = c / n0;
            hc[count] = c % n0;
            ++count;
        }
    if (hipMemcpyAsync(r0, hr, count * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c0, hc, count * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(SFG_EDEVICE, "kron_perturbed: upload failed");
    // Expansion it -> it + 1 for it = 1 .. k-1; the last one writes the
    // caller's arrays.
    for (uint32_t it = 1; it < k && count > 0; ++it) {
        const int g = grid_of(count);
        { ProfScope _ps("perturb_expand", s); pt_fanout<<<g, kPtThreads, 0, s>>>(a, it, count, r0, c0, fan); }
        const uint64_t nb = (count + kScanBlock - 1) / kScanBlock;
        pt_scan_sums<<<(int)nb, kPtThreads, 0, s>>>(fan, count, bsum);
        pt_scan_blocks<<<1, 1024, 0, s>>>(bsum, nb, total);
        pt_scan_apply<<<(int)nb, kPtThreads, 0, s>>>(fan, count, bsum, off);
        uint64_t next = 0;
        if (hipMemcpyAsync(&next, total, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return fail(SFG_EDEVICE, "kron_perturbed: %s", hipGetErrorString(hipGetLastError()));
        if (next > capacity)
            return fail(SFG_ENOSPACE, "kron_perturbed: iteration %u has %llu edges, capacity is %llu", it + 1,
                        (unsigned long long)next, (unsigned long long)capacity);
        ProfScope _ps("perturb_expand", s);
        if (it + 1 == k) {
            if (id_bytes == 4)
                pt_expand<int32_t><<<g, kPtThreads, 0, s>>>(a, it, count, r0, c0, off, next,
                                                            static_cast<int32_t *>(src), static_cast<int32_t *>(dst));
            else
                pt_expand<int64_t><<<g, kPtThreads, 0, s>>>(a, it, count, r0, c0, off, next,
                                                            static_cast<int64_t *>(src), static_cast<int64_t *>(dst));
        } else {
            pt_expand<uint32_t><<<g, kPtThreads, 0, s>>>(a, it, count, r0, c0, off, next, r1, c1);
            std::swap(r0, r1);
            std::swap(c0, c1);
        }
        count = next;
    }
    if (k == 1) {
        // The seed itself: widen the uploaded level to the id type.
        if (id_bytes == 4) {
            int32_t sr[64], sc[64];
            for (uint64_t i = 0; i < count; ++i) { sr[i] = (int32_t)hr[i]; sc[i] = (int32_t)hc[i]; }
            if (hipMemcpyAsync(src, sr, count * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(dst, sc, count * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(SFG_EDEVICE, "kron_perturbed: upload failed");
        } else {
            int64_t sr[64], sc[64];
            for (uint64_t i = 0; i < count; ++i) { sr[i] = hr[i]; sc[i] = hc[i]; }
            if (hipMemcpyAsync(src, sr, count * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(dst, sc, count * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(SFG_EDEVICE, "kron_perturbed: upload failed");
        }
    }
    if (hipMemcpyAsync(num_edges, &count, 8, hipMemcpyHostToDevice, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(SFG_EDEVICE, "kron_perturbed: %s", hipGetErrorString(hipGetLastError()));
    return check_launch("kron_perturbed");
}
