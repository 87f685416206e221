// Batched ensemble generation: many PBA and Kronecker graphs of uneven size
// and parameters generated, sorted and summarised together.
//
// A batch shares one vertex space (graph g owns ids [vbase_g, vbase_g + n_g))
// and one edge list: every PBA graph of the batch goes through one pass of
// each batched PBA kernel, every Kronecker graph through one launch of the
// batched sampler below, then a single CSR build sorts the union (its simple
// symmetrized CSR is the block-diagonal union of the members' CSRs) and the
// statistics kernels summarise all members at once.  Each member's edges,
// statistics and random streams are exactly those of the single-graph calls
// with the same graph id; only the launch count changes (about forty launches
// per batch instead of forty per graph).  Batches are cut greedily, in
// descriptor order, at max_batch_edges edges or 2^24 vertices.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "kron.hpp"
#include "pba.hpp"
#include "stats.hpp"

namespace sfg {
namespace {

constexpr int kKronThreads = 256;
constexpr int kKronItems = 8;  // edges per thread per workgroup pass

// One Kronecker member (device table).
struct KGraph {
    uint64_t edges, ebase, vbase;
    uint64_t lut_row, lut_col;
    uint32_t tm1[15];
    uint32_t k, n0, shift, pow2, tagword, key0, key1;
    uint64_t block0;  // first workgroup of this member
};

template <int NT> __device__ __forceinline__ uint32_t bucket_of(uint32_t w, const uint32_t *t) {
    uint32_t b = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i) b += (w > t[i]) ? 1u : 0u;
    return b;
}

__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    return make_u64(uniform32((uint32_t)x), uniform32((uint32_t)(x >> 32)));
}

// Workgroup b samples edges [(b - block0) * chunk, ...) of the member owning b.
// The member's parameters are the same for the whole workgroup, so they are
// moved from LDS into scalar registers: the Philox key schedule and the
// bucket thresholds then cost no vector instructions.
template <typename IdT, int NT>
__global__ __launch_bounds__(kKronThreads) void kron_batch(const KGraph *G, uint32_t count, IdT *__restrict__ src,
                                                           IdT *__restrict__ dst) {
    __shared__ KGraph s_g;
    if (threadIdx.x == 0) {
        uint32_t lo = 0, hi = count;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (G[mid].block0 <= blockIdx.x)
                lo = mid;
            else
                hi = mid;
        }
        s_g = G[lo];
    }
    __syncthreads();
    const uint64_t edges = uniform64(s_g.edges), ebase = uniform64(s_g.ebase), vbase = uniform64(s_g.vbase);
    const uint64_t lut_row = uniform64(s_g.lut_row), lut_col = uniform64(s_g.lut_col);
    const uint64_t block0 = uniform64(s_g.block0);
    uint32_t tm1[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) tm1[i] = uniform32(s_g.tm1[i]);
    const uint32_t k = uniform32(s_g.k), n0 = uniform32(s_g.n0), shift = uniform32(s_g.shift);
    const uint32_t pow2 = uniform32(s_g.pow2), tagword = uniform32(s_g.tagword);
    const uint32_t key0 = uniform32(s_g.key0), key1 = uniform32(s_g.key1);
    // Levels 4 blk .. 4 blk + nlev - 1 of edge e from Philox block blk.
    auto levels = [&](uint64_t e, uint32_t blk, uint32_t nlev, uint32_t &u, uint32_t &v) {
        const Block4 r = philox((uint32_t)e, (uint32_t)(e >> 32), blk, tagword, key0, key1);
        const uint32_t ws[4] = {r.w0, r.w1, r.w2, r.w3};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if ((uint32_t)i < nlev) {
                const uint32_t b = bucket_of<NT>(ws[i], tm1);
                const uint32_t rd = (uint32_t)(lut_row >> (4 * b)) & 15u;
                const uint32_t cd = (uint32_t)(lut_col >> (4 * b)) & 15u;
                if (pow2) {
                    u = (u << shift) | rd;
                    v = (v << shift) | cd;
                } else {
                    u = u * n0 + rd;
                    v = v * n0 + cd;
                }
            }
        }
    };
    const uint32_t full = k / 4, rest = k % 4;
    const uint64_t chunk = (uint64_t)kKronThreads * kKronItems;
    const uint64_t e0 = (blockIdx.x - block0) * chunk;
    for (int it = 0; it < kKronItems; ++it) {
        const uint64_t e = e0 + (uint64_t)it * kKronThreads + threadIdx.x;
        if (e >= edges) break;
        uint32_t u = 0, v = 0;  // below n0^k <= 2^32
        for (uint32_t blk = 0; blk < full; ++blk) levels(e, blk, 4, u, v);
        if (rest) levels(e, full, rest, u, v);
        src[ebase + e] = (IdT)(vbase + u);
        dst[ebase + e] = (IdT)(vbase + v);
    }
}

uint64_t desc_vertices(const sfg_graph_desc &d) {
    if (d.kind == SFG_GRAPH_PBA) return d.n;
    uint64_t nv = 1;
    for (uint32_t i = 0; i < d.k; ++i) nv *= d.n0;
    return nv;
}

uint64_t desc_edges(const sfg_graph_desc &d) { return d.kind == SFG_GRAPH_PBA ? d.n * d.m : d.num_edges; }

int check_desc(const sfg_graph_desc &d, uint32_t i) {
    if (d.kind == SFG_GRAPH_PBA) {
        PbaGraphSpec g{d.n, d.m, d.num_parts, d.p_inter, d.seed, d.graph_id, 0};
        return pba_check_spec(g, 8, "ensemble_generate");
    }
    if (d.kind != SFG_GRAPH_KRON) return fail(SFG_EINVAL, "ensemble_generate: descriptor %u has an unknown kind", i);
    if (d.n0 < 2 || d.n0 > 4) return fail(SFG_EINVAL, "ensemble_generate: descriptor %u: n0 must be in [2, 4]", i);
    if (d.k == 0 || d.k > 31) return fail(SFG_EINVAL, "ensemble_generate: descriptor %u: k must be in [1, 31]", i);
    if (d.graph_id >= (1u << 24)) return fail(SFG_EINVAL, "ensemble_generate: graph_id must be < 2^24");
    uint64_t nv = 1;
    for (uint32_t j = 0; j < d.k; ++j) {
        nv *= d.n0;
        if (nv > (1ull << 32)) return fail(SFG_ERANGE, "ensemble_generate: descriptor %u: n0^k > 2^32", i);
    }
    return SFG_OK;
}

// A batch also closes before its vertex space passes 2^24: the symmetrized
// sort key of a batch is two vertex ids wide, so up to 2^24 vertices it
// fits 48 bits and takes six 8-bit passes; one vertex more costs a seventh
// pass over every entry, more than the per-batch launches it saves.
constexpr uint64_t kBatchVertexCap = 1ull << 24;

// Greedy batches in descriptor order.
std::vector<std::pair<uint32_t, uint32_t>> cut_batches(const sfg_graph_desc *d, uint32_t count, uint64_t max_edges) {
    std::vector<std::pair<uint32_t, uint32_t>> out;
    uint32_t b0 = 0;
    uint64_t acc = 0, vacc = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const uint64_t e = desc_edges(d[i]), nv = desc_vertices(d[i]);
        if (i > b0 && (acc + e > max_edges || vacc + nv > kBatchVertexCap)) {
            out.push_back({b0, i});
            b0 = i;
            acc = vacc = 0;
        }
        acc += e;
        vacc += nv;
    }
    if (count > b0) out.push_back({b0, count});
    return out;
}

struct BatchPlan {
    uint64_t nv, E, E_pba, chunks;
    int id_bytes;
    std::vector<PbaGraphSpec> pba;
    std::vector<uint32_t> pba_idx, kron_idx;  // descriptor indices, in batch order
    size_t off_src, off_dst, off_gen, off_rp, off_col, off_ktab, off_stab, off_hist, off_scratch, total;
};

BatchPlan plan_batch(const sfg_graph_desc *d, uint32_t b0, uint32_t b1) {
    BatchPlan p;
    p.nv = p.E = p.E_pba = p.chunks = 0;
    // Vertex space and edge order: PBA members first, then Kronecker members.
    for (uint32_t i = b0; i < b1; ++i)
        if (d[i].kind == SFG_GRAPH_PBA) {
            p.pba.push_back(PbaGraphSpec{d[i].n, d[i].m, d[i].num_parts, d[i].p_inter, d[i].seed, d[i].graph_id, p.nv});
            p.pba_idx.push_back(i);
            p.nv += d[i].n;
            p.E += desc_edges(d[i]);
            p.chunks += stats_chunks_of(d[i].n);
        }
    p.E_pba = p.E;
    for (uint32_t i = b0; i < b1; ++i)
        if (d[i].kind != SFG_GRAPH_PBA) {
            p.kron_idx.push_back(i);
            const uint64_t nv = desc_vertices(d[i]);
            p.nv += nv;
            p.E += desc_edges(d[i]);
            p.chunks += stats_chunks_of(nv);
        }
    p.id_bytes = p.nv <= (1ull << 31) ? 4 : 8;
    const size_t gen = std::max(p.pba.empty() ? 0 : pba_batch_workspace_bytes(p.pba.data(), (uint32_t)p.pba.size()),
                                csr_workspace_bytes(std::max<uint64_t>(p.nv, 1), p.E, p.id_bytes,
                                                    SFG_CSR_SYMMETRIZE | SFG_CSR_SIMPLE));
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += align256(b);
        return r;
    };
    p.off_src = take(std::max<uint64_t>(p.E, 1) * p.id_bytes);
    p.off_dst = take(std::max<uint64_t>(p.E, 1) * p.id_bytes);
    p.off_gen = take(gen);  // PBA scratch, then reused by the CSR build
    p.off_rp = take((p.nv + 1) * 8);
    p.off_col = take(std::max<uint64_t>(2 * p.E, 1) * p.id_bytes);
    p.off_ktab = take(std::max<size_t>(p.kron_idx.size(), 1) * sizeof(KGraph));
    p.off_stab = take((b1 - b0) * sizeof(StatGraph));
    p.off_hist = take(32 * 8);
    p.off_scratch = take(stats_scratch_bytes(p.nv, p.chunks));
    p.total = o;
    return p;
}

int run_batch(const sfg_graph_desc *d, uint32_t b0, uint32_t b1, uint32_t samples, uint64_t stat_seed, uint64_t *hist,
              double *gamma, int64_t *closed, char *ws, size_t bytes, hipStream_t s) {
    BatchPlan P = plan_batch(d, b0, b1);
    if (bytes < P.total)
        return fail(SFG_ENOSPACE, "ensemble_generate: a batch needs %zu workspace bytes, %zu given", P.total, bytes);
    void *src = ws + P.off_src, *dst = ws + P.off_dst;
    // Tables (uploaded, then the host copies may die after the sync below).
    std::vector<KGraph> kt;
    uint64_t ebase = P.E_pba, vbase = 0, blocks = 0;
    for (const auto &g : P.pba) vbase += g.n;
    int nt_max = 0;
    for (uint32_t i : P.kron_idx) {
        SampleTable tab;
        memset(&tab, 0, sizeof(tab));
        int rc = build_sample_table(d[i].n0, d[i].initiator, tab);
        if (rc != SFG_OK) return rc;
        if (tab.nt > 15) return fail(SFG_EINVAL, "ensemble_generate: initiator with more than 15 thresholds");
        KGraph g;
        memset(&g, 0, sizeof(g));
        g.edges = d[i].num_edges;
        g.ebase = ebase;
        g.vbase = vbase;
        for (int j = 0; j < 15; ++j) g.tm1[j] = (uint32_t)j < tab.nt ? tab.tm1[j] : 0xFFFFFFFFu;
        for (uint32_t b = 0; b <= tab.nt; ++b) {
            g.lut_row |= (uint64_t)tab.row[b] << (4 * b);
            g.lut_col |= (uint64_t)tab.col[b] << (4 * b);
        }
        g.k = d[i].k;
        g.n0 = d[i].n0;
        g.pow2 = (d[i].n0 & (d[i].n0 - 1)) == 0;
        while ((1u << g.shift) < g.n0) ++g.shift;
        g.tagword = TAG_KRON | (d[i].graph_id << 8);
        g.key0 = (uint32_t)d[i].seed;
        g.key1 = (uint32_t)(d[i].seed >> 32);
        g.block0 = blocks;
        blocks += (g.edges + (uint64_t)kKronThreads * kKronItems - 1) / ((uint64_t)kKronThreads * kKronItems);
        nt_max = std::max(nt_max, (int)tab.nt);
        kt.push_back(g);
        ebase += g.edges;
        vbase += desc_vertices(d[i]);
    }
    std::vector<StatGraph> st;
    uint64_t chunk0 = 0, v = 0;
    auto add_stat = [&](uint32_t i) {
        const uint64_t n = desc_vertices(d[i]), E = desc_edges(d[i]);
        st.push_back(StatGraph{v, v + n, 2 * ((2 * E + n - 1) / n), chunk0, i, d[i].graph_id});
        v += n;
        chunk0 += stats_chunks_of(n);
    };
    for (uint32_t i : P.pba_idx) add_stat(i);
    for (uint32_t i : P.kron_idx) add_stat(i);
    KGraph *ktab = reinterpret_cast<KGraph *>(ws + P.off_ktab);
    StatGraph *stab = reinterpret_cast<StatGraph *>(ws + P.off_stab);
    if ((!kt.empty() && hipMemcpyAsync(ktab, kt.data(), kt.size() * sizeof(KGraph), hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(stab, st.data(), st.size() * sizeof(StatGraph), hipMemcpyHostToDevice, s) != hipSuccess)
        return check_launch("ensemble_generate: table upload");
    if (hipStreamSynchronize(s) != hipSuccess) return check_launch("ensemble_generate: table upload");

    // Generation.
    if (!P.pba.empty()) {
        int rc = pba_run_batch(P.pba.data(), (uint32_t)P.pba.size(), nullptr, nullptr, P.id_bytes, src, dst,
                               ws + P.off_gen, P.off_rp - P.off_gen, s);
        if (rc != SFG_OK) return rc;
    }
    if (!kt.empty()) {
        ProfScope _ps("kron_sample", s);
        const uint32_t kc = (uint32_t)kt.size();
        if (P.id_bytes == 4) {
            if (nt_max <= 3)
                kron_batch<int32_t, 3><<<(unsigned)blocks, kKronThreads, 0, s>>>(ktab, kc, (int32_t *)src, (int32_t *)dst);
            else
                kron_batch<int32_t, 15><<<(unsigned)blocks, kKronThreads, 0, s>>>(ktab, kc, (int32_t *)src, (int32_t *)dst);
        } else {
            if (nt_max <= 3)
                kron_batch<int64_t, 3><<<(unsigned)blocks, kKronThreads, 0, s>>>(ktab, kc, (int64_t *)src, (int64_t *)dst);
            else
                kron_batch<int64_t, 15><<<(unsigned)blocks, kKronThreads, 0, s>>>(ktab, kc, (int64_t *)src, (int64_t *)dst);
        }
    }
    // One CSR of the union; its histogram output is scratch (per-member
    // histograms come from the statistics pass).
    uint64_t *rp = reinterpret_cast<uint64_t *>(ws + P.off_rp);
    void *col = ws + P.off_col;
    const uint64_t *raw = nullptr;
    int rc = csr_build(std::max<uint64_t>(P.nv, 1), P.E, src, dst, P.id_bytes, SFG_CSR_SYMMETRIZE | SFG_CSR_SIMPLE, rp,
                       col, reinterpret_cast<uint64_t *>(ws + P.off_hist), nullptr, ws + P.off_gen,
                       P.off_rp - P.off_gen, s, &raw);
    if (rc != SFG_OK) return rc;
    return stats_enqueue(stab, (uint32_t)st.size(), P.chunks, P.nv, raw, rp, col, P.id_bytes, samples, stat_seed, hist,
                         gamma, closed, ws + P.off_scratch, s);
}

// Two library streams per device (default priority) on which consecutive
// batches alternate, each with its own half of the workspace: one batch's
// generation (VALU- and latency-bound) overlaps the other's sort
// (bandwidth-bound).  Results do not depend on the interleaving.
constexpr int kLanes = 2;
constexpr int kMaxDevs = 16;

bool lane_streams(hipStream_t out[kLanes]) {
    static std::mutex mu;
    static hipStream_t lanes[kMaxDevs][kLanes];
    static bool made[kMaxDevs];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevs) return false;
    std::lock_guard<std::mutex> lock(mu);
    if (!made[dev]) {
        for (int l = 0; l < kLanes; ++l)
            if (hipStreamCreateWithFlags(&lanes[dev][l], hipStreamNonBlocking) != hipSuccess) return false;
        made[dev] = true;
    }
    for (int l = 0; l < kLanes; ++l) out[l] = lanes[dev][l];
    return true;
}

size_t batch_need(const sfg_graph_desc *descs, const std::vector<std::pair<uint32_t, uint32_t>> &batches) {
    size_t need = 0;
    for (auto b : batches) need = std::max(need, plan_batch(descs, b.first, b.second).total);
    return align256(need);
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t ensemble_workspace_bytes(const sfg_graph_desc *descs, uint32_t count, uint64_t max_batch_edges) {
    if (!descs || count == 0) return 0;
    const auto batches = cut_batches(descs, count, std::max<uint64_t>(max_batch_edges, 1));
    // One workspace half per lane (a single batch needs one).
    return batch_need(descs, batches) * (batches.size() > 1 ? kLanes : 1);
}

extern "C" int ensemble_generate(const sfg_graph_desc *descs, uint32_t count, uint32_t num_samples,
                                 uint64_t stat_seed, uint64_t max_batch_edges, uint64_t *degree_hist32, double *gamma,
                                 int64_t *closed, void *workspace, size_t workspace_bytes, void *stream) {
    if (count == 0) return SFG_OK;
    if (!descs) return fail(SFG_EINVAL, "ensemble_generate: descs is NULL");
    if (!degree_hist32 || !gamma || !closed || !workspace) return fail(SFG_EINVAL, "ensemble_generate: NULL buffer");
    for (uint32_t i = 0; i < count; ++i) {
        int rc = check_desc(descs[i], i);
        if (rc != SFG_OK) return rc;
        if (descs[i].kind == SFG_GRAPH_KRON) {
            SampleTable tab;
            memset(&tab, 0, sizeof(tab));
            rc = build_sample_table(descs[i].n0, descs[i].initiator, tab);
            if (rc != SFG_OK) return rc;
        }
    }
    const auto batches = cut_batches(descs, count, std::max<uint64_t>(max_batch_edges, 1));
    const size_t need = batch_need(descs, batches);
    if (workspace_bytes < need)
        return fail(SFG_ENOSPACE, "ensemble_generate: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    // With room for two halves, batches alternate between the two lanes;
    // otherwise they run one after another on the caller's stream.
    hipStream_t lanes[kLanes];
    if (batches.size() < 2 || workspace_bytes < kLanes * need || !lane_streams(lanes)) {
        for (auto b : batches) {
            int rc = run_batch(descs, b.first, b.second, num_samples, stat_seed, degree_hist32, gamma, closed, ws,
                               workspace_bytes, s);
            if (rc != SFG_OK) return rc;
        }
        return SFG_OK;
    }
    // Lanes start after the work already on the caller's stream; the caller's
    // stream continues after both lanes.
    hipEvent_t start, done[kLanes];
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess)
        return fail(SFG_EDEVICE, "ensemble_generate: event creation failed");
    int created = 0;
    for (; created < kLanes; ++created)
        if (hipEventCreateWithFlags(&done[created], hipEventDisableTiming) != hipSuccess) break;
    int rc = created == kLanes ? SFG_OK : fail(SFG_EDEVICE, "ensemble_generate: event creation failed");
    if (rc == SFG_OK && hipEventRecord(start, s) != hipSuccess) rc = fail(SFG_EDEVICE, "ensemble_generate: event record failed");
    for (int l = 0; rc == SFG_OK && l < kLanes; ++l)
        if (hipStreamWaitEvent(lanes[l], start, 0) != hipSuccess) rc = fail(SFG_EDEVICE, "ensemble_generate: stream wait failed");
    for (size_t i = 0; rc == SFG_OK && i < batches.size(); ++i) {
        const int l = (int)(i % kLanes);
        rc = run_batch(descs, batches[i].first, batches[i].second, num_samples, stat_seed, degree_hist32, gamma,
                       closed, ws + l * need, need, lanes[l]);
    }
    // Join the lanes into the caller's stream, also after an error, so that
    // no lane still runs once the caller reuses the workspace.
    for (int l = 0; l < created; ++l) {
        if (hipEventRecord(done[l], lanes[l]) != hipSuccess || hipStreamWaitEvent(s, done[l], 0) != hipSuccess) {
            (void)hipStreamSynchronize(lanes[l]);
            if (rc == SFG_OK) rc = fail(SFG_EDEVICE, "ensemble_generate: joining the lanes failed");
        }
    }
    if (rc != SFG_OK)
        for (int l = 0; l < kLanes; ++l) (void)hipStreamSynchronize(lanes[l]);
    (void)hipEventDestroy(start);
    for (int l = 0; l < created; ++l) (void)hipEventDestroy(done[l]);
    return rc;
}
