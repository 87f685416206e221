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
//
// The whole ensemble runs on the caller's stream.  Every batch's tables (the
// Kronecker members, the PBA graph table, the statistics table) are built on
// the host and uploaded in one copy before the first batch, so the batches
// are a sequence of kernel launches with no host round trip; with
// SFG_ENSEMBLE_GRAPH that sequence is captured once into a HIP graph (cached
// per descriptor table, tuning, workspace and outputs) and every later call
// replays it as one graph launch.  The generation and statistics kernels are
// persistent: a grid of grid_per_cu workgroups per CU walks the batch's
// (member, tile) table.
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

// Tile b of the batch (ITEMS x 256 edges) belongs to the member whose block0
// is the last one <= b; workgroups walk the tiles persistently (b = blockIdx.x,
// blockIdx.x + gridDim.x, ...).  The member's parameters are the same for the
// whole tile, so they are moved from LDS into scalar registers: the Philox key
// schedule and the bucket thresholds then cost no vector instructions.
template <typename IdT, int NT, int ITEMS>
__global__ __launch_bounds__(kKronThreads) void kron_batch(const KGraph *G, uint32_t count, uint64_t tiles,
                                                           IdT *__restrict__ src, IdT *__restrict__ dst) {
    __shared__ KGraph s_g;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        if (threadIdx.x == 0) {
            uint32_t lo = 0, hi = count;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) / 2;
                if (G[mid].block0 <= tile)
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
        __syncthreads();  // s_g is rewritten by the next tile
        // Levels 5 blk .. 5 blk + nlev - 1 of edge e from Philox block blk.
        auto levels = [&](uint64_t e, uint32_t blk, uint32_t nlev, uint32_t &u, uint32_t &v) {
            const Block4 r = philox((uint32_t)e, (uint32_t)(e >> 32), blk, tagword, key0, key1);
            const uint32_t ws[5] = {r.w0, r.w1, r.w2, r.w3, level4_word(r)};
#pragma unroll
            for (int i = 0; i < 5; ++i) {
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
        const uint32_t full = k / 5, rest = k % 5;
        const uint64_t e0 = (tile - block0) * (uint64_t)(kKronThreads * ITEMS);
        for (int it = 0; it < ITEMS; ++it) {
            const uint64_t e = e0 + (uint64_t)it * kKronThreads + threadIdx.x;
            if (e >= edges) break;
            uint32_t u = 0, v = 0;  // below n0^k <= 2^32
            for (uint32_t blk = 0; blk < full; ++blk) levels(e, blk, 5, u, v);
            if (rest) levels(e, full, rest, u, v);
            src[ebase + e] = (IdT)(vbase + u);
            dst[ebase + e] = (IdT)(vbase + v);
        }
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

// One batch: its vertex space, edge list and workspace carving.  Tables of
// every batch live in a region of their own at the start of the workspace.
struct BatchPlan {
    uint32_t b0, b1;
    uint64_t nv, E, E_pba, chunks, kron_tiles;
    int id_bytes, nt_max;
    std::vector<PbaGraphSpec> pba;
    std::vector<uint32_t> pba_idx, kron_idx;  // descriptor indices, in batch order
    std::vector<KGraph> kt;
    std::vector<StatGraph> st;
    size_t off_src, off_dst, off_gen, off_rp, off_col, off_hist, off_scratch, total;  // in the batch region
    size_t tab_k, tab_s, tab_p;                                                      // in the table region
};

int plan_batch(const sfg_graph_desc *d, uint32_t b0, uint32_t b1, uint32_t items, BatchPlan &p) {
    p.b0 = b0;
    p.b1 = b1;
    p.nv = p.E = p.E_pba = p.chunks = p.kron_tiles = 0;
    p.nt_max = 0;
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
    const uint64_t tile_edges = (uint64_t)kKronThreads * items;
    for (uint32_t i = b0; i < b1; ++i)
        if (d[i].kind != SFG_GRAPH_PBA) {
            SampleTable tab;
            memset(&tab, 0, sizeof(tab));
            int rc = build_sample_table(d[i].n0, d[i].initiator, tab);
            if (rc != SFG_OK) return rc;
            if (tab.nt > 15) return fail(SFG_EINVAL, "ensemble_generate: initiator with more than 15 thresholds");
            const uint64_t nv = desc_vertices(d[i]);
            KGraph g;
            memset(&g, 0, sizeof(g));
            g.edges = d[i].num_edges;
            g.ebase = p.E;
            g.vbase = p.nv;
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
            g.block0 = p.kron_tiles;
            p.kron_tiles += (g.edges + tile_edges - 1) / tile_edges;
            p.nt_max = std::max(p.nt_max, (int)tab.nt);
            p.kt.push_back(g);
            p.kron_idx.push_back(i);
            p.nv += nv;
            p.E += desc_edges(d[i]);
            p.chunks += stats_chunks_of(nv);
        }
    uint64_t chunk0 = 0, v = 0;
    auto add_stat = [&](uint32_t i) {
        const uint64_t n = desc_vertices(d[i]), E = desc_edges(d[i]);
        p.st.push_back(StatGraph{v, v + n, 2 * ((2 * E + n - 1) / n), chunk0, i, d[i].graph_id});
        v += n;
        chunk0 += stats_chunks_of(n);
    };
    for (uint32_t i : p.pba_idx) add_stat(i);
    for (uint32_t i : p.kron_idx) add_stat(i);
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
    p.off_hist = take(32 * 8);
    p.off_scratch = take(stats_scratch_bytes(p.nv, p.chunks));
    p.total = o;
    return SFG_OK;
}

// Every batch's plan, the table region's layout and the batch region's size.
struct Ensemble {
    std::vector<BatchPlan> batches;
    size_t tables, region;  // bytes of the table region and of the (shared) batch region
};

int plan_ensemble(const sfg_graph_desc *descs, uint32_t count, uint64_t max_batch_edges, uint32_t items,
                  Ensemble &en) {
    const auto cuts = cut_batches(descs, count, std::max<uint64_t>(max_batch_edges, 1));
    en.batches.resize(cuts.size());
    en.tables = en.region = 0;
    for (size_t i = 0; i < cuts.size(); ++i) {
        BatchPlan &p = en.batches[i];
        int rc = plan_batch(descs, cuts[i].first, cuts[i].second, items, p);
        if (rc != SFG_OK) return rc;
        p.tab_k = en.tables;
        en.tables += align256(std::max<size_t>(p.kt.size(), 1) * sizeof(KGraph));
        p.tab_s = en.tables;
        en.tables += align256(p.st.size() * sizeof(StatGraph));
        p.tab_p = en.tables;
        en.tables += pba_tables_bytes(p.pba.data(), (uint32_t)p.pba.size());
        en.region = std::max(en.region, p.total);
    }
    en.tables = align256(en.tables);
    return SFG_OK;
}

void fill_tables(const Ensemble &en, std::vector<char> &blob) {
    blob.assign(en.tables, 0);
    for (const BatchPlan &p : en.batches) {
        if (!p.kt.empty()) memcpy(blob.data() + p.tab_k, p.kt.data(), p.kt.size() * sizeof(KGraph));
        memcpy(blob.data() + p.tab_s, p.st.data(), p.st.size() * sizeof(StatGraph));
        pba_tables_fill(p.pba.data(), (uint32_t)p.pba.size(), blob.data() + p.tab_p);
    }
}

template <typename IdT, int NT>
void launch_kron(int items, unsigned grid, const KGraph *G, uint32_t count, uint64_t tiles, void *src, void *dst,
                 hipStream_t s) {
    IdT *su = static_cast<IdT *>(src), *du = static_cast<IdT *>(dst);
    if (items == 4)
        kron_batch<IdT, NT, 4><<<grid, kKronThreads, 0, s>>>(G, count, tiles, su, du);
    else if (items == 16)
        kron_batch<IdT, NT, 16><<<grid, kKronThreads, 0, s>>>(G, count, tiles, su, du);
    else
        kron_batch<IdT, NT, 8><<<grid, kKronThreads, 0, s>>>(G, count, tiles, su, du);
}

// Kernel launches of one batch (its tables already on the device).
int enqueue_batch(const BatchPlan &P, const sfg_ensemble_tuning &tu, uint32_t samples, uint64_t stat_seed,
                  uint64_t *hist, double *gamma, int64_t *closed, char *tables, char *ws, hipStream_t s) {
    void *src = ws + P.off_src, *dst = ws + P.off_dst;
    const uint64_t cap = (uint64_t)device_cu_count() * tu.grid_per_cu;
    if (!P.pba.empty()) {
        int rc = pba_enqueue_batch(P.pba.data(), (uint32_t)P.pba.size(), P.id_bytes, src, dst, ws + P.off_gen,
                                   P.off_rp - P.off_gen, tables + P.tab_p, s);
        if (rc != SFG_OK) return rc;
    }
    if (!P.kt.empty()) {
        ProfScope _ps("kron_sample", s);
        const KGraph *ktab = reinterpret_cast<const KGraph *>(tables + P.tab_k);
        const uint32_t kc = (uint32_t)P.kt.size();
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(P.kron_tiles, cap));
        const int items = (int)tu.kron_items;
        if (P.id_bytes == 4) {
            if (P.nt_max <= 3)
                launch_kron<int32_t, 3>(items, grid, ktab, kc, P.kron_tiles, src, dst, s);
            else
                launch_kron<int32_t, 15>(items, grid, ktab, kc, P.kron_tiles, src, dst, s);
        } else {
            if (P.nt_max <= 3)
                launch_kron<int64_t, 3>(items, grid, ktab, kc, P.kron_tiles, src, dst, s);
            else
                launch_kron<int64_t, 15>(items, grid, ktab, kc, P.kron_tiles, src, dst, s);
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
    const StatGraph *stab = reinterpret_cast<const StatGraph *>(tables + P.tab_s);
    return stats_enqueue(stab, (uint32_t)P.st.size(), P.chunks, P.nv, raw, rp, col, P.id_bytes, samples, stat_seed,
                         hist, gamma, closed, ws + P.off_scratch, s,
                         (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(P.chunks, cap)));
}

int enqueue_all(const Ensemble &en, const sfg_ensemble_tuning &tu, uint32_t samples, uint64_t stat_seed,
                uint64_t *hist, double *gamma, int64_t *closed, char *ws, hipStream_t s) {
    char *tables = ws;
    char *region = ws + en.tables;
    for (const BatchPlan &p : en.batches) {
        int rc = enqueue_batch(p, tu, samples, stat_seed, hist, gamma, closed, tables, region, s);
        if (rc != SFG_OK) return rc;
    }
    return SFG_OK;
}

// ----------------------------------------------------------------------------- captured graphs
// A captured batch sequence is valid for exactly the arguments it was
// captured with: the descriptor table, samples, seed, tuning, workspace and
// output addresses, and the device.
struct Captured {
    int dev;
    std::vector<char> key;
    hipGraphExec_t exec;
};

std::vector<char> capture_key(const sfg_graph_desc *descs, uint32_t count, uint32_t samples, uint64_t stat_seed,
                              const sfg_ensemble_tuning &tu, const void *ws, size_t bytes, const void *hist,
                              const void *gamma, const void *closed) {
    std::vector<char> k(sizeof(sfg_graph_desc) * count);
    memcpy(k.data(), descs, k.size());
    auto put = [&](const void *p, size_t n) { k.insert(k.end(), (const char *)p, (const char *)p + n); };
    put(&count, sizeof(count));
    put(&samples, sizeof(samples));
    put(&stat_seed, sizeof(stat_seed));
    put(&tu, sizeof(tu));
    put(&ws, sizeof(ws));
    put(&bytes, sizeof(bytes));
    put(&hist, sizeof(hist));
    put(&gamma, sizeof(gamma));
    put(&closed, sizeof(closed));
    return k;
}

constexpr size_t kMaxCaptured = 8;
std::mutex g_cap_mu;
std::vector<Captured> g_captured;  // most recently used last

// The capture stream of the current device (non-blocking, default priority).
hipStream_t capture_stream() {
    static hipStream_t streams[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) return nullptr;
    return streams[dev];
}

// The graph of the batch sequence for these arguments: found in the cache or
// captured now.  Returns nullptr (and leaves the error message) if capture is
// not possible; the caller then enqueues the sequence directly.
hipGraphExec_t captured_graph(const Ensemble &en, const std::vector<char> &key, const sfg_ensemble_tuning &tu,
                              uint32_t samples, uint64_t stat_seed, uint64_t *hist, double *gamma, int64_t *closed,
                              char *ws) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(g_cap_mu);
    for (size_t i = 0; i < g_captured.size(); ++i)
        if (g_captured[i].dev == dev && g_captured[i].key == key) {
            Captured c = g_captured[i];
            g_captured.erase(g_captured.begin() + i);
            g_captured.push_back(c);
            return c.exec;
        }
    hipStream_t cs = capture_stream();
    if (!cs) return nullptr;
    (void)device_error_word();  // looked up outside the capture
    (void)device_cu_count();
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    const int rc = enqueue_all(en, tu, samples, stat_seed, hist, gamma, closed, ws, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc != SFG_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess || !exec) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (g_captured.size() >= kMaxCaptured) {
        (void)hipGraphExecDestroy(g_captured.front().exec);
        g_captured.erase(g_captured.begin());
    }
    g_captured.push_back(Captured{dev, key, exec});
    return exec;
}

int validate(const sfg_graph_desc *descs, uint32_t count) {
    for (uint32_t i = 0; i < count; ++i) {
        int rc = check_desc(descs[i], i);
        if (rc != SFG_OK) return rc;
    }
    return SFG_OK;
}

bool tuning_ok(const sfg_ensemble_tuning &tu) {
    return tu.max_batch_edges >= 1 && tu.grid_per_cu >= 1 && tu.grid_per_cu <= 64 &&
           (tu.kron_items == 4 || tu.kron_items == 8 || tu.kron_items == 16) &&
           (tu.flags & ~(uint32_t)SFG_ENSEMBLE_GRAPH) == 0;
}

sfg_ensemble_tuning default_tuning(uint64_t max_batch_edges) {
    sfg_ensemble_tuning tu;
    tu.max_batch_edges = max_batch_edges;
    tu.grid_per_cu = 8;
    tu.kron_items = 8;
    tu.flags = SFG_ENSEMBLE_GRAPH;
    return tu;
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t ensemble_workspace_bytes(const sfg_graph_desc *descs, uint32_t count, uint64_t max_batch_edges) {
    if (!descs || count == 0 || validate(descs, count) != SFG_OK) return 0;
    Ensemble en;
    // (the tile size changes no buffer size)
    if (plan_ensemble(descs, count, max_batch_edges, 8, en) != SFG_OK) return 0;
    return en.tables + en.region;
}

extern "C" int ensemble_generate_tuned(const sfg_graph_desc *descs, uint32_t count, uint32_t num_samples,
                                       uint64_t stat_seed, const sfg_ensemble_tuning *tuning, uint64_t *degree_hist32,
                                       double *gamma, int64_t *closed, void *workspace, size_t workspace_bytes,
                                       void *stream) {
    if (count == 0) return SFG_OK;
    if (!descs || !tuning) return fail(SFG_EINVAL, "ensemble_generate: descs or tuning is NULL");
    if (!degree_hist32 || !gamma || !closed || !workspace) return fail(SFG_EINVAL, "ensemble_generate: NULL buffer");
    const sfg_ensemble_tuning tu = *tuning;
    if (!tuning_ok(tu)) return fail(SFG_EINVAL, "ensemble_generate: bad tuning");
    int rc = validate(descs, count);
    if (rc != SFG_OK) return rc;
    Ensemble en;
    rc = plan_ensemble(descs, count, tu.max_batch_edges, tu.kron_items, en);
    if (rc != SFG_OK) return rc;
    const size_t need = en.tables + en.region;
    if (workspace_bytes < need)
        return fail(SFG_ENOSPACE, "ensemble_generate: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    if (!device_error_word()) return fail(SFG_EDEVICE, "ensemble_generate: no device");
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    // Every batch's tables in one upload (the host copy dies at return: wait).
    std::vector<char> blob;
    fill_tables(en, blob);
    if (hipMemcpyAsync(ws, blob.data(), blob.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return check_launch("ensemble_generate: table upload");
    if (tu.flags & SFG_ENSEMBLE_GRAPH) {
        const auto key = capture_key(descs, count, num_samples, stat_seed, tu, workspace, workspace_bytes,
                                     degree_hist32, gamma, closed);
        hipGraphExec_t exec = captured_graph(en, key, tu, num_samples, stat_seed, degree_hist32, gamma, closed, ws);
        if (exec) {
            if (hipGraphLaunch(exec, s) != hipSuccess) return check_launch("ensemble_generate: graph launch");
            return SFG_OK;
        }
    }
    rc = enqueue_all(en, tu, num_samples, stat_seed, degree_hist32, gamma, closed, ws, s);
    if (rc != SFG_OK) return rc;
    return check_launch("ensemble_generate");
}

extern "C" int ensemble_generate(const sfg_graph_desc *descs, uint32_t count, uint32_t num_samples,
                                 uint64_t stat_seed, uint64_t max_batch_edges, uint64_t *degree_hist32, double *gamma,
                                 int64_t *closed, void *workspace, size_t workspace_bytes, void *stream) {
    const sfg_ensemble_tuning tu = default_tuning(std::max<uint64_t>(max_batch_edges, 1));
    return ensemble_generate_tuned(descs, count, num_samples, stat_seed, &tu, degree_hist32, gamma, closed, workspace,
                                   workspace_bytes, stream);
}
