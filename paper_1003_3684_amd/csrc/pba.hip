// Parallel Barabasi-Albert generation (section "Parallel Barabasi-Albert (PBA)
// method", Fig. 1) on one GPU.
//
// The paper's processors become partitions of contiguous vertex blocks, and
// its two message exchanges become on-device passes:
//   draw1     phase 1: every slot j >= s of partition q is either terminal (a
//             faction partition for j < s, or an inter-faction partition) or
//             a pointer to a uniformly chosen earlier slot of q;
//   resolve   the copy chains are followed to their terminal label;
//   count     per-tile label histograms (the count messages c[q][l]);
//   scan      column prefix sums over (partition, tile) rows give, for every
//             tile and label, the position of its first request in the
//             label's selection list, plus D_l and the list bases;
//   draw2     phase 2: selection t of partition l is terminal (a seed-clique
//             vertex or an arrival vertex) or a pointer to an earlier
//             selection;
//   resolve   the same chain resolution over the selection lists;
//   subst     every slot takes the next endpoint of its label's list, in
//             slot order (a stable in-tile rank), and the edge list is
//             written.
//
// Chains are resolved in memory: a workgroup follows pointers to their
// terminal and writes the terminal back.  Partitions are bound to XCDs
// (workgroup b runs on XCD b mod 8) and every XCD walks its partitions tile
// by tile in slot order, so most pointers land in the already resolved,
// L2-resident prefix of the partition and a chain costs about one load.
// Output depends only on the draws, not on this schedule.
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"

namespace sfg {
namespace {

constexpr uint32_t kTerm = 0x80000000u;  // terminal flag of an encoded slot
constexpr int kXcd = 8;
constexpr int kDrawThreads = 256;
constexpr int kResThreads = 256;
constexpr int kResItems = 4;
constexpr int kResTile = kResThreads * kResItems;  // slots per resolve tile
constexpr int kSubThreads = 256;
constexpr uint32_t kMaxParts = 4096;

// Partition boundaries floor(q n / P), evaluated without 128-bit products.
__host__ __device__ __forceinline__ uint64_t part_start(uint64_t q, uint64_t n, uint64_t P) {
    const uint64_t qd = n / P, r = n % P;
    return q * qd + (q * r) / P;
}

struct Factions {
    // Ordered faction lists F(q) = fmem[foff[q] .. foff[q+1]) and the sorted
    // distinct members U(q) = umem[uoff[q] .. uoff[q+1]); null for F(q) = [q].
    const uint32_t *foff, *fmem, *uoff, *umem;
};

// The r-th partition (ascending) that is not in the sorted set U.
__device__ __forceinline__ uint32_t nonfaction(uint32_t r, const uint32_t *U, uint32_t u) {
    uint32_t x = r;
    for (uint32_t i = 0; i < u; ++i) {
        if (U[i] <= x)
            ++x;
        else
            break;
    }
    return x;
}

// ----------------------------------------------------------------------------- phase 1 draw
struct Draw1Args {
    uint64_t n, P;
    uint32_t m;
    uint32_t key0, key1, tagword;
    uint64_t thr_p;  // inter-faction threshold in [0, 2^32]
    Factions f;
    uint32_t *lab;
};

__global__ __launch_bounds__(kDrawThreads) void pba_draw1(Draw1Args a) {
    const uint32_t q = blockIdx.y;
    const uint64_t s0 = part_start(q, a.n, a.P), s1 = part_start(q + 1, a.n, a.P);
    const uint64_t nslots = (s1 - s0) * a.m;
    uint32_t s = 1, u = 1, self = q;
    const uint32_t *F = &self, *U = &self;
    if (a.f.foff) {
        F = a.f.fmem + a.f.foff[q];
        s = a.f.foff[q + 1] - a.f.foff[q];
        U = a.f.umem + a.f.uoff[q];
        u = a.f.uoff[q + 1] - a.f.uoff[q];
    }
    const uint32_t nnf = (uint32_t)a.P - u;
    const uint64_t stride = (uint64_t)gridDim.x * kDrawThreads;
    for (uint64_t j = (uint64_t)blockIdx.x * kDrawThreads + threadIdx.x; j < nslots; j += stride) {
        uint32_t enc;
        if (j < s) {
            enc = kTerm | F[j];
        } else {
            const Block4 w = philox((uint32_t)j, (uint32_t)(j >> 32), q, a.tagword, a.key0, a.key1);
            const uint64_t U64 = make_u64(w.w1, w.w2);
            if (nnf > 0 && (uint64_t)w.w0 < a.thr_p)
                enc = kTerm | nonfaction((uint32_t)uidx64(U64, nnf), U, u);
            else
                enc = (uint32_t)uidx64(U64, j);  // copy an earlier slot
        }
        a.lab[s0 * a.m + j] = enc;
    }
}

// ----------------------------------------------------------------------------- phase 2 draw
struct Draw2Args {
    uint64_t n, P, total;
    uint32_t key0, key1, tagword;
    const uint64_t *sbase;  // [P+1] list bases (prefix of D)
    uint32_t *sel;
};

__device__ __forceinline__ void pba_draw2_one(const Draw2Args &a, uint64_t g) {
    // partition l with sbase[l] <= g < sbase[l+1]
    uint32_t lo = 0, hi = (uint32_t)a.P;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (a.sbase[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const uint32_t l = lo;
    const uint64_t t = g - a.sbase[l];
    const uint64_t D = a.sbase[l + 1] - a.sbase[l];
    const uint64_t L = part_start(l + 1, a.n, a.P) - part_start(l, a.n, a.P);
    const Block4 w = philox((uint32_t)t, (uint32_t)(t >> 32), l, a.tagword, a.key0, a.key1);
    // Pool entry r of the first 2 + 2t: the seed clique (0, 1), an arrival
    // vertex floor(t' L / D) at even r, or the endpoint of selection t' at odd r.
    const uint64_t r = uidx64(make_u64(w.w0, w.w1), 2 + 2 * t);
    uint32_t enc;
    if (r < 2) {
        enc = kTerm | (uint32_t)r;
    } else if ((r & 1) == 0) {
        const uint64_t tp = (r - 2) >> 1;
        enc = kTerm | (uint32_t)((tp * L) / D);
    } else {
        enc = (uint32_t)((r - 3) >> 1);
    }
    a.sel[g] = enc;
}

__global__ __launch_bounds__(kDrawThreads) void pba_draw2(Draw2Args a) {
    const uint64_t stride = (uint64_t)gridDim.x * kDrawThreads;
    for (uint64_t g = (uint64_t)blockIdx.x * kDrawThreads + threadIdx.x; g < a.total; g += stride)
        pba_draw2_one(a, g);
}

// ----------------------------------------------------------------------------- chain resolution
// Segment q spans enc[base[q] .. base[q+1]); pointers are segment-local.
// Tiles of segment q are queued on XCD q mod 8, segment by segment, in order.
struct ResolveArgs {
    uint32_t *enc;
    const uint64_t *base;     // [P+1]
    const uint64_t *xprefix;  // [8][xstride] tile prefix per XCD queue
    const uint64_t *xtotal;   // [8]
    uint32_t *queues;         // [8] tile tickets
    uint32_t *err;
    uint32_t P, xstride;
};

__global__ __launch_bounds__(kResThreads) void pba_resolve(ResolveArgs a) {
    __shared__ uint64_t s_tile;
    __shared__ uint32_t s_seg;
    const int tid = threadIdx.x;
    const uint32_t home = blockIdx.x % kXcd;
    for (uint32_t att = 0; att < kXcd; ++att) {
        const uint32_t x = (home + att) % kXcd;
        const uint64_t total = a.xtotal[x];
        const uint64_t *pre = a.xprefix + (uint64_t)x * a.xstride;
        const uint32_t nseg = (a.P > x) ? (a.P - x + kXcd - 1) / kXcd : 0;
        for (;;) {
            if (tid == 0) {
                const uint64_t t = fetch_add_agent(&a.queues[x], 1u);
                s_tile = t;
                if (t < total) {
                    // last segment index i with pre[i] <= t
                    uint32_t lo = 0, hi = nseg;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) / 2;
                        if (pre[mid] <= t)
                            lo = mid;
                        else
                            hi = mid;
                    }
                    s_seg = lo;
                }
            }
            __syncthreads();
            const uint64_t t = s_tile;
            const uint32_t i = s_seg;
            __syncthreads();
            if (t >= total) break;
            const uint32_t q = x + kXcd * i;
            const uint64_t b0 = a.base[q];
            const uint64_t len = a.base[q + 1] - b0;
            const uint64_t first = (t - pre[i]) * kResTile;
            uint32_t *seg = a.enc + b0;
#pragma unroll
            for (int k = 0; k < kResItems; ++k) {
                const uint64_t j = first + (uint64_t)k * kResThreads + tid;
                if (j < len) {
                    uint32_t v = seg[j];
                    if (!(v & kTerm)) {
                        // Every hop goes to a strictly earlier slot; a value that
                        // does not is corrupt and ends the walk.
                        uint64_t cur = j;
                        while (!(v & kTerm)) {
                            if ((uint64_t)v >= cur) {
                                raise_device_error(a.err, DEVERR_CHAIN);
                                v = kTerm;
                                break;
                            }
                            cur = v;
                            v = seg[v];
                        }
                        seg[j] = v;
                    }
                }
            }
        }
    }
}

// Per-XCD queues of resolve tiles: prefix of tile counts over the segments
// q = x, x+8, ... of each XCD x.
__global__ void pba_tile_table(const uint64_t *base, uint32_t P, uint32_t xstride, uint64_t *xprefix,
                               uint64_t *xtotal, uint32_t *queues) {
    const uint32_t x = threadIdx.x;
    if (x >= kXcd) return;
    uint64_t acc = 0;
    uint32_t i = 0;
    for (uint32_t q = x; q < P; q += kXcd, ++i) {
        xprefix[(uint64_t)x * xstride + i] = acc;
        acc += (base[q + 1] - base[q] + kResTile - 1) / kResTile;
    }
    xprefix[(uint64_t)x * xstride + i] = acc;
    xtotal[x] = acc;
    queues[x] = 0;
}

__global__ void pba_phase1_bases(uint64_t n, uint64_t P, uint32_t m, uint64_t *base) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q <= P) base[q] = part_start(q, n, P) * m;
}

// ----------------------------------------------------------------------------- counting
// Tile (q, tau) covers slots [tau * CT, (tau+1) * CT) of partition q; its
// label histogram is row (q * T1 + tau) of H (P columns).
struct CountArgs {
    const uint32_t *lab;
    const uint64_t *base1;  // phase-1 bases [P+1]
    uint32_t *H;
    uint32_t P, T1, CT;
};

__global__ __launch_bounds__(256) void pba_count(CountArgs a) {
    extern __shared__ uint32_t s_h[];  // [P]
    const uint32_t q = blockIdx.y, tau = blockIdx.x;
    for (uint32_t l = threadIdx.x; l < a.P; l += 256) s_h[l] = 0;
    __syncthreads();
    const uint64_t b0 = a.base1[q], len = a.base1[q + 1] - b0;
    const uint64_t first = (uint64_t)tau * a.CT;
    const uint64_t last = std::min<uint64_t>(len, first + a.CT);
    for (uint64_t j = first + threadIdx.x; j < last; j += 256) atomicAdd(&s_h[a.lab[b0 + j] & ~kTerm], 1u);
    __syncthreads();
    uint32_t *row = a.H + ((uint64_t)q * a.T1 + tau) * a.P;
    for (uint32_t l = threadIdx.x; l < a.P; l += 256) row[l] = s_h[l];
}

// Column-wise exclusive scan of H (R rows x P columns) in three steps over
// groups of kScanRows rows.
constexpr int kScanRows = 256;

__global__ __launch_bounds__(256) void pba_scan_partial(const uint32_t *H, uint64_t R, uint32_t P, uint32_t *part) {
    const uint32_t col = blockIdx.y * 256 + threadIdx.x;
    if (col >= P) return;
    const uint64_t r0 = (uint64_t)blockIdx.x * kScanRows;
    const uint64_t r1 = std::min<uint64_t>(R, r0 + kScanRows);
    uint32_t acc = 0;
    for (uint64_t r = r0; r < r1; ++r) acc += H[r * P + col];
    part[(uint64_t)blockIdx.x * P + col] = acc;
}

__global__ __launch_bounds__(256) void pba_scan_groups(uint32_t *part, uint64_t groups, uint32_t P, uint64_t *D,
                                                       uint32_t *err) {
    const uint32_t col = blockIdx.x * 256 + threadIdx.x;
    if (col >= P) return;
    uint64_t acc = 0;
    for (uint64_t g = 0; g < groups; ++g) {
        const uint32_t c = part[g * P + col];
        part[g * P + col] = (uint32_t)acc;
        acc += c;
    }
    D[col] = acc;
    if (acc >= kTerm) raise_device_error(err, DEVERR_QUEUE);  // a list longer than 2^31 is unsupported
}

__global__ __launch_bounds__(256) void pba_scan_apply(uint32_t *H, uint64_t R, uint32_t P, const uint32_t *part) {
    const uint32_t col = blockIdx.y * 256 + threadIdx.x;
    if (col >= P) return;
    const uint64_t r0 = (uint64_t)blockIdx.x * kScanRows;
    const uint64_t r1 = std::min<uint64_t>(R, r0 + kScanRows);
    uint32_t acc = part[(uint64_t)blockIdx.x * P + col];
    for (uint64_t r = r0; r < r1; ++r) {
        const uint32_t c = H[r * P + col];
        H[r * P + col] = acc;
        acc += c;
    }
}

// List bases: sbase = exclusive prefix of D (single block).
__global__ __launch_bounds__(1024) void pba_list_bases(const uint64_t *D, uint32_t P, uint64_t *sbase) {
    __shared__ uint64_t s[1024];
    const uint32_t per = (P + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = std::min<uint32_t>(P, lo + per);
    uint64_t acc = 0;
    for (uint32_t i = lo; i < hi; ++i) acc += D[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t o = threadIdx.x >= (uint32_t)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += o;
        __syncthreads();
    }
    uint64_t run = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
    for (uint32_t i = lo; i < hi; ++i) {
        sbase[i] = run;
        run += D[i];
    }
    if (threadIdx.x == 1023) sbase[P] = s[1023];
}

// ----------------------------------------------------------------------------- substitution
// Tile (q, tau) of CT slots: 4 waves each walk a contiguous quarter in slot
// order.  The k-th occurrence of label l in the tile takes endpoint
// H[q,tau][l] + k of l's list (H holds the exclusive column prefix).
struct SubArgs {
    uint64_t n, P;
    uint32_t m, T1, CT, lbits;
    const uint32_t *lab;
    const uint64_t *base1;
    const uint32_t *H;
    const uint64_t *sbase;
    const uint32_t *sel;
    void *src, *dst;
};

__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

template <typename IdT> __global__ __launch_bounds__(kSubThreads) void pba_substitute(SubArgs a) {
    extern __shared__ uint32_t s_cnt[];  // [4][P]
    const uint32_t q = blockIdx.y, tau = blockIdx.x;
    const int tid = threadIdx.x, w = tid >> 6;
    const uint32_t lane = tid & 63;
    const uint32_t P = (uint32_t)a.P;
    for (uint32_t i = tid; i < 4 * P; i += kSubThreads) s_cnt[i] = 0;
    __syncthreads();
    const uint64_t b0 = a.base1[q], len = a.base1[q + 1] - b0;
    const uint64_t first = (uint64_t)tau * a.CT;
    const uint64_t last = std::min<uint64_t>(len, first + a.CT);
    const uint32_t quarter = a.CT / 4;
    const uint64_t wfirst = first + (uint64_t)w * quarter;
    const uint64_t wlast = std::min<uint64_t>(last, wfirst + quarter);
    uint32_t *cnt = s_cnt + (uint64_t)w * P;
    // Pass 1: per-wave label counts.
    for (uint64_t j = wfirst + lane; j < wlast; j += 64) atomicAdd(&cnt[a.lab[b0 + j] & ~kTerm], 1u);
    __syncthreads();
    // Per label: start of each wave's run inside the tile's share of the list.
    const uint32_t *hrow = a.H + ((uint64_t)q * a.T1 + tau) * P;
    for (uint32_t l = tid; l < P; l += kSubThreads) {
        uint32_t acc = hrow[l];
        for (int wv = 0; wv < 4; ++wv) {
            const uint32_t c = s_cnt[wv * P + l];
            s_cnt[wv * P + l] = acc;
            acc += c;
        }
    }
    __syncthreads();
    // Pass 2: slots in order; equal labels in a 64-slot step are ranked by lane.
    const uint64_t vstart = part_start(q, a.n, a.P);
    IdT *src = static_cast<IdT *>(a.src), *dst = static_cast<IdT *>(a.dst);
    for (uint64_t j0 = wfirst; j0 < wlast; j0 += 64) {
        const uint64_t j = j0 + lane;
        const bool valid = j < wlast;
        const uint32_t l = valid ? (a.lab[b0 + j] & ~kTerm) : 0;
        uint64_t peers = __ballot(valid);
        for (uint32_t b = 0; b < a.lbits; ++b) {
            const bool bit = (l >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        if (valid) {
            const uint32_t below = count_below(peers);
            const uint32_t k = cnt[l];
            if (below == 0) cnt[l] = k + (uint32_t)__popcll(peers);
            const uint64_t idx = a.sbase[l] + k + below;
            const uint64_t y = a.sel[idx] & ~kTerm;
            const uint64_t e = b0 + j;
            src[e] = (IdT)(vstart + j / a.m);
            dst[e] = (IdT)(part_start(l, a.n, a.P) + y);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ----------------------------------------------------------------------------- host
struct Plan {
    uint64_t n, E, P, Lmax;
    uint32_t m, T1, CT, xstride;
    uint64_t R, groups;
    size_t off_lab, off_sel, off_H, off_part, off_base1, off_sbase, off_D, off_xpre, off_xtot, off_queues,
        off_foff, off_fmem, off_uoff, off_umem, total;
};

uint32_t choose_ct(uint64_t P) {
    // Tiles of the count/substitution passes: large enough that the P x P
    // histogram rows stay a small fraction of the slot arrays.
    uint32_t ct = 4096;
    while (ct < 65536 && (uint64_t)ct < 16 * P) ct *= 2;
    return ct;
}

Plan make_plan(uint64_t n, uint32_t m, uint32_t P, uint64_t fmem_count) {
    Plan p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.m = m;
    p.P = P;
    p.E = n * m;
    p.Lmax = (n + P - 1) / P;
    p.CT = choose_ct(P);
    p.T1 = (uint32_t)((p.Lmax * m + p.CT - 1) / p.CT);
    p.R = (uint64_t)P * p.T1;
    p.groups = (p.R + kScanRows - 1) / kScanRows;
    p.xstride = (P + kXcd - 1) / kXcd + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align256(bytes);
        return r;
    };
    p.off_lab = take(p.E * 4);
    p.off_sel = take(p.E * 4);
    p.off_H = take(p.R * P * 4);
    p.off_part = take(p.groups * P * 4);
    p.off_base1 = take((P + 1) * 8);
    p.off_sbase = take((P + 1) * 8);
    p.off_D = take(P * 8);
    p.off_xpre = take((size_t)kXcd * p.xstride * 8);
    p.off_xtot = take(kXcd * 8);
    p.off_queues = take(2 * kXcd * 4);
    p.off_foff = take((P + 1) * 4);
    p.off_fmem = take(std::max<uint64_t>(fmem_count, 1) * 4);
    p.off_uoff = take((P + 1) * 4);
    p.off_umem = take(std::max<uint64_t>(fmem_count, 1) * 4);
    p.total = o;
    return p;
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t pba_workspace_bytes(uint64_t n, uint32_t m, uint32_t num_parts, uint64_t num_faction_members) {
    if (num_parts == 0 || m == 0 || n == 0) return 0;
    return make_plan(n, m, num_parts, num_faction_members).total;
}

extern "C" int pba_generate(uint64_t n, uint32_t m, uint32_t num_parts, double p_inter, const uint32_t *faction_off,
                            const uint32_t *faction_members, uint64_t seed, uint32_t graph_id, int id_bytes, void *src,
                            void *dst, void *workspace, size_t workspace_bytes, void *stream) {
    const uint32_t P = num_parts;
    if (m == 0) return fail(SFG_EINVAL, "pba_generate: m must be >= 1");
    if (P == 0 || P > kMaxParts) return fail(SFG_EINVAL, "pba_generate: num_parts must be in [1, %u]", kMaxParts);
    if (n < 2ull * P) return fail(SFG_EINVAL, "pba_generate: every partition needs >= 2 vertices (n >= 2 * num_parts)");
    if (!(p_inter >= 0.0 && p_inter <= 1.0)) return fail(SFG_EINVAL, "pba_generate: p_inter must be in [0, 1]");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "pba_generate: id_bytes must be 4 or 8");
    if (graph_id >= (1u << 24)) return fail(SFG_EINVAL, "pba_generate: graph_id must be < 2^24");
    if (!src || !dst || !workspace) return fail(SFG_EINVAL, "pba_generate: NULL buffer");
    if (n > (1ull << 40) || (uint64_t)m > (1ull << 20) || n * m > (1ull << 46))
        return fail(SFG_ERANGE, "pba_generate: n * m too large");
    if (id_bytes == 4 && n - 1 > 0x7FFFFFFFull) return fail(SFG_ERANGE, "pba_generate: n does not fit int32 ids");
    const uint64_t Lmax = (n + P - 1) / P;
    if (Lmax * m >= kTerm) return fail(SFG_ERANGE, "pba_generate: a partition holds >= 2^31 slots");
    // floor(t L / D) in 64 bits needs D * L < 2^64 with D <= n m.
    if ((unsigned __int128)(n * m) * Lmax >= ((unsigned __int128)1 << 64))
        return fail(SFG_ERANGE, "pba_generate: n * m * ceil(n / P) must be < 2^64");
    // Faction tables.
    std::vector<uint32_t> foff, fmem, uoff, umem;
    if (faction_off) {
        if (faction_off[0] != 0) return fail(SFG_EINVAL, "pba_generate: faction_off[0] must be 0");
        for (uint32_t q = 0; q < P; ++q) {
            if (faction_off[q + 1] < faction_off[q]) return fail(SFG_EINVAL, "pba_generate: faction_off is not monotone");
            // Copying needs an earlier slot: every partition starts from at
            // least one faction member.
            if (faction_off[q + 1] == faction_off[q])
                return fail(SFG_EINVAL, "pba_generate: partition %u has an empty faction list", q);
        }
        const uint32_t total = faction_off[P];
        if (total > 0 && !faction_members) return fail(SFG_EINVAL, "pba_generate: faction_members is NULL");
        foff.assign(faction_off, faction_off + P + 1);
        fmem.assign(faction_members, faction_members + total);
        for (uint32_t i = 0; i < total; ++i)
            if (fmem[i] >= P) return fail(SFG_EINVAL, "pba_generate: faction member %u >= num_parts", fmem[i]);
        uoff.resize(P + 1);
        uoff[0] = 0;
        for (uint32_t q = 0; q < P; ++q) {
            std::vector<uint32_t> u(fmem.begin() + foff[q], fmem.begin() + foff[q + 1]);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            umem.insert(umem.end(), u.begin(), u.end());
            uoff[q + 1] = (uint32_t)umem.size();
        }
    }
    Plan pl = make_plan(n, m, P, fmem.size());
    if (workspace_bytes < pl.total)
        return fail(SFG_ENOSPACE, "pba_generate: workspace has %zu bytes, needs %zu", workspace_bytes, pl.total);
    const size_t lds_sub = (size_t)4 * P * 4;
    uint32_t *err = device_error_word();
    if (!err) return fail(SFG_EDEVICE, "pba_generate: no device");

    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    uint32_t *lab = reinterpret_cast<uint32_t *>(ws + pl.off_lab);
    uint32_t *sel = reinterpret_cast<uint32_t *>(ws + pl.off_sel);
    uint32_t *H = reinterpret_cast<uint32_t *>(ws + pl.off_H);
    uint32_t *part = reinterpret_cast<uint32_t *>(ws + pl.off_part);
    uint64_t *base1 = reinterpret_cast<uint64_t *>(ws + pl.off_base1);
    uint64_t *sbase = reinterpret_cast<uint64_t *>(ws + pl.off_sbase);
    uint64_t *D = reinterpret_cast<uint64_t *>(ws + pl.off_D);
    uint64_t *xpre = reinterpret_cast<uint64_t *>(ws + pl.off_xpre);
    uint64_t *xtot = reinterpret_cast<uint64_t *>(ws + pl.off_xtot);
    uint32_t *queues = reinterpret_cast<uint32_t *>(ws + pl.off_queues);
    Factions fac{nullptr, nullptr, nullptr, nullptr};
    if (faction_off) {
        uint32_t *d_foff = reinterpret_cast<uint32_t *>(ws + pl.off_foff);
        uint32_t *d_fmem = reinterpret_cast<uint32_t *>(ws + pl.off_fmem);
        uint32_t *d_uoff = reinterpret_cast<uint32_t *>(ws + pl.off_uoff);
        uint32_t *d_umem = reinterpret_cast<uint32_t *>(ws + pl.off_umem);
        if (hipMemcpyAsync(d_foff, foff.data(), foff.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            (!fmem.empty() && hipMemcpyAsync(d_fmem, fmem.data(), fmem.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) ||
            hipMemcpyAsync(d_uoff, uoff.data(), uoff.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            (!umem.empty() && hipMemcpyAsync(d_umem, umem.data(), umem.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess))
            return check_launch("pba_generate: faction upload");
        // The host vectors die at return: wait for the copies.
        if (hipStreamSynchronize(s) != hipSuccess) return check_launch("pba_generate: faction upload");
        fac = Factions{d_foff, d_fmem, d_uoff, d_umem};
    }
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const int cus = device_cu_count();
    const int res_grid = cus * 8;

    // Phase 1.
    { ProfScope _ps("pba_tile_table", s); pba_phase1_bases<<<(P + 1 + 255) / 256, 256, 0, s>>>(n, P, m, base1); }
    Draw1Args d1{n, P, m, key0, key1, TAG_PBA1 | (graph_id << 8), 0, fac, lab};
    {
        double t = std::floor(p_inter * 4294967296.0);
        d1.thr_p = t <= 0.0 ? 0 : (t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t);
    }
    // Grid-stride launches: a dispatch's work-item count per dimension must
    // stay below 2^32.
    const uint64_t per_part = (pl.Lmax * m + kDrawThreads - 1) / kDrawThreads;
    dim3 g1((unsigned)std::min<uint64_t>(per_part, std::max<uint64_t>(1, (uint64_t)cus * 64 / P + 1)), P);
    { ProfScope _ps("pba_draw1", s); pba_draw1<<<g1, kDrawThreads, 0, s>>>(d1); }
    { ProfScope _ps("pba_tile_table", s); pba_tile_table<<<1, 64, 0, s>>>(base1, P, pl.xstride, xpre, xtot, queues); }
    { ProfScope _ps("pba_resolve", s); pba_resolve<<<res_grid, kResThreads, 0, s>>>(ResolveArgs{lab, base1, xpre, xtot, queues, err, P, pl.xstride}); }

    // Count exchange.
    dim3 gc(pl.T1, P);
    { ProfScope _ps("pba_count", s); pba_count<<<gc, 256, P * 4, s>>>(CountArgs{lab, base1, H, P, pl.T1, pl.CT}); }
    dim3 gs((unsigned)pl.groups, (P + 255) / 256);
    { ProfScope _ps("pba_scan", s); pba_scan_partial<<<gs, 256, 0, s>>>(H, pl.R, P, part); }
    { ProfScope _ps("pba_scan", s); pba_scan_groups<<<(P + 255) / 256, 256, 0, s>>>(part, pl.groups, P, D, err); }
    { ProfScope _ps("pba_scan", s); pba_scan_apply<<<gs, 256, 0, s>>>(H, pl.R, P, part); }
    { ProfScope _ps("pba_scan", s); pba_list_bases<<<1, 1024, 0, s>>>(D, P, sbase); }

    // Phase 2.
    Draw2Args d2{n, P, pl.E, key0, key1, TAG_PBA2 | (graph_id << 8), sbase, sel};
    { ProfScope _ps("pba_draw2", s); pba_draw2<<<(unsigned)std::min<uint64_t>((pl.E + kDrawThreads - 1) / kDrawThreads, (uint64_t)cus * 64), kDrawThreads, 0, s>>>(d2); }
    { ProfScope _ps("pba_tile_table", s); pba_tile_table<<<1, 64, 0, s>>>(sbase, P, pl.xstride, xpre, xtot, queues + kXcd); }
    { ProfScope _ps("pba_resolve", s); pba_resolve<<<res_grid, kResThreads, 0, s>>>(ResolveArgs{sel, sbase, xpre, xtot, queues + kXcd, err, P, pl.xstride}); }

    // Substitution.
    uint32_t lbits = 0;
    while ((1u << lbits) < P) ++lbits;
    SubArgs sa{n, P, m, pl.T1, pl.CT, lbits, lab, base1, H, sbase, sel, src, dst};
    dim3 gsub(pl.T1, P);
    if (id_bytes == 4)
        { ProfScope _ps("pba_substitute", s); pba_substitute<int32_t><<<gsub, kSubThreads, lds_sub, s>>>(sa); }
    else
        { ProfScope _ps("pba_substitute", s); pba_substitute<int64_t><<<gsub, kSubThreads, lds_sub, s>>>(sa); }
    return check_launch("pba_generate");
}
