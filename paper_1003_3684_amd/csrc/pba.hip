// Parallel Barabasi-Albert generation (section "Parallel Barabasi-Albert (PBA)
// method", Fig. 1) on one GPU, for one graph or a batch of graphs.
//
// The paper's processors become partitions of contiguous vertex blocks, and
// its two message exchanges become on-device passes.  A batch is a list of
// graphs; every (graph, partition) pair is a segment, and all passes run over
// all segments of the batch at once:
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
// terminal and writes the terminal back.  Segments are bound to XCDs
// (workgroup b runs on XCD b mod 8) and every XCD walks its segments tile
// by tile in slot order, so most pointers land in the already resolved,
// L2-resident prefix of the partition and a chain costs about one load.
// Output depends only on the draws, not on this schedule.
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "pba.hpp"

namespace sfg {
namespace {

constexpr uint32_t kTerm = 0x80000000u;  // bound of a partition's slot count and of a list's length
constexpr int kXcd = 8;
constexpr int kResThreads = 256;
constexpr int kResItems = 16;
constexpr int kResTile = kResThreads * kResItems;  // slots per resolve tile
constexpr int kSubThreads = 256;
constexpr uint32_t kMaxParts = 4096;
constexpr int kScanRows = 256;

// Partition boundaries floor(q n / P), evaluated without 128-bit products.
__host__ __device__ __forceinline__ uint64_t part_start(uint64_t q, uint64_t n, uint64_t P) {
    const uint64_t qd = n / P, r = n % P;
    return q * qd + (q * r) / P;
}

// floor(x / d) by multiply-high with magic = floor((2^32 - 1) / d) (32-bit)
// or floor((2^64 - 1) / d) (64-bit): the estimate is the quotient or one
// less, and one correction step makes it exact.
__device__ __forceinline__ uint32_t div_magic32(uint32_t x, uint32_t d, uint32_t magic) {
    uint32_t q = __umulhi(x, magic);
    if (x - q * d >= d) ++q;
    return q;
}
__device__ __forceinline__ uint64_t div_magic64(uint64_t x, uint64_t d, uint64_t magic) {
    uint64_t q = __umul64hi(x, magic);
    if (x - q * d >= d) ++q;
    return q;
}

// One graph of a batch (device table; a single graph travels by value).
struct PGraph {
    uint64_t n, vbase, ebase, thr_p, H0;
    uint32_t m, P, T1, CT, seg0;
    uint32_t key0, key1, tag1, tag2;
};

// Segment -> graph.  A single graph has segments 0..P-1 and no table.
struct Graphs {
    const PGraph *table;      // null for a single graph
    const uint32_t *seg_graph;
    PGraph one;
    __device__ __forceinline__ const PGraph &of_seg(uint32_t s, uint32_t &g) const {
        if (!table) {
            g = 0;
            return one;
        }
        g = seg_graph[s];
        return table[g];
    }
};

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

__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// ----------------------------------------------------------------------------- bases
__global__ void pba_bases1(Graphs G, uint32_t S, uint64_t total, uint64_t *base1) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > S) return;
    if (s == S) {
        base1[S] = total;
        return;
    }
    uint32_t g;
    const PGraph &p = G.of_seg(s, g);
    base1[s] = p.ebase + (uint64_t)p.m * part_start(s - p.seg0, p.n, p.P);
}

// ----------------------------------------------------------------------------- sentinels
__global__ void pba_fill32(uint32_t *p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ----------------------------------------------------------------------------- chain resolution
// A slot's phase-1 label and a selection's phase-2 endpoint are found by
// following copy pointers to a terminal draw.  Both passes run the draws
// themselves (Philox is counter-based, so any slot's draw can be recomputed
// anywhere): a thread draws its element, and while the draw points to an
// earlier element it reads that element's resolved value, or, if that one is
// not resolved yet (it still holds the sentinel every element starts from),
// draws it in turn.  Every pointer goes to a strictly earlier element, so a
// walk ends.  Segment s spans [base[s], base[s+1]) of the value array; tiles
// of segment s are queued on XCD s mod 8, segment by segment, in order, so
// most pointers land in the already resolved prefix of the segment, which
// stays in that XCD's L2 and the memory-side cache.
constexpr uint16_t kLabNone = 0xFFFFu;      // phase-1 label not resolved yet
constexpr uint32_t kSelNone = 0xFFFFFFFFu;  // phase-2 endpoint not resolved yet

struct ResolveArgs {
    Graphs G;
    Factions f;
    void *val;                // uint16_t labels (phase 1) or uint32_t endpoints (phase 2)
    const uint64_t *base;     // [S+1]
    const uint64_t *xprefix;  // [8][xstride] tile prefix per XCD queue
    const uint64_t *xtotal;   // [8]
    uint32_t *queues;         // [8] tile tickets
    uint32_t S, xstride;
};

// Phase-1 parameters of one partition (workgroup-uniform).  F and U are
// null for the default faction list [q].
struct Seg1 {
    uint32_t q, fs, u, nnf, tag, key0, key1;
    uint64_t thr_p;
    const uint32_t *F, *U;
};

// Terminal label of slot j of partition sg.q (labels: uint16_t, kLabNone
// while unresolved).
__device__ __forceinline__ uint32_t phase1_label(uint64_t j, const Seg1 &sg, const uint16_t *lab) {
    for (;;) {
        if (j < sg.fs) return sg.F ? sg.F[j] : sg.q;
        const Block4 w = philox((uint32_t)j, (uint32_t)(j >> 32), sg.q, sg.tag, sg.key0, sg.key1);
        const uint64_t U64 = make_u64(w.w1, w.w2);
        if (sg.nnf > 0 && (uint64_t)w.w0 < sg.thr_p) {
            const uint32_t r = (uint32_t)uidx64(U64, sg.nnf);
            return sg.U ? nonfaction(r, sg.U, sg.u) : r + (r >= sg.q ? 1u : 0u);
        }
        j = uidx64(U64, j);  // copy an earlier slot
        const uint32_t v = lab[j];
        if (v != kLabNone) return v;
    }
}

// Phase-2 parameters of one list (workgroup-uniform).
struct Seg2 {
    uint32_t l, tag, key0, key1;
    uint64_t L, D, magic;
};

// Endpoint (local vertex) of selection t of list sg.l: pool entry r of the
// first 2 + 2t is a seed-clique vertex (r < 2), the arrival floor(t' L / D)
// of selection t' = (r - 2) / 2 (even r), or the endpoint of selection
// (r - 3) / 2 (odd r).
__device__ __forceinline__ uint32_t phase2_endpoint(uint64_t t, const Seg2 &sg, const uint32_t *sel) {
    for (;;) {
        const Block4 w = philox((uint32_t)t, (uint32_t)(t >> 32), sg.l, sg.tag, sg.key0, sg.key1);
        const uint64_t r = uidx64(make_u64(w.w0, w.w1), 2 + 2 * t);
        if (r < 2) return (uint32_t)r;
        if ((r & 1) == 0) return (uint32_t)div_magic64(((r - 2) >> 1) * sg.L, sg.D, sg.magic);
        t = (r - 3) >> 1;
        const uint32_t v = sel[t];
        if (v != kSelNone) return v;
    }
}

template <int PHASE> __global__ __launch_bounds__(kResThreads) void pba_resolve(ResolveArgs a) {
    __shared__ uint64_t s_tile;
    __shared__ uint32_t s_seg;
    const int tid = threadIdx.x;
    const uint32_t home = blockIdx.x % kXcd;
    for (uint32_t att = 0; att < kXcd; ++att) {
        const uint32_t x = (home + att) % kXcd;
        const uint64_t total = a.xtotal[x];
        const uint64_t *pre = a.xprefix + (uint64_t)x * a.xstride;
        const uint32_t nseg = (a.S > x) ? (a.S - x + kXcd - 1) / kXcd : 0;
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
            const uint32_t sgi = x + kXcd * i;
            const uint64_t b0 = a.base[sgi];
            const uint64_t len = a.base[sgi + 1] - b0;
            const uint64_t first = (t - pre[i]) * kResTile;
            uint32_t g;
            const PGraph &p = a.G.of_seg(sgi, g);
            if (PHASE == 1) {
                Seg1 sg;
                sg.q = sgi - p.seg0;
                sg.fs = 1;
                sg.u = 1;
                sg.F = sg.U = nullptr;
                if (a.f.foff) {
                    sg.F = a.f.fmem + a.f.foff[sg.q];
                    sg.fs = a.f.foff[sg.q + 1] - a.f.foff[sg.q];
                    sg.U = a.f.umem + a.f.uoff[sg.q];
                    sg.u = a.f.uoff[sg.q + 1] - a.f.uoff[sg.q];
                }
                sg.nnf = p.P - sg.u;
                sg.thr_p = p.thr_p;
                sg.tag = p.tag1;
                sg.key0 = p.key0;
                sg.key1 = p.key1;
                uint16_t *lab = static_cast<uint16_t *>(a.val) + b0;
#pragma unroll 4
                for (int k = 0; k < kResItems; ++k) {
                    const uint64_t j = first + (uint64_t)k * kResThreads + tid;
                    if (j < len) lab[j] = (uint16_t)phase1_label(j, sg, lab);
                }
            } else {
                Seg2 sg;
                sg.l = sgi - p.seg0;
                sg.tag = p.tag2;
                sg.key0 = p.key0;
                sg.key1 = p.key1;
                sg.L = part_start(sg.l + 1, p.n, p.P) - part_start(sg.l, p.n, p.P);
                sg.D = len;
                sg.magic = len ? ~0ull / len : 0;
                uint32_t *sel = static_cast<uint32_t *>(a.val) + b0;
#pragma unroll 4
                for (int k = 0; k < kResItems; ++k) {
                    const uint64_t tt = first + (uint64_t)k * kResThreads + tid;
                    if (tt < len) sel[tt] = phase2_endpoint(tt, sg, sel);
                }
            }
        }
    }
}

// Per-XCD queues of resolve tiles: prefix of tile counts over the segments
// s = x, x+8, ... of each XCD x (one workgroup per XCD queue).
__global__ __launch_bounds__(1024) void pba_tile_table(const uint64_t *base, uint32_t S, uint32_t xstride,
                                                       uint64_t *xprefix, uint64_t *xtotal, uint32_t *queues) {
    __shared__ uint64_t sm[1024];
    const uint32_t x = blockIdx.x;
    const uint32_t nseg = S > x ? (S - x + kXcd - 1) / kXcd : 0;
    const uint32_t per = (nseg + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = std::min<uint32_t>(nseg, lo + per);
    uint64_t acc = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t sg = x + kXcd * i;
        acc += (base[sg + 1] - base[sg] + kResTile - 1) / kResTile;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t o = threadIdx.x >= (uint32_t)off ? sm[threadIdx.x - off] : 0;
        __syncthreads();
        sm[threadIdx.x] += o;
        __syncthreads();
    }
    uint64_t run = threadIdx.x > 0 ? sm[threadIdx.x - 1] : 0;
    uint64_t *pre = xprefix + (uint64_t)x * xstride;
    for (uint32_t i = lo; i < hi; ++i) {
        pre[i] = run;
        const uint32_t sg = x + kXcd * i;
        run += (base[sg + 1] - base[sg] + kResTile - 1) / kResTile;
    }
    if (threadIdx.x == 1023) {
        pre[nseg] = sm[1023];
        xtotal[x] = sm[1023];
        queues[x] = 0;
    }
}

// ----------------------------------------------------------------------------- counting
// Tile (q, tau) of graph g covers slots [tau * CT, (tau+1) * CT) of partition
// q; its label histogram is row H0 + (q * T1 + tau) of P columns.
struct CountArgs {
    Graphs G;
    const uint16_t *lab;
    const uint64_t *base1;
    uint32_t *H;
    uint32_t T1max;
};

__global__ __launch_bounds__(256) void pba_count(CountArgs a) {
    extern __shared__ uint32_t s_h[];  // [P]
    const uint32_t s = blockIdx.x / a.T1max, tau = blockIdx.x % a.T1max;
    uint32_t g;
    const PGraph &p = a.G.of_seg(s, g);
    if (tau >= p.T1) return;
    const uint32_t q = s - p.seg0;
    for (uint32_t l = threadIdx.x; l < p.P; l += 256) s_h[l] = 0;
    __syncthreads();
    const uint64_t b0 = a.base1[s], len = a.base1[s + 1] - b0;
    const uint64_t first = (uint64_t)tau * p.CT;
    const uint64_t last = std::min<uint64_t>(len, first + p.CT);
    // Eight labels per thread in flight, then their counts.
    for (uint64_t j0 = first + threadIdx.x; j0 < last; j0 += 256 * 8) {
        uint32_t l[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t j = j0 + (uint64_t)u * 256;
            l[u] = j < last ? a.lab[b0 + j] : 0u;
        }
        // The partition's own label is the most frequent one (every chain
        // that reaches the first slot ends there): its lanes are counted by
        // a ballot instead of contending for one LDS word.
        uint32_t own = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool in = j0 + (uint64_t)u * 256 < last;
            const bool mine = in && l[u] == q;
            own += (uint32_t)__popcll(__ballot(mine));
            if (in && !mine) atomicAdd(&s_h[l[u]], 1u);
        }
        if ((threadIdx.x & 63) == 0 && own) atomicAdd(&s_h[q], own);
    }
    __syncthreads();
    uint32_t *row = a.H + p.H0 + ((uint64_t)q * p.T1 + tau) * p.P;
    for (uint32_t l = threadIdx.x; l < p.P; l += 256) row[l] = s_h[l];
}

// In-place exclusive prefix sum of n words spaced stride apart, starting from
// acc; returns the total.  Sixteen loads go out together before their
// stores: in a load-store-load chain every load would also wait for the
// store before it.
__device__ __forceinline__ uint64_t scan_strided(uint32_t *x, uint64_t n, uint64_t stride, uint64_t acc) {
    constexpr int kBatch = 16;
    uint64_t r = 0;
    for (; r + kBatch <= n; r += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) v[u] = x[(r + u) * stride];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            x[(r + u) * stride] = (uint32_t)acc;
            acc += v[u];
        }
    }
    for (; r < n; ++r) {
        const uint32_t v = x[r * stride];
        x[r * stride] = (uint32_t)acc;
        acc += v;
    }
    return acc;
}

// Column-wise exclusive scan of every graph's H block.  Column c of the batch
// is label c - seg0 of the graph owning segment c; D[c] receives its total.
__global__ __launch_bounds__(256) void pba_scan_columns(Graphs G, uint32_t S, uint32_t *H, uint64_t *D,
                                                        uint32_t *err) {
    const uint32_t c = blockIdx.x * 256 + threadIdx.x;
    if (c >= S) return;
    uint32_t g;
    const PGraph &p = G.of_seg(c, g);
    const uint32_t l = c - p.seg0;
    const uint64_t rows = (uint64_t)p.P * p.T1;
    const uint64_t acc = scan_strided(H + p.H0 + l, rows, p.P, 0);
    D[c] = acc;
    if (acc >= kTerm) raise_device_error(err, DEVERR_QUEUE);  // a list longer than 2^31 is unsupported
}

// The same scan for one large graph, in three steps over groups of rows.
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
    const uint64_t acc = scan_strided(part + col, groups, P, 0);
    D[col] = acc;
    if (acc >= kTerm) raise_device_error(err, DEVERR_QUEUE);
}

__global__ __launch_bounds__(256) void pba_scan_apply(uint32_t *H, uint64_t R, uint32_t P, const uint32_t *part) {
    const uint32_t col = blockIdx.y * 256 + threadIdx.x;
    if (col >= P) return;
    const uint64_t r0 = (uint64_t)blockIdx.x * kScanRows;
    const uint64_t r1 = std::min<uint64_t>(R, r0 + kScanRows);
    scan_strided(H + r0 * P + col, r1 - r0, P, part[(uint64_t)blockIdx.x * P + col]);
}

// List bases: sbase = exclusive prefix of D over all segments (single block).
__global__ __launch_bounds__(1024) void pba_list_bases(const uint64_t *D, uint32_t S, uint64_t *sbase) {
    __shared__ uint64_t sm[1024];
    const uint32_t per = (S + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = std::min<uint32_t>(S, lo + per);
    uint64_t acc = 0;
    for (uint32_t i = lo; i < hi; ++i) acc += D[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t o = threadIdx.x >= (uint32_t)off ? sm[threadIdx.x - off] : 0;
        __syncthreads();
        sm[threadIdx.x] += o;
        __syncthreads();
    }
    uint64_t run = threadIdx.x > 0 ? sm[threadIdx.x - 1] : 0;
    for (uint32_t i = lo; i < hi; ++i) {
        sbase[i] = run;
        run += D[i];
    }
    if (threadIdx.x == 1023) sbase[S] = sm[1023];
}

// ----------------------------------------------------------------------------- substitution
// Tile (q, tau) of CT slots, taken in sub-tiles of kSubSlots slots in slot
// order.  The k-th slot of label l in the tile takes entry H[q,tau][l] + k of
// l's list (H holds the exclusive column prefix).  Each sub-tile is sorted by
// label in LDS -- stable ranks inside each wave's quarter from ballots over
// the label bits, then prefixes over the waves and over the labels (lane-match
// tables in LDS were slower: their 32 KB cost a workgroup per CU) -- so that one label's
// run of endpoints is loaded by consecutive lanes from consecutive addresses
// (one request per run instead of one per slot); the edges are then written
// in slot order.  Tiles are spread over the XCDs in contiguous ranges
// (workgroup b runs on XCD b mod 8), so neighbouring tiles of a partition,
// which read neighbouring pieces of the same lists, share an L2.
constexpr int kSubSlots = 2048;
constexpr int kSubWave = kSubSlots / 4;  // slots of each wave's quarter
constexpr int kSubSteps = kSubWave / 64;
static_assert(kSubThreads == 256, "four waves per substitution workgroup");

struct SubArgs {
    Graphs G;
    const uint16_t *lab;
    const uint64_t *base1;
    const uint32_t *H;
    const uint64_t *sbase;
    const uint32_t *sel;
    void *src, *dst;
    uint32_t T1max, Pmax;
    uint64_t tiles, per_xcd;
};

// Bytes of dynamic LDS of the substitution for up to Pmax labels.
size_t sub_lds_bytes(uint32_t Pmax) {
    return (size_t)Pmax * 8 + (size_t)kSubSlots * 4 + (size_t)4 * Pmax * 2 + (size_t)Pmax * 2 + (size_t)kSubSlots * 2 * 2;
}

template <typename IdT> __global__ __launch_bounds__(kSubThreads) void pba_substitute(SubArgs a) {
    extern __shared__ uint64_t s_dyn[];
    __shared__ uint32_t s_part[kSubThreads / 64];
    const uint64_t b = blockIdx.x;
    const uint64_t lt = (b % kXcd) * a.per_xcd + b / kXcd;
    if (lt >= a.tiles) return;
    const uint32_t s = (uint32_t)(lt / a.T1max), tau = (uint32_t)(lt % a.T1max);
    uint32_t g;
    const PGraph &p = a.G.of_seg(s, g);
    if (tau >= p.T1) return;
    const uint32_t q = s - p.seg0;
    const uint32_t P = p.P, Pm = a.Pmax;
    const int tid = threadIdx.x, w = tid >> 6;
    const uint32_t lane = tid & 63;
    // LDS carving (8-byte arrays first).
    uint64_t *s_cur = s_dyn;                                      // [Pm] next list entry of each label
    uint32_t *s_val = reinterpret_cast<uint32_t *>(s_cur + Pm);   // [kSubSlots] endpoints, slot order
    uint16_t *s_wcnt = reinterpret_cast<uint16_t *>(s_val + kSubSlots);  // [4][Pm]
    uint16_t *s_off = s_wcnt + 4 * Pm;                            // [Pm] label bases in sorted order
    uint16_t *s_lab = s_off + Pm;                                 // [kSubSlots] labels, slot order
    uint16_t *s_perm = s_lab + kSubSlots;                         // [kSubSlots] slot of each sorted position

    const uint64_t b0 = a.base1[s], len = a.base1[s + 1] - b0;
    const uint64_t first = (uint64_t)tau * p.CT;
    const uint64_t last = std::min<uint64_t>(len, first + p.CT);
    const uint32_t *hrow = a.H + p.H0 + ((uint64_t)q * p.T1 + tau) * P;
    const uint64_t *lbase = a.sbase + p.seg0;
    // Labels of this wave's quarter of a sub-tile.  Each sub-tile's labels
    // are loaded while the previous one is gathered and written (the first
    // sub-tile's while the list positions are set up).
    uint32_t lr[kSubSteps];
    auto load_labels = [&](uint64_t p0) {
        const uint32_t ns = (uint32_t)std::min<uint64_t>(kSubSlots, last - p0);
#pragma unroll
        for (int st = 0; st < kSubSteps; ++st) {
            const uint32_t i = (uint32_t)w * kSubWave + (uint32_t)st * 64 + lane;
            lr[st] = i < ns ? a.lab[b0 + p0 + i] : 0u;
        }
    };
    if (first < last) load_labels(first);
    for (uint32_t l = tid; l < P; l += kSubThreads) s_cur[l] = lbase[l] + hrow[l];
    __syncthreads();
    uint32_t lbits = 0;
    while ((1u << lbits) < P) ++lbits;
    const uint64_t vstart = p.vbase + part_start(q, p.n, P);
    // Per-element divisions by multiply-high: start(l) = l floor(n / P) +
    // floor(l (n mod P) / P) with l (n mod P) < P^2 <= 2^24, and the local
    // source j / m with j below the partition's slot count (< 2^31, checked
    // on the host).
    const uint64_t pq = p.n / P;
    const uint32_t pr = (uint32_t)(p.n % P), pmagic = 0xFFFFFFFFu / P, mmagic = 0xFFFFFFFFu / p.m;
    IdT *src = static_cast<IdT *>(a.src), *dst = static_cast<IdT *>(a.dst);
    uint16_t *wcnt = s_wcnt + (uint64_t)w * Pm;

    for (uint64_t pos0 = first; pos0 < last; pos0 += kSubSlots) {
        const uint32_t nsub = (uint32_t)std::min<uint64_t>(kSubSlots, last - pos0);
        for (uint32_t l = lane; l < P; l += 64) wcnt[l] = 0;
        // This wave's labels, and their stable ranks inside its quarter.
        uint32_t rr[kSubSteps];
#pragma unroll
        for (int st = 0; st < kSubSteps; ++st) {
            const uint32_t i = (uint32_t)w * kSubWave + (uint32_t)st * 64 + lane;
            if (i < nsub) s_lab[i] = (uint16_t)lr[st];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int st = 0; st < kSubSteps; ++st) {
            const uint32_t i = (uint32_t)w * kSubWave + (uint32_t)st * 64 + lane;
            const bool valid = i < nsub;
            const uint32_t l = lr[st];
            // The lanes holding the same label: every ballot over one label
            // bit keeps the lanes that agree with this lane on that bit.
            uint64_t peers = __ballot(valid);
            for (uint32_t bb = 0; bb < lbits; ++bb) {
                const bool bit = (l >> bb) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            if (!valid) peers = 0;
            const uint32_t below = count_below(peers);
            const uint32_t k = wcnt[l];
            rr[st] = k + below;
            __builtin_amdgcn_wave_barrier();
            if (valid && below == 0) wcnt[l] = (uint16_t)(k + (uint32_t)__popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // Per label: prefix over the waves; then the label bases of the
        // sorted order by a block scan over the labels (contiguous ranges of
        // labels per thread).
        const uint32_t per = (P + kSubThreads - 1) / kSubThreads;
        const uint32_t l0 = (uint32_t)tid * per, l1 = std::min<uint32_t>(P, l0 + per);
        uint32_t tsum = 0;
        for (uint32_t l = l0; l < l1; ++l) {
            uint32_t acc = 0;
#pragma unroll
            for (int wv = 0; wv < 4; ++wv) {
                const uint32_t c = s_wcnt[wv * Pm + l];
                s_wcnt[wv * Pm + l] = (uint16_t)acc;
                acc += c;
            }
            s_off[l] = (uint16_t)acc;  // the label's count, for now
            tsum += acc;
        }
        uint32_t x = tsum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= (uint32_t)off) x += y;
        }
        if (lane == 63) s_part[w] = x;
        __syncthreads();
        uint32_t run = x - tsum;
        for (int wv = 0; wv < w; ++wv) run += s_part[wv];
        for (uint32_t l = l0; l < l1; ++l) {
            const uint32_t c = s_off[l];
            s_off[l] = (uint16_t)run;
            run += c;
        }
        __syncthreads();
        // Sorted position of every slot.
#pragma unroll
        for (int st = 0; st < kSubSteps; ++st) {
            const uint32_t i = (uint32_t)w * kSubWave + (uint32_t)st * 64 + lane;
            if (i < nsub) {
                const uint32_t l = lr[st];
                s_perm[s_off[l] + s_wcnt[w * Pm + l] + rr[st]] = (uint16_t)i;
            }
        }
        __syncthreads();
        // Gather in sorted order: the lanes of one label's run read
        // consecutive list entries.  All of a thread's loads are issued
        // before any result is stored, so they are in flight together.
        {
            constexpr int kPerThread = kSubSlots / kSubThreads;
            uint32_t slot[kPerThread], v[kPerThread];
#pragma unroll
            for (int k = 0; k < kPerThread; ++k) {
                const uint32_t i = (uint32_t)k * kSubThreads + tid;
                slot[k] = i < nsub ? s_perm[i] : 0u;
                const uint32_t l = s_lab[slot[k]];
                v[k] = i < nsub ? a.sel[s_cur[l] + (i - s_off[l])] : 0u;
            }
            if (pos0 + kSubSlots < last) load_labels(pos0 + kSubSlots);
#pragma unroll
            for (int k = 0; k < kPerThread; ++k)
                if ((uint32_t)k * kSubThreads + tid < nsub) s_val[slot[k]] = v[k];
        }
        __syncthreads();
        // Edges in slot order.
        for (uint32_t i = tid; i < nsub; i += kSubThreads) {
            const uint64_t j = pos0 + i;
            const uint32_t l = s_lab[i];
            const uint64_t e = b0 + j;
            const uint64_t jm = div_magic32((uint32_t)j, p.m, mmagic);
            const uint64_t lstart = (uint64_t)l * pq + div_magic32(l * pr, P, pmagic);
            src[e] = (IdT)(vstart + jm);
            dst[e] = (IdT)(p.vbase + lstart + s_val[i]);
        }
        // Advance every label's list position by its count in this sub-tile.
        for (uint32_t l = tid; l < P; l += kSubThreads) {
            const uint32_t nxt = l + 1 < P ? s_off[l + 1] : nsub;
            s_cur[l] += nxt - s_off[l];
        }
        __syncthreads();
    }
}

// Whole-tile substitution of one graph with at most 1,024 labels (tiles of
// at most 16,384 slots).  One workgroup per CU walks a contiguous range of
// tiles of its XCD (so the 32 workgroups of an XCD hold neighbouring tiles,
// which read neighbouring pieces of every list), sorts each whole tile by
// label in LDS with the same stable ranks as above, and gathers every
// label's run of list entries for the tile at once: a run is one request
// instead of one per sub-tile.  The next tile's labels and list positions
// are loaded while the current tile is ranked, and tile coordinates come
// from the partition bounds, so no load waits on another inside a tile.
// LDS (138 KB) is reused: the permutation words (slot | label << 14) take
// the labels' space once every slot's label and rank are in registers, and
// the gathered values (local destinations) take the space of the per-wave
// counts and the ranks.
constexpr int kTileThreads = 1024;
constexpr int kTileWaves = kTileThreads / 64;
constexpr uint32_t kTileMax = 16384;
constexpr int kTilePer = (int)kTileMax / kTileThreads;  // slots of a thread
constexpr uint32_t kTilePmax = 1024;
static_assert(kTilePer == 16 && kTilePmax <= (uint32_t)kTileThreads, "one label per thread in the label scans");
static_assert(kTileMax <= (1u << 14), "a slot fits the permutation word's low 14 bits");

template <typename IdT> __global__ __launch_bounds__(kTileThreads) void pba_substitute_tile(SubArgs a) {
    __shared__ uint64_t s_cur[kTilePmax];                 // list entry of each label's first slot in the tile
    __shared__ uint16_t s_off[kTilePmax];                 // label bases in sorted order
    __shared__ uint32_t s_r1[kTileMax];  // labels in slot order (u16), then slot | label << 14 of each sorted position
    uint16_t *s_lab = reinterpret_cast<uint16_t *>(s_r1);
    uint32_t *s_perm = s_r1;
    __shared__ uint32_t s_part[kTileWaves];
    __shared__ uint32_t s_u[kTileMax];  // per-wave label counts [kTileWaves][Pm] and ranks [kTileMax], then values
    uint16_t *s_wcnt = reinterpret_cast<uint16_t *>(s_u);
    uint16_t *s_rank = s_wcnt + kTileWaves * kTilePmax;
    uint32_t *s_val = s_u;
    static_assert(kTileWaves * kTilePmax * 2 + kTileMax * 2 <= kTileMax * 4, "counts and ranks share the values' space");
    const PGraph &p = a.G.one;  // a single graph
    const uint32_t P = p.P;
    const uint32_t xcd = blockIdx.x % kXcd, nper = gridDim.x / kXcd;
    const uint64_t lt_end = std::min<uint64_t>(a.tiles, (uint64_t)(xcd + 1) * a.per_xcd);
    uint64_t lt = (uint64_t)xcd * a.per_xcd + blockIdx.x / kXcd;
    uint32_t lbits = 0;
    while ((1u << lbits) < P) ++lbits;
    const uint64_t pq = p.n / P;
    const uint32_t pr = (uint32_t)(p.n % P), pmagic = 0xFFFFFFFFu / P, mmagic = 0xFFFFFFFFu / p.m;
    IdT *src = static_cast<IdT *>(a.src), *dst = static_cast<IdT *>(a.dst);

    // Tile lt covers slots [first, first + nsub) of partition q, whose slots
    // start at b0; false for a tile past the partition's end.
    uint32_t q = 0, nsub = 0;
    uint64_t b0 = 0, first = 0;
    auto tile_of = [&](uint64_t t, uint32_t &tq, uint32_t &tn, uint64_t &tb0, uint64_t &tfirst) -> bool {
        tq = (uint32_t)(t / a.T1max);
        const uint32_t tau = (uint32_t)(t % a.T1max);
        if (tau >= p.T1) return false;
        // The partition's slots, from its vertex range (no loads).
        const uint64_t v0 = part_start(tq, p.n, P), v1 = part_start(tq + 1, p.n, P);
        tb0 = p.ebase + (uint64_t)p.m * v0;
        const uint64_t len = (uint64_t)p.m * (v1 - v0);
        tfirst = (uint64_t)tau * p.CT;
        if (tfirst >= len) return false;
        tn = (uint32_t)std::min<uint64_t>(p.CT, len - tfirst);
        return true;
    };
    // A tile's labels (thread: 16 slots, wave w holding slots w*1024 ..
    // w*1024+1023) and the two parts of label tid's list position.
    uint32_t lr[kTilePer];
    uint64_t cur_a = 0;
    uint32_t cur_b = 0;
    auto load_tile = [&](uint32_t tq, uint32_t tn, uint64_t tb0, uint64_t tfirst) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int st = 0; st < kTilePer; ++st) {
            const uint32_t i = (uint32_t)(tid >> 6) * 1024u + (uint32_t)st * 64u + (tid & 63);
            lr[st] = a.lab[tb0 + tfirst + (i < tn ? i : tn - 1)];
        }
        const uint32_t tau = (uint32_t)(tfirst / p.CT);
        if ((uint32_t)tid < P) {
            cur_a = a.sbase[p.seg0 + tid];
            cur_b = a.H[p.H0 + ((uint64_t)tq * p.T1 + tau) * P + tid];
        }
    };

    bool have = false;
    while (lt < lt_end && !(have = tile_of(lt, q, nsub, b0, first))) lt += nper;
    if (!have) return;
    load_tile(q, nsub, b0, first);
    while (have) {
        // Lane indices made opaque per tile, so that the compiler does not
        // keep every slot address of the loop live across it.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const uint32_t lane = (uint32_t)tid & 63u, w = (uint32_t)tid >> 6;
        // This tile's labels and list positions into LDS, counts cleared.
#pragma unroll
        for (int st = 0; st < kTilePer; ++st) {
            const uint32_t i = w * 1024u + (uint32_t)st * 64u + lane;
            if (i < nsub) s_lab[i] = (uint16_t)lr[st];
        }
        if ((uint32_t)tid < P) s_cur[tid] = cur_a + cur_b;
        uint16_t *wcnt = s_wcnt + w * kTilePmax;
        for (uint32_t l = lane; l < P; l += 64) wcnt[l] = 0;
        // The next tile's labels are loaded while this one is processed.
        uint32_t nq = 0, nn = 0;
        uint64_t nb0 = 0, nfirst = 0;
        bool next = false;
        lt += nper;
        while (lt < lt_end && !(next = tile_of(lt, nq, nn, nb0, nfirst))) lt += nper;
        if (next) load_tile(nq, nn, nb0, nfirst);
        __builtin_amdgcn_wave_barrier();
        // Stable ranks inside each wave's 1,024 slots: every ballot over one
        // label bit keeps the lanes that agree with this lane on that bit.
        // Four steps at a time, so that their ballot chains interleave.
        for (int st = 0; st < kTilePer; st += 4) {
            uint32_t ii[4], ll[4];
            bool vv[4];
            uint64_t pp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ii[u] = w * 1024u + (uint32_t)(st + u) * 64u + lane;
                vv[u] = ii[u] < nsub;
                ll[u] = vv[u] ? s_lab[ii[u]] : 0u;
                pp[u] = __ballot(vv[u]);
            }
            for (uint32_t bb = 0; bb < lbits; ++bb) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool bt = (ll[u] >> bb) & 1u;
                    const uint64_t m = __ballot(bt);
                    pp[u] &= bt ? m : ~m;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t pu = vv[u] ? pp[u] : 0ull;
                const uint32_t below = count_below(pu);
                const uint32_t kk = wcnt[ll[u]];
                s_rank[ii[u]] = (uint16_t)(kk + below);
                __builtin_amdgcn_wave_barrier();
                if (vv[u] && below == 0) wcnt[ll[u]] = (uint16_t)(kk + (uint32_t)__popcll(pu));
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        // Label tid: prefix over the waves, then the label bases by a block scan.
        uint32_t cnt = 0;
        if ((uint32_t)tid < P) {
#pragma unroll
            for (int wv = 0; wv < kTileWaves; ++wv) {
                const uint32_t c = s_wcnt[wv * kTilePmax + tid];
                s_wcnt[wv * kTilePmax + tid] = (uint16_t)cnt;
                cnt += c;
            }
        }
        uint32_t xs = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(xs, off, 64);
            if (lane >= (uint32_t)off) xs += y;
        }
        if (lane == 63) s_part[w] = xs;
        __syncthreads();
        uint32_t run = xs - cnt;
        for (uint32_t wv = 0; wv < w; ++wv) run += s_part[wv];
        if ((uint32_t)tid < P) s_off[tid] = (uint16_t)run;
        __syncthreads();
        // Sorted position of every slot (its label and rank first taken
        // into registers: the permutation overwrites the labels).
        uint32_t lk[kTilePer];
#pragma unroll
        for (int st = 0; st < kTilePer; ++st) {
            const uint32_t i = w * 1024u + (uint32_t)st * 64u + lane;
            lk[st] = i < nsub ? (uint32_t)s_lab[i] | ((uint32_t)s_rank[i] << 16) : 0u;
        }
        __syncthreads();
#pragma unroll 4
        for (int st = 0; st < kTilePer; ++st) {
            const uint32_t i = w * 1024u + (uint32_t)st * 64u + lane;
            if (i < nsub) {
                const uint32_t l = lk[st] & 0xFFFFu;
                s_perm[s_off[l] + s_wcnt[w * kTilePmax + l] + (lk[st] >> 16)] = i | (l << 14);
            }
        }
        __syncthreads();  // the counts are dead: their space takes the values
        // Gather in sorted order.
        uint32_t v[kTilePer];
#pragma unroll
        for (int k = 0; k < kTilePer; ++k) {
            const uint32_t i = (uint32_t)k * kTileThreads + tid;
            const uint32_t ic = i < nsub ? i : nsub - 1;  // a valid address for every lane
            const uint32_t l = s_perm[ic] >> 14;
            v[k] = a.sel[s_cur[l] + (ic - s_off[l])];
        }
        // Unconditional stores: a lane past the tile's end repeats the last
        // slot's store with the same value (a conditional store would let
        // the compiler sink its load behind the wait for all of them).
        // The values stored are the local destinations: the label's first
        // vertex plus the endpoint (below 2^32: checked on the host).
#pragma unroll
        for (int k = 0; k < kTilePer; ++k) {
            const uint32_t i = (uint32_t)k * kTileThreads + tid;
            const uint32_t x = s_perm[i < nsub ? i : nsub - 1];
            const uint32_t l = x >> 14;
            const uint32_t lstart = l * (uint32_t)pq + div_magic32(l * pr, P, pmagic);
            s_val[x & (kTileMax - 1)] = lstart + v[k];
        }
        __syncthreads();
        // Edges in slot order.
        const uint64_t vstart = p.vbase + part_start(q, p.n, P);
#pragma unroll 4
        for (int k = 0; k < kTilePer; ++k) {
            const uint32_t i = (uint32_t)k * kTileThreads + tid;
            if (i < nsub) {
                const uint64_t j = first + i;
                const uint64_t e = b0 + j;
                const uint64_t jm = div_magic32((uint32_t)j, p.m, mmagic);
                __builtin_nontemporal_store((IdT)(vstart + jm), &src[e]);
                __builtin_nontemporal_store((IdT)(p.vbase + s_val[i]), &dst[e]);
            }
        }
        __syncthreads();  // the labels, the values and s_cur are rewritten by the next tile
        have = next;
        q = nq;
        nsub = nn;
        b0 = nb0;
        first = nfirst;
    }
}

uint32_t choose_ct(uint64_t P) {
    // Tiles of the count/substitution passes: large enough that the P x P
    // histogram rows stay a small fraction of the slot arrays.
    uint32_t ct = 4096;
    while (ct < 65536 && (uint64_t)ct < 16 * P) ct *= 2;
    return ct;
}

}  // namespace

// ----------------------------------------------------------------------------- host
// Layout of a batch in the workspace.
struct PbaPlan {
    uint32_t count, S, T1max, Pmax, xstride;
    uint64_t E, Htotal, groups;
    bool grouped;  // one large graph: three-step column scan
    size_t off_lab, off_sel, off_H, off_part, off_base1, off_sbase, off_D, off_xpre, off_xtot, off_queues, off_foff,
        off_fmem, off_uoff, off_umem, total;
};

static PbaPlan plan_batch(const PbaGraphSpec *gs, uint32_t count, uint64_t fmem_count) {
    PbaPlan p;
    memset(&p, 0, sizeof(p));
    p.count = count;
    for (uint32_t g = 0; g < count; ++g) {
        const uint64_t Lmax = (gs[g].n + gs[g].P - 1) / gs[g].P;
        const uint32_t CT = choose_ct(gs[g].P);
        const uint32_t T1 = (uint32_t)((Lmax * gs[g].m + CT - 1) / CT);
        p.S += gs[g].P;
        p.E += gs[g].n * gs[g].m;
        p.Htotal += (uint64_t)gs[g].P * T1 * gs[g].P;
        p.T1max = std::max(p.T1max, T1);
        p.Pmax = std::max(p.Pmax, gs[g].P);
        if (count == 1) p.groups = ((uint64_t)gs[g].P * T1 + kScanRows - 1) / kScanRows;
    }
    p.grouped = count == 1 && p.groups > 16;
    p.xstride = (p.S + kXcd - 1) / kXcd + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align256(bytes);
        return r;
    };
    p.off_lab = take(p.E * 2);
    p.off_sel = take(p.E * 4);
    p.off_H = take(p.Htotal * 4);
    p.off_part = take(p.grouped ? p.groups * p.Pmax * 4 : 0);
    p.off_base1 = take((p.S + 1) * 8);
    p.off_sbase = take((p.S + 1) * 8);
    p.off_D = take(p.S * 8);
    p.off_xpre = take((size_t)kXcd * p.xstride * 8);
    p.off_xtot = take(kXcd * 8);
    p.off_queues = take(2 * kXcd * 4);
    p.off_foff = take(count == 1 ? (p.S + 1) * 4 : 0);
    p.off_fmem = take(count == 1 ? std::max<uint64_t>(fmem_count, 1) * 4 : 0);
    p.off_uoff = take(count == 1 ? (p.S + 1) * 4 : 0);
    p.off_umem = take(count == 1 ? std::max<uint64_t>(fmem_count, 1) * 4 : 0);
    p.total = o;
    return p;
}

size_t pba_batch_workspace_bytes(const PbaGraphSpec *gs, uint32_t count) { return plan_batch(gs, count, 0).total; }

int pba_check_spec(const PbaGraphSpec &g, int id_bytes, const char *who) {
    if (g.m == 0) return fail(SFG_EINVAL, "%s: m must be >= 1", who);
    if (g.P == 0 || g.P > kMaxParts) return fail(SFG_EINVAL, "%s: num_parts must be in [1, %u]", who, kMaxParts);
    if (g.n < 2ull * g.P) return fail(SFG_EINVAL, "%s: every partition needs >= 2 vertices (n >= 2 * num_parts)", who);
    if (!(g.p_inter >= 0.0 && g.p_inter <= 1.0)) return fail(SFG_EINVAL, "%s: p_inter must be in [0, 1]", who);
    if (g.graph_id >= (1u << 24)) return fail(SFG_EINVAL, "%s: graph_id must be < 2^24", who);
    if (g.n > (1ull << 40) || (uint64_t)g.m > (1ull << 20) || g.n * g.m > (1ull << 46))
        return fail(SFG_ERANGE, "%s: n * m too large", who);
    if (id_bytes == 4 && g.vbase + g.n - 1 > 0x7FFFFFFFull) return fail(SFG_ERANGE, "%s: ids do not fit int32", who);
    const uint64_t Lmax = (g.n + g.P - 1) / g.P;
    if (Lmax * g.m >= kTerm) return fail(SFG_ERANGE, "%s: a partition holds >= 2^31 slots", who);
    // floor(t L / D) in 64 bits needs D * L < 2^64 with D <= n m.
    if ((unsigned __int128)(g.n * g.m) * Lmax >= ((unsigned __int128)1 << 64))
        return fail(SFG_ERANGE, "%s: n * m * ceil(n / P) must be < 2^64", who);
    return SFG_OK;
}

// Device tables of a batch of more than one graph: the graph table and the
// segment -> graph map, as one blob (built on the host, uploaded by the caller).
static size_t tables_seg_offset(uint32_t count) { return align256((size_t)count * sizeof(PGraph)); }

static void build_table(const PbaGraphSpec *gs, uint32_t count, PGraph *table, uint32_t *seg_graph) {
    uint64_t ebase = 0, H0 = 0;
    uint32_t seg0 = 0;
    for (uint32_t g = 0; g < count; ++g) {
        const PbaGraphSpec &sp = gs[g];
        PGraph &p = table[g];
        memset(&p, 0, sizeof(p));
        const uint64_t Lmax = (sp.n + sp.P - 1) / sp.P;
        p.n = sp.n;
        p.vbase = sp.vbase;
        p.ebase = ebase;
        const double t = std::floor(sp.p_inter * 4294967296.0);
        p.thr_p = t <= 0.0 ? 0 : (t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t);
        p.m = sp.m;
        p.P = sp.P;
        p.CT = choose_ct(sp.P);
        p.T1 = (uint32_t)((Lmax * sp.m + p.CT - 1) / p.CT);
        p.H0 = H0;
        p.seg0 = seg0;
        p.key0 = (uint32_t)sp.seed;
        p.key1 = (uint32_t)(sp.seed >> 32);
        p.tag1 = TAG_PBA1 | (sp.graph_id << 8);
        p.tag2 = TAG_PBA2 | (sp.graph_id << 8);
        ebase += sp.n * sp.m;
        H0 += (uint64_t)sp.P * p.T1 * sp.P;
        if (seg_graph)
            for (uint32_t q = 0; q < sp.P; ++q) seg_graph[seg0 + q] = g;
        seg0 += sp.P;
    }
}

size_t pba_tables_bytes(const PbaGraphSpec *gs, uint32_t count) {
    if (count < 2) return 0;
    uint64_t S = 0;
    for (uint32_t g = 0; g < count; ++g) S += gs[g].P;
    return tables_seg_offset(count) + align256(S * 4);
}

void pba_tables_fill(const PbaGraphSpec *gs, uint32_t count, void *host) {
    if (count < 2) return;
    char *h = static_cast<char *>(host);
    build_table(gs, count, reinterpret_cast<PGraph *>(h), reinterpret_cast<uint32_t *>(h + tables_seg_offset(count)));
}

// Every pass of the generation for a planned batch, enqueued on s (kernel
// launches only: the sequence can be captured into a graph).
static int enqueue(const PbaPlan &pl, const Graphs &G, const Factions &fac, uint32_t count, uint32_t T1_single,
                   uint32_t P_single, int id_bytes, void *src, void *dst, char *ws, hipStream_t s, const char *who) {
    uint32_t *err = device_error_word();
    if (!err) return fail(SFG_EDEVICE, "%s: no device", who);
    uint16_t *lab = reinterpret_cast<uint16_t *>(ws + pl.off_lab);
    uint32_t *sel = reinterpret_cast<uint32_t *>(ws + pl.off_sel);
    uint32_t *H = reinterpret_cast<uint32_t *>(ws + pl.off_H);
    uint32_t *part = reinterpret_cast<uint32_t *>(ws + pl.off_part);
    uint64_t *base1 = reinterpret_cast<uint64_t *>(ws + pl.off_base1);
    uint64_t *sbase = reinterpret_cast<uint64_t *>(ws + pl.off_sbase);
    uint64_t *D = reinterpret_cast<uint64_t *>(ws + pl.off_D);
    uint64_t *xpre = reinterpret_cast<uint64_t *>(ws + pl.off_xpre);
    uint64_t *xtot = reinterpret_cast<uint64_t *>(ws + pl.off_xtot);
    uint32_t *queues = reinterpret_cast<uint32_t *>(ws + pl.off_queues);
    const int cus = device_cu_count();
    const int res_grid = cus * 8;
    const uint32_t S = pl.S;

    auto fill32 = [&](void *ptr, uint64_t words, uint32_t v) {
        if (!words) return;
        ProfScope _ps("pba_fill", s);
        const uint64_t want = (words + 255) / 256;
        pba_fill32<<<(unsigned)std::min<uint64_t>(want, (uint64_t)cus * 8), 256, 0, s>>>(static_cast<uint32_t *>(ptr),
                                                                                      words, v);
    };

    // Phase 1: every slot's label, drawn and resolved in one pass over
    // sentinel-initialised labels.
    { ProfScope _ps("pba_tile_table", s); pba_bases1<<<(S + 1 + 255) / 256, 256, 0, s>>>(G, S, pl.E, base1); }
    fill32(lab, (pl.E + 1) / 2, 0xFFFFFFFFu);
    { ProfScope _ps("pba_tile_table", s); pba_tile_table<<<kXcd, 1024, 0, s>>>(base1, S, pl.xstride, xpre, xtot, queues); }
    {
        ProfScope _ps("pba_resolve", s);
        pba_resolve<1><<<res_grid, kResThreads, 0, s>>>(ResolveArgs{G, fac, lab, base1, xpre, xtot, queues, S, pl.xstride});
    }

    // Count exchange.
    { ProfScope _ps("pba_count", s); pba_count<<<S * pl.T1max, 256, pl.Pmax * 4, s>>>(CountArgs{G, lab, base1, H, pl.T1max}); }
    if (pl.grouped) {
        const uint32_t P = P_single;
        const uint64_t R = (uint64_t)P * T1_single;
        dim3 gsc((unsigned)pl.groups, (P + 255) / 256);
        { ProfScope _ps("pba_scan", s); pba_scan_partial<<<gsc, 256, 0, s>>>(H, R, P, part); }
        { ProfScope _ps("pba_scan", s); pba_scan_groups<<<(P + 255) / 256, 256, 0, s>>>(part, pl.groups, P, D, err); }
        { ProfScope _ps("pba_scan", s); pba_scan_apply<<<gsc, 256, 0, s>>>(H, R, P, part); }
    } else {
        { ProfScope _ps("pba_scan", s); pba_scan_columns<<<(S + 255) / 256, 256, 0, s>>>(G, S, H, D, err); }
    }
    { ProfScope _ps("pba_scan", s); pba_list_bases<<<1, 1024, 0, s>>>(D, S, sbase); }

    // Phase 2: every selection's endpoint, drawn and resolved in one pass.
    fill32(sel, pl.E, kSelNone);
    { ProfScope _ps("pba_tile_table", s); pba_tile_table<<<kXcd, 1024, 0, s>>>(sbase, S, pl.xstride, xpre, xtot, queues + kXcd); }
    {
        ProfScope _ps("pba_resolve", s);
        pba_resolve<2><<<res_grid, kResThreads, 0, s>>>(ResolveArgs{G, fac, sel, sbase, xpre, xtot, queues + kXcd, S, pl.xstride});
    }

    // Substitution.
    const uint64_t tiles = (uint64_t)S * pl.T1max;
    const uint64_t per_xcd = (tiles + kXcd - 1) / kXcd;
    SubArgs sa{G, lab, base1, H, sbase, sel, src, dst, pl.T1max, pl.Pmax, tiles, per_xcd};
    const size_t lds = sub_lds_bytes(pl.Pmax);
    const unsigned gsub = (unsigned)(per_xcd * kXcd);
    {
        ProfScope _ps("pba_substitute", s);
        if (count == 1 && pl.Pmax <= kTilePmax && G.one.n < (1ull << 32)) {
            const unsigned gt = (unsigned)std::min<uint64_t>((uint64_t)cus, (per_xcd) * kXcd) / kXcd * kXcd;
            if (id_bytes == 4)
                pba_substitute_tile<int32_t><<<std::max(gt, (unsigned)kXcd), kTileThreads, 0, s>>>(sa);
            else
                pba_substitute_tile<int64_t><<<std::max(gt, (unsigned)kXcd), kTileThreads, 0, s>>>(sa);
        } else if (id_bytes == 4)
            pba_substitute<int32_t><<<gsub, kSubThreads, lds, s>>>(sa);
        else
            pba_substitute<int64_t><<<gsub, kSubThreads, lds, s>>>(sa);
    }
    return check_launch(who);
}

int pba_enqueue_batch(const PbaGraphSpec *gs, uint32_t count, int id_bytes, void *src, void *dst, void *workspace,
                      size_t workspace_bytes, const void *dev_tables, hipStream_t s) {
    const char *who = "ensemble_generate";
    if (count == 0) return SFG_OK;
    for (uint32_t g = 0; g < count; ++g) {
        int rc = pba_check_spec(gs[g], id_bytes, who);
        if (rc != SFG_OK) return rc;
    }
    const PbaPlan pl = plan_batch(gs, count, 0);
    if (!src || !dst || !workspace || (count > 1 && !dev_tables)) return fail(SFG_EINVAL, "%s: NULL buffer", who);
    if (workspace_bytes < pl.total)
        return fail(SFG_ENOSPACE, "%s: workspace has %zu bytes, needs %zu", who, workspace_bytes, pl.total);
    PGraph first;
    build_table(gs, 1, &first, nullptr);
    Graphs G;
    memset(&G, 0, sizeof(G));
    G.one = first;
    if (count > 1) {
        const char *t = static_cast<const char *>(dev_tables);
        G.table = reinterpret_cast<const PGraph *>(t);
        G.seg_graph = reinterpret_cast<const uint32_t *>(t + tables_seg_offset(count));
    }
    return enqueue(pl, G, Factions{nullptr, nullptr, nullptr, nullptr}, count, first.T1, first.P, id_bytes, src, dst,
                   static_cast<char *>(workspace), s, who);
}

// One graph (pba_generate), with optional faction tables.
int pba_run_batch(const PbaGraphSpec *gs, uint32_t count, const uint32_t *faction_off, const uint32_t *faction_members,
                  int id_bytes, void *src, void *dst, void *workspace, size_t workspace_bytes, hipStream_t s) {
    const char *who = "pba_generate";
    if (count != 1) return fail(SFG_EINVAL, "%s: one graph per call", who);
    int rc = pba_check_spec(gs[0], id_bytes, who);
    if (rc != SFG_OK) return rc;
    // Faction tables.
    std::vector<uint32_t> foff, fmem, uoff, umem;
    if (faction_off) {
        const uint32_t P = gs[0].P;
        if (faction_off[0] != 0) return fail(SFG_EINVAL, "%s: faction_off[0] must be 0", who);
        for (uint32_t q = 0; q < P; ++q) {
            if (faction_off[q + 1] < faction_off[q]) return fail(SFG_EINVAL, "%s: faction_off is not monotone", who);
            // Copying needs an earlier slot: every partition starts from at
            // least one faction member.
            if (faction_off[q + 1] == faction_off[q])
                return fail(SFG_EINVAL, "%s: partition %u has an empty faction list", who, q);
        }
        const uint32_t total = faction_off[P];
        if (total > 0 && !faction_members) return fail(SFG_EINVAL, "%s: faction_members is NULL", who);
        foff.assign(faction_off, faction_off + P + 1);
        fmem.assign(faction_members, faction_members + total);
        for (uint32_t i = 0; i < total; ++i)
            if (fmem[i] >= P) return fail(SFG_EINVAL, "%s: faction member %u >= num_parts", who, fmem[i]);
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
    const PbaPlan pl = plan_batch(gs, 1, fmem.size());
    if (!src || !dst || !workspace) return fail(SFG_EINVAL, "%s: NULL buffer", who);
    if (workspace_bytes < pl.total)
        return fail(SFG_ENOSPACE, "%s: workspace has %zu bytes, needs %zu", who, workspace_bytes, pl.total);
    char *ws = static_cast<char *>(workspace);
    PGraph first;
    build_table(gs, 1, &first, nullptr);
    Graphs G;
    memset(&G, 0, sizeof(G));
    G.one = first;
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
        fac = Factions{d_foff, d_fmem, d_uoff, d_umem};
        // The host tables die at return: wait for their copies.
        if (hipStreamSynchronize(s) != hipSuccess) return check_launch("pba_generate: faction upload");
    }
    return enqueue(pl, G, fac, 1, first.T1, first.P, id_bytes, src, dst, ws, s, who);
}

}  // namespace sfg

using namespace sfg;

extern "C" size_t pba_workspace_bytes(uint64_t n, uint32_t m, uint32_t num_parts, uint64_t num_faction_members) {
    if (num_parts == 0 || m == 0 || n == 0) return 0;
    PbaGraphSpec g{n, m, num_parts, 0.0, 0, 0, 0};
    return plan_batch(&g, 1, num_faction_members).total;
}

extern "C" int pba_generate(uint64_t n, uint32_t m, uint32_t num_parts, double p_inter, const uint32_t *faction_off,
                            const uint32_t *faction_members, uint64_t seed, uint32_t graph_id, int id_bytes, void *src,
                            void *dst, void *workspace, size_t workspace_bytes, void *stream) {
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "pba_generate: id_bytes must be 4 or 8");
    PbaGraphSpec g{n, m, num_parts, p_inter, seed, graph_id, 0};
    return pba_run_batch(&g, 1, faction_off, faction_members, id_bytes, src, dst, workspace, workspace_bytes,
                         as_stream(stream));
}
