// Edge list -> compressed sparse rows, and the degree histogram.
//
// Entries (src, dst) are packed into one unsigned key (src << db) | dst, with
// db = bits(n - 1) (rounded up to a whole digit when in-degrees are needed),
// and sorted by a least-significant-digit radix sort with 8-bit digits over
// the live key bits.  One histogram pass counts every digit of every pass;
// each digit pass is then a single "onesweep" kernel: workgroup b takes tile
// b (8,192 keys; workgroups start in id order, so every tile waited for is
// already running), ranks its keys stably in LDS, publishes its per-digit
// counts and finds the counts of all earlier tiles by decoupled look-back,
// then writes its keys digit run by digit run (coalesced).  One read and one
// write of every key per pass -- the pass is HBM-bound.  The first pass reads
// the edge arrays and packs keys on the fly, so no separate packing pass
// exists.
//
// After the sort, one streaming pass writes the columns, marks the first
// sorted position of every row (its row start) and counts repeated entries;
// with SIMPLE it also drops self-loops and repeats, compacting by a
// look-back scan.  Rows with no entry are filled by a reverse min-scan over
// the row starts.  The degree histogram counts deg(v) = out + in per vertex
// (the degree distributions of the paper's Results section).  For a directed
// CSR the in-degrees come from the sort itself: once the digit passes over
// the destination field are done the keys are ordered by destination, and the
// next pass marks where each destination's run starts (a column-start array
// filled like the row starts) -- no atomics.
#include <string.h>

#include <algorithm>

#include "common.hpp"

namespace sfg {
namespace {

constexpr int kPassThreads = 1024;
constexpr int kPassItems = 8;
constexpr int kPassTile = kPassThreads * kPassItems;  // keys per onesweep tile
constexpr int kPassWaves = kPassThreads / 64;
constexpr int kRadix = 256;
constexpr int kLookWindow = 2;  // predecessors read per lane and look-back round trip
constexpr int kLanesPerDigit = kPassThreads / kRadix;  // look-back lanes per digit

constexpr int kFinThreads = 256;
constexpr int kFinItems = 12;  // 3,072-entry finish tiles: six workgroups per CU with 8-byte keys
constexpr int kFinTile = kFinThreads * kFinItems;

constexpr int kScanChunk = 4096;  // vertices per chunk of the row fill scan
constexpr int kPrepUnroll = 4;    // keys per thread in flight in the histogram pass
constexpr int kPrepCopies = 4;    // interleaved copies of each LDS histogram
constexpr int kPrepBlocksPerCu = 4;

constexpr uint64_t kNoRow = ~0ull;

// Look-back status word: [63:58] pass tag, [57:56] flag, [55:0] count.
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
__device__ __forceinline__ uint64_t status_word(uint32_t tag, uint64_t flag, uint64_t v) {
    return ((uint64_t)tag << 58) | (flag << 56) | v;
}


__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// Sum-scan over the first 256 threads of a block (4 waves): returns the
// exclusive prefix of v and writes the total to *total.  All threads of the
// block must call it.
__device__ uint64_t block_exclusive_scan_256(uint64_t v, uint64_t *s_tmp /*[4]*/, uint64_t *total) {
    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const int w = tid >> 6;
    uint64_t x = tid < 256 ? v : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, 64);
        if (lane >= (uint32_t)off) x += y;
    }
    if (tid < 256 && lane == 63) s_tmp[w] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < w) base += s_tmp[i];
        tot += s_tmp[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - (tid < 256 ? v : 0);
}

// (u << wb) | v, with v cut to wb bits: an id outside [0, 2^wb) then changes
// only its own field, so the key digits always agree with what the histogram
// pass counts (whichever way it counts them) and no pass writes out of range.
template <typename IdT, typename KeyT> __device__ __forceinline__ KeyT pack(IdT u, IdT v, int wb) {
    using U = typename std::conditional<sizeof(IdT) == 4, uint32_t, uint64_t>::type;
    return ((KeyT)(U)u << wb) | ((KeyT)(U)v & (((KeyT)1 << wb) - 1));
}

// Key number idx of the (optionally symmetrized) entry sequence.
template <typename IdT, typename KeyT, bool SYM>
__device__ __forceinline__ KeyT entry_key(const IdT *src, const IdT *dst, uint64_t E, uint64_t idx, int wb) {
    if (!SYM || idx < E) return pack<IdT, KeyT>(src[idx], dst[idx], wb);
    const uint64_t j = idx - E;
    return pack<IdT, KeyT>(dst[j], src[j], wb);
}

// Key of entry idx with tb origin bits below it: entries at or after `split`
// come from the second graph (origin 1).
template <typename IdT, typename KeyT, bool SYM>
__device__ __forceinline__ KeyT tagged_key(const IdT *src, const IdT *dst, uint64_t E, uint64_t idx, int wb, int tb,
                                           uint64_t split) {
    const KeyT k = entry_key<IdT, KeyT, SYM>(src, dst, E, idx, wb);
    return tb ? (KeyT)((k << 1) | (KeyT)(idx >= split ? 1u : 0u)) : k;
}

// --------------------------------------------------------------------------- prepare
struct PrepArgs {
    uint64_t E, N;
    const void *src, *dst;
    uint64_t *ghist;   // [passes][256]
    int wb, passes;    // wb: width of the destination field
    int tb;            // origin bits below the entry (XOR mode)
    uint64_t split;    // first entry of origin 1
    int dbytes;        // SYM with a whole-byte destination field: its bytes, else 0
};

template <typename IdT, typename KeyT, bool SYM>
__global__ __launch_bounds__(256) void csr_prepare(PrepArgs a) {
    // kPrepCopies interleaved copies of every histogram, lane l counting in
    // copy l mod kPrepCopies: skewed digits (one value drawn by many lanes of
    // a wave) would otherwise serialise the LDS atomics on one address.
    __shared__ uint32_t s_h[8 * kRadix * kPrepCopies];
    for (int i = threadIdx.x; i < 8 * kRadix * kPrepCopies; i += 256) s_h[i] = 0;
    __syncthreads();
    const uint32_t copy = threadIdx.x % kPrepCopies;
    const IdT *src = static_cast<const IdT *>(a.src), *dst = static_cast<const IdT *>(a.dst);
    // kPrepUnroll keys per thread are loaded before any is counted, so that
    // enough loads are in flight to cover the memory latency.
    // Every edge is read once; with SYM its reversed entry is counted too.
    const uint64_t stride = (uint64_t)gridDim.x * 256 * kPrepUnroll;
    for (uint64_t i0 = (uint64_t)blockIdx.x * 256 * kPrepUnroll + threadIdx.x; i0 < a.E; i0 += stride) {
        IdT su[kPrepUnroll], du[kPrepUnroll];
#pragma unroll
        for (int u = 0; u < kPrepUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * 256;
            su[u] = i < a.E ? src[i] : (IdT)0;
            du[u] = i < a.E ? dst[i] : (IdT)0;
        }
#pragma unroll
        for (int u = 0; u < kPrepUnroll; ++u) {
            const uint64_t i = i0 + (uint64_t)u * 256;
            if (i >= a.E) break;
            if (SYM && a.dbytes) {
                // Key byte p of (u, v) and of (v, u) together is byte p mod
                // dbytes of u plus that of v: one count per byte of each end.
                using U = typename std::conditional<sizeof(IdT) == 4, uint32_t, uint64_t>::type;
                const uint64_t uu = (U)su[u], vv = (U)du[u];
                for (int q = 0; q < a.dbytes; ++q) {
                    atomicAdd(&s_h[(q * kRadix + (uint32_t)((uu >> (8 * q)) & 255)) * kPrepCopies + copy], 1u);
                    atomicAdd(&s_h[(q * kRadix + (uint32_t)((vv >> (8 * q)) & 255)) * kPrepCopies + copy], 1u);
                }
                continue;
            }
            KeyT k = pack<IdT, KeyT>(su[u], du[u], a.wb);
            if (a.tb) k = (KeyT)((k << 1) | (KeyT)(i >= a.split ? 1u : 0u));
            for (int p = 0; p < a.passes; ++p)
                atomicAdd(&s_h[(p * kRadix + (uint32_t)((k >> (8 * p)) & 255)) * kPrepCopies + copy], 1u);
            if (SYM) {
                const KeyT kr = pack<IdT, KeyT>(du[u], su[u], a.wb);
                for (int p = 0; p < a.passes; ++p)
                    atomicAdd(&s_h[(p * kRadix + (uint32_t)((kr >> (8 * p)) & 255)) * kPrepCopies + copy], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.passes * kRadix; i += 256) {
        // (with dbytes, pass p's histogram is the byte histogram p mod dbytes)
        const int row = (SYM && a.dbytes) ? (i / kRadix) % a.dbytes * kRadix + i % kRadix : i;
        uint32_t t = 0;
#pragma unroll
        for (int c = 0; c < kPrepCopies; ++c) t += s_h[row * kPrepCopies + c];
        if (t) atomicAdd((unsigned long long *)&a.ghist[i], (unsigned long long)t);
    }
}

// Exclusive scan of every pass's digit histogram -> bucket bases.
__global__ __launch_bounds__(256) void csr_digit_bases(const uint64_t *ghist, uint64_t *gbase) {
    __shared__ uint64_t s_tmp[4];
    const int p = blockIdx.x;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan_256(ghist[p * kRadix + threadIdx.x], s_tmp, &tot);
    gbase[p * kRadix + threadIdx.x] = ex;
}

template <typename T> __global__ void fill_kernel(T *p, uint64_t n, T v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// --------------------------------------------------------------------------- onesweep pass

struct PassArgs {
    uint64_t E, N;
    const void *src, *dst;  // first pass only
    const void *in;         // later passes
    void *out;
    uint64_t *status;       // [tiles][256]
    const uint64_t *gbase;  // [256] of this pass
    const uint64_t *ghist;  // [256] of this pass: digits no entry has skip the look-back
    uint32_t *err;
    uint64_t *csc;          // column starts (BOUND passes only)
    uint8_t *cmark;         // 1 where a column start was written (BOUND passes only)
    int wb, shift;          // wb: width of the destination field
    uint32_t tag;
    int tb;                 // origin bits below the entry (first pass, XOR mode)
    uint64_t split;         // first entry of origin 1
    uint64_t nv;            // vertices (BOUND passes write column starts below it)
};

// BOUND: the input keys are ordered by destination; mark the first position
// of every destination run in csc.
template <typename IdT, typename KeyT, bool SYM, bool FIRST, bool BOUND>
__global__ __launch_bounds__(kPassThreads, BOUND ? 6 : 8) void radix_pass(PassArgs a) {
    // s_keys holds the tile's keys in digit order after ranking; during the
    // ranking its first 32 KB serve as the per-wave lane-match tables.
    __shared__ KeyT s_keys[kPassTile];
    // 16-bit per-wave digit counters (8 KB); with the 64 KB key tile the block takes about 77 KB of LDS
    // (8-byte keys): two workgroups per CU.
    __shared__ uint16_t s_cnt[kPassWaves][kRadix];
    __shared__ uint16_t s_off[kRadix];
    __shared__ uint16_t s_tot[kRadix];
    __shared__ uint64_t s_gpos[kRadix];
    __shared__ uint64_t s_tmp[4];
    static_assert(sizeof(KeyT) * kPassTile >= sizeof(uint64_t) * kPassWaves * kRadix, "match tables do not fit");
    static_assert(kPassThreads % kRadix == 0 && 64 % kLanesPerDigit == 0, "look-back lane groups");
    uint64_t *s_match = reinterpret_cast<uint64_t *>(s_keys) + 0;  // [kPassWaves][256]

    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const int w = tid >> 6;
    for (int i = tid; i < kPassWaves * kRadix; i += kPassThreads) {
        (&s_cnt[0][0])[i] = 0;
        s_match[i] = 0;
    }
    __syncthreads();
    // Tile = workgroup id.  Workgroups are dispatched in id order, so every
    // tile this one waits for in the look-back was dispatched earlier and is
    // running or done: the smallest unfinished tile never waits.  (A ticket
    // counter would serialise the tiles on one device-coherent atomic.)
    const uint64_t tile = blockIdx.x;
    const uint64_t tile_base = tile * kPassTile;
    const uint64_t wbase = tile_base + (uint64_t)w * 64 * kPassItems;
    const bool full = tile_base + kPassTile <= a.N;

    KeyT k[kPassItems];
    uint32_t d[kPassItems];
#pragma unroll
    for (int i = 0; i < kPassItems; ++i) {
        const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
        const bool valid = full || idx < a.N;
        if (FIRST)
            k[i] = valid ? tagged_key<IdT, KeyT, SYM>(static_cast<const IdT *>(a.src), static_cast<const IdT *>(a.dst),
                                                       a.E, idx, a.wb, a.tb, a.split)
                         : (KeyT)0;
        else
            k[i] = valid ? static_cast<const KeyT *>(a.in)[idx] : (KeyT)0;
        d[i] = valid ? (uint32_t)(k[i] >> a.shift) & 255u : (uint32_t)kRadix;
    }

    if (BOUND) {
        // The key before position idx: the previous lane of the same item,
        // lane 63 of the previous item, or (first key of the wave) memory.
        const KeyT mask = ((KeyT)1 << a.wb) - 1;
        const KeyT *in = static_cast<const KeyT *>(a.in);
        KeyT carry = (wbase > 0 && wbase <= a.N) ? in[wbase - 1] : (KeyT)0;
#pragma unroll
        for (int i = 0; i < kPassItems; ++i) {
            const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
            KeyT prev = __shfl_up(k[i], 1, 64);
            if (lane == 0) prev = carry;
            carry = __shfl(k[i], 63, 64);
            // (ids at or above n are not vertices: never written, never a fault)
            if (idx < a.N && (idx == 0 || (k[i] & mask) != (prev & mask)) && (uint64_t)(k[i] & mask) < a.nv) {
                a.csc[(uint64_t)(k[i] & mask)] = idx;
                a.cmark[(uint64_t)(k[i] & mask)] = 1;
            }
        }
    }

    // Stable rank inside the wave.  For each group of 64 keys every lane ORs
    // its lane bit into the wave's match slot of its digit; reading the slot
    // back gives the lanes sharing the digit (OR is order-free, so the mask
    // is exact).  Lanes below this one in the mask come first; the lowest
    // lane of each digit advances the wave's counter and clears the slot.
    // LDS operations of one wave complete in program order.
    uint32_t r[kPassItems];
    uint64_t *match = s_match + w * kRadix;
    uint16_t *wcnt = s_cnt[w];
    const uint64_t my_bit = 1ull << lane;
#pragma unroll
    for (int i = 0; i < kPassItems; ++i) {
        const uint32_t di = d[i];
        const bool valid = di < kRadix;
        const uint32_t slot = valid ? di : 0;
        if (valid) atomicOr(reinterpret_cast<unsigned long long *>(&match[slot]), (unsigned long long)my_bit);
        __builtin_amdgcn_wave_barrier();
        const uint64_t peers = valid ? match[slot] : 0ull;
        const uint32_t below = count_below(peers);
        const uint32_t old = wcnt[slot];
        r[i] = old + below;
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) {
            wcnt[slot] = (uint16_t)(old + (uint32_t)__popcll(peers));
            match[slot] = 0;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // Per digit: prefix over the waves and the tile's count.
    uint32_t cnt = 0;
    if (tid < kRadix) {
        uint32_t acc = 0;
#pragma unroll
        for (int wv = 0; wv < kPassWaves; ++wv) {
            const uint32_t c = s_cnt[wv][tid];
            s_cnt[wv][tid] = (uint16_t)acc;
            acc += c;
        }
        cnt = acc;
        s_tot[tid] = (uint16_t)acc;
    }
    __syncthreads();

    // Decoupled look-back with kLanesPerDigit consecutive lanes per digit:
    // lane q of digit d's group reads kLookWindow predecessors, so one round
    // trip covers kLanesPerDigit kLookWindow earlier tiles.  Lane 0 of the
    // group publishes: the tile's own count first, its inclusive prefix once
    // known.
    // A digit that no entry of the pass has (known from the histogram pass)
    // has a zero prefix everywhere: its lanes neither publish nor walk.  Key
    // ranges that leave digit values unused (ids below a power of the radix,
    // generators with zero cells) save that part of the status traffic.
    const uint32_t dg = (uint32_t)tid / kLanesPerDigit, part = (uint32_t)tid % kLanesPerDigit;
    const uint64_t my_cnt = s_tot[dg];
    const bool used = a.ghist[dg] != 0;
    if (part == 0 && used)
        store_agent(a.status + tile * kRadix + dg, status_word(a.tag, tile == 0 ? kFlagIncl : kFlagAgg, my_cnt));

    uint64_t tot;
    const uint64_t ex = block_exclusive_scan_256(cnt, s_tmp, &tot);
    if (tid < kRadix) s_off[tid] = (uint16_t)ex;
    __syncthreads();

    // Scatter into LDS in digit order (the local order needs no global
    // offsets, and the keys leave the registers before the look-back).
#pragma unroll
    for (int i = 0; i < kPassItems; ++i)
        if (d[i] < kRadix) s_keys[s_off[d[i]] + s_cnt[w][d[i]] + r[i]] = k[i];

    uint64_t prefix = 0;
    if (tile > 0 && used) {
        uint64_t j = tile;  // tiles below j are still to be examined
        for (;;) {
            // This lane's predecessors: j - 1 - (part kLookWindow + i).  One
            // beyond tile 0 reads as an inclusive zero, which ends the walk.
            uint64_t v[kLookWindow];
#pragma unroll
            for (int i = 0; i < kLookWindow; ++i) {
                const uint64_t back = (uint64_t)part * kLookWindow + i;
                v[i] = j > back ? load_agent(a.status + (j - 1 - back) * kRadix + dg)
                                : status_word(a.tag, kFlagIncl, 0);
            }
            uint64_t sum = 0;
            bool found = false;
#pragma unroll
            for (int i = 0; i < kLookWindow; ++i) {
                if (found) break;
                const uint64_t back = (uint64_t)part * kLookWindow + i;
                uint32_t spins = 0;
                while ((uint32_t)(v[i] >> 58) != a.tag) {
                    if (++spins > kSpinLimit || ((spins & 1023) == 0 && load_agent(a.err) != 0)) {
                        raise_device_error(a.err, DEVERR_LOOKBACK);
                        v[i] = status_word(a.tag, kFlagIncl, 0);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    v[i] = load_agent(a.status + (j - 1 - back) * kRadix + dg);
                }
                sum += v[i] & ((1ull << 56) - 1);
                found = ((v[i] >> 56) & 3) == kFlagIncl;
            }
            // Combine the group, nearest predecessors first.
            const int lead = (int)(lane & ~(uint32_t)(kLanesPerDigit - 1));
            bool done = false;
#pragma unroll
            for (int q = 0; q < kLanesPerDigit; ++q) {
                const uint64_t sq = __shfl(sum, lead + q, 64);
                const int fq = __shfl((int)found, lead + q, 64);
                if (!done) {
                    prefix += sq;
                    done = fq != 0;
                }
            }
            if (done) break;
            j -= (uint64_t)kLanesPerDigit * kLookWindow;  // else a sentinel had ended the walk
        }
        if (part == 0) store_agent(a.status + tile * kRadix + dg, status_word(a.tag, kFlagIncl, prefix + my_cnt));
    }
    if (part == 0) s_gpos[dg] = prefix;
    __syncthreads();
    if (tid < kRadix) s_gpos[tid] = a.gbase[tid] + s_gpos[tid] - ex;
    __syncthreads();

    // Write the digit runs out, coalesced.
    const uint64_t rem = a.N - tile_base;
    const uint32_t nvalid = rem < (uint64_t)kPassTile ? (uint32_t)rem : (uint32_t)kPassTile;
    KeyT *out = static_cast<KeyT *>(a.out);
    for (uint32_t p = tid; p < nvalid; p += kPassThreads) {
        const KeyT key = s_keys[p];
        const uint32_t dd = (uint32_t)(key >> a.shift) & 255u;
        // Streaming store: the next pass reads the keys back from HBM anyway.
        __builtin_nontemporal_store(key, &out[s_gpos[dd] + p]);
    }
}

// --------------------------------------------------------------------------- finish
struct FinArgs {
    uint64_t N, n;
    const void *keys;
    void *col;
    uint64_t *rp;       // row starts in output (compacted) positions, written where a row starts
    uint64_t *rp_raw;   // row starts in sorted positions, or null
    uint8_t *mark;      // 1 where a row start was written (shared by rp and rp_raw)
    uint64_t *dups;     // [1] accumulated, or null
    uint64_t *status;   // [tiles] look-back words (SIMPLE)
    uint32_t *err;
    int wb;
};

__device__ __forceinline__ int fin_slot(int i) { return i + (i >> 4); }

// Non-SIMPLE finish: one streaming pass with no LDS.  Thread t of a block
// owns positions base + j*256 + t; the key before position idx comes from the
// previous lane (or, for lane 0, from memory).
template <typename IdT, typename KeyT>
__global__ __launch_bounds__(kFinThreads) void csr_finish_plain(FinArgs a) {
    __shared__ uint32_t s_dups[kFinThreads / 64];
    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const KeyT *K = static_cast<const KeyT *>(a.keys);
    IdT *col = static_cast<IdT *>(a.col);
    const KeyT mask = ((KeyT)1 << a.wb) - 1;
    uint32_t ndup = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kFinThreads;
    for (uint64_t idx = (uint64_t)blockIdx.x * kFinThreads + tid; idx - lane < a.N; idx += stride) {
        const bool valid = idx < a.N;
        const KeyT key = valid ? K[idx] : (KeyT)0;
        KeyT prev = __shfl_up(key, 1, 64);
        if (lane == 0 && idx > 0 && valid) prev = K[idx - 1];
        if (valid) {
            __builtin_nontemporal_store((IdT)(key & mask), &col[idx]);  // streaming output
            const uint64_t row = (uint64_t)(key >> a.wb);
            if ((idx == 0 || row != (uint64_t)(prev >> a.wb)) && row < a.n) {
                a.rp[row] = idx;
                if (a.rp_raw) a.rp_raw[row] = idx;
                a.mark[row] = 1;
            }
            ndup += (idx > 0 && key == prev) ? 1u : 0u;
            if (idx == a.N - 1) {
                a.rp[a.n] = a.N;
                if (a.rp_raw) a.rp_raw[a.n] = a.N;
                a.mark[a.n] = 1;
            }
        }
    }
    if (a.dups) {
        uint32_t x = ndup;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) s_dups[tid >> 6] = x;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (int i = 0; i < kFinThreads / 64; ++i) t += s_dups[i];
            if (t) atomicAdd((unsigned long long *)a.dups, (unsigned long long)t);
        }
    }
}

// Compacting finish.  SIMPLE (XOR = false): keep the first of every run of
// equal entries unless it is a self-loop.  XOR: the keys carry an origin bit
// below the entry (0 = first graph, whose entries are distinct; 1 = second
// graph, whose entries may repeat), so the first graph's copy of a pair sorts
// first; keep one copy of a pair present in exactly one of the two graphs.
// Output positions come from a look-back scan of the kept counts.
template <typename IdT, typename KeyT, bool XOR>
__global__ __launch_bounds__(kFinThreads) void csr_finish(FinArgs a) {
    constexpr int TB = XOR ? 1 : 0;  // origin bits below the entry
    // Blocked reads (kFinItems consecutive keys per thread) would hit few LDS
    // banks across the wave; one pad slot per 16 keys spreads them.  Slot 0 holds
    // the key before the tile, the last slot the key after it.
    // The same LDS later holds the tile's kept columns in output order, so
    // the column stores are coalesced; it is sized for 8-byte elements.
    constexpr size_t kKeyBytes = (kFinTile + kFinTile / 16 + 2) * sizeof(KeyT);
    constexpr size_t kColBytes = kFinTile * sizeof(IdT);
    __shared__ uint64_t s_raw[((kKeyBytes > kColBytes ? kKeyBytes : kColBytes) + 7) / 8];
    KeyT *s_keys = reinterpret_cast<KeyT *>(s_raw);
    IdT *s_col = reinterpret_cast<IdT *>(s_raw);
    __shared__ uint64_t s_tmp[4];
    __shared__ uint64_t s_base;
    __shared__ uint32_t s_dups[kFinThreads / 64];
    const int tid = threadIdx.x;
    const uint64_t tile = blockIdx.x;  // dispatch order (see radix_pass)
    const uint64_t t0 = tile * kFinTile;
    const KeyT *K = static_cast<const KeyT *>(a.keys);
    for (int i = tid; i < kFinTile; i += kFinThreads) {
        const uint64_t idx = t0 + i;
        s_keys[fin_slot(i + 1)] = idx < a.N ? K[idx] : (KeyT)0;
    }
    if (tid == 0) {
        s_keys[0] = t0 > 0 ? K[t0 - 1] : (KeyT)0;
        s_keys[fin_slot(kFinTile + 1)] = t0 + kFinTile < a.N ? K[t0 + kFinTile] : (KeyT)0;
    }
    __syncthreads();
    const KeyT mask = ((KeyT)1 << a.wb) - 1;
    // Blocked view: thread t owns positions t*kFinItems .. (t+1)*kFinItems-1.
    uint32_t keep_bits = 0, nkeep = 0, ndup = 0;
#pragma unroll
    for (int j = 0; j < kFinItems; ++j) {
        const int p = tid * kFinItems + j;
        const uint64_t idx = t0 + p;
        if (idx < a.N) {
            const KeyT key = s_keys[fin_slot(p + 1)], prev = s_keys[fin_slot(p)];
            bool keep;
            if (XOR) {
                const KeyT pair = key >> TB, next = s_keys[fin_slot(p + 2)];
                const bool first = idx == 0 || (prev >> TB) != pair;
                const bool alone = (key & 1) != 0 || idx + 1 >= a.N || (next >> TB) != pair;
                keep = first && alone;
            } else {
                const bool dup = idx > 0 && key == prev;
                ndup += dup;
                keep = !dup && (key >> a.wb) != (key & mask);
            }
            keep_bits |= (uint32_t)keep << j;
            nkeep += keep;
        }
    }
    // Exclusive scan of kept counts over the threads, then over tiles by a
    // decoupled look-back in which the first wavefront reads 64 predecessors
    // per round trip: the nearest one with an inclusive prefix ends the walk,
    // the counts of the ones before it are added.
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan_256(nkeep, s_tmp, &tot);
    if (tid < 64) {
        const uint32_t lane = tid;
        uint64_t *st = a.status + tile;
        uint64_t prefix = 0;
        if (tile == 0) {
            if (lane == 0) store_agent(st, status_word(1, kFlagIncl, tot));
        } else {
            if (lane == 0) store_agent(st, status_word(1, kFlagAgg, tot));
            uint64_t j = tile;  // this round reads tiles j-1 .. j-64
            for (;;) {
                const bool real = j > lane;
                const uint64_t *pj = a.status + (real ? j - 1 - lane : 0);
                uint64_t v = real ? load_agent(pj) : status_word(1, kFlagIncl, 0);
                uint32_t spins = 0;
                while ((uint32_t)(v >> 58) != 1u) {
                    if (++spins > kSpinLimit || ((spins & 1023) == 0 && load_agent(a.err) != 0)) {
                        raise_device_error(a.err, DEVERR_LOOKBACK);
                        v = status_word(1, kFlagIncl, 0);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    v = load_agent(pj);
                }
                const uint64_t incl = __ballot(((v >> 56) & 3) == kFlagIncl);
                const uint32_t first = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
                uint64_t c = lane <= first ? (v & ((1ull << 56) - 1)) : 0;
                for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
                prefix += c;
                if (incl) break;
                j -= 64;  // j > 64 here: a lane past tile 0 reads an inclusive zero
            }
            if (lane == 0) store_agent(st, status_word(1, kFlagIncl, prefix + tot));
        }
        if (lane == 0) s_base = prefix;
    }
    __syncthreads();
    const uint64_t cbase = s_base + ex;
    IdT *col = static_cast<IdT *>(a.col);
    uint64_t c = cbase;
    IdT vals[kFinItems];
#pragma unroll
    for (int j = 0; j < kFinItems; ++j) {
        const int p = tid * kFinItems + j;
        const uint64_t idx = t0 + p;
        vals[j] = 0;
        if (idx < a.N) {
            const KeyT key = s_keys[fin_slot(p + 1)] >> TB, prev = s_keys[fin_slot(p)] >> TB;
            const uint64_t row = (uint64_t)(key >> a.wb);
            if ((idx == 0 || row != (uint64_t)(prev >> a.wb)) && row < a.n) {
                a.rp[row] = c;
                if (a.rp_raw) a.rp_raw[row] = idx;
                a.mark[row] = 1;
            }
            vals[j] = (IdT)(key & mask);
            c += (keep_bits >> j) & 1u;
        }
    }
    // Kept columns to LDS in output order, then coalesced stores.
    __syncthreads();  // every read of the keys is done
    uint32_t r = (uint32_t)ex;
#pragma unroll
    for (int j = 0; j < kFinItems; ++j)
        if ((keep_bits >> j) & 1u) s_col[r++] = vals[j];
    __syncthreads();
    for (uint32_t i = tid; i < (uint32_t)tot; i += kFinThreads) __builtin_nontemporal_store(s_col[i], &col[s_base + i]);
    if (a.dups) {
        uint32_t x = ndup;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((tid & 63) == 0) s_dups[tid >> 6] = x;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (int i = 0; i < kFinThreads / 64; ++i) t += s_dups[i];
            if (t) atomicAdd((unsigned long long *)a.dups, (unsigned long long)t);
        }
    }
    // The last tile closes row n: total kept = base of this tile + its kept.
    if (t0 + kFinTile >= a.N && tid == kFinThreads - 1) {
        uint64_t tail = cbase;
        for (int j = 0; j < kFinItems; ++j) tail += (keep_bits >> j) & 1u;
        a.rp[a.n] = tail;
        if (a.rp_raw) a.rp_raw[a.n] = a.N;
        a.mark[a.n] = 1;
    }
}

// --------------------------------------------------------------------------- row fill
// mark[v] = 1 where rp[v] was written (a row with an entry; rp[n] always is).
// Afterwards every rp[v] holds the value of the first marked row at or after
// v.  Values at marked rows rise with the row, so that is a reverse running
// minimum, taken per chunk of kScanChunk rows: the first marked value of every
// chunk, an exclusive reverse scan over the chunks, then the chunk itself.
// Unmarked rows are written without being read, and only the marks are
// read for them.

// Marks of rows v0 .. v0+15 (v0 a multiple of 16) as a 16-bit mask.
__device__ __forceinline__ uint32_t load_marks16(const uint8_t *mark, uint64_t v0, uint64_t n1) {
    if (v0 + 16 <= n1) {
        const uint4 m = *reinterpret_cast<const uint4 *>(mark + v0);
        const uint32_t w[4] = {m.x, m.y, m.z, m.w};
        uint32_t bits = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int b = 0; b < 4; ++b) bits |= ((w[q] >> (8 * b)) & 1u) << (4 * q + b);
        return bits;
    }
    uint32_t bits = 0;
    for (uint64_t v = v0; v < n1; ++v) bits |= (uint32_t)(mark[v] & 1u) << (uint32_t)(v - v0);
    return bits;
}

__global__ __launch_bounds__(256) void rowfill_first(const uint64_t *rp, const uint8_t *mark, uint64_t n1,
                                                     uint64_t *cfirst) {
    __shared__ uint32_t s_first;
    if (threadIdx.x == 0) s_first = ~0u;
    __syncthreads();
    constexpr int per = kScanChunk / 256;
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk;
    const uint64_t v0 = c0 + (uint64_t)threadIdx.x * per;
    const uint32_t bits = v0 < n1 ? load_marks16(mark, v0, n1) : 0u;
    if (bits) atomicMin(&s_first, (uint32_t)threadIdx.x * per + (uint32_t)__builtin_ctz(bits));
    __syncthreads();
    if (threadIdx.x == 0) cfirst[blockIdx.x] = s_first == ~0u ? kNoRow : rp[c0 + s_first];
}

// Exclusive reverse min-scan of the chunk minima (single block).
__global__ __launch_bounds__(1024) void rowfill_chunks(uint64_t *cmin, uint64_t nchunks) {
    __shared__ uint64_t s[1024];
    const uint64_t per = (nchunks + 1023) / 1024;
    const uint64_t lo = (uint64_t)threadIdx.x * per, hi = min(lo + per, nchunks);
    uint64_t m = kNoRow;
    for (uint64_t c = lo; c < hi; ++c) m = min(m, cmin[c]);
    s[threadIdx.x] = m;
    __syncthreads();
    // inclusive suffix min over threads
    for (int off = 1; off < 1024; off <<= 1) {
        uint64_t other = threadIdx.x + off < 1024 ? s[threadIdx.x + off] : kNoRow;
        __syncthreads();
        s[threadIdx.x] = min(s[threadIdx.x], other);
        __syncthreads();
    }
    uint64_t run = threadIdx.x + 1 < 1024 ? s[threadIdx.x + 1] : kNoRow;
    for (uint64_t c = hi; c > lo; --c) {
        const uint64_t x = cmin[c - 1];
        cmin[c - 1] = run;  // minimum over later chunks
        run = min(run, x);
    }
}

__global__ __launch_bounds__(256) void rowfill_apply(uint64_t *rp, const uint8_t *mark, uint64_t n1,
                                                     const uint64_t *cnext) {
    constexpr int per = kScanChunk / 256;
    // Thread t owns rows t*per .. t*per+per-1 of the chunk; the results go
    // through LDS (one pad word per `per`) so the stores are coalesced.
    __shared__ uint64_t s_out[kScanChunk + kScanChunk / per];
    __shared__ uint64_t s[256];
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk;
    const uint64_t v0 = c0 + (uint64_t)threadIdx.x * per;
    const uint32_t bits = v0 < n1 ? load_marks16(mark, v0, n1) : 0u;
    uint64_t x[per];
    uint64_t m = kNoRow;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        x[j] = ((bits >> j) & 1u) ? rp[v0 + j] : kNoRow;  // marked rows only
        m = min(m, x[j]);
    }
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint64_t other = threadIdx.x + off < 256 ? s[threadIdx.x + off] : kNoRow;
        __syncthreads();
        s[threadIdx.x] = min(s[threadIdx.x], other);
        __syncthreads();
    }
    uint64_t run = min(cnext[blockIdx.x], threadIdx.x + 1 < 256 ? s[threadIdx.x + 1] : kNoRow);
#pragma unroll
    for (int j = per - 1; j >= 0; --j) {
        run = min(run, x[j]);
        s_out[threadIdx.x * (per + 1) + j] = run;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kScanChunk; i += 256) {
        const uint64_t v = c0 + i;
        if (v < n1) rp[v] = s_out[(i / per) * (per + 1) + i % per];
    }
}

// --------------------------------------------------------------------------- degree histogram
__device__ __forceinline__ int log2_bin(uint64_t d) {
    if (d == 0) return 0;
    const int b = 64 - __clzll(d);  // floor(log2 d) + 1
    return b > 31 ? 31 : b;
}

__global__ __launch_bounds__(256) void degree_hist_kernel(const uint64_t *rp_raw, const uint64_t *csc, uint64_t n,
                                                          uint64_t *hist) {
    __shared__ uint32_t s_h[32];
    if (threadIdx.x < 32) s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += stride) {
        uint64_t deg = rp_raw[v + 1] - rp_raw[v];
        if (csc) deg += csc[v + 1] - csc[v];
        atomicAdd(&s_h[log2_bin(deg)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32 && s_h[threadIdx.x]) atomicAdd((unsigned long long *)&hist[threadIdx.x], (unsigned long long)s_h[threadIdx.x]);
}

// --------------------------------------------------------------------------- host
int bits_for(uint64_t n) {  // bits to hold ids in [0, n)
    int b = 1;
    while (b < 64 && (n - 1) >> b) ++b;
    return b;
}

struct Plan {
    uint64_t n, E, N;
    int wb, db, kb, passes, key_bytes, dpasses;
    bool sym, simple, hist, directed_hist, xor_mode;
    int tb;
    uint64_t split;
    uint64_t pass_tiles, fin_tiles, chunks;
    // workspace carving
    size_t off_keysA, off_keysB, off_status, off_ghist, off_gbase, off_indeg, off_rpraw, off_mark,
        off_cmark, off_cmin, off_fstatus, total;
};

Plan make_plan(uint64_t n, uint64_t E, int id_bytes, uint32_t flags, bool want_hist, bool xor_mode = false,
               uint64_t split = 0) {
    Plan p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.E = E;
    p.sym = flags & SFG_CSR_SYMMETRIZE;
    p.simple = (flags & SFG_CSR_SIMPLE) || xor_mode;
    p.xor_mode = xor_mode;
    p.tb = xor_mode ? 1 : 0;
    p.split = split;
    p.N = p.sym ? 2 * E : E;
    p.wb = bits_for(n);
    p.hist = want_hist;
    p.directed_hist = want_hist && !p.sym;
    // With in-degrees wanted, the destination field fills whole digits so
    // that some pass boundary leaves the keys ordered by destination.
    p.db = p.directed_hist ? 8 * ((p.wb + 7) / 8) : p.wb;
    // Symmetrized: a whole-byte destination field lets the histogram pass
    // count bytes of the two endpoints instead of every digit of both keys;
    // taken when it costs no pass and no key width.
    if (p.sym && !xor_mode) {
        const int db8 = 8 * ((p.wb + 7) / 8);
        if ((p.wb + db8 + 7) / 8 == (2 * p.wb + 7) / 8 && (p.wb + db8 <= 32) == (2 * p.wb <= 32)) p.db = db8;
    }
    p.dpasses = p.db / 8;
    p.kb = p.wb + p.db + p.tb;
    p.passes = (p.kb + 7) / 8;
    p.key_bytes = p.kb <= 32 ? 4 : 8;
    p.pass_tiles = (p.N + kPassTile - 1) / kPassTile;
    p.fin_tiles = (p.N + kFinTile - 1) / kFinTile;
    p.chunks = (n + 1 + kScanChunk - 1) / kScanChunk;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align256(bytes);
        return r;
    };
    p.off_keysA = take(p.N * p.key_bytes);
    p.off_keysB = take(p.N * p.key_bytes);
    p.off_status = take(std::max<uint64_t>(p.pass_tiles, 1) * kRadix * 8);
    p.off_ghist = take(8 * kRadix * 8);
    p.off_gbase = take(8 * kRadix * 8);
    p.off_indeg = take(p.directed_hist ? (n + 1) * 8 : 0);
    p.off_rpraw = take(want_hist && p.simple ? (n + 1) * 8 : 0);
    p.off_mark = take(n + 1);
    p.off_cmark = take(p.directed_hist ? n + 1 : 0);
    p.off_cmin = take(std::max<uint64_t>(p.chunks, 1) * 8);
    p.off_fstatus = take(p.simple ? std::max<uint64_t>(p.fin_tiles, 1) * 8 : 0);
    p.total = o;
    (void)id_bytes;
    return p;
}

int fill_grid(uint64_t n) {
    const uint64_t want = (n + 255) / 256;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)device_cu_count() * 8));
}

template <typename T> void fill(T *p, uint64_t n, T v, hipStream_t s) {
    if (n) {
        ProfScope _ps("fill", s);
        fill_kernel<T><<<fill_grid(n), 256, 0, s>>>(p, n, v);
    }
}

void row_fill(uint64_t *rp, const uint8_t *mark, uint64_t n1, uint64_t *cmin, uint64_t chunks, hipStream_t s) {
    { ProfScope _ps("csr_rowfill", s); rowfill_first<<<(int)chunks, 256, 0, s>>>(rp, mark, n1, cmin); }
    { ProfScope _ps("csr_rowfill", s); rowfill_chunks<<<1, 1024, 0, s>>>(cmin, chunks); }
    { ProfScope _ps("csr_rowfill", s); rowfill_apply<<<(int)chunks, 256, 0, s>>>(rp, mark, n1, cmin); }
}

// Zero the mark bytes of rows [0, n1) (whole 32-bit words; the workspace
// carving rounds every region up to 256 bytes).
void clear_marks(uint8_t *mark, uint64_t n1, hipStream_t s) {
    fill<uint32_t>(reinterpret_cast<uint32_t *>(mark), (n1 + 3) / 4, 0u, s);
}

template <typename IdT, typename KeyT>
int run_csr(const Plan &P, const void *src, const void *dst, uint64_t *row_ptr, void *col, uint64_t *hist,
            uint64_t *dups, char *ws, hipStream_t s) {
    uint32_t *err = device_error_word();
    KeyT *keysA = reinterpret_cast<KeyT *>(ws + P.off_keysA);
    KeyT *keysB = reinterpret_cast<KeyT *>(ws + P.off_keysB);
    uint64_t *status = reinterpret_cast<uint64_t *>(ws + P.off_status);
    uint64_t *ghist = reinterpret_cast<uint64_t *>(ws + P.off_ghist);
    uint64_t *gbase = reinterpret_cast<uint64_t *>(ws + P.off_gbase);
    uint64_t *csc = P.directed_hist ? reinterpret_cast<uint64_t *>(ws + P.off_indeg) : nullptr;
    uint64_t *rp_raw_ws = (P.hist && P.simple) ? reinterpret_cast<uint64_t *>(ws + P.off_rpraw) : nullptr;
    uint64_t *cmin = reinterpret_cast<uint64_t *>(ws + P.off_cmin);
    uint8_t *mark = reinterpret_cast<uint8_t *>(ws + P.off_mark);
    uint8_t *cmark = P.directed_hist ? reinterpret_cast<uint8_t *>(ws + P.off_cmark) : nullptr;
    uint64_t *fstatus = P.simple ? reinterpret_cast<uint64_t *>(ws + P.off_fstatus) : nullptr;

    // Clear counters, histograms and look-back words (fill kernels, so the
    // sequence stays valid under stream capture).
    fill<uint64_t>(ghist, 8 * kRadix, 0, s);
    if (P.N) fill<uint64_t>(status, P.pass_tiles * kRadix, 0, s);
    if (fstatus && P.N) fill<uint64_t>(fstatus, P.fin_tiles, 0, s);
    // Row (and column) starts are written only where a row begins and
    // flagged in the mark bytes; the row fill completes the rest.
    clear_marks(mark, P.n + 1, s);
    if (csc) {
        clear_marks(cmark, P.n + 1, s);
        fill<uint64_t>(csc + P.n, 1, P.N, s);
        fill<uint8_t>(cmark + P.n, 1, 1, s);
    }
    if (dups) fill<uint64_t>(dups, 1, 0, s);
    if (hist) fill<uint64_t>(hist, 32, 0, s);

    if (P.N > 0) {
        PrepArgs pa{P.E, P.N, src, dst, ghist, P.db, P.passes, P.tb, P.split,
                    (P.sym && !P.xor_mode && P.db % 8 == 0) ? P.db / 8 : 0};
        // Every histogram workgroup stays resident (32 KB of LDS each).
        const int pg = (int)std::max<uint64_t>(1, std::min<uint64_t>((P.E + 255) / 256,
                                                                      (uint64_t)device_cu_count() * kPrepBlocksPerCu));
        if (P.sym)
            { ProfScope _ps("csr_prepare", s); csr_prepare<IdT, KeyT, true><<<pg, 256, 0, s>>>(pa); }
        else
            { ProfScope _ps("csr_prepare", s); csr_prepare<IdT, KeyT, false><<<pg, 256, 0, s>>>(pa); }
        { ProfScope _ps("csr_digit_bases", s); csr_digit_bases<<<P.passes, 256, 0, s>>>(ghist, gbase); }

        // Ping-pong so that the last pass lands in keysA.
        for (int p = 0; p < P.passes; ++p) {
            const int remaining = P.passes - 1 - p;  // passes after this one
            KeyT *out = (remaining % 2 == 0) ? keysA : keysB;
            KeyT *in = (remaining % 2 == 0) ? keysB : keysA;
            PassArgs a{P.E, P.N, src, dst, in, out, status, gbase + p * kRadix, ghist + p * kRadix, err,
                       csc, cmark, P.db, 8 * p, (uint32_t)(p + 1), P.tb, P.split, P.n};
            const int g = (int)P.pass_tiles;
            if (csc && p == P.dpasses) {
                { ProfScope _ps("radix_pass", s); radix_pass<IdT, KeyT, false, false, true><<<g, kPassThreads, 0, s>>>(a); }
            } else if (p == 0) {
                if (P.sym)
                    { ProfScope _ps("radix_pass", s); radix_pass<IdT, KeyT, true, true, false><<<g, kPassThreads, 0, s>>>(a); }
                else
                    { ProfScope _ps("radix_pass", s); radix_pass<IdT, KeyT, false, true, false><<<g, kPassThreads, 0, s>>>(a); }
            } else {
                { ProfScope _ps("radix_pass", s); radix_pass<IdT, KeyT, false, false, false><<<g, kPassThreads, 0, s>>>(a); }
            }
        }
        FinArgs fa{P.N, P.n, keysA, col, row_ptr, P.simple ? rp_raw_ws : nullptr, mark, dups, fstatus,
                   err, P.db};
        if (P.xor_mode)
            { ProfScope _ps("csr_finish", s); csr_finish<IdT, KeyT, true><<<(int)P.fin_tiles, kFinThreads, 0, s>>>(fa); }
        else if (P.simple)
            { ProfScope _ps("csr_finish", s); csr_finish<IdT, KeyT, false><<<(int)P.fin_tiles, kFinThreads, 0, s>>>(fa); }
        else
            { ProfScope _ps("csr_finish", s); csr_finish_plain<IdT, KeyT><<<fill_grid(P.N), kFinThreads, 0, s>>>(fa); }
    } else {
        fill<uint64_t>(row_ptr + P.n, 1, 0, s);
        if (rp_raw_ws) fill<uint64_t>(rp_raw_ws + P.n, 1, 0, s);
        fill<uint8_t>(mark + P.n, 1, 1, s);
    }
    row_fill(row_ptr, mark, P.n + 1, cmin, P.chunks, s);
    if (hist) {
        const uint64_t *raw = row_ptr;
        if (rp_raw_ws) {
            row_fill(rp_raw_ws, mark, P.n + 1, cmin, P.chunks, s);
            raw = rp_raw_ws;
        }
        if (csc) row_fill(csc, cmark, P.n + 1, cmin, P.chunks, s);
        { ProfScope _ps("degree_hist", s); degree_hist_kernel<<<fill_grid(P.n), 256, 0, s>>>(raw, csc, P.n, hist); }
    }
    return check_launch("edges_to_csr");
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t edges_to_csr_workspace_bytes(uint64_t n, uint64_t num_edges, int id_bytes, uint32_t flags) {
    return sfg::csr_workspace_bytes(n, num_edges, id_bytes, flags);
}

namespace sfg {

size_t csr_workspace_bytes(uint64_t n, uint64_t num_edges, int id_bytes, uint32_t flags) {
    if (n == 0) return 0;
    return make_plan(n, num_edges, id_bytes, flags, true).total;
}

int csr_build(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes, uint32_t flags,
              uint64_t *row_ptr, void *col, uint64_t *degree_hist32, uint64_t *num_duplicates, void *workspace,
              size_t workspace_bytes, hipStream_t s, const uint64_t **raw_rows) {
    if (n == 0) return fail(SFG_EINVAL, "edges_to_csr: n must be >= 1");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "edges_to_csr: id_bytes must be 4 or 8");
    if (flags & ~(uint32_t)(SFG_CSR_SYMMETRIZE | SFG_CSR_SIMPLE)) return fail(SFG_EINVAL, "edges_to_csr: bad flags");
    if (!row_ptr) return fail(SFG_EINVAL, "edges_to_csr: row_ptr is NULL");
    if (num_edges > 0 && (!src || !dst || !col)) return fail(SFG_EINVAL, "edges_to_csr: NULL edge or col buffer");
    if (id_bytes == 4 && n - 1 > 0x7FFFFFFFull) return fail(SFG_ERANGE, "edges_to_csr: n does not fit int32 ids");
    if (n > (1ull << 32)) return fail(SFG_ERANGE, "edges_to_csr: n > 2^32 does not fit a 64-bit key");
    if (num_edges > (1ull << 54)) return fail(SFG_ERANGE, "edges_to_csr: too many edges");
    const bool sym = flags & SFG_CSR_SYMMETRIZE;
    const uint64_t N = sym ? 2 * num_edges : num_edges;
    // One workgroup per tile: a dispatch's work-item count must stay below 2^32.
    if (N > (1ull << 36)) return fail(SFG_ERANGE, "edges_to_csr: more than 2^36 entries");
    Plan P = make_plan(n, num_edges, id_bytes, flags, degree_hist32 != nullptr);
    if (P.total > 0 && !workspace) return fail(SFG_EINVAL, "edges_to_csr: workspace is NULL");
    if (workspace_bytes < P.total)
        return fail(SFG_ENOSPACE, "edges_to_csr: workspace has %zu bytes, needs %zu", workspace_bytes, P.total);
    if (!device_error_word()) return fail(SFG_EDEVICE, "edges_to_csr: no device");
    char *ws = static_cast<char *>(workspace);
    if (raw_rows) *raw_rows = (P.hist && P.simple) ? reinterpret_cast<const uint64_t *>(ws + P.off_rpraw) : row_ptr;
    if (P.key_bytes == 4) {
        if (id_bytes == 4) return run_csr<int32_t, uint32_t>(P, src, dst, row_ptr, col, degree_hist32, num_duplicates, ws, s);
        return run_csr<int64_t, uint32_t>(P, src, dst, row_ptr, col, degree_hist32, num_duplicates, ws, s);
    }
    if (id_bytes == 4) return run_csr<int32_t, uint64_t>(P, src, dst, row_ptr, col, degree_hist32, num_duplicates, ws, s);
    return run_csr<int64_t, uint64_t>(P, src, dst, row_ptr, col, degree_hist32, num_duplicates, ws, s);
}

}  // namespace sfg

namespace sfg {

size_t csr_xor_workspace_bytes(uint64_t n, uint64_t num_entries) {
    return make_plan(n, num_entries, 8, 0, false, true, 0).total;
}

int csr_xor_build(uint64_t n, uint64_t num_entries, uint64_t split, const void *src, const void *dst, int id_bytes,
                  uint64_t *row_ptr, void *col, void *workspace, size_t workspace_bytes, hipStream_t s) {
    if (n > (1ull << 31)) return fail(SFG_ERANGE, "xor: n above 2^31 does not fit the tagged key");
    Plan P = make_plan(n, num_entries, id_bytes, 0, false, true, split);
    if (workspace_bytes < P.total)
        return fail(SFG_ENOSPACE, "xor: workspace has %zu bytes, needs %zu", workspace_bytes, P.total);
    char *ws = static_cast<char *>(workspace);
    if (P.key_bytes == 4) {
        if (id_bytes == 4) return run_csr<int32_t, uint32_t>(P, src, dst, row_ptr, col, nullptr, nullptr, ws, s);
        return run_csr<int64_t, uint32_t>(P, src, dst, row_ptr, col, nullptr, nullptr, ws, s);
    }
    if (id_bytes == 4) return run_csr<int32_t, uint64_t>(P, src, dst, row_ptr, col, nullptr, nullptr, ws, s);
    return run_csr<int64_t, uint64_t>(P, src, dst, row_ptr, col, nullptr, nullptr, ws, s);
}

}  // namespace sfg

extern "C" int edges_to_csr(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes,
                            uint32_t flags, uint64_t *row_ptr, void *col, uint64_t *degree_hist32,
                            uint64_t *num_duplicates, void *workspace, size_t workspace_bytes, void *stream) {
    return csr_build(n, num_edges, src, dst, id_bytes, flags, row_ptr, col, degree_hist32, num_duplicates, workspace,
                     workspace_bytes, as_stream(stream), nullptr);
}
