// Kronecker edge generation (section "Parallel Kronecker (PK) method", Fig. 2).
//
// Every edge is computed independently from its index e, so one launch covers
// any range of edges and needs no communication -- the one-GPU limit of the
// paper's processor groups, which split the meta-edges of each iteration
// among processors.
//
// Sample mode: per level one 32-bit Philox word chooses a cell of the
// initiator by comparison against cumulative thresholds; the row digit goes to
// the source id and the column digit to the destination id, most significant
// level first.  The kernel is bound by integer ALU work (Philox and the
// threshold compares), not by its 2 * id_bytes of HBM writes per edge.
//
// Enumerate mode: the base-e0 digits of e select seed edges, which is exactly
// the order in which the paper's depth-first meta-edge stack emits them.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kron.hpp"

namespace sfg {
namespace {

constexpr int kBlock = 256;
// The register-path sampler's LDS (byte counters, guide and packing tables,
// about 53 KB) allows three workgroups per CU: 1,024-thread workgroups give
// it the full 32 waves per CU to hide its LDS latency with.
constexpr int kFastBlock = 1024;

}  // namespace

int build_sample_table(uint32_t n0, const float *W, SampleTable &tab) {
    const uint32_t C = n0 * n0;
    std::vector<double> run(C);
    double S = 0.0;
    for (uint32_t c = 0; c < C; ++c) {
        const double w = (double)W[c];
        if (!(w >= 0.0) || std::isinf(w)) return fail(SFG_EINVAL, "kron_generate: initiator[%u] is not finite and >= 0", c);
        S = S + w;  // left-to-right binary64 running sum
        run[c] = S;
    }
    if (!(S > 0.0) || std::isinf(S)) return fail(SFG_EINVAL, "kron_generate: initiator sums to zero or overflows");
    // thr[c] = floor(S_c / T * 2^32) for c < C-1; thr[C-1] = 2^32 (never
    // reached).  A level's 24-bit uniform U selects #{c : 256 U >= thr[c]};
    // the kernels compare the whole 32-bit word w (U in its top 24 bits) with
    // thr rounded up to a multiple of 256, which selects the same cell
    // whatever w's low byte holds.
    std::vector<uint64_t> thr(C);
    for (uint32_t c = 0; c + 1 < C; ++c) {
        const double q = run[c] / S;
        const double t = std::floor(q * 4294967296.0);
        const uint64_t t32 = t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t;
        thr[c] = std::min<uint64_t>(1ull << 32, (t32 + 255) & ~255ull);
    }
    thr[C - 1] = 1ull << 32;
    // cell(w) = #{c < C-1 : w >= thr[c]}; thresholds equal to 0 always count.
    uint32_t base = 0;
    std::vector<uint64_t> distinct;
    for (uint32_t c = 0; c + 1 < C; ++c) {
        if (thr[c] == 0) {
            ++base;
        } else if (thr[c] < (1ull << 32)) {
            if (distinct.empty() || distinct.back() != thr[c]) distinct.push_back(thr[c]);
        }
    }
    tab.nt = (uint32_t)distinct.size();
    for (uint32_t i = 0; i < tab.nt; ++i) tab.tm1[i] = (uint32_t)(distinct[i] - 1);
    for (uint32_t b = 0; b <= tab.nt; ++b) {
        // w in [v_b, v_{b+1}) (with v_0 = 0): the cell counts thresholds <= v_b.
        const uint64_t vb = b == 0 ? 0 : distinct[b - 1];
        uint32_t cell = 0;
        for (uint32_t c = 0; c + 1 < C; ++c)
            if (thr[c] <= vb) ++cell;
        if (b == 0) cell = base;
        tab.row[b] = (uint8_t)(cell / n0);
        tab.col[b] = (uint8_t)(cell % n0);
    }
    return SFG_OK;
}

namespace {

// Kernel arguments of the register path (at most 15 distinct thresholds and
// digits below 16): thresholds live in scalar registers, the bucket-to-digit
// map in two 64-bit nibble tables.
struct FastArgs {
    uint64_t num_edges;  // edges written: e_begin .. e_begin + num_edges - 1
    uint64_t e_begin;
    uint32_t key0, key1, tagword, k;
    uint32_t n0, shift;
    uint32_t tm1[15];
    uint64_t lut_row, lut_col;
    // Byte counting (ByteCount): LDS rows, flushed into hist at the end;
    // optional sort keys.
    uint64_t *hist;
    int rows, row_mod, dst_row, dst_bytes, src_row, src_bytes;
    uint64_t *keys;
    int key_shift;
    uint64_t key_sym;  // offset of the reversed entries, or 0
    uint32_t *keys32;  // 4-byte keys (packed ids only)
    int pack_groups, pack_bits;
    const uint16_t *pack_tab;  // [2^pack_bits], see ByteCount
};

constexpr int kPackTabMax = 4096;  // group values of a packing table

constexpr int kCountRows = 8;    // byte-count rows a sampler workgroup keeps in LDS
constexpr int kCountCopies = 4;  // interleaved copies of every counter

template <int NT> __device__ __forceinline__ uint32_t bucket_of(uint32_t w, const uint32_t (&t)[15]) {
    uint32_t b = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i) b += (w > t[i]) ? 1u : 0u;
    return b;
}

// Guide table over the top kGuideBits bits of a word: for every prefix the
// row digit and the column digit of the cell (two byte tables, so that each
// digit is shifted into its id by a single instruction), unless a threshold
// falls inside the prefix's range of words (kStraddle in the row byte), where
// the word is compared against the thresholds.  The bucket count is monotone
// in the word, so equal buckets at both ends of a range make the entry exact
// for every word in it.
constexpr int kGuideBits = 13;
constexpr uint32_t kGuideSize = 1u << kGuideBits;
constexpr uint32_t kStraddle = 0x80;

// With CNT the kernel also counts the bytes of the ids it writes (ByteCount in
// kron.hpp): one LDS row of 256 counters per counted byte position, added
// into the global rows once per workgroup.  The counts are exact integers, so
// the result does not depend on the order in which lanes add them.
template <typename IdT, typename AccT, bool POW2, int NT, bool CNT>
__global__ __launch_bounds__(kFastBlock) void kron_sample_fast(FastArgs a, IdT *__restrict__ src, IdT *__restrict__ dst) {
    // With few thresholds the comparisons are cheaper than the table.
    constexpr bool kGuide = NT > 3;
    __shared__ uint8_t s_guide[kGuide ? 2 * kGuideSize : 1];  // row digits | kStraddle, then column digits
    // Lane l counts in copy l mod kCountCopies: lanes of a wave that draw the
    // same byte (frequent for skewed initiators) would otherwise serialise
    // their LDS atomics on one address.
    __shared__ uint32_t s_cnt[CNT ? kCountRows * 256 * kCountCopies : 1];
    __shared__ uint8_t s_pack[CNT && POW2 ? kPackTabMax : 1];
    const uint32_t copy = threadIdx.x % kCountCopies;
    if (CNT)
        for (uint32_t i = threadIdx.x; i < kCountRows * 256 * kCountCopies; i += kFastBlock) s_cnt[i] = 0;
    if (CNT && POW2 && a.pack_groups)
        for (uint32_t i = threadIdx.x; i < (1u << a.pack_bits); i += kFastBlock) s_pack[i] = (uint8_t)a.pack_tab[i];
    if (kGuide) {
        for (uint32_t i = threadIdx.x; i < kGuideSize; i += kFastBlock) {
            const uint32_t lo = i << (32 - kGuideBits), hi = lo | ((1u << (32 - kGuideBits)) - 1u);
            const uint32_t blo = bucket_of<NT>(lo, a.tm1), bhi = bucket_of<NT>(hi, a.tm1);
            const uint32_t rd = (uint32_t)(a.lut_row >> (4 * blo)) & 15u, cd = (uint32_t)(a.lut_col >> (4 * blo)) & 15u;
            s_guide[i] = (uint8_t)(rd | (blo == bhi ? 0u : kStraddle));
            s_guide[kGuideSize + i] = (uint8_t)cd;
        }
    }
    if (kGuide || CNT) __syncthreads();
    // Levels 5 blk .. 5 blk + nlev - 1 of edge (elo, ehi) from Philox block blk.
    auto levels = [&](uint32_t elo, uint32_t ehi, uint32_t blk, uint32_t nlev, AccT &u, AccT &v) {
        const Block4 r = philox(elo, ehi, blk, a.tagword, a.key0, a.key1);
        const uint32_t ws[5] = {r.w0, r.w1, r.w2, r.w3, level4_word(r)};
        // The block's table reads go out together; the rare words whose
        // prefix holds a threshold are decoded by comparison.
        uint32_t rd[5], cd[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const uint32_t g = ws[i] >> (32 - kGuideBits);
            rd[i] = kGuide ? (uint32_t)s_guide[g] : kStraddle;
            cd[i] = kGuide ? (uint32_t)s_guide[kGuideSize + g] : 0u;
        }
        if ((rd[0] | rd[1] | rd[2] | rd[3] | rd[4]) & kStraddle) {
#pragma unroll
            for (int i = 0; i < 5; ++i)
                if (rd[i] & kStraddle) {
                    const uint32_t b = bucket_of<NT>(ws[i], a.tm1);
                    rd[i] = (uint32_t)(a.lut_row >> (4 * b)) & 15u;
                    cd[i] = (uint32_t)(a.lut_col >> (4 * b)) & 15u;
                }
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            if ((uint32_t)i < nlev) {
                if (POW2) {
                    u = (u << a.shift) | (AccT)rd[i];
                    v = (v << a.shift) | (AccT)cd[i];
                } else {
                    u = u * a.n0 + (AccT)rd[i];
                    v = v * a.n0 + (AccT)cd[i];
                }
            }
        }
    };
    // Whole blocks of five levels first (no per-level test), then the rest.
    const uint32_t full = a.k / 5, rest = a.k % 5;
    const uint64_t stride = (uint64_t)gridDim.x * kFastBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kFastBlock + threadIdx.x; i < a.num_edges; i += stride) {
        AccT u = 0, v = 0;
        const uint64_t e = a.e_begin + i;  // the edge's index in the whole graph
        const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
        for (uint32_t blk = 0; blk < full; ++blk) levels(elo, ehi, blk, 5, u, v);
        if (rest) levels(elo, ehi, full, rest, u, v);
        src[i] = (IdT)u;
        dst[i] = (IdT)v;
        if (CNT) {
            // The sort works on packed ids when packing is on, else on the ids.
            AccT ku = u, kv = v;
            if (POW2 && a.pack_groups) {
                const AccT gmask = ((AccT)1 << a.pack_bits) - 1;
                ku = 0;
                kv = 0;
                for (int j = a.pack_groups - 1; j >= 0; --j) {
                    ku = (ku << 8) | (AccT)s_pack[(uint32_t)((u >> (a.pack_bits * j)) & gmask)];
                    kv = (kv << 8) | (AccT)s_pack[(uint32_t)((v >> (a.pack_bits * j)) & gmask)];
                }
                if (a.keys32) __builtin_nontemporal_store(((uint32_t)ku << a.key_shift) | (uint32_t)kv, &a.keys32[i]);
            }
            if (a.keys) {
                __builtin_nontemporal_store(((uint64_t)ku << a.key_shift) | (uint64_t)kv, &a.keys[i]);
                if (a.key_sym)
                    __builtin_nontemporal_store(((uint64_t)kv << a.key_shift) | (uint64_t)ku, &a.keys[a.key_sym + i]);
            }
#pragma unroll
            for (int q = 0; q < (int)sizeof(AccT); ++q) {
                if (q < a.dst_bytes)
                    atomicAdd(&s_cnt[((a.dst_row + q) * 256 + (uint32_t)((kv >> (8 * q)) & 255u)) * kCountCopies + copy], 1u);
                if (q < a.src_bytes)
                    atomicAdd(&s_cnt[((a.src_row + q) * 256 + (uint32_t)((ku >> (8 * q)) & 255u)) * kCountCopies + copy], 1u);
            }
        }
    }
    if (CNT) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < (uint32_t)a.rows * 256; i += kFastBlock) {
            const uint32_t slot = ((i >> 8) % (uint32_t)a.row_mod) * 256 + (i & 255u);
            uint32_t t = 0;
#pragma unroll
            for (int c = 0; c < kCountCopies; ++c) t += s_cnt[slot * kCountCopies + c];
            if (t) atomicAdd((unsigned long long *)&a.hist[i], (unsigned long long)t);
        }
    }
}

// General path: up to 255 distinct thresholds, searched in LDS.
struct GeneralArgs {
    uint64_t num_edges, e_begin;
    uint32_t key0, key1, tagword, k;
    uint32_t n0, nt;
};

template <typename IdT, typename AccT>
__global__ __launch_bounds__(kBlock) void kron_sample_general(GeneralArgs a, SampleTable tab, IdT *__restrict__ src,
                                                              IdT *__restrict__ dst) {
    __shared__ uint32_t s_t[256];
    __shared__ uint8_t s_row[256], s_col[256];
    for (uint32_t i = threadIdx.x; i < 256; i += kBlock) {
        s_t[i] = i < a.nt ? tab.tm1[i] : 0xFFFFFFFFu;
        s_row[i] = tab.row[i];
        s_col[i] = tab.col[i];
    }
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < a.num_edges; i += stride) {
        AccT u = 0, v = 0;
        const uint64_t e = a.e_begin + i;  // the edge's index in the whole graph
        const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
        for (uint32_t blk = 0; blk * 5 < a.k; ++blk) {
            const Block4 r = philox(elo, ehi, blk, a.tagword, a.key0, a.key1);
            const uint32_t ws[5] = {r.w0, r.w1, r.w2, r.w3, level4_word(r)};
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                if (blk * 5 + i < a.k) {
                    // b = #{j : w > s_t[j]}: binary search over the padded sorted table.
                    const uint32_t w = ws[i];
                    uint32_t b = 0;
#pragma unroll
                    for (uint32_t step = 128; step > 0; step >>= 1)
                        if (w > s_t[b + step - 1]) b += step;
                    u = u * a.n0 + s_row[b];
                    v = v * a.n0 + s_col[b];
                }
            }
        }
        src[i] = (IdT)u;
        dst[i] = (IdT)v;
    }
}

// Enumerate mode.  mask holds the 0/1 seed matrix (n0 <= 64) as bits; every
// block rebuilds the row-major list of nonzero cells in LDS.
struct EnumArgs {
    uint64_t num_edges, e_begin;
    uint32_t n0, e0, k;
    // Digits are taken in base `base` = e0, or e0^2 (two levels per step,
    // through a pair table) when e0 <= 64: `steps` steps, then one single
    // level if `odd`.  magic = floor((2^32 - 1) / base); place = n0 or n0^2.
    uint32_t pair, base, steps, odd, magic, place;
    uint32_t mask[128];
};

// Edge indices below 2^32 (IdxT = uint32_t) take their digits with a
// multiply-high by `magic`: the estimate is the quotient or one less, and one
// correction step makes it exact.  AccT holds ids (uint32_t when n0^k <= 2^32).
// A thread writes kEnumRun consecutive edges: they differ only in the lowest
// digit (the first step's), so after one full decomposition each further edge
// steps that digit and looks up its pair of table entries; a carry into the
// next digit (once per `base` edges) decomposes that edge afresh.  VEC: the
// run is stored with 16-byte vector stores (outputs 16-byte aligned).
constexpr int kEnumRun = 8;

template <typename IdT, typename IdxT, typename AccT, bool VEC>
__global__ __launch_bounds__(kBlock) void kron_enumerate_kernel(EnumArgs a, IdT *__restrict__ src,
                                                                IdT *__restrict__ dst) {
    __shared__ uint16_t s_r[4096], s_c[4096];    // seed edge -> (row, column)
    __shared__ uint16_t s_r2[4096], s_c2[4096];  // pair digit hi e0 + lo -> (r_hi n0 + r_lo, ...)
    __shared__ uint32_t s_wordbase[129];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < 128; ++i) {
            s_wordbase[i] = acc;
            acc += __popc(a.mask[i]);
        }
        s_wordbase[128] = acc;
    }
    __syncthreads();
    for (uint32_t wi = threadIdx.x; wi < 128; wi += kBlock) {
        uint32_t m = a.mask[wi], idx = s_wordbase[wi];
        while (m) {
            const uint32_t bit = __ffs(m) - 1;
            m &= m - 1;
            const uint32_t cell = wi * 32 + bit;
            s_r[idx] = (uint16_t)(cell / a.n0);
            s_c[idx] = (uint16_t)(cell % a.n0);
            ++idx;
        }
    }
    __syncthreads();
    const bool pair = a.pair != 0;
    if (pair) {
        for (uint32_t D = threadIdx.x; D < a.base; D += kBlock) {
            const uint32_t hi = D / a.e0, lo = D % a.e0;
            s_r2[D] = (uint16_t)(s_r[hi] * a.n0 + s_r[lo]);
            s_c2[D] = (uint16_t)(s_c[hi] * a.n0 + s_c[lo]);
        }
        __syncthreads();
    }
    const uint16_t *tr = pair ? s_r2 : s_r, *tc = pair ? s_c2 : s_c;
    // Ids of edge e (an index of the whole graph); d0 = its lowest digit.
    auto decompose = [&](uint64_t e, AccT &u, AccT &v, uint32_t &d0) {
        IdxT rest = (IdxT)e;
        AccT pw = 1;
        u = 0;
        v = 0;
        d0 = 0;
        for (uint32_t l = 0; l < a.steps; ++l) {  // least significant digits first
            IdxT q;
            uint32_t d;
            if (sizeof(IdxT) == 4) {
                q = (IdxT)__umulhi((uint32_t)rest, a.magic);
                d = (uint32_t)rest - (uint32_t)q * a.base;
                if (d >= a.base) {
                    ++q;
                    d -= a.base;
                }
            } else {
                q = rest / a.base;
                d = (uint32_t)(rest - q * a.base);
            }
            if (l == 0) d0 = d;
            rest = q;
            u += (AccT)tr[d] * pw;
            v += (AccT)tc[d] * pw;
            pw *= a.place;
        }
        if (a.odd) {  // the most significant level; rest < e0 here
            const uint32_t d = (uint32_t)rest < 4095u ? (uint32_t)rest : 4095u;
            u += (AccT)s_r[d] * pw;
            v += (AccT)s_c[d] * pw;
        }
    };
    // Stepping needs a lowest digit that is a table step (k = 1 has none).
    const bool step = a.steps > 0;
    const uint64_t runs = (a.num_edges + kEnumRun - 1) / kEnumRun;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < runs; r += stride) {
        const uint64_t i0 = r * kEnumRun;
        IdT su[kEnumRun], sv[kEnumRun];
        AccT u, v;
        uint32_t d0;
        decompose(a.e_begin + i0, u, v, d0);
        AccT uh = u - (AccT)tr[d0], vh = v - (AccT)tc[d0];
        su[0] = (IdT)u;
        sv[0] = (IdT)v;
#pragma unroll
        for (int j = 1; j < kEnumRun; ++j) {
            if (step && d0 + 1 < a.base) {
                ++d0;
                u = uh + (AccT)tr[d0];
                v = vh + (AccT)tc[d0];
            } else {
                decompose(a.e_begin + i0 + j, u, v, d0);
                uh = u - (AccT)tr[d0];
                vh = v - (AccT)tc[d0];
            }
            su[j] = (IdT)u;
            sv[j] = (IdT)v;
        }
        if (VEC && i0 + kEnumRun <= a.num_edges) {
            constexpr int kVec = 16 / sizeof(IdT);  // ids per 16-byte store
#pragma unroll
            for (int j = 0; j < kEnumRun; j += kVec) {
                uint4 ws, wd;
                memcpy(&ws, &su[j], 16);
                memcpy(&wd, &sv[j], 16);
                *reinterpret_cast<uint4 *>(src + i0 + j) = ws;
                *reinterpret_cast<uint4 *>(dst + i0 + j) = wd;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kEnumRun; ++j)
                if (i0 + j < a.num_edges) {
                    src[i0 + j] = su[j];
                    dst[i0 + j] = sv[j];
                }
        }
    }
}

// n0^k, or 0 if it exceeds 2^64 - 1.
uint64_t upow(uint64_t b, uint32_t k) {
    uint64_t r = 1;
    for (uint32_t i = 0; i < k; ++i) {
        if (r > UINT64_MAX / b) return 0;
        r *= b;
    }
    return r;
}

int grid_for(uint64_t items) {
    const uint64_t want = (items + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)device_cu_count() * 16;
    return (int)std::max<uint64_t>(1, std::min(want, cap));
}

int grid_fast(uint64_t items) {
    const uint64_t want = (items + kFastBlock - 1) / kFastBlock;
    const uint64_t cap = (uint64_t)device_cu_count() * 4;
    return (int)std::max<uint64_t>(1, std::min(want, cap));
}

template <typename IdT, typename AccT, bool POW2, bool CNT>
void launch_fast(const FastArgs &a, uint32_t nt, void *src, void *dst, hipStream_t s) {
    const int g = grid_fast(a.num_edges);
    IdT *S = static_cast<IdT *>(src), *D = static_cast<IdT *>(dst);
    if (nt <= 3)
        { ProfScope _ps("kron_sample", s); kron_sample_fast<IdT, AccT, POW2, 3, CNT><<<g, kFastBlock, 0, s>>>(a, S, D); }
    else if (nt <= 8)
        { ProfScope _ps("kron_sample", s); kron_sample_fast<IdT, AccT, POW2, 8, CNT><<<g, kFastBlock, 0, s>>>(a, S, D); }
    else
        { ProfScope _ps("kron_sample", s); kron_sample_fast<IdT, AccT, POW2, 15, CNT><<<g, kFastBlock, 0, s>>>(a, S, D); }
}

template <typename IdT, typename AccT>
void launch_fast_any(const FastArgs &a, bool pow2, bool cnt, uint32_t nt, void *src, void *dst, hipStream_t s) {
    if (pow2 && cnt)
        launch_fast<IdT, AccT, true, true>(a, nt, src, dst, s);
    else if (pow2)
        launch_fast<IdT, AccT, true, false>(a, nt, src, dst, s);
    else if (cnt)
        launch_fast<IdT, AccT, false, true>(a, nt, src, dst, s);
    else
        launch_fast<IdT, AccT, false, false>(a, nt, src, dst, s);
}

template <bool VEC>
void launch_enumerate(const EnumArgs &a, int id_bytes, bool idx32, bool acc32, int g, void *src, void *dst,
                      hipStream_t s) {
    if (id_bytes == 4 && idx32)  // int32 ids: n0^k <= 2^31
        kron_enumerate_kernel<int32_t, uint32_t, uint32_t, VEC><<<g, kBlock, 0, s>>>(a, (int32_t *)src, (int32_t *)dst);
    else if (id_bytes == 4)
        kron_enumerate_kernel<int32_t, uint64_t, uint32_t, VEC><<<g, kBlock, 0, s>>>(a, (int32_t *)src, (int32_t *)dst);
    else if (idx32 && acc32)
        kron_enumerate_kernel<int64_t, uint32_t, uint32_t, VEC><<<g, kBlock, 0, s>>>(a, (int64_t *)src, (int64_t *)dst);
    else if (idx32)
        kron_enumerate_kernel<int64_t, uint32_t, uint64_t, VEC><<<g, kBlock, 0, s>>>(a, (int64_t *)src, (int64_t *)dst);
    else if (acc32)
        kron_enumerate_kernel<int64_t, uint64_t, uint32_t, VEC><<<g, kBlock, 0, s>>>(a, (int64_t *)src, (int64_t *)dst);
    else
        kron_enumerate_kernel<int64_t, uint64_t, uint64_t, VEC><<<g, kBlock, 0, s>>>(a, (int64_t *)src, (int64_t *)dst);
}

// Whether a ByteCount request is one the register path can take: rows inside
// the LDS table, and per-workgroup counts that fit 32 bits.
bool count_ok(const ByteCount &bc, uint64_t count, int id_bytes) {
    if (!bc.hist || bc.rows < 1 || bc.rows > kCountRows || bc.row_mod < 1 || bc.row_mod > bc.rows) return false;
    if (bc.dst_bytes < 0 || bc.src_bytes < 0 || bc.dst_bytes > id_bytes || bc.src_bytes > id_bytes) return false;
    if (bc.dst_row < 0 || bc.src_row < 0 || bc.dst_row + bc.dst_bytes > kCountRows ||
        bc.src_row + bc.src_bytes > kCountRows)
        return false;
    if ((bc.keys || bc.keys32) && (bc.key_shift < 1 || bc.key_shift > 32)) return false;
    if (bc.pack_groups && (bc.pack_groups < 1 || bc.pack_bits < 1 || bc.pack_bits > 12 || !bc.pack_tab || bc.key_sym ||
                           (1 << bc.pack_bits) > kPackTabMax))
        return false;
    const uint64_t threads = (uint64_t)grid_fast(count) * kFastBlock;
    const uint64_t per_group = (count + threads - 1) / threads * kFastBlock;
    return 2 * per_group < (1ull << 32);
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" int kron_generate(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges, int mode,
                             uint64_t seed, uint32_t graph_id, int id_bytes, void *src, void *dst, void *stream) {
    return kron_generate_range(n0, initiator, k, num_edges, 0, num_edges, mode, seed, graph_id, id_bytes, src, dst,
                               stream);
}

extern "C" int kron_generate_range(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges,
                                   uint64_t e_begin, uint64_t count, int mode, uint64_t seed, uint32_t graph_id,
                                   int id_bytes, void *src, void *dst, void *stream) {
    return sfg::kron_generate_counted(n0, initiator, k, num_edges, e_begin, count, mode, seed, graph_id, id_bytes, src,
                                      dst, as_stream(stream), nullptr, nullptr);
}

namespace sfg {

int kron_generate_counted(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges, uint64_t e_begin,
                          uint64_t count, int mode, uint64_t seed, uint32_t graph_id, int id_bytes, void *src,
                          void *dst, hipStream_t s, const ByteCount *bc, bool *counted) {
    if (counted) *counted = false;
    if (n0 < 2) return fail(SFG_EINVAL, "kron_generate: n0 must be >= 2 (got %u)", n0);
    if (k == 0) return fail(SFG_EINVAL, "kron_generate: k must be >= 1");
    if (!initiator) return fail(SFG_EINVAL, "kron_generate: initiator is NULL");
    if (mode != SFG_KRON_SAMPLE && mode != SFG_KRON_ENUMERATE) return fail(SFG_EINVAL, "kron_generate: bad mode %d", mode);
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "kron_generate: id_bytes must be 4 or 8");
    if (graph_id >= (1u << 24)) return fail(SFG_EINVAL, "kron_generate: graph_id must be < 2^24");
    if (e_begin > num_edges || count > num_edges - e_begin)
        return fail(SFG_EINVAL, "kron_generate: edges [%llu, %llu + %llu) exceed the graph's %llu",
                    (unsigned long long)e_begin, (unsigned long long)e_begin, (unsigned long long)count,
                    (unsigned long long)num_edges);
    if (count > 0 && (!src || !dst)) return fail(SFG_EINVAL, "kron_generate: NULL output buffer");
    const uint64_t nv = upow(n0, k);
    const uint64_t max_id = id_bytes == 4 ? 0x7FFFFFFFull : 0x7FFFFFFFFFFFFFFFull;
    if (nv == 0 || nv - 1 > max_id)
        return fail(SFG_ERANGE, "kron_generate: %u^%u vertices do not fit %d-byte ids", n0, k, id_bytes);
    const bool acc32 = nv <= (1ull << 32);
    const bool pow2 = (n0 & (n0 - 1)) == 0;
    uint32_t shift = 0;
    while ((1u << shift) < n0) ++shift;

    if (mode == SFG_KRON_ENUMERATE) {
        if (n0 > 64) return fail(SFG_EINVAL, "kron_generate: enumerate mode needs n0 <= 64");
        EnumArgs a;
        memset(&a, 0, sizeof(a));
        uint32_t e0 = 0;
        for (uint32_t c = 0; c < n0 * n0; ++c) {
            const float w = initiator[c];
            if (!(w >= 0.0f) || std::isinf(w)) return fail(SFG_EINVAL, "kron_generate: initiator[%u] is not finite and >= 0", c);
            if (w > 0.0f) {
                a.mask[c / 32] |= 1u << (c % 32);
                ++e0;
            }
        }
        if (e0 == 0) return fail(SFG_EINVAL, "kron_generate: the seed graph has no edge");
        const uint64_t ne = upow(e0, k);
        if (ne == 0 || ne != num_edges)
            return fail(SFG_EINVAL, "kron_generate: enumerate mode writes e0^k = %u^%u edges, num_edges is %llu", e0, k,
                        (unsigned long long)num_edges);
        if (count == 0) return SFG_OK;
        a.num_edges = count;
        a.e_begin = e_begin;
        a.n0 = n0;
        a.e0 = e0;
        a.k = k;
        const bool pair = e0 <= 64;
        a.pair = pair ? 1u : 0u;
        a.base = pair ? e0 * e0 : e0;
        a.steps = pair ? k / 2 : k;
        a.odd = pair ? (k & 1) : 0;
        a.magic = 0xFFFFFFFFu / a.base;
        a.place = pair ? n0 * n0 : n0;
        const int g = grid_for((count + kEnumRun - 1) / kEnumRun);
        const bool idx32 = ne <= (1ull << 32);
        const bool vec = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
        ProfScope _ps("kron_enumerate", s);
        if (vec)
            launch_enumerate<true>(a, id_bytes, idx32, acc32, g, src, dst, s);
        else
            launch_enumerate<false>(a, id_bytes, idx32, acc32, g, src, dst, s);
        return check_launch("kron_generate(enumerate)");
    }

    if (n0 > 16) return fail(SFG_EINVAL, "kron_generate: sample mode needs n0 <= 16");
    SampleTable tab;
    memset(&tab, 0, sizeof(tab));
    int rc = build_sample_table(n0, initiator, tab);
    if (rc != SFG_OK) return rc;
    if (count == 0) return SFG_OK;
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t tagword = TAG_KRON | (graph_id << 8);
    if (tab.nt <= 15) {
        FastArgs a;
        memset(&a, 0, sizeof(a));
        a.num_edges = count;
        a.e_begin = e_begin;
        a.key0 = key0;
        a.key1 = key1;
        a.tagword = tagword;
        a.k = k;
        a.n0 = n0;
        a.shift = shift;
        for (int i = 0; i < 15; ++i) a.tm1[i] = (uint32_t)i < tab.nt ? tab.tm1[i] : 0xFFFFFFFFu;
        for (uint32_t b = 0; b <= tab.nt; ++b) {
            a.lut_row |= (uint64_t)tab.row[b] << (4 * b);
            a.lut_col |= (uint64_t)tab.col[b] << (4 * b);
        }
        const bool cnt = bc && count_ok(*bc, count, id_bytes) && (pow2 || !bc->pack_groups);
        if (cnt) {
            a.hist = bc->hist;
            a.rows = bc->rows;
            a.row_mod = bc->row_mod;
            a.dst_row = bc->dst_row;
            a.dst_bytes = bc->dst_bytes;
            a.src_row = bc->src_row;
            a.src_bytes = bc->src_bytes;
            a.keys = bc->keys;
            a.key_shift = bc->key_shift;
            a.key_sym = bc->key_sym ? count : 0;
            if (pow2) {
                a.keys32 = bc->keys32;
                a.pack_groups = bc->pack_groups;
                a.pack_bits = bc->pack_bits;
                a.pack_tab = bc->pack_tab;
            }
        }
        if (id_bytes == 4)
            launch_fast_any<int32_t, uint32_t>(a, pow2, cnt, tab.nt, src, dst, s);
        else if (acc32)
            launch_fast_any<int64_t, uint32_t>(a, pow2, cnt, tab.nt, src, dst, s);
        else
            launch_fast_any<int64_t, uint64_t>(a, pow2, cnt, tab.nt, src, dst, s);
        if (counted) *counted = cnt;
        return check_launch("kron_generate(sample)");
    }
    GeneralArgs a;
    a.num_edges = count;
    a.e_begin = e_begin;
    a.key0 = key0;
    a.key1 = key1;
    a.tagword = tagword;
    a.k = k;
    a.n0 = n0;
    a.nt = tab.nt;
    const int g = grid_for(count);
    if (id_bytes == 4)
        { ProfScope _ps("kron_sample", s); kron_sample_general<int32_t, uint32_t><<<g, kBlock, 0, s>>>(a, tab, (int32_t *)src, (int32_t *)dst); }
    else if (acc32)
        { ProfScope _ps("kron_sample", s); kron_sample_general<int64_t, uint32_t><<<g, kBlock, 0, s>>>(a, tab, (int64_t *)src, (int64_t *)dst); }
    else
        { ProfScope _ps("kron_sample", s); kron_sample_general<int64_t, uint64_t><<<g, kBlock, 0, s>>>(a, tab, (int64_t *)src, (int64_t *)dst); }
    return check_launch("kron_generate(sample, general)");
}

}  // namespace sfg
