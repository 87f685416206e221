// Community structure: the coarse adjacency matrix of an edge list, the view
// in which the paper's community figure (Results) shows the blocks of PBA
// graphs and the communities within communities of Kronecker graphs.
//
// counts[i][j] = #{edges (u, v) : floor(u B / n) = i, floor(v B / n) = j}.
// Up to kLdsBlocks^2 cells every workgroup counts in LDS (32-bit, flushed to
// the 64-bit global counts once at the end; a workgroup never sees 2^32
// edges); larger matrices count with global atomics.  Integer counts make the
// result independent of scheduling.
#include "common.hpp"

#include <algorithm>

namespace sfg {
namespace {

constexpr int kCommThreads = 256;
constexpr uint32_t kLdsBlocks = 64;  // 4,096 cells, 16 KB of LDS

template <typename IdT, bool LDS>
__global__ __launch_bounds__(kCommThreads) void block_count(uint64_t n, uint64_t E, const IdT *src, const IdT *dst,
                                                           uint32_t B, unsigned long long *counts) {
    __shared__ uint32_t s_c[LDS ? kLdsBlocks * kLdsBlocks : 1];
    // Small matrices keep 2 or 4 interleaved copies of every cell (lane l
    // counts in copy l mod copies): the edges of a skewed graph crowd into a
    // few cells, whose LDS atomics would otherwise serialise.
    const uint32_t cells = B * B;
    const uint32_t copies = !LDS ? 1u : cells * 4 <= kLdsBlocks * kLdsBlocks ? 4u : cells * 2 <= kLdsBlocks * kLdsBlocks ? 2u : 1u;
    const uint32_t copy = threadIdx.x % copies;
    if (LDS) {
        for (uint32_t i = threadIdx.x; i < cells * copies; i += kCommThreads) s_c[i] = 0;
        __syncthreads();
    }
    // floor(u B / n) by multiply-high (magic = floor((2^64 - 1) / n); the
    // estimate is the quotient or one less, one correction step makes it exact).
    const uint64_t magic = ~0ull / n;
    auto block_of = [&](uint64_t u) -> uint32_t {
        const uint64_t x = u * B;
        uint64_t q = __umul64hi(x, magic);
        if (x - q * n >= n) ++q;
        return (uint32_t)q;
    };
    const uint64_t stride = (uint64_t)gridDim.x * kCommThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kCommThreads + threadIdx.x; e < E; e += stride) {
        const uint64_t u = (uint64_t)src[e], v = (uint64_t)dst[e];
        if (u >= n || v >= n) continue;  // not a vertex: not counted
        const uint32_t bi = block_of(u), bj = block_of(v);
        if (LDS)
            atomicAdd(&s_c[(bi * B + bj) * copies + copy], 1u);
        else
            atomicAdd(&counts[(uint64_t)bi * B + bj], 1ull);
    }
    if (LDS) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cells; i += kCommThreads) {
            uint32_t t = 0;
            for (uint32_t c = 0; c < copies; ++c) t += s_c[i * copies + c];
            if (t) atomicAdd(&counts[i], (unsigned long long)t);
        }
    }
}

__global__ void zero_counts(unsigned long long *c, uint64_t m) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) c[i] = 0;
}

template <typename IdT>
void launch(uint64_t n, uint64_t E, const void *src, const void *dst, uint32_t B, uint64_t *counts, hipStream_t s) {
    auto *c = reinterpret_cast<unsigned long long *>(counts);
    const uint64_t cells = (uint64_t)B * B;
    zero_counts<<<(int)std::min<uint64_t>((cells + 255) / 256, 4096), 256, 0, s>>>(c, cells);
    if (E == 0) return;
    const int g = (int)std::max<uint64_t>(
        1, std::min<uint64_t>((E + kCommThreads - 1) / kCommThreads, (uint64_t)device_cu_count() * 8));
    const IdT *S = static_cast<const IdT *>(src), *D = static_cast<const IdT *>(dst);
    ProfScope _ps("block_count", s);
    if (B <= kLdsBlocks)
        block_count<IdT, true><<<g, kCommThreads, 0, s>>>(n, E, S, D, B, c);
    else
        block_count<IdT, false><<<g, kCommThreads, 0, s>>>(n, E, S, D, B, c);
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" int block_matrix(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes,
                            uint32_t blocks, uint64_t *counts, void *stream) {
    if (n == 0) return fail(SFG_EINVAL, "block_matrix: n must be >= 1");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "block_matrix: id_bytes must be 4 or 8");
    if (blocks == 0 || blocks > 4096) return fail(SFG_EINVAL, "block_matrix: blocks must be in [1, 4096]");
    if (blocks > n) return fail(SFG_EINVAL, "block_matrix: more blocks than vertices");
    if (n > (1ull << 48)) return fail(SFG_ERANGE, "block_matrix: n above 2^48");
    if (!counts || (num_edges > 0 && (!src || !dst))) return fail(SFG_EINVAL, "block_matrix: NULL buffer");
    hipStream_t s = as_stream(stream);
    if (id_bytes == 4)
        launch<int32_t>(n, num_edges, src, dst, blocks, counts, s);
    else
        launch<int64_t>(n, num_edges, src, dst, blocks, counts, s);
    return check_launch("block_matrix");
}
