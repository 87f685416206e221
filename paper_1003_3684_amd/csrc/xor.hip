// Randomized PK by exclusive OR (PK section, randomization): the adjacency
// matrix of the deterministic Kronecker power XOR that of a random graph.
//
// The Kronecker power's e0^k edges (enumerate mode, distinct pairs) and the
// random graph's num_random uniform pair draws are laid side by side in one
// edge list; the CSR build sorts them with an origin bit below every entry
// and keeps a pair once when exactly one of the two graphs holds it (repeated
// draws are one edge of the random graph).
#include <string.h>

#include <algorithm>

#include "common.hpp"


namespace sfg {
namespace {

constexpr uint32_t TAG_RANDOM = 6;
constexpr int kXorThreads = 256;

// Draw i: Philox block (i, 0, 0, tag 6 | gid << 8); row = uidx(w0 + 2^32 w1,
// n), column = uidx(w2 + 2^32 w3, n).
template <typename IdT>
__global__ __launch_bounds__(kXorThreads) void random_pairs(uint64_t count, uint64_t n, uint32_t key0, uint32_t key1,
                                                           uint32_t tagword, IdT *src, IdT *dst) {
    const uint64_t stride = (uint64_t)gridDim.x * kXorThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kXorThreads + threadIdx.x; i < count; i += stride) {
        const Block4 r = philox((uint32_t)i, (uint32_t)(i >> 32), 0, tagword, key0, key1);
        src[i] = (IdT)uidx64(make_u64(r.w0, r.w1), n);
        dst[i] = (IdT)uidx64(make_u64(r.w2, r.w3), n);
    }
}

struct XorSizes {
    uint64_t n, epk, total;
    size_t off_src, off_dst, off_csr, bytes;
};

int xor_sizes(uint32_t n0, const float *seed_matrix, uint32_t k, uint64_t num_random, int id_bytes, XorSizes *z) {
    if (n0 < 2 || n0 > 64) return fail(SFG_EINVAL, "kron_xor_random: n0 must be in [2, 64]");
    if (k == 0) return fail(SFG_EINVAL, "kron_xor_random: k must be >= 1");
    if (!seed_matrix) return fail(SFG_EINVAL, "kron_xor_random: NULL seed matrix");
    if (id_bytes != 4 && id_bytes != 8) return fail(SFG_EINVAL, "kron_xor_random: id_bytes must be 4 or 8");
    uint64_t e0 = 0;
    for (uint32_t c = 0; c < n0 * n0; ++c) {
        if (!(seed_matrix[c] >= 0.0f) || seed_matrix[c] > 3.0e38f)
            return fail(SFG_EINVAL, "kron_xor_random: bad seed entry %u", c);
        e0 += seed_matrix[c] != 0.0f;
    }
    if (e0 == 0) return fail(SFG_EINVAL, "kron_xor_random: the seed graph has no edge");
    uint64_t n = 1, epk = 1;
    for (uint32_t l = 0; l < k; ++l) {
        if (n > (1ull << 31) / n0) return fail(SFG_ERANGE, "kron_xor_random: n0^k above 2^31");
        n *= n0;
        if (epk > (1ull << 40) / e0) return fail(SFG_ERANGE, "kron_xor_random: e0^k above 2^40");
        epk *= e0;
    }
    if (id_bytes == 4 && n - 1 > 0x7FFFFFFFull) return fail(SFG_ERANGE, "kron_xor_random: ids do not fit int32");
    if (num_random > (1ull << 40)) return fail(SFG_ERANGE, "kron_xor_random: num_random above 2^40");
    // The sort takes one workgroup per tile of entries (see edges_to_csr).
    if (epk + num_random > (1ull << 34)) return fail(SFG_ERANGE, "kron_xor_random: more than 2^34 entries");
    z->n = n;
    z->epk = epk;
    z->total = epk + num_random;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += align256(b);
        return r;
    };
    z->off_src = take(z->total * id_bytes);
    z->off_dst = take(z->total * id_bytes);
    z->off_csr = take(csr_xor_workspace_bytes(n, z->total));
    z->bytes = o;
    return SFG_OK;
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t kron_xor_random_workspace_bytes(uint32_t n0, const float *seed_matrix, uint32_t k,
                                                  uint64_t num_random, int id_bytes) {
    XorSizes z;
    return xor_sizes(n0, seed_matrix, k, num_random, id_bytes, &z) == SFG_OK ? z.bytes : 0;
}

extern "C" int kron_xor_random(uint32_t n0, const float *seed_matrix, uint32_t k, uint64_t num_random, uint64_t seed,
                               uint32_t graph_id, int id_bytes, uint64_t *row_ptr, void *col, void *workspace,
                               size_t workspace_bytes, void *stream) {
    XorSizes z;
    int rc = xor_sizes(n0, seed_matrix, k, num_random, id_bytes, &z);
    if (rc != SFG_OK) return rc;
    if (graph_id >= (1u << 24)) return fail(SFG_EINVAL, "kron_xor_random: graph_id must be < 2^24");
    if (!row_ptr || !col) return fail(SFG_EINVAL, "kron_xor_random: NULL output");
    if (!workspace) return fail(SFG_EINVAL, "kron_xor_random: workspace is NULL");
    if (workspace_bytes < z.bytes)
        return fail(SFG_ENOSPACE, "kron_xor_random: workspace has %zu bytes, needs %zu", workspace_bytes, z.bytes);
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    char *src = ws + z.off_src, *dst = ws + z.off_dst;
    rc = kron_generate(n0, seed_matrix, k, z.epk, SFG_KRON_ENUMERATE, seed, graph_id, id_bytes, src, dst, stream);
    if (rc != SFG_OK) return rc;
    if (num_random) {
        const int g = (int)std::max<uint64_t>(
            1, std::min<uint64_t>((num_random + kXorThreads - 1) / kXorThreads, (uint64_t)device_cu_count() * 8));
        const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32), tagword = TAG_RANDOM | (graph_id << 8);
        ProfScope _ps("random_pairs", s);
        if (id_bytes == 4)
            random_pairs<int32_t><<<g, kXorThreads, 0, s>>>(num_random, z.n, key0, key1, tagword,
                                                            reinterpret_cast<int32_t *>(src) + z.epk,
                                                            reinterpret_cast<int32_t *>(dst) + z.epk);
        else
            random_pairs<int64_t><<<g, kXorThreads, 0, s>>>(num_random, z.n, key0, key1, tagword,
                                                            reinterpret_cast<int64_t *>(src) + z.epk,
                                                            reinterpret_cast<int64_t *>(dst) + z.epk);
    }
    return csr_xor_build(z.n, z.total, z.epk, src, dst, id_bytes, row_ptr, col, ws + z.off_csr,
                         workspace_bytes - z.off_csr, s);
}
