// Shared device and host helpers of libsfgen (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/sfgen.h"

namespace sfg {

// ----------------------------------------------------------------- host side
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int check_launch(const char *what);
hipStream_t as_stream(void *s);
int device_cu_count();

// Launch timing: while profiling is enabled (sfg_profile_enable), a
// ProfScope around a kernel launch records a pair of hipEvents on the launch
// stream (not while the stream is being captured into a graph), and
// sfg_profile_query sums their durations per kernel name.
struct ProfScope {
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
    int slot = -1;
    hipStream_t stream;
    const char *kname;
};

// CSR construction shared by edges_to_csr and the statistics entry points.
// raw_rows (optional) receives the device address of the row starts of the
// uncompacted entry list (n+1 values; inside the workspace when SIMPLE and a
// histogram are requested, else row_ptr itself).
size_t csr_workspace_bytes(uint64_t n, uint64_t num_edges, int id_bytes, uint32_t flags);
int csr_build(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes, uint32_t flags,
              uint64_t *row_ptr, void *col, uint64_t *degree_hist32, uint64_t *num_duplicates, void *workspace,
              size_t workspace_bytes, hipStream_t s, const uint64_t **raw_rows);

// CSR of the symmetric difference of two edge sets: entries [0, split) are the
// first graph (distinct pairs), entries [split, num_entries) the second (pairs
// may repeat); a pair is kept once when it is in exactly one of them.
size_t csr_xor_workspace_bytes(uint64_t n, uint64_t num_entries);
int csr_xor_build(uint64_t n, uint64_t num_entries, uint64_t split, const void *src, const void *dst, int id_bytes,
                  uint64_t *row_ptr, void *col, void *workspace, size_t workspace_bytes, hipStream_t s);

// Counter-word tags of the Philox streams.
enum : uint32_t { TAG_KRON = 1, TAG_PBA1 = 2, TAG_PBA2 = 3, TAG_WEDGE = 4 };

// Device address of the error word that kernels set when a bounded wait runs
// out (one word per device, defined in runtime.hip).
uint32_t *device_error_word();
enum : uint32_t { DEVERR_LOOKBACK = 1u, DEVERR_QUEUE = 2u, DEVERR_CHAIN = 4u };

// Bound of every inter-workgroup wait (iterations of a short sleep), about
// tens of milliseconds; a wait that runs out records a device error.
constexpr uint32_t kSpinLimit = 1u << 20;

// Round up to a multiple of 256 bytes (workspace carving granularity).
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Carves consecutive 256-byte aligned regions out of a workspace.
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T> T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += align256(count * sizeof(T));
        return p;
    }
};

// ----------------------------------------------------------------- device side

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of
// (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl increments between rounds.
struct Block4 {
    uint32_t w0, w1, w2, w3;
};

// Three-way XOR in one gfx950 instruction: v_bitop3_b32 with the truth
// table of a ^ b ^ c (0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

// The Kronecker sampler takes five 24-bit uniforms from a Philox block: the
// top 24 bits of words 0..3, and the low bytes of words 0, 1 and 2.  Each is
// used as a 32-bit word with its low 8 bits zero, so levels 0..3 read their
// word as it is (compared with thresholds that are multiples of 256, the low
// byte cannot change the cell) and level 4 reads this one.
__device__ __forceinline__ uint32_t level4_word(const Block4 &r) {
    return ((r.w0 & 255u) << 24) | ((r.w1 & 255u) << 16) | ((r.w2 & 255u) << 8);
}

// floor(U * R / 2^64): an index in [0, R) from a 64-bit uniform.
__device__ __forceinline__ uint64_t uidx64(uint64_t U, uint64_t R) { return __umul64hi(U, R); }

// floor(w * R / 2^32): an index in [0, R) from a 32-bit uniform.
__device__ __forceinline__ uint32_t uidx32(uint32_t w, uint32_t R) { return __umulhi(w, R); }

__device__ __forceinline__ uint64_t make_u64(uint32_t lo, uint32_t hi) {
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Device-coherent relaxed accesses used for inter-workgroup handshakes.
template <typename T> __device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ void store_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ T fetch_add_agent(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_device_error(uint32_t *word, uint32_t code) {
    __hip_atomic_fetch_or(word, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sfg
