// Test-only harness: Philox4x32-10 blocks from PyTorch's independent
// implementation (ATen/core/PhiloxRNGEngine.h), used to pin the oracle's
// Philox.  The engine's seed is the 64-bit key, its subsequence the counter's
// upper 64 bits and its offset the counter's lower 64 bits; four successive
// calls return the four words of one block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>

extern "C" void torch_philox_blocks(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int count) {
    for (int i = 0; i < count; ++i) {
        const uint32_t *c = ctr + 4 * i;
        const uint32_t *k = key + 2 * i;
        const uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
        const uint64_t subseq = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
        const uint64_t offset = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
        at::philox_engine eng(seed, subseq, offset);
        for (int w = 0; w < 4; ++w) out[4 * i + w] = eng();
    }
}
