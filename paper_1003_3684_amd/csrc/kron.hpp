// Internal interface of the Kronecker sampler shared with the ensemble
// generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfg {

// Thresholds of the sample mode in the form the kernels use.  With the
// distinct cumulative thresholds v_1 < v_2 < ... (those below 2^32, v_i >= 1),
// a word w selects bucket b = #{i : w > v_i - 1}; the cell is (row[b], col[b]).
struct SampleTable {
    uint32_t nt = 0;             // number of distinct thresholds >= 1
    uint32_t tm1[255];           // v_i - 1, ascending
    uint8_t row[256], col[256];  // cell digits of bucket b
};

// Binary64 thresholds floor(S_c / T * 2^32) of a float32 initiator (n0 x n0,
// row-major); returns SFG_EINVAL for a negative, non-finite or zero matrix.
int build_sample_table(uint32_t n0, const float *W, SampleTable &tab);

// Byte counts that a sampler launch can add while it writes the ids, in place
// of a later pass that reads the edge list to count them: byte q of every
// destination id is counted in row dst_row + q (q < dst_bytes), byte q of
// every source id in row src_row + q (q < src_bytes); at the end
// hist[r * 256 + value] (uint64) gains the count of row r mod row_mod, for
// every r < rows (rows <= 8).
// With keys set, the launch also writes the 8-byte sort key of every edge
// e: keys[e] = (src << key_shift) | dst, and with key_sym also
// keys[num_edges + e] = (dst << key_shift) | src (the reversed entry of a
// symmetrized CSR).
//
// Packed ids (pack_groups > 0, power-of-two n0, no key_sym): when the ids'
// base-n0 digits only take the values 0 .. r-1 (an initiator whose last rows
// and columns are zero), every group of g digits (pack_bits = g log2(n0)
// bits of the id, least significant group first) is replaced by its base-r
// value, one byte per group (r^g <= 255): pack(id) = sum_j
// pack_tab[group_j(id)] << 8 j.  pack is increasing, so keys of packed ids
// sort exactly like keys of the ids.  The counted bytes and the keys are
// then those of the packed ids (the written src / dst stay the ids); 4-byte
// keys go to keys32.  pack_tab (device, 2^pack_bits entries) holds for every
// group value the base-r value of the smallest digit-valid group >= it (low
// byte), plus 256 when the group itself is digit-valid.
struct ByteCount {
    uint64_t *hist;
    int rows, row_mod;
    int dst_row, dst_bytes, src_row, src_bytes;
    uint64_t *keys;
    int key_shift;
    bool key_sym;
    uint32_t *keys32;
    int pack_groups, pack_bits;
    const uint16_t *pack_tab;
};

// kron_generate_range with an optional ByteCount.  *counted tells whether the
// launch counted; the register-path sampler (sample mode, at most 15
// distinct thresholds) does, the other paths leave hist untouched.
int kron_generate_counted(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges, uint64_t e_begin,
                          uint64_t count, int mode, uint64_t seed, uint32_t graph_id, int id_bytes, void *src,
                          void *dst, hipStream_t s, const ByteCount *bc, bool *counted);

}  // namespace sfg
