// Internal interface of the Kronecker sampler shared with the ensemble
// generator.
#pragma once

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

}  // namespace sfg
