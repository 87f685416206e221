// Internal interface of the per-graph statistics shared by graph_stats and
// the ensemble generator.
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime.h>

namespace sfg {

// A graph owning vertices [v0, v1) of a (possibly shared) vertex space.
// dmin = 2 ceil(2E / n); chunk0 = index of its first statistics chunk; out =
// its index in the output arrays; gid = its Philox graph id.
struct StatGraph {
    uint64_t v0, v1, dmin, chunk0;
    uint32_t out, gid;
};

uint64_t stats_chunks_of(uint64_t n);
size_t stats_scratch_bytes(uint64_t nv, uint64_t total_chunks);

// Histograms, exponents and wedge counts of `count` graphs (table on the
// device) from the raw row starts and the simple CSR (rp, col) of their
// shared nv-vertex space.  Outputs are indexed by StatGraph::out.  grid:
// workgroups of the per-chunk pass (0 = one per chunk; fewer walk the chunks
// persistently, with the same results).  Kernel launches only.
int stats_enqueue(const StatGraph *G_dev, uint32_t count, uint64_t total_chunks, uint64_t nv, const uint64_t *raw,
                  const uint64_t *rp, const void *col, int id_bytes, uint32_t samples, uint64_t seed, uint64_t *hist,
                  double *gamma, int64_t *closed, void *scratch, hipStream_t s, uint32_t grid = 0);

}  // namespace sfg
