// Internal interface of the batched PBA passes (used by pba_generate and by
// the ensemble generator).
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime.h>

namespace sfg {

// One PBA graph: n vertices in P partitions, m edges per vertex, inter-faction
// probability p_inter, Philox seed and graph id.  Its vertex ids are offset by
// vbase in the output (0 for a single graph); its edges follow those of the
// previous graphs of the batch.
struct PbaGraphSpec {
    uint64_t n;
    uint32_t m, P;
    double p_inter;
    uint64_t seed;
    uint32_t graph_id;
    uint64_t vbase;
};

size_t pba_batch_workspace_bytes(const PbaGraphSpec *gs, uint32_t count);
int pba_check_spec(const PbaGraphSpec &g, int id_bytes, const char *who);

// One graph with optional faction tables (pba_generate).
int pba_run_batch(const PbaGraphSpec *gs, uint32_t count, const uint32_t *faction_off, const uint32_t *faction_members,
                  int id_bytes, void *src, void *dst, void *workspace, size_t workspace_bytes, hipStream_t s);

// A batch of graphs with default factions whose device tables (pba_tables_bytes
// bytes, built on the host by pba_tables_fill) the caller has uploaded to
// dev_tables; enqueues kernel launches only.  One graph needs no tables.
size_t pba_tables_bytes(const PbaGraphSpec *gs, uint32_t count);
void pba_tables_fill(const PbaGraphSpec *gs, uint32_t count, void *host);
int pba_enqueue_batch(const PbaGraphSpec *gs, uint32_t count, int id_bytes, void *src, void *dst, void *workspace,
                      size_t workspace_bytes, const void *dev_tables, hipStream_t s);

}  // namespace sfg
