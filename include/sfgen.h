/*
 * sfgen -- scale-free graph generation on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library libsfgen.so.  It implements the edge generators of
 * Yoo & Henderson, "Parallel Generation of Massive Scale-Free Graphs":
 *   - the parallel Barabasi-Albert method (PBA, two-phase preferential
 *     attachment; section "Parallel Barabasi-Albert (PBA) method", Fig. 1),
 *   - the Kronecker generator (section "Parallel Kronecker (PK) method",
 *     Fig. 2), both as the deterministic Kronecker power the paper expands
 *     and as the stochastic Kronecker model it cites in Related Work,
 * plus the conversion of an edge list to compressed sparse rows with a
 * degree histogram (the degree distributions of the Results section, Fig. 3).
 *
 * Conventions shared by every entry point:
 *   - All functions have C linkage, never throw, and return an int status:
 *     SFG_OK (0) or a negative SFG_E* code.  sfg_last_error() returns a
 *     thread-local message describing the last failure on the calling thread.
 *   - Every argument is validated on the host before anything is enqueued.
 *     On error nothing is enqueued and no output is touched.
 *   - Pointers documented "device" must point to device memory of the current
 *     HIP device; "host" pointers are read before the call returns and not
 *     retained.  The caller owns every buffer.  No entry point allocates
 *     device memory: scratch space is the caller's workspace, sized by the
 *     matching *_workspace_bytes function (edges_to_csr_noalloc uses a static
 *     array of the library instead).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; faults inside kernels surface at the
 *     next synchronisation of that stream.
 *   - id_bytes selects the vertex id type of edge and CSR arrays: 4 = int32,
 *     8 = int64.  Ids are nonnegative.
 *   - Every random choice is a draw of the counter-based generator
 *     Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`; the counter is
 *     (item_lo, item_hi, x, tag | graph_id << 8).  Outputs are a pure
 *     function of the arguments: independent of stream, workspace size above
 *     the minimum, launch configuration and batching.
 *   - A kernel that waits on another workgroup does so with a bounded spin.
 *     If the bound is ever exhausted the kernel records a device error and
 *     exits instead of hanging; sfg_device_error() reports it.
 */
#ifndef SFGEN_H
#define SFGEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SFG_OK = 0,
    SFG_EINVAL = -1,   /* malformed argument                                 */
    SFG_ERANGE = -2,   /* a size or id does not fit the chosen types         */
    SFG_ENOSPACE = -3, /* workspace smaller than *_workspace_bytes           */
    SFG_EDEVICE = -4   /* the HIP runtime reported an error                  */
};

enum { SFG_KRON_SAMPLE = 0, SFG_KRON_ENUMERATE = 1 };

enum {
    SFG_CSR_SYMMETRIZE = 1u, /* add (v,u) for every (u,v)                      */
    SFG_CSR_SIMPLE = 2u      /* drop self-loops and repeated (u,v) entries      */
};

/* Message for the last failing call on this thread ("" if none). */
const char *sfg_last_error(void);

/* ABI version of this header (incremented on incompatible change). */
int sfg_abi_version(void);

/* Device-side error word: 0 if no kernel has exhausted a bounded wait since
 * the last call, else a nonzero code.  Synchronises `stream` and clears the
 * word.  Returns SFG_OK and stores the word in *code. */
int sfg_device_error(void *stream, uint32_t *code);

/* Launch timing.  While enabled, every kernel launch of the library is
 * bracketed by a pair of hipEvents recorded on its stream.
 * sfg_profile_query waits for the recorded launches of the kernel called
 * `name` and returns how many there were and their summed duration in
 * milliseconds; sfg_profile_reset forgets all records.  Launches made while
 * the stream is being captured into a graph are not timed.  Kernel names:
 * "kron_sample", "kron_enumerate", "csr_prepare", "csr_digit_bases",
 * "radix_pass", "csr_finish", "csr_rowfill", "degree_hist", "fill",
 * "pba_fill", "pba_resolve", "pba_tile_table", "pba_count", "pba_scan",
 * "pba_substitute", "stats_chunks", "stats_gamma",
 * "stats_wedge_scan", "stats_wedge", "path_level", "block_count",
 * "random_pairs", "perturb_expand", "mlp_gemm", "mlp_elementwise",
 * "mlp_adam", "mlp_round", "mlp_rows", "mlp_wgrad", "mlp_update". */
int sfg_profile_enable(int on);
int sfg_profile_reset(void);
int sfg_profile_query(const char *name, uint64_t *launches, double *total_ms);

/* ------------------------------------------------------------------------
 * kron_generate -- Kronecker graph edges (section "Parallel Kronecker (PK)
 * method": Kronecker product of adjacency matrices, Fig. 2).
 *
 * n0, initiator: host array of n0*n0 float32, row-major, finite and >= 0.
 * k:             number of Kronecker levels; vertex ids lie in [0, n0^k).
 * mode SFG_KRON_SAMPLE: the stochastic model.  Edge e draws one cell per
 *     level, most significant level first, each with probability
 *     initiator[r][c] / sum(initiator); level l takes a 24-bit uniform U
 *     from the Philox block (e, l / 5, tag 1): the top 24 bits of word
 *     (l mod 5) for l mod 5 < 4, else the low bytes of words 0, 1, 2 (most
 *     significant first).  The cell is #{c : 256 U >= floor(S_c / T * 2^32)},
 *     binary64 cumulative thresholds.
 *     Row digits make the source id, column digits the destination id.
 *     Self-loops and repeated edges are kept.  Requires n0 <= 16.
 * mode SFG_KRON_ENUMERATE: the paper's deterministic Kronecker power.  The
 *     nonzero cells of the initiator are the seed graph's e0 edges in
 *     row-major order; edge e (in [0, e0^k)) takes the base-e0 digits of e,
 *     most significant first, as the seed edge expanded at each iteration.
 *     This is the order in which the paper's meta-edge stack emits edges.
 *     num_edges must equal e0^k; requires e0 <= 4096.  seed is unused.
 * num_edges:     edges to write (sample mode: any count).
 * src, dst:      device arrays of num_edges ids each (id_bytes wide).
 * Errors: EINVAL (n0 < 2, k == 0, bad initiator, bad mode, num_edges
 * mismatch in enumerate mode, NULL buffer with num_edges > 0, graph_id >=
 * 2^24); ERANGE (n0^k - 1 exceeds the id type).
 * ---------------------------------------------------------------------- */
int kron_generate(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges, int mode,
                  uint64_t seed, uint32_t graph_id, int id_bytes, void *src, void *dst, void *stream);

/* ------------------------------------------------------------------------
 * kron_generate_range -- edges [e_begin, e_begin + count) of the graph that
 * kron_generate(n0, initiator, k, num_edges, mode, seed, graph_id, ...)
 * writes, into src[0 .. count) and dst[0 .. count).  Every edge is a
 * function of its index alone (the PK meta-edges are independent, section
 * "Parallel Kronecker (PK) method"; in sample mode the index is the Philox
 * counter), so a graph can be generated in chunks, resumed after an
 * interruption from its last finished chunk, or split across devices, and
 * the pieces equal the corresponding slices of the one-call output.
 * kron_generate is this call with e_begin = 0 and count = num_edges.
 * Errors: those of kron_generate, and EINVAL when e_begin + count exceeds
 * num_edges.
 * ---------------------------------------------------------------------- */
int kron_generate_range(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges, uint64_t e_begin,
                        uint64_t count, int mode, uint64_t seed, uint32_t graph_id, int id_bytes, void *src,
                        void *dst, void *stream);

/* ------------------------------------------------------------------------
 * pba_generate -- parallel Barabasi-Albert edges (section "Parallel
 * Barabasi-Albert (PBA) method", Fig. 1).
 *
 * The paper's processors are num_parts partitions of contiguous vertex
 * blocks: partition q holds vertices [floor(q n / P), floor((q+1) n / P)).
 * Every vertex owns m edges, so the graph has n*m edges; edge e belongs to
 * vertex e / m (src[e] = e / m).
 *
 * Phase 1 (per partition q, slot j of its local edge list A): the first s_q
 *     slots take the partitions of q's faction list in order; a later slot,
 *     with probability p_inter, takes a uniformly chosen partition outside
 *     the faction list (an inter-faction edge), else copies the partition of
 *     a uniformly chosen earlier slot.  Draw: Philox block (j, q, tag 2):
 *     word 0 against floor(p_inter * 2^32), words 1-2 as a 64-bit uniform.
 * Count exchange: c[q][l] = occurrences of l in q's list; partition l
 *     receives D_l = sum_q c[q][l] requests, divided among requesters in
 *     ascending requester order.
 * Phase 2 (per partition l): D_l endpoints chosen by preferential attachment
 *     over l's vertices, growing from a 2-vertex clique: the t-th arrival is
 *     local vertex floor(t L_l / D_l) and its endpoint is a uniform entry of
 *     the endpoint pool of all earlier edges (Philox block (t, l, tag 3)).
 * Substitution: each occurrence of l in A is replaced, in slot order, by the
 *     next endpoint of the list l sent to this requester.
 *
 * faction_off:     host, num_parts+1 offsets into faction_members, or NULL for
 *                  the default F(q) = [q].
 * faction_members: host, faction_off[num_parts] partition ids (each <
 *                  num_parts); the list of q is the concatenation of the
 *                  members of q's factions, with repetition, and must not
 *                  be empty (slot 0 has no earlier slot to copy).
 * src, dst:        device, n*m ids each.
 * workspace:       device, at least pba_workspace_bytes(n, m, num_parts,
 *                  faction_off ? faction_off[num_parts] : 0) bytes, 256-byte
 *                  aligned.  Custom faction tables are copied into it
 *                  (the call waits for that copy before returning).
 * Errors: EINVAL (m == 0, num_parts == 0 or > 4096, n < 2*num_parts,
 * p_inter outside [0,1] or NaN, bad faction table, NULL buffers, graph_id >=
 * 2^24); ERANGE (n*m or n-1 do not fit, a partition holds >= 2^31 slots,
 * n*m*ceil(n/P) >= 2^64); ENOSPACE.  A partition that receives >= 2^31
 * requests is detected on the device (sfg_device_error).
 * ---------------------------------------------------------------------- */
size_t pba_workspace_bytes(uint64_t n, uint32_t m, uint32_t num_parts, uint64_t num_faction_members);
int pba_generate(uint64_t n, uint32_t m, uint32_t num_parts, double p_inter, const uint32_t *faction_off,
                 const uint32_t *faction_members, uint64_t seed, uint32_t graph_id, int id_bytes, void *src,
                 void *dst, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * edges_to_csr -- compressed sparse rows of an edge list.
 *
 * The entries (src[e], dst[e]) -- plus (dst[e], src[e]) with
 * SFG_CSR_SYMMETRIZE, so a self-loop appears twice -- are sorted ascending by
 * (row, column).  With SFG_CSR_SIMPLE, self-loops are dropped and repeated
 * entries are kept once.  row_ptr[v] = number of kept entries with row < v
 * (n+1 values); col holds the kept entries' columns in sorted order.
 *
 * n:               vertex count; every id must be < n.
 * row_ptr:         device, n+1 uint64.
 * col:             device, capacity num_edges (2*num_edges with SYMMETRIZE)
 *                  ids of id_bytes; with SIMPLE only row_ptr[n] are written.
 * degree_hist32:   device [32] uint64 or NULL.  Histogram of the degree
 *                  deg(v) = #{e : src[e] = v} + #{e : dst[e] = v} of the
 *                  input edge list: bin 0 counts degree 0, bin b (1..31)
 *                  counts 2^(b-1) <= deg < 2^b, degrees >= 2^30 go to bin 31.
 * num_duplicates:  device [1] uint64 or NULL: number of sorted positions
 *                  (before SIMPLE removal) whose entry equals the previous
 *                  one.
 * workspace:       device, edges_to_csr_workspace_bytes(...) bytes.
 * Errors: EINVAL (n == 0, bad flags, NULL buffers); ERANGE (ids or sizes do
 * not fit: n > 2^32, more than 2^34 entries -- edges, doubled when
 * symmetrized); ENOSPACE.  Ids outside [0, n) are not detected (the caller's
 * contract): the output is then unspecified, but no kernel writes or reads
 * outside the buffers on their account.
 * The sort's passes wait on earlier workgroups of the same launch (decoupled
 * look-back), which relies on the pass being the only such kernel on the
 * GPU: calls that sort (edges_to_csr, edges_to_csr_noalloc,
 * kron_generate_csr, graph_stats, kron_xor_random, ensemble_generate*) must
 * not overlap in time on one device, e.g. on two streams.  Their waits are
 * bounded: an overlap is reported through sfg_device_error, never a hang.
 * ---------------------------------------------------------------------- */
size_t edges_to_csr_workspace_bytes(uint64_t n, uint64_t num_edges, int id_bytes, uint32_t flags);
int edges_to_csr(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes, uint32_t flags,
                 uint64_t *row_ptr, void *col, uint64_t *degree_hist32, uint64_t *num_duplicates,
                 void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * edges_to_csr_noalloc -- edges_to_csr for callers that cannot allocate
 * device memory or pass a workspace: code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.
 *
 * Same arguments, outputs and errors as edges_to_csr, without the workspace:
 * the scratch space is a static device array of the library,
 * edges_to_csr_noalloc_max_bytes() bytes (64 MiB) per device, held from the
 * first use on that device until the process ends.  The call allocates
 * nothing (with launch timing off: sfg_profile_enable creates its timing
 * events on demand).  A problem whose edges_to_csr_workspace_bytes exceeds
 * the array fails with ERANGE before anything is enqueued (e.g. 1.5 M edges
 * over 2^20 vertices fit with every flag).  Every call on one device shares
 * that device's array and finds the last call's contents there (the call
 * clears what it needs): calls that overlap in time on one device -- on two
 * streams, or from two host threads without ordering -- race and must not be
 * made.
 * ---------------------------------------------------------------------- */
size_t edges_to_csr_noalloc_max_bytes(void);
int edges_to_csr_noalloc(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes,
                         uint32_t flags, uint64_t *row_ptr, void *col, uint64_t *degree_hist32,
                         uint64_t *num_duplicates, void *stream);

/* ------------------------------------------------------------------------
 * kron_generate_csr -- a Kronecker graph and its CSR in one call (the PK
 * method's generation, section "Parallel Kronecker (PK) method", followed by
 * the adjacency build of the Results section's analyses).
 *
 * Equivalent to kron_generate(n0, initiator, k, num_edges, mode, seed,
 * graph_id, id_bytes, src, dst, stream) followed by edges_to_csr(n0^k,
 * num_edges, src, dst, id_bytes, flags, row_ptr, col, degree_hist32,
 * num_duplicates, workspace, workspace_bytes, stream): every output, src and
 * dst included, is bit-identical to that pair's.  The difference is where the
 * sort's digit histogram is counted: when the CSR key's digits are whole
 * bytes of the ids (always with degree_hist32, else when bits(n0^k - 1) is a
 * multiple of 8; symmetrized, when edges_to_csr takes its whole-byte
 * destination field) and the sampler is the register path (sample mode, at
 * most 15 distinct initiator thresholds), the sampler counts the bytes of
 * the ids it writes, and the pass that would read the edge list back to
 * count them is skipped; with 8-byte sort keys it also writes every entry's
 * key into the workspace, so the first sort pass reads one key per entry
 * instead of both ids.  Otherwise the call runs the two steps unchanged.
 *
 * Arguments: those of kron_generate and edges_to_csr, with n = n0^k, which
 * must not exceed 2^32.  src and dst are outputs here (device, num_edges ids
 * each); the workspace is edges_to_csr_workspace_bytes(n0^k, num_edges,
 * id_bytes, flags) bytes and must not overlap src, dst or the outputs.
 * Errors: those of both calls, found before anything is launched.
 * ---------------------------------------------------------------------- */
int kron_generate_csr(uint32_t n0, const float *initiator, uint32_t k, uint64_t num_edges, int mode, uint64_t seed,
                      uint32_t graph_id, int id_bytes, void *src, void *dst, uint32_t flags, uint64_t *row_ptr,
                      void *col, uint64_t *degree_hist32, uint64_t *num_duplicates, void *workspace,
                      size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * graph_stats -- statistics of one edge list, as the paper characterises its
 * graphs (Results: degree distributions with fitted exponents, Fig. 3).
 *
 * degree_hist32: device [32] uint64, the histogram of edges_to_csr of
 *                deg(v) = out + in degree (a self-loop adds 2).
 * gamma:         device [1] double: the discrete power-law maximum-likelihood
 *                estimate of Clauset, Shalizi & Newman (2009),
 *                1 + N_t / sum_{d >= d_min} ln(d / (d_min - 1/2)) with
 *                d_min = 2 ceil(2E / n); NaN when no vertex reaches d_min.
 *                Summed in a fixed order: identical on every run and device.
 * closed:        device [1] int64: among num_samples wedges of the simple
 *                undirected graph (symmetrized, self-loops and repeats
 *                removed) -- centre v drawn with probability proportional to
 *                C(deg v, 2) from Philox block (i, 0, 0, tag 4), two distinct
 *                neighbours uniform -- the number whose ends are adjacent;
 *                -1 if the graph has no wedge.
 * workspace:     device, graph_stats_workspace_bytes(n, num_edges, id_bytes).
 * Errors: as edges_to_csr, plus EINVAL for NULL outputs or graph_id >= 2^24.
 * ---------------------------------------------------------------------- */
size_t graph_stats_workspace_bytes(uint64_t n, uint64_t num_edges, int id_bytes);
int graph_stats(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes, uint32_t num_samples,
                uint64_t seed, uint32_t graph_id, uint64_t *degree_hist32, double *gamma, int64_t *closed,
                void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * path_stats -- sampled shortest-path statistics (Results, Table 2: average
 * path length and diameter, both estimated by sampling).
 *
 * Breadth-first searches over the graph in CSR form from each given source:
 * out[0] = sum of d(s, v), out[1] = number of pairs, both over all sources s
 * and all vertices v != s reachable from s; out[2] = the largest such d (the
 * diameter estimate).  The average path length is out[0] / out[1].  Each
 * level looks at the neighbours listed in the CSR, so the CSR must be
 * symmetric (an undirected graph, e.g. edges_to_csr with
 * SFG_CSR_SYMMETRIZE | SFG_CSR_SIMPLE); repeated sources count once each.
 *
 * n, row_ptr:    device, n + 1 row starts (u64).
 * col:           device, row_ptr[n] ids (id_bytes wide), each < n.
 * sources:       host, num_sources vertex ids in [0, n) (the sample; read
 *                before the call returns).
 * out:           device, 3 u64.
 * workspace:     device, path_stats_workspace_bytes(n) (32 B per vertex).
 * The call searches 64 sources at a time and waits for the stream after
 * every level to decide whether the search is over, so it returns with the
 * work done.
 * Errors: EINVAL (n == 0, bad id_bytes, NULL buffers, a source outside
 * [0, n)); ENOSPACE.
 * ---------------------------------------------------------------------- */
size_t path_stats_workspace_bytes(uint64_t n);
int path_stats(uint64_t n, const uint64_t *row_ptr, const void *col, int id_bytes, const int64_t *sources,
               uint32_t num_sources, uint64_t *out, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * kron_perturbed -- randomized PK by temporary seed modification (PK section,
 * randomization: meta-edges added or deleted in the replacement phase of
 * every iteration by modifying the seed graph temporarily).
 *
 * The expansion of enumerate mode (nonzero entries of seed_matrix are the
 * seed's edges, iteration 1 is the seed itself), except that each meta-edge
 * (iteration i < k, row, col) is replaced by the edges of its own copy of the
 * seed in which an absent cell c is added with probability p_add and a
 * present cell deleted with probability p_del: word c mod 4 of Philox block
 * (row, col, i | (c / 4) << 8, tag 7 | graph_id << 8), compared as u64 with
 * floor(p 2^32).  Edges come out in the paper's meta-edge stack order (cell
 * order within every expansion, recursively); with p_add = p_del = 0 this is
 * kron_generate's enumerate mode entry for entry.
 *
 * n0 <= 8, n0^k <= 2^32.  capacity bounds the edges of every iteration (the
 * output arrays and the workspace are sized by it); an iteration above it
 * fails with ENOSPACE.  *num_edges (device u64) receives the edge count.
 * The call waits for the stream after every iteration (the next size comes
 * from the device).
 * workspace: device, kron_perturbed_workspace_bytes(capacity) (32 B per edge).
 * Errors: EINVAL (n0 outside [2, 8], k == 0, probabilities outside [0, 1],
 * bad seed entry or no edge, bad id_bytes, graph_id >= 2^24, NULL buffers);
 * ERANGE (n0^k > 2^32, k > 255, ids beyond int32 with id_bytes 4); ENOSPACE.
 * ---------------------------------------------------------------------- */
size_t kron_perturbed_workspace_bytes(uint64_t capacity);
int kron_perturbed(uint32_t n0, const float *seed_matrix, uint32_t k, double p_add, double p_del, uint64_t seed,
                   uint32_t graph_id, int id_bytes, uint64_t capacity, void *src, void *dst, uint64_t *num_edges,
                   void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * kron_xor_random -- randomized PK (PK section, randomization): the
 * adjacency matrix of the deterministic Kronecker power XOR that of a random
 * graph.
 *
 * The Kronecker power is kron_generate's enumerate mode on the 0/1 seed
 * (nonzero entries of seed_matrix are its edges): e0^k distinct pairs over
 * n = n0^k vertices.  The random graph is the set of distinct pairs among
 * num_random draws; draw i is Philox block (i, 0, 0, tag 6 | graph_id << 8),
 * row = uidx(w0 + 2^32 w1, n), column = uidx(w2 + 2^32 w3, n).  The result
 * holds every pair that is an edge of exactly one of the two graphs, as CSR
 * with columns ascending within each row; row_ptr[n] is its edge count.
 *
 * seed_matrix: host, n0 * n0 float32 (only zero / nonzero matters), n0 <= 64.
 * row_ptr:     device, n + 1 u64.
 * col:         device, room for e0^k + num_random ids (id_bytes wide).
 * workspace:   device, kron_xor_random_workspace_bytes(...).
 * Errors: EINVAL (n0 outside [2, 64], k == 0, a negative / NaN / infinite
 * entry, no edge in the seed, bad id_bytes, NULL buffers, graph_id >= 2^24);
 * ERANGE (n0^k > 2^31, e0^k or num_random > 2^40, e0^k + num_random > 2^34,
 * ids beyond int32 with id_bytes 4); ENOSPACE.  kron_xor_random_workspace_bytes returns 0 for
 * arguments that would be rejected.
 * ---------------------------------------------------------------------- */
size_t kron_xor_random_workspace_bytes(uint32_t n0, const float *seed_matrix, uint32_t k, uint64_t num_random,
                                       int id_bytes);
int kron_xor_random(uint32_t n0, const float *seed_matrix, uint32_t k, uint64_t num_random, uint64_t seed,
                    uint32_t graph_id, int id_bytes, uint64_t *row_ptr, void *col, void *workspace,
                    size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * block_matrix -- the coarse adjacency matrix of an edge list, the view in
 * which the paper shows community structure (Results, community figure:
 * blocks in PBA graphs, communities within communities in Kronecker graphs).
 *
 * counts[i * blocks + j] = number of edges (u, v) with floor(u blocks / n) = i
 * and floor(v blocks / n) = j.  Edges with an endpoint outside [0, n) are not
 * counted.
 * src, dst: device, num_edges ids each (id_bytes wide).
 * counts:   device, blocks * blocks u64, overwritten.
 * Errors: EINVAL (n == 0, bad id_bytes, blocks == 0, blocks > 4096,
 * blocks > n, NULL buffers); ERANGE (n > 2^48).
 * ---------------------------------------------------------------------- */
int block_matrix(uint64_t n, uint64_t num_edges, const void *src, const void *dst, int id_bytes, uint32_t blocks,
                 uint64_t *counts, void *stream);

/* ------------------------------------------------------------------------
 * ensemble_generate -- a batched ensemble of graphs (PBA and Kronecker
 * members of uneven size and parameters), each summarised by graph_stats
 * (the degree distributions and fitted exponents of the Results section,
 * Fig. 3, for thousands of graphs at once).
 *
 * Member i equals the single-graph call with the same parameters and graph
 * id: pba_generate(n, m, num_parts, p_inter, NULL, NULL, seed, graph_id, ...)
 * or kron_generate(n0, initiator, k, num_edges, SFG_KRON_SAMPLE, seed,
 * graph_id, ...), followed by graph_stats(..., num_samples, stat_seed,
 * graph_id, ...).  Its outputs go to degree_hist32[32 i .. 32 i + 31],
 * gamma[i] and closed[i] (device arrays of count entries), bit for bit the
 * single-graph results, whatever the tuning.
 *
 * Members are processed in batches cut greedily, in descriptor order, at
 * max_batch_edges edges or 2^24 vertices, whichever comes first (a single
 * member above either limit is a batch of its own): a batch shares one vertex
 * space and edge list and goes through each generation, sort and statistics
 * kernel once.  All batches run on `stream`, one after another.  The tables
 * of every batch are built on the host and uploaded in one copy at the start
 * (the call waits for it; descs is read before the call returns); the
 * batches are then kernel launches only.  ensemble_generate uses the default
 * tuning (grid_per_cu 8, kron_items 8, SFG_ENSEMBLE_GRAPH).
 * Kronecker members need n0 <= 4 and n0^k <= 2^32; PBA members use the
 * default factions.
 * workspace: device, ensemble_workspace_bytes(descs, count, max_batch_edges).
 * Errors: EINVAL / ERANGE as the single-graph calls, EINVAL for a bad tuning,
 * ENOSPACE.
 * ---------------------------------------------------------------------- */
enum { SFG_GRAPH_PBA = 0, SFG_GRAPH_KRON = 1 };

typedef struct {
    int32_t kind;         /* SFG_GRAPH_PBA or SFG_GRAPH_KRON          */
    uint32_t graph_id;    /* < 2^24                                    */
    uint64_t seed;        /* Philox key of the member's generation     */
    uint64_t n;           /* PBA: vertices                             */
    uint32_t m;           /* PBA: edges per vertex                     */
    uint32_t num_parts;   /* PBA: partitions                           */
    double p_inter;       /* PBA: inter-faction probability            */
    uint32_t n0;          /* Kronecker: initiator side (2..4)          */
    uint32_t k;           /* Kronecker: levels                         */
    uint64_t num_edges;   /* Kronecker: sampled edges                  */
    float initiator[16];  /* Kronecker: n0*n0 weights, row-major       */
} sfg_graph_desc;

size_t ensemble_workspace_bytes(const sfg_graph_desc *descs, uint32_t count, uint64_t max_batch_edges);
int ensemble_generate(const sfg_graph_desc *descs, uint32_t count, uint32_t num_samples, uint64_t stat_seed,
                      uint64_t max_batch_edges, uint64_t *degree_hist32, double *gamma, int64_t *closed,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Tuning of ensemble_generate_tuned (the choices of the autotuner; no choice
 * changes any result):
 *   max_batch_edges  the chunk schedule: the batch edge budget (>= 1);
 *   grid_per_cu      workgroups per compute unit of the persistent generation
 *                    and statistics kernels, which walk the batch's (member,
 *                    tile) table (1 .. 64);
 *   kron_items       edges per thread of a Kronecker sampling tile (4, 8 or
 *                    16; a tile is 256 threads);
 *   flags            SFG_ENSEMBLE_GRAPH: the batch sequence is captured once
 *                    into a HIP graph (on a library stream of default
 *                    priority) and launched on `stream` as one graph; the
 *                    graph is cached for the same descriptors, samples, seed,
 *                    tuning, workspace and outputs (eight per process, least
 *                    recently used dropped), so later identical calls replay
 *                    it.  If capture fails the sequence is enqueued directly. */
enum { SFG_ENSEMBLE_GRAPH = 1u };

typedef struct {
    uint64_t max_batch_edges;
    uint32_t grid_per_cu;
    uint32_t kron_items;
    uint32_t flags;
} sfg_ensemble_tuning;

int ensemble_generate_tuned(const sfg_graph_desc *descs, uint32_t count, uint32_t num_samples, uint64_t stat_seed,
                            const sfg_ensemble_tuning *tuning, uint64_t *degree_hist32, double *gamma,
                            int64_t *closed, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * MLP surrogate -- maps generator parameters to graph statistics; trained on
 * ensembles of generated graphs and inverted to choose parameters for a
 * target degree exponent (the generated graph, not the surrogate, decides
 * whether a result is accepted).
 *
 * Shape: d_in -> width -> ... -> width -> d_out with `hidden` SiLU layers
 * and a linear output layer.  params: device float32, for each layer W
 * (out x in, row-major) then b (out); mlp_param_count gives its length.
 * Every GEMM reads bfloat16 weights and inputs (round to nearest even) and
 * accumulates in float32 on the matrix cores; biases, activations and
 * gradients are float32.  Rounding points: Xb_0 = bf16(x); Z = Xb Wb^T + b;
 * next Xb = bf16(SiLU(Z)); backward dZb = bf16(dZ), dW = dZb^T Xb,
 * db = column sums of dZ, dH = dZb Wb.
 * workspace: device, mlp_workspace_bytes(shape, batch); mlp_forward leaves
 * the activations there for the following mlp_backward on the same batch.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t d_in, width, d_out, hidden;
} sfg_mlp_shape;

size_t mlp_param_count(const sfg_mlp_shape *shape);
size_t mlp_workspace_bytes(const sfg_mlp_shape *shape, uint32_t batch);
/* y: device [batch][d_out] from x: device [batch][d_in]. */
int mlp_forward(const sfg_mlp_shape *shape, uint32_t batch, const float *params, const float *x, float *y,
                void *workspace, size_t workspace_bytes, void *stream);
/* grad (device, param count; nullable) and dx (device [batch][d_in]; nullable,
 * the gradient with respect to x, passed straight through the input rounding)
 * from dy = dLoss/dy. */
int mlp_backward(const sfg_mlp_shape *shape, uint32_t batch, const float *params, const float *dy, float *grad,
                 float *dx, void *workspace, size_t workspace_bytes, void *stream);
/* loss = sum_{b,j} w_j mask_bj (y_bj - t_bj)^2 / batch and dy = dloss/dy;
 * mask [batch][d_out] and col_weight [d_out] are nullable (ones); loss is a
 * device float; workspace holds batch floats. */
int mlp_mse_grad(uint32_t batch, uint32_t d_out, const float *y, const float *target, const float *mask,
                 const float *col_weight, float *dy, float *loss, void *workspace, size_t workspace_bytes,
                 void *stream);
/* Adam (Kingma & Ba) with bias correction; step counts from 1. */
int adam_step(uint64_t count, float *params, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
              float eps, uint32_t step, void *stream);

/* The same update with the learning rate and the step counter in device
 * memory: the call first increments *step (device uint32, the number of
 * steps taken so far) and then applies step *step with learning rate *lr
 * (device float), so that a training step can be captured once into a HIP
 * graph and replayed while the schedule changes.  Bias corrections use the
 * device powf, so results may differ in the last bit from adam_step. */
int adam_step_device(uint64_t count, float *params, const float *grad, float *m, float *v, const float *lr,
                     float beta1, float beta2, float eps, uint32_t *step, void *stream);

/* One whole training step in four kernel launches: the forward pass, the
 * weighted squared-error loss and its gradient, the backward pass and Adam
 * (with the learning rate and the step counter in device memory, as
 * adam_step_device), with the rounding points above.  The first launch
 * rounds the weights to bfloat16 (row-major and transposed); the second
 * runs, for every block of 64 rows, the forward pass, the loss gradient and
 * the chain of activation gradients on the matrix cores with the layer
 * operand in LDS; the third computes every weight-gradient tile over each
 * 256-row slice of the batch on the matrix cores; the fourth sums the
 * slices and the per-block bias sums in a fixed order and applies Adam.
 * Results equal mlp_forward, mlp_mse_grad, mlp_backward and adam_step_device
 * up to the float32 summation order.
 * x, target, mask: device [rows of the data][d_in or d_out]; row r of the
 *   batch is row rows[r] of them (rows: device int64 [batch], or NULL for
 *   row r), so a shuffled batch needs no gather; mask and col_weight
 *   nullable (ones).
 * loss:  device float, the batch's loss (as mlp_mse_grad).
 * grad:  device [param count] or NULL: a copy of the gradient.
 * Layers at most 256 wide and at most 8 linear layers (EINVAL otherwise).
 * workspace: device, mlp_train_workspace_bytes(shape, batch). */
size_t mlp_train_workspace_bytes(const sfg_mlp_shape *shape, uint32_t batch);
int mlp_train_step(const sfg_mlp_shape *shape, uint32_t batch, float *params, const float *x, const float *target,
                   const float *mask, const float *col_weight, const int64_t *rows, float *m, float *v,
                   const float *lr, float beta1, float beta2, float eps, uint32_t *step, float *loss, float *grad,
                   void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SFGEN_H */
