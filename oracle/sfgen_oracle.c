/*
 * sfgen oracle -- plain, single-threaded, deliberately slow CPU implementation
 * of what the generators compute.  TEST INFRASTRUCTURE ONLY: it exists so the
 * GPU library can be checked against something written directly from the
 * paper (Yoo & Henderson, "Parallel Generation of Massive Scale-Free Graphs").
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source with the HIP library.
 *
 * Every step is taken in the order the paper (or the stated reading of it)
 * gives, with no blocking, fusion or reordering.  Integer work is exact;
 * floating point is binary64 compiled with -ffp-contract=off.
 *
 * Random numbers: the paper names no generator.  Every draw comes from
 * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel Random Numbers: As
 * Easy as 1, 2, 3", SC'11), keyed by the 64-bit seed, with the counter
 * (item_lo, item_hi, x, tag | graph_id << 8).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { TAG_KRON = 1, TAG_PBA1 = 2, TAG_PBA2 = 3, TAG_WEDGE = 4, TAG_RANDOM = 6, TAG_PERTURB = 7 };

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (SC'11 paper, section on Philox).  One round maps
 * (c0,c1,c2,c3) with key (k0,k1) to
 *   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
 * and the key is bumped by the Weyl constants between rounds.
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint64_t item, uint32_t x, uint32_t tag, uint32_t gid, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)item, (uint32_t)(item >> 32), x, tag | (gid << 8)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Index in [0, R) from a 64-bit uniform: floor(U * R / 2^64). */
uint64_t orc_uidx(uint64_t U, uint64_t R)
{
    return (uint64_t)(((u128)U * (u128)R) >> 64);
}

/* Index in [0, R) from a 32-bit uniform: floor(w * R / 2^32). */
static uint32_t uidx32(uint32_t w, uint32_t R)
{
    return (uint32_t)(((uint64_t)w * R) >> 32);
}

/* Bernoulli(p) threshold: an event happens when a 32-bit draw is below
 * floor(p * 2^32).  Multiplying by 2^32 is exact in binary64. */
uint64_t orc_bernoulli_threshold(double p)
{
    double t = floor(p * 4294967296.0);
    if (t <= 0.0) return 0;
    if (t >= 4294967296.0) return 4294967296ull;
    return (uint64_t)t;
}

/* Categorical thresholds for nonnegative float32 weights W[0..C-1]:
 * running sums in binary64, left to right; thr[c] = floor((S_c / T) * 2^32)
 * for c < C-1 and thr[C-1] = 2^32.  A 32-bit draw w selects cell
 * #{c < C-1 : w >= thr[c]}.  Returns -1 on a negative, non-finite or
 * all-zero weight vector. */
int orc_categorical_thresholds(const float *W, uint32_t C, uint64_t *thr)
{
    double S = 0.0;
    double *run = (double *)malloc(sizeof(double) * C);
    if (!run) return -1;
    for (uint32_t c = 0; c < C; ++c) {
        double w = (double)W[c];
        if (!(w >= 0.0) || isinf(w)) { free(run); return -1; }
        S = S + w;
        run[c] = S;
    }
    if (!(S > 0.0) || isinf(S)) { free(run); return -1; }
    for (uint32_t c = 0; c + 1 < C; ++c) {
        double q = run[c] / S;
        double t = floor(q * 4294967296.0);
        thr[c] = t >= 4294967296.0 ? 4294967296ull : (uint64_t)t;
    }
    thr[C - 1] = 4294967296ull;
    free(run);
    return 0;
}

static uint32_t cell_of(uint32_t w, const uint64_t *thr, uint32_t C)
{
    uint32_t c = 0;
    for (uint32_t i = 0; i + 1 < C; ++i)
        if ((uint64_t)w >= thr[i]) ++c;
    return c;
}

/* ---------------------------------------------------------------------------
 * Kronecker generator, sample mode.  The Kronecker power of the initiator
 * gives every cell (u, v) of the n0^k x n0^k matrix the probability
 * prod_l W[u_l][v_l] / T^k (Kronecker product section; the probabilistic
 * model of Leskovec et al. cited in Related Work).  Each edge descends k
 * levels, most significant digit first.  Level l takes a 24-bit uniform U
 * from the Philox block (e, l / 5, KRON): for l mod 5 = i < 4 the top 24
 * bits of word i, for l mod 5 = 4 the low bytes of words 0, 1 and 2 (most
 * significant first); the cell is the one the 32-bit thresholds give to
 * U * 256.  Edges e in [e_begin, e_end) are written to src[e - e_begin],
 * dst[e - e_begin].  Self-loops and duplicates are kept.
 * ------------------------------------------------------------------------- */
static uint32_t level_uniform24(const uint32_t blk[4], uint32_t i)
{
    if (i < 4) return blk[i] >> 8;
    return ((blk[0] & 255u) << 16) | ((blk[1] & 255u) << 8) | (blk[2] & 255u);
}

int orc_kron_sample(uint32_t n0, const float *W, uint32_t k, uint64_t e_begin, uint64_t e_end,
                    uint64_t seed, uint32_t gid, int64_t *src, int64_t *dst)
{
    uint32_t C = n0 * n0;
    uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * C);
    if (!thr) return -1;
    if (orc_categorical_thresholds(W, C, thr) != 0) { free(thr); return -1; }
    for (uint64_t e = e_begin; e < e_end; ++e) {
        uint64_t u = 0, v = 0;
        uint32_t blk[4] = {0, 0, 0, 0};
        for (uint32_t l = 0; l < k; ++l) {
            if (l % 5 == 0) draw(seed, e, l / 5, TAG_KRON, gid, blk);
            uint32_t c = cell_of(level_uniform24(blk, l % 5) << 8, thr, C);
            u = u * n0 + c / n0;
            v = v * n0 + c % n0;
        }
        src[e - e_begin] = (int64_t)u;
        dst[e - e_begin] = (int64_t)v;
    }
    free(thr);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Kronecker generator, enumerate mode: the paper's deterministic PK method
 * (Parallel Kronecker section, serial algorithm and Fig. 2).  A 0/1 seed
 * adjacency matrix is expanded k-1 times; every 1 becomes a copy of the seed
 * and every 0 a block of zeros.  A meta-edge is (iteration, row, col).  The
 * expansion uses the stack described there: pop the top meta-edge, emit it
 * if it is at the final iteration, otherwise push its children.  Children
 * and the initial seed edges are pushed in reverse row-major order so that
 * edges come out in row-major digit order.  Returns the number of edges
 * emitted, or -1 if it would exceed cap.
 * ------------------------------------------------------------------------- */
typedef struct { uint32_t iter; int64_t row, col; } meta_edge;

int64_t orc_kron_enumerate(uint32_t n0, const uint8_t *adj, uint32_t k, int64_t *src, int64_t *dst,
                           uint64_t cap)
{
    uint32_t e0 = 0;
    for (uint32_t c = 0; c < n0 * n0; ++c) e0 += adj[c] ? 1u : 0u;
    /* Depth-first expansion never holds more than e0 meta-edges per level. */
    size_t stack_cap = (size_t)e0 * (k + 1) + 1;
    meta_edge *stack = (meta_edge *)malloc(sizeof(meta_edge) * stack_cap);
    if (!stack) return -1;
    size_t top = 0;
    for (int64_t c = (int64_t)n0 * n0 - 1; c >= 0; --c)
        if (adj[c]) {
            meta_edge me = {1, c / n0, c % n0};
            stack[top++] = me;
        }
    int64_t emitted = 0;
    while (top > 0) {
        meta_edge me = stack[--top];
        if (me.iter == k) {
            if ((uint64_t)emitted >= cap) { free(stack); return -1; }
            src[emitted] = me.row;
            dst[emitted] = me.col;
            ++emitted;
            continue;
        }
        for (int64_t c = (int64_t)n0 * n0 - 1; c >= 0; --c)
            if (adj[c]) {
                meta_edge ch = {me.iter + 1, me.row * n0 + c / n0, me.col * n0 + c % n0};
                stack[top++] = ch;
            }
    }
    free(stack);
    return emitted;
}

/* ---------------------------------------------------------------------------
 * Parallel Barabasi-Albert (PBA), two-phase preferential attachment
 * (PBA section and Fig. 1).  The paper's processors are partitions q of
 * contiguous vertex blocks, start(q) = floor(q n / P).  Every vertex owns m
 * edge slots; slot j of partition q belongs to vertex start(q) + j / m.
 * ------------------------------------------------------------------------- */
static uint64_t part_start(uint64_t n, uint32_t P, uint32_t q)
{
    return (uint64_t)(((u128)q * n) / P);
}

/* Phase 1 for one partition: the local edge list A of labels.  The first s
 * slots take the faction list F in order; a later slot j becomes an
 * inter-faction edge to a uniformly chosen non-faction partition with
 * probability p, and otherwise copies the label of a uniformly chosen earlier
 * slot (uniform edge choice realises preferential attachment).
 * script, when non-NULL, replaces the random choice of slot j >= s by
 * script[j - s]: >= 0 copies that slot, < 0 takes label -1 - script[j - s]. */
int orc_pba_phase1(uint64_t nslots, uint32_t q, uint64_t thr_p, const uint32_t *F, uint32_t s,
                   const uint32_t *NF, uint32_t nnf, uint64_t seed, uint32_t gid,
                   const int64_t *script, uint32_t *label)
{
    for (uint64_t j = 0; j < nslots; ++j) {
        if (j < s) {
            label[j] = F[j];
            continue;
        }
        if (script) {
            int64_t a = script[j - s];
            label[j] = a >= 0 ? label[a] : (uint32_t)(-1 - a);
            continue;
        }
        uint32_t w[4];
        draw(seed, j, q, TAG_PBA1, gid, w);
        uint64_t U = (uint64_t)w[1] | ((uint64_t)w[2] << 32);
        if (nnf > 0 && (uint64_t)w[0] < thr_p)
            label[j] = NF[orc_uidx(U, nnf)];
        else
            label[j] = label[orc_uidx(U, j)];
    }
    return 0;
}

/* Phase 2 for one partition: D endpoints chosen by the standard preferential
 * attachment growth over the partition's L local vertices, seeded with a
 * 2-vertex clique.  The pool holds the endpoints of all edges so far:
 * pool[0] = 0, pool[1] = 1; the t-th arrival is local vertex
 * x_t = floor(t L / D), whose endpoint y_t is a uniformly chosen pool entry
 * among the first 2 + 2t; then pool[2+2t] = x_t and pool[3+2t] = y_t.  The
 * selection list is S[t] = y_t. */
int orc_pba_phase2(uint64_t D, uint64_t L, uint32_t q, uint64_t seed, uint32_t gid, uint32_t *S)
{
    if (D == 0) return 0;
    uint32_t *pool = (uint32_t *)malloc(sizeof(uint32_t) * (2 + 2 * D));
    if (!pool) return -1;
    pool[0] = 0;
    pool[1] = 1;
    for (uint64_t t = 0; t < D; ++t) {
        uint32_t x = (uint32_t)(((u128)t * L) / D);
        uint32_t w[4];
        draw(seed, t, q, TAG_PBA2, gid, w);
        uint64_t U = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        uint32_t y = pool[orc_uidx(U, 2 + 2 * t)];
        pool[2 + 2 * t] = x;
        pool[3 + 2 * t] = y;
        S[t] = y;
    }
    free(pool);
    return 0;
}

/* Substitution: every occurrence of partition l in A is replaced, in slot
 * order, by the next endpoint of the list partition l sent to this
 * requester; that list starts at S_l[off_row[l]].  S_l begins at
 * S + S_base[l] and its ids are local to partition l. */
int orc_pba_substitute(uint64_t nslots, const uint32_t *label, uint32_t P, const uint64_t *start,
                       const uint64_t *off_row, const uint64_t *S_base, const uint32_t *S, int64_t *dst)
{
    uint64_t *next = (uint64_t *)malloc(sizeof(uint64_t) * P);
    if (!next) return -1;
    for (uint32_t l = 0; l < P; ++l) next[l] = off_row[l];
    for (uint64_t j = 0; j < nslots; ++j) {
        uint32_t l = label[j];
        dst[j] = (int64_t)(start[l] + S[S_base[l] + next[l]]);
        next[l] += 1;
    }
    free(next);
    return 0;
}

/* Faction lists: F(q) = faction_members[faction_off[q] .. faction_off[q+1]),
 * or [q] when faction_off is NULL.  NF(q) = ascending partitions not in F(q). */
static uint32_t faction_list(const uint32_t *foff, const uint32_t *fmem, uint32_t q, const uint32_t **F,
                             uint32_t *self)
{
    if (!foff) {
        *self = q;
        *F = self;
        return 1;
    }
    *F = fmem + foff[q];
    return foff[q + 1] - foff[q];
}

/* The whole PBA generator.  Outputs: src/dst (n*m each, edge e = m*start(q)+j).
 * Optional outputs (NULL to skip): labels (n*m), counts (P*P, c[q][l]),
 * S (n*m, partition l's list at offset sum_{l'<l} D[l']). */
int orc_pba_generate(uint64_t n, uint32_t m, uint32_t P, double p, const uint32_t *foff,
                     const uint32_t *fmem, uint64_t seed, uint32_t gid, int64_t *src, int64_t *dst,
                     uint32_t *labels_out, uint64_t *counts_out, uint32_t *S_out)
{
    uint64_t E = n * m;
    uint64_t thr_p = orc_bernoulli_threshold(p);
    uint64_t *start = (uint64_t *)malloc(sizeof(uint64_t) * (P + 1));
    uint32_t *label = labels_out ? labels_out : (uint32_t *)malloc(sizeof(uint32_t) * (E ? E : 1));
    uint64_t *cnt = (uint64_t *)calloc((size_t)P * P, sizeof(uint64_t));
    uint64_t *D = (uint64_t *)calloc(P, sizeof(uint64_t));
    uint64_t *S_base = (uint64_t *)calloc(P + 1, sizeof(uint64_t));
    uint64_t *off = (uint64_t *)calloc((size_t)P * P, sizeof(uint64_t));
    uint32_t *S = S_out ? S_out : (uint32_t *)malloc(sizeof(uint32_t) * (E ? E : 1));
    uint32_t *NF = (uint32_t *)malloc(sizeof(uint32_t) * P);
    uint8_t *inF = (uint8_t *)malloc(P);
    int rc = -1;
    if (!start || !label || !cnt || !D || !S_base || !off || !S || !NF || !inF) goto done;
    /* Every processor draws from at least one faction: slot 0 has nothing
     * earlier to copy. */
    if (foff)
        for (uint32_t q = 0; q < P; ++q)
            if (foff[q + 1] <= foff[q]) goto done;
    for (uint32_t q = 0; q <= P; ++q) start[q] = part_start(n, P, q);

    /* Phase 1, every partition. */
    for (uint32_t q = 0; q < P; ++q) {
        uint64_t L = start[q + 1] - start[q];
        const uint32_t *F;
        uint32_t self;
        uint32_t s = faction_list(foff, fmem, q, &F, &self);
        memset(inF, 0, P);
        for (uint32_t i = 0; i < s; ++i) inF[F[i]] = 1;
        uint32_t nnf = 0;
        for (uint32_t r = 0; r < P; ++r)
            if (!inF[r]) NF[nnf++] = r;
        orc_pba_phase1(L * m, q, thr_p, F, s, NF, nnf, seed, gid, NULL, label + m * start[q]);
    }
    /* Count message: c[q][l] = occurrences of l in partition q's list. */
    for (uint32_t q = 0; q < P; ++q)
        for (uint64_t j = m * start[q]; j < m * start[q + 1]; ++j) cnt[(size_t)q * P + label[j]] += 1;
    /* Each partition l receives D[l] = sum_q c[q][l] requests, divided among
     * requesters in ascending requester order. */
    for (uint32_t l = 0; l < P; ++l) {
        uint64_t acc = 0;
        for (uint32_t q = 0; q < P; ++q) {
            off[(size_t)q * P + l] = acc;
            acc += cnt[(size_t)q * P + l];
        }
        D[l] = acc;
    }
    for (uint32_t l = 0; l < P; ++l) S_base[l + 1] = S_base[l] + D[l];
    /* Phase 2, every partition. */
    for (uint32_t l = 0; l < P; ++l)
        if (orc_pba_phase2(D[l], start[l + 1] - start[l], l, seed, gid, S + S_base[l]) != 0) goto done;
    /* Substitution and the source endpoints. */
    for (uint32_t q = 0; q < P; ++q) {
        uint64_t b = m * start[q];
        orc_pba_substitute(m * (start[q + 1] - start[q]), label + b, P, start, off + (size_t)q * P, S_base,
                           S, dst + b);
    }
    for (uint64_t e = 0; e < E; ++e) src[e] = (int64_t)(e / m);
    if (counts_out) memcpy(counts_out, cnt, sizeof(uint64_t) * P * P);
    rc = 0;
done:
    free(start);
    if (!labels_out) free(label);
    free(cnt);
    free(D);
    free(S_base);
    free(off);
    if (!S_out) free(S);
    free(NF);
    free(inF);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Compressed sparse rows: the entries sorted ascending by (row, column);
 * row_ptr[v] = number of kept entries with row < v; col = their columns in
 * sorted order.  flags & 1 (symmetrize): (v, u) is added for every (u, v), so
 * a self-loop appears twice.  flags & 2 (simple): self-loops are dropped and
 * an entry equal to the previous sorted entry is dropped.  dups = number of
 * sorted positions whose entry equals the previous one (counted before any
 * dropping).  Returns the number of kept entries, or -1.
 * ------------------------------------------------------------------------- */
static int cmp_pair(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

int64_t orc_edges_to_csr(uint64_t n, uint64_t E, const int64_t *src, const int64_t *dst, int flags,
                         uint64_t *row_ptr, int64_t *col, uint64_t *dups)
{
    int symmetrize = flags & 1, simple = flags & 2;
    uint64_t N = symmetrize ? 2 * E : E;
    int64_t *pairs = (int64_t *)malloc(sizeof(int64_t) * 2 * (N ? N : 1));
    if (!pairs) return -1;
    for (uint64_t e = 0; e < E; ++e) {
        pairs[2 * e] = src[e];
        pairs[2 * e + 1] = dst[e];
        if (symmetrize) {
            pairs[2 * (E + e)] = dst[e];
            pairs[2 * (E + e) + 1] = src[e];
        }
    }
    qsort(pairs, N, 2 * sizeof(int64_t), cmp_pair);
    for (uint64_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    uint64_t d = 0, kept = 0;
    for (uint64_t i = 0; i < N; ++i) {
        int repeat = i > 0 && pairs[2 * i] == pairs[2 * i - 2] && pairs[2 * i + 1] == pairs[2 * i - 1];
        if (repeat) ++d;
        if (simple && (repeat || pairs[2 * i] == pairs[2 * i + 1])) continue;
        row_ptr[pairs[2 * i] + 1] += 1;
        col[kept++] = pairs[2 * i + 1];
    }
    for (uint64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    *dups = d;
    free(pairs);
    return (int64_t)kept;
}

/* Degree of every vertex counting both endpoints of every edge (a self-loop
 * adds 2), and its 32-bin log2 histogram: bin 0 holds degree 0, bin b holds
 * degrees in [2^(b-1), 2^b), degrees from 2^30 up go to bin 31. */
int orc_degree_histogram(uint64_t n, uint64_t E, const int64_t *src, const int64_t *dst, uint64_t *deg,
                         uint64_t *hist)
{
    for (uint64_t v = 0; v < n; ++v) deg[v] = 0;
    for (uint64_t e = 0; e < E; ++e) {
        deg[src[e]] += 1;
        deg[dst[e]] += 1;
    }
    for (int b = 0; b < 32; ++b) hist[b] = 0;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t d = deg[v];
        int b = 0;
        while (b < 31 && d >= (1ull << b)) ++b;
        hist[b] += 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Graph statistics used to describe an ensemble member.
 * Tail exponent: the discrete power-law maximum-likelihood approximation of
 * Clauset, Shalizi & Newman (SIAM Review 2009, eq. 3.7):
 *   gamma = 1 + N_t / sum_{d_i >= d_min} ln(d_i / (d_min - 1/2)).
 * The paper fits gamma to degree distributions (Results, Fig. 3) and notes
 * that a finite mean degree implies gamma > 2.
 * ------------------------------------------------------------------------- */
double orc_gamma_mle(uint64_t n, const uint64_t *deg, uint64_t d_min)
{
    uint64_t nt = 0;
    double s = 0.0;
    for (uint64_t v = 0; v < n; ++v)
        if (deg[v] >= d_min && deg[v] > 0) {
            nt += 1;
            s += log((double)deg[v] / ((double)d_min - 0.5));
        }
    if (nt == 0 || !(s > 0.0)) return NAN;
    return 1.0 + (double)nt / s;
}

/* Simple undirected graph: both orientations of every non-loop edge, sorted,
 * duplicates removed.  row_ptr has n+1 entries; col must hold 2E entries.
 * Returns the number of entries kept. */
int64_t orc_simple_csr(uint64_t n, uint64_t E, const int64_t *src, const int64_t *dst, uint64_t *row_ptr,
                       int64_t *col)
{
    int64_t *pairs = (int64_t *)malloc(sizeof(int64_t) * 4 * (E ? E : 1));
    if (!pairs) return -1;
    uint64_t N = 0;
    for (uint64_t e = 0; e < E; ++e) {
        if (src[e] == dst[e]) continue;
        pairs[2 * N] = src[e];
        pairs[2 * N + 1] = dst[e];
        ++N;
        pairs[2 * N] = dst[e];
        pairs[2 * N + 1] = src[e];
        ++N;
    }
    qsort(pairs, N, 2 * sizeof(int64_t), cmp_pair);
    uint64_t k = 0;
    for (uint64_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    for (uint64_t i = 0; i < N; ++i) {
        if (i > 0 && pairs[2 * i] == pairs[2 * i - 2] && pairs[2 * i + 1] == pairs[2 * i - 1]) continue;
        row_ptr[pairs[2 * i] + 1] += 1;
        col[k++] = pairs[2 * i + 1];
    }
    for (uint64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    free(pairs);
    return (int64_t)k;
}

static int has_neighbor(const uint64_t *row_ptr, const int64_t *col, int64_t v, int64_t w)
{
    uint64_t lo = row_ptr[v], hi = row_ptr[v + 1];
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < w) lo = mid + 1;
        else hi = mid;
    }
    return lo < row_ptr[v + 1] && col[lo] == w;
}

/* Wedge sampling on a simple undirected CSR (Results: the clustering the
 * paper compares is estimated here by sampled wedges).  Sample i picks the
 * centre v with probability proportional to C(d_v, 2) -- the first vertex
 * whose inclusive prefix of C(d, 2) exceeds a uniform index in [0, total) --
 * then two distinct neighbours a != b uniformly; the wedge is closed when a
 * and b are adjacent.
 *
 * orc_wedge_draws writes (v, a, b) of samples 0 .. num_samples-1 into out[3 i
 * .. 3 i + 2] (a and b are the neighbours' ids) and returns the number of
 * closed ones; orc_wedge_closed returns only that number.  Both return -1 if
 * the graph has no wedge (out is then untouched). */
int64_t orc_wedge_draws(uint64_t n, const uint64_t *row_ptr, const int64_t *col, uint32_t num_samples,
                        uint64_t seed, uint32_t gid, int64_t *out)
{
    uint64_t *pre = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!pre) return -1;
    uint64_t acc = 0;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t d = row_ptr[v + 1] - row_ptr[v];
        acc += d >= 2 ? d * (d - 1) / 2 : 0;
        pre[v] = acc; /* inclusive prefix of C(d, 2) */
    }
    if (acc == 0) { free(pre); return -1; }
    int64_t closed = 0;
    for (uint32_t i = 0; i < num_samples; ++i) {
        uint32_t w[4];
        draw(seed, i, 0, TAG_WEDGE, gid, w);
        uint64_t target = orc_uidx((uint64_t)w[0] | ((uint64_t)w[1] << 32), acc);
        /* centre: the first v whose inclusive prefix exceeds target */
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (pre[mid] > target) hi = mid;
            else lo = mid + 1;
        }
        uint64_t v = lo;
        uint32_t d = (uint32_t)(row_ptr[v + 1] - row_ptr[v]);
        uint32_t a = uidx32(w[2], d);
        uint32_t b = uidx32(w[3], d - 1);
        if (b >= a) b += 1;
        int64_t na = col[row_ptr[v] + a], nb = col[row_ptr[v] + b];
        closed += has_neighbor(row_ptr, col, na, nb);
        if (out) {
            out[3 * (uint64_t)i] = (int64_t)v;
            out[3 * (uint64_t)i + 1] = na;
            out[3 * (uint64_t)i + 2] = nb;
        }
    }
    free(pre);
    return closed;
}

int64_t orc_wedge_closed(uint64_t n, const uint64_t *row_ptr, const int64_t *col, uint32_t num_samples,
                         uint64_t seed, uint32_t gid)
{
    return orc_wedge_draws(n, row_ptr, col, num_samples, seed, gid, NULL);
}

/* ------------------------------------------------------------------------
 * Sampled path statistics (Results, Table 2: average shortest-path length and
 * diameter estimated by sampling).  A breadth-first search from every given
 * source over the CSR graph (unweighted; the caller passes the simple
 * undirected CSR).  Outputs: the sum of d(s, v) and the number of pairs over
 * all sources s and vertices v != s reachable from s, and the largest such
 * distance (the sampled eccentricity maximum, the diameter estimate).
 * ---------------------------------------------------------------------- */
void orc_path_stats(uint64_t n, const uint64_t *row_ptr, const int64_t *col, const int64_t *sources,
                    uint32_t num_sources, uint64_t *sum_out, uint64_t *pairs_out, uint64_t *max_out)
{
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    uint64_t sum = 0, pairs = 0, mx = 0;
    for (uint32_t i = 0; i < num_sources; ++i) {
        for (uint64_t v = 0; v < n; ++v) dist[v] = -1;
        int64_t s = sources[i];
        uint64_t head = 0, tail = 0;
        dist[s] = 0;
        queue[tail++] = s;
        while (head < tail) {
            int64_t u = queue[head++];
            for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int64_t x = col[e];
                if (dist[x] < 0) {
                    dist[x] = dist[u] + 1;
                    queue[tail++] = x;
                    sum += (uint64_t)dist[x];
                    pairs += 1;
                    if ((uint64_t)dist[x] > mx) mx = (uint64_t)dist[x];
                }
            }
        }
    }
    *sum_out = sum;
    *pairs_out = pairs;
    *max_out = mx;
    free(dist);
    free(queue);
}

/* ------------------------------------------------------------------------
 * Randomized PK by exclusive OR (PK section, randomization): the adjacency
 * matrix of the deterministic Kronecker power XOR that of a random graph.
 * The random graph is the set of distinct pairs among num_random uniform
 * draws: draw i is Philox block (i, 0, 0, tag 6 | gid << 8), row =
 * uidx(w0 + 2^32 w1, n), column = uidx(w2 + 2^32 w3, n).  A pair is an edge
 * of the result when it is an edge of exactly one of the two graphs.
 * Output: CSR of the result (rows ascending, columns ascending), returns the
 * number of edges, or -1 on allocation failure.  row_ptr has n + 1 entries,
 * col room for e0^k + num_random.
 * ---------------------------------------------------------------------- */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t orc_kron_xor_random(uint32_t n0, const uint8_t *adj, uint32_t k, uint64_t num_random, uint64_t seed,
                            uint32_t gid, uint64_t *row_ptr, int64_t *col)
{
    uint32_t e0 = 0;
    for (uint32_t c = 0; c < n0 * n0; ++c) e0 += adj[c] ? 1u : 0u;
    uint64_t epk = 1, n = 1;
    for (uint32_t l = 0; l < k; ++l) { epk *= e0; n *= n0; }
    int64_t *ps = (int64_t *)malloc(sizeof(int64_t) * (epk ? epk : 1));
    int64_t *pd = (int64_t *)malloc(sizeof(int64_t) * (epk ? epk : 1));
    uint64_t *pk = (uint64_t *)malloc(sizeof(uint64_t) * (epk ? epk : 1));
    uint64_t *rk = (uint64_t *)malloc(sizeof(uint64_t) * (num_random ? num_random : 1));
    if (!ps || !pd || !pk || !rk) { free(ps); free(pd); free(pk); free(rk); return -1; }
    orc_kron_enumerate(n0, adj, k, ps, pd, epk);
    for (uint64_t e = 0; e < epk; ++e) pk[e] = (uint64_t)ps[e] * n + (uint64_t)pd[e];
    for (uint64_t i = 0; i < num_random; ++i) {
        uint32_t w[4];
        draw(seed, i, 0, TAG_RANDOM, gid, w);
        uint64_t a = orc_uidx((uint64_t)w[0] | ((uint64_t)w[1] << 32), n);
        uint64_t b = orc_uidx((uint64_t)w[2] | ((uint64_t)w[3] << 32), n);
        rk[i] = a * n + b;
    }
    qsort(pk, epk, sizeof(uint64_t), cmp_u64);
    qsort(rk, num_random, sizeof(uint64_t), cmp_u64);
    /* Merge the two sorted lists; the random list may repeat a pair. */
    uint64_t i = 0, j = 0, out = 0;
    for (uint64_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    while (i < epk || j < num_random) {
        uint64_t key;
        int in_pk = 0, in_rand = 0;
        if (j >= num_random || (i < epk && pk[i] <= rk[j])) key = pk[i]; else key = rk[j];
        while (i < epk && pk[i] == key) { in_pk = 1; ++i; }
        while (j < num_random && rk[j] == key) { in_rand = 1; ++j; }
        if (in_pk != in_rand) {
            col[out++] = (int64_t)(key % n);
            row_ptr[key / n + 1] += 1;
        }
    }
    for (uint64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    free(ps); free(pd); free(pk); free(rk);
    return (int64_t)out;
}

/* ------------------------------------------------------------------------
 * Randomized PK by temporary seed modification (PK section, randomization):
 * the meta-edge stack of orc_kron_enumerate, except that every meta-edge of
 * iteration i < k is replaced by the edges of a perturbed copy of the seed:
 * an absent cell c is added with probability p_add, a present one deleted
 * with probability p_del.  The draws of meta-edge (i, row, col) come from
 * Philox blocks (row, col, i | b << 8, tag 7 | gid << 8), b = c / 4, word
 * c mod 4, compared with floor(p 2^32).  The seed's own edges (iteration 1)
 * are not perturbed.  Emits edges in stack order; returns their number, or
 * -1 when more than cap would be written.
 * ---------------------------------------------------------------------- */
int64_t orc_kron_perturbed(uint32_t n0, const uint8_t *adj, uint32_t k, double p_add, double p_del, uint64_t seed,
                           uint32_t gid, int64_t *src, int64_t *dst, uint64_t cap)
{
    const uint32_t C = n0 * n0;
    const uint64_t thr_add = orc_bernoulli_threshold(p_add), thr_del = orc_bernoulli_threshold(p_del);
    size_t stack_cap = (size_t)C * (k + 1) + 1;
    meta_edge *stack = (meta_edge *)malloc(sizeof(meta_edge) * stack_cap);
    uint8_t *cell = (uint8_t *)malloc(C ? C : 1);
    if (!stack || !cell) { free(stack); free(cell); return -1; }
    size_t top = 0;
    for (int64_t c = (int64_t)C - 1; c >= 0; --c)
        if (adj[c]) {
            meta_edge me = {1, c / n0, c % n0};
            stack[top++] = me;
        }
    int64_t emitted = 0;
    while (top > 0) {
        meta_edge me = stack[--top];
        if (me.iter == k) {
            if ((uint64_t)emitted >= cap) { free(stack); free(cell); return -1; }
            src[emitted] = me.row;
            dst[emitted] = me.col;
            ++emitted;
            continue;
        }
        /* the temporarily modified seed of this meta-edge */
        for (uint32_t c = 0; c < C; ++c) {
            uint32_t w[4];
            uint32_t ctr[4] = {(uint32_t)me.row, (uint32_t)me.col, me.iter | ((c / 4) << 8), TAG_PERTURB | (gid << 8)};
            uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            orc_philox4x32_10(ctr, key, w);
            uint64_t x = w[c % 4];
            cell[c] = adj[c] ? (x < thr_del ? 0 : 1) : (x < thr_add ? 1 : 0);
        }
        for (int64_t c = (int64_t)C - 1; c >= 0; --c)
            if (cell[c]) {
                meta_edge ch = {me.iter + 1, me.row * n0 + c / n0, me.col * n0 + c % n0};
                stack[top++] = ch;
            }
    }
    free(stack);
    free(cell);
    return emitted;
}
