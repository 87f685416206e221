"""CPU oracle for the scale-free graph generators -- TEST INFRASTRUCTURE.

A plain, single-threaded, obviously-correct implementation of what the GPU
library computes, written from the paper (Yoo & Henderson, "Parallel
Generation of Massive Scale-Free Graphs") and checked against what the paper
and the mathematics fix (see tests/test_oracle_*.py).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
product path never does.  It shares no code with the HIP library.

The arithmetic lives in ``sfgen_oracle.c`` (built by ``oracle/build.py`` into
``liboracle.so``) and, for the MLP surrogate, in ``oracle/mlp.py`` (numpy
float64).  This module only marshals numpy arrays into the C functions.
"""
import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
        "orc_uidx": (C.c_uint64, [C.c_uint64, C.c_uint64]),
        "orc_bernoulli_threshold": (C.c_uint64, [C.c_double]),
        "orc_categorical_thresholds": (C.c_int, [f32p, C.c_uint32, u64p]),
        "orc_kron_sample": (C.c_int, [C.c_uint32, f32p, C.c_uint32, C.c_uint64, C.c_uint64,
                                      C.c_uint64, C.c_uint32, i64p, i64p]),
        "orc_kron_enumerate": (C.c_int64, [C.c_uint32, u8p, C.c_uint32, i64p, i64p, C.c_uint64]),
        "orc_pba_phase1": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint64, u32p, C.c_uint32, u32p,
                                     C.c_uint32, C.c_uint64, C.c_uint32, C.c_void_p, u32p]),
        "orc_pba_phase2": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, u32p]),
        "orc_pba_substitute": (C.c_int, [C.c_uint64, u32p, C.c_uint32, u64p, u64p, u64p, u32p, i64p]),
        "orc_pba_generate": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_double, C.c_void_p,
                                       C.c_void_p, C.c_uint64, C.c_uint32, i64p, i64p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]),
        "orc_edges_to_csr": (C.c_int64, [C.c_uint64, C.c_uint64, i64p, i64p, C.c_int, u64p, i64p, u64p]),
        "orc_degree_histogram": (C.c_int, [C.c_uint64, C.c_uint64, i64p, i64p, u64p, u64p]),
        "orc_gamma_mle": (C.c_double, [C.c_uint64, u64p, C.c_uint64]),
        "orc_simple_csr": (C.c_int64, [C.c_uint64, C.c_uint64, i64p, i64p, u64p, i64p]),
        "orc_wedge_closed": (C.c_int64, [C.c_uint64, u64p, i64p, C.c_uint32, C.c_uint64, C.c_uint32]),
        "orc_wedge_draws": (C.c_int64, [C.c_uint64, u64p, i64p, C.c_uint32, C.c_uint64, C.c_uint32, i64p]),
        "orc_path_stats": (None, [C.c_uint64, u64p, i64p, i64p, C.c_uint32, u64p, u64p, u64p]),
        "orc_kron_xor_random": (C.c_int64, [C.c_uint32, u8p, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32,
                                            u64p, i64p]),
        "orc_kron_perturbed": (C.c_int64, [C.c_uint32, u8p, C.c_uint32, C.c_double, C.c_double, C.c_uint64,
                                           C.c_uint32, i64p, i64p, C.c_uint64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------- primitives
def philox(ctr, key):
    """Philox4x32-10 block for counter (4 x u32) and key (2 x u32)."""
    out = np.zeros(4, np.uint32)
    _load().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def uidx(U: int, R: int) -> int:
    return int(_load().orc_uidx(U, R))


def bernoulli_threshold(p: float) -> int:
    return int(_load().orc_bernoulli_threshold(p))


def categorical_thresholds(W) -> np.ndarray:
    W = np.ascontiguousarray(W, np.float32).ravel()
    thr = np.zeros(W.size, np.uint64)
    if _load().orc_categorical_thresholds(W, W.size, thr) != 0:
        raise ValueError("initiator must be finite, nonnegative and not all zero")
    return thr


def cell_probabilities(W) -> np.ndarray:
    """Exact probability of each cell for a level's 24-bit uniform U: cell c
    takes the U with thr[c - 1] <= 256 U < thr[c], i.e. U in
    [ceil(thr[c - 1] / 256), ceil(thr[c] / 256))."""
    thr = categorical_thresholds(W).astype(np.uint64)
    up = ((thr + np.uint64(255)) // np.uint64(256)).astype(np.float64)
    prev = np.concatenate([[0.0], up[:-1]])
    return (up - prev) / 2.0 ** 24


# --------------------------------------------------------------------- Kronecker
def kron_sample(n0, W, k, num_edges, seed, graph_id=0, e_begin=0):
    """Edges [e_begin, e_begin + num_edges) of the sampled Kronecker graph."""
    W = np.ascontiguousarray(W, np.float32).ravel()
    assert W.size == n0 * n0
    src = np.zeros(num_edges, np.int64)
    dst = np.zeros(num_edges, np.int64)
    rc = _load().orc_kron_sample(n0, W, k, e_begin, e_begin + num_edges, seed, graph_id, src, dst)
    if rc != 0:
        raise ValueError("bad initiator")
    return src, dst


def kron_enumerate(adj, k):
    """The paper's deterministic Kronecker power, expanded with the meta-edge stack."""
    adj = np.ascontiguousarray(np.asarray(adj) != 0, np.uint8)
    n0 = adj.shape[0]
    e0 = int(adj.sum())
    cap = e0 ** k
    src = np.zeros(cap, np.int64)
    dst = np.zeros(cap, np.int64)
    got = _load().orc_kron_enumerate(n0, adj.ravel(), k, src, dst, cap)
    assert got == cap, (got, cap)
    return src, dst


# --------------------------------------------------------------------- PBA
def partition_starts(n, P):
    return np.array([(q * n) // P for q in range(P + 1)], np.uint64)


def pba_phase1(nslots, q, p, F, NF, seed, graph_id=0, script=None):
    F = np.ascontiguousarray(F, np.uint32)
    nnf = len(NF)
    NF = np.ascontiguousarray(NF, np.uint32) if nnf else np.zeros(1, np.uint32)
    label = np.zeros(max(nslots, 1), np.uint32)
    sc = None if script is None else np.ascontiguousarray(script, np.int64)
    _load().orc_pba_phase1(nslots, q, bernoulli_threshold(p), F, len(F), NF, nnf,
                           seed, graph_id, _ptr(sc), label)
    return label[:nslots]


def pba_phase2(D, L, q, seed, graph_id=0):
    S = np.zeros(max(D, 1), np.uint32)
    _load().orc_pba_phase2(D, L, q, seed, graph_id, S)
    return S[:D]


def pba_substitute(label, P, start, off_row, S_base, S):
    dst = np.zeros(max(len(label), 1), np.int64)
    _load().orc_pba_substitute(len(label), np.ascontiguousarray(label, np.uint32), P,
                               np.ascontiguousarray(start, np.uint64), np.ascontiguousarray(off_row, np.uint64),
                               np.ascontiguousarray(S_base, np.uint64), np.ascontiguousarray(S, np.uint32), dst)
    return dst[:len(label)]


def pba_generate(n, m, P, p, seed, graph_id=0, faction_off=None, faction_members=None, extras=False):
    """Full PBA edge list (src, dst) as int64; with extras also labels, counts, S."""
    E = n * m
    src = np.zeros(max(E, 1), np.int64)
    dst = np.zeros(max(E, 1), np.int64)
    foff = None if faction_off is None else np.ascontiguousarray(faction_off, np.uint32)
    fmem = None if faction_members is None else np.ascontiguousarray(faction_members, np.uint32)
    if foff is not None and fmem is None:
        fmem = np.zeros(1, np.uint32)
    labels = np.zeros(max(E, 1), np.uint32) if extras else None
    counts = np.zeros(P * P, np.uint64) if extras else None
    S = np.zeros(max(E, 1), np.uint32) if extras else None
    rc = _load().orc_pba_generate(n, m, P, p, _ptr(foff), _ptr(fmem), seed, graph_id, src, dst,
                                  _ptr(labels), _ptr(counts), _ptr(S))
    if rc != 0:
        raise ValueError("oracle PBA failed (empty faction list or out of memory)")
    if extras:
        return src[:E], dst[:E], labels[:E], counts.reshape(P, P), S[:E]
    return src[:E], dst[:E]


# --------------------------------------------------------------------- CSR and stats
def edges_to_csr(n, src, dst, symmetrize=False, simple=False):
    """(row_ptr, col, dups) of the sorted entry list; see orc_edges_to_csr."""
    src = np.ascontiguousarray(src, np.int64)
    dst = np.ascontiguousarray(dst, np.int64)
    E = src.size
    N = 2 * E if symmetrize else E
    row_ptr = np.zeros(n + 1, np.uint64)
    col = np.zeros(max(N, 1), np.int64)
    dups = np.zeros(1, np.uint64)
    kept = _load().orc_edges_to_csr(n, E, src, dst, int(bool(symmetrize)) | (2 if simple else 0), row_ptr, col, dups)
    if kept < 0:
        raise MemoryError("oracle CSR failed")
    return row_ptr, col[:kept], int(dups[0])


def degree_histogram(n, src, dst):
    src = np.ascontiguousarray(src, np.int64)
    dst = np.ascontiguousarray(dst, np.int64)
    deg = np.zeros(max(n, 1), np.uint64)
    hist = np.zeros(32, np.uint64)
    _load().orc_degree_histogram(n, src.size, src, dst, deg, hist)
    return deg[:n], hist


def gamma_mle(deg, d_min):
    deg = np.ascontiguousarray(deg, np.uint64)
    return float(_load().orc_gamma_mle(deg.size, deg, int(d_min)))


def gamma_dmin(n, num_edges):
    """d_min = 2 * ceil(mean degree), mean degree = 2E / n."""
    return 2 * ((2 * num_edges + n - 1) // n)


def simple_csr(n, src, dst):
    src = np.ascontiguousarray(src, np.int64)
    dst = np.ascontiguousarray(dst, np.int64)
    row_ptr = np.zeros(n + 1, np.uint64)
    col = np.zeros(max(2 * src.size, 1), np.int64)
    k = _load().orc_simple_csr(n, src.size, src, dst, row_ptr, col)
    return row_ptr, col[:k]


def wedge_closed(n, row_ptr, col, num_samples, seed, graph_id=0):
    row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
    col = np.ascontiguousarray(col, np.int64)
    if col.size == 0:
        col = np.zeros(1, np.int64)
    return int(_load().orc_wedge_closed(n, row_ptr, col, num_samples, seed, graph_id))


def wedge_draws(n, row_ptr, col, num_samples, seed, graph_id=0):
    """(closed count, [num_samples, 3] array of (centre, a, b)) of the wedge
    samples; (-1, None) when the graph has no wedge."""
    row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
    col = np.ascontiguousarray(col, np.int64)
    if col.size == 0:
        col = np.zeros(1, np.int64)
    out = np.zeros((max(num_samples, 1), 3), np.int64)
    closed = int(_load().orc_wedge_draws(n, row_ptr, col, num_samples, seed, graph_id, out))
    return (closed, out[:num_samples]) if closed >= 0 else (-1, None)


def path_stats(n, row_ptr, col, sources):
    """(sum of distances, reachable pairs, largest distance) of breadth-first
    searches from `sources` over the CSR graph (Results, Table 2)."""
    row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
    col = np.ascontiguousarray(col, np.int64)
    if col.size == 0:
        col = np.zeros(1, np.int64)
    src = np.ascontiguousarray(sources, np.int64)
    out = np.zeros(3, np.uint64)
    _load().orc_path_stats(n, row_ptr, col, src, src.size, out[0:1], out[1:2], out[2:3])
    return int(out[0]), int(out[1]), int(out[2])


def kron_xor_random(adj, k, num_random, seed, graph_id=0):
    """CSR (row_ptr, col) of the deterministic Kronecker power XOR the random
    graph of num_random uniform pair draws (PK section, randomization)."""
    adj = np.ascontiguousarray(np.asarray(adj) != 0, np.uint8)
    n0 = adj.shape[0]
    e0 = int(adj.sum())
    n = n0 ** k
    row_ptr = np.zeros(n + 1, np.uint64)
    col = np.zeros(max(e0 ** k + num_random, 1), np.int64)
    m = _load().orc_kron_xor_random(n0, adj, k, num_random, seed, graph_id, row_ptr, col)
    if m < 0:
        raise MemoryError("oracle XOR graph")
    return row_ptr, col[:m]


def kron_perturbed(adj, k, p_add, p_del, seed, graph_id=0, cap=None):
    """Kronecker power with the seed temporarily modified at every expansion
    (PK section, randomization); (src, dst) in stack order."""
    adj = np.ascontiguousarray(np.asarray(adj) != 0, np.uint8)
    n0 = adj.shape[0]
    if cap is None:
        cap = (n0 * n0) ** k
    src = np.zeros(max(cap, 1), np.int64)
    dst = np.zeros(max(cap, 1), np.int64)
    m = _load().orc_kron_perturbed(n0, adj, k, p_add, p_del, seed, graph_id, src, dst, cap)
    if m < 0:
        raise ValueError("more than cap edges")
    return src[:m], dst[:m]


def block_matrix(n, src, dst, blocks):
    """Coarse adjacency matrix (the adjacency-matrix view of the paper's
    community figure, Results): counts[i][j] = number of edges (u, v) with
    floor(u B / n) = i and floor(v B / n) = j, B = blocks."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    bi = (src * blocks) // n
    bj = (dst * blocks) // n
    counts = np.zeros((blocks, blocks), np.uint64)
    np.add.at(counts, (bi, bj), 1)
    return counts


def graph_stats(n, src, dst, num_samples, seed, graph_id=0):
    """(degree histogram, gamma estimate, closed-wedge count) of one graph."""
    deg, hist = degree_histogram(n, src, dst)
    g = gamma_mle(deg, gamma_dmin(n, len(src)))
    rp, col = simple_csr(n, src, dst)
    closed = wedge_closed(n, rp, col, num_samples, seed, graph_id)
    return hist, g, closed


__all__ = [k for k in list(globals()) if not k.startswith("_") and k not in ("C", "math", "os", "np")]
