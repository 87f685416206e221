"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks it against
an independent implementation (PyTorch's Philox header, exact rational
arithmetic, numpy), a worked example printed in the paper, a closed form, an
invariant, or a textbook special case.
"""
import json
import math
import os
import subprocess
import sys
from fractions import Fraction
from itertools import product

import numpy as np
import pytest
from scipy import stats

from paper_1003_3684_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    import ctypes
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    out = tmp_path_factory.mktemp("philox") / "libtorchphilox.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", f"-I{inc}",
                    os.path.join(GOLDEN, "philox_torch_harness.cpp"), "-o", str(out)], check=True)
    lib = ctypes.CDLL(str(out))
    p32 = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    lib.torch_philox_blocks.argtypes = [p32, p32, p32, ctypes.c_int]
    lib.torch_philox_blocks.restype = None

    def blocks(ctr, key):
        ctr = np.ascontiguousarray(ctr, np.uint32)
        key = np.ascontiguousarray(key, np.uint32)
        outv = np.zeros((ctr.shape[0], 4), np.uint32)
        lib.torch_philox_blocks(ctr, key, outv, ctr.shape[0])
        return outv
    return blocks


def test_philox_matches_torch_header(orc, torch_philox):
    """10^4 random (counter, key) pairs plus the extreme words 0 and 2^32-1."""
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(10_000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(10_000, 2), dtype=np.uint64).astype(np.uint32)
    edge = np.array([0, 0xFFFFFFFF], np.uint32)
    ectr = np.array(list(product(edge, repeat=4)), np.uint32)
    ekey = np.array(list(product(edge, repeat=2)), np.uint32)
    ctr = np.concatenate([ctr, np.repeat(ectr, len(ekey), axis=0)])
    key = np.concatenate([key, np.tile(ekey, (len(ectr), 1))])
    ref = torch_philox(ctr, key)
    got = np.array([orc.philox(c, k) for c, k in zip(ctr, key)])
    np.testing.assert_array_equal(got, ref)


# ----------------------------------------------------------------------------- thresholds
def _exact_thresholds(W):
    W = [Fraction(float(x)) for x in np.asarray(W, np.float32).ravel()]
    T = sum(W)
    out, S = [], Fraction(0)
    for c, w in enumerate(W):
        S += w
        out.append(math.floor(S / T * 2 ** 32) if c < len(W) - 1 else 2 ** 32)
    return np.array(out, np.uint64)


@pytest.mark.parametrize("W", [wl.KRON_K20["initiator"], wl.KRON_SCALE["initiator"], wl.KRON_SCALE_B["initiator"]])
def test_thresholds_exact_on_configs(orc, W):
    """binary64 running sums give the exact rational thresholds on every configured initiator."""
    np.testing.assert_array_equal(orc.categorical_thresholds(W), _exact_thresholds(W))


def test_thresholds_random(orc):
    """On random initiators the binary64 recipe is within one unit of the exact
    floor; an off-by-one is only possible at a rounding boundary and is rare."""
    rng = np.random.default_rng(2)
    mism = 0
    for _ in range(300):
        n0 = int(rng.integers(2, 5))
        W = rng.uniform(0, 1, size=n0 * n0).astype(np.float32)
        W[rng.uniform(size=W.size) < 0.2] = 0
        if W.sum() == 0:
            continue
        a, b = orc.categorical_thresholds(W).astype(np.int64), _exact_thresholds(W).astype(np.int64)
        assert np.max(np.abs(a - b)) <= 1
        mism += int(np.any(a != b))
    assert mism <= 3


def test_bernoulli_threshold(orc):
    assert orc.bernoulli_threshold(0.1) == 429_496_729
    assert orc.bernoulli_threshold(0.0) == 0
    assert orc.bernoulli_threshold(1.0) == 2 ** 32
    assert orc.bernoulli_threshold(0.5) == 2 ** 31


def test_uidx_is_floor(orc):
    rng = np.random.default_rng(3)
    for _ in range(2000):
        U, R = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2)), int(rng.integers(1, 2 ** 40))
        assert orc.uidx(U, R) == (U * R) >> 64


# ----------------------------------------------------------------------------- Kronecker sample
def _cell_probs(orc, W):
    return orc.cell_probabilities(W)


@pytest.mark.parametrize("n0,k,W", [
    (2, 3, [[0.6, 0.25], [0.1, 0.05]]),
    (3, 2, [[0.3, 0.1, 0.05], [0.2, 0.02, 0.1], [0.0, 0.15, 0.08]]),
    (2, 6, [[0.35, 0.25], [0.22, 0.18]]),
])
@pytest.mark.parametrize("seed", [11, 12])
def test_kron_chi_square_tiny(orc, n0, k, W, seed):
    """Every (u, v) cell of the n0^k x n0^k matrix is hit with probability
    prod_l p(u_l, v_l), the Kronecker product of the quantized initiator
    (brute-force enumeration of all cells, chi-square over 10^6 edges).  The
    initiators are asymmetric, so a transposed digit would fail; k = 6 spans
    a whole Philox block of five levels (the fifth built from the low bytes
    of three words) and the first level of the next, so levels that shared
    random bits would fail too."""
    E = 1_000_000
    src, dst = orc.kron_sample(n0, W, k, E, seed)
    nv = n0 ** k
    counts = np.bincount(src * nv + dst, minlength=nv * nv)
    p = _cell_probs(orc, W).reshape(n0, n0)
    expect = np.zeros((nv, nv))
    for u in range(nv):
        for v in range(nv):
            pr = 1.0
            for l in range(k):
                pr *= p[(u // n0 ** (k - 1 - l)) % n0, (v // n0 ** (k - 1 - l)) % n0]
            expect[u, v] = pr * E
    mask = expect.ravel() > 0
    assert counts[~mask].sum() == 0
    chi2 = ((counts[mask] - expect.ravel()[mask]) ** 2 / expect.ravel()[mask]).sum()
    pval = stats.chi2.sf(chi2, mask.sum() - 1)
    assert pval > 1e-4, (chi2, mask.sum(), pval)


def test_kron_zero_one_support(orc):
    """With a 0/1 initiator (the Fig. 2 seed) every edge is a nonzero of the
    Kronecker power, and all 11^k nonzeros are equally likely."""
    adj = wl.FIG2_SEED
    k = 2
    src, dst = orc.kron_sample(5, adj.astype(np.float32), k, 200_000, 5)
    G2 = np.kron(adj, adj)
    assert np.all(G2[src, dst] == 1)
    counts = np.bincount(src * 25 + dst, minlength=625)[G2.ravel() == 1]
    assert counts.size == 121
    assert stats.chisquare(counts).pvalue > 1e-4


def _kron_stats_closed_forms(orc, W, k, E):
    p = _cell_probs(orc, W)
    n0 = int(round(math.sqrt(p.size)))
    P = p.reshape(n0, n0)
    rho = P.sum(axis=1)
    sum_sq_outdeg = E + E * (E - 1) * float((rho ** 2).sum()) ** k
    outdeg0 = E * float(rho[0]) ** k
    # expected number of distinct cells hit: sum over digit-count compositions
    C = p.size
    logfact = [math.lgamma(i + 1) for i in range(k + 1)]
    distinct = 0.0

    def comps(rem, parts):
        if parts == 1:
            yield (rem,)
            return
        for a in range(rem + 1):
            for rest in comps(rem - a, parts - 1):
                yield (a,) + rest
    for a in comps(k, C):
        if any(a[c] > 0 and p[c] == 0 for c in range(C)):
            continue
        logmult = logfact[k] - sum(logfact[x] for x in a)
        logpi = sum(a[c] * math.log(p[c]) for c in range(C) if a[c])
        pi = math.exp(logpi)
        distinct += math.exp(logmult) * -math.expm1(E * math.log1p(-pi))
    return sum_sq_outdeg, outdeg0, E - distinct


def test_kron_k20_moments_and_duplicates(orc):
    """2x2 initiator, k = 20, 2^24 edges: second moment of the out-degree,
    the expected out-degree of vertex 0 and the expected number of repeated
    edges all match their closed forms (about 3.22e10, 6.93e4 and 6.91e5)."""
    c = wl.KRON_K20
    E, k = c["num_edges"], c["k"]
    src, dst = orc.kron_sample(2, c["initiator"], k, E, c["seed"])
    out = np.bincount(src, minlength=2 ** k).astype(np.float64)
    s2, d0, dups = _kron_stats_closed_forms(orc, c["initiator"], k, E)
    assert abs(s2 - 3.2201e10) / 3.2201e10 < 1e-3
    assert abs((out ** 2).sum() - s2) / s2 < 0.01
    assert abs(out[0] - d0) < 6 * math.sqrt(d0)
    _, _, got_dups = orc.edges_to_csr(2 ** k, src, dst)
    assert abs(got_dups - dups) / dups < 0.01, (got_dups, dups)
    assert abs(dups - 6.914e5) / 6.914e5 < 2e-3


def test_kron_tail_exponent_above_two(orc):
    """The paper observes gamma > 2 for its Kronecker graphs (Results, Fig. 3)."""
    c = wl.KRON_K20
    src, dst = orc.kron_sample(2, c["initiator"], 16, 1 << 20, 3)
    deg, _ = orc.degree_histogram(1 << 16, src, dst)
    g = orc.gamma_mle(deg, orc.gamma_dmin(1 << 16, 1 << 20))
    assert g > 2.0


# ----------------------------------------------------------------------------- Kronecker enumerate
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_kron_enumerate_equals_kronecker_power(orc, k):
    """The stack expansion of the Fig. 2 seed yields exactly the nonzeros of
    G1 (x) ... (x) G1: 121 edges on 25 vertices at k = 2 (Fig. 2(c)), 14,641
    edges on 625 vertices at k = 4 (Fig. 2(d))."""
    adj = wl.FIG2_SEED
    src, dst = orc.kron_enumerate(adj, k)
    G = adj
    for _ in range(k - 1):
        G = np.kron(G, adj)
    assert src.size == 11 ** k
    r, cidx = np.nonzero(G)
    assert set(zip(src.tolist(), dst.tolist())) == set(zip(r.tolist(), cidx.tolist()))
    assert len(set(zip(src.tolist(), dst.tolist()))) == src.size


@pytest.mark.parametrize("n0,k,density,seed", [(5, 3, None, 0), (4, 5, 0.5, 1), (7, 3, 0.3, 2)])
def test_kron_enumerate_stack_order(orc, n0, k, density, seed):
    """The depth-first stack emits edge e as the seed edges named by the
    base-e0 digits of e, most significant first (the order the GPU computes
    in closed form)."""
    if density is None:
        adj = wl.FIG2_SEED
    else:
        rng = np.random.default_rng(seed)
        adj = (rng.uniform(size=(n0, n0)) < density).astype(np.uint8)
        adj[0, 0] = 1
    nz = np.argwhere(adj)  # row-major
    e0 = len(nz)
    src, dst = orc.kron_enumerate(adj, k)
    e = np.arange(e0 ** k)
    u = np.zeros_like(e)
    v = np.zeros_like(e)
    for l in range(k):
        d = (e // e0 ** (k - 1 - l)) % e0
        u = u * n0 + nz[d, 0]
        v = v * n0 + nz[d, 1]
    np.testing.assert_array_equal(src, u)
    np.testing.assert_array_equal(dst, v)


# ----------------------------------------------------------------------------- PBA
def test_pba_fig1_replay(orc):
    """Fig. 1: P0's list starts with its faction members in order, copies
    earlier slots, requests 4 endpoints from P1 and 3 from P0 and P2, and
    substituting P1's list 8, 7, 5, 8 gives Fig. 1(b)."""
    fx = json.load(open(os.path.join(GOLDEN, "fig1_pba.json")))
    L, m = fx["vertices_per_partition"], fx["m"]
    F = fx["faction_list_P0"]
    script = fx["scripted_copy_indices_j4_to_j9"]
    lab = orc.pba_phase1(L * m, 0, 0.0, F, [3], seed=0, script=script)
    np.testing.assert_array_equal(lab, fx["fig1a_v_partition"])
    counts = np.bincount(lab, minlength=4)
    assert counts[0] == fx["counts_requested_from"]["P0"]
    assert counts[1] == fx["counts_requested_from"]["P1"]
    assert counts[2] == fx["counts_requested_from"]["P2"]
    start = np.array([0, 5, 10, 15, 20], np.uint64)
    S1 = np.array(fx["list_sent_by_P1"], np.uint32) - 5
    # lists of P0 and P2 are not shown in the figure: use markers 100+ to tell them apart
    S = np.concatenate([np.full(3, 95, np.uint32), S1, np.full(3, 90, np.uint32)])
    S_base = np.array([0, 3, 7, 10], np.uint64)
    dst = orc.pba_substitute(lab, 4, start, np.zeros(4, np.uint64), S_base, S)
    got = [str(d) if l == 1 else f"P{l}" for l, d in zip(lab, dst)]
    assert got == fx["fig1b_v"]
    src_row = np.arange(L * m) // m
    np.testing.assert_array_equal(src_row, fx["fig1a_u"])


def _check_pba_invariants(orc, n, m, P, p, seed, foff=None, fmem=None):
    src, dst, lab, cnt, S = orc.pba_generate(n, m, P, p, seed, 0, foff, fmem, extras=True)
    E = n * m
    assert src.size == E
    np.testing.assert_array_equal(src, np.arange(E) // m)  # every vertex owns m slots
    start = orc.partition_starts(n, P).astype(np.int64)
    L = np.diff(start)
    # rows of c sum to each partition's slot count; columns give D
    np.testing.assert_array_equal(cnt.sum(axis=1), L * m)
    D = cnt.sum(axis=0)
    # each edge's endpoint lies in the partition named by its label
    part_of_dst = np.searchsorted(start, dst, side="right") - 1
    np.testing.assert_array_equal(part_of_dst, lab.astype(np.int64))
    # phase 2 never attaches to a vertex that has not arrived yet
    base = np.concatenate([[0], np.cumsum(D)]).astype(np.int64)
    for l in range(P):
        t = np.arange(D[l])
        if D[l] == 0:
            continue
        x = (t * L[l]) // D[l]
        assert np.all(S[base[l]:base[l + 1]] <= np.maximum(1, x))
    # total degree is exactly 2 n m
    deg, _ = orc.degree_histogram(n, src, dst)
    assert deg.sum() == 2 * E
    return src, dst, lab, cnt


@pytest.mark.parametrize("n,m,P,p,seed", [(65536, 4, 64, 0.1, 1), (1001, 3, 7, 0.5, 2), (40, 2, 20, 1.0, 3),
                                          (500, 5, 1, 0.3, 4)])
def test_pba_invariants(orc, n, m, P, p, seed):
    _check_pba_invariants(orc, n, m, P, p, seed)


def test_pba_invariants_factions(orc):
    off = np.array([0, 4, 6, 7, 9], np.uint32)
    mem = np.array([1, 2, 0, 1, 1, 3, 2, 0, 3], np.uint32)
    _, _, lab, _ = _check_pba_invariants(orc, 4000, 2, 4, 0.2, 7, off, mem)
    # the first s slots of every partition are its faction list, in order
    start = orc.partition_starts(4000, 4).astype(np.int64)
    for q in range(4):
        F = mem[off[q]:off[q + 1]]
        np.testing.assert_array_equal(lab[2 * start[q]:2 * start[q] + len(F)], F)


def test_pba_empty_faction_rejected(orc):
    """Slot 0 of a partition with no faction member would have nothing earlier to copy."""
    with pytest.raises(ValueError):
        orc.pba_generate(40, 2, 4, 0.1, 1, 0, np.array([0, 1, 1, 2, 3], np.uint32), np.array([1, 2, 3], np.uint32))


def test_pba_p0_is_textbook_ba(orc):
    """With p = 0 and singleton factions every partition is an independent
    Barabasi-Albert graph grown from a 2-vertex clique by the edge-copy rule:
    vertex x = j // m arrives m times and attaches to a uniformly chosen
    endpoint of the edges so far.  A direct loop over the same draws matches."""
    n, m, P, seed = 600, 3, 3, 21
    src, dst = orc.pba_generate(n, m, P, 0.0, seed)
    start = orc.partition_starts(n, P).astype(np.int64)
    for q in range(P):
        L = int(start[q + 1] - start[q])
        pool = [0, 1]
        for j in range(L * m):
            w = orc.philox([j & 0xFFFFFFFF, j >> 32, q, 3], [seed & 0xFFFFFFFF, seed >> 32])
            U = int(w[0]) | (int(w[1]) << 32)
            y = pool[(U * len(pool)) >> 64]
            pool += [j // m, y]
            e = m * start[q] + j
            assert src[e] == start[q] + j // m
            assert dst[e] == start[q] + y


def test_pba_p0_degree_law(orc):
    """At p = 0 the degree distribution approaches the Barabasi-Albert law
    P(k) = 2m(m+1) / (k(k+1)(k+2)) (Bollobas et al. 2001; Dorogovtsev et al.
    2000), a power law with exponent 3."""
    n, m = 1 << 20, 3
    src, dst = orc.pba_generate(n, m, 1, 0.0, 99)
    deg, _ = orc.degree_histogram(n, src, dst)
    ks = np.arange(m, 31)
    emp = np.array([(deg == k).mean() for k in ks])
    theory = 2 * m * (m + 1) / (ks * (ks + 1) * (ks + 2))
    assert np.all(np.abs(emp / theory - 1) < 0.12), np.round(emp / theory, 3)
    g = orc.gamma_mle(deg, 4 * m)
    assert 2.7 < g < 3.3


def test_pba_polya_martingale(orc):
    """At p = 0 the share of a label with multiplicity a in a faction list of
    length s is a Polya urn: its expectation stays a / s."""
    P = 300
    off = np.arange(0, 3 * P + 1, 3, dtype=np.uint32)
    mem = np.array([[(q + 1) % P, (q + 1) % P, (q + 2) % P] for q in range(P)], np.uint32).ravel()
    src, dst, lab, cnt, S = orc.pba_generate(P * 50, 4, P, 0.0, 5, 0, off, mem, extras=True)
    share = np.array([cnt[q, (q + 1) % P] / cnt[q].sum() for q in range(P)])
    se = share.std(ddof=1) / math.sqrt(P)
    assert abs(share.mean() - 2 / 3) < 4 * se, (share.mean(), se)


def test_pba_urn_recursion(orc):
    """Copies may copy remote labels, so the realised remote share obeys
    E[R_{j+1}] = E[R_j] (1 + (1-p)/j) + p; for 4,096 slots and p = 0.1 that is
    0.547 (mean over the 64 partitions of the small configuration)."""
    c = wl.PBA_SMALL
    src, dst, lab, cnt, S = orc.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], c["seed"], extras=True)
    P = c["num_parts"]
    N = c["n"] // P * c["m"]
    R = 0.0
    for j in range(1, N):
        R = R * (1 + (1 - c["p_inter"]) / j) + c["p_inter"]
    expect = R / N
    assert abs(expect - 0.547) < 1e-3
    frac = np.array([1 - cnt[q, q] / cnt[q].sum() for q in range(P)])
    t = (frac.mean() - expect) / (frac.std(ddof=1) / math.sqrt(P))
    assert abs(t) < 4, (frac.mean(), expect)


# ----------------------------------------------------------------------------- CSR and degrees
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_csr_matches_numpy(orc, flags):
    rng = np.random.default_rng(40 + flags)
    n, E = 300, 5000
    src = rng.integers(0, n, size=E)
    dst = np.minimum(rng.zipf(1.6, size=E) - 1, n - 1)
    rp, col, dups = orc.edges_to_csr(n, src, dst, symmetrize=bool(flags & 1), simple=bool(flags & 2))
    s, d = (np.concatenate([src, dst]), np.concatenate([dst, src])) if flags & 1 else (src, dst)
    order = np.lexsort((d, s))
    s, d = s[order], d[order]
    key = s * n + d
    assert dups == int(np.sum(key[1:] == key[:-1]))
    if flags & 2:
        keep = np.ones(key.size, bool)
        keep[1:] = key[1:] != key[:-1]
        keep &= s != d
        s, d = s[keep], d[keep]
    np.testing.assert_array_equal(col, d)
    np.testing.assert_array_equal(rp, np.concatenate([[0], np.cumsum(np.bincount(s, minlength=n))]))


def test_degree_histogram_matches_numpy(orc):
    rng = np.random.default_rng(9)
    n, E = 1000, 20000
    src = np.minimum(rng.zipf(1.4, size=E) - 1, n - 1)
    dst = rng.integers(0, n, size=E)
    deg, hist = orc.degree_histogram(n, src, dst)
    np.testing.assert_array_equal(deg, np.bincount(src, minlength=n) + np.bincount(dst, minlength=n))
    bins = np.where(deg == 0, 0, np.minimum(31, np.floor(np.log2(np.maximum(deg, 1))).astype(int) + 1))
    np.testing.assert_array_equal(hist, np.bincount(bins, minlength=32))


# ----------------------------------------------------------------------------- statistics
def test_gamma_closed_form_constant_degrees(orc):
    d_min = 8
    deg = np.full(1000, d_min, np.uint64)
    assert abs(orc.gamma_mle(deg, d_min) - (1 + 1 / math.log(d_min / (d_min - 0.5)))) < 1e-12


@pytest.mark.parametrize("alpha", [2.2, 2.5, 3.0])
def test_gamma_recovers_power_law(orc, alpha):
    """Degrees drawn from a power law with exponent alpha above d_min: the
    estimator recovers alpha (Clauset, Shalizi & Newman 2009)."""
    rng = np.random.default_rng(int(alpha * 10))
    d_min = 10
    x = (d_min - 0.5) * (1 - rng.uniform(size=1_000_000)) ** (-1 / (alpha - 1))
    deg = np.floor(x + 0.5).astype(np.uint64)
    g = orc.gamma_mle(deg, d_min)
    assert abs(g - alpha) < 0.02, g


def _transitivity(n, rp, col):
    A = np.zeros((n, n), np.int64)
    for v in range(n):
        A[v, col[rp[v]:rp[v + 1]]] = 1
    tri = np.trace(A @ A @ A) / 6
    d = A.sum(1)
    wedges = (d * (d - 1) // 2).sum()
    return 3 * tri / wedges


def _simple_undirected_numpy(n, src, dst):
    """Row starts and columns of the simple undirected graph: both
    orientations of every non-loop edge, repeats removed (numpy.unique)."""
    u = np.concatenate([src, dst]).astype(np.int64)
    v = np.concatenate([dst, src]).astype(np.int64)
    keep = u != v
    key = np.unique(u[keep] * n + v[keep])
    rows, cols = key // n, key % n
    return np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.uint64), cols


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_simple_csr_matches_numpy_unique(orc, seed):
    """The simple undirected graph the wedge statistics run on: self-loops
    dropped, both orientations, every pair once.  Inputs carry many
    self-loops and repeated pairs in both orientations."""
    rng = np.random.default_rng(300 + seed)
    n, E = 64, 3000
    src = rng.integers(0, n, size=E)
    dst = np.where(rng.uniform(size=E) < 0.2, src, rng.integers(0, n, size=E))  # ~20 % self-loops
    dup = rng.integers(0, E, size=E // 4)
    src = np.concatenate([src, dst[dup], src[dup]])  # repeats, reversed and straight
    dst = np.concatenate([dst, src[dup], dst[dup]])
    assert np.any(src == dst)
    rp, col = orc.simple_csr(n, src, dst)
    erp, ecol = _simple_undirected_numpy(n, src, dst)
    np.testing.assert_array_equal(rp, erp)
    np.testing.assert_array_equal(col, ecol)
    assert not np.any(np.repeat(np.arange(n), np.diff(rp.astype(np.int64))) == col)  # no loop survives
    # the same graph through the general CSR with SYMMETRIZE | SIMPLE
    rp2, col2, _ = orc.edges_to_csr(n, src, dst, symmetrize=True, simple=True)
    np.testing.assert_array_equal(rp2, erp)
    np.testing.assert_array_equal(col2, ecol)


def _wedge_boundary_graph():
    """A small simple graph whose vertex order puts vertices without wedges
    (degree 0 or 1) first and right after each boundary of the cumulative
    C(d, 2) list, so that sampled indices equal to a prefix value are common."""
    edges = [(0, 1), (1, 4), (4, 5), (4, 6), (5, 6), (6, 8), (3, 8), (8, 9), (9, 10), (10, 11), (12, 13),
             (13, 14), (14, 12), (14, 15)]
    n = 17  # vertices 2, 7 and 16 are isolated
    a = np.array(edges, np.int64)
    return n, a[:, 0], a[:, 1]


@pytest.mark.parametrize("case", ["boundary", "random_sparse"])
def test_wedge_centres_brute_force(orc, case):
    """Every sampled centre is the vertex the definition picks: the first
    vertex whose inclusive running sum of C(d, 2) exceeds the sampled index
    floor(U acc / 2^64), found here by a plain linear scan.  Every centre has
    degree >= 2, its two ends are distinct neighbours, and 'closed' is the
    adjacency of the two ends (a set lookup)."""
    if case == "boundary":
        n, src, dst = _wedge_boundary_graph()
    else:
        rng = np.random.default_rng(77)
        n = 400
        src = rng.integers(0, n, size=300)
        dst = rng.integers(0, n, size=300)
    rp, col = orc.simple_csr(n, src, dst)
    rp = rp.astype(np.int64)
    nbrs = [set(col[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
    deg = [len(s) for s in nbrs]
    cum, acc = [], 0
    for d in deg:
        acc += d * (d - 1) // 2
        cum.append(acc)
    N, seed, gid = 4000, 29, 3
    closed, draws = orc.wedge_draws(n, rp.astype(np.uint64), col, N, seed, gid)
    expect_closed = 0
    for i in range(N):
        w = orc.philox([i, 0, 0, 4 | (gid << 8)], [seed & 0xFFFFFFFF, seed >> 32])
        U = int(w[0]) | (int(w[1]) << 32)
        target = (U * acc) >> 64
        v = 0
        while cum[v] <= target:
            v += 1
        c, a, b = (int(x) for x in draws[i])
        assert c == v, (i, target, c, v)
        assert deg[c] >= 2
        assert a != b and a in nbrs[c] and b in nbrs[c]
        expect_closed += b in nbrs[a]
    assert closed == expect_closed
    assert closed == orc.wedge_closed(n, rp.astype(np.uint64), col, N, seed, gid)


def test_wedges_special_graphs(orc):
    # complete graph: every wedge closed; star and cycle: none
    n = 12
    u, v = np.triu_indices(n, 1)
    rp, col = orc.simple_csr(n, u, v)
    assert orc.wedge_closed(n, rp, col, 10_000, 1) == 10_000
    rp, col = orc.simple_csr(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    assert orc.wedge_closed(n, rp, col, 10_000, 1) == 0
    rp, col = orc.simple_csr(n, np.arange(n), (np.arange(n) + 1) % n)
    assert orc.wedge_closed(n, rp, col, 10_000, 1) == 0
    rp, col = orc.simple_csr(3, np.array([0]), np.array([1]))
    assert orc.wedge_closed(3, rp, col, 10, 1) == -1  # no wedge at all


def test_wedges_estimate_transitivity(orc):
    """The closed share of sampled wedges estimates the global clustering
    coefficient 3 x triangles / wedges (binomial tolerance)."""
    rng = np.random.default_rng(5)
    n = 200
    src = rng.integers(0, n, size=1500)
    dst = (src + rng.integers(1, 8, size=1500)) % n
    rp, col = orc.simple_csr(n, src, dst)
    tau = _transitivity(n, rp, col)
    N = 10_000
    closed = orc.wedge_closed(n, rp, col, N, 17)
    sd = math.sqrt(N * tau * (1 - tau))
    assert abs(closed - N * tau) < 5 * sd, (closed, N * tau)


# --------------------------------------------------------------------------- sampled path statistics
def _csr_of_undirected(n, pairs):
    """Simple undirected CSR of an explicit edge list (numpy, independent of the oracle)."""
    if len(pairs):
        a = np.array(pairs, np.int64)
        u = np.concatenate([a[:, 0], a[:, 1]])
        v = np.concatenate([a[:, 1], a[:, 0]])
        keep = u != v
        key = np.unique(u[keep] * n + v[keep])
        u, v = key // n, key % n
    else:
        u = v = np.zeros(0, np.int64)
    rp = np.zeros(n + 1, np.uint64)
    np.add.at(rp, u + 1, 1)
    return np.cumsum(rp).astype(np.uint64), v.astype(np.int64)


def test_path_stats_closed_forms(orc):
    # path P_n from one end: distances 1..n-1
    n = 50
    rp, col = _csr_of_undirected(n, [(i, i + 1) for i in range(n - 1)])
    assert orc.path_stats(n, rp, col, [0]) == (n * (n - 1) // 2, n - 1, n - 1)
    # cycle C_n: two vertices at every distance below n/2, one at n/2 when n is even
    for n in (9, 10):
        rp, col = _csr_of_undirected(n, [(i, (i + 1) % n) for i in range(n)])
        h = (n - 1) // 2
        want = 2 * h * (h + 1) // 2 + (n // 2 if n % 2 == 0 else 0)
        assert orc.path_stats(n, rp, col, [3]) == (want, n - 1, n // 2)
    # star: centre 0; a leaf sees the centre at 1 and the other leaves at 2
    n = 12
    rp, col = _csr_of_undirected(n, [(0, i) for i in range(1, n)])
    assert orc.path_stats(n, rp, col, [0]) == (n - 1, n - 1, 1)
    assert orc.path_stats(n, rp, col, [5]) == (1 + 2 * (n - 2), n - 1, 2)
    # hypercube Q_d: distance = Hamming distance, summing to d 2^(d-1)
    d = 7
    n = 1 << d
    rp, col = _csr_of_undirected(n, [(v, v ^ (1 << b)) for v in range(n) for b in range(d)])
    assert orc.path_stats(n, rp, col, [0, 77]) == (2 * d * (1 << (d - 1)), 2 * (n - 1), d)
    # two components: only reachable pairs count
    rp, col = _csr_of_undirected(6, [(0, 1), (1, 2), (3, 4)])
    assert orc.path_stats(6, rp, col, [0, 3, 5]) == (1 + 2 + 1, 3, 2)


def test_path_stats_match_scipy_bfs(orc):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(8)
    for n, m in ((60, 90), (200, 260), (300, 2000)):
        pairs = list(zip(rng.integers(0, n, m), rng.integers(0, n, m)))
        rp, col = _csr_of_undirected(n, pairs)
        A = csr_matrix((np.ones(col.size), col, rp.astype(np.int64)), shape=(n, n))
        srcs = rng.integers(0, n, 7)
        D = shortest_path(A, method="D", unweighted=True, indices=srcs)
        fin = np.isfinite(D) & (D > 0)
        want = (int(D[fin].sum()), int(fin.sum()), int(D[fin].max()) if fin.any() else 0)
        assert orc.path_stats(n, rp, col, srcs) == want


# --------------------------------------------------------------------------- communities (block matrix)
def test_block_matrix_of_kronecker_power_is_a_kronecker_power(orc):
    # The deterministic Kronecker power of a 0/1 seed: coarsened to n0^l
    # blocks, every nonzero cell of the l-th power of the seed holds the
    # e0^(k-l) edges expanded from it -- the communities within communities.
    from paper_1003_3684_amd import workloads as wl
    seed = wl.FIG2_SEED
    n0, e0, k = seed.shape[0], int(seed.sum()), 4
    src, dst = orc.kron_enumerate(seed, k)
    n = n0 ** k
    power = np.ones((1, 1), np.int64)
    for l in range(0, k + 1):
        B = n0 ** l
        got = orc.block_matrix(n, src, dst, B)
        np.testing.assert_array_equal(got, power * e0 ** (k - l))
        power = np.kron(power, seed.astype(np.int64))


def test_block_matrix_uneven_blocks(orc):
    # n = 10 vertices in B = 3 blocks: vertex v is in block floor(3 v / 10),
    # so the blocks are {0..3}, {4..6}, {7..9}.
    src = np.array([0, 3, 4, 6, 7, 9, 9], np.int64)
    dst = np.array([9, 4, 3, 6, 0, 7, 9], np.int64)
    want = np.array([[0, 1, 1],
                     [1, 1, 0],
                     [1, 0, 2]], np.uint64)
    np.testing.assert_array_equal(orc.block_matrix(10, src, dst, 3), want)
    assert orc.block_matrix(10, src, dst, 1)[0, 0] == 7


# --------------------------------------------------------------------------- randomized PK by XOR
def _dense(n, rp, col):
    A = np.zeros((n, n), np.uint8)
    for u in range(n):
        A[u, col[int(rp[u]):int(rp[u + 1])]] = 1
    return A


def test_kron_xor_random_brute_force(orc):
    # Adjacency of the Kronecker power by numpy.kron, the random graph from
    # the Philox primitive and the uidx map directly (uidx(U, R) =
    # floor(U R / 2^64), checked here with Python integers), XOR elementwise.
    seed_m = np.array([[1, 1, 0], [1, 0, 1], [0, 1, 1]], np.uint8)
    k, M, seed, gid = 3, 400, 77, 5
    n = 3 ** k
    A = np.ones((1, 1), np.uint8)
    for _ in range(k):
        A = np.kron(A, seed_m)
    R = np.zeros((n, n), np.uint8)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(M):
        w = orc.philox([i & 0xFFFFFFFF, i >> 32, 0, 6 | (gid << 8)], key)
        a = ((int(w[0]) | (int(w[1]) << 32)) * n) >> 64
        b = ((int(w[2]) | (int(w[3]) << 32)) * n) >> 64
        R[a, b] = 1
    rp, col = orc.kron_xor_random(seed_m, k, M, seed, gid)
    np.testing.assert_array_equal(_dense(n, rp, col), A ^ R)
    # columns ascending within every row
    for u in range(n):
        c = col[int(rp[u]):int(rp[u + 1])]
        assert np.all(np.diff(c) > 0)
    assert len(col) == int(A.sum()) + int(R.sum()) - 2 * int((A & R).sum())


def test_kron_xor_without_random_graph_is_the_power(orc):
    from paper_1003_3684_amd import workloads as wl
    rp, col = orc.kron_xor_random(wl.FIG2_SEED, 2, 0, 1)
    A = np.kron(wl.FIG2_SEED, wl.FIG2_SEED)
    np.testing.assert_array_equal(_dense(25, rp, col), A)


# --------------------------------------------------------------------------- randomized PK by seed modification
def test_perturbed_without_changes_is_the_power(orc):
    from paper_1003_3684_amd import workloads as wl
    s0, d0 = orc.kron_enumerate(wl.FIG2_SEED, 4)
    s1, d1 = orc.kron_perturbed(wl.FIG2_SEED, 4, 0.0, 0.0, 5)
    np.testing.assert_array_equal(s0, s1)
    np.testing.assert_array_equal(d0, d1)


def test_perturbed_extremes_are_kronecker_products(orc):
    # p_add = p_del = 1 flips every cell at every expansion: the graph is
    # seed (x) complement (x) ... (x) complement.  p_del = 1, p_add = 0
    # deletes everything below the first iteration.
    seed_m = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 0]], np.uint8)
    k = 4
    comp = 1 - seed_m
    A = seed_m.astype(np.int64)
    for _ in range(k - 1):
        A = np.kron(A, comp)
    s, d = orc.kron_perturbed(seed_m, k, 1.0, 1.0, 9)
    n = 3 ** k
    got = np.zeros((n, n), np.int64)
    got[s, d] += 1
    np.testing.assert_array_equal(got, A)
    s, d = orc.kron_perturbed(seed_m, k, 0.0, 1.0, 9)
    assert s.size == 0
    s, d = orc.kron_perturbed(seed_m, 1, 0.7, 0.7, 9)  # one level: the seed itself
    assert s.size == int(seed_m.sum())


def test_perturbed_subset_and_expected_size(orc):
    from paper_1003_3684_amd import workloads as wl
    seed_m = wl.FIG2_SEED
    n0, e0, k = 5, 11, 5
    n = n0 ** k
    base = set(zip(*orc.kron_enumerate(seed_m, k)))
    # additions only: a superset of the power; deletions only: a subset
    up = set(zip(*orc.kron_perturbed(seed_m, k, 0.02, 0.0, 3)))
    down = set(zip(*orc.kron_perturbed(seed_m, k, 0.0, 0.1, 3)))
    assert base < up and down < base
    # every meta-edge expands independently: E|G_k| = e0 f^(k-1) with
    # f = e0 (1 - p_del) + (n0^2 - e0) p_add
    p_add, p_del = 0.05, 0.1
    f = e0 * (1 - p_del) + (n0 * n0 - e0) * p_add
    sizes = [orc.kron_perturbed(seed_m, k, p_add, p_del, s)[0].size for s in range(24)]
    assert abs(np.mean(sizes) / (e0 * f ** (k - 1)) - 1) < 0.04
    # distinct meta-edges give distinct edges
    s, d = orc.kron_perturbed(seed_m, k, p_add, p_del, 1)
    assert np.unique(s * n + d).size == s.size


# ----------------------------------------------------------------------------- PBA brute force
# Tiny instances whose every outcome is enumerated with its exact probability
# from the process as the PBA section states it (phase 1: the faction prefix,
# then an inter-faction draw with probability p or a copy of a uniformly
# chosen earlier slot; phase 2: preferential attachment grown from a 2-vertex
# clique, each endpoint a uniform pick from the endpoints so far;
# substitution in slot order), written here as a probability tree rather
# than a simulation, against the oracle's outcome frequencies over seeds.

def _exact_p(p):
    return Fraction(int(math.floor(p * 2 ** 32)), 2 ** 32)  # the Bernoulli threshold over 2^32


def _phase1_tree(nslots, q, other, pe):
    """{labels: probability} for one partition with F(q) = [q] and one
    non-faction partition `other`."""
    out = {}

    def rec(lab, pr):
        j = len(lab)
        if j == nslots:
            out[tuple(lab)] = out.get(tuple(lab), 0) + pr
            return
        if j == 0:
            return rec([q], pr)
        rec(lab + [other], pr * pe)
        for i in range(j):
            rec(lab + [lab[i]], pr * (1 - pe) / j)

    rec([], Fraction(1))
    return out


def _phase2_tree(D, L):
    """{S: probability}: arrival t is local vertex floor(t L / D); its
    endpoint is one of the 2 + 2t pool entries, uniformly."""
    out = {}

    def rec(pool, S, pr):
        t = len(S)
        if t == D:
            out[tuple(S)] = out.get(tuple(S), 0) + pr
            return
        x = t * L // D
        for y in pool:
            rec(pool + [x, y], S + [y], pr / len(pool))

    rec([0, 1], [], Fraction(1))
    return out


def _chi2_against(exact, observed, n):
    cats = sorted(exact, key=lambda k: -exact[k])
    exp = np.array([float(exact[c]) * n for c in cats])
    obs = np.array([observed.get(c, 0) for c in cats], np.float64)
    assert set(observed) <= set(exact), "an outcome of probability zero occurred"
    big = exp >= 5
    e = np.append(exp[big], exp[~big].sum())
    o = np.append(obs[big], obs[~big].sum())
    if e[-1] == 0:
        e, o = e[:-1], o[:-1]
    return stats.chisquare(o, e).pvalue


def test_pba_phase1_brute_force(orc):
    pe = _exact_p(0.3)
    exact = _phase1_tree(4, 0, 1, pe)
    assert sum(exact.values()) == 1
    n = 30000
    seen = {}
    for s in range(n):
        lab = tuple(int(x) for x in orc.pba_phase1(4, 0, 0.3, [0], [1], s))
        seen[lab] = seen.get(lab, 0) + 1
    assert _chi2_against(exact, seen, n) > 1e-3


def test_pba_phase2_brute_force(orc):
    exact = _phase2_tree(4, 3)
    assert sum(exact.values()) == 1
    n = 30000
    seen = {}
    for s in range(n):
        S = tuple(int(x) for x in orc.pba_phase2(4, 3, 1, s))
        seen[S] = seen.get(S, 0) + 1
    assert _chi2_against(exact, seen, n) > 1e-3


def test_pba_whole_graph_brute_force(orc):
    """P = 2 partitions of L = 2 vertices, m = 1, p = 0.3: the exact law of the
    whole destination list."""
    pe = _exact_p(0.3)
    L, start = 2, [0, 2]
    exact = {}
    t0, t1 = _phase1_tree(2, 0, 1, pe), _phase1_tree(2, 1, 0, pe)
    for (l0, p0), (l1, p1) in product(t0.items(), t1.items()):
        labels = [list(l0), list(l1)]
        D = [sum(row.count(l) for row in labels) for l in range(2)]
        # requester q's share of partition l's list starts after the shares
        # of the requesters before it (ascending order)
        off = [[sum(labels[r].count(l) for r in range(q)) for l in range(2)] for q in range(2)]
        for (S0, a0), (S1, a1) in product(_phase2_tree(D[0], L).items() if D[0] else [((), 1)],
                                          _phase2_tree(D[1], L).items() if D[1] else [((), 1)]):
            S = [S0, S1]
            dst = []
            for q in range(2):
                used = [0, 0]
                for l in labels[q]:
                    dst.append(start[l] + S[l][off[q][l] + used[l]])
                    used[l] += 1
            key = tuple(dst)
            exact[key] = exact.get(key, 0) + p0 * p1 * a0 * a1
    assert sum(exact.values()) == 1
    n = 30000
    seen = {}
    for s in range(n):
        _, dst = orc.pba_generate(4, 1, 2, 0.3, s)
        key = tuple(int(x) for x in dst)
        seen[key] = seen.get(key, 0) + 1
    assert _chi2_against(exact, seen, n) > 1e-3
