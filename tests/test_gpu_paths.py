"""Sampled shortest-path statistics (Results, Table 2) on the GPU against the
oracle's breadth-first searches and against closed forms: sums of distances,
reachable pairs and the largest distance must agree exactly."""
import numpy as np
import pytest

from paper_1003_3684_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _undirected_csr(n, pairs):
    a = np.array(pairs, np.int64).reshape(-1, 2)
    u = np.concatenate([a[:, 0], a[:, 1]])
    v = np.concatenate([a[:, 1], a[:, 0]])
    keep = u != v
    key = np.unique(u[keep] * n + v[keep])
    u, v = key // n, key % n
    rp = np.zeros(n + 1, np.uint64)
    np.add.at(rp, u + 1, 1)
    return np.cumsum(rp).astype(np.uint64), v.astype(np.int64)


def _gpu(sfg, n, rp, col, sources, id_bytes=4):
    import torch
    rp_d = torch.tensor(rp.astype(np.int64), device="cuda")
    col_d = torch.tensor(col.astype(np.int32 if id_bytes == 4 else np.int64), device="cuda")
    if col_d.numel() == 0:
        col_d = torch.zeros(1, dtype=col_d.dtype, device="cuda")
    out = sfg.path_stats(n, rp_d, col_d, sources)
    torch.cuda.synchronize()
    return tuple(int(x) for x in out.cpu().numpy())


@pytest.mark.parametrize("id_bytes", [4, 8])
def test_closed_forms(sfg, orc, id_bytes):
    n = 50
    rp, col = _undirected_csr(n, [(i, i + 1) for i in range(n - 1)])
    assert _gpu(sfg, n, rp, col, [0], id_bytes) == (n * (n - 1) // 2, n - 1, n - 1)
    # star with a heavy centre (degree above the one-lane limit)
    n = 1001
    rp, col = _undirected_csr(n, [(0, i) for i in range(1, n)])
    assert _gpu(sfg, n, rp, col, [0, 7], id_bytes) == ((n - 1) + 1 + 2 * (n - 2), 2 * (n - 1), 2)
    d = 7
    n = 1 << d
    rp, col = _undirected_csr(n, [(v, v ^ (1 << b)) for v in range(n) for b in range(d)])
    srcs = list(range(0, n, 3))  # 43 sources
    assert _gpu(sfg, n, rp, col, srcs, id_bytes) == (len(srcs) * d * (1 << (d - 1)), len(srcs) * (n - 1), d)
    rp, col = _undirected_csr(6, [(0, 1), (1, 2), (3, 4)])
    assert _gpu(sfg, 6, rp, col, [0, 3, 5, 5], id_bytes) == (4, 3, 2)


@pytest.mark.parametrize("kind", ["pba", "kron"])
def test_generated_graphs_match_oracle(sfg, orc, kind):
    import torch
    if kind == "pba":
        n, E = 6000, 6000 * 3
        src, dst = sfg.pba_generate(n, 3, 8, 0.2, seed=5)
    else:
        k = 12
        n, E = 1 << k, 16 << k
        src, dst = sfg.kron_generate(2, [[0.57, 0.19], [0.19, 0.05]], k, E, seed=9)
    rp, col, _, _ = sfg.edges_to_csr(n, src, dst, flags=sfg.CSR_SYMMETRIZE | sfg.CSR_SIMPLE)
    torch.cuda.synchronize()
    kept = int(rp[-1])
    sources = np.random.default_rng(2).integers(0, n, 150)  # three groups, the last partial
    out = sfg.path_stats(n, rp, col[:max(kept, 1)], sources)
    torch.cuda.synchronize()
    got = tuple(int(x) for x in out.cpu().numpy())
    want = orc.path_stats(n, rp.cpu().numpy().astype(np.uint64), col[:kept].cpu().numpy().astype(np.int64), sources)
    assert got == want
    assert want[1] > 0 and 1 <= want[2] < 64


def test_errors(sfg):
    import torch
    from paper_1003_3684_amd.native import SfgenError
    rp, col = _undirected_csr(4, [(0, 1), (2, 3)])
    rp_d = torch.tensor(rp.astype(np.int64), device="cuda")
    col_d = torch.tensor(col.astype(np.int32), device="cuda")
    with pytest.raises(SfgenError):
        sfg.path_stats(4, rp_d, col_d, [4])
    with pytest.raises(SfgenError):
        sfg.path_stats(4, rp_d, col_d, [0], ws=sfg.workspace(8))
    assert _gpu(sfg, 4, rp, col, []) == (0, 0, 0)
