"""GPU parity of edges_to_csr against the oracle (bit-exact rows, columns,
duplicate counts and degree histograms)."""
import numpy as np
import pytest

from paper_1003_3684_amd import workloads as wl

pytestmark = pytest.mark.gpu

FLAG_SETS = [0, 1, 2, 3]  # directed, symmetrized, simple, symmetrized+simple


def _gpu_csr(sfg, n, src_np, dst_np, flags, id_bytes):
    import torch
    dt = torch.int32 if id_bytes == 4 else torch.int64
    src = torch.as_tensor(np.asarray(src_np), dtype=dt).cuda()
    dst = torch.as_tensor(np.asarray(dst_np), dtype=dt).cuda()
    rp, col, hist, dups = sfg.edges_to_csr(n, src, dst, flags=flags)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    return rp.cpu().numpy(), col.cpu().numpy(), hist.cpu().numpy(), int(dups.item())


def _check(sfg, orc, n, src, dst, flags, id_bytes):
    rp, col, hist, dups = _gpu_csr(sfg, n, src, dst, flags, id_bytes)
    orp, ocol, odups = orc.edges_to_csr(n, src, dst, symmetrize=bool(flags & 1), simple=bool(flags & 2))
    _, ohist = orc.degree_histogram(n, src, dst)
    np.testing.assert_array_equal(rp.astype(np.uint64), orp)
    kept = int(orp[-1])
    np.testing.assert_array_equal(col[:kept].astype(np.int64), ocol)
    assert dups == odups
    np.testing.assert_array_equal(hist.astype(np.uint64), ohist)


@pytest.mark.parametrize("flags", FLAG_SETS)
def test_csr_kron_k20(sfg, orc, flags):
    """The 2^24-edge Kronecker graph: directed CSR with about 691 k repeated edges."""
    c = wl.KRON_K20
    src, dst = orc.kron_sample(c["n0"], c["initiator"], c["k"], c["num_edges"], c["seed"])
    _check(sfg, orc, c["n0"] ** c["k"], src, dst, flags, 4)


@pytest.mark.parametrize("flags", FLAG_SETS)
def test_csr_pba_small(sfg, orc, flags):
    c = wl.PBA_SMALL
    src, dst = orc.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], c["seed"])
    _check(sfg, orc, c["n"], src, dst, flags, 4)


@pytest.mark.parametrize("trial", range(16))
def test_csr_random(sfg, orc, trial):
    rng = np.random.default_rng(500 + trial)
    n = int(rng.choice([1, 2, 3, 17, 1000, 65536, 65537, 1 << 20, (1 << 24) + 3]))
    E = int(rng.choice([0, 1, 5, 8191, 8192, 8193, 100_000, 300_001]))
    id_bytes = 8 if trial % 2 else 4
    if rng.uniform() < 0.5:  # skewed ids, many repeats and self-loops
        src = np.minimum(rng.zipf(1.5, size=E) - 1, n - 1)
        dst = np.minimum(rng.zipf(1.8, size=E) - 1, n - 1)
    else:
        src = rng.integers(0, n, size=E)
        dst = rng.integers(0, n, size=E)
    flags = int(rng.integers(0, 4))
    _check(sfg, orc, n, src.astype(np.int64), dst.astype(np.int64), flags, id_bytes)


def test_csr_wide_ids(sfg):
    """n = 2^31 - 1 (62 live key bits): columns match a lexicographic sort and
    row starts match binary searches at sampled rows (row_ptr stays on the GPU)."""
    import torch
    rng = np.random.default_rng(3)
    n = (1 << 31) - 1
    E = 50_000
    src = np.concatenate([rng.integers(n - 1000, n, size=E - 10), np.full(10, n - 1)])
    dst = rng.integers(0, n, size=E)
    s = torch.as_tensor(src, dtype=torch.int64).cuda()
    d = torch.as_tensor(dst, dtype=torch.int64).cuda()
    rp, col, hist, dups = sfg.edges_to_csr(n, s, d, flags=0)
    torch.cuda.synchronize()
    order = np.lexsort((dst, src))
    np.testing.assert_array_equal(col.cpu().numpy(), dst[order])
    ss = src[order]
    rows = np.concatenate([[0, 1, n - 1001, n - 1, n], rng.integers(n - 1100, n, size=200)])
    got = rp[torch.as_tensor(rows).cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, np.searchsorted(ss, rows, side="left"))
    key = src * n + dst
    assert int(dups.item()) == E - len(np.unique(key))
    del rp
    torch.cuda.empty_cache()


def test_csr_all_loops_and_empty(sfg, orc):
    n = 10
    src = np.array([3, 3, 3, 7, 7], np.int64)
    dst = src.copy()
    for flags in FLAG_SETS:
        _check(sfg, orc, n, src, dst, flags, 4)
    for flags in FLAG_SETS:
        _check(sfg, orc, n, np.zeros(0, np.int64), np.zeros(0, np.int64), flags, 4)


@pytest.mark.parametrize("order", ["ascending", "descending", "blocks"])
@pytest.mark.parametrize("flags", [0, 1])
def test_csr_sorted_inputs(sfg, orc, order, flags):
    """Inputs already ordered by source (or in reverse, or in sorted blocks):
    each digit value of the last pass sits in a few tiles only, so most
    tiles' runs follow a run of an earlier, non-adjacent tile or of another
    digit -- the cases the last pass settles after the sort."""
    rng = np.random.default_rng({"ascending": 1, "descending": 2, "blocks": 3}[order] + 10 * flags)
    n, E = (1 << 20) + 5, 200_003
    src = rng.integers(0, n, size=E)
    dst = rng.integers(0, n, size=E)
    if order == "ascending":
        src = np.sort(src)
    elif order == "descending":
        src = np.sort(src)[::-1].copy()
    else:
        src = np.concatenate([np.sort(b) for b in np.array_split(src, 7)])
    dst[::97] = src[::97]  # some self-loops
    dst[1::89] = dst[0:-1:89][: len(dst[1::89])]  # some repeated pairs next to each other
    src[1::89] = src[0:-1:89][: len(src[1::89])]
    for ib in (4, 8):
        _check(sfg, orc, n, src, dst, flags, ib)


def test_entry_count_limit(sfg):
    """More than 2^34 entries (edges, doubled when symmetrized) is ERANGE,
    found before any buffer is touched: with one workgroup per tile a
    dispatch's work-item count stays below 2^32."""
    import torch
    lib = sfg.load()
    t = torch.zeros(64, dtype=torch.int64, device="cuda")
    p = t.data_ptr()
    for num_edges, flags in (((1 << 34) + 1, 0), ((1 << 33) + 1, sfg.CSR_SYMMETRIZE)):
        rc = lib.edges_to_csr(1000, num_edges, p, p, 8, flags, p, p, None, None, p, 1 << 62, None)
        assert rc == sfg.SFG_ERANGE, (num_edges, flags, rc)
    torch.cuda.synchronize()
    assert int(t.abs().sum().item()) == 0
