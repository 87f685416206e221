"""edges_to_csr at full size, in the configurations the benchmark runs, checked
on the GPU by invariants that pin the CSR exactly (no CPU sort of billions
of entries is needed):

* the benchmark step: 5 x 2^30 Kronecker edges (3x3 initiator padded to
  4x4, 15 levels, int64 ids) generated and sorted by the one-call
  kron_generate_csr (the sampler counts the sort's histogram), directed CSR
  with duplicate count and degree histogram: sampled edges equal the
  oracle's, row starts are the exclusive scan of the source counts, every
  row is sorted, the multiset of (row, column) equals that of (src, dst)
  (64-bit sum of a mixing function of the packed pair), the duplicate count
  equals the repeated sorted positions, and the histogram equals the one of
  out-degree + in-degree;
* the PBA workload at 2^27 vertices: symmetrized simple CSR: no self-loops,
  strictly increasing rows, and the entry set equals the distinct non-loop
  pairs of the edge list in both directions."""
import numpy as np
import pytest

from paper_1003_3684_amd import workloads as wl

pytestmark = pytest.mark.gpu

CH = 1 << 28  # elements per chunk of the checks


def _mix(x):
    """A fixed 64-bit mixing function (wrapping int64 arithmetic)."""
    import torch
    x = x * 0x5DEECE66D + 0xB
    x = x ^ (x >> 29)
    x = x * -7046029254386353131
    return x ^ (x >> 32)


def _hash_pairs(a, b, shift):
    import torch
    tot = torch.zeros((), dtype=torch.int64, device=a.device)
    for i in range(0, a.numel(), CH):
        tot += _mix(a[i:i + CH].long() * (1 << shift) + b[i:i + CH].long()).sum()
    return int(tot)


def _counts(ids, n):
    import torch
    c = torch.zeros(n, dtype=torch.int64, device=ids.device)
    for i in range(0, ids.numel(), CH):
        c += torch.bincount(ids[i:i + CH].long(), minlength=n)
    return c


def _row_hash(rp, col, n, shift, rows=1 << 24):
    """Sum of _mix(row << shift | col) over the CSR entries, rows in blocks."""
    import torch
    tot = torch.zeros((), dtype=torch.int64, device=col.device)
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        lo, hi = int(rp[r0]), int(rp[r1])
        if hi == lo:
            continue
        cnt = rp[r0 + 1:r1 + 1] - rp[r0:r1]
        row = torch.repeat_interleave(torch.arange(r0, r1, device=col.device), cnt)
        tot += _mix(row * (1 << shift) + col[lo:hi].long()).sum()
    return int(tot)


def _row_starts_mask(rp, n, total):
    import torch
    starts = torch.zeros(total, dtype=torch.bool, device=rp.device)
    nonempty = rp[1:] > rp[:-1]
    starts[rp[:-1][nonempty]] = True
    return starts


def _sampled_edges(orc, c, src, dst, chunk=4096, n_random=500):
    """Chunks at the start, across 2^32 and at the ragged end, and random
    single edges, each equal to the oracle's."""
    import torch
    E = c["num_edges"]
    for s in (0, (1 << 32) - chunk // 2, E - chunk):
        os_, od = orc.kron_sample(c["n0"], c["initiator"], c["k"], chunk, c["seed"], 0, e_begin=s)
        np.testing.assert_array_equal(src[s:s + chunk].cpu().numpy(), os_)
        np.testing.assert_array_equal(dst[s:s + chunk].cpu().numpy(), od)
    idx = np.sort(np.random.default_rng(c["seed"] + 1).integers(0, E, size=n_random))
    gi = torch.as_tensor(idx, device="cuda")
    gs, gd = src[gi].cpu().numpy(), dst[gi].cpu().numpy()
    for j, e in enumerate(idx):
        os_, od = orc.kron_sample(c["n0"], c["initiator"], c["k"], 1, c["seed"], 0, e_begin=int(e))
        assert gs[j] == os_[0] and gd[j] == od[0], int(e)


@pytest.mark.timeout(900)
def test_bench_csr_at_full_size(sfg, orc):
    import torch
    c = wl.KRON_SCALE
    n, E = c["n0"] ** c["k"], c["num_edges"]
    print(f"case {c['name']}: n={n} E={E}", flush=True)
    src, dst, rp, col, hist, dups = sfg.kron_generate_csr(c["n0"], c["initiator"], c["k"], E, seed=c["seed"],
                                                          id_bytes=8, flags=0)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    torch.cuda.empty_cache()
    _sampled_edges(orc, c, src, dst)
    assert int(rp[0]) == 0 and int(rp[n]) == E
    out = rp[1:] - rp[:-1]
    assert int(out.min()) >= 0
    assert torch.equal(out, _counts(src, n))
    indeg = _counts(dst, n)
    deg = out + indeg
    del indeg
    bins = torch.zeros(n, dtype=torch.int64, device="cuda")
    for b in range(31):
        bins += (deg >= (1 << b)).long()
    del deg
    np.testing.assert_array_equal(torch.bincount(bins, minlength=32).cpu().numpy(), hist.cpu().numpy())
    del bins
    starts = _row_starts_mask(rp, n, E)
    ndup = 0
    for i in range(1, E, CH):
        j = min(E, i + CH)
        a, b, s = col[i - 1:j - 1], col[i:j], starts[i:j]
        assert bool(((b >= a) | s).all()), "a row is not sorted"
        ndup += int(((b == a) & ~s).sum())
    del starts
    assert ndup == int(dups)
    assert int(col.min()) >= 0 and int(col.max()) < n
    assert _hash_pairs(src, dst, 30) == _row_hash(rp, col, n, 30)
    del src, dst, rp, col
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_pba_symmetric_simple_csr_at_scale(sfg):
    import torch
    c = wl.PBA_SCALE[1]
    n, E = c["n"], c["n"] * c["m"]
    print(f"case {c['name']}: n={n} E={E}", flush=True)
    src, dst = sfg.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], seed=c["seed"])
    rp, col, hist, dups = sfg.edges_to_csr(n, src, dst, flags=sfg.CSR_SYMMETRIZE | sfg.CSR_SIMPLE)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    torch.cuda.empty_cache()
    kept = int(rp[n])
    assert int(rp[0]) == 0 and int((rp[1:] - rp[:-1]).min()) >= 0
    col = col[:kept]
    starts = _row_starts_mask(rp, n, kept)
    for i in range(1, kept, CH):
        j = min(kept, i + CH)
        assert bool(((col[i:j] > col[i - 1:j - 1]) | starts[i:j]).all()), "a row is not strictly increasing"
    del starts
    # distinct non-loop pairs of the edge list, both directions
    u, v = src.long(), dst.long()
    keys = torch.cat([u * n + v, v * n + u])
    keys = keys[(keys // n) != (keys % n)]
    keys = torch.unique(keys)
    assert keys.numel() == kept
    ref = int(_mix((keys // n) * (1 << 27) + keys % n).sum())
    assert ref == _row_hash(rp, col, n, 27)
