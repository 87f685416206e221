"""edges_to_csr at full size, in the configurations the benchmark runs, checked
on the GPU by invariants that pin the CSR exactly (no CPU sort of billions
of entries is needed):

* the benchmark step: 5 x 2^30 Kronecker edges (3x3 initiator padded to
  4x4, 15 levels, int64 ids) generated and sorted by the one-call
  kron_generate_csr (the sampler counts the sort's histogram), directed CSR
  with duplicate count and degree histogram; the same for the unpadded 3x3
  initiator at 19 levels (3^19 ids).  Every one of the 5 x 2^30 edges equals
  the oracle's: the oracle regenerates the edge list in chunks of 2^26 on
  all host cores (the oracle is plain C called through ctypes, so threads
  run it in parallel) and each chunk is compared byte for byte with the
  device's.  Row starts are the exclusive scan of the source counts, every
  row is sorted, the multiset of (row, column) equals that of (src, dst)
  (64-bit sum of a mixing function of the packed pair), the duplicate count
  equals the repeated sorted positions, and the histogram equals the one of
  out-degree + in-degree;
* the PBA workload at 2^27 vertices (whose edges the PBA tests compare with
  the oracle in full): the symmetrized CSR with degree histogram and
  duplicate count, at p = 0.01, 0.1 and 0.3, by the same invariants over
  both orientations of every edge; and the symmetrized simple CSR: no
  self-loops, strictly increasing rows, and the entry set equals the
  distinct non-loop pairs of the edge list in both directions."""
import os
import time
from concurrent.futures import ThreadPoolExecutor

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


ORACLE_CHUNK = 1 << 26  # edges per oracle chunk of the full comparison


def _host_threads():
    """Oracle threads: the host cores this process may use, at most 16 (the
    share of the host that goes with one GPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def _all_edges_equal_oracle(orc, c, src, dst):
    """Every edge [0, E) of the device's edge list equals the oracle's: the
    oracle regenerates chunks of ORACLE_CHUNK edges in parallel threads and
    each is compared byte for byte with the device chunk copied to the host."""
    import torch
    E = c["num_edges"]
    chunks = [(s, min(E, s + ORACLE_CHUNK)) for s in range(0, E, ORACLE_CHUNK)]
    threads = _host_threads()
    host_s = torch.empty(ORACLE_CHUNK, dtype=src.dtype, pin_memory=True)
    host_d = torch.empty(ORACLE_CHUNK, dtype=dst.dtype, pin_memory=True)

    def oracle_chunk(r):
        return orc.kron_sample(c["n0"], c["initiator"], c["k"], r[1] - r[0], c["seed"], 0, e_begin=r[0])

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        # at most 2 x threads chunks in flight (each 1 GiB of oracle output)
        pending = [ex.submit(oracle_chunk, r) for r in chunks[:2 * threads]]
        nxt = len(pending)
        for i, (s, e) in enumerate(chunks):
            os_, od = pending[i].result()
            pending[i] = None
            if nxt < len(chunks):
                pending.append(ex.submit(oracle_chunk, chunks[nxt]))
                nxt += 1
            m = e - s
            host_s[:m].copy_(src[s:e])
            host_d[:m].copy_(dst[s:e])
            if not (np.array_equal(host_s[:m].numpy(), os_) and np.array_equal(host_d[:m].numpy(), od)):
                bad = np.nonzero((host_s[:m].numpy() != os_) | (host_d[:m].numpy() != od))[0]
                raise AssertionError(f"{c['name']}: {bad.size} edges of chunk [{s}, {e}) differ from the oracle, "
                                     f"first at edge {s + int(bad[0])}")
            if i % 16 == 15:
                print(f"  {c['name']}: edges [0, {e}) equal the oracle ({time.perf_counter() - t0:.0f} s, "
                      f"{threads} threads)", flush=True)
    print(f"  {c['name']}: all {E} edges equal the oracle in {time.perf_counter() - t0:.0f} s", flush=True)


def _check_directed_csr(c, n, E, src, dst, rp, col, hist, dups, shift):
    """The directed CSR of (src, dst) with histogram and duplicate count, by
    exact invariants (no sort on the host)."""
    import torch
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
    assert _hash_pairs(src, dst, shift) == _row_hash(rp, col, n, shift)


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("case", ["padded_4x4_k15", "unpadded_3x3_k19"])
def test_bench_csr_at_full_size(sfg, orc, case):
    import torch
    c = wl.KRON_SCALE if case == "padded_4x4_k15" else wl.KRON_SCALE_B
    n, E = c["n0"] ** c["k"], c["num_edges"]
    shift = max(1, (n - 1).bit_length())
    print(f"case {c['name']}: n={n} E={E}", flush=True)
    src, dst, rp, col, hist, dups = sfg.kron_generate_csr(c["n0"], c["initiator"], c["k"], E, seed=c["seed"],
                                                          id_bytes=8, flags=0)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    torch.cuda.empty_cache()
    _all_edges_equal_oracle(orc, c, src, dst)
    _check_directed_csr(c, n, E, src, dst, rp, col, hist, dups, shift)
    del src, dst, rp, col
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("idx", [0, 1, 2])
def test_pba_symmetrized_csr_at_scale(sfg, idx):
    """The 2^27-vertex PBA workload's symmetrized CSR (both orientations of
    every edge, loops twice, repeats kept) with histogram and duplicate
    count, at p = 0.01, 0.1 and 0.3."""
    import torch
    c = wl.PBA_SCALE[idx]
    n, E = c["n"], c["n"] * c["m"]
    print(f"case {c['name']}: symmetrized CSR, n={n} E={E}", flush=True)
    src, dst = sfg.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], seed=c["seed"])
    rp, col, hist, dups = sfg.edges_to_csr(n, src, dst, flags=sfg.CSR_SYMMETRIZE)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    N = 2 * E
    assert int(rp[0]) == 0 and int(rp[n]) == N
    rows = rp[1:] - rp[:-1]
    deg = _counts(src, n) + _counts(dst, n)
    assert torch.equal(rows, deg)  # symmetrized: row v holds deg(v) entries
    bins = torch.zeros(n, dtype=torch.int64, device="cuda")
    for b in range(31):
        bins += (deg >= (1 << b)).long()
    np.testing.assert_array_equal(torch.bincount(bins, minlength=32).cpu().numpy(), hist.cpu().numpy())
    del bins, deg, rows
    starts = _row_starts_mask(rp, n, N)
    ndup = 0
    for i in range(1, N, CH):
        j = min(N, i + CH)
        a, b, s = col[i - 1:j - 1], col[i:j], starts[i:j]
        assert bool(((b >= a) | s).all()), "a row is not sorted"
        ndup += int(((b == a) & ~s).sum())
    del starts
    assert ndup == int(dups)
    assert _hash_pairs(torch.cat([src, dst]), torch.cat([dst, src]), 27) == _row_hash(rp, col, n, 27)


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
