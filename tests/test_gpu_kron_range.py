"""Range generation of Kronecker graphs: edges [e_begin, e_begin + count)
equal the oracle's at edge indices far beyond 2^32 (the Philox counter's
high word), across the low word's wrap, and at the tail of the 5 x 2^30
workload; enumerate-mode ranges equal slices of the one-call output; and a
chunked run interrupted mid-way and resumed equals the one-call graph."""
import numpy as np
import pytest

from paper_1003_3684_amd import chunked, workloads as wl

pytestmark = pytest.mark.gpu

CASES = [
    # (name, n0, initiator, k, num_edges, e_begin, count, id_bytes, seed)
    ("kron2x2_k20_beyond_2^33", 2, wl.KRON_K20["initiator"], 20, 1 << 34, (1 << 33) + 5, 100_003, 4, 7),
    ("kron3x3pad4_k15_tail", 4, wl.KRON_SCALE["initiator"], 15, 5 << 30, (5 << 30) - 77_777, 77_777, 8, 13),
    ("kron3x3_k19_low_word_wrap", 3, wl.KRON_SCALE_B["initiator"], 19, 1 << 40, (1 << 32) - 1000, 3000, 8, 13),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_range_matches_oracle(sfg, orc, case):
    import torch
    _, n0, W, k, ne, e_begin, count, id_bytes, seed = case
    src, dst = sfg.kron_generate_range(n0, W, k, ne, e_begin, count, seed=seed, id_bytes=id_bytes)
    torch.cuda.synchronize()
    os_, od = orc.kron_sample(n0, W, k, count, seed, e_begin=e_begin)
    np.testing.assert_array_equal(src.cpu().numpy().astype(np.int64), os_)
    np.testing.assert_array_equal(dst.cpu().numpy().astype(np.int64), od)


def test_range_general_path(sfg, orc):
    """More than 15 thresholds (LDS search path), across the counter's low-word wrap."""
    rng = np.random.default_rng(55)
    W = rng.uniform(0.0, 1.0, size=(6, 6)).astype(np.float32)
    e_begin, count = (1 << 32) - 2000, 5001
    src, dst = sfg.kron_generate_range(6, W, 5, 1 << 36, e_begin, count, seed=3, graph_id=9, id_bytes=4)
    os_, od = orc.kron_sample(6, W, 5, count, 3, graph_id=9, e_begin=e_begin)
    np.testing.assert_array_equal(src.cpu().numpy().astype(np.int64), os_)
    np.testing.assert_array_equal(dst.cpu().numpy().astype(np.int64), od)


def test_range_enumerate_is_a_slice(sfg):
    seed = wl.FIG2_SEED.astype(np.float32)
    full_s, full_d = sfg.kron_generate(5, seed, 4, 11 ** 4, mode=sfg.KRON_ENUMERATE)
    for b, c in ((0, 1), (1000, 4001), (11 ** 4 - 7, 7), (11 ** 4, 0)):
        s, d = sfg.kron_generate_range(5, seed, 4, 11 ** 4, b, c, mode=sfg.KRON_ENUMERATE)
        assert np.array_equal(s.cpu().numpy(), full_s[b:b + c].cpu().numpy())
        assert np.array_equal(d.cpu().numpy(), full_d[b:b + c].cpu().numpy())


def test_range_errors(sfg):
    W = wl.KRON_K20["initiator"]
    with pytest.raises(sfg.SfgenError):
        sfg.kron_generate_range(2, W, 20, 1000, 900, 101)
    with pytest.raises(sfg.SfgenError):
        sfg.kron_generate_range(2, W, 20, 1000, 1001, 0)


def test_chunked_resume_equals_one_call(sfg):
    """2^24 edges in ragged chunks; the sink fails once on chunk 2, the run
    resumes from the cursor, and the delivered chunks equal the one-call graph."""
    import torch
    c = wl.KRON_K20
    full_s, full_d = sfg.kron_generate(c["n0"], c["initiator"], c["k"], c["num_edges"], seed=c["seed"])
    out_s = np.full(c["num_edges"], -1, np.int64)
    out_d = np.full(c["num_edges"], -1, np.int64)
    failed = []

    def sink(ci, e_begin, s, d):
        if ci == 2 and not failed:
            failed.append(ci)
            raise IOError("injected failure")
        out_s[e_begin:e_begin + s.numel()] = s.cpu().numpy()
        out_d[e_begin:e_begin + d.numel()] = d.cpu().numpy()

    kw = dict(chunk_edges=3_000_017, sink=sink, seed=c["seed"])
    with pytest.raises(chunked.ChunkInterrupted) as info:
        chunked.kron_chunks(c["n0"], c["initiator"], c["k"], c["num_edges"], **kw)
    assert info.value.next_chunk == 2
    assert (out_s[2 * 3_000_017:] == -1).all()
    total = chunked.kron_chunks(c["n0"], c["initiator"], c["k"], c["num_edges"], start_chunk=2, **kw)
    assert total == 6
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out_s, full_s.cpu().numpy())
    np.testing.assert_array_equal(out_d, full_d.cpu().numpy())
