"""Host logic of range-chunked generation with resume, with a stand-in
generator (edge e -> (3e, 7e + 1)) so that no GPU is needed."""
import numpy as np
import pytest

from paper_1003_3684_amd import chunked


def _gen(e_begin, count):
    e = np.arange(e_begin, e_begin + count, dtype=np.int64)
    return 3 * e, 7 * e + 1


def _run(num_edges, chunk, fail_at=None, start=0, out=None):
    out = out if out is not None else {}
    failed = []

    def sink(c, e_begin, s, d):
        if c == fail_at and not failed:
            failed.append(c)
            raise OSError("injected")
        assert c not in out
        out[c] = (e_begin, s.copy(), d.copy())

    total = chunked.kron_chunks(2, [[1, 1], [1, 1]], 3, num_edges, chunk_edges=chunk, sink=sink, gen=_gen,
                                start_chunk=start)
    return total, out


def _joined(out):
    keys = sorted(out)
    return np.concatenate([out[c][1] for c in keys]), np.concatenate([out[c][2] for c in keys])


@pytest.mark.parametrize("num_edges,chunk", [(10, 3), (9, 3), (1, 5), (100_001, 7_919)])
def test_chunks_cover_the_graph(num_edges, chunk):
    total, out = _run(num_edges, chunk)
    assert total == chunked.num_chunks(num_edges, chunk) == len(out)
    s, d = _joined(out)
    e = np.arange(num_edges)
    assert np.array_equal(s, 3 * e) and np.array_equal(d, 7 * e + 1)
    assert [out[c][0] for c in sorted(out)] == list(range(0, num_edges, chunk))


@pytest.mark.parametrize("fail_at", [0, 1, 5, 12])
def test_interrupt_and_resume(fail_at):
    num_edges, chunk = 100_001, 7_919  # 13 chunks, the last one short
    out = {}
    with pytest.raises(chunked.ChunkInterrupted) as info:
        _run(num_edges, chunk, fail_at=fail_at, out=out)
    assert info.value.next_chunk == fail_at and sorted(out) == list(range(fail_at))
    total, out = _run(num_edges, chunk, start=info.value.next_chunk, out=out)
    assert total == 13 and sorted(out) == list(range(13))
    ref_total, ref = _run(num_edges, chunk)
    for a, b in zip(_joined(out), _joined(ref)):
        assert np.array_equal(a, b)


def test_edge_cases():
    total, out = _run(0, 4)
    assert total == 0 and out == {}
    total, out = _run(12, 4, start=3)
    assert total == 3 and out == {}
    with pytest.raises(ValueError):
        _run(12, 4, start=4)
    with pytest.raises(ValueError):
        _run(12, 0)
