"""Range-chunked Kronecker generation that can be resumed.

Every Kronecker edge is a function of its index alone, so a graph too large
to hold at once (or a run that may be interrupted) is generated in chunks of
consecutive edges with ``kron_generate_range``: chunk c covers edges
[c * chunk_edges, min((c + 1) * chunk_edges, num_edges)).  Each chunk is
written into one pair of reusable device buffers and handed to ``sink``
(which copies it out, writes it to disk, or consumes it), in chunk order.  The
only state is the cursor: the index of the first chunk not yet delivered.

If the generator or the sink raises, the exception is re-raised as
``ChunkInterrupted`` carrying that cursor; calling ``kron_chunks`` again with
``start_chunk=cursor`` continues, and the chunks delivered over both calls
are exactly those of an uninterrupted run.
"""


class ChunkInterrupted(RuntimeError):
    """Generation stopped before chunk `next_chunk`; every earlier chunk was
    delivered to the sink."""

    def __init__(self, next_chunk, cause):
        super().__init__(f"interrupted before chunk {next_chunk} finished: {cause!r}")
        self.next_chunk = next_chunk
        self.cause = cause


def num_chunks(num_edges, chunk_edges):
    if chunk_edges <= 0:
        raise ValueError("chunk_edges must be positive")
    return (num_edges + chunk_edges - 1) // chunk_edges


def kron_chunks(n0, initiator, k, num_edges, *, chunk_edges, sink, mode=0, seed=0, graph_id=0, id_bytes=4,
                start_chunk=0, gen=None, stream=None):
    """Deliver chunks start_chunk .. last to sink(c, e_begin, src, dst) and
    return the number of chunks of the graph.  `gen` defaults to the GPU
    kron_generate_range; src and dst are views of reused buffers, valid only
    during the sink call."""
    total = num_chunks(num_edges, chunk_edges)
    if not 0 <= start_chunk <= total:
        raise ValueError(f"start_chunk {start_chunk} outside [0, {total}]")
    if gen is None:
        import torch

        from . import native

        dt = torch.int32 if id_bytes == 4 else torch.int64
        cap = min(chunk_edges, num_edges)
        bufs = (torch.empty(cap, dtype=dt, device="cuda"), torch.empty(cap, dtype=dt, device="cuda"))

        def gen(e_begin, count):
            s, d = bufs[0][:count], bufs[1][:count]
            native.kron_generate_range(n0, initiator, k, num_edges, e_begin, count, mode=mode, seed=seed,
                                       graph_id=graph_id, id_bytes=id_bytes, src=s, dst=d, stream=stream)
            return s, d
    for c in range(start_chunk, total):
        e_begin = c * chunk_edges
        count = min(chunk_edges, num_edges - e_begin)
        try:
            src, dst = gen(e_begin, count)
            sink(c, e_begin, src, dst)
        except Exception as exc:  # the cursor stays at c: chunk c was not delivered
            raise ChunkInterrupted(c, exc) from exc
    return total
