"""Autotuner for the chunk schedule of the batched ensemble.

``ensemble_generate`` cuts its member table, in order, into batches of at most
``max_batch_edges`` edges (and 2^24 vertices); every batch goes through each
generation, sort and statistics kernel once.  Larger budgets mean fewer
launches and fewer per-batch scans; smaller ones shorter sort keys, shorter
pointer chains per batch and a smaller workspace.  The best budget depends on
the table and on the GPU, so it is measured: each candidate budget runs the
whole table once, the fastest is kept, and the choice is cached per (GPU
architecture, table bucket) in a JSON file (``$SFGEN_TUNE_CACHE``, default
``~/.cache/sfgen/tune.json``).

Results never depend on the choice.  Every candidate's statistics are
compared with the first candidate's, bit for bit, and a difference raises.

Kernel tile sizes (onesweep tiles, resolve tiles, finish tiles) are fixed at
compile time; the budget is the schedule that varies with the workload.
"""
import json
import os

CANDIDATES = tuple(1 << b for b in range(25, 31))  # 2^25 .. 2^30 edges per batch
DEFAULT_BATCH_EDGES = 1 << 30


def cache_path():
    return os.environ.get("SFGEN_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "sfgen",
                                                              "tune.json")


def _edges(r):
    return r["n"] * r["m"] if r["kind"] == "pba" else r["num_edges"]


def _vertices(r):
    return r["n"] if r["kind"] == "pba" else r["n0"] ** r["k"]


def table_key(rows, arch):
    """Cache key: the architecture and the bit lengths of the member count,
    the total edge count and the total vertex count (tables within a factor
    of two of each other share a schedule)."""
    count = len(rows)
    edges = sum(_edges(r) for r in rows)
    verts = sum(_vertices(r) for r in rows)
    return f"{arch}/ensemble/g{count.bit_length()}/e{edges.bit_length()}/v{verts.bit_length()}"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(entries, path=None):
    """Write the cache atomically (a reader never sees half a file)."""
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_arch(device=0):
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def best_batch_edges(rows, *, arch=None, path=None, default=DEFAULT_BATCH_EDGES):
    """The cached budget for this table, or `default` if it was never tuned."""
    arch = arch or device_arch()
    entry = load_cache(path).get(table_key(rows, arch))
    if isinstance(entry, dict) and isinstance(entry.get("best"), int) and entry["best"] > 0:
        return entry["best"]
    return default


def tune_ensemble(rows, *, candidates=CANDIDATES, num_samples=10_000, stat_seed=0, path=None, save=True):
    """Run the whole table once per candidate budget (after one warm-up call)
    and return {"best", "seconds": {budget: s}, "key"}; the choice is cached
    unless save is False.  Raises if any candidate's statistics differ."""
    import numpy as np
    import torch

    from . import native as sfg

    if not candidates:
        raise ValueError("no candidate budgets")
    candidates = sorted({int(c) for c in candidates})
    descs = sfg.graph_descs(rows)
    count = len(rows)
    ws = sfg.workspace(max(sfg.ensemble_workspace_bytes(descs, c) for c in candidates))
    out = (torch.empty((count, 32), dtype=torch.int64, device="cuda"),
           torch.empty(count, dtype=torch.float64, device="cuda"),
           torch.empty(count, dtype=torch.int64, device="cuda"))
    warm = min(count, 64)
    sfg.ensemble_generate(sfg.graph_descs(rows[:warm]), num_samples=num_samples, stat_seed=stat_seed,
                          max_batch_edges=candidates[0], ws=ws, out=tuple(t[:warm] for t in out))
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    seconds, ref = {}, None
    for c in candidates:
        a.record()
        sfg.ensemble_generate(descs, num_samples=num_samples, stat_seed=stat_seed, max_batch_edges=c, ws=ws,
                              out=out)
        b.record()
        torch.cuda.synchronize()
        seconds[c] = a.elapsed_time(b) / 1e3
        got = tuple(t.cpu().numpy() for t in out)
        if ref is None:
            ref = got
        elif not (np.array_equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])
                  and np.array_equal(got[1], ref[1], equal_nan=True)):
            raise RuntimeError(f"ensemble statistics differ between batch budgets {candidates[0]} and {c}")
    del ws
    best = min(seconds, key=seconds.get)
    key = table_key(rows, device_arch())
    if save:
        entries = load_cache(path)
        entries[key] = {"best": best, "seconds": {str(c): s for c, s in seconds.items()}}
        save_cache(entries, path)
    return {"best": best, "seconds": seconds, "key": key}
