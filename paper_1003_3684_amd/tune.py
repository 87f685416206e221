"""Autotuner of the batched ensemble: chunk schedule, persistent grid and tile.

``ensemble_generate_tuned`` takes three choices (``sfg_ensemble_tuning``):

* the chunk schedule: the member table is cut, in order, into batches of at
  most ``max_batch_edges`` edges (and 2^24 vertices), and every batch goes
  through each generation, sort and statistics kernel once.  Larger budgets
  mean fewer launches and per-batch scans; smaller ones shorter sort keys and
  a smaller workspace;
* ``grid_per_cu``: workgroups per compute unit of the persistent generation
  and statistics kernels, which walk the batch's (member, tile) table;
* ``kron_items``: edges per thread of a Kronecker sampling tile (4, 8 or 16).

The best choice depends on the table and on the GPU, so it is measured by
coordinate descent: the budgets first (at the default grid and tile), then
the tiles at the best budget, then the grids at the best budget and tile;
each candidate runs the whole table once (captured into a HIP graph, as it
runs in use) and the fastest is kept.  The choice is cached per (GPU
architecture, table bucket) in a JSON file (``$SFGEN_TUNE_CACHE``, default
``~/.cache/sfgen/tune.json``).

Results never depend on the choice.  Every candidate's statistics are
compared with the first candidate's, bit for bit, and a difference raises.
"""
import json
import os

CANDIDATES = tuple(1 << b for b in range(25, 31))  # 2^25 .. 2^30 edges per batch
GRID_CANDIDATES = (2, 4, 8, 16)  # persistent workgroups per CU
ITEM_CANDIDATES = (4, 8, 16)     # edges per thread of a Kronecker tile
DEFAULT_BATCH_EDGES = 1 << 30
DEFAULT_GRID, DEFAULT_ITEMS = 8, 8


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


def best_tuning(rows, *, arch=None, path=None):
    """(budget, grid_per_cu, kron_items) cached for this table; the defaults
    for whatever was never tuned."""
    arch = arch or device_arch()
    entry = load_cache(path).get(table_key(rows, arch))
    budget, grid, items = DEFAULT_BATCH_EDGES, DEFAULT_GRID, DEFAULT_ITEMS
    if isinstance(entry, dict):
        if isinstance(entry.get("best"), int) and entry["best"] > 0:
            budget = entry["best"]
        if entry.get("grid_per_cu") in GRID_CANDIDATES:
            grid = entry["grid_per_cu"]
        if entry.get("kron_items") in ITEM_CANDIDATES:
            items = entry["kron_items"]
    return budget, grid, items


def tune_ensemble(rows, *, candidates=CANDIDATES, grids=GRID_CANDIDATES, items=ITEM_CANDIDATES, num_samples=10_000,
                  stat_seed=0, path=None, save=True):
    """Coordinate descent over the budget, the tile and the grid (after one
    warm-up call); returns {"best", "grid_per_cu", "kron_items", "seconds":
    {budget: s}, "tile_seconds": {items: s}, "grid_seconds": {grid: s},
    "key"}.  The choice is cached unless save is False.  Raises if any
    candidate's statistics differ from the first one's, or if a kernel
    reported a device error."""
    import numpy as np
    import torch

    from . import native as sfg

    if not candidates or not grids or not items:
        raise ValueError("no candidates")
    candidates = sorted({int(c) for c in candidates})
    grids = sorted({int(g) for g in grids})
    items = sorted({int(i) for i in items})
    descs = sfg.graph_descs(rows)
    count = len(rows)
    ws = sfg.workspace(max(sfg.ensemble_workspace_bytes(descs, c) for c in candidates))
    out = (torch.empty((count, 32), dtype=torch.int64, device="cuda"),
           torch.empty(count, dtype=torch.float64, device="cuda"),
           torch.empty(count, dtype=torch.int64, device="cuda"))
    warm = min(count, 64)
    sfg.ensemble_generate(sfg.graph_descs(rows[:warm]), num_samples=num_samples, stat_seed=stat_seed,
                          ws=ws, out=tuple(t[:warm] for t in out), check=True,
                          tuning=sfg.ensemble_tuning(candidates[0], DEFAULT_GRID, DEFAULT_ITEMS))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ref = []

    def run(budget, grid, item):
        tu = sfg.ensemble_tuning(budget, grid, item)
        # first call captures the batch sequence into a graph; the timed one replays it
        sfg.ensemble_generate(descs, num_samples=num_samples, stat_seed=stat_seed, ws=ws, out=out, tuning=tu)
        a.record()
        sfg.ensemble_generate(descs, num_samples=num_samples, stat_seed=stat_seed, ws=ws, out=out, tuning=tu)
        b.record()
        torch.cuda.synchronize()
        if sfg.device_error() != 0:
            raise RuntimeError(f"ensemble: device error with tuning {(budget, grid, item)}")
        got = tuple(t.cpu().numpy() for t in out)
        if not ref:
            ref.append(got)
        elif not (np.array_equal(got[0], ref[0][0]) and np.array_equal(got[2], ref[0][2])
                  and np.array_equal(got[1], ref[0][1], equal_nan=True)):
            raise RuntimeError(f"ensemble statistics differ with tuning {(budget, grid, item)}")
        return a.elapsed_time(b) / 1e3

    grid0 = DEFAULT_GRID if DEFAULT_GRID in grids else grids[0]
    item0 = DEFAULT_ITEMS if DEFAULT_ITEMS in items else items[0]
    seconds = {c: run(c, grid0, item0) for c in candidates}
    best = min(seconds, key=seconds.get)
    tile_seconds = {i: (seconds[best] if i == item0 else run(best, grid0, i)) for i in items}
    best_item = min(tile_seconds, key=tile_seconds.get)
    grid_seconds = {g: (tile_seconds[best_item] if g == grid0 else run(best, g, best_item)) for g in grids}
    best_grid = min(grid_seconds, key=grid_seconds.get)
    del ws
    key = table_key(rows, device_arch())
    if save:
        entries = load_cache(path)
        entries[key] = {"best": best, "grid_per_cu": best_grid, "kron_items": best_item,
                        "seconds": {str(c): s for c, s in seconds.items()},
                        "tile_seconds": {str(i): s for i, s in tile_seconds.items()},
                        "grid_seconds": {str(g): s for g, s in grid_seconds.items()}}
        save_cache(entries, path)
    return {"best": best, "grid_per_cu": best_grid, "kron_items": best_item, "seconds": seconds,
            "tile_seconds": tile_seconds, "grid_seconds": grid_seconds, "key": key}
