"""The ensemble autotuner on the GPU: batch budgets from one member per batch
to the whole table in one batch, three tile sizes and four persistent grids
give bit-identical statistics (the tuner raises otherwise), the fastest is
cached, and every combination of tile, grid and graph capture reproduces
the plain per-graph statistics."""
import numpy as np
import pytest

from paper_1003_3684_amd import tune, workloads as wl

pytestmark = pytest.mark.gpu


def test_tuner_invariance_and_cache(sfg, tmp_path):
    import torch
    rows = wl.small_ensemble_table(48)
    path = str(tmp_path / "tune.json")
    cands = (1 << 12, 1 << 16, 1 << 20, 1 << 30)
    res = tune.tune_ensemble(rows, candidates=cands, num_samples=2000, stat_seed=3, path=path)
    assert res["best"] in cands and set(res["seconds"]) == set(cands)
    assert set(res["tile_seconds"]) == set(tune.ITEM_CANDIDATES) and set(res["grid_seconds"]) == set(tune.GRID_CANDIDATES)
    assert all(s > 0 for s in res["seconds"].values())
    assert tune.best_batch_edges(rows, path=path) == res["best"]
    assert tune.best_tuning(rows, path=path) == (res["best"], res["grid_per_cu"], res["kron_items"])
    # The chosen budget reproduces the statistics of the one-member batches.
    descs = sfg.graph_descs(rows)
    a = sfg.ensemble_generate(descs, num_samples=2000, stat_seed=3, max_batch_edges=res["best"])
    b = sfg.ensemble_generate(descs, num_samples=2000, stat_seed=3, max_batch_edges=1 << 12)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    np.testing.assert_array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    np.testing.assert_array_equal(a[2].cpu().numpy(), b[2].cpu().numpy())
    np.testing.assert_array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


def test_every_tile_grid_and_capture_gives_the_same_statistics(sfg):
    import itertools

    import torch
    rows = wl.small_ensemble_table(32, seed=41)
    descs = sfg.graph_descs(rows)
    ref = None
    for budget, grid, items, graph in itertools.product((1 << 14, 1 << 24), (1, 2, 16), tune.ITEM_CANDIDATES,
                                                         (False, True)):
        out = sfg.ensemble_generate(descs, num_samples=1000, stat_seed=6, check=True,
                                    tuning=sfg.ensemble_tuning(budget, grid, items, graph))
        got = [t.cpu().numpy() for t in out]
        if ref is None:
            ref = got
            continue
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b, err_msg=str((budget, grid, items, graph)))
    torch.cuda.synchronize()
