"""The ensemble schedule autotuner on the GPU: four batch budgets, from one
member per batch to the whole table in one batch, give bit-identical
statistics (the tuner raises otherwise), and the fastest is cached."""
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
    assert all(s > 0 for s in res["seconds"].values())
    assert tune.best_batch_edges(rows, path=path) == res["best"]
    # The chosen budget reproduces the statistics of the one-member batches.
    descs = sfg.graph_descs(rows)
    a = sfg.ensemble_generate(descs, num_samples=2000, stat_seed=3, max_batch_edges=res["best"])
    b = sfg.ensemble_generate(descs, num_samples=2000, stat_seed=3, max_batch_edges=1 << 12)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    np.testing.assert_array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    np.testing.assert_array_equal(a[2].cpu().numpy(), b[2].cpu().numpy())
    np.testing.assert_array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
