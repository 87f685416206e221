"""Host logic of the ensemble schedule autotuner: cache keys, cache file
round trip and the fallback when nothing was tuned (no GPU needed)."""
import json

from paper_1003_3684_amd import tune, workloads as wl


def test_table_key_buckets():
    def pba(n, count=10):
        return [dict(kind="pba", n=n, m=4)] * count

    k1 = tune.table_key(pba(1000), "gfx950")
    assert k1 == "gfx950/ensemble/g4/e16/v14"  # 10 members, 40,000 edges, 10,000 vertices
    assert tune.table_key(pba(1100), "gfx950") == k1  # within the same powers of two
    assert tune.table_key(pba(3000), "gfx950") != k1
    assert tune.table_key(pba(1000, 20), "gfx950") != k1
    assert tune.table_key(pba(1000), "gfx942") != k1
    kron = [dict(kind="kron", n0=2, k=10, num_edges=16 << 10)]
    assert tune.table_key(kron, "gfx950") == "gfx950/ensemble/g1/e15/v11"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    rows = wl.small_ensemble_table(16)
    assert tune.best_batch_edges(rows, arch="gfx950", path=path) == tune.DEFAULT_BATCH_EDGES
    key = tune.table_key(rows, "gfx950")
    tune.save_cache({key: {"best": 1 << 27, "seconds": {"134217728": 0.5}}}, path)
    assert json.load(open(path))[key]["best"] == 1 << 27
    assert tune.best_batch_edges(rows, arch="gfx950", path=path) == 1 << 27
    assert tune.best_batch_edges(rows, arch="gfx942", path=path, default=7) == 7


def test_bad_cache_falls_back(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    rows = wl.small_ensemble_table(8)
    assert tune.load_cache(str(path)) == {}
    assert tune.best_batch_edges(rows, arch="gfx950", path=str(path), default=5) == 5
    path.write_text(json.dumps({tune.table_key(rows, "gfx950"): {"best": "x"}}))
    assert tune.best_batch_edges(rows, arch="gfx950", path=str(path), default=5) == 5
