"""Host-side input recipes: faction topologies and the ensemble table."""
import numpy as np

from paper_1003_3684_amd import workloads as wl


def test_faction_groups_block_and_overlap():
    off, mem = wl.faction_groups(16, 4)
    assert off.size == 17 and off[-1] == mem.size == 16 * 4
    for q in range(16):
        lst = mem[off[q]:off[q + 1]]
        g = q * 4 // 16
        assert sorted(lst) == list(range(4 * g, 4 * g + 4))
        assert q in lst  # every partition is in its own faction
    off, mem = wl.faction_groups(16, 4, overlap=True)
    for q in range(16):
        g = q * 4 // 16
        lst = mem[off[q]:off[q + 1]]
        assert set(lst) == set(range(4 * g, 4 * g + 4)) | set(range(4 * ((g + 1) % 4), 4 * ((g + 1) % 4) + 4))
    # uneven group sizes still cover every partition exactly once per group
    off, mem = wl.faction_groups(10, 3)
    assert sorted(set(mem.tolist())) == list(range(10))


def test_ensemble_table_recipe():
    rows = wl.ensemble_table(64, seed=17)
    assert len(rows) == 64
    for g, r in enumerate(rows):
        assert r["graph_id"] == g
        if g % 2 == 0:
            assert r["kind"] == "pba" and 2 ** 10 <= r["n"] <= 2 ** 20 and 2 <= r["m"] <= 8
            assert 0.0 <= r["p_inter"] <= 0.5 and r["num_parts"] == 64
        else:
            W = np.asarray(r["initiator"], np.float64)
            assert r["kind"] == "kron" and 10 <= r["k"] <= 20 and r["num_edges"] == 16 << r["k"]
            np.testing.assert_allclose(W.sum(axis=1), 1.0, rtol=1e-6)
