"""Randomized PK by temporary seed modification (PK section): the GPU's
level-synchronous expansion equals the oracle's meta-edge stack entry for
entry, including edge order, and reduces to enumerate mode without changes."""
import numpy as np
import pytest

from paper_1003_3684_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIG2 = wl.FIG2_SEED.astype(np.float32)
SEED3 = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 0]], np.float32)
ONES8 = np.ones((8, 8), np.float32)


@pytest.mark.parametrize("seed_m,k,p_add,p_del,id_bytes", [
    (FIG2, 1, 0.3, 0.3, 4),       # the seed itself
    (FIG2, 4, 0.0, 0.0, 4),       # the deterministic power
    (FIG2, 6, 0.05, 0.1, 4),      # ~1.5 M edges, several scan blocks
    (SEED3, 9, 0.2, 0.3, 8),      # 64-bit ids
    (SEED3, 5, 1.0, 1.0, 4),      # every cell flipped: seed (x) complement^4
    (SEED3, 4, 0.0, 1.0, 4),      # everything deleted below the first level
    # ~58 children per meta-edge: a workgroup's children overflow its LDS
    # staging area and are written directly
    (ONES8, 3, 0.0, 0.1, 4),
    (ONES8, 3, 0.0, 0.1, 8),
])
def test_matches_oracle(sfg, orc, seed_m, k, p_add, p_del, id_bytes):
    import torch
    n0 = seed_m.shape[0]
    cap = 4_000_000
    src, dst = sfg.kron_perturbed(n0, seed_m, k, p_add, p_del, cap, seed=17, graph_id=2, id_bytes=id_bytes)
    torch.cuda.synchronize()
    os_, od = orc.kron_perturbed(seed_m, k, p_add, p_del, 17, 2, cap=cap)
    np.testing.assert_array_equal(src.cpu().numpy().astype(np.int64), os_)
    np.testing.assert_array_equal(dst.cpu().numpy().astype(np.int64), od)


def test_no_change_equals_enumerate(sfg):
    import torch
    a = sfg.kron_perturbed(5, FIG2, 5, 0.0, 0.0, 11 ** 5, seed=3)
    b = sfg.kron_generate(5, FIG2, 5, 11 ** 5, mode=sfg.KRON_ENUMERATE)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_capacity_error(sfg):
    from paper_1003_3684_amd.native import SfgenError
    with pytest.raises(SfgenError):
        sfg.kron_perturbed(5, FIG2, 4, 0.0, 0.0, 11 ** 4 - 1)
    with pytest.raises(SfgenError):
        sfg.kron_perturbed(9, np.ones((9, 9), np.float32), 2, 0.0, 0.0, 100)
