"""Randomized PK by XOR with a random graph (PK section): the GPU CSR equals
the oracle's bit for bit, across tile boundaries, with repeated random pairs
and pairs shared with the Kronecker power; and the SIMPLE CSR path it shares
its finish kernel with is unchanged."""
import numpy as np
import pytest

from paper_1003_3684_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED3 = np.array([[1, 1, 0], [1, 0, 1], [0, 1, 1]], np.float32)


@pytest.mark.parametrize("seed_m,k,M,id_bytes", [
    (SEED3, 3, 400, 4),                       # tiny: many collisions and repeats
    (SEED3, 9, 50_000, 4),                    # 3^9 ids, several finish tiles
    (wl.FIG2_SEED.astype(np.float32), 6, 3_000_000, 8),  # 11^6 + 3e6 entries, 64-bit ids
    (wl.FIG2_SEED.astype(np.float32), 5, 0, 4),           # no random graph: the power itself
])
def test_xor_matches_oracle(sfg, orc, seed_m, k, M, id_bytes):
    import torch
    rp, col = sfg.kron_xor_random(seed_m.shape[0], seed_m, k, M, seed=91, graph_id=3, id_bytes=id_bytes)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    orp, ocol = orc.kron_xor_random(seed_m, k, M, 91, 3)
    np.testing.assert_array_equal(rp.cpu().numpy().astype(np.uint64), orp)
    m = int(orp[-1])
    np.testing.assert_array_equal(col[:m].cpu().numpy().astype(np.int64), ocol)


def test_xor_errors(sfg):
    from paper_1003_3684_amd.native import SfgenError
    with pytest.raises(SfgenError):
        sfg.kron_xor_random(3, np.zeros((3, 3), np.float32), 2, 10)
    with pytest.raises(SfgenError):
        sfg.kron_xor_random(2, np.ones((2, 2), np.float32), 32, 10)  # 2^32 vertices
