"""edges_to_csr_noalloc (the CSR build on the library's static scratch array)
against edges_to_csr with a caller workspace, through the C ABI: two calls in
a row on the same device, the second with a smaller input (the scratch array
keeps the first call's contents), plus the size limit."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _edges(rng, n, E):
    import torch
    src = rng.integers(0, n, E)
    dst = np.minimum(rng.zipf(1.5, E) - 1, n - 1)
    return (torch.tensor(src, dtype=torch.int32, device="cuda"), torch.tensor(dst, dtype=torch.int32, device="cuda"))


def _noalloc(lib, n, src, dst, flags, sfg):
    """The new entry point called through the C ABI on caller-owned outputs."""
    import torch
    E = src.numel()
    N = 2 * E if flags & sfg.CSR_SYMMETRIZE else E
    rp = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
    col = torch.full((max(N, 1),), -1, dtype=src.dtype, device="cuda")
    hist = torch.full((32,), -1, dtype=torch.int64, device="cuda")
    dups = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.edges_to_csr_noalloc(n, E, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), 4, flags,
                                  C.c_void_p(rp.data_ptr()), C.c_void_p(col.data_ptr()), C.c_void_p(hist.data_ptr()),
                                  C.c_void_p(dups.data_ptr()), s)
    assert rc == 0, lib.sfg_last_error()
    return rp, col, hist, dups


@pytest.mark.parametrize("flags", [0, 1, 3])
def test_noalloc_equals_workspace_call_twice(sfg, flags):
    import torch
    lib = sfg.load()
    rng = np.random.default_rng(40 + flags)
    # first call near the scratch limit, second one smaller (stale scratch)
    for n, E in ((1 << 20, 1_500_000), (40_000, 300_001)):
        src, dst = _edges(rng, n, E)
        need = sfg.edges_to_csr_workspace_bytes(n, E, 4, flags)
        assert need <= lib.edges_to_csr_noalloc_max_bytes()
        rp, col, hist, dups = _noalloc(lib, n, src, dst, flags, sfg)
        rp2, col2, hist2, dups2 = sfg.edges_to_csr(n, src, dst, flags=flags)
        torch.cuda.synchronize()
        assert sfg.device_error() == 0
        kept = int(rp2[n])
        assert torch.equal(rp, rp2)
        assert torch.equal(col[:kept], col2[:kept])
        assert torch.equal(hist, hist2) and torch.equal(dups, dups2)


def test_noalloc_size_limit(sfg):
    import torch
    lib = sfg.load()
    cap = lib.edges_to_csr_noalloc_max_bytes()
    E = cap // 8  # 8-byte keys twice over: more than the scratch holds
    need = sfg.edges_to_csr_workspace_bytes(1 << 20, E, 4, 0)
    assert need > cap
    src = torch.zeros(E, dtype=torch.int32, device="cuda")
    with pytest.raises(sfg.SfgenError) as ei:
        sfg.edges_to_csr_noalloc(1 << 20, src, src)
    assert ei.value.code == sfg.SFG_ERANGE
