"""The C-ABI library loads and exports every function include/sfgen.h declares,
and host-side validation rejects bad arguments before anything is enqueued
(these calls never reach a kernel, so they run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfgen.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


@pytest.fixture(scope="module")
def lib():
    import torch  # (torch first: one shared HIP runtime)
    from paper_1003_3684_amd import native
    return native.load()


@pytest.fixture
def host_only():
    """The validation tests pass fake device addresses; they are host-logic
    tests and must never reach a kernel, so they do not run where a GPU is."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("host validation tests use fake device pointers")


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("kron_generate", "pba_generate", "pba_workspace_bytes", "edges_to_csr",
                     "edges_to_csr_workspace_bytes", "sfg_last_error", "sfg_abi_version", "sfg_device_error"):
        assert required in names, names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in sfgen.h but not exported"


def test_binding_covers_every_declared_symbol():
    from paper_1003_3684_amd import native
    for name in _declared_functions():
        assert name in native.SIGNATURES, f"{name} has no binding signature"


def test_abi_version(lib):
    assert lib.sfg_abi_version() == 1


def _W(x):
    a = np.ascontiguousarray(x, np.float32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def test_kron_validation(lib, host_only):
    _, w = _W([0.5, 0.2, 0.2, 0.1])
    dummy = ctypes.c_void_p(16)
    assert lib.kron_generate(1, w, 3, 10, 0, 1, 0, 4, dummy, dummy, None) == -1   # n0 < 2
    assert lib.kron_generate(2, w, 0, 10, 0, 1, 0, 4, dummy, dummy, None) == -1   # k = 0
    assert lib.kron_generate(2, w, 3, 10, 7, 1, 0, 4, dummy, dummy, None) == -1   # mode
    assert lib.kron_generate(2, w, 3, 10, 0, 1, 0, 3, dummy, dummy, None) == -1   # id bytes
    assert lib.kron_generate(2, w, 3, 10, 0, 1, 1 << 24, 4, dummy, dummy, None) == -1  # graph id
    assert lib.kron_generate(2, w, 3, 10, 0, 1, 0, 4, None, dummy, None) == -1    # NULL
    assert lib.kron_generate(2, w, 32, 10, 0, 1, 0, 4, dummy, dummy, None) == -2  # 2^32 ids in int32
    assert lib.kron_generate(2, w, 64, 10, 0, 1, 0, 8, dummy, dummy, None) == -2  # 2^64 ids
    _, wneg = _W([0.5, -0.2, 0.2, 0.1])
    assert lib.kron_generate(2, wneg, 3, 10, 0, 1, 0, 4, dummy, dummy, None) == -1
    _, wnan = _W([0.5, float("nan"), 0.2, 0.1])
    assert lib.kron_generate(2, wnan, 3, 10, 0, 1, 0, 4, dummy, dummy, None) == -1
    _, wzero = _W([0, 0, 0, 0])
    assert lib.kron_generate(2, wzero, 3, 10, 0, 1, 0, 4, dummy, dummy, None) == -1
    # enumerate mode: num_edges must be e0^k
    _, w01 = _W([1, 1, 0, 1])
    assert lib.kron_generate(2, w01, 3, 26, 1, 0, 0, 4, dummy, dummy, None) == -1
    assert b"e0^k" in lib.sfg_last_error()


def test_pba_validation(lib, host_only):
    d = ctypes.c_void_p(256)
    big = 1 << 40
    assert lib.pba_generate(100, 0, 4, 0.1, None, None, 1, 0, 4, d, d, d, big, None) == -1    # m = 0
    assert lib.pba_generate(100, 2, 0, 0.1, None, None, 1, 0, 4, d, d, d, big, None) == -1    # P = 0
    assert lib.pba_generate(100, 2, 4097, 0.1, None, None, 1, 0, 4, d, d, d, big, None) == -1  # P too big
    assert lib.pba_generate(7, 2, 4, 0.1, None, None, 1, 0, 4, d, d, d, big, None) == -1      # n < 2P
    assert lib.pba_generate(100, 2, 4, 1.5, None, None, 1, 0, 4, d, d, d, big, None) == -1    # p > 1
    assert lib.pba_generate(100, 2, 4, float("nan"), None, None, 1, 0, 4, d, d, d, big, None) == -1
    assert lib.pba_generate(100, 2, 4, 0.1, None, None, 1, 0, 4, d, d, d, 10, None) == -3     # workspace
    assert lib.pba_generate(1 << 32, 2, 4, 0.1, None, None, 1, 0, 4, d, d, d, big, None) == -2  # int32 ids
    off = np.array([0, 1, 1, 2, 9], np.uint32)
    mem = np.array([0, 7, 1, 1, 1, 1, 1, 1, 1], np.uint32)  # member 7 >= P
    assert lib.pba_generate(100, 2, 4, 0.1, off.ctypes.data_as(ctypes.c_void_p), mem.ctypes.data_as(ctypes.c_void_p),
                            1, 0, 4, d, d, d, big, None) == -1
    empty = np.array([0, 1, 1, 2, 3], np.uint32)  # partition 1 has no faction member
    assert lib.pba_generate(100, 2, 4, 0.1, empty.ctypes.data_as(ctypes.c_void_p),
                            mem.ctypes.data_as(ctypes.c_void_p), 1, 0, 4, d, d, d, big, None) == -1
    assert b"empty faction" in lib.sfg_last_error()
    bad = np.array([0, 2, 1, 2, 3], np.uint32)  # not monotone
    assert lib.pba_generate(100, 2, 4, 0.1, bad.ctypes.data_as(ctypes.c_void_p), mem.ctypes.data_as(ctypes.c_void_p),
                            1, 0, 4, d, d, d, big, None) == -1


def test_csr_validation(lib, host_only):
    d = ctypes.c_void_p(256)
    assert lib.edges_to_csr(0, 10, d, d, 4, 0, d, d, None, None, d, 1 << 30, None) == -1   # n = 0
    assert lib.edges_to_csr(10, 10, d, d, 4, 8, d, d, None, None, d, 1 << 30, None) == -1  # flags
    assert lib.edges_to_csr(10, 10, d, d, 5, 0, d, d, None, None, d, 1 << 30, None) == -1  # id bytes
    assert lib.edges_to_csr(10, 10, d, d, 4, 0, None, d, None, None, d, 1 << 30, None) == -1  # row_ptr
    assert lib.edges_to_csr(1 << 33, 10, d, d, 8, 0, d, d, None, None, d, 1 << 62, None) == -2  # n > 2^32
    need = lib.edges_to_csr_workspace_bytes(1000, 5000, 4, 1)
    assert need > 0
    assert lib.edges_to_csr(1000, 5000, d, d, 4, 1, d, d, d, None, d, need - 1, None) == -3


def test_kron_csr_validation(lib, host_only):
    """kron_generate_csr checks the generator's and the CSR build's arguments
    before anything is launched."""
    _, w = _W([0.5, 0.2, 0.2, 0.1])
    d = ctypes.c_void_p(256)
    need = lib.edges_to_csr_workspace_bytes(1 << 10, 5000, 4, 0)
    assert need > 0

    def call(n0=2, k=10, E=5000, mode=0, graph_id=0, ib=4, flags=0, rp=d, ws=need, W=w):
        return lib.kron_generate_csr(n0, W, k, E, mode, 1, graph_id, ib, d, d, flags, rp, d, d, d, d, ws, None)

    assert call(n0=1) == -1                 # n0 < 2
    assert call(k=0) == -1                  # k = 0
    assert call(k=33) == -2                 # 2^33 vertices: no 64-bit key
    assert call(flags=8) == -1              # bad flags
    assert call(ib=3) == -1                 # id bytes
    assert call(rp=None) == -1              # row_ptr
    assert call(ws=need - 1) == -3          # workspace
    assert lib.edges_to_csr_workspace_bytes(1 << 10, 5000, 4, 1) > need  # symmetrized: twice the entries
    assert call(flags=1, ws=need) == -3


def test_workspace_sizes_monotone(lib):
    a = lib.pba_workspace_bytes(1 << 20, 4, 64, 0)
    b = lib.pba_workspace_bytes(1 << 21, 4, 64, 0)
    assert 0 < a < b
    assert lib.pba_workspace_bytes(1 << 20, 4, 64, 1000) >= a
    assert lib.edges_to_csr_workspace_bytes(1 << 20, 1 << 22, 4, 0) < lib.edges_to_csr_workspace_bytes(1 << 20, 1 << 22, 4, 1)
