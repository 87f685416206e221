"""Thin Python binding of libsfgen.so.

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of generation and CSR construction runs in the library's
HIP kernels.  Function names follow the C ABI in include/sfgen.h.  There is no
CPU fallback: if the library or a GPU is missing, calls raise.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfgen.so")

SFG_OK, SFG_EINVAL, SFG_ERANGE, SFG_ENOSPACE, SFG_EDEVICE = 0, -1, -2, -3, -4
KRON_SAMPLE, KRON_ENUMERATE = 0, 1
CSR_SYMMETRIZE, CSR_SIMPLE = 1, 2

_ERRNAMES = {SFG_EINVAL: "EINVAL", SFG_ERANGE: "ERANGE", SFG_ENOSPACE: "ENOSPACE", SFG_EDEVICE: "EDEVICE"}


class SfgenError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_vp, _u32, _u64, _i32, _dbl, _sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_double, C.c_size_t

# name -> (restype, argtypes); the order follows include/sfgen.h.
SIGNATURES = {
    "sfg_last_error": (C.c_char_p, []),
    "sfg_abi_version": (_i32, []),
    "sfg_device_error": (_i32, [_vp, C.POINTER(_u32)]),
    "sfg_profile_enable": (_i32, [_i32]),
    "sfg_profile_reset": (_i32, []),
    "sfg_profile_query": (_i32, [C.c_char_p, C.POINTER(_u64), C.POINTER(C.c_double)]),
    "kron_generate": (_i32, [_u32, _vp, _u32, _u64, _i32, _u64, _u32, _i32, _vp, _vp, _vp]),
    "kron_generate_range": (_i32, [_u32, _vp, _u32, _u64, _u64, _u64, _i32, _u64, _u32, _i32, _vp, _vp, _vp]),
    "pba_workspace_bytes": (_sz, [_u64, _u32, _u32, _u64]),
    "pba_generate": (_i32, [_u64, _u32, _u32, _dbl, _vp, _vp, _u64, _u32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "edges_to_csr_workspace_bytes": (_sz, [_u64, _u64, _i32, _u32]),
    "edges_to_csr": (_i32, [_u64, _u64, _vp, _vp, _i32, _u32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "edges_to_csr_noalloc_max_bytes": (_sz, []),
    "edges_to_csr_noalloc": (_i32, [_u64, _u64, _vp, _vp, _i32, _u32, _vp, _vp, _vp, _vp, _vp]),
    "kron_generate_csr": (_i32, [_u32, _vp, _u32, _u64, _i32, _u64, _u32, _i32, _vp, _vp, _u32, _vp, _vp, _vp, _vp,
                                 _vp, _sz, _vp]),
    "graph_stats_workspace_bytes": (_sz, [_u64, _u64, _i32]),
    "graph_stats": (_i32, [_u64, _u64, _vp, _vp, _i32, _u32, _u64, _u32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "path_stats_workspace_bytes": (_sz, [_u64]),
    "block_matrix": (_i32, [_u64, _u64, _vp, _vp, _i32, _u32, _vp, _vp]),
    "kron_xor_random_workspace_bytes": (_sz, [_u32, _vp, _u32, _u64, _i32]),
    "kron_perturbed_workspace_bytes": (_sz, [_u64]),
    "kron_perturbed": (_i32, [_u32, _vp, _u32, _dbl, _dbl, _u64, _u32, _i32, _u64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "kron_xor_random": (_i32, [_u32, _vp, _u32, _u64, _u64, _u32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "path_stats": (_i32, [_u64, _vp, _vp, _i32, _vp, _u32, _vp, _vp, _sz, _vp]),
    "ensemble_workspace_bytes": (_sz, [_vp, _u32, _u64]),
    "ensemble_generate": (_i32, [_vp, _u32, _u32, _u64, _u64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ensemble_generate_tuned": (_i32, [_vp, _u32, _u32, _u64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mlp_param_count": (_sz, [_vp]),
    "mlp_workspace_bytes": (_sz, [_vp, _u32]),
    "mlp_forward": (_i32, [_vp, _u32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mlp_backward": (_i32, [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "mlp_mse_grad": (_i32, [_u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "adam_step": (_i32, [_u64, _vp, _vp, _vp, _vp, C.c_float, C.c_float, C.c_float, C.c_float, _u32, _vp]),
    "adam_step_device": (_i32, [_u64, _vp, _vp, _vp, _vp, _vp, C.c_float, C.c_float, C.c_float, _vp, _vp]),
    "mlp_train_workspace_bytes": (_sz, [_vp, _u32]),
    "mlp_train_step": (_i32, [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_float, C.c_float, C.c_float,
                              _vp, _vp, _vp, _vp, _sz, _vp]),
}


class MlpShape(C.Structure):
    """sfg_mlp_shape of include/sfgen.h."""
    _fields_ = [("d_in", C.c_uint32), ("width", C.c_uint32), ("d_out", C.c_uint32), ("hidden", C.c_uint32)]


class GraphDesc(C.Structure):
    """sfg_graph_desc of include/sfgen.h."""
    _fields_ = [("kind", C.c_int32), ("graph_id", C.c_uint32), ("seed", C.c_uint64), ("n", C.c_uint64),
                ("m", C.c_uint32), ("num_parts", C.c_uint32), ("p_inter", C.c_double), ("n0", C.c_uint32),
                ("k", C.c_uint32), ("num_edges", C.c_uint64), ("initiator", C.c_float * 16)]


GRAPH_PBA, GRAPH_KRON = 0, 1
ENSEMBLE_GRAPH = 1


class EnsembleTuning(C.Structure):
    """sfg_ensemble_tuning of include/sfgen.h."""
    _fields_ = [("max_batch_edges", C.c_uint64), ("grid_per_cu", C.c_uint32), ("kron_items", C.c_uint32),
                ("flags", C.c_uint32)]


def ensemble_tuning(max_batch_edges=1 << 28, grid_per_cu=8, kron_items=8, graph=True):
    return EnsembleTuning(max_batch_edges, grid_per_cu, kron_items, ENSEMBLE_GRAPH if graph else 0)


def load(path: str = LIB_PATH):
    """Load libsfgen.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or python -m paper_1003_3684_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(lib, name):
            continue
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != SFG_OK:
        raise SfgenError(rc, load().sfg_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _idtype(id_bytes):
    if id_bytes == 4:
        return torch.int32
    if id_bytes == 8:
        return torch.int64
    raise ValueError("id_bytes must be 4 or 8")


def _require_cuda():
    if not torch.cuda.is_available():
        raise RuntimeError("sfgen needs a HIP device; no CPU path exists")


def workspace(nbytes, device="cuda"):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def device_error(stream=None):
    code = _u32(0)
    _check(load().sfg_device_error(_stream(stream), C.byref(code)))
    return int(code.value)


def profile_enable(on=True):
    _check(load().sfg_profile_enable(1 if on else 0))


def profile_reset():
    _check(load().sfg_profile_reset())


def profile_query(name):
    """(launches, total_ms) of the timed launches of kernel `name`."""
    n, ms = _u64(0), C.c_double(0.0)
    _check(load().sfg_profile_query(name.encode(), C.byref(n), C.byref(ms)))
    return int(n.value), float(ms.value)


# ----------------------------------------------------------------------------- Kronecker
def kron_generate(n0, initiator, k, num_edges, *, mode=KRON_SAMPLE, seed=0, graph_id=0, id_bytes=4,
                  src=None, dst=None, stream=None):
    """Kronecker edges into device tensors (allocated if not given)."""
    _require_cuda()
    lib = load()
    W = torch.as_tensor(initiator, dtype=torch.float32).contiguous().reshape(-1)
    if W.numel() != n0 * n0:
        raise ValueError("initiator must have n0*n0 entries")
    dt = _idtype(id_bytes)
    if src is None:
        src = torch.empty(num_edges, dtype=dt, device="cuda")
    if dst is None:
        dst = torch.empty(num_edges, dtype=dt, device="cuda")
    _check(lib.kron_generate(n0, C.c_void_p(W.data_ptr()), k, num_edges, mode, seed, graph_id, id_bytes,
                             _ptr(src), _ptr(dst), _stream(stream)))
    return src, dst


def kron_generate_range(n0, initiator, k, num_edges, e_begin, count, *, mode=KRON_SAMPLE, seed=0, graph_id=0,
                        id_bytes=4, src=None, dst=None, stream=None):
    """Edges [e_begin, e_begin + count) of the graph kron_generate(n0, initiator,
    k, num_edges, ...) writes, into device tensors of count ids."""
    _require_cuda()
    lib = load()
    W = torch.as_tensor(initiator, dtype=torch.float32).contiguous().reshape(-1)
    if W.numel() != n0 * n0:
        raise ValueError("initiator must have n0*n0 entries")
    dt = _idtype(id_bytes)
    if src is None:
        src = torch.empty(count, dtype=dt, device="cuda")
    if dst is None:
        dst = torch.empty(count, dtype=dt, device="cuda")
    _check(lib.kron_generate_range(n0, C.c_void_p(W.data_ptr()), k, num_edges, e_begin, count, mode, seed, graph_id,
                                   id_bytes, _ptr(src), _ptr(dst), _stream(stream)))
    return src, dst


# ----------------------------------------------------------------------------- PBA
def pba_workspace_bytes(n, m, num_parts, num_faction_members=0):
    return int(load().pba_workspace_bytes(n, m, num_parts, num_faction_members))


def pba_generate(n, m, num_parts, p_inter, *, seed=0, graph_id=0, faction_off=None, faction_members=None,
                 id_bytes=4, src=None, dst=None, ws=None, stream=None):
    """Parallel Barabasi-Albert edges into device tensors."""
    _require_cuda()
    lib = load()
    dt = _idtype(id_bytes)
    E = n * m
    if src is None:
        src = torch.empty(E, dtype=dt, device="cuda")
    if dst is None:
        dst = torch.empty(E, dtype=dt, device="cuda")
    foff = fmem = None
    nmem = 0
    if faction_off is not None:
        import numpy as np
        foff = np.ascontiguousarray(faction_off, np.uint32)
        nmem = int(foff[-1])
        fmem = np.ascontiguousarray(faction_members if faction_members is not None else [], np.uint32)
        if fmem.size == 0:
            fmem = np.zeros(1, np.uint32)
    need = pba_workspace_bytes(n, m, num_parts, nmem)
    if ws is None:
        ws = workspace(need)
    _check(lib.pba_generate(n, m, num_parts, float(p_inter),
                            None if foff is None else foff.ctypes.data_as(_vp),
                            None if fmem is None else fmem.ctypes.data_as(_vp),
                            seed, graph_id, id_bytes, _ptr(src), _ptr(dst), _ptr(ws), ws.numel(), _stream(stream)))
    return src, dst


# ----------------------------------------------------------------------------- CSR
def edges_to_csr_workspace_bytes(n, num_edges, id_bytes, flags):
    return int(load().edges_to_csr_workspace_bytes(n, num_edges, id_bytes, flags))


def edges_to_csr(n, src, dst, *, flags=0, want_hist=True, want_dups=True, row_ptr=None, col=None, ws=None,
                 stream=None):
    """CSR of (src, dst): returns (row_ptr, col, hist32 or None, dups tensor or None)."""
    _require_cuda()
    lib = load()
    assert src.dtype == dst.dtype and src.numel() == dst.numel()
    id_bytes = src.element_size()
    E = src.numel()
    N = 2 * E if flags & CSR_SYMMETRIZE else E
    if row_ptr is None:
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=src.device)
    if col is None:
        col = torch.empty(max(N, 1), dtype=src.dtype, device=src.device)
    hist = torch.empty(32, dtype=torch.int64, device=src.device) if want_hist else None
    dups = torch.empty(1, dtype=torch.int64, device=src.device) if want_dups else None
    need = edges_to_csr_workspace_bytes(n, E, id_bytes, flags)
    if ws is None:
        ws = workspace(need, src.device)
    _check(lib.edges_to_csr(n, E, _ptr(src), _ptr(dst), id_bytes, flags, _ptr(row_ptr), _ptr(col), _ptr(hist),
                            _ptr(dups), _ptr(ws), ws.numel(), _stream(stream)))
    return row_ptr, col, hist, dups


def edges_to_csr_noalloc(n, src, dst, *, flags=0, want_hist=True, want_dups=True, row_ptr=None, col=None,
                         stream=None):
    """edges_to_csr with the library's static scratch array as its workspace
    (no device allocation inside the call when row_ptr and col are given);
    returns (row_ptr, col, hist32 or None, dups tensor or None)."""
    _require_cuda()
    lib = load()
    assert src.dtype == dst.dtype and src.numel() == dst.numel()
    E = src.numel()
    N = 2 * E if flags & CSR_SYMMETRIZE else E
    if row_ptr is None:
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=src.device)
    if col is None:
        col = torch.empty(max(N, 1), dtype=src.dtype, device=src.device)
    hist = torch.empty(32, dtype=torch.int64, device=src.device) if want_hist else None
    dups = torch.empty(1, dtype=torch.int64, device=src.device) if want_dups else None
    _check(lib.edges_to_csr_noalloc(n, E, _ptr(src), _ptr(dst), src.element_size(), flags, _ptr(row_ptr), _ptr(col),
                                    _ptr(hist), _ptr(dups), _stream(stream)))
    return row_ptr, col, hist, dups


def kron_generate_csr(n0, initiator, k, num_edges, *, mode=KRON_SAMPLE, seed=0, graph_id=0, id_bytes=4, flags=0,
                      want_hist=True, want_dups=True, src=None, dst=None, row_ptr=None, col=None, ws=None,
                      stream=None):
    """kron_generate followed by edges_to_csr in one library call (the sampler
    counts the sort's digit histogram): returns (src, dst, row_ptr, col,
    hist32 or None, dups tensor or None)."""
    _require_cuda()
    lib = load()
    W = torch.as_tensor(initiator, dtype=torch.float32).contiguous().reshape(-1)
    if W.numel() != n0 * n0:
        raise ValueError("initiator must have n0*n0 entries")
    n = n0 ** k
    if n > 1 << 32:
        raise ValueError(f"{n0}^{k} vertices exceed 2^32")
    dt = _idtype(id_bytes)
    N = 2 * num_edges if flags & CSR_SYMMETRIZE else num_edges
    if src is None:
        src = torch.empty(num_edges, dtype=dt, device="cuda")
    if dst is None:
        dst = torch.empty(num_edges, dtype=dt, device="cuda")
    if row_ptr is None:
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    if col is None:
        col = torch.empty(max(N, 1), dtype=dt, device="cuda")
    hist = torch.empty(32, dtype=torch.int64, device="cuda") if want_hist else None
    dups = torch.empty(1, dtype=torch.int64, device="cuda") if want_dups else None
    if ws is None:
        ws = workspace(edges_to_csr_workspace_bytes(n, num_edges, id_bytes, flags))
    _check(lib.kron_generate_csr(n0, C.c_void_p(W.data_ptr()), k, num_edges, mode, seed, graph_id, id_bytes,
                                 _ptr(src), _ptr(dst), flags, _ptr(row_ptr), _ptr(col), _ptr(hist), _ptr(dups),
                                 _ptr(ws), ws.numel(), _stream(stream)))
    return src, dst, row_ptr, col, hist, dups


# ----------------------------------------------------------------------------- statistics
def graph_stats_workspace_bytes(n, num_edges, id_bytes):
    return int(load().graph_stats_workspace_bytes(n, num_edges, id_bytes))


def graph_stats(n, src, dst, *, num_samples=10_000, seed=0, graph_id=0, ws=None, out=None, stream=None):
    """(hist32, gamma, closed) device tensors for one edge list."""
    _require_cuda()
    lib = load()
    id_bytes = src.element_size()
    E = src.numel()
    if out is None:
        out = (torch.empty(32, dtype=torch.int64, device=src.device), torch.empty(1, dtype=torch.float64, device=src.device),
               torch.empty(1, dtype=torch.int64, device=src.device))
    hist, gamma, closed = out
    if ws is None:
        ws = workspace(graph_stats_workspace_bytes(n, E, id_bytes), src.device)
    _check(lib.graph_stats(n, E, _ptr(src), _ptr(dst), id_bytes, num_samples, seed, graph_id, _ptr(hist), _ptr(gamma),
                           _ptr(closed), _ptr(ws), ws.numel(), _stream(stream)))
    return hist, gamma, closed


# ----------------------------------------------------------------------------- ensemble
def path_stats_workspace_bytes(n):
    return int(load().path_stats_workspace_bytes(n))


def path_stats(n, row_ptr, col, sources, *, ws=None, out=None, stream=None):
    """(sum of BFS distances, reachable pairs, largest distance) from `sources`
    over a symmetric CSR; returns the device tensor of 3 u64 (as int64)."""
    _require_cuda()
    lib = load()
    import numpy as np
    srcs = np.ascontiguousarray(sources, np.int64)
    if out is None:
        out = torch.empty(3, dtype=torch.int64, device=row_ptr.device)
    if ws is None:
        ws = workspace(path_stats_workspace_bytes(n), row_ptr.device)
    _check(lib.path_stats(n, _ptr(row_ptr), _ptr(col), col.element_size(), srcs.ctypes.data_as(_vp), srcs.size,
                          _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def kron_perturbed(n0, seed_matrix, k, p_add, p_del, capacity, *, seed=0, graph_id=0, id_bytes=4, ws=None,
                   stream=None):
    """Kronecker expansion with the seed modified per meta-edge: returns
    (src, dst) device tensors trimmed to the edge count."""
    _require_cuda()
    lib = load()
    import numpy as np
    W = np.ascontiguousarray(seed_matrix, np.float32).reshape(-1)
    if W.size != n0 * n0:
        raise ValueError("seed matrix must have n0*n0 entries")
    dt = _idtype(id_bytes)
    src = torch.empty(max(capacity, 1), dtype=dt, device="cuda")
    dst = torch.empty(max(capacity, 1), dtype=dt, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    if ws is None:
        ws = workspace(lib.kron_perturbed_workspace_bytes(capacity))
    _check(lib.kron_perturbed(n0, W.ctypes.data_as(_vp), k, float(p_add), float(p_del), seed, graph_id, id_bytes,
                              capacity, _ptr(src), _ptr(dst), _ptr(cnt), _ptr(ws), ws.numel(), _stream(stream)))
    m = int(cnt.item())
    return src[:m], dst[:m]


def kron_xor_random(n0, seed_matrix, k, num_random, *, seed=0, graph_id=0, id_bytes=4, ws=None, stream=None):
    """CSR (row_ptr, col[:row_ptr[n]]) of the Kronecker power of a 0/1 seed XOR
    the random graph of num_random uniform pair draws."""
    _require_cuda()
    lib = load()
    import numpy as np
    W = np.ascontiguousarray(seed_matrix, np.float32).reshape(-1)
    if W.size != n0 * n0:
        raise ValueError("seed matrix must have n0*n0 entries")
    e0 = int((W != 0).sum())
    n = n0 ** k
    need = int(lib.kron_xor_random_workspace_bytes(n0, W.ctypes.data_as(_vp), k, num_random, id_bytes))
    if need == 0:  # rejected arguments: let the library say why, before allocating anything
        _check(lib.kron_xor_random(n0, W.ctypes.data_as(_vp), k, num_random, seed, graph_id, id_bytes, None, None,
                                   None, 0, _stream(stream)))
    if ws is None:
        ws = workspace(need)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(max(e0 ** k + num_random, 1), dtype=_idtype(id_bytes), device="cuda")
    _check(lib.kron_xor_random(n0, W.ctypes.data_as(_vp), k, num_random, seed, graph_id, id_bytes, _ptr(row_ptr),
                               _ptr(col), _ptr(ws), ws.numel(), _stream(stream)))
    return row_ptr, col


def block_matrix(n, src, dst, blocks, *, out=None, stream=None):
    """Coarse adjacency matrix [blocks, blocks] (int64 device tensor)."""
    _require_cuda()
    assert src.dtype == dst.dtype and src.numel() == dst.numel()
    if out is None:
        out = torch.empty((blocks, blocks), dtype=torch.int64, device=src.device)
    _check(load().block_matrix(n, src.numel(), _ptr(src), _ptr(dst), src.element_size(), blocks, _ptr(out),
                               _stream(stream)))
    return out


def graph_descs(rows):
    """ctypes array of GraphDesc from dicts (kind 'pba' or 'kron')."""
    arr = (GraphDesc * len(rows))()
    for d, r in zip(arr, rows):
        d.graph_id = r["graph_id"]
        d.seed = r["seed"]
        if r["kind"] == "pba":
            d.kind, d.n, d.m, d.num_parts, d.p_inter = GRAPH_PBA, r["n"], r["m"], r["num_parts"], r["p_inter"]
        else:
            import numpy as np
            W = np.asarray(r["initiator"], np.float32).ravel()
            d.kind, d.n0, d.k, d.num_edges = GRAPH_KRON, r["n0"], r["k"], r["num_edges"]
            for i, x in enumerate(W):
                d.initiator[i] = float(x)
    return arr


def ensemble_workspace_bytes(descs, max_batch_edges):
    return int(load().ensemble_workspace_bytes(C.cast(descs, _vp), len(descs), max_batch_edges))


def ensemble_generate(descs, *, num_samples=10_000, stat_seed=0, max_batch_edges=1 << 28, ws=None, out=None,
                      stream=None, tuning=None, check=False):
    """Batched ensemble: returns (hist [count,32], gamma [count], closed [count]) device tensors.
    tuning: an EnsembleTuning (ensemble_tuning(...)); None = the library's
    default tuning with this max_batch_edges.  check: synchronise and raise
    SfgenError(EDEVICE) if a kernel reported a device error."""
    _require_cuda()
    lib = load()
    count = len(descs)
    if out is None:
        out = (torch.empty((count, 32), dtype=torch.int64, device="cuda"),
               torch.empty(count, dtype=torch.float64, device="cuda"),
               torch.empty(count, dtype=torch.int64, device="cuda"))
    hist, gamma, closed = out
    budget = tuning.max_batch_edges if tuning is not None else max_batch_edges
    if ws is None:
        ws = workspace(ensemble_workspace_bytes(descs, budget))
    if tuning is None:
        _check(lib.ensemble_generate(C.cast(descs, _vp), count, num_samples, stat_seed, max_batch_edges, _ptr(hist),
                                     _ptr(gamma), _ptr(closed), _ptr(ws), ws.numel(), _stream(stream)))
    else:
        _check(lib.ensemble_generate_tuned(C.cast(descs, _vp), count, num_samples, stat_seed, C.byref(tuning),
                                           _ptr(hist), _ptr(gamma), _ptr(closed), _ptr(ws), ws.numel(),
                                           _stream(stream)))
    if check:
        code = device_error(stream)
        if code:
            raise SfgenError(SFG_EDEVICE, f"ensemble_generate: device error word {code}")
    return hist, gamma, closed


# ----------------------------------------------------------------------------- MLP surrogate
def mlp_shape(d_in, width=256, d_out=34, hidden=3):
    return MlpShape(d_in, width, d_out, hidden)


def mlp_param_count(shape):
    return int(load().mlp_param_count(C.byref(shape)))


def mlp_workspace_bytes(shape, batch):
    return int(load().mlp_workspace_bytes(C.byref(shape), batch))


def mlp_forward(shape, params, x, ws, y=None, stream=None):
    lib = load()
    B = x.shape[0]
    if y is None:
        y = torch.empty((B, shape.d_out), dtype=torch.float32, device=x.device)
    _check(lib.mlp_forward(C.byref(shape), B, _ptr(params), _ptr(x), _ptr(y), _ptr(ws), ws.numel(), _stream(stream)))
    return y


def mlp_backward(shape, params, dy, ws, grad=None, dx=None, want_grad=True, want_dx=False, stream=None):
    lib = load()
    B = dy.shape[0]
    if want_grad and grad is None:
        grad = torch.empty(mlp_param_count(shape), dtype=torch.float32, device=dy.device)
    if want_dx and dx is None:
        dx = torch.empty((B, shape.d_in), dtype=torch.float32, device=dy.device)
    _check(lib.mlp_backward(C.byref(shape), B, _ptr(params), _ptr(dy), _ptr(grad if want_grad else None),
                            _ptr(dx if want_dx else None), _ptr(ws), ws.numel(), _stream(stream)))
    return grad, dx


def mlp_mse_grad(y, target, ws, mask=None, col_weight=None, dy=None, loss=None, stream=None):
    lib = load()
    B, D = y.shape
    if dy is None:
        dy = torch.empty_like(y)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=y.device)
    _check(lib.mlp_mse_grad(B, D, _ptr(y), _ptr(target), _ptr(mask), _ptr(col_weight), _ptr(dy), _ptr(loss), _ptr(ws),
                            ws.numel(), _stream(stream)))
    return dy, loss


def adam_step_device(params, grad, m, v, lr_dev, step_dev, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """Adam with the learning rate (float32 [1]) and the step counter (int32
    [1], incremented by the call) in device memory: capturable into a graph."""
    assert lr_dev.dtype == torch.float32 and step_dev.dtype == torch.int32
    _check(load().adam_step_device(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), _ptr(lr_dev), beta1,
                                   beta2, eps, _ptr(step_dev), _stream(stream)))


def mlp_train_workspace_bytes(shape, batch):
    return int(load().mlp_train_workspace_bytes(C.byref(shape), batch))


def mlp_train_step(shape, batch, params, x, target, m, v, lr_dev, step_dev, ws, *, rows=None, mask=None,
                   col_weight=None, loss=None, grad=None, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One fused training step (forward, loss gradient, backward, Adam) in four
    launches; returns the device loss (float32 [1]).  rows: int64 [batch]
    device indices into x / target / mask, or None for the first `batch` rows."""
    assert lr_dev.dtype == torch.float32 and step_dev.dtype == torch.int32
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
    if rows is not None:
        assert rows.dtype == torch.int64 and rows.numel() == batch
    _check(load().mlp_train_step(C.byref(shape), batch, _ptr(params), _ptr(x), _ptr(target), _ptr(mask),
                                 _ptr(col_weight), _ptr(rows), _ptr(m), _ptr(v), _ptr(lr_dev), beta1, beta2, eps,
                                 _ptr(step_dev), _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(), _stream(stream)))
    return loss


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().adam_step(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), lr, beta1, beta2, eps, step,
                            _stream(stream)))
