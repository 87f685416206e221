#!/usr/bin/env python3
"""Benchmark of the scale-free graph generation hot path on one MI355X.

A step is one pass of the hot path over the 1-billion-vertex-scale Kronecker
workload: sample 5 x 2^30 edges from a 3x3 initiator zero-padded to 4x4 with
15 levels (2^30 vertex ids, int64 endpoints, ~80 GB edge list), then sort them
into compressed sparse rows with the repeated-edge count and the 32-bin degree
histogram -- one library call (kron_generate_csr), in which the sampler also
counts the sort's digit histogram.  The same step as two calls (kron_generate,
then edges_to_csr with its own histogram pass) is timed beside it.  Inputs are synthetic and produced on the GPU by the generator
itself; every buffer is resident in HBM before the timed region starts.

One JSON line is printed.  Besides the headline edges/s it carries the
roofline of the dominant kernel (the radix-sort pass), the CPU oracle timed
on a bounded sample of the same workload, the PBA workload (2^27 vertices,
m = 5, 1,024 partitions), PBA generation at the paper's largest size (2^30
vertices, m = 5), the batched-versus-plain ensemble rate (4,096 PBA and
Kronecker graphs with their statistics, batch budget from the autotuner),
the enumerated Kronecker power of the Fig. 2 seed, the two randomized PK
variants and the block matrix on that seed, and one surrogate training step.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("csr.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1003_3684_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_from_profile(kernel_hash):
    """HBM bytes per radix-pass launch from the committed rocprofv3 counter
    summary, or None if it was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "radix_pass_kron_scale_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _valu_per_edge_from_profile():
    """VALU wave-instructions per edge of the Kronecker sampler from the
    committed rocprofv3 SQ-counter summary, or None if it was taken on a
    different sampler source."""
    h = hashlib.sha256()
    for f in ("kron.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1003_3684_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    path = os.path.join(ROOT, "profiles", "kron_sample_kron_scale_valu.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    try:
        return float(vals["valu_instructions_per_edge"])
    except (KeyError, ValueError):
        return None


# Algorithmic HBM bytes per PBA edge, from the method's data flow: a slot's
# label written and read twice at 2 B (6), a 4-byte rank per slot for the
# exchange written and read (8; here the ranks stay in LDS), the selection
# lists written and gathered (8), the edge written (8) -- about 30 B.
PBA_BYTES_PER_EDGE = 30


def _pba_profile_values():
    """HBM bytes per PBA generation at 2^27 and 2^30 vertices from the
    committed rocprofv3 counter summary, or {} if it was taken on a different
    source of the PBA kernels."""
    h = hashlib.sha256()
    for f in ("pba.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1003_3684_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    path = os.path.join(ROOT, "profiles", "pba_kernels_n2e27_n2e30.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#") and not line.startswith("##"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("pba_source_sha256_16") != h.hexdigest()[:16]:
        return {}
    out = {}
    for key in ("hbm_bytes_per_generation_n2e27", "hbm_bytes_per_generation_n2e30"):
        try:
            out[key] = float(vals[key])
        except (KeyError, ValueError):
            pass
    return out


def _pba_roofline(edges, ms, traffic):
    """The PBA generation against HBM: PBA_BYTES_PER_EDGE per edge over the
    generation's time (all its passes), beside the bytes the counters saw."""
    achieved = edges * PBA_BYTES_PER_EDGE / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
            "traffic": traffic, "kernel": "pba_generate (all passes)", "algorithmic_bytes_per_edge": PBA_BYTES_PER_EDGE,
            "note": "the chain walks are bound by L2 misses of one random read per element (see the PBA profile)"}


def _host_info():
    """CPU model, usable cores and RAM of the host the CPU baseline ran on."""
    model, ram = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu": model, "usable_cores": cores, "ram_gib": ram}


class _OneCore:
    """Pins the calling thread (the one that runs the oracle) to one host core
    for the duration of a with-block and restores its affinity after."""

    def __enter__(self):
        self.saved = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
        self.core = min(self.saved) if self.saved else None
        if self.saved:
            os.sched_setaffinity(0, {self.core})
        return self

    def __exit__(self, *exc):
        if self.saved:
            os.sched_setaffinity(0, self.saved)
        return False


def _oracle_config_times(wl, full_cfg3):
    """The oracle on the test configurations, each in full: PBA n = 65,536
    (generation + symmetrized CSR), Kronecker 2x2 at 20 levels (2^24 edges,
    generation + directed CSR with duplicate count), and -- with full_cfg3 --
    PBA at 2^27 vertices, p = 0.1 (generation + symmetrized CSR + degree
    histogram)."""
    import oracle
    out = {}

    def pba(c):
        t0 = time.perf_counter()
        src, dst = oracle.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], c["seed"])
        t1 = time.perf_counter()
        oracle.edges_to_csr(c["n"], src, dst, symmetrize=True)
        oracle.degree_histogram(c["n"], src, dst)
        t2 = time.perf_counter()
        E = c["n"] * c["m"]
        return {"edges": E, "gen_s": t1 - t0, "csr_s": t2 - t1, "edges_per_s": E / (t2 - t0)}

    out[wl.PBA_SMALL["name"]] = pba(wl.PBA_SMALL)
    c = wl.KRON_K20
    t0 = time.perf_counter()
    src, dst = oracle.kron_sample(c["n0"], c["initiator"], c["k"], c["num_edges"], c["seed"])
    t1 = time.perf_counter()
    oracle.edges_to_csr(c["n0"] ** c["k"], src, dst)
    t2 = time.perf_counter()
    out[c["name"]] = {"edges": c["num_edges"], "gen_s": t1 - t0, "csr_s": t2 - t1,
                      "edges_per_s": c["num_edges"] / (t2 - t0)}
    del src, dst
    if full_cfg3:
        out[wl.PBA_SCALE[1]["name"]] = pba(wl.PBA_SCALE[1])
    return out


def _cpu_baseline(cfg, sample_edges, wl=None, full_cfg3=False):
    """The oracle, pinned to one host core, on the first `sample_edges` edges
    of the workload: sampling plus CSR of that sample; scaled to edges/s.
    Beside it, the oracle's times on the small configurations in full."""
    import numpy as np
    import oracle
    n = cfg["n0"] ** cfg["k"]
    with _OneCore() as pin:
        t0 = time.perf_counter()
        src, dst = oracle.kron_sample(cfg["n0"], cfg["initiator"], cfg["k"], sample_edges, cfg["seed"])
        t1 = time.perf_counter()
        oracle.edges_to_csr(n, src, dst)
        oracle.degree_histogram(n, src, dst)
        t2 = time.perf_counter()
        del src, dst
        # the per-vertex part of the CSR and histogram (row starts and degrees
        # of all n vertices), paid once per graph whatever its edge count
        none = np.zeros(0, np.int64)
        t3 = time.perf_counter()
        oracle.edges_to_csr(n, none, none)
        oracle.degree_histogram(n, none, none)
        t_vertex = time.perf_counter() - t3
        configs = _oracle_config_times(wl, full_cfg3) if wl is not None else None
        pinned = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    per_edge = max(t2 - t0 - t_vertex, 1e-9) / sample_edges
    E = cfg["num_edges"]
    out = {"value": E / (t_vertex + per_edge * E), "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": f"first {sample_edges} edges of the workload: oracle Kronecker sampling ({t1 - t0:.1f} s) "
                     f"+ CSR sort and degree histogram ({t2 - t1:.1f} s, of which {t_vertex:.1f} s is the "
                     f"per-vertex part over all {n} vertices), one thread pinned to host core {pin.core}; value = "
                     f"all {E} edges over (per-vertex time + sample time per edge x {E})",
           "sample_edges_per_s": sample_edges / (t2 - t0), "pinned_cores": pinned, "host": _host_info()}
    if configs is not None:
        out["configs"] = configs
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=1 << 25, help="edges in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on the 2^27-vertex PBA configuration in full (minutes)")
    ap.add_argument("--no-extras", action="store_true", help="skip the PBA and ensemble extras")
    ap.add_argument("--only", choices=("pba", "cpu", "surrogate", "mlp"), default=None,
                    help="run only one part and print its JSON: 'pba' = PBA generation at 2^27 and 2^30 vertices "
                         "with per-kernel times (for profiling runs); 'cpu' = the CPU oracle baseline; 'mlp' = the "
                         "surrogate's training step, fused and unfused")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy three times (the reference kernel of known "
                         "size for scaling the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": a.numel() * 8,
                          "bytes_written_per_copy": a.numel() * 8, "copies": 3}), flush=True)
        return
    if args.only == "cpu":
        from paper_1003_3684_amd import workloads as wl
        print(json.dumps({"cpu_baseline": _cpu_baseline(wl.KRON_SCALE, args.cpu_sample, wl, args.cpu_full)}),
              flush=True)
        return
    if args.only == "surrogate":
        import torch
        from paper_1003_3684_amd import native as sfg
        from paper_1003_3684_amd import workloads as wl
        sfg.load()
        print(json.dumps({"surrogate": _bench_surrogate(sfg, wl, torch)}), flush=True)
        return
    if args.only == "mlp":
        import torch
        from paper_1003_3684_amd import native as sfg
        sfg.load()
        print(json.dumps({"mlp_step": _bench_mlp(sfg, torch)}), flush=True)
        return
    if args.only == "pba":
        import torch
        from paper_1003_3684_amd import native as sfg
        from paper_1003_3684_amd import workloads as wl
        sfg.load()
        print(json.dumps({"pba": _bench_pba(sfg, wl, torch, paths=False),
                          "pba_paper_scale": _bench_pba_paper(sfg, wl, torch)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU sharding is a design note, "
              "not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1003_3684_amd import native as sfg
    from paper_1003_3684_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    sfg.load()
    cfg = wl.KRON_SCALE
    n0, W, k, E, seed = cfg["n0"], cfg["initiator"], cfg["k"], cfg["num_edges"], cfg["seed"]
    n = n0 ** k
    flags = 0  # directed CSR
    dt = torch.int64
    src = torch.empty(E, dtype=dt, device="cuda")
    dst = torch.empty(E, dtype=dt, device="cuda")
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(E, dtype=dt, device="cuda")
    hist = torch.empty(32, dtype=torch.int64, device="cuda")
    dups = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = sfg.workspace(sfg.edges_to_csr_workspace_bytes(n, E, 8, flags))
    stream = torch.cuda.current_stream()
    lib = sfg.load()
    import ctypes as C
    Wt = torch.as_tensor(W, dtype=torch.float32).contiguous().reshape(-1)
    wptr = C.c_void_p(Wt.data_ptr())
    sptr = C.c_void_p(stream.cuda_stream)

    def step():
        # One call: the sampler writes the edge list and counts the sort's
        # digit histogram; the CSR build follows on the same stream.
        rc = lib.kron_generate_csr(n0, wptr, k, E, 0, seed, 0, 8, C.c_void_p(src.data_ptr()),
                                   C.c_void_p(dst.data_ptr()), flags, C.c_void_p(row_ptr.data_ptr()),
                                   C.c_void_p(col.data_ptr()), C.c_void_p(hist.data_ptr()),
                                   C.c_void_p(dups.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(), sptr)
        assert rc == 0, lib.sfg_last_error()

    def two_call_step():
        rc = lib.kron_generate(n0, wptr, k, E, 0, seed, 0, 8, C.c_void_p(src.data_ptr()),
                               C.c_void_p(dst.data_ptr()), sptr)
        assert rc == 0, lib.sfg_last_error()
        rc = lib.edges_to_csr(n, E, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), 8, flags,
                              C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col.data_ptr()), C.c_void_p(hist.data_ptr()),
                              C.c_void_p(dups.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(), sptr)
        assert rc == 0, lib.sfg_last_error()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    sfg.profile_reset()
    sfg.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sfg.profile_enable(False)
    assert sfg.device_error() == 0
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    edges_per_s = E / (ms_per_step / 1e3)
    fused_hist = hist.clone()

    kernels = {}
    for name in ("kron_sample", "csr_prepare", "radix_pass", "csr_run_starts", "csr_finish", "csr_rowfill", "fill",
                 "csr_digit_bases"):
        cnt, tot = sfg.profile_query(name)
        if cnt:
            kernels[name] = {"launches_per_step": cnt // args.steps, "ms_per_step": tot / args.steps}
    # Radix pass roofline: in the one-call path the sampler writes the 8-byte
    # keys, so every pass reads one key and writes one key (the last pass: one
    # 8-byte column) -- 16 B per entry and pass.
    passes = kernels["radix_pass"]["launches_per_step"]
    radix_bytes = E * 16 * passes
    radix_ms = kernels["radix_pass"]["ms_per_step"]
    achieved = radix_bytes / (radix_ms / 1e3) / 1e9
    traffic = _traffic_from_profile(_kernel_source_hash())
    gen_ms = kernels["kron_sample"]["ms_per_step"]
    total_kernel_ms = sum(v["ms_per_step"] for v in kernels.values())
    # The sampler is bound by VALU issue: 256 CUs x 4 SIMDs x 2.4 GHz / 4
    # cycles per wave64 instruction; its instruction count per edge comes from
    # the committed SQ-counter profile (null when the source has changed).
    valu_peak = 256 * 4 * 2.4e9 / 4
    vpe = _valu_per_edge_from_profile()
    # (the sampler writes src, dst and the sort key: 24 B per edge)
    generation = {"edges_per_s": E / (gen_ms / 1e3), "write_GBs": 24 * E / (gen_ms / 1e3) / 1e9, "bound": "alu",
                  "valu_instr_per_edge": vpe,
                  "alu_frac": None if vpe is None else vpe * E / 64 / (gen_ms / 1e3) / valu_peak,
                  "alu_peak_wave_instr_per_s": valu_peak}
    result = {
        "metric": "edges/s + achieved HBM GB/s at 1B-vertex scale; batched vs plain graphs/s",
        "value": edges_per_s,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (generated on the GPU by the Kronecker sampler, seed 13)",
        "config": {"workload": cfg["name"], "generator": "kronecker-sample", "n0": n0, "levels": k,
                   "vertices": n, "edges": E, "id_bytes": 8, "csr": "directed, duplicate count, degree histogram",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "radix_pass",
                     "algorithmic_bytes_per_step": radix_bytes, "launches_per_step": passes},
        "kernels": kernels,
        "generation": generation,
        "csr_edges_per_s": E / ((total_kernel_ms - gen_ms) / 1e3),
    }
    if not args.no_extras:
        # The same step as two library calls (kron_generate, then edges_to_csr
        # with its own histogram pass over the edge list), for comparison.
        two_call_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            two_call_step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert sfg.device_error() == 0
        result["two_call_step"] = {"ms_per_step": (t1 - t0) * 1e3 / 3,
                                   "degree_hist_identical": bool(torch.equal(hist, fused_hist))}
    del src, dst, row_ptr, col, ws
    torch.cuda.empty_cache()

    if not args.no_extras:
        result["extras"] = {"pba": _bench_pba(sfg, wl, torch), "pba_paper_scale": _bench_pba_paper(sfg, wl, torch),
                            "ensemble": _bench_ensemble(sfg, wl, torch),
                            "kron_enumerate": _bench_enumerate(sfg, wl, torch),
                            "randomized_pk": _bench_randomized_pk(sfg, wl, torch), "mlp": _bench_mlp(sfg, torch),
                            "surrogate": _bench_surrogate(sfg, wl, torch)}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = _cpu_baseline(cfg, args.cpu_sample, wl, full_cfg3=args.cpu_full)
    print(json.dumps(result), flush=True)


PBA_KERNELS = ("pba_fill", "pba_resolve", "pba_tile_table", "pba_count", "pba_scan", "pba_substitute")


def _pba_breakdown(sfg, gen, reps):
    """Per-kernel milliseconds per generation, from the library's launch events."""
    sfg.profile_reset()
    sfg.profile_enable(True)
    for _ in range(reps):
        gen()
    sfg.profile_enable(False)
    out = {}
    for name in PBA_KERNELS:
        cnt, tot = sfg.profile_query(name)
        if cnt:
            out[name] = {"launches": cnt // reps, "ms": tot / reps}
    return out


def _bench_pba_paper(sfg, wl, torch, reps=2):
    """PBA generation at the paper's largest size: 2^30 vertices, m = 5
    (5.4e9 edges, int32), 1,024 partitions, p = 0.1; edge list only, as the
    paper times it.  For context, the paper generates 1 billion vertices and
    5 billion edges in under 13 s on a 1,024-processor cluster."""
    c = wl.PBA_PAPER
    E = c["n"] * c["m"]
    src = torch.empty(E, dtype=torch.int32, device="cuda")
    dst = torch.empty(E, dtype=torch.int32, device="cuda")
    ws = sfg.workspace(sfg.pba_workspace_bytes(c["n"], c["m"], c["num_parts"]))

    def gen():
        sfg.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], seed=c["seed"], src=src, dst=dst, ws=ws)

    gen()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        gen()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    kernels = _pba_breakdown(sfg, gen, reps)
    del src, dst, ws
    torch.cuda.empty_cache()
    return {"workload": c["name"], "edges": E, "gen_ms": ms, "gen_edges_per_s": E / (ms / 1e3),
            "kernels": kernels,
            "roofline": _pba_roofline(E, ms, _pba_profile_values().get("hbm_bytes_per_generation_n2e30")),
            "paper_context": "under 13 s for 1e9 vertices and 5e9 edges on 1,024 processors of a cluster"}


def _bench_pba(sfg, wl, torch, reps=3, paths=True):
    """PBA at 2^27 vertices, m = 5, 1,024 partitions, p = 0.1: generation plus
    the symmetrized CSR with degree histogram."""
    c = wl.PBA_SCALE[1]
    E = c["n"] * c["m"]
    src = torch.empty(E, dtype=torch.int32, device="cuda")
    dst = torch.empty(E, dtype=torch.int32, device="cuda")
    ws = sfg.workspace(max(sfg.pba_workspace_bytes(c["n"], c["m"], c["num_parts"]),
                           sfg.edges_to_csr_workspace_bytes(c["n"], E, 4, sfg.CSR_SYMMETRIZE)))
    rp = torch.empty(c["n"] + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(2 * E, dtype=torch.int32, device="cuda")

    def gen():
        sfg.pba_generate(c["n"], c["m"], c["num_parts"], c["p_inter"], seed=c["seed"], src=src, dst=dst, ws=ws)

    def csr():
        sfg.edges_to_csr(c["n"], src, dst, flags=sfg.CSR_SYMMETRIZE, row_ptr=rp, col=col, ws=ws)

    gen()
    csr()
    torch.cuda.synchronize()
    a, b, d = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a.record()
    for _ in range(reps):
        gen()
    b.record()
    for _ in range(reps):
        csr()
    d.record()
    torch.cuda.synchronize()
    gen_ms, csr_ms = a.elapsed_time(b) / reps, b.elapsed_time(d) / reps
    out = {"workload": c["name"], "edges": E, "gen_ms": gen_ms, "gen_edges_per_s": E / (gen_ms / 1e3),
           "csr_ms": csr_ms, "step_edges_per_s": E / ((gen_ms + csr_ms) / 1e3),
           "kernels": _pba_breakdown(sfg, gen, reps),
           "roofline": _pba_roofline(E, gen_ms, _pba_profile_values().get("hbm_bytes_per_generation_n2e27"))}
    if not paths:
        del src, dst, rp, col, ws
        torch.cuda.empty_cache()
        return out
    # Table 2 analogue: average path length and diameter estimate from 64
    # sampled sources, on the symmetrized graph.
    import numpy as np
    del ws
    torch.cuda.empty_cache()
    sources = np.random.default_rng(c["seed"]).integers(0, c["n"], 64)
    pws = sfg.workspace(sfg.path_stats_workspace_bytes(c["n"]))
    t0 = time.perf_counter()
    res = sfg.path_stats(c["n"], rp, col, sources, ws=pws).cpu().numpy()
    path_s = time.perf_counter() - t0
    out["paths"] = {"sources": 64, "avg_path_length": float(res[0]) / max(int(res[1]), 1),
                    "diameter_estimate": int(res[2]), "seconds": path_s}
    del src, dst, rp, col, pws
    torch.cuda.empty_cache()
    return out


def _timed(torch, fn, reps=3):
    """Milliseconds per call of fn on the current stream (after one warm-up)."""
    out = fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        out = fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps, out


def _bench_randomized_pk(sfg, wl, torch, k=8):
    """The paper's two randomizations of the PK power and the community
    report, on the Fig. 2 seed at 8 levels (11^8 = 2.1e8 edges, 5^8
    vertices, int32 ids): the seed modified per meta-edge expansion
    (p_add = p_del = 0.05), the power XOR a random graph of 10^8 uniform
    pair draws (sorted into one CSR), and the 25 x 25 block matrix of the
    modified graph."""
    W = wl.FIG2_SEED.astype("float32")
    n = 5 ** k
    cap = 3 * 10 ** 8
    ws = sfg.workspace(sfg.load().kron_perturbed_workspace_bytes(cap))
    ms1, (src, dst) = _timed(torch, lambda: sfg.kron_perturbed(5, W, k, 0.05, 0.05, cap, seed=5, ws=ws))
    m = src.numel()
    ms3, _ = _timed(torch, lambda: sfg.block_matrix(n, src, dst, 25))
    del src, dst, ws
    torch.cuda.empty_cache()
    R = 10 ** 8
    ms2, (rp, col) = _timed(torch, lambda: sfg.kron_xor_random(5, W, k, R, seed=5))
    kept = int(rp[n])
    del rp, col
    torch.cuda.empty_cache()
    return {"workload": f"fig2_seed_k{k}",
            "modified_seed": {"edges": m, "ms": ms1, "edges_per_s": m / (ms1 / 1e3)},
            "xor_random": {"power_edges": 11 ** k, "random_pairs": R, "kept": kept, "ms": ms2,
                           "entries_per_s": (11 ** k + R) / (ms2 / 1e3)},
            "block_matrix": {"edges": m, "blocks": 25, "ms": ms3, "edges_per_s": m / (ms3 / 1e3)}}


def _bench_enumerate(sfg, wl, torch, k=9, reps=5):
    """The paper's deterministic Kronecker power of the Fig. 2 seed (11 edges,
    5 vertices) at 9 levels: 11^9 edges, int32 ids; bound by HBM writes."""
    E = 11 ** k
    src = torch.empty(E, dtype=torch.int32, device="cuda")
    dst = torch.empty(E, dtype=torch.int32, device="cuda")
    W = wl.FIG2_SEED.astype("float32")

    def run():
        sfg.kron_generate(5, W, k, E, mode=sfg.KRON_ENUMERATE, src=src, dst=dst)

    run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        run()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    gbs = 8 * E / (ms / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"workload": f"fig2_seed_k{k}", "edges": E, "ms": ms, "edges_per_s": E / (ms / 1e3),
            "write_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}


def _bench_mlp(sfg, torch, batch=4096, steps=50):
    """One surrogate training step (forward, masked MSE gradient, backward,
    Adam) at batch 4,096 on the 10 -> 256 x 3 -> 34 network."""
    shape = sfg.mlp_shape(10, 256, 34, 3)
    P = sfg.mlp_param_count(shape)
    g = torch.Generator(device="cuda").manual_seed(3)
    params = (torch.randn(P, device="cuda", generator=g) * 0.05).contiguous()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    x = torch.randn(batch, 10, device="cuda", generator=g)
    t = torch.randn(batch, 34, device="cuda", generator=g)
    ws = sfg.workspace(sfg.mlp_workspace_bytes(shape, batch))
    lws = sfg.workspace(4 * batch)

    def step(i):
        y = sfg.mlp_forward(shape, params, x, ws)
        dy, _ = sfg.mlp_mse_grad(y, t, lws)
        grad, _ = sfg.mlp_backward(shape, params, dy, ws)
        sfg.adam_step(params, grad, m, v, i + 1, lr=1e-3)

    step(0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        step(i + 1)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    # The same step captured once into a HIP graph (learning rate and step
    # counter in device memory) and replayed.
    y, dy = torch.empty(batch, 34, device="cuda"), torch.empty(batch, 34, device="cuda")
    loss, grad = torch.empty(1, device="cuda"), torch.empty_like(params)
    lr_dev = torch.full((1,), 1e-3, device="cuda")
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")

    def gstep():
        sfg.mlp_forward(shape, params, x, ws, y=y)
        sfg.mlp_mse_grad(y, t, lws, dy=dy, loss=loss)
        sfg.mlp_backward(shape, params, dy, ws, grad=grad)
        sfg.adam_step_device(params, grad, m, v, lr_dev, step_dev)

    gstep()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gstep()
    a.record()
    for _ in range(steps):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    ms_graph = a.elapsed_time(b) / steps
    del graph
    # The fused step: forward, loss gradient, backward and Adam in four launches.
    tws = sfg.workspace(sfg.mlp_train_workspace_bytes(shape, batch))

    def fstep():
        sfg.mlp_train_step(shape, batch, params, x, t, m, v, lr_dev, step_dev, tws, loss=loss)

    fstep()
    torch.cuda.synchronize()
    sfg.profile_reset()
    sfg.profile_enable(True)
    a.record()
    for _ in range(steps):
        fstep()
    b.record()
    torch.cuda.synchronize()
    sfg.profile_enable(False)
    ms_fused = a.elapsed_time(b) / steps
    kern = {}
    for name in ("mlp_round", "mlp_rows", "mlp_wgrad", "mlp_update"):
        cnt, tot = sfg.profile_query(name)
        kern[name] = tot / max(cnt, 1)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fstep()
    a.record()
    for _ in range(steps):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    ms_fused_graph = a.elapsed_time(b) / steps
    del graph
    macs = 10 * 256 + 2 * 256 * 256 + 256 * 34
    flops = 3 * 2 * batch * macs  # forward, input gradients, weight gradients
    return {"batch": batch, "ms_per_step": ms_fused, "ms_per_step_graph": ms_fused_graph,
            "launches_per_step": 4, "kernel_ms": kern,
            "unfused_ms_per_step": ms, "unfused_ms_per_step_graph": ms_graph, "unfused_launches_per_step": 26,
            "samples_per_s": batch / (ms_fused / 1e3), "tflops": flops / (ms_fused / 1e3) / 1e12,
            "mfma_peak_tflops_bf16": 2500.0,
            "note": "fused step: bf16 weights, then one launch runs forward, loss gradient and the "
                    "activation-gradient chain per 64-row block, one computes the weight-gradient tiles per "
                    "256-row slice, one sums the slices and applies Adam; a 256-wide network at batch 4,096 "
                    "stays latency-bound, far below the matrix-core roofline"}


def _bench_surrogate(sfg, wl, torch, graphs=100_000):
    """The surrogate trained on `graphs` graphs of the ensemble recipe (made
    by ensemble_generate) and inverted for the exponents 2.1 .. 3.0 on the
    2x2 Kronecker family at 14 levels: generator runs and seconds per target,
    with the surrogate-guided search and with the generator-only search, each
    answer judged by the generator."""
    from paper_1003_3684_amd import surrogate as sg
    res = sg.ensemble_study(wl.ensemble_table(graphs, seed=19))
    res["workload"] = f"ensemble_recipe_{graphs}_graphs_seed19"
    torch.cuda.empty_cache()
    return res


def _bench_ensemble(sfg, wl, torch, samples=10_000, stat_seed=5,
                    candidates=(1 << 26, 1 << 27, 1 << 28, 1 << 30)):
    """Graphs/s of the batched ensemble entry point against the same 4,096
    graphs made one by one (generator call, then the statistics call), with
    the statistics compared member by member.  The tuning (batch budget, tile
    size, persistent grid) is chosen first by the autotuner (each candidate
    runs the whole table; the tuner checks that all give the same
    statistics); the batched run is the captured graph of the batch sequence,
    replayed, and the same tuning enqueued without a graph is timed beside it."""
    import numpy as np
    from paper_1003_3684_amd import tune
    rows = wl.ensemble_table()
    tuned = tune.tune_ensemble(rows, candidates=candidates, num_samples=samples, stat_seed=stat_seed, save=False)
    max_batch_edges = tuned["best"]
    torch.cuda.empty_cache()
    descs = sfg.graph_descs(rows)
    count = len(rows)
    edges = sum(r["n"] * r["m"] if r["kind"] == "pba" else r["num_edges"] for r in rows)
    out = (torch.empty((count, 32), dtype=torch.int64, device="cuda"),
           torch.empty(count, dtype=torch.float64, device="cuda"),
           torch.empty(count, dtype=torch.int64, device="cuda"))
    ws = sfg.workspace(sfg.ensemble_workspace_bytes(descs, max_batch_edges))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(graph):
        tu = sfg.ensemble_tuning(max_batch_edges, tuned["grid_per_cu"], tuned["kron_items"], graph)
        sfg.ensemble_generate(descs, num_samples=samples, stat_seed=stat_seed, ws=ws, out=out, tuning=tu)
        torch.cuda.synchronize()
        a.record()
        sfg.ensemble_generate(descs, num_samples=samples, stat_seed=stat_seed, ws=ws, out=out, tuning=tu)
        b.record()
        torch.cuda.synchronize()
        assert sfg.device_error() == 0
        return a.elapsed_time(b) / 1e3, [t.cpu().numpy() for t in out]

    eager_s, eager_out = timed(False)
    batched_s, (bh, bg, bc) = timed(True)
    graph_same = all(np.array_equal(x, y, equal_nan=True) for x, y in zip((bh, bg, bc), eager_out))
    del ws
    torch.cuda.empty_cache()

    def nv(r):
        return r["n"] if r["kind"] == "pba" else r["n0"] ** r["k"]

    def ne(r):
        return r["n"] * r["m"] if r["kind"] == "pba" else r["num_edges"]

    emax = max(ne(r) for r in rows)
    nmax = max(nv(r) for r in rows)
    src = torch.empty(emax, dtype=torch.int32, device="cuda")
    dst = torch.empty(emax, dtype=torch.int32, device="cuda")
    pws = sfg.workspace(max(sfg.pba_workspace_bytes(r["n"], r["m"], r["num_parts"]) for r in rows if r["kind"] == "pba"))
    sws = sfg.workspace(sfg.graph_stats_workspace_bytes(nmax, emax, 4))
    ph = torch.empty((count, 32), dtype=torch.int64, device="cuda")
    pg = torch.empty(count, dtype=torch.float64, device="cuda")
    pc = torch.empty(count, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    for i, r in enumerate(rows):
        E = ne(r)
        s_, d_ = src[:E], dst[:E]
        if r["kind"] == "pba":
            sfg.pba_generate(r["n"], r["m"], r["num_parts"], r["p_inter"], seed=r["seed"], graph_id=r["graph_id"],
                             src=s_, dst=d_, ws=pws)
        else:
            sfg.kron_generate(r["n0"], r["initiator"], r["k"], E, seed=r["seed"], graph_id=r["graph_id"], src=s_,
                              dst=d_)
        sfg.graph_stats(nv(r), s_, d_, num_samples=samples, seed=stat_seed, graph_id=r["graph_id"], ws=sws,
                        out=(ph[i], pg[i:i + 1], pc[i:i + 1]))
    b.record()
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t0
    plain_s = a.elapsed_time(b) / 1e3
    same = bool(np.array_equal(bh, ph.cpu().numpy()) and np.array_equal(bc, pc.cpu().numpy())
                and np.array_equal(bg, pg.cpu().numpy(), equal_nan=True))
    del src, dst, pws, sws
    torch.cuda.empty_cache()
    return {"workload": f"ensemble_{count}_graphs_seed17", "graphs": count, "edges": edges,
            "wedge_samples": samples,
            "tuning": {"max_batch_edges": max_batch_edges, "grid_per_cu": tuned["grid_per_cu"],
                       "kron_items": tuned["kron_items"]},
            "tuner_seconds": {"budget": {str(c): round(t, 4) for c, t in tuned["seconds"].items()},
                              "kron_items": {str(c): round(t, 4) for c, t in tuned["tile_seconds"].items()},
                              "grid_per_cu": {str(c): round(t, 4) for c, t in tuned["grid_seconds"].items()}},
            "batched_s": batched_s, "batched_graphs_per_s": count / batched_s,
            "batched_edges_per_s": edges / batched_s, "batched_launch": "one captured HIP graph, replayed",
            "batched_no_graph_s": eager_s, "batched_no_graph_graphs_per_s": count / eager_s,
            "plain_s": plain_s, "plain_wall_s": plain_wall, "plain_graphs_per_s": count / plain_s,
            "speedup": plain_s / batched_s, "stats_identical": same and graph_same}


if __name__ == "__main__":
    main()
