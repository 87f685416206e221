"""Host logic of bench.py (no GPU): the hash-guarded readers of the committed
profile summaries, the host description in the CPU baseline, and the refusal
of multi-GPU runs."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1003_3684_amd" / "csrc").mkdir(parents=True)
    monkeypatch.setattr(mod, "ROOT", str(tmp_path))
    return mod


def _write(path, text):
    with open(path, "w") as f:
        f.write(text)


def test_traffic_reader_checks_the_source_hash(bench, tmp_path):
    prof = tmp_path / "profiles" / "radix_pass_kron_scale_counters.txt"
    assert bench._traffic_from_profile("abc") is None  # no file
    _write(prof, "# comment: x\nkernel_source_sha256_16: abc\nhbm_bytes_per_launch: 1.5e+11\n")
    assert bench._traffic_from_profile("abc") == 1.5e11
    assert bench._traffic_from_profile("abd") is None  # kernel changed since the counters
    _write(prof, "kernel_source_sha256_16: abc\nhbm_bytes_per_launch: n/a\n")
    assert bench._traffic_from_profile("abc") is None  # malformed value


def test_kernel_hash_covers_the_sort_sources(bench, tmp_path):
    csrc = tmp_path / "paper_1003_3684_amd" / "csrc"
    _write(csrc / "csr.hip", "a")
    _write(csrc / "common.hpp", "b")
    h0 = bench._kernel_source_hash()
    assert h0 == hashlib.sha256(b"ab").hexdigest()[:16]
    _write(csrc / "common.hpp", "c")
    assert bench._kernel_source_hash() != h0


def test_valu_reader_checks_the_sampler_hash(bench, tmp_path):
    csrc = tmp_path / "paper_1003_3684_amd" / "csrc"
    _write(csrc / "kron.hip", "kernel")
    _write(csrc / "common.hpp", "shared")
    h = hashlib.sha256(b"kernelshared").hexdigest()[:16]
    prof = tmp_path / "profiles" / "kron_sample_kron_scale_valu.txt"
    assert bench._valu_per_edge_from_profile() is None
    _write(prof, f"kernel_source_sha256_16: {h}\nvalu_instructions_per_edge: 280.6\n")
    assert bench._valu_per_edge_from_profile() == 280.6
    _write(csrc / "kron.hip", "kernel, edited")
    assert bench._valu_per_edge_from_profile() is None


def test_pba_traffic_reader_checks_the_pba_hash(bench, tmp_path):
    csrc = tmp_path / "paper_1003_3684_amd" / "csrc"
    _write(csrc / "pba.hip", "pba")
    _write(csrc / "common.hpp", "shared")
    h = hashlib.sha256(b"pbashared").hexdigest()[:16]
    prof = tmp_path / "profiles" / "pba_kernels_n2e27_n2e30.txt"
    assert bench._pba_profile_values() == {}
    _write(prof, f"# note: x\n## PBA generation, 2^27 vertices: 7 generations\npba_source_sha256_16: {h}\n"
                 "hbm_bytes_per_generation_n2e27: 2.5e+10\nhbm_bytes_per_generation_n2e30: n/a\n")
    assert bench._pba_profile_values() == {"hbm_bytes_per_generation_n2e27": 2.5e10}  # malformed value dropped
    _write(csrc / "pba.hip", "pba, edited")
    assert bench._pba_profile_values() == {}
    roof = bench._pba_roofline(1000, 1.0, None)
    assert roof["achieved"] == 1000 * bench.PBA_BYTES_PER_EDGE / 1e-3 / 1e9 and roof["traffic"] is None
    assert roof["frac"] == roof["achieved"] / roof["peak"]


def test_host_info(bench):
    info = bench._host_info()
    assert set(info) == {"cpu", "usable_cores", "ram_gib"}
    assert info["usable_cores"] >= 1
    assert info["ram_gib"] is None or info["ram_gib"] > 0


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
