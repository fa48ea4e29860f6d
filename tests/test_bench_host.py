"""Host-side checks of bench.py: the single-GPU contract and the committed
rocprofv3 summaries it reads (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_reader_checks_the_source_digest(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    digest = bench.source_digest()              # of the (empty) source tree under tmp_path
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_x.txt").write_text(f"# title\n| a | b |\nhbm_bytes_per_call: 123\nsource_digest: {digest}\n")
    (prof / "traffic_y.txt").write_text("hbm_bytes_per_call: 456\nsource_digest: 0000000000000000\n")
    assert bench.read_traffic("x") == 123.0
    assert bench.read_traffic("y") is None      # counters taken from other kernel sources
    assert bench.read_traffic("z") is None      # no summary


@pytest.mark.parametrize("name", ["traffic_pfb_backward_b32_s8192_c1024_t16.txt",
                                  "traffic_pfb_execute_b32_s8192_c1024_t16.txt",
                                  "conversions_fir_c4096_t16_s32768.txt",
                                  "traffic_fir_fft_c4096_t16_s32768.txt"])
def test_committed_counter_summaries_match_the_kernel_sources(name):
    """The counter summaries that bench.py reports were taken from the
    kernel sources in this tree (else its `traffic` would read null)."""
    kv = bench.read_profile(name)
    assert kv is not None, f"profiles/{name} is missing or was taken from other kernel sources"
    if name.startswith("traffic_pfb"):
        alg = float(kv["algorithmic_bytes_per_call"])
        hbm = float(kv["hbm_bytes_per_call"])
        assert 0.95 * alg < hbm < 1.5 * alg
