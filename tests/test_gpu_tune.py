"""The library's tuner times candidate tile shapes on the device and records
the fastest in a cache file that later plans read (PFB_TUNE_CACHE)."""
import os

import numpy as np
import pytest

import oracle
from paper_1511_03599_amd import synth
from helpers import SPEC_TOL, FIR_TOL, c128, rel_l2, taps_to_device, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("C,T,S,flags", [(1024, 16, 2048, 0), (512, 8, 1000, 1), (4096, 4, 300, 0)])
def test_tune_writes_cache_and_plans_use_it(dev, tmp_path, monkeypatch, C, T, S, flags):
    from paper_1511_03599_amd import pfb
    cache = str(tmp_path / "tune.txt")
    p0 = pfb.Plan(C, T, S, 1, "c64", flags)
    p0.tune(cache)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1
    fields = lines[0].split()
    assert fields[0].startswith("gfx")
    assert [int(v) for v in fields[1:6]] == [0, C, T, 1, S]
    kv = dict(f.split("=") for f in fields[6:])
    monkeypatch.setenv("PFB_TUNE_CACHE", cache)
    p1 = pfb.Plan(C, T, S, 1, "c64", flags)
    info = p1.info()
    if int(kv["path"]) == 0:
        assert info["path"] == "fused"
    elif flags & pfb.FIR_ONLY:
        assert info["fir_cpt"] == int(kv["fir_cpt"]) and info["fir_rows"] == int(kv["fir_sb"])
    else:
        assert info["path"] == "split" and info["fir_cpt"] == int(kv["fir_cpt"])
    # the tuned plan computes the same thing
    st = synth.noise_stream(1, C, T, S, 900 + C)
    out = p1.execute(to_device(st.x, dev), taps_to_device(st.h, dev))
    if flags & pfb.FIR_ONLY:
        assert rel_l2(c128(out), oracle.fir(st.x, st.h)) <= FIR_TOL
    else:
        rows = [0, S // 2, S - 1]
        for s in rows:
            Yr = oracle.pfb_forward(st.x[:, s:s + T], st.h)
            assert rel_l2(c128(out[0, s]), Yr[0, 0]) <= SPEC_TOL


def test_damaged_cache_falls_back_to_defaults(dev, tmp_path, monkeypatch):
    from paper_1511_03599_amd import pfb
    cache = tmp_path / "bad.txt"
    cache.write_text("garbage line\ngfx950 0 1024 16\n\x00\x01 nonsense path=zz\n")
    monkeypatch.setenv("PFB_TUNE_CACHE", str(cache))
    a = pfb.Plan(1024, 16, 512, 1, "c64").info()
    monkeypatch.setenv("PFB_TUNE_CACHE", str(tmp_path / "missing.txt"))
    b = pfb.Plan(1024, 16, 512, 1, "c64").info()
    monkeypatch.delenv("PFB_TUNE_CACHE")
    c = pfb.Plan(1024, 16, 512, 1, "c64").info()
    assert a == b == c


def test_cache_entry_carries_over_to_other_lengths(dev, tmp_path, monkeypatch):
    """An entry for one (B, S) serves other batch sizes and lengths of the
    same dtype, C and T with its shape-independent choices (here the split
    path) and the built-in tile sizes; other C or T are untouched; an exact
    entry wins over a nearer one."""
    import torch
    from paper_1511_03599_amd import pfb
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{arch} 0 1024 16 1 1000 path=1 fir_cpt=1 fir_sb=64 bwd_sb=64\n"
                     f"{arch} 0 1024 16 2 3000 path=0 fused_sb=32\n")
    monkeypatch.setenv("PFB_TUNE_CACHE", str(cache))
    near = pfb.Plan(1024, 16, 900, 1, "c64").info()     # nearest: the (1, 1000) line
    assert near["path"] == "split" and near["fir_cpt"] == 1
    assert near["fir_rows"] == 32                        # the built-in FIR tile height, not 64
    assert pfb.Plan(1024, 16, 2900, 2, "c64").info()["path"] == "fused"   # nearest: (2, 3000)
    assert pfb.Plan(1024, 16, 3000, 2, "c64").info()["fir_rows"] == 32     # exact entry
    assert pfb.Plan(1024, 8, 900, 1, "c64").info()["path"] == "fused"     # other T: defaults
    st = synth.noise_stream(1, 1024, 16, 900, 950)
    out = pfb.Plan(1024, 16, 900, 1, "c64").execute(to_device(st.x, dev), taps_to_device(st.h, dev))
    for s in (0, 450, 899):
        Yr = oracle.pfb_forward(st.x[:, s:s + 16], st.h)
        assert rel_l2(c128(out[0, s]), Yr[0, 0]) <= SPEC_TOL
