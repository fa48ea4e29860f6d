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
