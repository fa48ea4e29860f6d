"""Batched multi-beam plans: one persistent launch over beams of uneven C, T
and S. Each beam must equal a separate plain single-stream launch bit for bit
(same FIR accumulation order and the same transform), and match the oracle."""
import numpy as np
import pytest

import oracle
from paper_1511_03599_amd import synth
from helpers import SPEC_TOL, c128, rel_l2, say, taps_to_device, to_device

pytestmark = pytest.mark.gpu

BEAMS = [(32, 4, 100), (128, 32, 1500), (8192, 8, 70), (1024, 16, 1031), (4096, 3, 90), (256, 1, 64),
         (2048, 32, 33), (512, 17, 260), (64, 8, 5000), (8192, 32, 40), (512, 64, 300), (8192, 40, 50),
         (256, 12, 20000)]


def make_beams(beams, seed):
    xs, hs = [], []
    for i, (C, T, S) in enumerate(beams):
        st = synth.noise_stream(1, C, T, S, seed + i)
        xs.append(st.x[0])
        hs.append(synth.random_taps(C, T, seed + 100 + i))
    return xs, hs


def test_batched_equals_separate_plain_launches(dev):
    import torch
    from paper_1511_03599_amd import pfb
    xs, hs = make_beams(BEAMS, 1000)
    xd = [to_device(x, dev) for x in xs]
    hd = [taps_to_device(h, dev) for h in hs]
    bp = pfb.BatchedPlan(BEAMS)
    Ys = bp.execute(xd, hd)
    torch.cuda.synchronize()
    for i, (C, T, S) in enumerate(BEAMS):
        say(f"beam {i}: C={C} T={T} S={S}")
        ref = pfb.Plan(C, T, S, 1, "c64", pfb.PLAIN).execute(xd[i][None].contiguous(), hd[i])
        assert np.array_equal(Ys[i].cpu().numpy(), ref[0].cpu().numpy()), i
        rows = sorted(set([0, S - 1, S // 2]))
        for s in rows:
            Yr = oracle.pfb_forward(xs[i][None, s:s + T], hs[i])
            assert rel_l2(c128(Ys[i][s]), Yr[0, 0]) <= SPEC_TOL, (i, s)


def test_batched_replays_and_pointer_changes(dev):
    """The recorded graph replays correctly, and new buffers are picked up."""
    import torch
    from paper_1511_03599_amd import pfb
    beams = BEAMS[:5]
    xs, hs = make_beams(beams, 2000)
    xd = [to_device(x, dev) for x in xs]
    hd = [taps_to_device(h, dev) for h in hs]
    bp = pfb.BatchedPlan(beams)
    first = [Y.cpu().numpy() for Y in bp.execute(xd, hd)]
    Ys = [torch.empty((S, C), dtype=torch.complex64, device=dev) for (C, T, S) in beams]
    for rep in range(3):
        for Y in Ys:
            Y.zero_()
        torch.cuda.synchronize()
        bp.execute(xd, hd, Ys)
        torch.cuda.synchronize()
        for a, Y in zip(first, Ys):
            assert np.array_equal(a, Y.cpu().numpy()), rep
    # new inputs in new buffers
    xs2, hs2 = make_beams(beams, 3000)
    xd2 = [to_device(x, dev) for x in xs2]
    hd2 = [taps_to_device(h, dev) for h in hs2]
    out2 = bp.execute(xd2, hd2)
    torch.cuda.synchronize()
    for i, (C, T, S) in enumerate(beams):
        Yr = oracle.pfb_forward(xs2[i][None, 0:T], hs2[i])
        assert rel_l2(c128(out2[i][0]), Yr[0, 0]) <= SPEC_TOL


def test_batched_rejects_bad_beams(dev):
    from paper_1511_03599_amd import pfb
    with pytest.raises(pfb.PFBError):
        pfb.BatchedPlan([(1000, 4, 10)])
    with pytest.raises(pfb.PFBError):
        pfb.BatchedPlan([(1024, 65, 10)])
    with pytest.raises(pfb.PFBError):
        pfb.BatchedPlan([])


def test_batched_tile_size_from_cache(dev, tmp_path, monkeypatch):
    """A tuned tile size (here the smallest, so beams split into many tiles
    with ragged last tiles) gives the same bits as the default one."""
    import torch
    from paper_1511_03599_amd import pfb
    beams = [(8192, 8, 100), (1024, 16, 1031), (128, 4, 3000), (2048, 32, 77)]
    xs, hs = make_beams(beams, 4000)
    xd = [to_device(x, dev) for x in xs]
    hd = [taps_to_device(h, dev) for h in hs]
    ref = [Y.cpu().numpy() for Y in pfb.BatchedPlan(beams).execute(xd, hd)]
    torch.cuda.synchronize()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    total = sum(C * S for (C, T, S) in beams)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{arch} batched {len(beams)} {total} tile_kib=16\n")
    monkeypatch.setenv("PFB_TUNE_CACHE", str(cache))
    out = pfb.BatchedPlan(beams).execute(xd, hd)
    torch.cuda.synchronize()
    for i in range(len(beams)):
        say(f"beam {i}: {beams[i]}")
        assert np.array_equal(out[i].cpu().numpy(), ref[i]), i


def test_batched_tuner_writes_cache(dev, tmp_path):
    from paper_1511_03599_amd import pfb
    beams = [(1024, 16, 2000), (256, 8, 4000)]
    cache = tmp_path / "tune.txt"
    pfb.BatchedPlan.tune(beams, str(cache))
    lines = [l for l in cache.read_text().splitlines() if " batched " in l]
    assert len(lines) == 1
    f = lines[0].split()
    assert f[1] == "batched" and int(f[2]) == 2 and int(f[3]) == 1024 * 2000 + 256 * 4000
    kib = int(f[4].split("=")[1])
    assert kib in (64, 128, 256, 512, 1024, 2048, 4096)
