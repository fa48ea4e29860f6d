"""GPU parity of the hand-written adjoint against the FP64 oracle adjoint
(itself pinned to finite differences and the dot-product identity on the
CPU). Tolerances: relative L2 <= 1e-5 for the sample gradient and <= 1e-4
for the tap gradient."""
import numpy as np
import pytest

import oracle
from paper_1511_03599_amd import synth
from helpers import GH_TOL, GX_TOL, c128, rel_l2, say, taps_to_device, to_device

pytestmark = pytest.mark.gpu


def pfbmod():
    from paper_1511_03599_amd import pfb
    return pfb


def adjoint_kind_cache(tmp_path, monkeypatch, C, T, S, B, ws):
    """A tuning-cache entry that selects the wave-specialised (ws=1) or the
    single-role (ws=0) fused adjoint."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / f"tune{ws}.txt"
    cache.write_text(f"{arch} 0 {C} {T} {B} {S} path=-1 bwd_ws={ws}\n")
    monkeypatch.setenv("PFB_TUNE_CACHE", str(cache))


@pytest.mark.parametrize("C,T,S,B", [(32, 4, 20, 2), (256, 8, 100, 2), (1024, 16, 80, 3), (4096, 5, 10, 1),
                                     (64, 64, 100, 1), (1024, 33, 70, 1), (512, 1, 40, 2), (128, 16, 600, 1),
                                     (1024, 16, 700, 2), (256, 3, 530, 1), (512, 13, 257, 2),
                                     (384, 8, 50, 2), (3072, 4, 12, 1), (105, 16, 40, 1),
                                     (1024, 7, 300, 2), (1024, 2, 45, 1), (1024, 16, 1, 1), (1024, 4, 3, 2),
                                     (512, 16, 1000, 1), (512, 5, 17, 3), (2048, 8, 20, 1), (8192, 4, 6, 2)])
@pytest.mark.parametrize("mode", ["default", "split", "single_role", "wave_specialised"])
def test_backward_parity(dev, C, T, S, B, mode, tmp_path, monkeypatch):
    import torch
    pfb = pfbmod()
    say(f"backward C={C} T={T} S={S} B={B} {mode}")
    x = synth.quantise(synth.complex_gaussian((B, S + T - 1, C), 700 + C), "c64")
    h = synth.random_taps(C, T, 701)
    gY = synth.quantise(synth.complex_gaussian((B, S, C), 702), "c64")
    if mode in ("single_role", "wave_specialised"):
        adjoint_kind_cache(tmp_path, monkeypatch, C, T, S, B, int(mode == "wave_specialised"))
    plan = pfb.Plan(C, T, S, B, "c64", pfb.NO_FUSE if mode == "split" else 0)
    kind = plan.info()["backward_kind"]
    if mode == "split" or not (C in (256, 512, 1024) and T <= 16):
        assert kind == "split"
    elif mode == "default":
        assert kind == "fused", kind
    else:
        assert kind == ("fused" if mode == "single_role" else "fused_ws"), kind
    gx, gh = plan.backward(to_device(x, dev), taps_to_device(h, dev), to_device(gY, dev))
    torch.cuda.synchronize()
    gx_r, gh_r = oracle.pfb_adjoint(x, h, gY)
    assert rel_l2(c128(gx), gx_r) <= GX_TOL
    assert rel_l2(gh.cpu().numpy().astype(np.float64), gh_r) <= GH_TOL


@pytest.mark.parametrize("C,T,S", [(256, 8, 50), (512, 16, 70), (1024, 16, 90), (1024, 3, 40)])
def test_backward_only_one_output(dev, C, T, S):
    pfb = pfbmod()
    say(f"backward one output C={C} T={T} S={S}")
    x = synth.quantise(synth.complex_gaussian((1, S + T - 1, C), 710), "c64")
    h = synth.random_taps(C, T, 711)
    gY = synth.quantise(synth.complex_gaussian((1, S, C), 712), "c64")
    plan = pfb.Plan(C, T, S, 1, "c64")
    gx_r, gh_r = oracle.pfb_adjoint(x, h, gY)
    gx, gh = plan.backward(to_device(x, dev), taps_to_device(h, dev), to_device(gY, dev), want_gh=False)
    assert gh is None and rel_l2(c128(gx), gx_r) <= GX_TOL
    gx, gh = plan.backward(to_device(x, dev), taps_to_device(h, dev), to_device(gY, dev), want_gx=False)
    assert gx is None and rel_l2(gh.cpu().numpy().astype(np.float64), gh_r) <= GH_TOL


def test_tap_gradient_reproducible(dev):
    pfb = pfbmod()
    C, T, S, B = 1024, 16, 300, 4
    x = synth.quantise(synth.complex_gaussian((B, S + T - 1, C), 720), "c64")
    h = synth.random_taps(C, T, 721)
    gY = synth.quantise(synth.complex_gaussian((B, S, C), 722), "c64")
    plan = pfb.Plan(C, T, S, B, "c64")
    args = (to_device(x, dev), taps_to_device(h, dev), to_device(gY, dev))
    a = plan.backward(*args)
    b = plan.backward(*args)
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


def test_autograd_function_leakage_loss(dev):
    """Learnable taps against the out-of-channel power of off-centre tones:
    torch autograd through the library's forward and adjoint matches the
    oracle's adjoint of the oracle's loss gradient."""
    import torch
    pfb = pfbmod()
    st = synth.tone_streams(B=4, C=256, T=8, S=64, seed=731)
    x = to_device(st.x, dev)
    h = taps_to_device(st.h, dev).requires_grad_(True)
    xr = x.clone().requires_grad_(True)
    Y = pfb.PFBFunction.apply(xr, h)
    mask = torch.ones(Y.shape, device=dev)
    for b, k in enumerate(st.tone_bins):
        mask[b, :, int(k)] = 0
    loss = (mask * (Y.real ** 2 + Y.imag ** 2)).sum()
    loss.backward()
    Yr = oracle.pfb_forward(st.x, st.h)
    L, gY = oracle.leakage_loss(Yr, st.tone_bins)
    gx_r, gh_r = oracle.pfb_adjoint(st.x, st.h, gY)
    assert abs(loss.item() - L) <= 1e-4 * L
    assert rel_l2(h.grad.cpu().numpy().astype(np.float64), gh_r) <= GH_TOL
    assert rel_l2(c128(xr.grad), gx_r) <= GX_TOL


@pytest.mark.parametrize("C,T,S,B", [(1024, 16, 700, 2), (512, 8, 333, 1), (256, 4, 1000, 3), (1024, 5, 64, 1)])
def test_wave_specialised_adjoint_equals_single_role(dev, C, T, S, B, tmp_path, monkeypatch):
    """Both fused adjoint kernels do the same operations in the same order:
    identical bits for gx and for the tap gradient."""
    pfb = pfbmod()
    say(f"ws vs single-role C={C} T={T} S={S} B={B}")
    x = synth.quantise(synth.complex_gaussian((B, S + T - 1, C), 740), "c64")
    h = synth.random_taps(C, T, 741)
    gY = synth.quantise(synth.complex_gaussian((B, S, C), 742), "c64")
    args = (to_device(x, dev), taps_to_device(h, dev), to_device(gY, dev))
    adjoint_kind_cache(tmp_path, monkeypatch, C, T, S, B, 1)
    p1 = pfb.Plan(C, T, S, B, "c64")
    assert p1.info()["backward_kind"] == "fused_ws"
    a = [t.cpu().numpy() for t in p1.backward(*args)]
    adjoint_kind_cache(tmp_path, monkeypatch, C, T, S, B, 0)
    p2 = pfb.Plan(C, T, S, B, "c64")
    assert p2.info()["backward_kind"] == "fused"
    b = [t.cpu().numpy() for t in p2.backward(*args)]
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
