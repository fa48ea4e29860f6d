"""Streaming plans: consecutive calls continue the streams, so k calls of S
new raw spectra each equal one call over the concatenated input (with T-1
zero spectra in front: the state before the first call). Checked bit for bit
against the one-shot plan (same kernels, same arithmetic) and against the
FP64 oracle on the concatenated stream."""
import numpy as np
import pytest

import oracle
from paper_1511_03599_amd import synth
from helpers import SPEC_TOL, FIR_TOL, c128, rel_l2_per_stream, say, taps_to_device, to_device

pytestmark = pytest.mark.gpu


def pfbmod():
    from paper_1511_03599_amd import pfb
    return pfb


@pytest.mark.parametrize("C,T,S,B,k,dtype,flags", [
    (1024, 16, 100, 2, 4, "c64", 0),      # fused path
    (256, 8, 333, 1, 3, "c64", 0),
    (4096, 5, 20, 1, 5, "c64", 0),        # split path
    (512, 16, 64, 2, 3, "ci16", 0),
    (256, 12, 50, 1, 4, "ci8", 0),
    (128, 4, 7, 3, 6, "cf16", 0),         # S < T-1: history spans calls
    (1024, 16, 200, 1, 3, "c64", 4),      # NO_FUSE
    (1000, 9, 40, 2, 3, "c64", 1),        # FIR only, any C
    (256, 1, 30, 1, 3, "c64", 0),         # T = 1: nothing carried
])
def test_streaming_equals_one_shot(dev, C, T, S, B, k, dtype, flags):
    import torch
    pfb = pfbmod()
    say(f"streaming C={C} T={T} S={S} B={B} calls={k} {dtype} flags={flags}")
    st = synth.noise_stream(B, C, 1, k * S, 1300 + C + T, dtype=dtype)  # k*S raw spectra
    new = st.x                                                          # [B, k*S, C(,2)]
    h = synth.random_taps(C, T, 1301)
    # one-shot reference input: T-1 zero spectra, then everything
    pad = np.zeros((B, T - 1) + new.shape[2:], dtype=new.dtype)
    full = np.concatenate([pad, new], axis=1)
    one = pfb.Plan(C, T, k * S, B, dtype, flags)
    ref = one.execute(to_device(full, dev), taps_to_device(h, dev)).cpu().numpy()
    plan = pfb.Plan(C, T, S, B, dtype, flags | pfb.STREAMING)
    buf = plan.stream_buffer(dev)
    hd = taps_to_device(h, dev)
    outs = []
    for i in range(k):
        buf[:, T - 1:] = to_device(np.ascontiguousarray(new[:, i * S:(i + 1) * S]), dev)
        outs.append(plan.execute_stream(buf, hd).cpu().numpy())
    got = np.concatenate(outs, axis=1)
    assert np.array_equal(got, ref)
    want = oracle.fir(full, h) if flags & 1 else oracle.pfb_forward(full, h)
    tol = FIR_TOL if flags & 1 else SPEC_TOL
    assert max(rel_l2_per_stream(c128(torch.from_numpy(got)), want)) <= tol


def test_stream_reset_and_state_errors(dev):
    import torch
    pfb = pfbmod()
    C, T, S = 256, 8, 40
    st = synth.noise_stream(1, C, T, S, 1310)
    h = taps_to_device(synth.random_taps(C, T, 1311), dev)
    plan = pfb.Plan(C, T, S, 1, "c64", pfb.STREAMING)
    buf = plan.stream_buffer(dev)
    new = to_device(st.x[:, T - 1:], dev)
    buf[:, T - 1:] = new
    first = plan.execute_stream(buf, h).cpu().numpy()
    buf[:, T - 1:] = new
    second = plan.execute_stream(buf, h).cpu().numpy()
    assert not np.array_equal(first, second)       # history from call 1 is used
    plan.reset_stream()
    buf[:, T - 1:] = new
    again = plan.execute_stream(buf, h).cpu().numpy()
    assert np.array_equal(first, again)            # reset: zeros again
    plain = pfb.Plan(C, T, S, 1, "c64")
    with pytest.raises(pfb.PFBError):
        plain.execute_stream(buf, h)
    with pytest.raises(pfb.PFBError):
        plain.reset_stream()


def test_stream_pipeline_matches_one_shot(dev):
    """Host chunks through the three-stream pipeline (pinned memory,
    overlapped copies) give the bits of one call over the whole stream."""
    import torch
    pfb = pfbmod()
    C, T, S, B, k = 1024, 16, 256, 2, 5
    st = synth.noise_stream(B, C, 1, k * S, 1320, dtype="ci16")
    new = st.x
    h = synth.random_taps(C, T, 1321)
    pad = np.zeros((B, T - 1) + new.shape[2:], dtype=new.dtype)
    full = np.concatenate([pad, new], axis=1)
    ref = pfb.Plan(C, T, k * S, B, "ci16").execute(to_device(full, dev), taps_to_device(h, dev)).cpu().numpy()
    plan = pfb.Plan(C, T, S, B, "ci16", pfb.STREAMING)
    pipe = pfb.StreamPipeline(plan, taps_to_device(h, dev))
    chunks = [torch.from_numpy(np.ascontiguousarray(new[:, i * S:(i + 1) * S])).pin_memory() for i in range(k)]
    outs = [torch.empty((B, S, C), dtype=torch.complex64).pin_memory() for _ in range(k)]
    pipe.run(chunks, outs)
    got = np.concatenate([o.numpy() for o in outs], axis=1)
    assert np.array_equal(got, ref)
