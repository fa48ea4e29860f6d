"""The allocation-free adjoint (pfb_backward_noalloc) against the plan-based
adjoint (pfb_backward) through the C ABI: the same relative L2 tolerances as
the oracle parity tests (1e-5 for the sample gradient, 1e-4 for the tap
gradient), on two calls in a row, the second with a smaller input; and a
problem whose partials exceed the scratch is rejected on the host."""
import numpy as np
import pytest

from paper_1511_03599_amd import synth
from helpers import GH_TOL, GX_TOL, c128, rel_l2, say, taps_to_device, to_device

pytestmark = pytest.mark.gpu


def inputs(C, T, S, B, seed, dev):
    x = synth.quantise(synth.complex_gaussian((B, S + T - 1, C), seed), "c64")
    h = synth.random_taps(C, T, seed + 1)
    gY = synth.quantise(synth.complex_gaussian((B, S, C), seed + 2), "c64")
    return to_device(x, dev), taps_to_device(h, dev), to_device(gY, dev)


def test_noalloc_adjoint_matches_plan_adjoint(dev):
    import torch
    from paper_1511_03599_amd import pfb
    for (C, T, S, B), seed in (((1024, 16, 900, 3), 800), ((512, 8, 130, 1), 810), ((1024, 5, 40, 2), 820)):
        say(f"noalloc adjoint C={C} T={T} S={S} B={B}")
        x, h, gY = inputs(C, T, S, B, seed, dev)
        gx_p, gh_p = pfb.Plan(C, T, S, B, "c64").backward(x, h, gY)
        gx_n, gh_n = pfb.backward_noalloc(x, h, gY)
        torch.cuda.synchronize()
        ex = rel_l2(c128(gx_n), c128(gx_p))
        eh = rel_l2(gh_n.cpu().numpy().astype(np.float64), gh_p.cpu().numpy().astype(np.float64))
        say(f"  gx rel L2 {ex:.2e}, gh rel L2 {eh:.2e}, bit-equal "
            f"{torch.equal(gx_n, gx_p) and torch.equal(gh_n, gh_p)}")
        assert ex <= GX_TOL and eh <= GH_TOL
        # one output at a time
        gx1, none = pfb.backward_noalloc(x, h, gY, want_gh=False)
        assert none is None and rel_l2(c128(gx1), c128(gx_p)) <= GX_TOL
        none, gh1 = pfb.backward_noalloc(x, h, gY, want_gx=False)
        assert none is None
        assert rel_l2(gh1.cpu().numpy().astype(np.float64), gh_p.cpu().numpy().astype(np.float64)) <= GH_TOL


def test_noalloc_rejects_what_does_not_fit(dev):
    import ctypes
    import torch
    from paper_1511_03599_amd import pfb
    L = pfb.lib()
    t = torch.zeros(64, dtype=torch.complex64, device=dev)
    p = ctypes.c_void_p(t.data_ptr())
    # partials of 600 streams x 16 taps x 1024 channels exceed the scratch
    d = pfb.make_desc(1024, 16, 16, 600, "c64", 0)
    assert L.pfb_backward_noalloc(ctypes.byref(d), p, p, p, p, p, None) == pfb.PFB_E_UNSUPPORTED
    assert b"scratch" in L.pfb_last_error()
    # shapes outside the fused adjoint, other types, flags
    for args in ((2048, 16, 16, 1, "c64", 0), (1024, 32, 16, 1, "c64", 0), (1024, 16, 16, 1, "ci16", 0)):
        d = pfb.make_desc(*args)
        assert L.pfb_backward_noalloc(ctypes.byref(d), p, p, p, p, p, None) == pfb.PFB_E_UNSUPPORTED
    d = pfb.make_desc(1024, 16, 16, 1, "c64", pfb.NO_FUSE)
    assert L.pfb_backward_noalloc(ctypes.byref(d), p, p, p, p, p, None) == pfb.PFB_E_INVALID
    torch.cuda.synchronize()
