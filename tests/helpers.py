"""Shared helpers for the GPU parity tests (test infrastructure)."""
import sys

import numpy as np

FIR_TOL = 2e-6     # relative L2 of the filtered spectra vs the FP64 oracle
SPEC_TOL = 1e-5    # relative L2 of the frequency spectra
GX_TOL = 1e-5      # relative L2 of the sample gradient
GH_TOL = 1e-4      # relative L2 of the tap gradient (long FP32 reductions)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(stored: np.ndarray, dev):
    """Stored stream (numpy, trailing re/im axis) -> torch tensor in the
    library's layout: complex64 for c64, (..., 2) int16/int8/float16 else."""
    import torch
    if stored.dtype == np.float32:
        t = torch.from_numpy(np.ascontiguousarray(stored)).to(dev)
        return torch.view_as_complex(t).contiguous()
    return torch.from_numpy(np.ascontiguousarray(stored)).to(dev)


def taps_to_device(h, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(h, dtype=np.float32)).to(dev)


def c128(t) -> np.ndarray:
    if isinstance(t, np.ndarray):
        return t.astype(np.complex128)
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    ref = np.asarray(ref)
    d = np.linalg.norm((got - ref).ravel())
    n = np.linalg.norm(ref.ravel())
    return float(d / n) if n > 0 else float(d)


def rel_l2_per_stream(got, ref):
    return [rel_l2(got[b], ref[b]) for b in range(ref.shape[0])]
