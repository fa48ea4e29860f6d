"""Host-only checks of the Python binding's argument validation and of the
byte / FLOP formulas the benchmark reports. No GPU: the validation helpers run
on CPU tensors with the device requirement switched off, so every rejection
below is the one a GPU caller would get before any pointer reaches a kernel."""
import pytest
import torch

from paper_1511_03599_amd import metrics, pfb


B, S, T, C = 2, 5, 4, 8
ROWS = S + T - 1


def ok_x(dtype):
    if dtype == "c64":
        return torch.zeros((B, ROWS, C), dtype=torch.complex64)
    return torch.zeros((B, ROWS, C, 2), dtype=pfb.STORAGE_DTYPES[dtype])


@pytest.mark.parametrize("dtype", ["c64", "ci16", "ci8", "cf16"])
def test_samples_accepted_in_the_plan_layout(dtype):
    pfb.check_samples(ok_x(dtype), B, ROWS, C, dtype, cuda=False)


def test_c64_samples_may_carry_a_float_pair_axis():
    pfb.check_samples(torch.zeros((B, ROWS, C, 2), dtype=torch.float32), B, ROWS, C, "c64", cuda=False)


@pytest.mark.parametrize("dtype", ["ci16", "ci8", "cf16"])
def test_low_precision_samples_without_pair_axis_rejected(dtype):
    """A missing trailing re/im axis would make the kernel read twice the
    buffer's size."""
    x = torch.zeros((B, ROWS, C), dtype=pfb.STORAGE_DTYPES[dtype])
    with pytest.raises(pfb.PFBError):
        pfb.check_samples(x, B, ROWS, C, dtype, cuda=False)


@pytest.mark.parametrize("bad", [
    torch.zeros((B, ROWS, C, 1), dtype=torch.int16),          # wrong pair axis
    torch.zeros((B, ROWS + 1, C, 2), dtype=torch.int16),      # wrong row count
    torch.zeros((B, ROWS, C, 2, 1), dtype=torch.int16),       # extra axis
    torch.zeros((B, ROWS, C, 2), dtype=torch.int8),           # wrong storage type
    torch.zeros((B, ROWS, 2, C), dtype=torch.int16).transpose(2, 3),  # not contiguous
])
def test_malformed_samples_rejected(bad):
    with pytest.raises(pfb.PFBError):
        pfb.check_samples(bad, B, ROWS, C, "ci16", cuda=False)


def test_c64_samples_of_wrong_shape_rejected():
    for bad in (torch.zeros((B, ROWS, C + 1), dtype=torch.complex64),
                torch.zeros((ROWS, C), dtype=torch.complex64),
                torch.zeros((B, ROWS, C), dtype=torch.complex128),
                torch.zeros((B, ROWS, C, 3), dtype=torch.float32)):
        with pytest.raises(pfb.PFBError):
            pfb.check_samples(bad, B, ROWS, C, "c64", cuda=False)


def test_conjugate_views_rejected():
    """data_ptr() of a conj view points at the unconjugated values."""
    x = ok_x("c64").conj()
    assert x.is_conj()
    with pytest.raises(pfb.PFBError, match="conjugate"):
        pfb.check_samples(x, B, ROWS, C, "c64", cuda=False)
    Y = torch.zeros((B, S, C), dtype=torch.complex64).conj()
    with pytest.raises(pfb.PFBError, match="conjugate"):
        pfb.check_array(Y, "Y", (B, S, C), torch.complex64, cuda=False)
    # resolving the bit makes a plain tensor that passes
    pfb.check_array(Y.resolve_conj(), "Y", (B, S, C), torch.complex64, cuda=False)


def test_cpu_tensor_rejected_when_a_device_is_required():
    with pytest.raises(pfb.PFBError, match="CUDA"):
        pfb.check_samples(ok_x("c64"), B, ROWS, C, "c64")
    with pytest.raises(pfb.PFBError, match="CUDA"):
        pfb.check_array(torch.zeros((T, C)), "taps", (T, C), torch.float32)


@pytest.mark.parametrize("shape,dtype", [
    ((B, S, C + 1), torch.complex64),      # too small or too large an output
    ((B, S - 1, C), torch.complex64),
    ((B * S * C,), torch.complex64),       # right size, wrong shape
    ((B, S, C), torch.float32),
    ((B, S, C, 2), torch.float32),
])
def test_outputs_of_wrong_shape_or_type_rejected(shape, dtype):
    with pytest.raises(pfb.PFBError):
        pfb.check_array(torch.zeros(shape, dtype=dtype), "Y", (B, S, C), torch.complex64, cuda=False)


def test_outputs_on_another_device_rejected():
    t = torch.zeros((T, C), dtype=torch.float32)
    with pytest.raises(pfb.PFBError, match="on"):
        pfb.check_array(t, "gh", (T, C), torch.float32, cuda=False, device=torch.device("meta"))


def test_non_tensor_rejected():
    with pytest.raises(pfb.PFBError):
        pfb.check_array([1.0], "taps", (1,), torch.float32, cuda=False)


def test_tap_limits_match_the_header():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "pfb.h")).read()
    assert int(re.search(r"#define PFB_MAX_TAPS (\d+)", hdr).group(1)) == pfb.MAX_TAPS
    assert int(re.search(r"#define PFB_MAX_TAPS_WINDOW (\d+)", hdr).group(1)) == pfb.MAX_TAPS_WINDOW


# --- metric arithmetic (values of the workload table, worked by hand) ----------

def test_fir_bytes_of_the_tap_sweep():
    """C=1024, S=65536, T=16, complex64: (65551 + 65536) * 1024 * 8 bytes of
    samples plus 16 * 1024 * 4 bytes of taps, about 1.074 GB."""
    b = metrics.fir_bytes(1, 65536, 1024, 16)
    assert b == (65551 + 65536) * 1024 * 8 + 16 * 1024 * 4
    assert abs(b / 1e9 - 1.074) < 1e-3


@pytest.mark.parametrize("dtype,gb", [("ci8", 1.343), ("ci16", 1.611), ("cf16", 1.611), ("c64", 2.148)])
def test_fir_bytes_of_the_precision_workload(dtype, gb):
    """C=4096, T=16, S=32768: input at the storage size, output complex64."""
    b = metrics.fir_bytes(1, 32768, 4096, 16, dtype)
    assert b == 32783 * 4096 * metrics.BYTES_PER_SAMPLE[dtype] + 16 * 4096 * 4 + 32768 * 4096 * 8
    assert abs(b / 1e9 - gb) < 1e-3


def test_differentiable_workload_bytes():
    """B=32, S=8192, C=1024, T=16: forward about 4.30 GB, adjoint (gY in, x
    in, gx out, taps in, tap gradient out) about 6.45 GB."""
    fwd = metrics.pfb_fused_bytes(32, 8192, 1024, 16)
    bwd = metrics.backward_fused_bytes(32, 8192, 1024, 16)
    assert fwd == 32 * 8207 * 1024 * 8 + 16 * 1024 * 4 + 32 * 8192 * 1024 * 8
    assert bwd == 32 * 8192 * 1024 * 8 + 2 * 32 * 8207 * 1024 * 8 + 2 * 16 * 1024 * 4
    assert abs(fwd / 1e9 - 4.30) < 5e-3
    assert abs(bwd / 1e9 - 6.45) < 5e-3


def test_split_bytes_add_the_stand_alone_transform():
    assert metrics.pfb_split_bytes(1, 100, 64, 8) == metrics.fir_bytes(1, 100, 64, 8) + 2 * 100 * 64 * 8
    assert metrics.fft_bytes(3, 10, 32) == 2 * 3 * 10 * 32 * 8


def test_flop_counts():
    """Eq. (3): 2 S C (2T - 1); the tap sweep at T=64 is about 17.05 GFLOP,
    the precision workload about 8.32 GFLOP; the transform count 5 C log2 C
    per spectrum gives 3.36 GFLOP for the tap sweep."""
    assert metrics.effective_flops(1, 100, 10) == 3800.0
    assert abs(metrics.effective_flops(65536, 1024, 64) / 1e9 - 17.05) < 0.01
    assert abs(metrics.effective_flops(32768, 4096, 16) / 1e9 - 8.32) < 0.01
    assert abs(metrics.fft_flops(1024, 65536) / 1e9 - 3.36) < 0.01
