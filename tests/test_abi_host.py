"""Host-only checks of the C ABI: the library loads, exports every function
that include/pfb.h declares, and rejects invalid descriptors on the host
before touching a device. No compute calls (they need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pfb_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1511_03599_amd import pfb
    if not os.path.exists(pfb.LIB_PATH):
        pytest.skip("libpfb.so not built")
    return pfb.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("pfb_plan_create", "pfb_execute", "pfb_backward", "pfb_plan_create_batched",
                 "pfb_execute_batched", "pfb_tune", "pfb_tune_batched", "pfb_plan_destroy", "pfb_status_str",
                 "pfb_execute_stream", "pfb_stream_reset", "pfb_plan_create_vegas", "pfb_execute_vegas",
                 "pfb_last_error", "pfb_plan_get_info"):
        assert want in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1511_03599_amd import pfb
    assert sorted(pfb.EXPORTED) == declared_functions()


def _create(L, **kw):
    from paper_1511_03599_amd import pfb
    d = pfb.make_desc(**{"channels": 64, "taps": 4, "spectra": 16, **kw})
    h = ctypes.c_void_p(1234)
    st = L.pfb_plan_create(ctypes.byref(d), ctypes.byref(h))
    return st, h.value


@pytest.mark.parametrize("kw,code", [
    ({"channels": 0}, 1), ({"taps": 0}, 1), ({"spectra": 0}, 1), ({"batch": 0}, 1),
    ({"taps": 1025}, 2), ({"channels": 44}, 2), ({"channels": 16}, 2), ({"channels": 16384}, 2),
    ({"channels": 8190}, 2), ({"channels": 13 * 64}, 2),
    ({"dtype": "c64", "flags": 1 << 10}, 1),
    ({"dtype": "c64", "flags": 32}, 2), ({"dtype": "ci8", "taps": 17, "flags": 32}, 2),
    ({"channels": 1 << 30, "spectra": 1 << 40, "flags": 1}, 1),
])
def test_invalid_descriptors_rejected_on_host(L, kw, code):
    st, h = _create(L, **kw)
    assert st == code
    assert h is None
    assert L.pfb_last_error().decode()


def test_unknown_dtype_rejected(L):
    from paper_1511_03599_amd import pfb
    d = pfb.Desc(64, 4, 16, 1, 7, 0)
    h = ctypes.c_void_p()
    assert L.pfb_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1


def test_null_arguments(L):
    assert L.pfb_plan_create(None, None) == 1
    assert L.pfb_execute(None, None, None, None, None, None) == 1
    assert L.pfb_backward(None, None, None, None, None, None, None) == 1
    assert L.pfb_execute_stream(None, None, None, None, None, None) == 1
    assert L.pfb_stream_reset(None, None) == 1
    assert L.pfb_execute_vegas(None, None, None, None, None) == 1
    h = ctypes.c_void_p()
    assert L.pfb_plan_create_vegas(48, 2, 4, 10, 0, ctypes.byref(h)) == 2    # C_V not a power of two
    assert L.pfb_plan_create_vegas(64, 0, 4, 10, 0, ctypes.byref(h)) == 1    # no sub-band
    assert L.pfb_plan_create_vegas(64, 2, 0, 10, 0, ctypes.byref(h)) == 1    # no tap
    assert L.pfb_plan_destroy(None) == 0
    assert L.pfb_status_str(0) == b"PFB_OK"
    assert b"INVALID" in L.pfb_status_str(1)
