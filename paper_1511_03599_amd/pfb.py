"""Python binding of libpfb.so (the C ABI in include/pfb.h).

Argument marshalling only: tensors are passed to the library as device
pointers together with torch's current HIP stream, and every step of the
computation runs in the library's kernels. There is no fallback: if the
library is missing or a call fails, a PFBError is raised.

Tensor conventions (all on the GPU, contiguous):
  x   [B, S+T-1, C] complex64, or [B, S+T-1, C, 2] int16 / int8 / float16
  h   [T, C] float32
  Y   [B, S, C] complex64 (frequency spectra), y likewise (filtered spectra)
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfb.so")

# pfb_status
PFB_OK, PFB_E_INVALID, PFB_E_UNSUPPORTED, PFB_E_NOMEM, PFB_E_HIP, PFB_E_STATE = range(6)
# pfb_dtype
DTYPE_CODES = {"c64": 0, "ci16": 1, "ci8": 2, "cf16": 3}
# flags
FIR_ONLY, NO_FUSE, PLAIN, STREAMING, CONVERT_PER_USE = 1, 4, 8, 16, 32
PATH_NAMES = {0: "fused", 1: "split", 2: "fir_only"}
MAX_TAPS = 1024          # PFB_MAX_TAPS: forward and FIR-only plans
MAX_TAPS_WINDOW = 64     # PFB_MAX_TAPS_WINDOW: backward and batched plans
STORAGE_DTYPES = {"ci16": torch.int16, "ci8": torch.int8, "cf16": torch.float16}


class PFBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("taps", ctypes.c_int32), ("spectra", ctypes.c_int64),
                ("batch", ctypes.c_int32), ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("fir_rows", ctypes.c_int32), ("fir_cpt", ctypes.c_int32),
                ("padded_taps", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("chunk_rows", ctypes.c_int64), ("backward_fused", ctypes.c_int32),
                ("fused_ws", ctypes.c_int32), ("backward_rows", ctypes.c_int32)]


EXPORTED = ("pfb_plan_create", "pfb_execute", "pfb_execute_stream", "pfb_stream_reset", "pfb_backward",
            "pfb_backward_noalloc", "pfb_plan_create_batched", "pfb_execute_batched", "pfb_plan_create_vegas", "pfb_execute_vegas",
            "pfb_tune", "pfb_tune_batched", "pfb_plan_get_info", "pfb_plan_destroy", "pfb_status_str",
            "pfb_last_error")

_lib = None


def lib():
    """Load libpfb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PFBError(PFB_E_STATE, f"{LIB_PATH} is missing: build it with "
                                    "`python -m paper_1511_03599_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    L.pfb_plan_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    L.pfb_execute.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pfb_execute_stream.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pfb_stream_reset.argtypes = [vp, vp]
    L.pfb_plan_create_vegas.argtypes = [i32, i32, i32, ctypes.c_int64, i32, ctypes.POINTER(vp)]
    L.pfb_execute_vegas.argtypes = [vp, vp, vp, vp, vp]
    L.pfb_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pfb_backward_noalloc.argtypes = [ctypes.POINTER(Desc), vp, vp, vp, vp, vp, vp]
    L.pfb_plan_create_batched.argtypes = [i32, ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    L.pfb_execute_batched.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.pfb_tune.argtypes = [ctypes.POINTER(Desc), ctypes.c_char_p]
    L.pfb_tune_batched.argtypes = [i32, ctypes.POINTER(Desc), ctypes.c_char_p]
    L.pfb_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.pfb_plan_destroy.argtypes = [vp]
    L.pfb_status_str.argtypes = [st]
    L.pfb_status_str.restype = ctypes.c_char_p
    L.pfb_last_error.argtypes = []
    L.pfb_last_error.restype = ctypes.c_char_p
    for f in ("pfb_plan_create", "pfb_execute", "pfb_execute_stream", "pfb_stream_reset", "pfb_backward",
              "pfb_backward_noalloc", "pfb_plan_create_batched", "pfb_execute_batched", "pfb_plan_create_vegas", "pfb_execute_vegas",
              "pfb_tune", "pfb_tune_batched", "pfb_plan_get_info", "pfb_plan_destroy"):
        getattr(L, f).restype = st
    _lib = L
    return L


def check(status: int):
    if status != PFB_OK:
        msg = lib().pfb_last_error().decode(errors="replace")
        raise PFBError(status, msg or lib().pfb_status_str(status).decode())


def make_desc(channels, taps, spectra, batch=1, dtype="c64", flags=0) -> Desc:
    return Desc(int(channels), int(taps), int(spectra), int(batch), DTYPE_CODES[dtype], int(flags))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def dtype_of(x: torch.Tensor) -> str:
    if x.dtype == torch.complex64:
        return "c64"
    if x.dtype == torch.float32 and x.shape[-1] == 2:
        return "c64"
    return {torch.int16: "ci16", torch.int8: "ci8", torch.float16: "cf16"}[x.dtype]


def _plain_tensor(t, name: str, cuda: bool):
    """Common checks of a tensor handed to the library as a raw pointer."""
    if not isinstance(t, torch.Tensor):
        raise PFBError(PFB_E_INVALID, f"{name} must be a torch.Tensor")
    if cuda and not t.is_cuda:
        raise PFBError(PFB_E_INVALID, f"{name} must be a CUDA (HIP) tensor")
    if t.is_conj() or t.is_neg():
        # data_ptr() ignores the lazy conjugate / negative bits, so the
        # kernels would read or fill the unconjugated values
        raise PFBError(PFB_E_INVALID, f"{name} has its conjugate or negative bit set; "
                                      "call resolve_conj() / resolve_neg() first")
    if not t.is_contiguous():
        raise PFBError(PFB_E_INVALID, f"{name} must be contiguous")


def check_samples(x, B: int, rows: int, C: int, dtype: str, name: str = "x", cuda: bool = True,
                  lead: tuple | None = None):
    """A sample array of the plan's element type: complex64 [*lead] (or
    float32 [*lead, 2]) for c64, [*lead, 2] of int16 / int8 / float16
    otherwise; lead defaults to (B, rows, C). Raises PFBError otherwise."""
    _plain_tensor(x, name, cuda)
    lead = (B, rows, C) if lead is None else tuple(lead)
    if dtype == "c64":
        ok = (x.dtype == torch.complex64 and tuple(x.shape) == lead) or \
             (x.dtype == torch.float32 and tuple(x.shape) == lead + (2,))
        want = f"complex64 {list(lead)}"
    else:
        ok = x.dtype == STORAGE_DTYPES[dtype] and tuple(x.shape) == lead + (2,)
        want = f"{STORAGE_DTYPES[dtype]} {list(lead + (2,))}"
    if not ok:
        raise PFBError(PFB_E_INVALID, f"{name} must be {want} for a {dtype} plan, "
                                      f"got {x.dtype} {list(x.shape)}")


def check_array(t, name: str, shape: tuple, dtype, cuda: bool = True, device=None):
    """A dense array of exactly `shape` and `dtype` (on `device` if given)."""
    _plain_tensor(t, name, cuda)
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise PFBError(PFB_E_INVALID, f"{name} must be {dtype} {list(shape)}, got {t.dtype} {list(t.shape)}")
    if device is not None and t.device != device:
        raise PFBError(PFB_E_INVALID, f"{name} is on {t.device}, the other arguments on {device}")


class Plan:
    """One filter-bank problem: B streams of S filtered spectra, C channels,
    T taps, input element type `dtype`."""

    def __init__(self, channels, taps, spectra, batch=1, dtype="c64", flags=0):
        self.C, self.T, self.S, self.B = int(channels), int(taps), int(spectra), int(batch)
        self.dtype, self.flags = dtype, int(flags)
        d = make_desc(channels, taps, spectra, batch, dtype, flags)
        h = ctypes.c_void_p()
        check(lib().pfb_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    @property
    def rows(self):
        return self.S + self.T - 1

    def info(self) -> dict:
        i = PlanInfo()
        check(lib().pfb_plan_get_info(self._h, ctypes.byref(i)))
        return {"path": PATH_NAMES.get(i.path, i.path), "fir_rows": i.fir_rows, "fir_cpt": i.fir_cpt,
                "padded_taps": i.padded_taps, "workspace_bytes": i.workspace_bytes,
                "chunk_rows": i.chunk_rows, "backward_fused": bool(i.backward_fused),
                "backward_kind": ("split", "fused", "fused_ws")[i.backward_fused],
                "fused_ws": bool(i.fused_ws), "backward_rows": i.backward_rows}

    def _check_x(self, x):
        check_samples(x, self.B, self.rows, self.C, self.dtype)

    def _check_h(self, h, device=None):
        check_array(h, "taps", (self.T, self.C), torch.float32, device=device)

    def _check_out(self, t, name, device):
        check_array(t, name, (self.B, self.S, self.C), torch.complex64, device=device)

    def execute(self, x, h, Y=None, y=None, stream=None):
        """Forward pass. Returns Y (or y for a FIR-only plan)."""
        self._check_x(x)
        self._check_h(h, x.device)
        out_shape = (self.B, self.S, self.C)
        if y is not None:
            self._check_out(y, "y", x.device)
        if self.flags & FIR_ONLY:
            if y is None:
                y = torch.empty(out_shape, dtype=torch.complex64, device=x.device)
            check(lib().pfb_execute(self._h, _ptr(x), _ptr(h), _ptr(y), None, _stream(stream)))
            return y
        if Y is None:
            Y = torch.empty(out_shape, dtype=torch.complex64, device=x.device)
        else:
            self._check_out(Y, "Y", x.device)
        check(lib().pfb_execute(self._h, _ptr(x), _ptr(h), _ptr(y), _ptr(Y), _stream(stream)))
        return Y

    def stream_buffer(self, device=None) -> torch.Tensor:
        """An input buffer for execute_stream: [B, S+T-1, C] of the plan's
        dtype; write each call's new raw spectra into buf[:, T-1:]."""
        shape = (self.B, self.rows, self.C)
        if self.dtype == "c64":
            return torch.zeros(shape, dtype=torch.complex64, device=device)
        tdt = {"ci16": torch.int16, "ci8": torch.int8, "cf16": torch.float16}[self.dtype]
        return torch.zeros(shape + (2,), dtype=tdt, device=device)

    def execute_stream(self, xbuf, h, Y=None, y=None, stream=None):
        """Streaming forward pass (plan created with STREAMING): xbuf holds the
        call's S new raw spectra in rows T-1.. of each stream; rows 0..T-2 are
        overwritten with the spectra carried from the previous call."""
        if not self.flags & STREAMING:
            raise PFBError(PFB_E_STATE, "execute_stream needs a plan created with STREAMING")
        self._check_x(xbuf)
        self._check_h(h, xbuf.device)
        out_shape = (self.B, self.S, self.C)
        if y is not None:
            self._check_out(y, "y", xbuf.device)
        if self.flags & FIR_ONLY:
            if y is None:
                y = torch.empty(out_shape, dtype=torch.complex64, device=xbuf.device)
            check(lib().pfb_execute_stream(self._h, _ptr(xbuf), _ptr(h), _ptr(y), None, _stream(stream)))
            return y
        if Y is None:
            Y = torch.empty(out_shape, dtype=torch.complex64, device=xbuf.device)
        else:
            self._check_out(Y, "Y", xbuf.device)
        check(lib().pfb_execute_stream(self._h, _ptr(xbuf), _ptr(h), _ptr(y), _ptr(Y), _stream(stream)))
        return Y

    def reset_stream(self, stream=None):
        """Forget the carried spectra (the next call starts from zeros)."""
        check(lib().pfb_stream_reset(self._h, _stream(stream)))

    def backward(self, x, h, gY, gx=None, gh=None, want_gx=True, want_gh=True, stream=None):
        """Adjoint pass for a real loss with frequency-spectra gradient gY.
        Returns (gx, gh); either is None when not requested."""
        if self.dtype != "c64":
            raise PFBError(PFB_E_UNSUPPORTED, "backward needs a complex64 plan")
        check_array(gY, "gY", (self.B, self.S, self.C), torch.complex64)
        dev = gY.device
        self._check_h(h, dev)
        if want_gh or x is not None:
            self._check_x(x)
            if x.device != dev:
                raise PFBError(PFB_E_INVALID, f"x is on {x.device}, gY on {dev}")
        if want_gx:
            if gx is None:
                gx = torch.empty((self.B, self.rows, self.C), dtype=torch.complex64, device=dev)
            else:
                check_array(gx, "gx", (self.B, self.rows, self.C), torch.complex64, device=dev)
        if want_gh:
            if gh is None:
                gh = torch.empty((self.T, self.C), dtype=torch.float32, device=dev)
            else:
                check_array(gh, "gh", (self.T, self.C), torch.float32, device=dev)
        check(lib().pfb_backward(self._h, _ptr(x), _ptr(h), _ptr(gY), _ptr(gx if want_gx else None),
                                 _ptr(gh if want_gh else None), _stream(stream)))
        return (gx if want_gx else None), (gh if want_gh else None)

    def tune(self, cache_path: str):
        """Run the library's tuner for this plan's descriptor (writes one line
        to `cache_path`; plans created later read it via PFB_TUNE_CACHE)."""
        d = make_desc(self.C, self.T, self.S, self.B, self.dtype, self.flags)
        check(lib().pfb_tune(ctypes.byref(d), cache_path.encode()))

    def close(self):
        if getattr(self, "_h", None):
            lib().pfb_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan:
    """Many independent single-stream beams (complex64), each with its own
    (C, T, S), run by one persistent kernel launch per call."""

    def __init__(self, beams):
        """beams: list of (C, T, S) tuples."""
        self.beams = [(int(C), int(T), int(S)) for (C, T, S) in beams]
        h = ctypes.c_void_p()
        check(lib().pfb_plan_create_batched(len(self.beams), self._descs(self.beams), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def _descs(beams):
        return (Desc * len(beams))(*[make_desc(C, T, S, 1, "c64", 0) for (C, T, S) in beams])

    @staticmethod
    def tune(beams, cache_path: str):
        """Time the tile sizes for this beam table and append the fastest to
        the tuning cache (read by plans created later via PFB_TUNE_CACHE)."""
        beams = [(int(C), int(T), int(S)) for (C, T, S) in beams]
        check(lib().pfb_tune_batched(len(beams), BatchedPlan._descs(beams), cache_path.encode()))

    def execute(self, xs, hs, Ys=None, stream=None):
        n = len(self.beams)
        if len(xs) != n or len(hs) != n:
            raise PFBError(PFB_E_INVALID, "one x and one taps tensor per beam")
        if Ys is None:
            Ys = [torch.empty((S, C), dtype=torch.complex64, device=xs[0].device)
                  for (C, T, S) in self.beams]
        if len(Ys) != n:
            raise PFBError(PFB_E_INVALID, "one Y tensor per beam")
        dev = xs[0].device
        for i, ((C, T, S), x, h, Y) in enumerate(zip(self.beams, xs, hs, Ys)):
            lead = (S + T - 1, C) if x.dim() == 2 else (1, S + T - 1, C)
            check_samples(x, 1, S + T - 1, C, "c64", name=f"x[{i}]", lead=lead)
            check_array(h, f"taps[{i}]", (T, C), torch.float32, device=dev)
            if x.device != dev:
                raise PFBError(PFB_E_INVALID, f"x[{i}] is on {x.device}, x[0] on {dev}")
            if Y.dim() == 2:
                check_array(Y, f"Y[{i}]", (S, C), torch.complex64, device=dev)
            else:
                check_array(Y, f"Y[{i}]", (1, S, C), torch.complex64, device=dev)
        P = ctypes.c_void_p * n
        xa = P(*[x.data_ptr() for x in xs])
        ha = P(*[h.data_ptr() for h in hs])
        Ya = P(*[Y.data_ptr() for Y in Ys])
        check(lib().pfb_execute_batched(self._h, xa, ha, Ya, _stream(stream)))
        return Ys

    def close(self):
        if getattr(self, "_h", None):
            lib().pfb_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VegasPlan:
    """Polarisation-interleaved sub-bands: x [S+T-1, nsub, C, 2] (+ trailing
    re/im axis for integer and float16 types) -> Y complex64 [S, nsub, C, 2],
    one C-channel filter bank per sub-band and polarisation with the same
    taps h [T, C]."""

    def __init__(self, channels, subbands, taps, spectra, dtype="c64"):
        self.C, self.NS, self.T, self.S = int(channels), int(subbands), int(taps), int(spectra)
        self.dtype = dtype
        h = ctypes.c_void_p()
        check(lib().pfb_plan_create_vegas(self.C, self.NS, self.T, self.S, DTYPE_CODES[dtype], ctypes.byref(h)))
        self._h = h

    def execute(self, x, h, Y=None, stream=None):
        lead = (self.S + self.T - 1, self.NS, self.C, 2)
        check_samples(x, 1, 0, 0, self.dtype, lead=lead)
        check_array(h, "taps", (self.T, self.C), torch.float32, device=x.device)
        if Y is None:
            Y = torch.empty((self.S, self.NS, self.C, 2), dtype=torch.complex64, device=x.device)
        else:
            check_array(Y, "Y", (self.S, self.NS, self.C, 2), torch.complex64, device=x.device)
        check(lib().pfb_execute_vegas(self._h, _ptr(x), _ptr(h), _ptr(Y), _stream(stream)))
        return Y

    def close(self):
        if getattr(self, "_h", None):
            lib().pfb_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StreamPipeline:
    """Real-time use of a STREAMING plan: chunks of raw spectra arrive in
    (pinned) host memory and their frequency spectra go back to host memory.
    Three streams overlap the host-to-device copy of chunk i+1, the filter
    bank of chunk i and the device-to-host copy of chunk i-1; two device input
    buffers and two output buffers alternate. The filter bank itself is the
    plan's (pfb_execute_stream); this class only orders copies and launches."""

    def __init__(self, plan: Plan, h: torch.Tensor, device=None):
        if not plan.flags & STREAMING or plan.flags & FIR_ONLY:
            raise PFBError(PFB_E_STATE, "StreamPipeline needs a STREAMING (not FIR-only) plan")
        self.plan, self.h = plan, h
        dev = device if device is not None else h.device
        self.bufs = [plan.stream_buffer(dev), plan.stream_buffer(dev)]
        self.outs = [torch.empty((plan.B, plan.S, plan.C), dtype=torch.complex64, device=dev) for _ in range(2)]
        self.s_in, self.s_run, self.s_out = torch.cuda.Stream(dev), torch.cuda.Stream(dev), torch.cuda.Stream(dev)
        self.ev_in = [torch.cuda.Event() for _ in range(2)]
        self.ev_run = [torch.cuda.Event() for _ in range(2)]
        self.ev_out = [torch.cuda.Event() for _ in range(2)]
        self.used = [False, False]

    def run(self, host_chunks, host_outs):
        """host_chunks[i]: [B, S, C] (or [B, S, C, 2]) pinned host tensor of
        chunk i's new raw spectra; host_outs[i]: pinned complex64 [B, S, C]
        receiving its frequency spectra. Returns when all copies are done."""
        T = self.plan.T
        for i, (src, dst) in enumerate(zip(host_chunks, host_outs)):
            k = i % 2
            with torch.cuda.stream(self.s_in):
                if self.used[k]:
                    self.s_in.wait_event(self.ev_run[k])   # buffer k free again
                self.bufs[k][:, T - 1:].copy_(src, non_blocking=True)
                self.ev_in[k].record(self.s_in)
            with torch.cuda.stream(self.s_run):
                self.s_run.wait_event(self.ev_in[k])
                if self.used[k]:
                    self.s_run.wait_event(self.ev_out[k])  # output k copied out
                self.plan.execute_stream(self.bufs[k], self.h, Y=self.outs[k], stream=self.s_run)
                self.ev_run[k].record(self.s_run)
            with torch.cuda.stream(self.s_out):
                self.s_out.wait_event(self.ev_run[k])
                dst.copy_(self.outs[k], non_blocking=True)
                self.ev_out[k].record(self.s_out)
            self.used[k] = True
        self.s_out.synchronize()


def backward_noalloc(x, h, gY, gx=None, gh=None, want_gx=True, want_gh=True, stream=None):
    """pfb_backward_noalloc: the adjoint without a plan and without device
    allocation inside the library (outputs are allocated here unless given).
    x: complex64 [B, S+T-1, C]; h: float32 [T, C]; gY: complex64 [B, S, C].
    Returns (gx, gh); either is None when not requested."""
    check_array(gY, "gY", tuple(gY.shape), torch.complex64)
    if gY.dim() != 3:
        raise PFBError(PFB_E_INVALID, "gY must be complex64 [B, S, C]")
    B, S, C = gY.shape
    T = h.shape[0] if h.dim() == 2 else -1
    dev = gY.device
    check_array(h, "taps", (T, C), torch.float32, device=dev)
    rows = S + T - 1
    if want_gh or x is not None:
        check_samples(x, B, rows, C, "c64")
        if x.device != dev:
            raise PFBError(PFB_E_INVALID, f"x is on {x.device}, gY on {dev}")
    if want_gx:
        if gx is None:
            gx = torch.empty((B, rows, C), dtype=torch.complex64, device=dev)
        else:
            check_array(gx, "gx", (B, rows, C), torch.complex64, device=dev)
    if want_gh:
        if gh is None:
            gh = torch.empty((T, C), dtype=torch.float32, device=dev)
        else:
            check_array(gh, "gh", (T, C), torch.float32, device=dev)
    d = make_desc(C, T, S, B, "c64", 0)
    check(lib().pfb_backward_noalloc(ctypes.byref(d), _ptr(x), _ptr(h), _ptr(gY), _ptr(gx if want_gx else None),
                                     _ptr(gh if want_gh else None), _stream(stream)))
    return (gx if want_gx else None), (gh if want_gh else None)


_plan_cache: dict = {}


def cached_plan(C, T, S, B=1, dtype="c64", flags=0) -> Plan:
    key = (C, T, S, B, dtype, flags, torch.cuda.current_device())
    p = _plan_cache.get(key)
    if p is None:
        p = Plan(C, T, S, B, dtype, flags)
        _plan_cache[key] = p
    return p


class PFBFunction(torch.autograd.Function):
    """Y = PFB(x, h) with the library's hand-written adjoint as backward.
    x: complex64 [B, S+T-1, C]; h: float32 [T, C]; Y: complex64 [B, S, C].
    Gradients follow torch's complex convention (dL/dRe + i dL/dIm)."""

    @staticmethod
    def forward(ctx, x, h):
        B, rows, C = x.shape
        T = h.shape[0]
        plan = cached_plan(C, T, rows - T + 1, B, "c64", 0)
        x = x.resolve_conj().resolve_neg().contiguous()
        h = h.resolve_neg().contiguous()
        Y = plan.execute(x, h)
        ctx.save_for_backward(x, h)
        ctx.plan = plan
        return Y

    @staticmethod
    def backward(ctx, gY):
        x, h = ctx.saved_tensors
        need_x, need_h = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gY = gY.resolve_conj().resolve_neg().contiguous()
        gx, gh = ctx.plan.backward(x, h, gY, want_gx=need_x, want_gh=need_h)
        return gx, gh


def pfb(x, h):
    return PFBFunction.apply(x, h)
