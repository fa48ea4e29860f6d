"""Benchmark of the MI355X polyphase filter bank.

One step = one pass of the whole hot path over one batch of synthetic input
already resident in HBM: the forward filter bank (ingest + convert, FIR, FFT,
write) followed by its adjoint (inverse FFT, sample gradient, tap gradient).
Workload: the differentiable filter bank, 32 streams x 8192 filtered spectra,
C = 1024 channels, T = 16 taps, complex64 off-centre tones, Hamming-windowed
sinc taps, a seeded complex64 frequency-spectra gradient.

Prints ONE JSON line. `value` is the real-time sample rate in Msamples/s
(new input samples B*S*C per second of the fwd+bwd step). The same step on the
plain comparator (unfused FIR launch then FFT launch, split adjoint) is timed
beside it, and the oracle is timed on bounded samples on the host cores.
Unless --quick is given, `extras` adds the other workloads: the forward pass
over T in {4..64} at C=1024 (one stream of 65536 spectra, also timed fwd+bwd),
the split adjoint where no fused kernel applies (C=4096 at T=16, C=1024 at
T=32), the low-precision inputs at C=4096 with their errors against FP64, the
64-beam batched launch against 64 separate plain launches, and the layouts
of the later rows (streaming, non-power-of-two channel counts, sub-bands).

Before timing the 64-beam launch it runs the library's batched tuner
(pfb_tune_batched) and uses its tile size; `--tune all` also tunes the
headline plan, `--tune none` uses built-in choices throughout. `--only`
runs one extra alone (for profiling) and `--copy-calibration` ends with
three plain 512 MiB device copies whose counter readings calibrate the
FETCH_SIZE / WRITE_SIZE summaries under profiles/.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--quick]
                    [--tune none|batched|all] [--only precision|sweep|batched]
                    [--copy-calibration]
"""
from __future__ import annotations

import argparse
import glob
import tempfile
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8000.0  # GB/s, MI355X published
METRIC = "PFB Msamples/s and HBM GB/s (% of 8 TB/s) vs plain FP32 path, fwd+bwd"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1511_03599_amd", "csrc")
    files = [f for ext in ("*.hip", "*.h", "*.cpp") for f in glob.glob(os.path.join(src, ext))]
    for f in sorted(files):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_profile(fname: str):
    """The `key: value` lines of a committed rocprofv3 summary under
    profiles/, or None when there is none or the kernel sources changed
    since its counters were taken."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    return kv


def read_traffic(name: str):
    """HBM bytes per launch from profiles/traffic_<name>.txt (FETCH_SIZE +
    WRITE_SIZE, calibrated), or None."""
    kv = read_profile(f"traffic_{name}.txt")
    try:
        return float(kv["hbm_bytes_per_call"]) if kv else None
    except (KeyError, ValueError):
        return None


def time_calls(fn, n, stream):
    """Average ms per call of fn over n back-to-back calls, HIP events on the
    stream the library launches on."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(n):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / n


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(B, S, C, T, seed):
    """The oracle (plain FP64 C, OpenMP) timed on bounded samples of the
    step's workload, each part on its own: the FIR (Algorithm 1), the DFT
    (Eq. (2), direct O(C^2) per spectrum), the inverse DFT of the gradient,
    and the two FIR adjoints; once on all host threads and once on one.
    Each part's time is scaled linearly from its sample to the whole step
    (B*S spectra) -- the DFT parts are therefore extrapolated -- and `value`
    is B*S*C over the sum, on all threads."""
    import oracle
    from paper_1511_03599_amd import synth
    fir_rows, dft_rows = 16384, 3072  # about 10 s of host work in all
    st = synth.noise_stream(1, C, T, fir_rows, seed, fast=True)
    x = oracle._as_c128(st.x)
    h = st.h.astype("float64")
    g = synth.complex_gaussian((1, fir_rows, C), seed + 1)
    spec = g[:, :dft_rows]
    oracle.fir(x[:, :T + 1], h)  # load the library, warm the threads

    def parts():
        out = {}
        t0 = time.perf_counter()
        oracle.fir(x, h)
        out["fir"] = (time.perf_counter() - t0) / fir_rows
        t0 = time.perf_counter()
        oracle.dft(spec, -1)
        out["dft"] = (time.perf_counter() - t0) / dft_rows
        t0 = time.perf_counter()
        oracle.dft(spec, +1)
        out["inverse_dft"] = (time.perf_counter() - t0) / dft_rows
        t0 = time.perf_counter()
        oracle.fir_adjoint_x(g, h)
        oracle.fir_adjoint_h(g, x, T)
        out["fir_adjoints"] = (time.perf_counter() - t0) / fir_rows
        return out

    def report(per_row):
        step = sum(per_row.values()) * B * S
        res = {"value": round(B * S * C / step / 1e6, 4), "step_s": round(step, 2),
               "fir_msamples_s": round(C / per_row["fir"] / 1e6, 2),
               "fir_gflops": round(2 * C * (2 * T - 1) / per_row["fir"] / 1e9, 2),
               "dft_msamples_s": round(C / per_row["dft"] / 1e6, 3),
               "dft_gflops": round(8.0 * C * C / per_row["dft"] / 1e9, 2)}
        return res

    nthreads = oracle.num_threads()
    all_cores = report(parts())
    oracle.set_num_threads(1)
    try:
        one_core = report(parts())
    finally:
        oracle.set_num_threads(nthreads)
    return {"value": all_cores["value"], "unit": "Msamples/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"FP64 oracle parts timed separately on samples of the {B}x{S}-spectrum, C={C}, "
                      f"T={T} step: FIR and both FIR adjoints on {fir_rows} spectra, DFT and inverse DFT "
                      f"(direct O(C^2)) on {dft_rows} spectra, each scaled linearly to {B * S} spectra "
                      f"(DFT parts extrapolated)",
            "all_cores": all_cores, "one_core": one_core}


def extras_sweep(dev, stream, C, S):
    import torch
    from paper_1511_03599_amd import metrics, pfb, synth
    out = {}
    Y = torch.empty((1, S, C), dtype=torch.complex64, device=dev)
    for T in (4, 8, 16, 32, 64, 128, 192):
        st = synth.noise_stream(1, C, T, S, synth.seed_for(2, T), fast=True)
        x = torch.view_as_complex(torch.from_numpy(st.x)).to(dev).contiguous()
        h = torch.from_numpy(st.h).to(dev)
        p = pfb.Plan(C, T, S, 1, "c64")
        pf = pfb.Plan(C, T, S, 1, "c64", pfb.FIR_ONLY)
        for _ in range(3):
            p.execute(x, h, Y=Y)
            pf.execute(x, h, y=Y)
        tp = time_calls(lambda: p.execute(x, h, Y=Y), 20, stream)
        tf = time_calls(lambda: pf.execute(x, h, y=Y), 20, stream)
        out[str(T)] = {
            "pfb_ms": round(tp, 5), "pfb_msamples_s": round(S * C / tp / 1e3, 1),
            "pfb_gbs": round(metrics.pfb_fused_bytes(1, S, C, T) / tp / 1e6, 1), "path": p.info()["path"],
            "fir_ms": round(tf, 5), "fir_gbs": round(metrics.fir_bytes(1, S, C, T) / tf / 1e6, 1),
            "fir_gflops": round(metrics.effective_flops(S, C, T) / tf / 1e6, 1),
            "fir_frac_valu": round(metrics.effective_flops(S, C, T) / tf / 1e9 / metrics.FP32_VALU_PEAK_TFLOPS, 4)}
        del x, p, pf
    return out


def precision_errors(dev, C, T, S):
    """Error of each input type against FP64 on one seeded stream of S
    spectra (C channels, T taps): `binding` is the GPU spectra against the
    oracle on the same quantised input (the parity bar); `vs_unquantised` is
    the GPU spectra against the oracle on the Gaussian before quantisation
    (informational: it includes the quantisation noise itself)."""
    import numpy as np
    import torch
    import oracle
    from paper_1511_03599_amd import pfb, synth
    out = {}
    h = synth.windowed_sinc_taps(C, T)
    hd = torch.from_numpy(h).to(dev)
    for dt, sigma in (("ci8", 16.0), ("ci16", 2000.0), ("cf16", 1.0), ("c64", 1.0)):
        xc = synth.complex_gaussian((1, S + T - 1, C), synth.seed_for(3, 50), sigma=sigma * np.sqrt(2.0)
                                    if dt in ("ci8", "ci16") else 1.0)
        xq = synth.quantise(xc, dt)
        xd = torch.from_numpy(np.ascontiguousarray(xq)).to(dev)
        if dt == "c64":
            xd = torch.view_as_complex(xd).contiguous()
        Y = pfb.Plan(C, T, S, 1, dt).execute(xd, hd).cpu().numpy().astype(np.complex128)
        Yq = oracle.pfb_forward(xq, h)
        Yc = oracle.pfb_forward(xc, h)
        n = np.linalg.norm
        out[dt] = {"binding_rel_l2": float(f"{n(Y - Yq) / n(Yq):.3e}"),
                   "vs_unquantised_rel_l2": float(f"{n(Y - Yc) / n(Yc):.3e}")}
    return out


def extras_precision(dev, stream):
    """C=4096, T=16, 32768 spectra in each input type (device-generated
    inputs of each type's distribution): the FIR alone and the whole filter
    bank; the FIR alone again with four input buffers used in turn (about
    1.1 GB of int8 input and more for the other types, beyond the 256 MB
    last-level cache, so every call reads its input from HBM); and the
    convert-per-use comparator (each stored sample converted at every tap,
    2T conversions per output) beside this library's convert-at-load FIR (2
    conversions per input sample). Bytes use each type's sample size.
    Errors per type on a 64-spectrum sample."""
    import torch
    from paper_1511_03599_amd import metrics, pfb, synth
    C, T, S = 4096, 16, 32768
    out = {}
    Y = torch.empty((1, S, C), dtype=torch.complex64, device=dev)
    h = torch.from_numpy(synth.windowed_sinc_taps(C, T)).to(dev)
    for dt in ("ci8", "ci16", "cf16", "c64"):
        xs = [synth.device_quantised_noise((1, S + T - 1, C), dt, synth.seed_for(3, 10 + k), dev) for k in range(4)]
        x = xs[0]
        p = pfb.Plan(C, T, S, 1, dt)
        pf = pfb.Plan(C, T, S, 1, dt, pfb.FIR_ONLY)
        for _ in range(3):
            p.execute(x, h, Y=Y)
            pf.execute(x, h, y=Y)
        tp = time_calls(lambda: p.execute(x, h, Y=Y), 10, stream)
        tf = time_calls(lambda: pf.execute(x, h, y=Y), 10, stream)
        k = [0]

        def rotating():
            pf.execute(xs[k[0] % 4], h, y=Y)
            k[0] += 1
        tr = time_calls(rotating, 12, stream)
        fb = metrics.fir_bytes(1, S, C, T, dt)
        r = {"pfb_ms": round(tp, 4), "pfb_msamples_s": round(S * C / tp / 1e3, 1),
             "pfb_gbs": round(metrics.pfb_fused_bytes(1, S, C, T, dt) / tp / 1e6, 1),
             "fir_ms": round(tf, 4), "fir_gbs": round(fb / tf / 1e6, 1),
             "fir_rotating_inputs_ms": round(tr, 4), "fir_rotating_inputs_gbs": round(fb / tr / 1e6, 1),
             "path": p.info()["path"]}
        if dt != "c64":
            pu = pfb.Plan(C, T, S, 1, dt, pfb.FIR_ONLY | pfb.CONVERT_PER_USE)
            for _ in range(2):
                pu.execute(x, h, y=Y)
            tu = time_calls(lambda: pu.execute(x, h, y=Y), 10, stream)
            at_load = 2 * (S + T - 1) * C
            per_use = 2 * T * S * C
            r.update({"fir_convert_per_use_ms": round(tu, 4), "fir_convert_per_use_gbs": round(fb / tu / 1e6, 1),
                      "per_use_slowdown": round(tu / tf, 3),
                      "conversions_at_load": at_load, "conversions_per_use": per_use,
                      "gconversions_s_at_load": round(at_load / tf / 1e6, 1),
                      "gconversions_s_per_use": round(per_use / tu / 1e6, 1)})
            del pu
        out[dt] = r
        del x, xs, p, pf
        torch.cuda.empty_cache()
    err = precision_errors(dev, C, T, 64)
    for dt in err:
        out[dt].update(err[dt])
    # conversion instructions counted by rocprofv3 (SQ_INSTS_VALU_CVT, per
    # wave instruction, x64 lanes) in the committed summary of this workload
    kv = read_profile("conversions_fir_c4096_t16_s32768.txt")
    if kv:
        for dt in ("ci8", "ci16", "cf16"):
            try:
                at = float(kv[f"{dt}.at_load.cvt_per_input_sample"])
                pu = float(kv[f"{dt}.per_use.cvt_per_input_sample"])
            except (KeyError, ValueError):
                continue
            n_in = (S + T - 1) * C
            r = out[dt]
            r["counted_cvt_per_input_sample"] = {"at_load": at, "per_use": pu}
            r["counted_gconversions_s_at_load"] = round(at * n_in / r["fir_ms"] / 1e6, 1)
            r["counted_gconversions_s_per_use"] = round(pu * n_in / r["fir_convert_per_use_ms"] / 1e6, 1)
    return out


def tune_cache() -> str:
    """This run's tuning-cache file (a fresh temporary file per run)."""
    global _TUNE_CACHE
    if _TUNE_CACHE is None:
        _TUNE_CACHE = os.path.join(tempfile.mkdtemp(prefix="pfb_tune_"), "cache.txt")
    return _TUNE_CACHE


_TUNE_CACHE = None


def extras_batched(dev, stream, tune=True):
    """64 beams of uneven C, T, S: one persistent launch vs 64 separate plain
    launches, and vs 64 launches of the default plans, on one stream."""
    import torch
    from paper_1511_03599_amd import metrics, pfb, synth
    beams = synth.beam_table()
    desc = [(b.C, b.T, b.S) for b in beams]
    xs = [synth.device_noise((b.S + b.T - 1, b.C), b.seed, dev) for b in beams]
    hs = [torch.from_numpy(synth.windowed_sinc_taps(b.C, b.T)).to(dev) for b in beams]
    Ys = [torch.empty((b.S, b.C), dtype=torch.complex64, device=dev) for b in beams]
    tuned_tile = None
    if tune:
        # the batched tile size from the tuner (pfb_tune_batched, which
        # times 64 KiB - 4 MiB tiles), read by the plan created below
        pfb.BatchedPlan.tune(desc, tune_cache())
        os.environ["PFB_TUNE_CACHE"] = tune_cache()
        tuned_tile = open(tune_cache()).read().strip().splitlines()[-1]
    bp = pfb.BatchedPlan(desc)
    for _ in range(2):
        bp.execute(xs, hs, Ys)
    tb = time_calls(lambda: bp.execute(xs, hs, Ys), 5, stream)
    del bp
    plains = [pfb.Plan(C, T, S, 1, "c64", pfb.PLAIN) for (C, T, S) in desc]

    def run_plain():
        for p, x, h, Y in zip(plains, xs, hs, Ys):
            p.execute(x[None], h, Y=Y[None])
    run_plain()
    tpl = time_calls(run_plain, 3, stream)
    del plains
    # the same beams as 64 launches of this library's default plans (fused
    # where the beam allows, else the split path with its default tiles)
    defaults = [pfb.Plan(C, T, S, 1, "c64") for (C, T, S) in desc]

    def run_default():
        for p, x, h, Y in zip(defaults, xs, hs, Ys):
            p.execute(x[None], h, Y=Y[None])
    run_default()
    tdf = time_calls(run_default, 3, stream)
    del defaults
    samples = sum(S * C for (C, T, S) in desc)
    fused_bytes = sum(metrics.pfb_fused_bytes(1, S, C, T) for (C, T, S) in desc)
    return {"beams": len(desc), "msamples": round(samples / 1e6, 1), "ms": round(tb, 3),
            "msamples_s": round(samples / tb / 1e3, 1), "gbs": round(fused_bytes / tb / 1e6, 1),
            "frac_hbm": round(fused_bytes / tb / 1e6 / HBM_PEAK, 4),
            "plain_64_launches_ms": round(tpl, 3), "speedup_vs_plain": round(tpl / tb, 3),
            "default_64_launches_ms": round(tdf, 3), "tuned": tuned_tile}


def extras_streaming(dev, stream):
    """Real-time use: 8 consecutive chunks of 16384 new spectra (C=1024,
    T=16, int16 samples) through a STREAMING plan. Compute-only: chunks
    already in HBM. End-to-end: chunks from pinned host memory, frequency
    spectra back to pinned host memory, copies overlapped with the filter
    bank on three streams (StreamPipeline); this rate includes PCIe and is
    never the headline value."""
    import torch
    from paper_1511_03599_amd import pfb, synth
    C, T, S, k = 1024, 16, 16384, 8
    plan = pfb.Plan(C, T, S, 1, "ci16", pfb.STREAMING)
    h = torch.from_numpy(synth.windowed_sinc_taps(C, T)).to(dev)
    g = torch.Generator().manual_seed(1511400)
    chunks = [torch.randint(-2000, 2000, (1, S, C, 2), dtype=torch.int16, generator=g).pin_memory()
              for _ in range(k)]
    outs = [torch.empty((1, S, C), dtype=torch.complex64).pin_memory() for _ in range(k)]
    buf = plan.stream_buffer(dev)
    Y = torch.empty((1, S, C), dtype=torch.complex64, device=dev)
    buf[:, T - 1:].copy_(chunks[0].to(dev))
    for _ in range(3):
        plan.execute_stream(buf, h, Y=Y)
    t_comp = time_calls(lambda: plan.execute_stream(buf, h, Y=Y), 20, stream)
    pipe = pfb.StreamPipeline(plan, h)
    pipe.run(chunks[:2], outs[:2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipe.run(chunks, outs)
    torch.cuda.synchronize()
    t_e2e = (time.perf_counter() - t0) * 1e3 / k
    samples = S * C
    bytes_pcie = samples * (4 + 8)
    return {"chunk_spectra": S, "chunks": k, "compute_ms_per_chunk": round(t_comp, 4),
            "compute_msamples_s": round(samples / t_comp / 1e3, 1),
            "end_to_end_ms_per_chunk": round(t_e2e, 4),
            "end_to_end_msamples_s": round(samples / t_e2e / 1e3, 1),
            "end_to_end_pcie_gbs": round(bytes_pcie / t_e2e / 1e6, 1)}


def extras_mixed_radix(dev, stream):
    """Channel counts that are not powers of two (mixed-radix transform on the
    split path) beside their power-of-two neighbours: T=16, 2^27 samples."""
    import torch
    from paper_1511_03599_amd import metrics, pfb, synth
    out = {}
    for C in (2048, 3072, 4096, 6144):
        T, S = 16, (1 << 27) // C
        x = synth.device_noise((1, S + T - 1, C), 1511500 + C, dev)
        h = torch.from_numpy(synth.windowed_sinc_taps(C, T)).to(dev)
        Y = torch.empty((1, S, C), dtype=torch.complex64, device=dev)
        p = pfb.Plan(C, T, S, 1, "c64")
        for _ in range(2):
            p.execute(x, h, Y=Y)
        t = time_calls(lambda: p.execute(x, h, Y=Y), 10, stream)
        out[str(C)] = {"pfb_ms": round(t, 4), "pfb_msamples_s": round(S * C / t / 1e3, 1),
                       "path": p.info()["path"],
                       "fused_bytes_gbs": round(metrics.pfb_fused_bytes(1, S, C, T) / t / 1e6, 1)}
        del p, x, Y
    return out


def extras_subbands(dev, stream):
    """Polarisation-interleaved sub-band layout at the size of the paper's
    spectrometer comparison: 2 * 4096 channels * 8 sub-bands = 65536 columns,
    int8 samples, 2048 filtered spectra, T = 16 and 64."""
    import torch
    from paper_1511_03599_amd import pfb, synth
    CV, NS, S = 4096, 8, 2048
    out = {}
    for T in (16, 64):
        g = torch.Generator().manual_seed(1511600 + T)
        x = torch.randint(-100, 100, (S + T - 1, NS, CV, 2, 2), dtype=torch.int8, generator=g).to(dev)
        h = torch.from_numpy(synth.windowed_sinc_taps(CV, T)).to(dev)
        p = pfb.VegasPlan(CV, NS, T, S, "ci8")
        Y = torch.empty((S, NS, CV, 2), dtype=torch.complex64, device=dev)
        for _ in range(2):
            p.execute(x, h, Y=Y)
        t = time_calls(lambda: p.execute(x, h, Y=Y), 10, stream)
        samples = S * NS * CV * 2
        out[str(T)] = {"ms": round(t, 4), "msamples_s": round(samples / t / 1e3, 1)}
        del p, x, Y
    return out


def extras_split_adjoint(dev, stream):
    """The adjoint where no fused kernel applies (split path: inverse
    transform, reversed-tap FIR, tap-gradient partials and reduction), one
    complex64 stream of 2^27 samples: C=4096 at T=16 and C=1024 at T=32.
    GB/s counts the adjoint's minimum bytes (read gY and x, write gx)."""
    import torch
    from paper_1511_03599_amd import metrics, pfb, synth
    out = {}
    for C, T in ((4096, 16), (1024, 32)):
        S = (1 << 27) // C
        x = synth.device_noise((1, S + T - 1, C), 1511700 + C, dev)
        h = torch.from_numpy(synth.windowed_sinc_taps(C, T)).to(dev)
        gY = synth.device_noise((1, S, C), 1511800 + C, dev)
        gx = torch.empty_like(x)
        gh = torch.empty((T, C), dtype=torch.float32, device=dev)
        p = pfb.Plan(C, T, S, 1, "c64")
        for _ in range(2):
            p.backward(x, h, gY, gx=gx, gh=gh)
        t = time_calls(lambda: p.backward(x, h, gY, gx=gx, gh=gh), 10, stream)
        bb = metrics.backward_fused_bytes(1, S, C, T)
        out[f"c{C}_t{T}"] = {"bwd_ms": round(t, 4), "backward_kind": p.info()["backward_kind"],
                             "min_bytes_gbs": round(bb / t / 1e6, 1)}
        del p, x, gY, gx
    return out


def extras_single_stream(dev, stream):
    """One stream of 65536 spectra, C=1024, T=16 (the tap-sweep workload at
    16 taps): forward, adjoint and the fwd+bwd step, complex64 noise."""
    import torch
    from paper_1511_03599_amd import metrics, pfb, synth
    B, S, C, T = 1, 65536, 1024, 16
    x = synth.device_noise((B, S + T - 1, C), synth.seed_for(2, T), dev)
    h = torch.from_numpy(synth.windowed_sinc_taps(C, T)).to(dev)
    gY = synth.device_noise((B, S, C), synth.seed_for(2, 100 + T), dev)
    Y = torch.empty((B, S, C), dtype=torch.complex64, device=dev)
    gx = torch.empty_like(x)
    gh = torch.empty((T, C), dtype=torch.float32, device=dev)
    p = pfb.Plan(C, T, S, B, "c64")
    for _ in range(3):
        p.execute(x, h, Y=Y)
        p.backward(x, h, gY, gx=gx, gh=gh)
    tf = time_calls(lambda: p.execute(x, h, Y=Y), 20, stream)
    tb = time_calls(lambda: p.backward(x, h, gY, gx=gx, gh=gh), 20, stream)
    fb, bb = metrics.pfb_fused_bytes(B, S, C, T), metrics.backward_fused_bytes(B, S, C, T)
    return {"fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4), "fwd_gbs": round(fb / tf / 1e6, 1),
            "bwd_gbs": round(bb / tb / 1e6, 1), "fwd_bwd_msamples_s": round(B * S * C / (tf + tb) / 1e3, 1)}


def calibration_copies(dev):
    """Three plain 512 MiB device-to-device copies: the known traffic that
    scales the FETCH_SIZE and WRITE_SIZE counters in the profiles."""
    import torch
    a = torch.empty(1 << 26, dtype=torch.complex64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the headline step")
    ap.add_argument("--only", choices=["precision", "sweep", "batched"], default=None,
                    help="run only the named extra and print it as the JSON line (for profiling)")
    ap.add_argument("--tune", choices=["none", "batched", "all"], default="batched",
                    help="run the library's tuner before timing: for the 64-beam batched launch (default), "
                         "for every workload, or not at all")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three plain 512 MiB device copies (counter calibration for profiles)")
    args = ap.parse_args()

    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or ws > 1:
        print("bench.py runs on one GPU: the library runs each problem on one GPU (streams and beams "
              "would shard across GPUs with no communication); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1511_03599_amd import metrics, pfb, synth

    if args.only:
        dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream()
        if args.only == "precision":
            res = {"precision_c4096_t16_s32768": extras_precision(dev, stream)}
        elif args.only == "sweep":
            res = {"tap_sweep_c1024_s65536": extras_sweep(dev, stream, 1024, 65536)}
        else:
            res = {"batched_64_beams": extras_batched(dev, stream, args.tune != "none")}
        if args.copy_calibration:
            calibration_copies(dev)
        print(json.dumps(res), flush=True)
        return

    B, S, C, T = 32, 8192, 1024, 16
    dev = torch.device("cuda:0")
    log(f"bench: B={B} S={S} C={C} T={T}: generating input")
    x = synth.device_tone_streams(B, C, T, S, synth.seed_for(5), dev)
    h = torch.from_numpy(synth.windowed_sinc_taps(C, T)).to(dev)
    gY = synth.device_noise((B, S, C), synth.seed_for(5, 2), dev)
    Y = torch.empty((B, S, C), dtype=torch.complex64, device=dev)
    gx = torch.empty((B, S + T - 1, C), dtype=torch.complex64, device=dev)
    gh = torch.empty((T, C), dtype=torch.float32, device=dev)

    # With --tune all, tile shapes from the library's tuner (pfb_tune,
    # before any timing): its entry for this shape is read by the plans
    # created below, and by the other workloads' plans as the nearest entry
    # of their shape. By default the headline uses the built-in choices:
    # the tuner's picks at this shape measured no faster (2.17 against
    # 2.13 ms per step), its own timings of the candidates being this close.
    tuned = None
    if args.tune == "all":
        t0 = time.perf_counter()
        pfb.Plan(C, T, S, B, "c64").tune(tune_cache())
        os.environ["PFB_TUNE_CACHE"] = tune_cache()
        tuned = {"seconds": round(time.perf_counter() - t0, 2), "entry": open(tune_cache()).read().strip()}
        log(f"bench: tuned in {tuned['seconds']} s: {tuned['entry']}")
    plan = pfb.Plan(C, T, S, B, "c64")
    plain = pfb.Plan(C, T, S, B, "c64", pfb.PLAIN)
    stream = torch.cuda.current_stream()

    def step(p):
        p.execute(x, h, Y=Y)
        p.backward(x, h, gY, gx=gx, gh=gh)

    info = plan.info()
    log(f"bench: plan {info}")
    for _ in range(args.warmup):
        step(plan)
    torch.cuda.synchronize()
    t_step = time_calls(lambda: step(plan), args.steps, stream)
    torch.cuda.synchronize()
    log(f"bench: step {t_step:.4f} ms")

    # per-call times of the two halves (same stream, HIP events)
    t_fwd = time_calls(lambda: plan.execute(x, h, Y=Y), args.steps, stream)
    t_bwd = time_calls(lambda: plan.backward(x, h, gY, gx=gx, gh=gh), args.steps, stream)
    for _ in range(2):
        step(plain)
    t_plain = time_calls(lambda: step(plain), max(3, args.steps // 4), stream)
    t_plain_fwd = time_calls(lambda: plain.execute(x, h, Y=Y), max(3, args.steps // 4), stream)
    torch.cuda.synchronize()
    log(f"bench: fwd {t_fwd:.4f} ms, bwd {t_bwd:.4f} ms, plain step {t_plain:.4f} ms")

    fwd_bytes = metrics.pfb_fused_bytes(B, S, C, T)
    bwd_bytes = metrics.backward_fused_bytes(B, S, C, T)
    samples = B * S * C
    value = samples / (t_step * 1e-3) / 1e6
    step_gbs = (fwd_bytes + bwd_bytes) / (t_step * 1e-3) / 1e9

    # dominant kernel of the step: the adjoint (one fused kernel plus the
    # small fixed-order tap-gradient reduction) or the fused forward kernel
    if t_bwd >= t_fwd:
        name = {"fused": "fused_bwd_kernel+gh_reduce_kernel", "fused_ws": "fused_bwd_ws_kernel+gh_reduce_kernel",
                "split": "split_adjoint"}[info["backward_kind"]]
        t_dom, b_dom, tkey = t_bwd, bwd_bytes, f"pfb_backward_b{B}_s{S}_c{C}_t{T}"
    else:
        name = {"fused": "fused_fwd_ws_kernel" if info["fused_ws"] else "fused_fwd_pipe_kernel"}.get(
            info["path"], "split_forward")
        t_dom, b_dom, tkey = t_fwd, fwd_bytes, f"pfb_execute_b{B}_s{S}_c{C}_t{T}"
    achieved = b_dom / (t_dom * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK, 4), "traffic": read_traffic(tkey), "kernel": name,
            "algorithmic_bytes_per_launch": b_dom, "launch_ms": round(t_dom, 5)}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"differentiable pfb fwd+bwd, {B} streams x {S} spectra, C={C}, T={T}, "
                               f"complex64 off-centre tones, seeded gradient",
                   "channels": C, "taps": T, "spectra": S, "streams": B, "path": info["path"],
                   "backward_kind": info["backward_kind"], "fused_rows": info["fir_rows"],
                   "backward_rows": info["backward_rows"], "tuned": tuned},
        "hbm_gbs": round(step_gbs, 1), "hbm_frac": round(step_gbs / HBM_PEAK, 4),
        "fwd_ms": round(t_fwd, 5), "bwd_ms": round(t_bwd, 5),
        "fwd_gbs": round(fwd_bytes / t_fwd / 1e6, 1), "bwd_gbs": round(bwd_bytes / t_bwd / 1e6, 1),
        "fwd_frac": round(fwd_bytes / t_fwd / 1e6 / HBM_PEAK, 4),
        "bwd_frac": round(bwd_bytes / t_bwd / 1e6 / HBM_PEAK, 4),
        "plain": {"ms_per_step": round(t_plain, 5), "value": round(samples / (t_plain * 1e-3) / 1e6, 1),
                  "fwd_ms": round(t_plain_fwd, 5), "speedup": round(t_plain / t_step, 3)},
        "roofline": roof,
    }
    del plain

    if not args.quick:
        del x, gx, gY, Y
        torch.cuda.empty_cache()
        log("bench: tap sweep")
        extras = {"tap_sweep_c1024_s65536": extras_sweep(dev, stream, 1024, 65536)}
        log("bench: single stream fwd+bwd")
        extras["single_stream_b1_s65536_c1024_t16"] = extras_single_stream(dev, stream)
        torch.cuda.empty_cache()
        log("bench: split adjoint")
        extras["split_adjoint_2p27"] = extras_split_adjoint(dev, stream)
        torch.cuda.empty_cache()
        log("bench: low-precision inputs")
        extras["precision_c4096_t16_s32768"] = extras_precision(dev, stream)
        torch.cuda.empty_cache()
        log("bench: batched beams")
        extras["batched_64_beams"] = extras_batched(dev, stream, args.tune != "none")
        torch.cuda.empty_cache()
        log("bench: mixed-radix channel counts")
        extras["mixed_radix_t16"] = extras_mixed_radix(dev, stream)
        torch.cuda.empty_cache()
        log("bench: sub-band layout")
        extras["subbands_cv4096_n8_ci8"] = extras_subbands(dev, stream)
        torch.cuda.empty_cache()
        log("bench: streaming")
        extras["streaming_c1024_t16_ci16"] = extras_streaming(dev, stream)
        out["extras"] = extras

    if args.copy_calibration:
        calibration_copies(dev)

    if not args.no_cpu:
        log("bench: timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(B, S, C, T, synth.seed_for(5, 7))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
