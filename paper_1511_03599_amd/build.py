"""Build the HIP library libpfb.so for gfx950 (in-tree, next to this file).

    python -m paper_1511_03599_amd.build [--jobs N] [--changed]

Every source under csrc/ is compiled by hipcc to an object in _build/, then
linked into libpfb.so. By default the build recompiles everything (it is the
"does it build" check as well as the build); --changed recompiles only the
sources whose object is older than the source or than any header in csrc/
or include/.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpfb.so")
ARCH = "gfx950"

# Packed FP32 instructions are switched off for the device code: every FP32
# operation is issued as a plain VALU instruction. Floating-point contraction
# is off: the kernels write their fused multiply-adds explicitly, so the
# rounding of every result is fixed by the source and identical on every
# code path (fused, split, batched).
HIP_FLAGS = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    obj = _obj(src)
    cmd = [hipcc(), *HIP_FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{out}")
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def _obj(src: str) -> str:
    return os.path.join(BUILD, os.path.basename(src) + ".o")


def _stale(src: str) -> bool:
    obj = _obj(src)
    if not os.path.exists(obj):
        return True
    headers = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))
    newest = max([os.path.getmtime(src)] + [os.path.getmtime(h) for h in headers])
    return os.path.getmtime(obj) < newest


def build(jobs: int | None = None, verbose: bool = False, changed_only: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if changed_only else srcs
    jobs = jobs or min(max(1, len(todo)), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [_obj(s) for s in srcs]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--changed", action="store_true", help="recompile only out-of-date sources")
    args = ap.parse_args()
    build(args.jobs, verbose=True, changed_only=args.changed)


if __name__ == "__main__":
    main()
