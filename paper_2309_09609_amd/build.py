"""Builds libswsearch.so for gfx950 with hipcc (in-tree, next to this file).

The 16-bit sweep compares biased integers with half-float maximum
instructions, and most of those integers (1..1023) are subnormal halves, so
every kernel must run with f16 denormals preserved (the hardware's f16/f64
denormal mode 3, the default).  ``build()`` refuses flags that change it and
checks the mode recorded in every kernel descriptor of the build.
"""
from __future__ import annotations

import os
import re
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libswsearch.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("sw_kernels.hip", "sw_align.hip", "sw_pair.hip",
                                                           "sw_noalloc.hip", "sw_api.cpp")]
HIP_SOURCES = [s for s in SOURCES if s.endswith(".hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         # packed FP32 instructions stay off (the kernels are integer-only anyway)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]
# Extra hipcc flags may be given in SWSEARCH_HIPCC_FLAGS (checked by check_flags).
EXTRA_ENV = "SWSEARCH_HIPCC_FLAGS"


def check_flags(flags) -> None:
    """Raise ValueError for flags that may flush f16 subnormals or let the
    compiler assume away infinities and NaNs (which mark saturated cells)."""
    for f in flags:
        bad = (f.startswith("-fdenormal-fp-math") and not f.endswith("=ieee")) or \
            f in ("-ffast-math", "-ffinite-math-only", "-fno-honor-nans", "-fno-honor-infinities",
                  "-funsafe-math-optimizations", "-ffp-model=fast", "-fgpu-flush-denormals-to-zero",
                  "-fcuda-flush-denormals-to-zero")
        if bad:
            raise ValueError(f"hipcc flag {f!r} is not allowed: the 16-bit sweep needs f16 subnormals preserved "
                             f"and infinities/NaNs kept")


def denormal_modes(flags, sources=None) -> dict:
    """{kernel: f16/f64 denormal mode} from the device assembly of the HIP sources (default: all) built
    with flags."""
    modes = {}
    for src in sources or HIP_SOURCES:
        r = subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", src, "-o", "-"], capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError(f"hipcc failed building the device assembly of {src}")
        name = None
        for line in r.stdout.splitlines():
            m = re.match(r"\s*\.amdhsa_kernel\s+(\S+)", line)
            if m:
                name = m.group(1)
            m = re.match(r"\s*\.amdhsa_float_denorm_mode_16_64\s+(\d+)", line)
            if m and name:
                modes[name] = int(m.group(1))
    return modes


def build(verbose: bool = False) -> str:
    extra = shlex.split(os.environ.get(EXTRA_ENV, ""))
    check_flags(extra)
    flags = FLAGS + extra
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *flags, "-shared", *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    modes = denormal_modes(flags)          # the device assembly, built meanwhile
    out, _ = proc.communicate()
    if proc.returncode != 0:
        sys.stderr.write(out)
        raise RuntimeError("hipcc failed building libswsearch.so")
    flushing = sorted(k for k, v in modes.items() if v != 3)
    if not modes or flushing:
        os.remove(tmp)
        raise RuntimeError(f"kernels built without f16 subnormals preserved: {flushing or 'no kernel found'}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"{len(modes)} kernels, f16/f64 denormal mode 3 (preserve) in every descriptor", flush=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
