"""Build the HIP library ``libphotonmc.so`` for gfx950 with hipcc (in-tree).

The walk is FP32 with FP contraction off, so every launch shape produces the
same bits; packed-FP32 instruction selection is disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libphotonmc.so")
SOURCES = [os.path.join(CSRC, "photonmc.hip"), os.path.join(CSRC, "batch.hip"), os.path.join(CSRC, "spinodal.hip"),
           os.path.join(CSRC, "analytics.hip"), os.path.join(CSRC, "metrics.hip"),
           os.path.join(CSRC, "noalloc.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("philox.hpp", "walk.hpp", "internal.hpp", "select.hpp")] + [
    os.path.join(INCLUDE, "photonmc.h"), os.path.join(INCLUDE, "spinodal.h"), os.path.join(INCLUDE, "analytics.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _run(cmd: list[str]) -> str:
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    errs = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + errs)
    return errs


def build_library(verbose: bool = False, out: str = LIB, defines: tuple[str, ...] = ()) -> str:
    """Compile the library (always; the caller decides when): each source to an object
    in parallel under ``_build/``, then one link."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(ROOT, "_build", os.path.basename(out) + ".obj")
    os.makedirs(objdir, exist_ok=True)
    flags = [f for f in HIPCC_FLAGS if f != "-shared"] + [f"-D{d}" for d in defines]
    objs = [os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o") for src in SOURCES]
    cmds = [[hipcc(), *flags, f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        msgs = list(ex.map(_run, cmds))
    msgs.append(_run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out + ".tmp"]))
    if verbose and any(m.strip() for m in msgs):
        print("\n".join(m for m in msgs if m.strip()))
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
