"""Compile the HIP library (libtds.so) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libtds.so"
BUILD = PKG / "_build"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # the pair decision is pinned to an exact operation order: no contraction
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{ROOT / 'include'}",
]
SOURCES = ["tds_kernels.hip", "tds_traj.hip", "tds_greedy.hip", "tds_api.cpp", "tds_server.cpp"]
# vector-ALU issue-rate probes for the benchmark's peak figures (own library)
PROBE_LIB = PKG / "libtds_probe.so"
PROBE_SOURCES = ["tds_probe.hip"]


def build(verbose: bool = False, extra: list[str] | None = None, out: Path | None = None) -> Path:
    """Compile libtds.so (or `out`, with `extra` compiler flags); with the
    default output also the probe library."""
    if out is None:
        _link(PROBE_LIB, PROBE_SOURCES, BUILD, verbose, extra)
        return _link(LIB, SOURCES, BUILD, verbose, extra)
    lib = Path(out)
    return _link(lib, SOURCES, lib.parent / (lib.stem + "_build"), verbose, extra)


def _link(lib: Path, sources: list[str], bdir: Path, verbose: bool, extra: list[str] | None) -> Path:
    bdir.mkdir(parents=True, exist_ok=True)
    objs = []
    for src in sources:
        obj = bdir / (Path(src).stem + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC, *COMMON, *(extra or []), *lang, "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib.with_suffix(f".so.tmp{os.getpid()}")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
