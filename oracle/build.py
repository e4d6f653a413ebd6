"""Compile the oracle (plain C, FP64, OpenMP) into a shared library.

Test infrastructure only. ``build()`` returns the path of the library;
``defines``/``src_text`` let a test compile a modified copy elsewhere.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
SRC = HERE / "oracle.c"
BUILD_DIR = HERE / "_build"
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Werror"]


def build(out: Path | None = None, src_text: str | None = None, force: bool = False) -> Path:
    text = SRC.read_text() if src_text is None else src_text
    tag = hashlib.sha1(text.encode()).hexdigest()[:12]
    out_dir = BUILD_DIR if out is None else Path(out)
    out_dir.mkdir(parents=True, exist_ok=True)
    lib = out_dir / f"liboracle_{tag}.so"
    if lib.exists() and not force:
        return lib
    src = out_dir / f"oracle_{tag}.c"
    src.write_text(text)
    tmp = lib.with_suffix(f".so.tmp{os.getpid()}")
    flags = CFLAGS if src_text is None else [f for f in CFLAGS if f != "-Werror"]
    subprocess.run(["gcc", *flags, str(src), "-o", str(tmp), "-lm"], check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(force=True))
