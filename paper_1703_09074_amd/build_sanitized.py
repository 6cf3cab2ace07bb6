"""Builds a copy of librcp whose host code runs under AddressSanitizer and
UndefinedBehaviorSanitizer, for the CPU tests of the C interface:

    python -m paper_1703_09074_amd.build_sanitized

The C interface, argument checking, workspace layout and batch program
builder (rcp_api.cpp) are compiled with both sanitizers on the host side
only; the kernels are the ordinary objects of build.py (compiled here when
missing).  The library links the sanitizer runtime dynamically, so a process
that loads it needs that runtime first in its library list (LD_PRELOAD of
``runtime()``).  Output: _build/librcp_san.so, never the product library.
"""
from __future__ import annotations

import os
import subprocess
import sys

from . import build as _b

SAN_LIB = os.path.join(_b.BUILD, "librcp_san.so")
# every sanitizer flag applies to the host pass only
SAN_FLAGS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
             "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()
SAN_LINK = "-shared-libasan -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()


def runtime() -> str:
    """Path of the shared AddressSanitizer runtime of hipcc's clang."""
    clang = os.path.join(os.path.dirname(os.path.realpath(_b._hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True, check=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        raise RuntimeError("AddressSanitizer runtime not found")
    return out


def _fresh(obj: str, src: str) -> bool:
    return os.path.exists(obj) and os.path.getmtime(obj) >= os.path.getmtime(src)


def build(verbose: bool = False) -> str:
    os.makedirs(_b.BUILD, exist_ok=True)
    objs = []
    for src in _b.SOURCES:
        path = os.path.join(_b.CSRC, src)
        stem = os.path.splitext(src)[0]
        if src.endswith(".cpp"):
            obj = os.path.join(_b.BUILD, stem + "_san.o")
            cmd = [_b._hipcc(), "-x", "hip"] + _b.HIP_FLAGS + SAN_FLAGS + ["-g", "-c", path, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        else:
            obj = os.path.join(_b.BUILD, stem + ".o")
            if not _fresh(obj, path):
                obj = _b._compile(src)
        objs.append(obj)
    tmp = SAN_LIB + ".tmp"
    cmd = [_b._hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN_LINK + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
