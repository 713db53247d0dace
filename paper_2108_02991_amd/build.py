"""Builds libsparkling.so in-tree with hipcc for gfx950.

Usage: python -m paper_2108_02991_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT = PKG / "libsparkling.so"
BUILD_DIR = ROOT / "_build"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["sweep.hip", "reduce.hip", "project.hip", "field.hip", "fftfield.hip", "fmm.hip",
           "probe.hip", "api.cpp"]

# Packed FP32 instructions are disabled: scalar and float2 code must not be
# turned into v_pk_* FP32 operations on this target.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    # host symbols other than the C ABI stay out of the dynamic symbol table
    "-Xarch_host", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", str(ROOT / "include"), "-I", str(CSRC),
]


def _compile(src: str, extra, bdir: Path) -> Path:
    obj = bdir / (Path(src).stem + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", str(CSRC / src), "-o", str(obj)]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(extra_flags=(), out: Path | None = None, build_dir: Path | None = None) -> Path:
    """Compile every source and link libsparkling.so (next to this file by default).

    extra_flags may override the sweep tunables of spk_internal.h, e.g.
    ["-DSPK_TARGETS_F32=8"]; such variants should go to another `out`.
    """
    out = Path(out) if out else OUT
    bdir = Path(build_dir) if build_dir else BUILD_DIR
    bdir.mkdir(parents=True, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra_flags), bdir), SOURCES))
    tmp = out.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp),
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


# Host-side sanitizers for the debug build: every flag goes to the host pass
# only (-Xarch_host), device code is compiled as usual.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build_sanitized(out_dir) -> Path:
    """libsparkling.so with AddressSanitizer and UndefinedBehaviorSanitizer in
    its host code (argument validation, planning, workspace layout).  Load it
    with SPK_LIBRARY set to the returned path in a process started with
    clang's ASan runtime in LD_PRELOAD (asan_runtime())."""
    out_dir = Path(out_dir)
    return build(SANITIZE_HOST, out=out_dir / "libsparkling_asan_ubsan.so", build_dir=out_dir)


def asan_runtime() -> str:
    """Path of the ASan runtime of the compiler behind hipcc."""
    clang = Path(HIPCC).resolve().parent.parent / "lib" / "llvm" / "bin" / "clang"
    if not clang.exists():
        clang = Path("/opt/rocm/llvm/bin/clang")
    r = subprocess.run([str(clang), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    return r.stdout.strip()


if __name__ == "__main__":
    print(build(sys.argv[1:]))
