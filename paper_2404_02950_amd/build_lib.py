"""Build libshamr.so for gfx950 with hipcc (run on any machine with ROCm; no GPU needed).

    python -m paper_2404_02950_amd.build_lib

Flags that matter for the numerics: -ffp-contract=off (no fused multiply-add, so the
float results follow the written operation order) and packed FP32 instructions
disabled (-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libshamr.so")

ARCH = os.environ.get("SHAMR_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall"]

HIP_SOURCES = ["kernels.hip", "kernels_hilap.hip", "kernels_ko.hip", "kernels_ko_lds.hip", "kernels_fused.hip", "kernels_stream.hip", "runtime.cpp"]
HOST_SOURCES = ["cluster.cpp", "local_regrid.cpp"]


# the device-code sources each kernel family is compiled from
KERNEL_SOURCES = {
    "fused": ("kernels_fused.hip", "sh_device.h", "sh_internal.h"),
    "stage": ("kernels.hip", "kernels_hilap.hip", "kernels_ko.hip", "kernels_ko_lds.hip", "sh_stage.h", "sh_device.h", "sh_internal.h"),
}


def kernel_family(kernel: str) -> str:
    """'fused' for the fused step (k_fused_step, fused_* bench names), else 'stage'."""
    return "fused" if ("fused" in kernel) else "stage"


def kernel_source_sha(family: str = "fused") -> str:
    """SHA-256 over the sources of one kernel family; counter summaries record it so a
    figure taken on other kernels is not reported for these."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libshamr)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:2])} ... (exit {r.returncode})")
    return r


# Host-code sanitizer build (a debugging aid, run on the CPU only): AddressSanitizer and
# UndefinedBehaviorSanitizer on the host side of every source (the device code is built as
# usual), all host code compiled by ROCm's clang so that one sanitizer runtime serves it.
SAN_BUILD = os.path.join(PKG, "_build_san")
SAN_LIB = os.path.join(SAN_BUILD, "libshamr_san.so")
SAN_HIP = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _clangxx() -> str:
    c = os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "llvm", "bin", "clang++")
    return os.path.realpath(c) if os.path.exists(c) else "/opt/rocm/llvm/bin/clang++"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source (in parallel) and link libshamr.so; returns the library path.
    With ``sanitize``, build the host-sanitizer variant in _build_san/ instead."""
    from concurrent.futures import ThreadPoolExecutor
    out_dir = SAN_BUILD if sanitize else BUILD
    lib = SAN_LIB if sanitize else LIB
    os.makedirs(out_dir, exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", INCLUDE, "-I", CSRC]
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        extra = SAN_HIP if sanitize else []
        cmds.append([hipcc] + HIP_FLAGS + extra + inc + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        if sanitize:
            cmds.append([_clangxx()] + HOST_FLAGS + ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
                        + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
        else:
            cmds.append(["g++"] + HOST_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=max(1, min(len(cmds), os.cpu_count() or 1))) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = lib + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if sanitize:
        link += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    _run(link, verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
