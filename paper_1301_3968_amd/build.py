"""Build libdedisp.so (HIP, gfx950) in-tree with hipcc.

Every HIP translation unit is compiled for gfx950 only, without packed-fp32
instruction selection and without floating-point contraction (the host delay
arithmetic must reproduce floor/ceil of the stated double expressions).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdedisp.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["plan.cpp", "api.cpp", "kernels_basic.hip", "kernels_search.hip", "kernels_f32.hip",
           "kernels_mfma.hip"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(HERE, "..", "include"),
]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer (device code is left as it is);
# the library then needs the sanitizer runtime preloaded into the process.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
SAN_LIB = os.path.join(HERE, "libdedisp_san.so")


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False) -> str:
    """Compile every source and link the library; with sanitize, a host-sanitized copy
    (libdedisp_san.so, for host-side checks on a machine without a GPU)."""
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    lib_path = SAN_LIB if sanitize else LIB
    extra = SANITIZE_HOST if sanitize else []
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [hipcc] + lang + COMMON + extra + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = lib_path + ".tmp"
    link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-shared-libsan"] if sanitize else ["-Wl,--no-undefined"]
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + link + [
        "-L", os.path.join(ROCM, "lib"), "-lamdhip64"]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout)
    os.replace(tmp, lib_path)
    return lib_path


PROBE_SRC = os.path.join(CSRC, "probe_lds.hip")
PROBE_BIN = os.path.join(HERE, "probe_lds")


def build_probe(verbose: bool = False) -> str:
    """Compile the LDS read-rate measurement program (not part of the library)."""
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    cmd = [hipcc, "-x", "hip"] + [f for f in COMMON if f != "-fPIC"] + [PROBE_SRC, "-o", PROBE_BIN]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode != 0:
        raise RuntimeError("probe build failed:\n" + out.stdout)
    return PROBE_BIN


def _wait(procs):
    errs = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            errs.append(f"{src}:\n{text}")
        elif "warning" in text and os.environ.get("DEDISP_BUILD_VERBOSE"):
            print(text)
    if errs:
        raise RuntimeError("compile failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
