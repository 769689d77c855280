"""Build the HIP library (gfx950) in-tree: paper_2503_17743_amd/libmoc.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmoc.so")
SOURCES = ["plan.cpp", "sweep.hip", "api.cpp", "server.cpp"]
ARCH = os.environ.get("MOC_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"-I{ROOT}/include",
              "-Wall", "-Wno-unused-result"]
    # packed FP32 instructions are kept out of generated device code
    dev = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-munsafe-fp-atomics"]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc] + common + dev + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd = [hipcc, "-x", "hip"] + common + dev + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l
                         and "not a recognized feature" not in l)
        if text.strip() and verbose:
            print(text)
        if p.returncode != 0:
            failed.append((src, text))
    if failed:
        for src, text in failed:
            print(f"--- {src} failed ---\n{text}", file=sys.stderr)
        raise RuntimeError("HIP library build failed")
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
