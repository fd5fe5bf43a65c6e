"""Build the HIP library liblbib.so for gfx950, in-tree.

Usage: python -m paper_1907_00080_amd.build   (or build() from Python).
Every call recompiles (sources in parallel) and refuses a library whose
kernels use private (scratch) memory.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbib.so")
SOURCES = ["engine.hip", "k_lattice.hip", "k_lagrangian.hip", "k_adjoint.hip", "k_repulsion.hip", "k_observe.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _llvm_tool(name: str) -> str:
    for d in ("/opt/rocm/lib/llvm/bin", "/opt/rocm/llvm/bin"):
        path = os.path.join(d, name)
        if os.path.exists(path):
            return path
    return name


def private_segments(obj: str, workdir: str) -> dict:
    """Kernel name -> private (scratch) bytes per lane, read from the gfx950
    code object compiled into `obj`."""
    base = os.path.join(workdir, os.path.basename(obj))
    sections = subprocess.run([_llvm_tool("llvm-readelf"), "-S", "--wide", obj], check=True,
                              capture_output=True, text=True).stdout
    if ".hip_fatbin" not in sections:
        return {}   # host code only
    subprocess.run([_llvm_tool("llvm-objcopy"), "--dump-section", f".hip_fatbin={base}.fat", obj],
                   check=True, capture_output=True)
    subprocess.run([_llvm_tool("clang-offload-bundler"), "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={base}.fat",
                    f"--output={base}.elf", "--unbundle"], check=True, capture_output=True)
    notes = subprocess.run([_llvm_tool("llvm-readelf"), "--notes", f"{base}.elf"], check=True,
                           capture_output=True, text=True).stdout
    out, name = {}, None
    for line in notes.splitlines():
        line = line.strip()
        if line.startswith(".name:"):
            name = line.split(":", 1)[1].strip()
        elif line.startswith(".private_segment_fixed_size:") and name is not None:
            out[name] = int(line.split(":", 1)[1])
    return out


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), check that no kernel
    spills register arrays to private memory (a silent slowdown of the
    latency-bound kernels), then link liblbib.so."""
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include")]
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="lbib_build_") as work:
        def compile_one(src: str) -> str:
            obj = os.path.join(work, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc()] + flags + inc + ["-c", "-o", obj, os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            return obj
        jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
        with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
            objs = list(pool.map(compile_one, SOURCES))
        spills = {}
        for obj in objs:
            spills.update({k: v for k, v in private_segments(obj, work).items() if v > 0})
        if spills:
            lines = "\n".join(f"  {k}: {v} bytes" for k, v in sorted(spills.items()))
            raise RuntimeError("kernels with private (scratch) memory per lane:\n" + lines)
        cmd = [hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp] + objs
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking liblbib.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
