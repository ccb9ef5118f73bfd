"""Build libcoloc.so (and the input generator's libsynth.so) for gfx950.

Every HIP translation unit is compiled with hipcc for gfx950 only, with
packed FP32 instructions disabled, then linked into one shared library next
to this file.  Run: python -m paper_2501_16909_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["k_memory.hip", "k_compute.hip", "k_dense.hip", "k_util.hip", "k_decode.hip", "runtime.hip",
           "serve.hip", "decode.hip"]
LIB = os.path.join(HERE, "libcoloc.so")
SYNTH_SRC = os.path.join(ROOT, "synth", "fill.hip")
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth.so")


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-FP32 feature switch; that note is noise
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, s.replace(".hip", ".o")) for s in SOURCES]
    jobs = [[HIPCC, *FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    jobs.append([HIPCC, *FLAGS, "-shared", SYNTH_SRC, "-o", SYNTH_LIB + ".tmp"])
    workers = min(len(jobs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    _run([HIPCC, *FLAGS, "-shared", *objs, "-o", LIB + ".tmp"])
    os.replace(LIB + ".tmp", LIB)
    os.replace(SYNTH_LIB + ".tmp", SYNTH_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
