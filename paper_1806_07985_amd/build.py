"""Build the gfx950 HIP library ``lib/libnncp.so`` in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIB_DIR, "libnncp.so")
SOURCES = ["pm_plan.hip", "pm_kernels.hip", "pm16_kernels.hip", "pm16_bf16.hip", "pm16_f16.hip", "pm16_bf16_mt.hip",
           "pm16_f16_mt.hip", "small_kernels.hip",
           "driver.hip", "server.cpp", "noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object (in parallel) and link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = os.path.join(ROOT, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    os.makedirs(LIB_DIR, exist_ok=True)
    incs = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, *incs, "-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-fPIC", "-std=c++17", "-Wno-unused-result", *incs, "-c", src,
                   "-o", obj]
        log = open(obj + ".log", "w")
        procs.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT)))
        log.close()
        while True:
            running = [p for _, p in procs if p.poll() is None]
            if len(running) < jobs:
                break
            running[0].wait()
    failed = []
    for src, p in procs:
        p.wait()
        with open(os.path.join(obj_dir, os.path.basename(src) + ".o.log")) as f:
            out = f.read()
        lines = [ln for ln in out.splitlines()
                 if "packed-fp32-ops" not in ln and "unknown target feature" not in ln
                 and not ln.strip().endswith("warning generated.")
                 and not ln.strip().endswith("warnings generated.")]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError("hipcc failed:\n" + msg)
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
