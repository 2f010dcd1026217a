"""Every global load and store of the partial-MTTKRP kernels stays inside its
buffer, for the plans the library makes (host check, no GPU).

tests/pm_address_emulator.cpp walks every work-group, wave and lane of a plan
the way the kernels address the tensor and the output (vector loads, masked
element loads near the end, loads prefetched past a wave's range, groups that
stream several M tiles or i1 stages). It is built against the library with
hipcc and run over ragged, tiny, tall, skinny and benchmark-family shapes for
FP32, BF16 and FP16 storage.
"""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1806_07985_amd", "lib")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SHAPES = [(60, 50, 40), (33, 47, 29), (64, 40, 24, 10), (40, 36, 30), (20, 18, 22), (1024, 300), (128, 64, 33, 9),
          (3012, 12, 10), (300, 20, 10), (60, 200, 200), (36, 300, 120), (9, 8, 16), (7, 11, 13), (1, 1, 1), (1, 5, 1),
          (2, 3), (5, 1), (1, 7), (3, 1, 2), (12, 10, 9, 8, 7), (1152, 70000), (1030, 66000), (37, 29, 23),
          (200000, 40), (40, 200000), (199999, 37), (37, 199999), (4096, 64, 64), (64, 64, 4096), (1000, 100, 100),
          (333, 333, 333), (48, 2000, 33), (384, 1400, 16), (128, 128, 128, 128), (64, 64, 64, 200), (640, 30, 500),
          (64, 5, 8200), (128, 3, 4500), (64, 64, 9000), (128, 2, 8300)]


def _cases():
    rng = np.random.default_rng(0)
    shapes = list(SHAPES)
    shapes += [tuple(int(x) for x in rng.integers(32, 257, size=3)) for _ in range(8)]
    out = []
    for d in shapes:
        for s in range(1, len(d)):
            IL, IR = math.prod(d[:s]), math.prod(d[s:])
            for R in (5, 24, 50, 64):
                for dt in (0, 1, 2):
                    out.append(f"{dt} {IL} {IR} {d[s]} {d[0]} {R}")
    return out


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if not os.path.exists(os.path.join(LIB_DIR, "libnncp.so")):
        pytest.fail("libnncp.so is not built")
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("emu") / "pm_address_emulator")
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1806_07985_amd", "csrc"), os.path.join(ROOT, "tests", "pm_address_emulator.cpp"),
           "-o", exe, "-L", LIB_DIR, "-lnncp", f"-Wl,-rpath,{LIB_DIR}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_every_access_in_bounds(emulator):
    cases = _cases()
    r = subprocess.run([emulator], input="\n".join(cases) + "\n", capture_output=True, text=True, timeout=600)
    failed = [line for line in r.stdout.splitlines() if line.startswith("FAIL") or "OOB" in line]
    print(r.stdout.splitlines()[-1])
    assert r.returncode == 0 and not failed, "\n".join(failed[:20])
    assert f"{len(cases)} cases" in r.stdout.splitlines()[-1]
