"""Batched plans (GPU): members advanced together by persistent work-list
kernels give the same results as the same plans run alone, and agree with the
FP64 oracle.

A member keeps the kernels, tiles and summation order of its stand-alone run
(its tiling depends on its own shape only), so alone and in the mix the
factors must be bitwise equal; the oracle bound is the FP32-mode 1e-5.
"""

import numpy as np
import pytest

import oracle as O
from tolerances import TRAJ_TOL
from paper_1806_07985_amd import inputs

pytestmark = pytest.mark.gpu

# (dims, R, update, split, dtype, wg_kib): mixed orders, ranks, updates, storage
JOBS = [
    ((40, 30, 20), 8, "hals", 0, "f32", 8),
    ((24, 20, 18, 6), 16, "mu", 2, "f32", 4),
    ((30, 28, 26), 32, "hals", 1, "bf16", 4),
    ((12, 10, 9, 8, 7), 4, "hals", 3, "f32", 1),
    ((64, 48, 40), 24, "hals", 2, "f16", 16),
    ((50, 33, 17), 50, "hals", 0, "f32", 2),
    ((37, 29, 23), 12, "hals", 1, "f32", 0),
    ((64, 40, 1000), 16, "hals", 1, "bf16", 0),   # tall right node with J == 1: its own kernel family
    ((60, 300, 120), 10, "hals", 1, "bf16", 0),   # the same, masked form (I_L % 8 == 4, ragged I1)
]


def _tensor(dims, R, dt, seed):
    import torch
    from paper_1806_07985_amd import native
    X, _ = inputs.planted(dims, R, 0.01, seed=seed, dtype=np.float32)
    flat = torch.from_numpy(np.ascontiguousarray(X.ravel(order="F")))
    if dt == "f32":
        return flat.cuda(), X.astype(np.float64)
    q = flat.to({"bf16": torch.bfloat16, "f16": torch.float16}[dt])
    return q.cuda(), q.to(torch.float64).numpy().reshape(dims, order="F")


def _make(job, seed, graph=True):
    from paper_1806_07985_amd import native
    dims, R, update, split, dt, kib = job
    Xd, X64 = _tensor(dims, R, dt, seed)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=seed + 1)]
    Hd = [native.factor_to_device(h) for h in H0]
    plan = native.Plan(Xd, list(dims), R, Hd, update=update, split=split, graph=graph, pm_wg_kib=kib)
    return dict(plan=plan, X=Xd, H=Hd, H0=H0, X64=X64)


def test_batch_members_equal_alone_bitwise(gpu_lib):
    import torch
    from paper_1806_07985_amd import native
    iters = 6
    alone = []
    for j, job in enumerate(JOBS):
        print(f"case alone {job}", flush=True)
        m = _make(job, 100 + 10 * j)
        m["fit"] = m["plan"].run(iters)
        alone.append(m)
    batch = native.Batch()
    mixed = []
    for j, job in enumerate(JOBS):
        m = _make(job, 100 + 10 * j, graph=False)
        batch.add(m["plan"])
        mixed.append(m)
    print(f"case batch of {len(batch)} {batch.stats()}", flush=True)
    batch.run(iters)
    for job, a, b in zip(JOBS, alone, mixed):
        fa, fb = a["fit"], b["plan"].fits()
        assert len(fb) == iters
        assert np.array_equal(fa, fb), (job, fa, fb)
        for ha, hb in zip(a["H"], b["H"]):
            assert torch.equal(ha, hb), job
    batch.close()


def test_batch_matches_oracle(gpu_lib):
    from paper_1806_07985_amd import native
    iters = 12
    batch = native.Batch()
    ms = []
    for j, job in enumerate(JOBS):
        m = _make(job, 300 + 10 * j, graph=False)
        batch.add(m["plan"])
        ms.append(m)
    batch.run(iters)
    for job, m in zip(JOBS, ms):
        dims, R, update, split, dt, kib = job
        lam = m["plan"].finish()
        ref = O.nncp(m["X64"], [h.astype(np.float64) for h in m["H0"]], iters, update=update)
        errs = [np.linalg.norm(native.factor_to_host(h) - r) / np.linalg.norm(r) for h, r in zip(m["H"], ref["H"])]
        fit_err = float(np.max(np.abs(m["plan"].fits() - np.asarray(ref["fit"]))))
        lam_err = float(np.max(np.abs(lam - ref["lam"]) / ref["lam"]))
        print(f"case oracle {job}: factors {max(errs):.1e} lam {lam_err:.1e} fit {fit_err:.1e}", flush=True)
        tol = TRAJ_TOL[dt]
        assert max(errs) < tol and lam_err < tol and fit_err < tol
    batch.close()


def test_batch_membership_changes(gpu_lib):
    """Members join and leave between ticks; each member's result equals its
    stand-alone run of the same number of iterations."""
    import torch
    from paper_1806_07985_amd import native
    jobs = JOBS[:4]
    batch = native.Batch()
    ms = [_make(job, 500 + 10 * j, graph=False) for j, job in enumerate(jobs)]
    batch.add(ms[0]["plan"])
    batch.add(ms[1]["plan"])
    batch.run(3)
    batch.add(ms[2]["plan"])
    batch.run(2)
    batch.remove(ms[0]["plan"])     # member 0 leaves after 5 iterations
    batch.add(ms[3]["plan"])
    batch.run(4)
    done = {0: 5, 1: 9, 2: 6, 3: 4}
    for j, job in enumerate(jobs):
        a = _make(job, 500 + 10 * j)
        fa = a["plan"].run(done[j])
        fb = ms[j]["plan"].fits()
        print(f"case membership {job}: iters {len(fb)}", flush=True)
        assert np.array_equal(fa, fb)
        for ha, hb in zip(a["H"], ms[j]["H"]):
            assert torch.equal(ha, hb)
    batch.close()
