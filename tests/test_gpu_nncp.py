"""End-to-end parity of the GPU NNCP driver with the FP64 oracle.

The tolerance in FP32 mode is 1e-5 relative on every factor (Frobenius norm of
the difference of the unit-column factors over the norm of the oracle's), on
lambda and on every recorded fit. The oracle runs on exactly the FP32 tensor
and FP32 starting factors the GPU receives.
"""

import numpy as np
import pytest

import oracle as O
from tolerances import TRAJ_TOL
from paper_1806_07985_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _run_gpu(X32, H0, R, iters, update="hals", split=0, graph=True, lam=None):
    from paper_1806_07985_amd import native
    Xd = native.tensor_to_device(X32)
    Hd = [native.factor_to_device(h) for h in H0]
    out = native.nncp(Xd, list(X32.shape), R, iters, Hd, lam=lam, update=update, split=split, graph=graph)
    out["H"] = [native.factor_to_host(h) for h in Hd]
    return out


def _run_oracle(X32, H0, iters, update="hals", lam=None):
    H32 = [np.asarray(h, dtype=np.float32).astype(np.float64) for h in H0]
    return O.nncp(X32.astype(np.float64), H32, iters, update=update, lam0=lam)


def _compare(g, o, tol=TOL, fits=True):
    errs = []
    for Hg, Ho in zip(g["H"], o["H"]):
        errs.append(np.linalg.norm(Hg - Ho) / np.linalg.norm(Ho))
    # a component that both sides drive to zero has lambda 0: judged against the largest lambda
    lo = np.abs(np.asarray(o["lam"]))
    lam_err = np.max(np.abs(g["lam"] - o["lam"]) / np.where(lo > 0, lo, np.max(lo)))
    fit_err = np.max(np.abs(np.asarray(g["fit"]) - np.asarray(o["fit"])) / np.abs(np.asarray(o["fit"]))) if fits else 0.0
    print(f"factor errs {['%.2e' % e for e in errs]} lam {lam_err:.2e} fit {fit_err:.2e}", flush=True)
    assert max(errs) <= tol, errs
    assert lam_err <= tol, lam_err
    assert fit_err <= tol, fit_err


def test_one_outer_iteration(gpu_lib):
    dims, R = (30, 24, 20, 12), 6
    X, _ = inputs.planted(dims, R, 0.01, seed=101, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=102)]
    for upd in ("hals", "mu"):
        print(f"case one-step {upd}", flush=True)
        _compare(_run_gpu(X, H0, R, 1, upd), _run_oracle(X, H0, 1, upd), tol=2e-6)


def test_trajectory_3way_60x50x40_rank5(gpu_lib):
    """60x50x40 planted rank 5 + 1% noise, HALS, 20 iterations, split {1,2}|{3}."""
    dims, R = (60, 50, 40), 5
    X64, _ = inputs.planted(dims, R, 0.01, seed=1)
    X = X64.astype(np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=2)]
    ref = _run_oracle(X, H0, 20)
    for split in (2, 1):
        print(f"case C1 split={split}", flush=True)
        _compare(_run_gpu(X, H0, R, 20, split=split), ref)


@pytest.mark.parametrize("update", ["hals", "mu"])
def test_trajectory_4way(gpu_lib, update):
    dims, R = (20, 18, 16, 14), 8
    X, _ = inputs.planted(dims, R, 0.01, seed=11, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=12)]
    ref = _run_oracle(X, H0, 30, update)
    for split in (2, 1, 3):
        print(f"case 4way {update} split={split}", flush=True)
        _compare(_run_gpu(X, H0, R, 30, update, split=split), ref)


def test_trajectory_5way_and_2way(gpu_lib):
    for dims, R in [((8, 7, 6, 5, 4), 4), ((70, 45), 7)]:
        X, _ = inputs.planted(dims, R, 0.02, seed=21, dtype=np.float32)
        H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=22)]
        print(f"case dims={dims}", flush=True)
        _compare(_run_gpu(X, H0, R, 15), _run_oracle(X, H0, 15))


def test_graph_replay_is_bitwise_equal_to_eager(gpu_lib):
    dims, R = (24, 22, 20), 7
    X, _ = inputs.planted(dims, R, 0.01, seed=31, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=32)]
    a = _run_gpu(X, H0, R, 12, graph=True)
    b = _run_gpu(X, H0, R, 12, graph=False)
    for Ha, Hb in zip(a["H"], b["H"]):
        assert np.array_equal(Ha, Hb)
    assert np.array_equal(a["fit"], b["fit"]) and np.array_equal(a["lam"], b["lam"])


def test_resume_from_finished_state(gpu_lib):
    """Running 6 + 6 iterations through finish() equals 12 iterations (to tolerance)."""
    from paper_1806_07985_amd import native
    dims, R = (26, 20, 18), 5
    X, _ = inputs.planted(dims, R, 0.01, seed=41, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=42)]
    Xd = native.tensor_to_device(X)
    Hd = [native.factor_to_device(h) for h in H0]
    plan = native.Plan(Xd, list(dims), R, Hd)
    f1 = plan.run(6)
    lam1 = plan.finish()
    f2 = plan.run(6)
    lam2 = plan.finish()
    plan.close()
    ref = _run_oracle(X, H0, 12)
    g = dict(H=[native.factor_to_host(h) for h in Hd], lam=lam2, fit=np.concatenate([f1, f2]))
    _compare(g, ref)


def test_zero_column_stays_zero(gpu_lib):
    dims, R = (15, 12, 10), 4
    X, _ = inputs.planted(dims, 3, 0.01, seed=51, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=52)]
    H0[1][:, 2] = 0.0
    g = _run_gpu(X, H0, R, 5)
    o = _run_oracle(X, H0, 5)
    for H in g["H"]:
        assert np.all(H[:, 2] == 0.0)
    assert g["lam"][2] == 0.0 and o["lam"][2] == 0.0
    keep = [0, 1, 3]
    for Hg, Ho in zip(g["H"], o["H"]):
        assert np.linalg.norm(Hg[:, keep] - Ho[:, keep]) <= TOL * np.linalg.norm(Ho[:, keep])


def test_lambda_input_scales_the_model(gpu_lib):
    dims, R = (12, 11, 10), 3
    X, _ = inputs.planted(dims, R, 0.01, seed=61, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=62)]
    lam = np.array([2.0, 0.5, 3.0])
    _compare(_run_gpu(X, H0, R, 4, lam=lam), _run_oracle(X, H0, 4, lam=lam))


@pytest.mark.parametrize("dims,R,dt", [((30, 24, 20), 6, "f32"), ((16, 14, 12, 10), 8, "f32"),
                                       ((10, 9, 8, 7, 6), 4, "f32"), ((40, 30), 5, "f32"),
                                       ((20, 18, 16, 14), 8, "bf16")])
def test_no_tree_matches_oracle_and_tree(gpu_lib, dims, R, dt):
    """Every mode's MTTKRP straight from the tensor (the tree-less baseline) gives
    the oracle's trajectory, like the dimension tree."""
    import torch
    from paper_1806_07985_amd import native
    print(f"case no-tree dims={dims} R={R} {dt}", flush=True)
    X, _ = inputs.planted(dims, R, 0.01, seed=21, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=22)]
    flat = torch.from_numpy(np.ascontiguousarray(X.ravel(order="F")))
    if dt == "bf16":
        flat = flat.to(torch.bfloat16)
    X64 = flat.to(torch.float64).numpy().reshape(dims, order="F")
    out = {}
    for nt in (False, True):
        Hd = [native.factor_to_device(h) for h in H0]
        r = native.nncp(flat.cuda(), list(dims), R, 10, Hd, no_tree=nt)
        out[nt] = ([native.factor_to_host(h) for h in Hd], r["lam"], r["fit"])
    ref = O.nncp(X64, [h.astype(np.float64) for h in H0], 10)
    tol = TRAJ_TOL[dt]
    for nt in (False, True):
        H, lam, fit = out[nt]
        errs = [np.linalg.norm(h - rh) / np.linalg.norm(rh) for h, rh in zip(H, ref["H"])]
        print(f"  no_tree={nt}: factors {max(errs):.1e} fit {np.max(np.abs(fit - ref['fit'])):.1e}", flush=True)
        assert max(errs) < tol and np.max(np.abs(fit - np.asarray(ref["fit"]))) < tol


@pytest.mark.parametrize("dims,R,update,sweeps", [((30, 24, 20), 6, "hals", 10), ((16, 14, 12, 10), 40, "hals", 5),
                                                  ((24, 20, 18), 80, "hals", 4), ((20, 18, 16), 8, "mu", 6),
                                                  ((22, 20, 18), 70, "mu", 3)])
def test_inner_sweeps_match_oracle(gpu_lib, dims, R, update, sweeps):
    """Several update sweeps per block update (towards the exact NNLS block
    solve) give the oracle's trajectory with the same number of sweeps; both
    update kernels (rank <= 64 in registers, larger ranks through LDS)."""
    from paper_1806_07985_amd import native
    print(f"case inner sweeps dims={dims} R={R} {update} sweeps={sweeps}", flush=True)
    X, _ = inputs.planted(dims, min(R, 8), 0.02, seed=51, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=52)]
    Xd = native.tensor_to_device(X)
    Hd = [native.factor_to_device(h) for h in H0]
    g = native.nncp(Xd, list(dims), R, 6, Hd, update=update, inner_sweeps=sweeps)
    g["H"] = [native.factor_to_host(h) for h in Hd]
    o = O.nncp(X.astype(np.float64), [h.astype(np.float64) for h in H0], 6, update=update, inner_sweeps=sweeps)
    _compare(g, o)


def test_inner_sweeps_in_batch_equal_alone(gpu_lib):
    """A member with several sweeps per block computes the same bits in a batch."""
    import torch
    from paper_1806_07985_amd import native
    dims, R = (26, 22, 20), 12
    X, _ = inputs.planted(dims, R, 0.02, seed=53, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=54)]
    res = []
    for batched in (False, True):
        Xd = native.tensor_to_device(X)
        Hd = [native.factor_to_device(h) for h in H0]
        plan = native.Plan(Xd, list(dims), R, Hd, inner_sweeps=7, graph=not batched)
        if batched:
            b = native.Batch()
            b.add(plan)
            b.run(5)
            b.close()
            fit = plan.fits()
        else:
            fit = plan.run(5)
        res.append((fit, [h.clone() for h in Hd]))
    assert np.array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert torch.equal(a, b)


def test_inner_sweeps_above_maximum_rejected(gpu_lib):
    from paper_1806_07985_amd import native
    dims, R = (8, 7, 6), 3
    X, _ = inputs.planted(dims, R, 0.02, seed=55, dtype=np.float32)
    Hd = [native.factor_to_device(h.astype(np.float32)) for h in inputs.init_factors(dims, R, seed=56)]
    with pytest.raises(Exception):
        native.nncp(native.tensor_to_device(X), list(dims), R, 1, Hd, inner_sweeps=100001)


@pytest.mark.parametrize("dims,R,dt", [((24, 20, 18, 16), 8, "f32"), ((40, 36, 30), 12, "bf16"),
                                       ((12, 10, 9, 8, 7), 4, "f32")])
def test_autotune_split_picks_the_fastest_timed_split(gpu_lib, dims, R, dt):
    """Every root split is timed; the returned one is the fastest; the factors
    are left untouched; a plan on that split still matches the oracle."""
    import torch
    from paper_1806_07985_amd import native
    print(f"case autotune dims={dims} R={R} {dt}", flush=True)
    X, _ = inputs.planted(dims, R, 0.01, seed=61, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=62)]
    flat = torch.from_numpy(np.ascontiguousarray(X.ravel(order="F")))
    if dt == "bf16":
        flat = flat.to(torch.bfloat16)
    X64 = flat.to(torch.float64).numpy().reshape(dims, order="F")
    Xd = flat.cuda()
    Hd = [native.factor_to_device(h) for h in H0]
    best, ms = native.autotune_split(Xd, list(dims), R, Hd, reps=2)
    print(f"  best split {best}, ms {ms}", flush=True)
    assert len(ms) == len(dims) - 1 and all(t > 0 for t in ms)
    assert 1 <= best <= len(dims) - 1 and ms[best - 1] == min(ms)
    for h, h0 in zip(Hd, H0):
        assert np.array_equal(native.factor_to_host(h), h0)
    r = native.nncp(Xd, list(dims), R, 5, Hd, split=best)
    ref = O.nncp(X64, [h.astype(np.float64) for h in H0], 5)
    tol = TRAJ_TOL[dt]
    assert np.max(np.abs(r["fit"] - np.asarray(ref["fit"]))) < tol


@pytest.mark.parametrize("dims,R", [((12, 10, 5000), 16), ((8, 6, 1500), 40)])
def test_multichunk_gram_and_fit_match_oracle(gpu_lib, dims, R):
    """A last mode long enough that its Gram (and the fit) is summed over several
    row chunks, with one and two R x R entries per thread."""
    print(f"case multichunk dims={dims} R={R}", flush=True)
    X, _ = inputs.planted(dims, min(R, 6), 0.02, seed=71, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=72)]
    g = _run_gpu(X, H0, R, 5)
    o = _run_oracle(X, H0, 5)
    _compare(g, o)
