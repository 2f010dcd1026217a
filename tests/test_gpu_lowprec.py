"""Parity of the BF16 / FP16 tensor path against the FP64 oracle (GPU).

The tensor is rounded to BF16 or FP16 on the CPU (torch, round to nearest
even); the GPU streams those 16-bit values and the oracle sees the same values
widened to FP64, so these tests measure only the arithmetic of the 16-bit path
(the storage rounding itself is the workload, not an error).

Tolerances follow from the arithmetic. The first contracted factor enters the
MFMA as a sum of values of the tensor's 16-bit type as exact as an FP32 value
(FP16 hi + lo, BF16 hi + mid + lo); products are exact in FP32 and summed in
FP32 over at most one i1 block per Khatri-Rao row group before the FP32
column-scaled accumulation. Each partial-MTTKRP entry is therefore within
2e-6 of sum |x||k| (a bound; typical errors are ~10x smaller). Whole
trajectories use the per-storage bounds of tests/tolerances.py.
"""

import numpy as np
import pytest

import oracle as O
from tolerances import TRAJ_TOL
from paper_1806_07985_amd import inputs

pytestmark = pytest.mark.gpu

DTYPES = ["bf16", "f16"]


def _torch_dtype(name):
    import torch
    return {"bf16": torch.bfloat16, "f16": torch.float16}[name]


def _quantized(X, name):
    """(device 16-bit tensor, FP64 host copy of the same values)."""
    import torch
    from paper_1806_07985_amd import native
    flat = torch.from_numpy(np.ascontiguousarray(np.asarray(X, dtype=np.float32).ravel(order="F")))
    q = flat.to(_torch_dtype(name))
    Xq = q.to(torch.float64).numpy().reshape(X.shape, order="F")
    return q.to("cuda"), Xq


PM_CASES = [
    ((60, 50, 40), 5, 2),
    ((60, 50, 40), 5, 1),
    ((33, 47, 29), 8, 1),        # ragged: masked loads on both sides
    ((64, 40, 24, 10), 32, 2),
    ((40, 36, 30), 50, 1),       # four column blocks, padded
    ((20, 18, 22), 100, 2),      # column chunks of 64
    ((1024, 300), 24, 1),
    ((128, 64, 33, 9), 50, 1),   # the hyperspectral shape family, small
    ((3012, 12, 10), 10, 1),     # the fMRI shape family: I_L % 8 == 4, ragged I1 (8-byte loads)
    ((300, 20, 10), 10, 2),      # I_L % 8 == 0 but I1 ragged: 8-byte loads on full k-steps
    ((60, 200, 200), 10, 1),     # tall right node with J == 1, masked form (I_L % 8 == 4, ragged I1)
    ((36, 300, 120), 24, 1),     # the same with two column blocks
    ((9, 8, 16), 6, 2),          # I_L % 8 == 0, odd I1 with J > 1: column offsets not 16-byte aligned
    ((7, 11, 13), 5, 1),         # every extent odd
]


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("dims,R,s", PM_CASES)
@pytest.mark.parametrize("side", [0, 1])
def test_partial_mttkrp_16bit(gpu_lib, dt, dims, R, s, side):
    from paper_1806_07985_amd import native
    print(f"case pm16 {dt} dims={dims} R={R} s={s} side={side}", flush=True)
    rng = np.random.default_rng(hash((dims, R, s)) % 1000)
    X = rng.random(dims).astype(np.float32)
    H = [rng.random((d, R)).astype(np.float32) for d in dims]
    Xd, Xq = _quantized(X, dt)
    Hd = [native.factor_to_device(h) for h in H]
    T = native.partial_mttkrp(Xd, list(dims), s, side, Hd, R).cpu().numpy().T
    H64 = [h.astype(np.float64) for h in H]
    fn = O.partial_mttkrp_left if side == 0 else O.partial_mttkrp_right
    ref = fn(Xq, H64, s).reshape(-1, R, order="F")
    bound = fn(np.abs(Xq), H64, s).reshape(-1, R, order="F")
    err = np.abs(T - ref)
    print(f"  max error / sum|x||k| {float(np.max(err / (bound + 1e-30))):.2e}", flush=True)
    assert np.all(err <= 2e-6 * bound + 1e-30), float(np.max(err / (bound + 1e-30)))


# Tall right nodes whose first mode does not fit one LDS block: the work-group
# walks the i1 blocks in turn (fast 16-byte path and the masked path).
@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("dims,R", [((1152, 70000), 40), ((1030, 66000), 20)])
def test_partial_mttkrp_16bit_staged_right(gpu_lib, dt, dims, R):
    from paper_1806_07985_amd import native
    print(f"case pm16 staged {dt} dims={dims} R={R}", flush=True)
    rng = np.random.default_rng(R)
    X = rng.random(dims, dtype=np.float32)
    H = [rng.random((d, R)).astype(np.float32) for d in dims]
    Xd, Xq = _quantized(X, dt)
    Hd = [native.factor_to_device(h) for h in H]
    T = native.partial_mttkrp(Xd, list(dims), 1, 1, Hd, R).cpu().numpy().T
    ref = Xq.T @ H[0].astype(np.float64)
    bound = np.abs(Xq).T @ H[0].astype(np.float64)
    assert np.all(np.abs(T - ref) <= 2e-6 * bound), float(np.max(np.abs(T - ref) / bound))
    # the left node of the same matrix (short output, split over K)
    T = native.partial_mttkrp(Xd, list(dims), 1, 0, Hd, R).cpu().numpy().T
    ref = Xq @ H[1].astype(np.float64)
    bound = np.abs(Xq) @ H[1].astype(np.float64)
    assert np.all(np.abs(T - ref) <= 2e-6 * bound), float(np.max(np.abs(T - ref) / bound))


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("dims,R,split,update,iters", [
    ((60, 50, 40), 5, 2, "hals", 20),
    ((20, 18, 16, 14), 8, 2, "hals", 15),
    ((20, 18, 16, 14), 8, 1, "mu", 15),
    ((12, 10, 9, 8, 7), 4, 3, "hals", 10),
])
def test_nncp_16bit_matches_oracle_on_stored_values(gpu_lib, dt, dims, R, split, update, iters):
    from paper_1806_07985_amd import native
    print(f"case nncp16 {dt} dims={dims} R={R} split={split} {update}", flush=True)
    X, _ = inputs.planted(dims, R, 0.01, seed=3, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=4)]
    Xd, Xq = _quantized(X, dt)
    Hd = [native.factor_to_device(h) for h in H0]
    out = native.nncp(Xd, list(dims), R, iters, Hd, update=update, split=split)
    ref = O.nncp(Xq, [h.astype(np.float64) for h in H0], iters, update=update)
    errs = [np.linalg.norm(native.factor_to_host(h) - r) / np.linalg.norm(r) for h, r in zip(Hd, ref["H"])]
    lam_err = float(np.max(np.abs(out["lam"] - ref["lam"]) / ref["lam"]))
    fit_err = float(np.max(np.abs(np.asarray(out["fit"]) - np.asarray(ref["fit"]))))
    print(f"  factor errs {['%.1e' % e for e in errs]} lam {lam_err:.1e} fit {fit_err:.1e}", flush=True)
    # per-storage bounds (tests/tolerances.py)
    tol = TRAJ_TOL[dt]
    assert max(errs) < tol and lam_err < tol and fit_err < tol


def test_quantized_fit_close_to_fp32_fit(gpu_lib):
    """Equal fit: the model found from the BF16-stored tensor, scored against the
    original FP32 tensor in FP64 (oracle), is within 1e-4 of the FP32 run's."""
    from paper_1806_07985_amd import native
    dims, R, iters = (48, 40, 36, 12), 8, 60
    X, _ = inputs.planted(dims, R, 0.02, seed=11, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=12)]
    X64 = X.astype(np.float64)
    fits = {}
    for dt in ["f32", "bf16", "f16"]:
        if dt == "f32":
            Xd = native.tensor_to_device(X)
        else:
            Xd, _ = _quantized(X, dt)
        Hd = [native.factor_to_device(h) for h in H0]
        out = native.nncp(Xd, list(dims), R, iters, Hd, split=2)
        H = [native.factor_to_host(h) for h in Hd]
        fits[dt] = 1.0 - O.relerr_explicit(X64, out["lam"], H)
    print(f"fit vs FP32 tensor: {fits}", flush=True)
    assert abs(fits["bf16"] - fits["f32"]) < 1e-4
    assert abs(fits["f16"] - fits["f32"]) < 1e-4


def test_bf16_rank64_full_lds_block_alone_and_batched(gpu_lib):
    """BF16 at rank 64 keeps three 64-column term rows per i1 in LDS; with a
    full 384-row i1 block and a long j range (one work-group per column tile,
    from a large per-group share of the tensor) the per-(j, column) scales are
    what is left of the CU's 160 KiB, so the j block is cut below 64. The plan
    still follows the oracle, and the same plan advanced in a batch (graph of
    kernel nodes sized for the largest LDS the variant can ask for) gives
    bitwise the same factors."""
    import torch
    from paper_1806_07985_amd import native
    dims, R, split, iters = (384, 1400, 16), 64, 2, 3
    print(f"case bf16 full lds block dims={dims} R={R}", flush=True)
    X, _ = inputs.planted(dims, R, 0.01, seed=61, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=62)]
    Xd, Xq = _quantized(X, "bf16")
    Ha = [native.factor_to_device(h) for h in H0]
    out = native.nncp(Xd, list(dims), R, iters, Ha, split=split, pm_wg_kib=1 << 14)
    ref = O.nncp(Xq, [h.astype(np.float64) for h in H0], iters)
    errs = [np.linalg.norm(native.factor_to_host(h) - r) / np.linalg.norm(r) for h, r in zip(Ha, ref["H"])]
    fit_err = float(np.max(np.abs(np.asarray(out["fit"]) - np.asarray(ref["fit"]))))
    print(f"  factor errs {['%.1e' % e for e in errs]} fit {fit_err:.1e}", flush=True)
    assert max(errs) < TRAJ_TOL["bf16"] and fit_err < TRAJ_TOL["bf16"]
    # the same plan alone (graph) and advanced by a batch: the unnormalised factors
    Hc = [native.factor_to_device(h) for h in H0]
    alone = native.Plan(Xd, list(dims), R, Hc, split=split, pm_wg_kib=1 << 14)
    alone.run(iters)
    Hb = [native.factor_to_device(h) for h in H0]
    plan = native.Plan(Xd, list(dims), R, Hb, split=split, pm_wg_kib=1 << 14, graph=False)
    batch = native.Batch()
    batch.add(plan)
    batch.run(iters)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(Hc, Hb))
    assert np.array_equal(alone.fits(), plan.fits())
    batch.close()
    plan.close()
    alone.close()
