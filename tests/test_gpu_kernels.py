"""Per-step parity of the HIP kernels against the FP64 oracle (GPU).

Inputs are seeded and synthetic; the oracle sees exactly the values the GPU
sees (the FP32 tensor and FP32 factors, widened to FP64). Tolerances follow
from the arithmetic: FP32 MFMA products summed in FP32 for 16 or 32 terms and
then in FP64, so each MTTKRP entry is off by a few units of 2^-24 relative to
sum |x k|; multi-TTV, Gram and update arithmetic are FP64.
"""

import math

import numpy as np
import pytest

import oracle as O
from paper_1806_07985_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(gpu_lib):
    import torch
    return torch.device("cuda:0")


def _setup(dims, R, seed, signed=False):
    rng = np.random.default_rng(seed)
    X = rng.random(dims).astype(np.float32)
    if signed:
        X = (X - 0.5).astype(np.float32)
    H = [rng.random((d, R)).astype(np.float32) for d in dims]
    return X, H


def _to_gpu(X, H):
    from paper_1806_07985_amd import native
    Xd = native.tensor_to_device(X)
    Hd = [native.factor_to_device(h) for h in H]
    return Xd, Hd


def _absbound(Xabs, Habs, fn, *args):
    """sum |x| |k| computed by the oracle on absolute values (error scale)."""
    return fn(Xabs, Habs, *args)


PM_CASES = [
    ((60, 50, 40), 5, 2),        # C1 shape, both sides
    ((60, 50, 40), 5, 1),
    ((33, 47, 29), 8, 1),        # ragged: I_L not a multiple of 4 (scalar loads)
    ((33, 47, 29), 16, 2),
    ((64, 40, 24, 10), 32, 2),   # two 16-column blocks
    ((40, 36, 30), 50, 1),       # four column blocks with padding
    ((24, 20, 18, 6), 64, 2),
    ((20, 18, 22), 100, 2),      # more than 64 columns: column chunks
    ((7, 3), 3, 1),              # tiny matrix
    ((1024, 300), 24, 1),        # long reduction, many splits
    ((64, 1040, 8), 32, 1),      # left: three i1 blocks (352, 352, 336 rows) with FP32 chains of 2 steps;
                                 # the short last block has an odd step count (chains must end with each j)
    # FP32 right node staged through LDS (first mode a multiple of 64, long output):
    ((64, 5, 8200), 20, 2),      # two M tiles per group, ragged last tile, j rotation
    ((128, 3, 4500), 50, 2),     # four column blocks (one 16-column group per wave), three tiles per group
    ((64, 64, 9000), 32, 2),     # split K over three j blocks (FP64 partials)
    ((128, 2, 8300), 12, 1),     # one column block, J = 1, five tiles per group
]


@pytest.mark.parametrize("dims,R,s", PM_CASES)
@pytest.mark.parametrize("side", [0, 1])
def test_partial_mttkrp_matches_oracle(gpu_lib, dims, R, s, side):
    from paper_1806_07985_amd import native
    print(f"case pm dims={dims} R={R} s={s} side={side}", flush=True)
    X, H = _setup(dims, R, seed=hash((dims, R, s)) % 1000)
    Xd, Hd = _to_gpu(X, H)
    T = native.partial_mttkrp(Xd, list(dims), s, side, Hd, R).cpu().numpy().T
    X64 = X.astype(np.float64)
    H64 = [h.astype(np.float64) for h in H]
    fn = O.partial_mttkrp_left if side == 0 else O.partial_mttkrp_right
    ref = fn(X64, H64, s)
    ref = ref.reshape(-1, R, order="F")
    bound = fn(np.abs(X64), [np.abs(h) for h in H64], s).reshape(-1, R, order="F")
    err = np.abs(T - ref)
    assert T.shape == ref.shape
    # FP32 products, FP64 sums after every 16-32 terms: well below 1e-6 of sum |x k|
    assert np.all(err <= 1e-6 * bound + 1e-30), float(np.max(err / (bound + 1e-30)))


def test_partial_mttkrp_signed_data(gpu_lib):
    from paper_1806_07985_amd import native
    dims, R, s = (48, 36, 20), 16, 1
    X, H = _setup(dims, R, seed=5, signed=True)
    Xd, Hd = _to_gpu(X, H)
    for side in (0, 1):
        T = native.partial_mttkrp(Xd, list(dims), s, side, Hd, R).cpu().numpy().T
        fn = O.partial_mttkrp_left if side == 0 else O.partial_mttkrp_right
        ref = fn(X.astype(np.float64), [h.astype(np.float64) for h in H], s).reshape(-1, R, order="F")
        bound = fn(np.abs(X.astype(np.float64)), [h.astype(np.float64) for h in H], s).reshape(-1, R, order="F")
        assert np.all(np.abs(T - ref) <= 1e-6 * bound)


@pytest.mark.parametrize("node_dims,R", [((30, 20, 10), 8), ((128, 128), 32), ((33, 9), 50), ((7, 5, 3, 2), 5),
                                         ((100, 1300), 16)])
def test_mttv_matches_oracle(gpu_lib, node_dims, R):
    import torch
    from paper_1806_07985_amd import native
    rng = np.random.default_rng(len(node_dims) * 100 + R)
    T = rng.random(tuple(node_dims) + (R,))
    Hs = [rng.random((d, R)).astype(np.float32) for d in node_dims]
    Td = native.tensor_to_device(T)
    # trailing: contract modes 2.. with their factors
    out = native.mttv(Td, list(node_dims), 0, [native.factor_to_device(h) for h in Hs[1:]], R)
    ref = O.mttv_trail(T, [h.astype(np.float64) for h in Hs[1:]])
    got = out.cpu().numpy().T
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    # leading: contract mode 1
    out = native.mttv(Td, list(node_dims), 1, [native.factor_to_device(Hs[0])], R)
    ref = O.mttv_lead(T, Hs[0].astype(np.float64)).reshape(-1, R, order="F")
    got = out.cpu().numpy().T
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("dims,R", [((12, 10, 8), 4), ((9, 8, 7, 6), 8), ((6, 5, 4, 3, 5), 3), ((40, 30), 6)])
def test_tree_mttkrp_every_mode_and_split_matches_direct(gpu_lib, dims, R):
    from paper_1806_07985_amd import native
    X, H = _setup(dims, R, seed=len(dims) * 7 + R)
    Xd, Hd = _to_gpu(X, H)
    X64 = X.astype(np.float64)
    H64 = [h.astype(np.float64) for h in H]
    for s in range(1, len(dims)):
        for n in range(len(dims)):
            print(f"case tree dims={dims} R={R} s={s} n={n}", flush=True)
            M = native.mttkrp(Xd, list(dims), s, n, Hd, R).cpu().numpy().T
            ref = O.mttkrp_direct(X64, H64, n)
            np.testing.assert_allclose(M, ref, rtol=5e-7)


@pytest.mark.parametrize("I,R", [(1, 1), (37, 5), (128, 32), (1344, 50), (300, 64), (90, 100),
                                 (5000, 16), (2000, 40), (700, 45), (1030, 33)])
def test_gram_matches_oracle(gpu_lib, I, R):
    """Single and several row chunks, one, two and four R x R entries per thread."""
    from paper_1806_07985_amd import native
    rng = np.random.default_rng(I + R)
    H = rng.random((I, R)).astype(np.float32)
    G = native.gram(native.factor_to_device(H), I, R).cpu().numpy()
    np.testing.assert_allclose(G, O.gram(H.astype(np.float64)), rtol=1e-13)


@pytest.mark.parametrize("update", ["hals", "mu"])
@pytest.mark.parametrize("I,R", [(50, 5), (128, 32), (333, 50), (64, 64), (40, 100)])
def test_nls_update_matches_oracle(gpu_lib, update, I, R):
    import torch
    from paper_1806_07985_amd import native
    rng = np.random.default_rng(I * 3 + R)
    K = rng.random((4 * R + 10, R))
    S = K.T @ K
    S = S / np.sqrt(np.outer(np.diag(S), np.diag(S)))  # unit diagonal, like normalised factors
    A = rng.random((I, 4 * R + 10))
    M = A @ K / np.sqrt(np.diag(K.T @ K))
    Hn = rng.random((I, R)).astype(np.float32)
    lam = rng.random(R) + 0.5
    dev = torch.device("cuda:0")
    Hd = native.factor_to_device(Hn)
    Md = torch.from_numpy(np.ascontiguousarray(M.T)).to(dev)
    lam_t, G = native.nls_update(Md, Hd, I, R, torch.from_numpy(S).to(dev),
                                 torch.from_numpy(lam).to(dev), update)
    upd = O.hals_update if update == "hals" else O.mu_update
    W = upd(Hn.astype(np.float64) * lam[None, :], S, M)
    Href, lref = O.normalize_columns(W)
    got = native.factor_to_host(Hd)
    assert np.linalg.norm(got - Href) <= 1e-6 * np.linalg.norm(Href)
    np.testing.assert_allclose(lam_t.cpu().numpy(), lref, rtol=1e-6)
    np.testing.assert_allclose(G.cpu().numpy(), O.gram(Href), rtol=1e-6, atol=1e-7)


def test_norm_sq_and_quantize(gpu_lib):
    import torch
    from paper_1806_07985_amd import native
    rng = np.random.default_rng(3)
    x = (rng.random(1_000_003) * 3).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    assert abs(native.norm_sq(xd) - float(np.sum(x.astype(np.float64) ** 2))) <= 1e-12 * np.sum(x.astype(np.float64) ** 2)
    qb = native.quantize(xd, "bf16")
    ref_b = torch.from_numpy(x).to(torch.bfloat16)  # CPU rounding: nearest even
    assert torch.equal(qb.cpu().view(torch.int16), ref_b.view(torch.int16))
    qh = native.quantize(xd, "f16")
    ref_h = torch.from_numpy(x.astype(np.float16))
    assert torch.equal(qh.cpu().view(torch.int16), ref_h.view(torch.int16))
    # alpha of the stored low-precision tensor
    a = native.norm_sq(qb)
    ref = float(np.sum(ref_b.float().numpy().astype(np.float64) ** 2))
    assert abs(a - ref) <= 1e-12 * ref
