"""Dimension trees of every shape on the GPU (Section IV-A allows any binary
tree over contiguous mode ranges; option tree_peel picks, per internal node of
three or more modes, {a} | {a+1..b} or {a..b-1} | {b}).

Every tree computes the direct MTTKRP exactly (in exact arithmetic), so every
shape must follow the oracle's trajectory at the FP32-mode bound; a tree also
behaves the same alone and in a batch, and the autotuner times every shape.
"""

import numpy as np
import pytest

import oracle as O
from paper_1806_07985_amd import inputs

pytestmark = pytest.mark.gpu


def _shapes(a, b, m, out):
    """Every internal-split mask of the node {a..b} (peel-first before peel-last)."""
    if b - a < 2:
        out.append(m)
        return
    _shapes(a + 1, b, m, out)
    _shapes(a, b - 1, m | (1 << (a * 8 + b)), out)


def _trees(N):
    out = []
    for s in range(1, N):
        left, right = [], []
        _shapes(0, s - 1, 0, left)
        _shapes(s, N - 1, 0, right)
        out += [(s, l | r) for l in left for r in right]
    return out


@pytest.mark.parametrize("dims,R", [((8, 7, 6, 5, 4), 6), ((6, 5, 4, 7), 5), ((5, 4, 3, 3, 4, 3), 3)])
def test_every_tree_matches_oracle(gpu_lib, dims, R):
    from paper_1806_07985_amd import native
    X, _ = inputs.planted(dims, R, 0.01, seed=31, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=32)]
    iters = 6
    ref = O.nncp(X.astype(np.float64), [h.astype(np.float64) for h in H0], iters)
    Xd = native.tensor_to_device(X)
    trees = _trees(len(dims))
    print(f"case trees {dims}: {len(trees)} trees", flush=True)
    for s, peel in trees:
        Hd = [native.factor_to_device(h) for h in H0]
        out = native.nncp(Xd, list(dims), R, iters, Hd, split=s, peel=peel)
        errs = [np.linalg.norm(native.factor_to_host(h) - r) / np.linalg.norm(r) for h, r in zip(Hd, ref["H"])]
        fit_err = float(np.max(np.abs(np.asarray(out["fit"]) - np.asarray(ref["fit"]))))
        lam_err = float(np.max(np.abs(out["lam"] - ref["lam"]) / np.max(ref["lam"])))
        print(f"  split {s} peel {peel:#x}: factors {max(errs):.1e} lam {lam_err:.1e} fit {fit_err:.1e}", flush=True)
        assert max(errs) <= 1e-5 and lam_err <= 1e-5 and fit_err <= 1e-5


def test_tree_shapes_in_a_batch_equal_alone(gpu_lib):
    """Plans of different tree shapes (and one without the tree) advanced in one
    batch give bitwise the factors of the same plans run alone."""
    import torch
    from paper_1806_07985_amd import native
    dims, R = (10, 9, 8, 7, 6), 8
    X, _ = inputs.planted(dims, R, 0.01, seed=41, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=42)]
    Xd = native.tensor_to_device(X)
    configs = [dict(split=2, peel=0), dict(split=2, peel=1 << (2 * 8 + 4)), dict(split=1, peel=1 << (1 * 8 + 4)),
               dict(split=3, peel=1 << (0 * 8 + 2)), dict(split=2, no_tree=True)]
    iters = 5
    alone, mixed = [], []
    for c in configs:
        Ha = [native.factor_to_device(h) for h in H0]
        pa = native.Plan(Xd, list(dims), R, Ha, **c)
        pa.run(iters)
        alone.append((pa, Ha))
        Hb = [native.factor_to_device(h) for h in H0]
        mixed.append((native.Plan(Xd, list(dims), R, Hb, graph=False, **c), Hb))
    batch = native.Batch()
    for p_, _ in mixed:
        batch.add(p_)
    batch.run(iters)
    torch.cuda.synchronize()
    for c, (pa, Ha), (pb, Hb) in zip(configs, alone, mixed):
        same = all(torch.equal(x, y) for x, y in zip(Ha, Hb))
        print(f"case batch tree {c}: equal alone {same}", flush=True)
        assert same
        assert np.array_equal(pa.fits(), pb.fits())
    batch.close()
    for p_, _ in alone + mixed:
        p_.close()


def test_autotune_tree_times_every_shape(gpu_lib):
    from paper_1806_07985_amd import native
    dims, R = (12, 11, 10, 9, 8), 8
    X, _ = inputs.planted(dims, R, 0.01, seed=51, dtype=np.float32)
    H0 = [h.astype(np.float32) for h in inputs.init_factors(dims, R, seed=52)]
    Xd = native.tensor_to_device(X)
    Hd = [native.factor_to_device(h) for h in H0]
    s, peel, rows = native.autotune_tree(Xd, list(dims), R, Hd, reps=2)
    trees = _trees(len(dims))
    print(f"case autotune: best split {s} peel {peel:#x} of {len(rows)}", flush=True)
    assert [(r[0], r[1]) for r in rows] == trees
    assert all(r[2] > 0 for r in rows)
    assert (s, peel) in trees and min(r[2] for r in rows) == [r[2] for r in rows if (r[0], r[1]) == (s, peel)][0]
