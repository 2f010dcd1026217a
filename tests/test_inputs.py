"""The slab-wise device generator (CPU run): mode order, the closed-form
||X_c||, the noise level, and the storage rounding."""

import numpy as np
import pytest

import oracle as O
from paper_1806_07985_amd import inputs


def _factors(dims, R, seed):
    import torch
    g = torch.Generator()
    g.manual_seed(seed)
    return [torch.rand((d, R), generator=g, dtype=torch.float32).double().numpy() for d in dims]


@pytest.mark.parametrize("dims,slab", [((5, 4, 6), 160), ((3, 4, 2, 5), 100), ((7, 9), 1 << 20)])
def test_noise_free_slabs_are_the_cp_model(dims, slab):
    R = 3
    X = inputs.planted_device_slabs(dims, R, 0.0, seed=5, dtype="f32", device="cpu", slab_bytes=slab)
    Xn = X.double().numpy().reshape(dims, order="F")
    model = O.model_tensor_cp(np.ones(R), _factors(dims, R, 5))
    np.testing.assert_allclose(Xn, model, rtol=2e-6, atol=1e-6)


def test_noise_level_and_bf16_rounding():
    import torch
    dims, R = (30, 20, 24), 4
    X = inputs.planted_device_slabs(dims, R, 0.05, seed=6, dtype="f32", device="cpu", slab_bytes=30 * 20 * 4 * 5)
    model = O.model_tensor_cp(np.ones(R), _factors(dims, R, 6)).ravel(order="F")
    x = X.double().numpy()
    rel = np.linalg.norm(x - model) / np.linalg.norm(model)
    assert abs(rel - 0.05) < 2e-3  # the clamp at zero never bites: the model is far above the noise
    Xb = inputs.planted_device_slabs(dims, R, 0.05, seed=6, dtype="bf16", device="cpu", slab_bytes=30 * 20 * 4 * 5)
    assert Xb.dtype == torch.bfloat16
    assert torch.equal(Xb, X.to(torch.bfloat16))
