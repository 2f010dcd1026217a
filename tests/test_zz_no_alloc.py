"""The entry point that allocates nothing (nncp_norm_sq_noalloc) against the
allocating one (nncp_norm_sq), through the C ABI on the GPU.

Both run the same kernel with the same grid and summation order, so the bar is
bit equality; the FP64 sum of the same values on the host is checked as well
(the squares are exact in FP64, so only the summation order differs: 1e-12).
Two calls in a row, the second on a smaller input, show that the shared static
scratch (block partials, arrival counter) carries nothing from one call into
the next.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
def test_norm_sq_noalloc_matches_allocating_entry(gpu_lib, dt):
    import torch
    from paper_1806_07985_amd import native
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dt]
    g = torch.Generator().manual_seed(17)
    # first call: a large input (the full 1024-group grid), then a smaller ragged one
    # (fewer groups, n % 8 != 0, and an element-aligned but not 16-byte-aligned base)
    big = torch.rand(50_000_003, generator=g).to(tdt)
    small = torch.rand(123_457, generator=g).to(tdt)
    cases = [("big", big.to("cuda")), ("small", small.to("cuda")[1:])]
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for name, X in cases:
        print(f"case noalloc {dt} {name} n={X.numel()}", flush=True)
        native.norm_sq_noalloc(X, out)
        torch.cuda.synchronize()
        got = float(out.item())
        ref = native.norm_sq(X)
        host = float(np.sum(X.cpu().to(torch.float64).numpy() ** 2))
        print(f"  noalloc {got!r} alloc {ref!r} host {host!r}", flush=True)
        assert got == ref
        assert abs(got - host) <= 1e-12 * host


def test_norm_sq_noalloc_rejects_bad_arguments(gpu_lib):
    import ctypes
    from paper_1806_07985_amd import native
    L = native.lib()
    assert L.nncp_norm_sq_noalloc(None, 0, 10, None, None) == -1
    buf = ctypes.c_double(0.0)
    assert L.nncp_norm_sq_noalloc(ctypes.addressof(buf), 0, 0, ctypes.addressof(buf), None) == -1
    assert L.nncp_norm_sq_noalloc(ctypes.addressof(buf), 7, 10, ctypes.addressof(buf), None) == -1
