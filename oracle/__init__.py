"""FP64 CPU oracle for nonnegative CP decomposition (test infrastructure).

This package is the checker, not the product. Only the test suite, the
smoke check and the benchmark's CPU-baseline leg import it; the GPU library
and its Python binding never do, and they share no code with it.

Everything here is plain NumPy in float64, written from the paper
(Ballard, Hayashi, Kannan: Parallel Nonnegative CP Decomposition of Dense
Tensors), one function per step, each citing the passage it follows.
"""

from .nncp_oracle import *  # noqa: F401,F403
from .nncp_oracle import __all__  # noqa: F401
