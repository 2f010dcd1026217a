"""Parity bounds of the GPU path against the FP64 oracle, per tensor storage.

Each bound is on the normwise relative error of every unit-column factor, the
relative error of lambda and the error of every recorded fit, over whole
trajectories (tens of outer iterations from the same start as the oracle, the
oracle running on the same stored tensor values), and over one iteration of
the full-size workloads.

All three storage types share one bound, 1e-5, the bound set for FP32 mode,
because the 16-bit path adds no rounding of its own beyond the tensor's
storage, which is the workload itself:

* "f32": products are exact FP32 MFMA products, partial sums are folded into
  FP64 before they reach ~0.2 ulp of error, the tree temporaries, the update
  and the Gram/fit arithmetic are FP64; the factors are stored in FP32.
* "f16" / "bf16": the first contracted factor enters the MFMA as a sum of
  16-bit values as exact as an FP32 value (FP16 hi + lo, 22 bits; BF16
  hi + mid + lo, 24 bits), products are exact in FP32, and the sums and tree
  temporaries are FP32 instead of FP64: an MTTKRP entry carries a relative
  error of a few 2^-24 times sqrt(terms) of sum |x||k| (~1e-7 to 1e-6).

The block updates then amplify these errors by the conditioning of the
subproblem S (high at R = 50 with overlapping components), and a trajectory
carries them on. Measured on MI355X: FP32 up to 3.5e-6 (128^4, 50 iterations),
FP16 up to 4.2e-6 and BF16 up to 5.6e-6 (the 1024x1344x33x9 R = 50 tensor,
lambda after one iteration). 1e-5 is below 2x the largest of these and 500x
below the BF16 storage rounding of the tensor itself (2^-9); with the two-term
BF16 split of earlier builds (16 bits, 2^-17 per entry) one iteration of the
same tensor was already 1.9e-5 off, which this bound rejects.
"""

TRAJ_TOL = {"f32": 1e-5, "f16": 1e-5, "bf16": 1e-5}
