"""FP64 CPU oracle for motion-focus recognition (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the HIP path
is checked against.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg import it; the product library never does, and it shares no
code with the HIP kernels or the C ABI.  Everything runs in NumPy float64.

Contents
  vit     -- the multi-view ViT forward that regresses per-frame camera pose
             (the foundation-model stage of Sec. 2.2; sizes from the workloads)
  motion  -- sliding-window schedule and incremental anchoring (Sec. 2.2),
             camera centres, discrete acceleration and the focus projection
             (Sec. 2.3, Eq. 1-6), and the Gaussian motion-focus map (Eq. 7)
  pipeline-- the whole stream: windows -> forward -> chaining -> focus -> map

Parity status: every function below is pinned by the CPU tests in
tests/test_oracle_*.py (brute force, closed forms, invariants and library
routines).  The composition of the network as a whole has no external pin
(no trained weights, no printed values): "parity unpinned" beyond its
individually pinned parts.
"""
from . import vit, motion, pipeline  # noqa: F401
