"""CPU FP64 oracle of the learnable multigrid V-cycle and its adjoint.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and by
the benchmark's CPU-baseline leg.  The GPU product path never imports it, and
it shares no code with the GPU path.
"""
