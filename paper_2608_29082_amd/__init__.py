"""Learnable graph-convolution multigrid V-cycle on AMD Instinct MI355X.

The numerical work runs in the HIP library libmgl.so (C ABI in
include/mgl.h); this package holds its build step, its Python binding, the
autograd wrapper used for training and the request loop used for serving.
"""
__all__ = ["binding", "autograd", "serve", "build"]
