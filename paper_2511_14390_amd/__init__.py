"""Differentiable direct-form IIR filtering on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libfilt.so`` built from the HIP
sources in ``csrc/`` (``build.py``); this package only marshals arguments to it
(:mod:`.filt`) and wraps it in a ``torch.autograd.Function``
(:mod:`.autograd`).  Importing the package does not load the library;
the first call does, and fails loudly if it has not been built.
"""
__all__ = ["filt", "autograd", "workloads"]
