"""MI355X-native electromagnetic particle-in-cell time step (gfx950, HIP).

The compute path is the C-ABI library ``libpic355.so`` built from ``csrc/``;
``_lib`` is a thin ctypes binding with the same entry-point names, and
``rollout`` wraps forward and adjoint steps in a ``torch.autograd.Function``.
Importing this package loads nothing; the library is loaded on first use and
an error is raised if it is missing.
"""
__all__ = ["workloads", "lib", "rollout"]
