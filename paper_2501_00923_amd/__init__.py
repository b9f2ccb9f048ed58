"""MI355X-native discrete-velocity BGK primal/adjoint solver and wall shape
sensitivity (Yuan & Wu, arXiv 2501.00923).

Submodules are imported lazily: ``inputs`` (seeded synthetic grids and
workloads) needs only numpy; ``dvm`` (the binding to the HIP library)
needs torch and the built ``libdvm.so``.
"""
__all__ = ["inputs", "dvm"]
