"""MI355X-native parallel Riccati Newton-step (KKT) solver.

The solver itself is the HIP library behind ``include/rs.h``; ``rs`` is its
Python binding and ``workloads`` draws the seeded synthetic problems.
"""
__all__ = ["rs", "workloads", "build"]
