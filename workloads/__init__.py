"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds no arithmetic of the simulation method: it only writes
circuit text in the project's IR and draws seeded random tensors.  Fault
sampling, pre-screening, MPS simulation and re-weighting live elsewhere.
"""
