"""CPU oracle for the batched exact-MPS cultivation-shot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes anything here; only the tests, the graft entry's smoke check and the
bench's CPU-baseline leg do.  The oracle shares no code with the library: it
has its own IR parser, its own fault sampler twin, a dense state vector, a
plain FP64 MPS (LAPACK SVD), a symbolic-sign stabiliser pre-screen and the
subset-sampling estimators, each written from the paper:

- ``ir``           circuit text -> op list (the project's own IR format)
- ``sampler``      subset-sampling fault draws (Section 4.1), SplitMix64
- ``statevector``  dense complex128 simulation of one shot (Sections 3.1, 4)
- ``mps``          FP64 MPS, exact up to 1e-12 sigma_0 (Section 3.1; Section
                   5.1 "exact regime")
- ``prescreen``    stabiliser-propagation offline screening (Section 4.2)
- ``estimators``   Eq. (reweight), Eq. (estimators), the truncation bound B
                   (Appendix "Systematics") and the loss multiplier
                   (Appendix "Losses")

Every function names the passage it follows.  Functions whose result no
paper value, closed form, invariant or brute force pins are marked
"parity unpinned" in their docstring.
"""
