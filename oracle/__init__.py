"""FP64 CPU oracle for the SI-CTMRG move -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow reference that the GPU path is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it; the product library never does, and it
shares no code with the HIP path (the two meet only through the seeded inputs
of the ``synth`` module).

Every function cites the passage of Zhang & Corboz, "Fast two-dimensional
tensor-network contraction via subspace iteration", that it follows.  The
paper's equations are tensor diagrams; the matrix reading used here (index
order, which bond each enlarged-corner product is open at, sign and cutoff
rules) is written out in the module docstring of :mod:`oracle.ctmrg`.

The reverse-mode reference of one move (:mod:`oracle.adjoint`, PyTorch CPU
autograd in float64) is imported explicitly; it is pinned to central finite
differences of the NumPy move.

Parity status: every function is pinned by ``tests/test_oracle_*.py``
(Onsager/Yang closed forms, exact product states, Eckart-Young, k = N
reduction of subspace iteration to the SVD, gauge and rotation invariances,
brute-force network values).
"""
from .ctmrg import *  # noqa: F401,F403
