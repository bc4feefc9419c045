"""CPU oracle of the mu-mode integrator -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct FP64 / complex128 numpy code written from
the paper (Caliari, Cassini, Einkemmer, Ostermann, Zivcovich, "A mu-mode
integrator for solving evolution equations in Kronecker form").  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
it.  The HIP library never calls it, and it shares no code with the library:
the only common module is ``synth`` (seeded input draws).

Tensors are numpy arrays indexed U[i_1, ..., i_d] (paper index order).

Modules
-------
mumode     mu-mode product (Definition 2.1), Tucker operator / integrator
           (equation dd-tensor), Kronecker-matrix cross-checks (Section 2).
operators  1-D finite-difference generators, exponentials of symmetric /
           Hermitian generators, Hermite functions and Gauss-Hermite
           quadrature (Section 3).
schemes    Strang-split Gross-Pitaevskii step, harmonic-oscillator Hermite
           step with time-dependent potential, monitors (mass, energy).

Parity status per function is listed in each module docstring.
"""
from . import mumode, operators, schemes  # noqa: F401
