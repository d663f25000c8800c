"""FP64 CPU oracle for the selected Green's-function solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or
links anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU path:
it is plain numpy/LAPACK in complex128, written from the paper's statement of
the problem (Eq. 2 with the G row of Table I, selected BT entries, Section II-A).

Two independent implementations of the same result:
  dense_selected  - the plain definition: assemble M(E), invert it densely,
                    form G^< = G^R Sigma^< G^R^H, keep the BT blocks.
  rgf_selected    - the block recurrences of recursive Green's functions
                    (block Gaussian elimination, Section IV-A), step by step.
Observables (transmission, contact and bond currents) live in observables.py;
the screened Coulomb (W) system of Table I in wsystem.py; the FPX storage
formats of Section V-A in fpx.py.

Parity is pinned (tests/test_oracle_*.py) by closed forms of a uniform chain
and a uniform strip, exact rational brute force on tiny systems, and the
structural invariants of lesser/greater/retarded functions.
"""
from .rgf_oracle import dense_selected, rgf_selected, assemble_dense, schur_complements, OUTPUT_KEYS  # noqa: F401
from .observables import transmission_left, contact_current_left, bond_currents, rel_fro_err  # noqa: F401
from .wsystem import w_assemble, w_selected, w_as_g_problem  # noqa: F401
from .fpx import fpx_round, fpx_encode, fpx_decode, fpx_codes, FPX_BITS  # noqa: F401
