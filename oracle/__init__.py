"""FP64 CPU oracle of the OK-action operator M and its BiCGStab solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library; the
only common module is the seeded input generator ``paper_1311_5029_amd.inputs``,
which holds none of the operator's arithmetic.

Modules
-------
basis      Pauli and Dirac matrices (the W basis), gamma5 conjugation Gamma(X).
lattice    periodic shifts, colour and spin multiplication on NumPy fields.
clover     clover field strength F_{mu nu}, chromo-magnetic B_i, electric E_i.
route_b    M applied term by term from the links (operator composition).
route_a    the precalculation matrices W as printed in the paper, the 27-term
           apply (Eq. minFlopForm) and the 14-block shifted apply (Eq. FinalForm).
free       free-field symbol, plane-wave eigenvalues, FFT point-source solutions.
dense      dense assembly of M on tiny lattices.
bicgstab   plain FP64 BiCGStab (van der Vorst) on any operator.
net        the gauge-covariant linear stencil network: forward, adjoint, gradients.

Every function is vectorised over sites with NumPy; no blocking, fusion or
reordering beyond the definitions it cites.

Parity unpinned (no independent check exists): the physical values of the
stand-in coefficient set, and the overall sign/normalisation of F relative to
the conventions of the OK action's original definition (only its relation to
the textbook Wilson-clover term is pinned).
"""
