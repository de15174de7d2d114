"""CPU FP64 oracle for the density-fitted JK / generalized-Fock path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the paper's natural-orbital-functional method
computes in each orbital-optimisation iteration.  It exists to check the HIP
library against.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import it; the library never does, and the
two share no code (the oracle reads no header, kernel, table or helper of the
HIP path).

Citations name the paper's sections and equations (DoNOF 2.0, arXiv
2512.13550).  Every function is written from the mathematics, in the paper's
notation, with library primitives (matmul, expm, eigh) as its only building
blocks.

Pin status (what each function is checked against, in tests/test_oracle_*.py):
  dfjk.mo_transform / jk      pinned: explicit four-index ERIs, invariants
  dfjk.energy                 pinned: spin-orbital 2RDM brute force, closed-shell HF
  dfjk.gen_fock               pinned: finite-difference orbital gradient,
                              textbook AO closed-shell Fock matrix
  functionals (pnof5, pnof7)  parity unpinned as functionals (their formulas are
                              cited out of the paper); the Delta/Pi -> cJ/cK
                              mapping they feed is pinned by the 2RDM brute force;
                              PNOF7 also: equal to PNOF5 for one subspace and for
                              0/1 occupations, exact interpair energy drop, finite
                              differences of dE/dn
  occupations.*               pinned: sum rule, bounds, finite differences
  rotation.*                  pinned: orthogonality, closed forms; the orthonormality
                              check written out as a double loop, the closed-form
                              error -3/4 E^2 + 1/4 E^3 left by one repair step
  mlp.*                       pinned: finite differences, hand-checked tiny net
  nlop.*                      pinned: exact on polynomial dipoles, analytic
                              derivatives of a smooth dipole, hand-made
                              selection cases, Hellmann-Feynman (dipole equals
                              minus the field derivative of SCF energies), the
                              stencil weights and Romberg denominators the paper
                              prints (tests/golden/nlop_formulas.json)
  solver.solve                pinned: closed-shell HF minimum equal to a DIIS
                              Roothaan SCF; stationarity (lambda symmetric, ON
                              gradient zero) and variational checks at the end;
                              the orbitals stay orthonormal over the run
"""
