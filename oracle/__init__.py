"""Plain FP64 CPU oracle for TDA-risp (test infrastructure only).

This package is the checker of the HIP path, not part of it. Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library and its Python binding never do.
It shares no code with the HIP path: the two meet only in the seeded inputs made by ``synth``.

Everything here is NumPy/SciPy in float64, written for a reader to check against the paper by eye:

* ``integrals``: McMurchie-Davidson Hermite-Gaussian 2- and 3-centre integrals over primitive
  Cartesian Gaussians for the Coulomb operator 1/r and the attenuated operator erf(w r)/r (the latter
  enters the range-separated exchange operator of the section on exchange-space truncation), the
  Boys function from the regularised incomplete gamma function, and the diagonal 4-centre integrals
  used by Schwarz screening. Deliberately a different algorithm from the Obara-Saika kernels.
* ``risp``: auxiliary-basis selection, the energy window, shell-pair screening, the RI factors
  through a Cholesky split of the metric, the dense TDA-risp matrix A (eq. TDA-risp), its matrix-free
  product sigma = A X, a block Davidson solver and the dense eigensolver.

Pins: every function is checked in the CPU test suite against quantities fixed by mathematics
(closed forms, numerical quadrature, brute-force 4-index sums, invariants); see the oracle tests.
The absolute excitation energies of the paper's molecules are parity unpinned: the paper prints no
small worked example, and its benchmark molecules and orbitals are not available.
"""
