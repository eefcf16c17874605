"""Seeded synthetic inputs for TDA-risp: geometry, AO shells, MO coefficients and energies.

This module produces the *inputs* of the method (what the paper's problem statement takes in:
geometry, AO and auxiliary radii, MO coefficients, orbital energies). It holds none of the method's
own arithmetic: no electron-repulsion integrals, no RI factors, no response matrix. The only integral
it evaluates is the AO overlap S, which the method never uses; it is needed to make the synthetic MO
coefficients orthonormal (C = S^-1/2 Q).

Both the FP64 oracle and the HIP path read these inputs; neither imports the other.
"""
from .molecule import (  # noqa: F401
    ANGSTROM_TO_BOHR, HARTREE_TO_EV, AO_EXPONENTS, COVALENT_RADIUS_ANGSTROM,
    Molecule, make_config0, make_chain_ring, make_system, config_system, random_trial_vectors,
)
