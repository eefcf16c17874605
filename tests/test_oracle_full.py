"""Pins of the full TDDFT-risp oracle (oracle/full.py): A and B against a brute-force 4-index
assembly, the eigenpairs against the non-Hermitian form of eq. tddft, the matrix-free products
against the dense ones, and the exchange-free and TDA limits."""
import numpy as np
import pytest

from oracle import full as FU
from oracle import integrals as I
from oracle import risp as R
from tests.test_oracle_risp import tiny_molecule


@pytest.fixture(scope="module")
def tiny():
    return tiny_molecule()


def brute_AB(mol, prm):
    """A and B element by element from explicit 4-index RI integrals ((P|Q)^-1 by inversion)."""
    auxJ, auxK = R.select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    C = mol.mo_coeff
    o = mol.nocc
    v = C.shape[1] - o
    e = mol.mo_energy
    V3 = I.int3c(mol.coords, mol.shells, auxJ)
    ao4 = np.einsum("mnP,PQ,klQ->mnkl", V3, np.linalg.inv(I.int2c(mol.coords, auxJ)), V3, optimize=True)
    mo4 = np.einsum("mnkl,mp,nq,kr,ls->pqrs", ao4, C, C, C, C, optimize=True)
    V3x = prm.c_x * I.int3c(mol.coords, mol.shells, auxK) + prm.beta * I.int3c(mol.coords, mol.shells, auxK, prm.omega)
    V2x = prm.c_x * I.int2c(mol.coords, auxK) + prm.beta * I.int2c(mol.coords, auxK, prm.omega)
    ao4x = np.einsum("mnP,PQ,klQ->mnkl", V3x, np.linalg.inv(V2x), V3x, optimize=True)
    mo4x = np.einsum("mnkl,mp,nq,kr,ls->pqrs", ao4x, C, C, C, C, optimize=True)
    occK, virK = R.window_sets(e, o, prm.window_ev, prm.window_mode)
    occK, virK = set(occK.tolist()), set(virK.tolist())
    A = np.zeros((o * v, o * v))
    B = np.zeros((o * v, o * v))
    for i in range(o):
        for a in range(v):
            for j in range(o):
                for b in range(v):
                    ca = 2.0 * mo4[i, o + a, j, o + b]
                    A[i * v + a, j * v + b] = ca + ((e[o + a] - e[i]) if (i == j and a == b) else 0.0)
                    B[i * v + a, j * v + b] = ca
                    if i in occK and j in occK and a in virK and b in virK:
                        A[i * v + a, j * v + b] -= mo4x[i, j, o + a, o + b]
                        B[i * v + a, j * v + b] -= mo4x[i, o + b, j, o + a]
    return A, B


@pytest.mark.parametrize("window", [40.0, 25.0])
def test_A_and_B_match_brute_force(tiny, window):
    prm = R.Params(window_ev=window, schwarz_tau=0.0)
    F = R.build_factors(tiny, prm)
    X = FU.exchange_ia_factor(tiny, prm)
    Ab, Bb = brute_AB(tiny, prm)
    ApB, AmB = FU.dense_ApB_AmB(F, X)
    assert np.abs(0.5 * (ApB + AmB) - Ab).max() <= 1e-12 * np.abs(Ab).max()
    # the same absolute bar as A (B's elements are 2 orders smaller than A's diagonal; the brute force
    # inverts the metrics explicitly)
    assert np.abs(0.5 * (ApB - AmB) - Bb).max() <= 1e-12 * np.abs(Ab).max()
    assert np.abs(Bb - Bb.T).max() <= 1e-12 * np.abs(Ab).max()  # B symmetric (real orbitals), as A
    if window == 25.0:
        assert len(F.virK) < F.nvir


def test_eigenpairs_match_eq_tddft_non_hermitian(tiny):
    prm = R.Params(schwarz_tau=0.0)
    F = R.build_factors(tiny, prm)
    ApB, AmB = FU.dense_ApB_AmB(F, FU.exchange_ia_factor(tiny, prm))
    assert np.linalg.eigvalsh(AmB).min() > 0.0  # stable ground state on these inputs
    n = 6
    om, XpY, XmY = FU.full_eigh(ApB, AmB, n)
    A, B = 0.5 * (ApB + AmB), 0.5 * (ApB - AmB)
    # [[A, B], [-B, -A]] [X; Y] = Omega [X; Y]: eigenvalues in +-Omega pairs
    big = np.block([[A, B], [-B, -A]])
    w = np.linalg.eigvals(big)
    pos = np.sort(w.real[w.real > 0])[:n]
    assert np.abs(w.imag).max() < 1e-9
    assert np.abs(pos - om).max() <= 1e-10 * om.max()
    # the pair equations and the normalisation
    for k in range(n):
        assert np.abs(ApB @ XpY[k] - om[k] * XmY[k]).max() <= 1e-10
        assert np.abs(AmB @ XmY[k] - om[k] * XpY[k]).max() <= 1e-10
        assert abs(XpY[k] @ XmY[k] - 1.0) <= 1e-12
        X, Y = 0.5 * (XpY[k] + XmY[k]), 0.5 * (XpY[k] - XmY[k])
        assert abs(X @ X - Y @ Y - 1.0) <= 1e-12  # the symplectic norm of eq. tddft


def test_full_energies_below_tda_and_exchange_free_limit(tiny):
    prm = R.Params(schwarz_tau=0.0)
    F = R.build_factors(tiny, prm)
    ApB, AmB = FU.dense_ApB_AmB(F, FU.exchange_ia_factor(tiny, prm))
    om, _, _ = FU.full_eigh(ApB, AmB, 8)
    tda = np.linalg.eigvalsh(R.dense_A(F))[:8]
    assert np.all(om <= tda + 1e-12)  # full TDDFT lies below TDA state by state on these inputs
    # no exchange: A - B is the diagonal of orbital gaps and the factor is empty
    p0 = R.Params(schwarz_tau=0.0, c_x=0.0, beta=0.0)
    F0 = R.build_factors(tiny, p0)
    X0 = FU.exchange_ia_factor(tiny, p0)
    assert X0.shape[0] == 0
    _, AmB0 = FU.dense_ApB_AmB(F0, X0)
    assert np.abs(AmB0 - np.diag(F0.de.ravel())).max() <= 1e-15 * np.abs(F0.de).max()


def test_matrix_free_products_match_dense(tiny):
    prm = R.Params(window_ev=25.0, schwarz_tau=0.0)
    F = R.build_factors(tiny, prm)
    Xf = FU.exchange_ia_factor(tiny, prm)
    ApB, AmB = FU.dense_ApB_AmB(F, Xf)
    rng = np.random.default_rng(3)
    V = rng.normal(size=(4, F.nocc, F.nvir))
    P, M = FU.sigma_pm(F, Xf, V)
    Vf = V.reshape(4, -1)
    assert np.abs(P.reshape(4, -1) - Vf @ ApB.T).max() <= 1e-12 * np.abs(P).max()
    assert np.abs(M.reshape(4, -1) - Vf @ AmB.T).max() <= 1e-12 * np.abs(M).max()
