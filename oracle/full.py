"""Full TDDFT-risp (A and B) in plain FP64 (oracle; test infrastructure only).

The symplectic problem of eq. tddft with the matrices of eq. hessian, XC kernel dropped and the
integrals approximated as in TDA-risp (eq. TDDFT-axs_approx_integral, minimal auxiliary basis,
range-separated exchange operator J^ in its own metric, 40 eV exchange window):

  A_{ia,jb} = (e_a - e_i) d_ij d_ab + 2 (ia|jb) - [window] (ij|J^|ab)     (eq. TDA-risp)
  B_{ia,jb} =                         2 (ia|jb) - [window] (ib|J^|ja)
  (A + B) = de + 4 (ia|jb) - [window] ((ij|J^|ab) + (ib|J^|ja))
  (A - B) = de              - [window] ((ij|J^|ab) - (ib|J^|ja))

Reading: the Coulomb part of A + B is 4 (ia|jb) (2 from A, 2 from B), so that A and B are those
of eq. TDA-risp and of the closed-shell singlet; the printed eq. hessian shows 2 (ia|jb), which
contradicts eq. TDA-risp. [window] keeps i, j in occK' and a, b in virK' as for A.

RI: (ia|jb) = sum_P B^P_ia B^P_jb (the Coulomb factor of oracle.risp) and
(ib|J^|ja) = sum_P Bx^P_ib Bx^P_ja with Bx^P_ia = sum_Q (ia|J^|Q)(L^-T)_QP over the window, the
extra exchange factor that only full TDDFT needs (Fig. tensors_shape, T_ia^P'), built with the same
Cholesky factor L of the J^ metric as Bx_ij and Bx_ab.

Eigenpairs: with A - B = L L^T (positive definite here), the symmetric problem
L^T (A + B) L c = Omega^2 c gives X + Y = L c / sqrt(Omega) and X - Y = L^-T c sqrt(Omega), which
satisfy (A + B)(X + Y) = Omega (X - Y), (A - B)(X - Y) = Omega (X + Y) and (X + Y).(X - Y) = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import risp as R


def exchange_ia_factor(mol, prm: R.Params = R.Params(), pair_mask=None):
    """Bx^P_ia [nK][noK][nvK] over the window (combined reading of the exchange operator)."""
    if prm.rsh_mode != "combined":
        raise NotImplementedError("the full-TDDFT factor follows the combined reading")
    coords, shells = mol.coords, mol.shells
    auxJ, auxK = R.select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    if pair_mask is None:
        _, pair_mask, _ = R.schwarz_pairs(coords, shells, auxJ, prm.schwarz_tau)
    C = mol.mo_coeff
    nocc = mol.nocc
    occK, virK = R.window_sets(mol.mo_energy, nocc, prm.window_ev, prm.window_mode)
    CoK, CvK = C[:, :nocc][:, occK], C[:, nocc:][:, virK]
    noK, nvK = len(occK), len(virK)
    if (prm.c_x == 0.0 and prm.beta == 0.0) or noK == 0 or nvK == 0:
        return np.zeros((0, noK, nvK))
    V2 = R._operator_int2c(coords, auxK, prm.c_x, prm.beta, prm.omega)
    Tia = R._transformed(coords, shells, auxK, prm.c_x, prm.beta, prm.omega, pair_mask, CoK, CvK)
    L = np.linalg.cholesky(V2)
    nK = V2.shape[0]
    return np.ascontiguousarray(sla.solve_triangular(L, Tia.reshape(nK, -1), lower=True)).reshape(Tia.shape)


def dense_B(F: R.Factors, Bx_ia) -> np.ndarray:
    """B [nocc*nvir, nocc*nvir], row index i*nvir + a."""
    o, v = F.nocc, F.nvir
    Bf = F.B_ia.reshape(F.B_ia.shape[0], o * v)
    B = 2.0 * Bf.T @ Bf
    if Bx_ia.shape[0]:
        # (ib|J^|ja) = sum_P Bx_ib Bx_ja, element [i, a, j, b]
        K = np.einsum("Pib,Pja->iajb", Bx_ia, Bx_ia, optimize=True)
        B4 = B.reshape(o, v, o, v)
        ix = np.ix_(F.occK, F.virK, F.occK, F.virK)
        B4[ix] -= K
    return B


def dense_ApB_AmB(F: R.Factors, Bx_ia):
    A = R.dense_A(F)
    B = dense_B(F, Bx_ia)
    return A + B, A - B


def sigma_pm(F: R.Factors, Bx_ia, V):
    """((A + B) V, (A - B) V) for a block V [m][nocc][nvir], matrix-free.

    With J V = sum_P B_ia (B^P . V), KA V the exchange term of A (oracle.risp.sigma) and
    KB V_ia = sum_P sum_jb Bx_ib Bx_ja V_jb over the window:
    (A + B) V = de V + 4 J V - KA V - KB V,  (A - B) V = de V - KA V + KB V.
    """
    V = np.asarray(V, dtype=np.float64)
    m = V.shape[0]
    o, v = F.nocc, F.nvir
    Bf = F.B_ia.reshape(F.B_ia.shape[0], o * v)
    JV = ((Bf @ V.reshape(m, o * v).T).T @ Bf).reshape(m, o, v)
    deV = F.de[None] * V
    AV = R.sigma(F, V)  # de V + 2 J V - KA V
    KA = deV + 2.0 * JV - AV
    KB = np.zeros_like(V)
    if Bx_ia.shape[0]:
        Vw = np.ascontiguousarray(V[:, F.occK][:, :, F.virK])  # [m][j][b]
        Kw = np.zeros_like(Vw)
        for P in range(Bx_ia.shape[0]):
            H = np.einsum("ib,mjb->mij", Bx_ia[P], Vw, optimize=True)  # H_mij = sum_b Bx_ib V_jb
            Kw += np.einsum("mij,ja->mia", H, Bx_ia[P], optimize=True)  # sum_j H_ij Bx_ja
        KB[np.ix_(np.arange(m), F.occK, F.virK)] = Kw
    return deV + 4.0 * JV - KA - KB, deV - KA + KB


def full_eigh(ApB, AmB, n):
    """Lowest n excitation energies Omega and amplitudes X + Y, X - Y [n][ov] (normalised so that
    (X + Y).(X - Y) = 1), through the symmetric form L^T (A + B) L with A - B = L L^T."""
    L = np.linalg.cholesky(AmB)
    S = L.T @ ApB @ L
    w, c = np.linalg.eigh(0.5 * (S + S.T))
    w, c = w[:n], c[:, :n]
    om = np.sqrt(w)
    XpY = (L @ c) / np.sqrt(om)[None, :]
    XmY = sla.solve_triangular(L, c, lower=True, trans="T") * np.sqrt(om)[None, :]
    return om, XpY.T, XmY.T
