"""TDA-risp in plain FP64 (oracle; test infrastructure only, never imported by the HIP path).

The matrix of eq. TDA-risp, with the XC kernel dropped, the RI approximation of
eq. TDDFT-axs_approx_integral, the minimal auxiliary basis of eq. gr without hydrogen functions,
the exchange-space energy window (section on exchange-space truncation) and the range-separated
exchange operator J^ = (alpha + beta erf(omega r))/r of eq. RSH / eq. K_mia_RSH:

  A_{ia,jb} = (e_a - e_i) d_ij d_ab + 2 sum_P B^P_ia B^P_jb
              - [i,j in occK' and a,b in virK'] sum_P Bx^P_ij Bx^P_ab

* B^P_pq = sum_Q (pq|Q) (L^-T)_QP with (P|Q) = L L^T over the Coulomb auxiliary basis (s + p on every
  non-hydrogen atom). Then sum_P B_ia B_jb = sum_PQ (ia|P)(P|Q)^-1(Q|jb), the RI integral. The paper
  writes the exchange factors as T_ij = (ij|Q)(Q|P)^-1 and T_ab = (ab|P); the symmetric Cholesky split
  used here gives the same product and is unique, so factors can be compared element by element.
* Bx: the same construction over the exchange auxiliary basis (one s function per non-hydrogen atom)
  with the operator J^ in both the three-centre integrals and the metric ("combined" reading: one RI
  in the J^ metric, as in eq. K_mia_RSH). For a global hybrid beta = 0 and J^ = c_x/r, so the exchange
  block equals c_x (ij|ab)_RI. The "split" reading stacks sqrt(alpha) RI(1/r) and sqrt(beta) RI(erf)
  along P, each in its own metric.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import integrals as I

HARTREE_TO_EV = 27.211386245988  # CODATA 2018


@dataclass
class Params:
    c_x: float = 0.22  # alpha: full-range exact-exchange fraction
    beta: float = 0.78  # long-range erf part (omegaB97X-family: alpha + beta = 1)
    omega: float = 0.2  # bohr^-1
    window_ev: float = 40.0
    window_mode: str = "absolute"  # or "frontier"
    rsh_mode: str = "combined"  # or "split"
    theta: float = 0.2
    h_in_aux: bool = False
    schwarz_tau: float = 1e-10


# ----------------------------------------------------------------------------------------------
# Auxiliary basis (eq. gr; hydrogen omitted; Coulomb: s+p, exchange: s)
# ----------------------------------------------------------------------------------------------
def select_aux(Z, aux_radius, theta=0.2, h_in_aux=False):
    """Auxiliary shells [(atom, l, exponent, 1.0)] for the Coulomb (s and p) and exchange (s) terms.

    One uncontracted primitive per shell with exponent theta / R_A^2 (eq. gr). Atoms with Z == 1 get
    no auxiliary functions unless h_in_aux. Coulomb order: per atom s then p; exchange: s per atom.
    """
    J, K = [], []
    for a, z in enumerate(Z):
        if z == 1 and not h_in_aux:
            continue
        e = theta / float(aux_radius[a]) ** 2
        J.append((a, 0, e, 1.0))
        J.append((a, 1, e, 1.0))
        K.append((a, 0, e, 1.0))
    return J, K


# ----------------------------------------------------------------------------------------------
# Energy window (section on exchange-space truncation)
# ----------------------------------------------------------------------------------------------
def window_sets(mo_energy, nocc, window_ev=40.0, mode="absolute"):
    """Occupied and virtual orbitals kept in the exchange term, ascending, 0-based within each space.

    absolute: keep occupied i with e_i * H2EV > -window and virtual a with e_a * H2EV < window.
    frontier: keep i with (e_LUMO - e_i) * H2EV < window and a with (e_a - e_HOMO) * H2EV < window.
    """
    e = np.asarray(mo_energy, dtype=np.float64)
    eo, ev = e[:nocc], e[nocc:]
    if mode == "absolute":
        occ = np.nonzero(eo * HARTREE_TO_EV > -window_ev)[0]
        vir = np.nonzero(ev * HARTREE_TO_EV < window_ev)[0]
    elif mode == "frontier":
        occ = np.nonzero((ev[0] - eo) * HARTREE_TO_EV < window_ev)[0]
        vir = np.nonzero((ev - eo[-1]) * HARTREE_TO_EV < window_ev)[0]
    else:
        raise ValueError(mode)
    return occ.astype(np.int32), vir.astype(np.int32)


# ----------------------------------------------------------------------------------------------
# Shell-pair screening (Schwarz)
# ----------------------------------------------------------------------------------------------
def schwarz_pairs(coords, shells, aux_shells, tau):
    """Kept shell pairs (A >= B) with Q_AB * Q_aux >= tau, sorted by (A, B); plus the ratio array.

    Q_AB = max sqrt((mu nu|mu nu)) over the functions of the two shells and Q_aux = max_P sqrt((P|P))
    over the given auxiliary functions. tau = 0 keeps every pair.
    Returns (pairs [npair, 2] int32, mask [nsh, nsh] bool (symmetric), ratio Q_AB Q_aux / tau or None).
    """
    Qab = I.schwarz_diag(coords, shells)
    Vaux = I.int2c(coords, aux_shells)
    qaux = float(np.sqrt(np.max(np.diag(Vaux))))
    nsh = len(shells)
    A, B = np.tril_indices(nsh)
    vals = Qab[A, B] * qaux
    keep = vals >= tau
    pairs = np.stack([A[keep], B[keep]], axis=1).astype(np.int32)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    pairs = pairs[order]
    mask = np.zeros((nsh, nsh), dtype=bool)
    mask[pairs[:, 0], pairs[:, 1]] = True
    mask[pairs[:, 1], pairs[:, 0]] = True
    ratio = vals / tau if tau > 0 else None
    return pairs, mask, ratio


# ----------------------------------------------------------------------------------------------
# RI factors
# ----------------------------------------------------------------------------------------------
def _operator_int3c(coords, shells, aux, alpha, beta, omega, mask, aux_idx=None):
    """(mu nu| alpha/r + beta erf(omega r)/r |P)."""
    out = 0.0
    if alpha != 0.0:
        out = alpha * I.int3c(coords, shells, aux, None, mask, aux_idx)
    if beta != 0.0:
        out = out + beta * I.int3c(coords, shells, aux, omega, mask, aux_idx)
    return out


def _operator_int2c(coords, aux, alpha, beta, omega):
    out = 0.0
    if alpha != 0.0:
        out = alpha * I.int2c(coords, aux)
    if beta != 0.0:
        out = out + beta * I.int2c(coords, aux, omega)
    return out


def cholesky_split(V3_mo, V2):
    """B[P, ...] with sum_P B^P_pq B^P_rs = (pq|P)(P|Q)^-1(Q|rs): B = L^-1 (Q|pq), (P|Q) = L L^T."""
    L = np.linalg.cholesky(V2)
    shp = V3_mo.shape
    Bflat = sla.solve_triangular(L, V3_mo.reshape(shp[0], -1), lower=True)
    # C order: the solver returns Fortran order, whose reshape would be a strided view
    return np.ascontiguousarray(Bflat).reshape(shp), L


@dataclass
class Factors:
    nocc: int
    nvir: int
    de: np.ndarray  # [nocc, nvir] e_a - e_i
    B_ia: np.ndarray  # [naux_J, nocc, nvir]
    Bx_ij: np.ndarray  # [nKaux, noK, noK]
    Bx_ab: np.ndarray  # [nKaux, nvK, nvK]
    occK: np.ndarray
    virK: np.ndarray
    L_J: np.ndarray = field(repr=False, default=None)
    L_K: np.ndarray = field(repr=False, default=None)
    pairs: np.ndarray = field(repr=False, default=None)


def build_factors(mol, prm: Params = Params(), pair_mask=None) -> Factors:
    """All RI factors of the TDA-risp matrix for a synth.Molecule-like object."""
    coords = mol.coords
    shells = mol.shells
    auxJ, auxK = select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    if pair_mask is None:
        pairs, pair_mask, _ = schwarz_pairs(coords, shells, auxJ, prm.schwarz_tau)
    else:
        pairs = None
    C = mol.mo_coeff
    nocc = mol.nocc
    Co, Cv = C[:, :nocc], C[:, nocc:]
    occK, virK = window_sets(mol.mo_energy, nocc, prm.window_ev, prm.window_mode)
    CoK, CvK = Co[:, occK], Cv[:, virK]
    # Coulomb factor (integrals evaluated a few auxiliary shells at a time to bound memory)
    Tia = _transformed(coords, shells, auxJ, 1.0, 0.0, None, pair_mask, Co, Cv)
    B_ia, L_J = cholesky_split(Tia, I.int2c(coords, auxJ))
    # exchange factors in the J^ metric
    Bx_ij, Bx_ab, L_K = _exchange_factors(coords, shells, auxK, prm, pair_mask, CoK, CvK)
    e = mol.mo_energy
    de = e[None, nocc:] - e[:nocc, None]
    return Factors(nocc=nocc, nvir=C.shape[1] - nocc, de=de, B_ia=B_ia, Bx_ij=Bx_ij, Bx_ab=Bx_ab,
                   occK=occK, virK=virK, L_J=L_J, L_K=L_K, pairs=pairs)


def _transformed(coords, shells, aux, alpha, beta, omega, mask, Cl, Cr, chunk=8):
    """T~[P][p][q] = sum_mu nu Cl[mu][p] (mu nu| alpha/r + beta erf(omega r)/r |P) Cr[nu][q]."""
    out = []
    for s0 in range(0, len(aux), chunk):
        idx = list(range(s0, min(len(aux), s0 + chunk)))
        V3 = _operator_int3c(coords, shells, aux, alpha, beta, omega, mask, idx)
        out.append(np.einsum("mp,mnP,nq->Ppq", Cl, V3, Cr, optimize=True))
    return np.concatenate(out, axis=0)


def _exchange_factors(coords, shells, auxK, prm, pair_mask, CoK, CvK):
    def one(alpha, beta):
        V2 = _operator_int2c(coords, auxK, alpha, beta, prm.omega)
        Tij = _transformed(coords, shells, auxK, alpha, beta, prm.omega, pair_mask, CoK, CoK)
        Tab = _transformed(coords, shells, auxK, alpha, beta, prm.omega, pair_mask, CvK, CvK)
        L = np.linalg.cholesky(V2)
        nK = V2.shape[0]
        Bij = np.ascontiguousarray(sla.solve_triangular(L, Tij.reshape(nK, -1), lower=True)).reshape(Tij.shape)
        Bab = np.ascontiguousarray(sla.solve_triangular(L, Tab.reshape(nK, -1), lower=True)).reshape(Tab.shape)
        return Bij, Bab, L

    noK, nvK = CoK.shape[1], CvK.shape[1]
    if prm.c_x == 0.0 and prm.beta == 0.0:
        return np.zeros((0, noK, noK)), np.zeros((0, nvK, nvK)), None
    if prm.rsh_mode == "combined":
        return one(prm.c_x, prm.beta)
    if prm.rsh_mode == "split":
        parts = []
        if prm.c_x != 0.0:
            parts.append(one(prm.c_x, 0.0))
        if prm.beta != 0.0:
            parts.append(one(0.0, prm.beta))
        Bij = np.concatenate([p[0] for p in parts])
        Bab = np.concatenate([p[1] for p in parts])
        return Bij, Bab, None
    raise ValueError(prm.rsh_mode)


# ----------------------------------------------------------------------------------------------
# The matrix and its product with trial vectors
# ----------------------------------------------------------------------------------------------
def dense_A(F: Factors) -> np.ndarray:
    """A [nocc*nvir, nocc*nvir], row index i*nvir + a."""
    o, v = F.nocc, F.nvir
    Bf = F.B_ia.reshape(F.B_ia.shape[0], o * v)
    A = 2.0 * Bf.T @ Bf
    A[np.diag_indices(o * v)] += F.de.ravel()
    if F.Bx_ij.shape[0]:
        K = np.einsum("Pij,Pab->iajb", F.Bx_ij, F.Bx_ab, optimize=True)
        A4 = A.reshape(o, v, o, v)
        ix = np.ix_(F.occK, F.virK, F.occK, F.virK)
        A4[ix] -= K
    return A


def diag_A(F: Factors) -> np.ndarray:
    """Diagonal of A [nocc][nvir]: e_a - e_i + 2 sum_P B^P_ia^2 - [i in occK', a in virK'] sum_P Bx^P_ii Bx^P_aa."""
    d = F.de + 2.0 * np.einsum("Pia,Pia->ia", F.B_ia, F.B_ia)
    if F.Bx_ij.shape[0]:
        bii = np.einsum("Pii->Pi", F.Bx_ij)
        baa = np.einsum("Paa->Pa", F.Bx_ab)
        d[np.ix_(F.occK, F.virK)] -= bii.T @ baa
    return d


def sigma(F: Factors, X: np.ndarray, coulomb=None) -> np.ndarray:
    """sigma = A X for a block X [m][nocc][nvir], matrix-free.

    sigma = de*X + 2 sum_P B^P_ia (sum_jb B^P_jb X_mjb) - scatter_window(K), where the exchange part
    K_mia = sum_P sum_jb Bx^P_ij Bx^P_ab X_mjb runs over the window only. `coulomb`: the Coulomb
    term 2 J [m][nocc][nvir] computed elsewhere (coulomb_ao) in place of the one from B_ia.
    """
    X = np.asarray(X, dtype=np.float64)
    m = X.shape[0]
    o, v = F.nocc, F.nvir
    out = F.de[None] * X
    if coulomb is None:
        Bf = F.B_ia.reshape(F.B_ia.shape[0], o * v)
        Y = Bf @ X.reshape(m, o * v).T  # [P, m]
        out += 2.0 * (Y.T @ Bf).reshape(m, o, v)
    else:
        out += coulomb
    if F.Bx_ij.shape[0]:
        Xw = np.ascontiguousarray(X[:, F.occK][:, :, F.virK])  # [m, noK, nvK] (contiguous for BLAS)
        K = np.zeros_like(Xw)
        for P in range(F.Bx_ij.shape[0]):
            M = Xw @ F.Bx_ab[P]  # M^P_mja = sum_b Xw_mjb Bx^P_ba (Bx^P_ab is symmetric in a, b)
            K += F.Bx_ij[P] @ M  # K_mia += sum_j Bx^P_ij M^P_mja (matmul broadcast over m)
        out[np.ix_(np.arange(m), F.occK, F.virK)] -= K
    return out


def coulomb_ao(mol, X: np.ndarray, prm: Params = Params(), pair_mask=None) -> np.ndarray:
    """2 J_mia by the AO-density route (section on on-the-fly Coulomb evaluation), no stored T_ia.

    D_m = C_occ X_m C_vir^T (AO transition density); R_Q = sum_(mu nu) (mu nu|Q) D_m,mu nu;
    R~ solves (P|Q) R~ = R; U_m = sum_P (mu nu|P) R~_P; J_m = C_occ^T U_m C_vir. The same Schwarz pair
    mask as build_factors (by default), so J equals the stored-factor route up to rounding.
    Returns [m][nocc][nvir].
    """
    coords, shells = mol.coords, mol.shells
    auxJ, _ = select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    if pair_mask is None:
        _, pair_mask, _ = schwarz_pairs(coords, shells, auxJ, prm.schwarz_tau)
    C = mol.mo_coeff
    nocc = mol.nocc
    Co, Cv = C[:, :nocc], C[:, nocc:]
    X = np.asarray(X, dtype=np.float64)
    D = np.einsum("mi,kia,na->kmn", Co, X, Cv, optimize=True)
    V3 = I.int3c(coords, shells, auxJ, None, pair_mask)  # [mu][nu][P]
    R = np.einsum("mnP,kmn->Pk", V3, D, optimize=True)
    Rt = sla.cho_solve(sla.cho_factor(I.int2c(coords, auxJ), lower=True), R)
    U = np.einsum("mnP,Pk->kmn", V3, Rt, optimize=True)
    return 2.0 * np.einsum("mi,kmn,na->kia", Co, U, Cv, optimize=True)


def sigma_ao(F: Factors, mol, X: np.ndarray, prm: Params = Params()) -> np.ndarray:
    """sigma = A X with the Coulomb term from coulomb_ao (F supplies the gaps and exchange factors)."""
    X = np.asarray(X, dtype=np.float64)
    return sigma(F, X, coulomb=coulomb_ao(mol, X, prm))


def sigma_rows_chunk(mol, prm: Params, pair_mask, kind, shell_idx, D, rows_i, rows_a):
    """Integral work of sigma_rows for one chunk of auxiliary shells (no reduction across chunks).

    kind "J": Coulomb auxiliary shells shell_idx. Returns (R [nP][m], Tq [nP][r]) with
    R_Pm = sum_(mu nu) (mu nu|P) D_m,mu nu (D_m = C_occ X_m C_vir^T, the AO transition density, so
    R_Pm = sum_ia (ia|P) X_m,ia) and Tq_Pr = (i_r a_r|P).
    kind "K": exchange auxiliary shells shell_idx with the operator J^ = c_x/r + beta erf(omega r)/r.
    Returns (Ti [nP][r][noK], Ta [nP][r][nvK]) with Ti_Prj = (i_r j|J^|P) for j in occK' and
    Ta_Prb = (a_r b|J^|P) for b in virK'.
    """
    coords, shells = mol.coords, mol.shells
    auxJ, auxK = select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    C = mol.mo_coeff
    nocc = mol.nocc
    Co, Cv = C[:, :nocc], C[:, nocc:]
    if kind == "J":
        V3 = I.int3c(coords, shells, auxJ, None, pair_mask, list(shell_idx))  # [mu][nu][P]
        nao, nP = V3.shape[0], V3.shape[2]
        m = D.shape[0]
        R = V3.reshape(nao * nao, nP).T @ np.asarray(D).reshape(m, nao * nao).T  # [P][m]
        iu, inv = np.unique(rows_i, return_inverse=True)
        H = np.einsum("mu,mnP->unP", Co[:, iu], V3, optimize=True)  # (i nu|P)
        Tq = np.einsum("rnP,nr->Pr", H[inv], Cv[:, rows_a], optimize=True)
        return R, Tq
    if kind == "K":
        V3 = _operator_int3c(coords, shells, auxK, prm.c_x, prm.beta, prm.omega, pair_mask, list(shell_idx))
        occK, virK = window_sets(mol.mo_energy, nocc, prm.window_ev, prm.window_mode)
        Hi = np.einsum("mr,mnP->rnP", Co[:, rows_i], V3, optimize=True)
        Ha = np.einsum("mr,mnP->rnP", Cv[:, rows_a], V3, optimize=True)
        Ti = np.einsum("rnP,nj->Prj", Hi, Co[:, occK], optimize=True)
        Ta = np.einsum("rnP,nb->Prb", Ha, Cv[:, virK], optimize=True)
        return Ti, Ta
    raise ValueError(kind)


def sigma_rows_tasks(mol, prm: Params = Params(), j_chunk=4, k_chunk=8):
    """The (kind, shell_idx) chunks that sigma_rows evaluates, Coulomb first."""
    auxJ, auxK = select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    tasks = [("J", tuple(range(s, min(len(auxJ), s + j_chunk)))) for s in range(0, len(auxJ), j_chunk)]
    tasks += [("K", tuple(range(s, min(len(auxK), s + k_chunk)))) for s in range(0, len(auxK), k_chunk)]
    return tasks


def sigma_rows(mol, X, rows, prm: Params = Params(), pair_mask=None, run_chunks=None, D=None):
    """Selected elements of sigma = A X straight from the integrals, without storing any factor.

    rows: flat indices r = i*nvir + a. Returns [m][len(rows)]. For each row (i, a):
      sigma_m,ia = (e_a - e_i) X_m,ia + 2 sum_P B^P_ia Y^P_m - [i in occK', a in virK'] K_m,ia,
      B = L_J^-1 (Q|ia), Y = L_J^-1 R with R_Q = sum_jb (jb|Q) X_m,jb (formed from the AO transition
      density, as in coulomb_ao), and K_m,ia = sum_P sum_(j,b in window) Bx^P_ij X_m,jb Bx^P_ab with
      Bx = L_K^-1 (pq|J^|Q) in the J^ metric (eq. K_mia_RSH, combined reading).
    This is the same matrix as build_factors/sigma; only the needed rows of the factors are formed, so
    it runs at sizes whose factors do not fit in host memory. run_chunks(tasks, D, rows_i, rows_a):
    optional replacement of the serial loop over sigma_rows_chunk (e.g. a process pool), returning
    the chunk results in task order; D: optional precomputed AO transition densities [m][nao][nao].
    """
    if prm.rsh_mode != "combined":
        raise NotImplementedError("sigma_rows implements the combined reading of the exchange operator")
    coords, shells = mol.coords, mol.shells
    auxJ, auxK = select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    if pair_mask is None:
        _, pair_mask, _ = schwarz_pairs(coords, shells, auxJ, prm.schwarz_tau)
    C = mol.mo_coeff
    nocc, nvir = mol.nocc, C.shape[1] - mol.nocc
    Co, Cv = C[:, :nocc], C[:, nocc:]
    X = np.asarray(X, dtype=np.float64)
    m = X.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    ri, ra = rows // nvir, rows % nvir
    if D is None and run_chunks is None:
        D = np.einsum("mi,kia,na->kmn", Co, X, Cv, optimize=True)
    tasks = sigma_rows_tasks(mol, prm)
    if run_chunks is None:
        res = [sigma_rows_chunk(mol, prm, pair_mask, k, idx, D, ri, ra) for k, idx in tasks]
    else:
        res = list(run_chunks(tasks, D, ri, ra))
    nJt = sum(1 for t in tasks if t[0] == "J")
    R = np.concatenate([r[0] for r in res[:nJt]], axis=0)  # [naux_J][m]
    Tq = np.concatenate([r[1] for r in res[:nJt]], axis=0)  # [naux_J][r]
    LJ = np.linalg.cholesky(I.int2c(coords, auxJ))
    B = sla.solve_triangular(LJ, Tq, lower=True)
    Y = sla.solve_triangular(LJ, R, lower=True)
    e = mol.mo_energy
    out = (e[nocc + ra] - e[ri])[None, :] * X.reshape(m, -1)[:, rows] + 2.0 * (Y.T @ B)
    if (prm.c_x != 0.0 or prm.beta != 0.0) and len(auxK):
        occK, virK = window_sets(e, nocc, prm.window_ev, prm.window_mode)
        Ti = np.concatenate([r[0] for r in res[nJt:]], axis=0)  # [nK][r][noK]
        Ta = np.concatenate([r[1] for r in res[nJt:]], axis=0)  # [nK][r][nvK]
        LK = np.linalg.cholesky(_operator_int2c(coords, auxK, prm.c_x, prm.beta, prm.omega))
        nK, nr = Ti.shape[0], Ti.shape[1]
        Bi = sla.solve_triangular(LK, Ti.reshape(nK, -1), lower=True).reshape(Ti.shape)
        Ba = sla.solve_triangular(LK, Ta.reshape(nK, -1), lower=True).reshape(Ta.shape)
        Xw = X[:, occK][:, :, virK]  # [m][noK][nvK]
        inw = np.isin(ri, occK) & np.isin(ra, virK)
        for r in np.nonzero(inw)[0]:
            # K_m = sum_P Bi[P, r, :] Xw_m Ba[P, r, :]
            G = np.einsum("Pj,Pb->jb", Bi[:, r, :], Ba[:, r, :], optimize=True)
            out[:, r] -= np.einsum("mjb,jb->m", Xw, G, optimize=True)
    return out


def lowest_eigh(A, n):
    w, U = np.linalg.eigh(A)
    return w[:n], U[:, :n].T


# ----------------------------------------------------------------------------------------------
# Block Davidson (section on large-system Davidson diagonalisation)
# ----------------------------------------------------------------------------------------------
@dataclass
class DavidsonResult:
    energies: np.ndarray
    vectors: np.ndarray  # [nstates, nocc*nvir]
    iters: int
    restarts: int
    nsigma: int
    converged: bool
    resid: list


def davidson(F: Factors, nstates, tol=1e-6, block=None, max_space=None, max_iter=200, sigma_fn=None, diag=None,
             verbose=False):
    """Block Davidson for the lowest eigenpairs of A (FP64).

    Guess: unit vectors at the lowest d = e_a - e_i (or `diag`, e.g. diag_A(F)), ties by (i, a). Each
    iteration: Rayleigh-Ritz on the subspace, residuals r_k = A x_k - theta_k x_k for the lowest
    `block` Ritz pairs, corrections t_k = r_k / (theta_k - d) (|theta - d| floored at 1e-8), two-pass
    classical Gram-Schmidt against the subspace, drop vectors whose norm falls below 1e-6. Converged when ||r_k|| < tol for
    k < nstates. When the subspace would exceed max_space, restart from the current Ritz vectors and
    recompute their products A V.
    """
    o, v = F.nocc, F.nvir
    n = o * v
    if block is None:
        block = min(2 * nstates, 30)
    block = min(block, n)
    if max_space is None:
        max_space = max(8 * block, nstates + 2 * block)
    sig = sigma_fn or (lambda X: sigma(F, X.reshape(-1, o, v)).reshape(-1, n))
    d = (F.de if diag is None else np.asarray(diag)).ravel()
    order = np.lexsort((np.arange(n), d))[:block]  # stable: ties keep (i, a) order
    V = np.zeros((block, n))
    V[np.arange(block), order] = 1.0
    W = sig(V)
    nsig = block
    restarts = 0
    resid = []
    for it in range(1, max_iter + 1):
        H = V @ W.T
        H = 0.5 * (H + H.T)
        theta, y = np.linalg.eigh(H)
        k = min(block, len(theta))
        theta, y = theta[:k], y[:, :k]
        Xr = y.T @ V
        R = y.T @ W - theta[:, None] * Xr
        rn = np.linalg.norm(R, axis=1)
        resid.append(rn[:nstates].copy())
        if verbose:
            print(f"oracle davidson iteration {it}: subspace {V.shape[0]}, max residual {rn[:nstates].max():.3e}",
                  flush=True)
        if np.all(rn[:nstates] < tol):
            return DavidsonResult(theta[:nstates], Xr[:nstates], it, restarts, nsig, True, resid)
        todo = [j for j in range(k) if rn[j] >= tol]
        den = theta[todo, None] - d[None, :]
        den = np.where(np.abs(den) < 1e-8, np.where(den < 0, -1e-8, 1e-8), den)
        T = R[todo] / den
        T = T / np.linalg.norm(T, axis=1, keepdims=True)  # drop test below is relative to unit length
        if V.shape[0] + T.shape[0] > max_space:
            # restart: keep the Ritz vectors, recompute A V for consistency
            V = Xr
            W = sig(V)
            nsig += V.shape[0]
            restarts += 1
        for _ in range(2):
            T = T - (T @ V.T) @ V
        keep = []
        for j in range(T.shape[0]):
            t = T[j]
            for q in keep:
                t = t - np.dot(T[q], t) * T[q]
            t = t - (t @ V.T) @ V
            nt = np.linalg.norm(t)
            if nt > 1e-6:
                T[j] = t / nt
                keep.append(j)
        T = T[keep]
        if T.shape[0] == 0:
            break
        WT = sig(T)
        nsig += T.shape[0]
        V = np.vstack([V, T])
        W = np.vstack([W, WT])
    H = V @ W.T
    theta, y = np.linalg.eigh(0.5 * (H + H.T))
    return DavidsonResult(theta[:nstates], (y[:, :nstates].T @ V), max_iter, restarts, nsig, False, resid)
