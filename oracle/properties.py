"""Transition properties of TDA-risp states in plain FP64 (oracle; test infrastructure only).

For the excitation n with energy Omega_n and unit-normalised amplitudes X_n (the Davidson output),
the paper's oscillator and rotatory strengths (eq. oscillator_strength, eq. rotator_strength) in
the dipole-length form with TDA amplitudes (Y = 0 in eq. transition and eq. transition_magnetic):

  mu_0n = sqrt(2) sum_ia r_ia X_nia          f_0n = 2/3 Omega_n |mu_0n|^2
  m_0n  = sqrt(2) sum_ia (r x nabla)_ia X_nia    R_0n = 1/2 mu_0n . m_0n

r_ia = <i| r - O |a> and (r x nabla)_ia = <i| (r - O) x nabla |a> over the real MOs (a real
antisymmetric operator); O is the gauge origin. The sqrt(2) makes the spin-adapted closed-shell
singlet of a unit-normalised X (the paper writes the sums over spin orbitals).

AO integrals over normalised primitive Cartesian Gaussians follow the McMurchie-Davidson route of
oracle.integrals: one Cartesian direction of <a|b> is E^{ij}_0 sqrt(pi/p), of <a|x - O_x|b> is
(E^{ij}_1 + (P_x - O_x) E^{ij}_0) sqrt(pi/p), and the derivative of the ket primitive is
d/dx x_B^j exp(-b x_B^2) = j x_B^(j-1) exp(...) - 2 b x_B^(j+1) exp(...).

Spectra: each state's strength spread with a unit-area Lorentzian of half width at half maximum
gamma (the paper's figures use 0.05 eV): S(E) = sum_n s_n (gamma/pi) / ((E - Omega_n)^2 + gamma^2).
"""
from __future__ import annotations

import math

import numpy as np

from . import integrals as I


def _one_dim(i, j, A, B, a, b, O):
    """1-D factors for primitives of powers i (centre A, exponent a) and j (B, b), all arrays:
    overlap S, moment M = <x - O>, and ket derivative D = <i| d/dx |j>; without the Gaussian prefactor
    exp(-mu X_AB^2), which the caller applies once per pair."""
    p = a + b
    P = (a * A + b * B) / p
    s = np.sqrt(math.pi / p)

    def S1(ii, jj):
        if jj < 0:
            return 0.0 * p
        return I.hermite_E(ii, jj, P - A, P - B, p)[0] * s

    E = I.hermite_E(i, j, P - A, P - B, p)
    S = E[0] * s
    E1 = E[1] if len(E) > 1 else 0.0 * p
    M = (E1 + (P - O) * E[0]) * s
    D = j * S1(i, j - 1) - 2.0 * b * S1(i, j + 1)
    return S, M, D


def ao_dipole_and_rxdel(coords, shells, origin=(0.0, 0.0, 0.0)):
    """AO matrices <mu| r - O |nu> [3][nao][nao] and <mu| (r - O) x nabla |nu> [3][nao][nao].

    Evaluated for all shell pairs of one angular-momentum class at a time (arrays over the pairs)."""
    coords = np.asarray(coords, dtype=np.float64)
    O = np.asarray(origin, dtype=np.float64)
    off, nao = I.shell_offsets(shells)
    off = np.array(off)
    ls = np.array([s[1] for s in shells])
    cen = np.array([coords[s[0]] for s in shells]).reshape(-1, 3)
    ex = np.array([s[2] for s in shells], dtype=np.float64)
    cf = np.array([s[3] for s in shells], dtype=np.float64)
    dip = np.zeros((3, nao, nao))
    rxd = np.zeros((3, nao, nao))
    for la in (0, 1):
        for lb in (0, 1):
            SA, SB = np.nonzero(ls == la)[0], np.nonzero(ls == lb)[0]
            if len(SA) == 0 or len(SB) == 0:
                continue
            pa, pb = np.meshgrid(SA, SB, indexing="ij")
            pa, pb = pa.ravel(), pb.ravel()
            A, B, a, b = cen[pa], cen[pb], ex[pa], ex[pb]
            mu = a * b / (a + b)
            K = np.exp(-mu * np.sum((A - B) ** 2, axis=1))
            for ia, compA in enumerate(I.cart_components(la)):
                na = I.primitive_norm(a, compA) * cf[pa]
                for ib, compB in enumerate(I.cart_components(lb)):
                    nb = I.primitive_norm(b, compB) * cf[pb]
                    S, M, D = zip(*[_one_dim(compA[d], compB[d], A[:, d], B[:, d], a, b, O[d]) for d in range(3)])
                    pre = K * na * nb
                    r, c = off[pa] + ia, off[pb] + ib
                    dip[0, r, c] = pre * M[0] * S[1] * S[2]
                    dip[1, r, c] = pre * S[0] * M[1] * S[2]
                    dip[2, r, c] = pre * S[0] * S[1] * M[2]
                    # (r x nabla)_x = y d/dz - z d/dy, cyclic
                    rxd[0, r, c] = pre * S[0] * (M[1] * D[2] - D[1] * M[2])
                    rxd[1, r, c] = pre * S[1] * (M[2] * D[0] - D[2] * M[0])
                    rxd[2, r, c] = pre * S[2] * (M[0] * D[1] - D[0] * M[1])
    return dip, rxd


def mo_transition_integrals(mol, origin=(0.0, 0.0, 0.0)):
    """r_ia and (r x nabla)_ia as [3][nocc][nvir] over the occupied and virtual MOs."""
    dip, rxd = ao_dipole_and_rxdel(mol.coords, mol.shells, origin)
    C = mol.mo_coeff
    Co, Cv = C[:, :mol.nocc], C[:, mol.nocc:]
    r_ia = np.einsum("mi,cmn,na->cia", Co, dip, Cv, optimize=True)
    l_ia = np.einsum("mi,cmn,na->cia", Co, rxd, Cv, optimize=True)
    return r_ia, l_ia


def transition_moments(r_ia, l_ia, X):
    """mu_0n, m_0n [n][3] for amplitudes X [n][nocc][nvir] (unit rows)."""
    X = np.asarray(X, dtype=np.float64)
    mu = math.sqrt(2.0) * np.einsum("cia,nia->nc", r_ia, X, optimize=True)
    m = math.sqrt(2.0) * np.einsum("cia,nia->nc", l_ia, X, optimize=True)
    return mu, m


def oscillator_strengths(omega, mu):
    """f_0n = 2/3 Omega_n |mu_0n|^2 (eq. oscillator_strength)."""
    return 2.0 / 3.0 * np.asarray(omega) * np.sum(np.asarray(mu) ** 2, axis=1)


def rotatory_strengths(mu, m):
    """R_0n = 1/2 mu_0n . m_0n (eq. rotator_strength)."""
    return 0.5 * np.sum(np.asarray(mu) * np.asarray(m), axis=1)


def spectrum(energies_grid, omega, strengths, hwhm):
    """Lorentzian-broadened stick spectrum sum_n s_n (gamma/pi) / ((E - Omega_n)^2 + gamma^2)."""
    E = np.asarray(energies_grid, dtype=np.float64)[:, None]
    w = np.asarray(omega, dtype=np.float64)[None, :]
    g = float(hwhm)
    return np.sum(np.asarray(strengths)[None, :] * (g / math.pi) / ((E - w) ** 2 + g * g), axis=1)


def properties(mol, omega, X, origin=(0.0, 0.0, 0.0)):
    """mu, m [n][3], f [n], R [n] for the states (omega [n], X [n][nocc][nvir])."""
    r_ia, l_ia = mo_transition_integrals(mol, origin)
    mu, m = transition_moments(r_ia, l_ia, X)
    return mu, m, oscillator_strengths(omega, mu), rotatory_strengths(mu, m)
