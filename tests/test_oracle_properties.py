"""Pins of the oracle's transition properties (oracle/properties.py) against closed forms, numerical
quadrature and the symmetry of the operators (no GPU)."""
import math

import numpy as np
import pytest

import synth
from oracle import integrals as I
from oracle import properties as PR
from oracle import risp as R


def _prim(coords, shell, comp, pts):
    """A normalised primitive and its gradient on points [n][3]."""
    k, l, e, c = shell
    d = pts - np.asarray(coords[k])
    n = float(I.primitive_norm(e, comp)) * c
    g = n * np.exp(-e * np.sum(d * d, axis=1))
    poly = np.prod([d[:, q] ** comp[q] for q in range(3)], axis=0)
    val = poly * g
    grad = []
    for q in range(3):
        dpoly = comp[q] * np.prod([d[:, r] ** (comp[r] - (1 if r == q else 0)) for r in range(3)], axis=0)
        grad.append(dpoly * g - 2.0 * e * d[:, q] * val)
    return val, np.stack(grad, axis=1)


def test_closed_forms_same_centre():
    # <p_x| (r x nabla)_z |p_y> = +1 and <p_y| (r x nabla)_z |p_x> = -1 for normalised p on one centre
    # (L_z = -i (x d_y - y d_x)); <s| x |p_x> = 1 / (2 sqrt(a)); <s| r |s> = the centre
    a = 0.45
    coords = np.array([[0.3, -0.2, 0.7]])
    shells = [(0, 0, a, 1.0), (0, 1, a, 1.0)]
    dip, rxd = PR.ao_dipole_and_rxdel(coords, shells, origin=coords[0])
    px, py = 1, 2
    assert abs(rxd[2, px, py] - 1.0) < 1e-13 and abs(rxd[2, py, px] + 1.0) < 1e-13
    assert abs(rxd[0, 2, 3] - 1.0) < 1e-13  # <p_y| (r x nabla)_x |p_z> = +1 (cyclic)
    assert abs(dip[0, 0, px] - 1.0 / (2.0 * math.sqrt(a))) < 1e-13
    dip0, _ = PR.ao_dipole_and_rxdel(coords, shells)
    assert np.allclose(dip0[:, 0, 0], coords[0], atol=1e-14)


def test_dipole_and_rxdel_vs_quadrature():
    # two atoms with s and p shells of different exponents, off-origin gauge point; trapezoid rule on a
    # fine grid (spectrally accurate for Gaussians)
    coords = np.array([[0.0, 0.0, 0.0], [1.1, -0.6, 0.8]])
    shells = [(0, 0, 0.45, 1.0), (0, 1, 0.45, 1.0), (1, 0, 1.35, 1.0), (1, 1, 0.15 * 3, 1.0)]
    O = np.array([0.2, 0.3, -0.4])
    dip, rxd = PR.ao_dipole_and_rxdel(coords, shells, origin=O)
    h, L = 0.09, 7.5
    ax = np.arange(-L, L + 1e-9, h)
    X, Y, Z = np.meshgrid(ax + 0.55, ax - 0.3, ax + 0.4, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    w = h ** 3
    funcs = []
    for s in shells:
        for comp in I.cart_components(s[1]):
            funcs.append(_prim(coords, s, comp, pts))
    rO = pts - O
    for mu in range(len(funcs)):
        for nu in range(len(funcs)):
            va, _ = funcs[mu]
            vb, gb = funcs[nu]
            for c in range(3):
                q = np.sum(va * rO[:, c] * vb) * w
                assert abs(q - dip[c, mu, nu]) < 1e-9, (mu, nu, c)
            cross = np.cross(rO, gb)  # ((r - O) x nabla) phi_b
            for c in range(3):
                q = np.sum(va * cross[:, c]) * w
                assert abs(q - rxd[c, mu, nu]) < 1e-9, (mu, nu, c)


def test_operator_symmetry_and_origin_shift():
    mol = synth.make_config0()
    dip, rxd = PR.ao_dipole_and_rxdel(mol.coords, mol.shells)
    assert np.abs(dip - dip.transpose(0, 2, 1)).max() < 1e-13
    assert np.abs(rxd + rxd.transpose(0, 2, 1)).max() < 1e-12  # r x nabla is anti-Hermitian (real)
    # a shifted gauge origin changes r by a constant times the overlap
    O = np.array([0.7, -1.1, 0.4])
    dip2, _ = PR.ao_dipole_and_rxdel(mol.coords, mol.shells, origin=O)
    diff = dip - dip2  # = O_c * S
    Sx = diff[0] / O[0]
    assert np.abs(diff[1] - O[1] * Sx).max() < 1e-12 and np.abs(diff[2] - O[2] * Sx).max() < 1e-12
    assert np.allclose(np.diag(Sx), 1.0, atol=1e-13)  # normalised primitives


def _transform(mol, Q):
    """The molecule under the orthogonal map r -> Q r: coordinates, and the p components of every
    MO rotate like a vector; s components are unchanged."""
    import copy
    m2 = copy.copy(mol)
    m2.coords = mol.coords @ Q.T
    C = mol.mo_coeff.copy()
    off, _ = I.shell_offsets(mol.shells)
    for k, (atom, l, e, c) in enumerate(mol.shells):
        if l == 1:
            C[off[k]:off[k] + 3] = Q @ C[off[k]:off[k] + 3]
    m2.mo_coeff = C
    return m2


def test_strengths_rotation_invariant_and_mirror_flips_rotatory():
    mol = synth.make_config0()
    rng = np.random.default_rng(4)
    X = rng.normal(size=(3, mol.nocc, mol.nvir))
    X /= np.linalg.norm(X.reshape(3, -1), axis=1)[:, None, None]
    omega = np.array([0.2, 0.25, 0.3])
    com = mol.coords.mean(axis=0)
    mu, m, f, Rr = PR.properties(mol, omega, X, origin=com)
    assert np.all(f > 0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    M = np.diag([1.0, 1.0, -1.0])  # mirror z -> -z
    for T, sign in ((Q, 1.0), (M, -1.0), (Q @ M, -1.0)):
        m2 = _transform(mol, T)
        mu2, mm2, f2, R2 = PR.properties(m2, omega, X, origin=T @ com)
        assert np.allclose(mu2, mu @ T.T, atol=1e-11)
        assert np.allclose(f2, f, rtol=1e-11, atol=1e-15)
        assert np.allclose(R2, sign * Rr, rtol=1e-9, atol=1e-14)  # pseudoscalar
    # a translated molecule with the origin moved along gives the same strengths
    m3 = _transform(mol, np.eye(3))
    m3.coords = mol.coords + np.array([3.0, -2.0, 1.0])
    _, _, f3, R3 = PR.properties(m3, omega, X, origin=com + np.array([3.0, -2.0, 1.0]))
    assert np.allclose(f3, f, rtol=1e-10) and np.allclose(R3, Rr, rtol=1e-8, atol=1e-14)


def test_spectrum_area_and_peak():
    omega = np.array([0.2, 0.3])
    s = np.array([0.7, 0.1])
    g = 0.05 / R.HARTREE_TO_EV
    E = np.linspace(-40.0, 40.0, 2_000_001)
    S = PR.spectrum(E, omega, s, g)
    area = np.sum(S) * (E[1] - E[0])
    assert abs(area - s.sum()) < 2e-3 * s.sum()  # Lorentzian tails beyond +-40 Ha carry ~1e-5
    peak = PR.spectrum(np.array([0.2]), omega[:1], s[:1], g)[0]
    assert abs(peak - s[0] / (math.pi * g)) < 1e-12 * peak
