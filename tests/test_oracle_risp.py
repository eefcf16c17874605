"""Pins of the oracle's TDA-risp matrix, factors, product and eigensolvers.

The brute-force reference assembles A element by element from 4-index AO integrals built with the
explicit inverse of the metric, (mu nu|P)(P|Q)^-1(Q|kappa lambda), transformed to the MO basis by a
separate 4-index contraction, with the window applied by explicit membership tests (eq. TDA-risp,
eq. TDDFT-axs_approx_integral, eq. K_mia_RSH and the exchange-space window).
"""
import numpy as np
import pytest

import synth
from oracle import integrals as I
from oracle import risp as R

H2EV = 27.211386245988


def tiny_molecule(seed=7):
    """3 C + 2 H, a few bohr apart; nao = 37, nocc = 7, nvir = 30."""
    rng = np.random.default_rng(seed)
    C = np.array([[0.0, 0.0, 0.0], [1.42, 0.1, -0.05], [2.1, 1.25, 0.2]]) + rng.uniform(-0.1, 0.1, (3, 3))
    H = np.array([[-0.6, -0.9, 0.3], [2.9, 1.6, -0.7]])
    ss = np.random.SeedSequence(seed).spawn(2)
    return synth.make_system(C, H, np.random.default_rng(ss[0]), np.random.default_rng(ss[1]), seed, "tiny5")


def brute_A(mol, prm):
    auxJ, auxK = R.select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    C = mol.mo_coeff
    o = mol.nocc
    v = C.shape[1] - o
    e = mol.mo_energy
    # Coulomb: (mu nu|k l)_RI with the explicit inverse
    V3 = I.int3c(mol.coords, mol.shells, auxJ)
    Vinv = np.linalg.inv(I.int2c(mol.coords, auxJ))
    ao4 = np.einsum("mnP,PQ,klQ->mnkl", V3, Vinv, V3, optimize=True)
    mo4 = np.einsum("mnkl,mp,nq,kr,ls->pqrs", ao4, C, C, C, C, optimize=True)
    # exchange operator J^ = c_x/r + beta erf(omega r)/r, one RI in its own metric
    V3x = prm.c_x * I.int3c(mol.coords, mol.shells, auxK) + prm.beta * I.int3c(mol.coords, mol.shells, auxK, prm.omega)
    V2x = prm.c_x * I.int2c(mol.coords, auxK) + prm.beta * I.int2c(mol.coords, auxK, prm.omega)
    ao4x = np.einsum("mnP,PQ,klQ->mnkl", V3x, np.linalg.inv(V2x), V3x, optimize=True)
    mo4x = np.einsum("mnkl,mp,nq,kr,ls->pqrs", ao4x, C, C, C, C, optimize=True)
    occK, virK = R.window_sets(e, o, prm.window_ev, prm.window_mode)
    occK, virK = set(occK.tolist()), set(virK.tolist())
    A = np.zeros((o * v, o * v))
    for i in range(o):
        for a in range(v):
            for j in range(o):
                for b in range(v):
                    val = 2.0 * mo4[i, o + a, j, o + b]
                    if i == j and a == b:
                        val += e[o + a] - e[i]
                    if i in occK and j in occK and a in virK and b in virK:
                        val -= mo4x[i, j, o + a, o + b]
                    A[i * v + a, j * v + b] = val
    return A


@pytest.fixture(scope="module")
def tiny():
    return tiny_molecule()


@pytest.mark.parametrize("window", [40.0, 25.0])
def test_dense_A_matches_brute_force(tiny, window):
    prm = R.Params(window_ev=window, schwarz_tau=0.0)
    F = R.build_factors(tiny, prm)
    A = R.dense_A(F)
    Ab = brute_A(tiny, prm)
    assert np.abs(A - Ab).max() <= 1e-12 * np.abs(Ab).max()
    if window == 25.0:  # the window must actually cut something in this case
        assert len(F.virK) < F.nvir


def test_exchange_factor_slices_symmetric(tiny):
    # (pq|P) is symmetric in (p, q), and the metric split acts on P only, so every slice of the
    # windowed exchange factors is symmetric; the GPU build relies on it for T_ab (it forms the
    # upper triangle and mirrors it)
    F = R.build_factors(tiny, R.Params())
    for B in (F.Bx_ab, F.Bx_ij):
        assert B.shape[0] > 0 and B.shape[1] > 1
        assert np.abs(B - np.swapaxes(B, 1, 2)).max() <= 1e-13 * np.abs(B).max()


def test_A_symmetric_and_coulomb_psd(tiny):
    F = R.build_factors(tiny, R.Params(schwarz_tau=0.0))
    A = R.dense_A(F)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    Bf = F.B_ia.reshape(F.B_ia.shape[0], -1)
    J = 2.0 * Bf.T @ Bf
    lam = np.linalg.eigvalsh(J)
    assert lam.min() >= -1e-12 * lam.max()


def test_factor_split_equals_explicit_inverse(tiny):
    auxJ, _ = R.select_aux(tiny.Z, tiny.aux_radius)
    V3 = I.int3c(tiny.coords, tiny.shells, auxJ)
    V2 = I.int2c(tiny.coords, auxJ)
    B, L = R.cholesky_split(V3.transpose(2, 0, 1).copy(), V2)
    assert np.abs(L @ L.T - V2).max() <= 1e-14 * np.abs(V2).max()
    lhs = np.einsum("Pmn,Pkl->mnkl", B, B)
    rhs = np.einsum("mnP,PQ,klQ->mnkl", V3, np.linalg.inv(V2), V3)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_window_infinite_equals_untruncated_and_zero_removes_exchange(tiny):
    o = tiny.nocc
    full = R.dense_A(R.build_factors(tiny, R.Params(window_ev=1e9, schwarz_tau=0.0)))
    # untruncated exchange coded separately: (ij|ab) over all orbitals
    F = R.build_factors(tiny, R.Params(window_ev=1e9, schwarz_tau=0.0))
    assert len(F.occK) == o and len(F.virK) == F.nvir
    noex = R.dense_A(R.build_factors(tiny, R.Params(c_x=0.0, beta=0.0, schwarz_tau=0.0)))
    K = np.einsum("Pij,Pab->iajb", F.Bx_ij, F.Bx_ab).reshape(full.shape)
    assert np.abs((noex - K) - full).max() <= 1e-13 * np.abs(full).max()
    zero = R.dense_A(R.build_factors(tiny, R.Params(window_ev=0.0, schwarz_tau=0.0)))
    assert np.abs(zero - noex).max() <= 1e-14 * np.abs(noex).max()


def test_no_coulomb_no_exchange_gives_orbital_gaps(tiny):
    F = R.build_factors(tiny, R.Params(c_x=0.0, beta=0.0, schwarz_tau=0.0))
    F.B_ia[...] = 0.0
    w = np.linalg.eigvalsh(R.dense_A(F))
    assert np.array_equal(w, np.sort(F.de.ravel())) or np.abs(w - np.sort(F.de.ravel())).max() <= 1e-15


def test_weyl_bound_without_exchange(tiny):
    F = R.build_factors(tiny, R.Params(c_x=0.0, beta=0.0, schwarz_tau=0.0))
    w = np.linalg.eigvalsh(R.dense_A(F))
    d = np.sort(F.de.ravel())
    assert np.all(w >= d - 1e-13)


def test_energies_translation_and_aux_scaling_invariant(tiny):
    prm = R.Params(schwarz_tau=0.0)
    w0 = np.linalg.eigvalsh(R.dense_A(R.build_factors(tiny, prm)))[:6]
    shifted = tiny_molecule()
    shifted.coords = shifted.coords + np.array([2.0, -1.0, 0.5])
    w1 = np.linalg.eigvalsh(R.dense_A(R.build_factors(shifted, prm)))[:6]
    assert np.abs(w0 - w1).max() <= 1e-12
    # RI is invariant under a nonsingular rescaling of the auxiliary functions
    orig = R.select_aux

    def scaled(Z, rad, theta=0.2, h=False):
        J, K = orig(Z, rad, theta, h)
        return ([(a, l, e, 1.7 + 0.1 * k) for k, (a, l, e, _) in enumerate(J)],
                [(a, l, e, 0.6 + 0.2 * k) for k, (a, l, e, _) in enumerate(K)])

    R.select_aux = scaled
    try:
        w2 = np.linalg.eigvalsh(R.dense_A(R.build_factors(tiny, prm)))[:6]
    finally:
        R.select_aux = orig
    assert np.abs(w0 - w2).max() <= 1e-12


def test_rsh_split_equals_combined_when_beta_zero_or_omega_large(tiny):
    for kw in (dict(beta=0.0), dict(omega=1e6)):
        a = R.dense_A(R.build_factors(tiny, R.Params(rsh_mode="combined", schwarz_tau=0.0, **kw)))
        b = R.dense_A(R.build_factors(tiny, R.Params(rsh_mode="split", schwarz_tau=0.0, **kw)))
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()
    a = R.dense_A(R.build_factors(tiny, R.Params(rsh_mode="combined", schwarz_tau=0.0)))
    b = R.dense_A(R.build_factors(tiny, R.Params(rsh_mode="split", schwarz_tau=0.0)))
    assert np.abs(a - b).max() > 1e-8  # the two readings differ in general


def test_sigma_equals_dense_product(tiny):
    F = R.build_factors(tiny, R.Params(window_ev=25.0))
    A = R.dense_A(F)
    X = synth.random_trial_vectors(5, F.nocc, F.nvir, 3)
    S = R.sigma(F, X)
    ref = (A @ X.reshape(5, -1).T).T.reshape(S.shape)
    assert np.abs(S - ref).max() <= 1e-13 * np.abs(ref).max()
    # bilinear symmetry and linearity
    Y = synth.random_trial_vectors(5, F.nocc, F.nvir, 4)
    assert abs(np.sum(Y * R.sigma(F, X)) - np.sum(X * R.sigma(F, Y))) <= 1e-13
    assert np.abs(R.sigma(F, 2 * X - Y) - (2 * S - R.sigma(F, Y))).max() <= 1e-13


@pytest.mark.parametrize("tau", [0.0, 1e-10])
def test_coulomb_ao_route_equals_stored_factor_route(tiny, tau):
    # two different orders of the same contraction: C_occ^T [(mu nu|P)(P|Q)^-1(Q|kl)] C_vir applied
    # to the AO density C_occ X C_vir^T, against 2 B_ia^T (B_ia X) from the Cholesky-split factors
    prm = R.Params(schwarz_tau=tau)
    F = R.build_factors(tiny, prm)
    X = synth.random_trial_vectors(4, F.nocc, F.nvir, 9)
    Bf = F.B_ia.reshape(F.B_ia.shape[0], -1)
    ref = 2.0 * (Bf.T @ (Bf @ X.reshape(4, -1).T)).T.reshape(X.shape)
    got = R.coulomb_ao(tiny, X, prm)
    # rounding of the two orders differs by ~1e-12 relative (the metric solve amplifies it); a
    # dropped or transposed term changes the result at order one
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    # the whole product through the AO route equals the dense matrix
    S = R.sigma_ao(F, tiny, X, prm)
    dense = (R.dense_A(F) @ X.reshape(4, -1).T).T.reshape(X.shape)
    assert np.abs(S - dense).max() <= 1e-11 * np.abs(dense).max()


def test_coulomb_ao_route_symmetric_psd_and_linear(tiny):
    # J is a Gram matrix in the Coulomb metric: symmetric and positive semi-definite, and linear in X
    prm = R.Params()
    F = R.build_factors(tiny, prm)
    X = synth.random_trial_vectors(3, F.nocc, F.nvir, 21)
    Y = synth.random_trial_vectors(3, F.nocc, F.nvir, 22)
    JX, JY = R.coulomb_ao(tiny, X, prm), R.coulomb_ao(tiny, Y, prm)
    scale = np.abs(JX).max() * np.abs(Y).max() * Y[0].size
    for k in range(3):
        assert abs(np.sum(Y[k] * JX[k]) - np.sum(X[k] * JY[k])) <= 1e-13 * scale
        assert np.sum(X[k] * JX[k]) >= 0.0
    assert np.abs(R.coulomb_ao(tiny, 2 * X - Y, prm) - (2 * JX - JY)).max() <= 1e-11 * np.abs(JX).max()
    # a zero trial vector gives zero
    assert np.all(R.coulomb_ao(tiny, np.zeros_like(X[:1]), prm) == 0.0)


def test_diag_A_equals_dense_diagonal(tiny):
    for prm in (R.Params(window_ev=25.0), R.Params(rsh_mode="split")):
        F = R.build_factors(tiny, prm)
        ref = np.diag(R.dense_A(F)).reshape(F.nocc, F.nvir)
        assert np.abs(R.diag_A(F) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_window_sets_by_hand():
    e = np.array([-2.0, -40.0 / H2EV, -39.0 / H2EV, -0.3, 0.1, 1.0, 40.0 / H2EV, 1.5, 3.0])
    occ, vir = R.window_sets(e, 4, 40.0)
    assert occ.tolist() == [2, 3]  # -40 eV exactly is not kept (strict)
    assert vir.tolist() == [0, 1]  # 40 eV exactly is not kept; 1.5 Ha = 40.8 eV is dropped
    # frontier: LUMO = 0.1 Ha, HOMO = -0.3 Ha; (0.1 - e_i) eV = 41.7 for i = 2, 10.9 for i = 3;
    # (e_a + 0.3) eV = 10.9, 35.4, 48.2, 49.0, 89.8
    occ, vir = R.window_sets(e, 4, 40.0, "frontier")
    assert occ.tolist() == [3] and vir.tolist() == [0, 1]
    occ, vir = R.window_sets(e, 4, 1e9)
    assert occ.tolist() == [0, 1, 2, 3] and vir.tolist() == [0, 1, 2, 3, 4]


def test_select_aux_counts():
    mol = synth.make_config0()
    J, K = R.select_aux(mol.Z, mol.aux_radius)
    nC = int(np.sum(mol.Z == 6))
    assert sum(1 if l == 0 else 3 for (_, l, _, _) in J) == 4 * nC == 48
    assert len(K) == nC and all(l == 0 for (_, l, _, _) in K)
    assert all(mol.Z[a] == 6 for (a, _, _, _) in J)
    e = J[0][2]
    assert e == pytest.approx(0.2 / (0.76 * synth.ANGSTROM_TO_BOHR) ** 2)
    J2, K2 = R.select_aux(mol.Z, mol.aux_radius, h_in_aux=True)
    assert len(K2) == mol.natm


def test_screening_limits_and_monotone():
    mol = tiny_molecule()
    auxJ, _ = R.select_aux(mol.Z, mol.aux_radius)
    nsh = len(mol.shells)
    p0, _, _ = R.schwarz_pairs(mol.coords, mol.shells, auxJ, 0.0)
    assert len(p0) == nsh * (nsh + 1) // 2
    prev = None
    for tau in (1e-12, 1e-6, 1e-3, 1e-1):
        p, mask, ratio = R.schwarz_pairs(mol.coords, mol.shells, auxJ, tau)
        s = set(map(tuple, p.tolist()))
        if prev is not None:
            assert s <= prev
        prev = s
    assert len(prev) < len(p0)


def test_davidson_matches_eigh_config0():
    mol = synth.make_config0()
    F = R.build_factors(mol, R.Params())
    w, U = R.lowest_eigh(R.dense_A(F), 5)
    r = R.davidson(F, 5, tol=1e-7)
    assert r.converged
    assert np.abs(r.energies - w).max() <= 1e-10
    for k in range(5):
        assert abs(abs(np.dot(r.vectors[k], U[k])) - 1.0) <= 1e-8
    r2 = R.davidson(F, 5, tol=1e-7, max_space=30)
    assert r2.converged and r2.restarts > 0
    assert np.abs(r2.energies - w).max() <= 1e-10


def test_screening_changes_energies_negligibly():
    mol = synth.make_config0()
    A1 = R.dense_A(R.build_factors(mol, R.Params(schwarz_tau=1e-10)))
    A0 = R.dense_A(R.build_factors(mol, R.Params(schwarz_tau=0.0)))
    w1 = np.linalg.eigvalsh(A1)[:5]
    w0 = np.linalg.eigvalsh(A0)[:5]
    assert np.abs(w1 - w0).max() <= 1e-8


def test_davidson_diag_preconditioner_matches_eigh_config0():
    """The diagonal-of-A guess and preconditioner path (the one that wrote the 300-atom reference
    energies) against dense eigh, with and without restarts (Davidson section: the converged
    eigenpairs do not depend on the guess or the preconditioner; a guess that misses a low root or a
    wrong ordering of the guess shows up as a wrong energy here)."""
    mol = synth.make_config0()
    F = R.build_factors(mol, R.Params())
    A = R.dense_A(F)
    w, U = R.lowest_eigh(A, 5)
    d = R.diag_A(F)
    # the diagonal differs from the plain gaps, so this path is really a different guess
    assert np.abs(d - F.de).max() > 1e-3
    assert not np.array_equal(np.argsort(d.ravel(), kind="stable")[:10], np.argsort(F.de.ravel(), kind="stable")[:10])
    for max_space in (None, 30):
        r = R.davidson(F, 5, tol=1e-7, diag=d, max_space=max_space)
        assert r.converged
        if max_space == 30:
            assert r.restarts > 0
        assert np.abs(r.energies - w).max() <= 1e-10
        for k in range(5):
            assert abs(abs(np.dot(r.vectors[k], U[k])) - 1.0) <= 1e-8
            # a true eigenpair of the dense matrix
            res = A @ r.vectors[k] - r.energies[k] * r.vectors[k]
            assert np.linalg.norm(res) <= 1e-7


def brute_A_split(mol, prm):
    """A with the split reading of the range-separated exchange assembled from 4-index AO integrals:
    c_x (mu nu|P)(P|Q)^-1(Q|kl) + beta (mu nu|erf|P)(P|erf|Q)^-1(Q|erf|kl), each block inverting its
    own metric (eq. RSH with one RI per operator)."""
    auxJ, auxK = R.select_aux(mol.Z, mol.aux_radius, prm.theta, prm.h_in_aux)
    C = mol.mo_coeff
    o = mol.nocc
    v = C.shape[1] - o
    e = mol.mo_energy
    V3 = I.int3c(mol.coords, mol.shells, auxJ)
    ao4 = np.einsum("mnP,PQ,klQ->mnkl", V3, np.linalg.inv(I.int2c(mol.coords, auxJ)), V3, optimize=True)
    mo4 = np.einsum("mnkl,mp,nq,kr,ls->pqrs", ao4, C, C, C, C, optimize=True)
    V3p = I.int3c(mol.coords, mol.shells, auxK)
    V3e = I.int3c(mol.coords, mol.shells, auxK, prm.omega)
    ao4x = (prm.c_x * np.einsum("mnP,PQ,klQ->mnkl", V3p, np.linalg.inv(I.int2c(mol.coords, auxK)), V3p, optimize=True)
            + prm.beta * np.einsum("mnP,PQ,klQ->mnkl", V3e, np.linalg.inv(I.int2c(mol.coords, auxK, prm.omega)), V3e,
                                   optimize=True))
    mo4x = np.einsum("mnkl,mp,nq,kr,ls->pqrs", ao4x, C, C, C, C, optimize=True)
    occK, virK = R.window_sets(e, o, prm.window_ev, prm.window_mode)
    wo = np.zeros(o, bool)
    wo[occK] = True
    wv = np.zeros(v, bool)
    wv[virK] = True
    A = 2.0 * mo4[:o, o:, :o, o:].copy()
    A[np.arange(o)[:, None], np.arange(v)[None, :], np.arange(o)[:, None], np.arange(v)[None, :]] += \
        e[None, o:] - e[:o, None]
    Kx = mo4x[:o, :o, o:, o:].transpose(0, 2, 1, 3)  # [i][a][j][b] = (ij|J^|ab)
    win = wo[:, None, None, None] & wv[None, :, None, None] & wo[None, None, :, None] & wv[None, None, None, :]
    A -= np.where(win, Kx, 0.0)
    return A.reshape(o * v, o * v)


def test_dense_A_split_rsh_matches_brute_force(tiny):
    """Split reading with both parts present (c_x and beta non-zero, finite omega): each RI block in
    its own metric. Inverting the plain metric for the erf block, or the combined metric for both,
    changes A at order 1e-3 relative here, far above the 1e-12 bar."""
    prm = R.Params(rsh_mode="split", window_ev=25.0, schwarz_tau=0.0)
    assert prm.c_x != 0.0 and prm.beta != 0.0 and 0.0 < prm.omega < 10.0
    F = R.build_factors(tiny, prm)
    A = R.dense_A(F)
    Ab = brute_A_split(tiny, prm)
    assert np.abs(A - Ab).max() <= 1e-12 * np.abs(Ab).max()
    # the erf block in the plain metric is a different matrix (so the test can tell them apart)
    auxJ, auxK = R.select_aux(tiny.Z, tiny.aux_radius)
    V3e = I.int3c(tiny.coords, tiny.shells, auxK, prm.omega)
    wrong = np.einsum("mnP,PQ,klQ->mnkl", V3e, np.linalg.inv(I.int2c(tiny.coords, auxK)), V3e)
    right = np.einsum("mnP,PQ,klQ->mnkl", V3e, np.linalg.inv(I.int2c(tiny.coords, auxK, prm.omega)), V3e)
    assert np.abs(wrong - right).max() > 1e-6 * np.abs(right).max()
    # and the combined reading differs from the split one at these parameters
    Ac = R.dense_A(R.build_factors(tiny, R.Params(rsh_mode="combined", window_ev=25.0, schwarz_tau=0.0)))
    assert np.abs(Ac - Ab).max() > 1e-6 * np.abs(Ab).max()


def test_schwarz_keep_rule_by_hand():
    """Keep rule of the screening (section on on-the-fly Coulomb evaluation, screened AO pairs):
    (A >= B) is kept iff Q_AB * max_P sqrt((P|P)) >= tau with Q_AB from the four-centre diagonal and
    the maximum over the Coulomb (s + p) auxiliary basis. tau is set to exactly the value of one
    same-shell pair, so the list separates >= from >, drops a same-shell pair and a p-s pair, and
    drops more than 10 % of the pairs. Dropped pairs must satisfy the Schwarz bound on the actual
    three-centre integrals."""
    mol = tiny_molecule()
    sh = mol.shells
    nsh = len(sh)
    auxJ0, auxK = R.select_aux(mol.Z, mol.aux_radius)
    # In the production basis s and p share an exponent and the s function has the largest (P|P),
    # so the Coulomb and exchange maxima coincide; more diffuse p functions here make them differ, so the
    # test can tell which basis the rule uses.
    auxJ = [(a, l, e * (0.1 if l == 1 else 1.0), c) for (a, l, e, c) in auxJ0]
    assert np.sqrt(np.max(np.diag(I.int2c(mol.coords, auxJ0)))) == np.sqrt(np.max(np.diag(I.int2c(mol.coords, auxK))))
    Qab = I.schwarz_diag(mol.coords, sh)
    qJ = float(np.sqrt(np.max(np.diag(I.int2c(mol.coords, auxJ)))))
    qK = float(np.sqrt(np.max(np.diag(I.int2c(mol.coords, auxK)))))
    assert qJ > qK
    diag_vals = sorted(set(Qab[a, a] * qJ for a in range(nsh)))
    tau = diag_vals[1]  # the second-smallest same-shell value: the smallest same-shell pairs are dropped

    def by_hand(q, strict=False):
        out = []
        for a in range(nsh):
            for b in range(a + 1):
                v = Qab[a, b] * q
                if (v > tau) if strict else (v >= tau):
                    out.append((a, b))
        return out

    want = by_hand(qJ)
    got, mask, ratio = R.schwarz_pairs(mol.coords, sh, auxJ, tau)
    assert [tuple(p) for p in got.tolist()] == want
    dropped = [(a, b) for a in range(nsh) for b in range(a + 1) if (a, b) not in set(want)]
    npair = nsh * (nsh + 1) // 2
    assert 0.1 * npair <= len(dropped) < npair
    assert any(a == b for a, b in dropped)
    assert any(sh[a][1] != sh[b][1] for a, b in dropped)  # a p-s pair
    # plausible mistakes give different lists at this tau
    assert by_hand(qJ, strict=True) != want          # '>' instead of '>='
    assert by_hand(qK) != want                        # exchange (s-only) auxiliary maximum
    assert [(a, b) for a in range(nsh) for b in range(a + 1) if Qab[a, b] >= tau] != want  # Q_AB alone
    # every dropped pair's integrals are below tau in magnitude (Schwarz inequality)
    V3 = I.int3c(mol.coords, sh, auxJ)
    off, nf = I.shell_offsets(sh)
    off = off + [nf]
    for a, b in dropped:
        blk = V3[off[a]:off[a + 1], off[b]:off[b + 1], :]
        assert np.abs(blk).max() < tau
    # the factor build screens with the Coulomb basis
    F = R.build_factors(mol, R.Params(schwarz_tau=1e-3))
    ref, _, _ = R.schwarz_pairs(mol.coords, sh, auxJ0, 1e-3)
    assert np.array_equal(F.pairs, ref) and len(ref) < npair


def test_sigma_rows_equals_full_sigma():
    """sigma_rows (rows of sigma from the integrals, no stored factor; used for the full-size sampled
    references) equals the stored-factor sigma at the same rows, inside and outside the window, for
    the 20-atom molecule, with the default and a 10 eV window."""
    mol = synth.make_config0()
    X = synth.random_trial_vectors(3, mol.nocc, mol.nvir, 7)
    nv = mol.nvir
    for window in (40.0, 10.0):
        prm = R.Params(window_ev=window)
        F = R.build_factors(mol, prm)
        nvk = len(F.virK)
        rows = np.array([0, 5, nvk - 1, nvk, nv - 1, 3 * nv + 90, (mol.nocc - 1) * nv + nvk - 1,
                         mol.nocc * nv - 1])
        want = R.sigma(F, X).reshape(3, -1)[:, rows]
        got = R.sigma_rows(mol, X, rows, prm)
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
        # the exchange part is present (dropping it changes the in-window rows)
        F0 = R.build_factors(mol, R.Params(window_ev=window, c_x=0.0, beta=0.0))
        assert np.abs(R.sigma(F0, X).reshape(3, -1)[:, rows] - want).max() > 1e-4 * np.abs(want).max()
