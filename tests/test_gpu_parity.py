"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bit-exact: window index sets and screened pair lists. FP64 integrals: 1e-12 relative. Factors and
sigma: element by element. Excitation energies: 1e-6 Ha (FP64 / FP32 paths), 2e-5 Ha (BF16 with the
FP32 correction pass).
"""
import numpy as np
import pytest

import synth
from oracle import integrals as OI
from oracle import risp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mol0():
    return synth.make_config0()


@pytest.fixture(scope="module")
def tiny():
    from tests.test_oracle_risp import tiny_molecule
    return tiny_molecule()


@pytest.fixture(scope="module")
def oracle0(mol0):
    return R.build_factors(mol0, R.Params())


# Element-wise bar for BF16 sigma, relative to the largest element. Every stored factor element
# carries a relative rounding error of at most u = 2^-8 (8-bit significand) after its exact
# power-of-two scale; the products accumulate in FP32, so an element of sigma is a sum of many
# products whose rounding errors are independent and largely cancel: the measured error is ~1e-4 of
# the largest element. The bar, 1e-3 (u / 4), is ten times that: a wrong power-of-two scale on one
# auxiliary slice (a factor 2 on 1/48 of the Coulomb sum at 20 atoms) or a dropped small term moves
# sigma by ~1e-2 and fails it.
BF16_SIGMA_TOL = 1e-3


def _params(**kw):
    import paper_2603_29257_amd as P
    return P.Params(**kw)


# ---------------------------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------------------------
def test_window_sets_bit_exact(ctx, mol0):
    import paper_2603_29257_amd as P
    cases = [(mol0.mo_energy, mol0.nocc, 40.0)]
    H2EV = 27.211386245988
    e = np.array([-2.0, -40.0 / H2EV, -39.0 / H2EV, -0.3, 0.1, 1.0, 40.0 / H2EV, 1.5, 3.0])
    cases += [(e, 4, 40.0), (e, 4, 0.0), (e, 4, 1e9), (mol0.mo_energy, mol0.nocc, 16.0)]
    for (ee, no, w) in cases:
        for mode, name in ((P.WIN_ABSOLUTE, "absolute"), (P.WIN_FRONTIER, "frontier")):
            o, v = ctx.window(ee, no, w, mode)
            ro, rv = R.window_sets(ee, no, w, name)
            assert o.tolist() == ro.tolist() and v.tolist() == rv.tolist(), (w, name)


@pytest.mark.parametrize("which", ["tiny", "grid20"])
def test_screening_bit_exact(ctx, which, tiny, mol0):
    import paper_2603_29257_amd as P
    mol = tiny if which == "tiny" else mol0
    sysc = P.System(mol)
    auxJ, _ = R.select_aux(mol.Z, mol.aux_radius)
    for tau in (1e-10, 1e-4, 1e-2):
        ref, _, ratio = R.schwarz_pairs(mol.coords, mol.shells, auxJ, tau)
        # margin audit: no pair so close to the threshold that rounding could decide it
        assert np.min(np.abs(ratio - 1.0)) > 1e-12
        got = ctx.screen(sysc, auxJ, tau)
        assert got.shape == ref.shape and np.array_equal(got, ref), tau


def test_select_aux_matches_oracle(ctx, mol0):
    import paper_2603_29257_amd as P
    J, K = ctx.select_aux(P.System(mol0), _params())
    rJ, rK = R.select_aux(mol0.Z, mol0.aux_radius)
    assert J == rJ and K == rK


@pytest.mark.parametrize("omega", [0.0, 0.2])
def test_int2c_fp64(ctx, mol0, omega):
    import paper_2603_29257_amd as P
    auxJ, _ = R.select_aux(mol0.Z, mol0.aux_radius)
    got = ctx.int2c(P.System(mol0), auxJ, omega)
    ref = OI.int2c(mol0.coords, auxJ, omega if omega > 0 else None)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("omega", [0.0, 0.2, 1.7])
def test_int3c_fp64_tiny_all_classes(ctx, tiny, omega):
    import paper_2603_29257_amd as P
    auxJ, _ = R.select_aux(tiny.Z, tiny.aux_radius)
    got = ctx.int3c(P.System(tiny), auxJ, omega=omega)
    ref = OI.int3c(tiny.coords, tiny.shells, auxJ, omega if omega > 0 else None).transpose(2, 0, 1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_int3c_fp64_screened_config0(ctx, mol0):
    import paper_2603_29257_amd as P
    auxJ, _ = R.select_aux(mol0.Z, mol0.aux_radius)
    pairs, mask, _ = R.schwarz_pairs(mol0.coords, mol0.shells, auxJ, 1e-10)
    sel = [0, 1, 7, 22, 23]  # s and p shells at several atoms, a ragged subset
    got = np.concatenate([ctx.int3c(P.System(mol0), auxJ, k, k + 1, 0.0, 1e-10) for k in sel])
    ref = OI.int3c(mol0.coords, mol0.shells, auxJ, None, mask, sel).transpose(2, 0, 1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------------------------------------
# factors, sigma, eigenpairs at the 20-atom size
# ---------------------------------------------------------------------------------------------
def _gpu_factors(ctx, mol, **kw):
    import paper_2603_29257_amd as P
    sysc = P.System(mol)
    return ctx.build_factors(sysc, _params(**kw))


def test_factors_fp64_elementwise(ctx, mol0, oracle0):
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.FP64)
    assert F.naux_j == oracle0.B_ia.shape[0] and F.naux_k == oracle0.Bx_ij.shape[0]
    assert F.nocc_k == len(oracle0.occK) and F.nvir_k == len(oracle0.virK)
    assert F.npair == len(oracle0.pairs)
    Tia = F.tensor("t_ia").cpu().numpy()
    Tij = F.tensor("t_ij").cpu().numpy().transpose(1, 0, 2)
    Tab = F.tensor("t_ab").cpu().numpy()
    for got, ref, name in ((Tia, oracle0.B_ia, "ia"), (Tij, oracle0.Bx_ij, "ij"), (Tab, oracle0.Bx_ab, "ab")):
        err = np.abs(got - ref).max() / np.abs(ref).max()
        _print(f"T_{name} FP64 max rel err {err:.3e}")
        # rounding-order differences (integral algorithm, summation order) of ~1e-14 are amplified by
        # the metric (sqrt(cond) ~ 1.5e3) and the cancellation of the MO transform (~1e3)
        assert err <= 5e-8, name
    assert F.tensor("occ_k").cpu().numpy().tolist() == oracle0.occK.tolist()
    assert F.tensor("vir_k").cpu().numpy().tolist() == oracle0.virK.tolist()
    F.free()


def test_factors_fp32_and_bf16_storage(ctx, mol0, oracle0):
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.FP32)
    Tia = F.tensor("t_ia").cpu().numpy().astype(np.float64)
    err = np.abs(Tia - oracle0.B_ia).max() / np.abs(oracle0.B_ia).max()
    _print(f"T_ia FP32 max rel err {err:.3e}")
    assert err <= 1e-6
    F.free()
    F = _gpu_factors(ctx, mol0, precision=P.BF16)
    s = F.tensor("scale_ia").cpu().numpy().astype(np.float64)
    Tia = F.tensor("t_ia").float().cpu().numpy().astype(np.float64) * s[:, None, None]
    assert np.all(np.log2(s) == np.round(np.log2(s)))  # powers of two
    rowmax = np.abs(oracle0.B_ia).reshape(len(s), -1).max(axis=1)
    assert np.all(s >= rowmax) and np.all(s < 2 * rowmax)
    err = np.abs(Tia - oracle0.B_ia).max() / np.abs(oracle0.B_ia).max()
    _print(f"T_ia BF16 max rel err {err:.3e}")
    assert err <= 2 ** -8
    # stored rows are padded to 8 elements (16 bytes) with zeros
    d = F.desc
    assert d.ld_ia % 8 == 0 and d.ld_ia - 8 < d.nocc * d.nvir <= d.ld_ia
    assert d.ld_ij % 8 == 0 and d.ld_ij - 8 < d.nocc_k <= d.ld_ij
    assert d.ld_ab % 8 == 0 and d.ld_ab - 8 < d.nvir_k <= d.ld_ab
    for name, n in (("t_ia", d.nocc * d.nvir), ("t_ij", d.nocc_k), ("t_ab", d.nvir_k), ("t_ij_lo", d.nocc_k),
                    ("t_ab_lo", d.nvir_k)):
        full = F.tensor(name, padded=True).float().cpu().numpy()
        assert np.all(full[..., n:] == 0), name
    # hi + lo BF16 parts of the exchange factors (correction pass): T / scale to about 2^-17
    sk = F.tensor("scale_k").cpu().numpy().astype(np.float64)
    hi = F.tensor("t_ab").float().cpu().numpy().astype(np.float64)
    lo = F.tensor("t_ab_lo").float().cpu().numpy().astype(np.float64)
    ref = oracle0.Bx_ab
    # T_ab's own scale is s_k / s_ij; compare after scaling both parts back with it
    hij = F.tensor("t_ij").float().cpu().numpy().astype(np.float64)  # [i][P][j]
    lij = F.tensor("t_ij_lo").float().cpu().numpy().astype(np.float64)
    sij = np.array([2.0 ** np.ceil(np.log2(np.abs(oracle0.Bx_ij[p]).max())) for p in range(len(sk))])
    sab = sk / sij
    for name, h, l, r, sc in (("t_ab", hi, lo, ref, sab[:, None, None]),
                              ("t_ij", hij.transpose(1, 0, 2), lij.transpose(1, 0, 2), oracle0.Bx_ij, sij[:, None, None])):
        e_hi = np.abs(h * sc - r).max() / np.abs(r).max()
        e_sp = np.abs((h + l) * sc - r).max() / np.abs(r).max()
        _print(f"{name} BF16 hi max rel err {e_hi:.3e}, hi + lo {e_sp:.3e}")
        assert e_hi <= 2 ** -8 and e_sp <= 2 ** -16
    F.free()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_diagonal_of_A(ctx, mol0, oracle0, prec):
    # FP64 diagonal from the FP64 factors in every storage precision (guess and preconditioner)
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec])
    got = F.tensor("diag_a").cpu().numpy()
    ref = R.diag_A(oracle0)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _print(f"diag(A) {prec} max rel err {err:.3e}")
    assert err <= 1e-9
    F.free()
    # the AO route leaves the Coulomb part out
    F = _gpu_factors(ctx, mol0, precision=P.FP64, j_mode=P.J_AO_DIRECT)
    got = F.tensor("diag_a").cpu().numpy()
    Bf = oracle0.B_ia
    ref_ao = ref - 2.0 * np.einsum("Pia,Pia->ia", Bf, Bf)
    assert np.abs(got - ref_ao).max() <= 1e-9 * np.abs(ref_ao).max()
    F.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_factors_chunked_build_identical(ctx, mol0, prec):
    # tiny build chunks (one occupied / window-virtual orbital per chunk) give the same stored factors
    import paper_2603_29257_amd as P
    F1 = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec])
    F2 = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec], build_chunk_kib=16)
    for name in ("t_ia", "t_ij", "t_ab", "diag_a") + (("scale_ia", "scale_k") if prec == "bf16" else ()):
        a = F1.tensor(name, padded=True).double().cpu().numpy()
        b = F2.tensor(name, padded=True).double().cpu().numpy()
        assert np.array_equal(a, b), name
    F1.free()
    F2.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_t_ab_slices_exactly_symmetric(ctx, mol0, prec):
    # T^P_ab is symmetric in (a, b): the build forms the upper triangle and mirrors the strict lower
    # one, so every stored slice (BF16: both halves) equals its transpose bit for bit, whether the
    # window virtuals are transformed in one chunk or one orbital at a time
    import paper_2603_29257_amd as P
    for kib in (0, 16):
        F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec], build_chunk_kib=kib)
        for name in ("t_ab", "t_ab_lo") if prec == "bf16" else ("t_ab",):
            t = F.tensor(name).double().cpu().numpy()
            assert t.shape[1] == t.shape[2] == F.nvir_k and t.shape[1] > 1
            assert np.array_equal(t, np.swapaxes(t, 1, 2)), (name, kib)
        F.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("m", [1, 7, 30])
def test_sigma_matches_oracle(ctx, mol0, oracle0, prec, m):
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec])
    X = synth.random_trial_vectors(m, F.nocc, F.nvir, 11)
    ref = R.sigma(oracle0, X)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd = torch.tensor(X, dtype=dt, device=ctx.device)
    got = ctx.sigma(F, Xd).cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _print(f"sigma {prec} m={m} max rel err {err:.3e}")
    tol = {"fp64": 1e-9, "fp32": 2e-6, "bf16": BF16_SIGMA_TOL}[prec]
    assert err <= tol
    F.free()


@pytest.mark.parametrize("m", [40, 70])
def test_sigma_bf16_wide_blocks(ctx, mol0, oracle0, m):
    # more than 32 vectors (two MFMA column tiles in the Coulomb kernels) and more than 64 (the
    # Coulomb passes run in groups of 64)
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.BF16)
    X = synth.random_trial_vectors(m, F.nocc, F.nvir, 17)
    ref = R.sigma(oracle0, X)
    got = ctx.sigma(F, torch.tensor(X, dtype=torch.float32, device=ctx.device)).cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _print(f"sigma bf16 m={m} max rel err {err:.3e}")
    assert err <= BF16_SIGMA_TOL
    # each row depends on its own trial vector only (summation splits may differ with the block size)
    one = ctx.sigma(F, torch.tensor(X[m - 1:m], dtype=torch.float32, device=ctx.device)).cpu().numpy()
    assert np.abs(one[0] - got[m - 1]).max() <= 1e-5 * np.abs(got[m - 1]).max()
    F.free()


def test_sigma_repeatable_after_other_work(ctx, mol0):
    # workspaces grow with earlier calls (the FP32 correction pass); results must not depend on that
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.BF16)
    X = torch.tensor(synth.random_trial_vectors(10, F.nocc, F.nvir, 5), dtype=torch.float32, device=ctx.device)
    s1 = ctx.sigma(F, X).cpu().numpy()
    e1, _, _ = ctx.davidson(F, 5, tol=1e-5)
    s2 = ctx.sigma(F, X).cpu().numpy()
    e2, _, _ = ctx.davidson(F, 5, tol=1e-5)
    assert np.array_equal(s1, s2)
    assert np.array_equal(e1, e2)
    F.free()


def test_sigma_bilinear_symmetry_fp32(ctx, mol0):
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.FP32)
    X = torch.tensor(synth.random_trial_vectors(3, F.nocc, F.nvir, 1), dtype=torch.float32, device=ctx.device)
    Y = torch.tensor(synth.random_trial_vectors(3, F.nocc, F.nvir, 2), dtype=torch.float32, device=ctx.device)
    a = (Y.double() * ctx.sigma(F, X).double()).sum(dim=(1, 2))
    b = (X.double() * ctx.sigma(F, Y).double()).sum(dim=(1, 2))
    assert torch.max(torch.abs(a - b)).item() <= 1e-6
    F.free()


@pytest.mark.parametrize("prec,tol_e", [("fp64", 1e-6), ("fp32", 1e-6), ("bf16", 2e-5)])
def test_davidson_energies_config0(ctx, mol0, oracle0, prec, tol_e):
    import paper_2603_29257_amd as P
    w, U = R.lowest_eigh(R.dense_A(oracle0), 5)
    F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec])
    e, vec, info = ctx.davidson(F, 5, tol=1e-6 if prec == "fp64" else 1e-5)
    _print(f"davidson {prec}: iters {info.iters} restarts {info.restarts} corr {info.correction_iters} "
           f"max |dE| {np.abs(e - w).max():.3e}")
    assert info.converged
    assert np.abs(e - w).max() <= tol_e
    for k in range(5):
        gap = min(abs(w[k] - w[j]) for j in range(5) if j != k)
        if gap >= 1e-4:
            assert abs(abs(np.dot(vec[k].astype(np.float64), U[k])) - 1.0) <= 1e-4
    F.free()


def test_davidson_bf16_stage_alone_vs_oracle(ctx, mol0, oracle0):
    """BF16 products without the FP32 correction pass: the energies carry the BF16 storage error of
    the factors (about 2e-4 Ha on this molecule by the precision study), so the bar is 1e-3 Ha per
    state; a percent-level defect in the BF16 factors (a wrong slice scale) moves the energies by
    more."""
    import paper_2603_29257_amd as P
    w, _ = R.lowest_eigh(R.dense_A(oracle0), 5)
    F = _gpu_factors(ctx, mol0, precision=P.BF16)
    e, _, info = ctx.davidson(F, 5, tol=1e-5, correction_pass=False, allow_notconv=True)
    err = np.abs(e - w)
    _print(f"davidson bf16 stage only: iters {info.iters}, per-state |dE| {err}")
    assert info.correction_iters == 0
    assert err.max() <= 1e-3
    F.free()


def test_davidson_restart_same_answer(ctx, mol0, oracle0):
    import paper_2603_29257_amd as P
    w, _ = R.lowest_eigh(R.dense_A(oracle0), 5)
    F = _gpu_factors(ctx, mol0, precision=P.FP64)
    e, _, info = ctx.davidson(F, 5, tol=1e-7, max_space=30)
    assert info.converged and info.restarts > 0
    assert np.abs(e - w).max() <= 1e-8
    F.free()


# method variants: readings of the exchange operator and window, auxiliary-basis choice
_VARIANTS = {
    "rsh_split": (dict(rsh_mode=1), dict(rsh_mode="split")),
    "window_frontier": (dict(window_mode=1), dict(window_mode="frontier")),
    "window_10ev": (dict(window_ev=10.0), dict(window_ev=10.0)),
    "window_0ev": (dict(window_ev=0.0), dict(window_ev=0.0)),
    "h_in_aux": (dict(h_in_aux=True), dict(h_in_aux=True)),
    "global_hybrid": (dict(beta=0.0), dict(beta=0.0)),
    "no_exchange": (dict(c_x=0.0, beta=0.0), dict(c_x=0.0, beta=0.0)),
}


@pytest.mark.parametrize("variant", sorted(_VARIANTS))
def test_sigma_method_variants_fp64(ctx, mol0, variant):
    import paper_2603_29257_amd as P
    gp, op = _VARIANTS[variant]
    ref_f = R.build_factors(mol0, R.Params(**op))
    F = _gpu_factors(ctx, mol0, precision=P.FP64, **gp)
    assert F.naux_j == ref_f.B_ia.shape[0]
    assert F.nocc_k == len(ref_f.occK) and F.nvir_k == len(ref_f.virK)
    # an empty window keeps no exchange factors on the device
    assert F.naux_k == (ref_f.Bx_ij.shape[0] if F.nocc_k and F.nvir_k else 0)
    X = synth.random_trial_vectors(4, F.nocc, F.nvir, 23)
    ref = R.sigma(ref_f, X)
    got = ctx.sigma(F, torch.tensor(X, dtype=torch.float64, device=ctx.device)).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    dg = np.abs(F.tensor("diag_a").cpu().numpy() - R.diag_A(ref_f)).max() / np.abs(R.diag_A(ref_f)).max()
    _print(f"sigma FP64 {variant}: naux_k {F.naux_k} window {F.nocc_k}x{F.nvir_k} max rel err {err:.3e}, diag {dg:.3e}")
    assert err <= 1e-9 and dg <= 1e-9
    F.free()


# ---------------------------------------------------------------------------------------------
# Coulomb term by the AO-density route (no stored T_ia; integrals regenerated per sigma block)
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("m", [1, 7, 70])
def test_sigma_ao_route_matches_oracle(ctx, mol0, oracle0, prec, m):
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec], j_mode=P.J_AO_DIRECT)
    assert not F.desc.t_ia
    with pytest.raises(ValueError):
        F.tensor("t_ia")
    X = synth.random_trial_vectors(m, F.nocc, F.nvir, 13)
    ref = R.sigma_ao(oracle0, mol0, X)
    dt = torch.float64 if prec == "fp64" else torch.float32
    got = ctx.sigma(F, torch.tensor(X, dtype=dt, device=ctx.device)).cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _print(f"sigma AO route {prec} m={m} max rel err {err:.3e}")
    # the Coulomb term is FP64 in every precision; FP32 and BF16 errors come from the exchange term
    # and the FP32 X / sigma
    tol = {"fp64": 1e-9, "fp32": 2e-6, "bf16": BF16_SIGMA_TOL}[prec]
    assert err <= tol
    F.free()


def test_sigma_ao_route_equals_stored_route_fp64(ctx, mol0):
    import paper_2603_29257_amd as P
    Fm = _gpu_factors(ctx, mol0, precision=P.FP64)
    Fa = _gpu_factors(ctx, mol0, precision=P.FP64, j_mode=P.J_AO_DIRECT)
    X = torch.tensor(synth.random_trial_vectors(5, Fm.nocc, Fm.nvir, 3), dtype=torch.float64, device=ctx.device)
    a = ctx.sigma(Fm, X).cpu().numpy()
    b = ctx.sigma(Fa, X).cpu().numpy()
    err = np.abs(a - b).max() / np.abs(a).max()
    _print(f"sigma AO vs stored route FP64 max rel diff {err:.3e}")
    assert err <= 1e-10
    Fm.free()
    Fa.free()


def test_davidson_ao_route_energies_config0(ctx, mol0, oracle0):
    import paper_2603_29257_amd as P
    w, _ = R.lowest_eigh(R.dense_A(oracle0), 5)
    F = _gpu_factors(ctx, mol0, precision=P.FP32, j_mode=P.J_AO_DIRECT)
    e, _, info = ctx.davidson(F, 5, tol=1e-5)
    _print(f"davidson AO route fp32: iters {info.iters} max |dE| {np.abs(e - w).max():.3e}")
    assert info.converged
    assert np.abs(e - w).max() <= 1e-6
    F.free()


def test_ao_route_rejected_by_serving(ctx, mol0):
    import paper_2603_29257_amd as P
    with pytest.raises(P.RispError):
        ctx.submit(P.System(mol0), _params(j_mode=P.J_AO_DIRECT), 3)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_davidson_spilled_subspace_identical(ctx, mol0, prec):
    # the subspace in pinned host memory runs the same kernels on the same values (a BF16 stage
    # tolerance of 1e-4 keeps that stage long enough to restart in a subspace of 40)
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec])
    e1, v1, i1 = ctx.davidson(F, 5, tol=1e-5, max_space=40, bf16_tol=1e-4)
    e2, v2, i2 = ctx.davidson(F, 5, tol=1e-5, max_space=40, spill=True, bf16_tol=1e-4)
    assert i1.restarts > 0 and i1.iters == i2.iters
    assert np.array_equal(e1, e2) and np.array_equal(v1, v2)
    F.free()


def test_errors_are_reported(ctx, mol0):
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.FP32)
    with pytest.raises(ValueError):
        ctx.sigma(F, torch.zeros((2, 3, 4), device=ctx.device))
    with pytest.raises(P.RispError):
        ctx.davidson(F, 0)
    F.free()
    bad = synth.make_config0()
    bad.nocc = bad.mo_coeff.shape[1]
    with pytest.raises(P.RispError):
        _gpu_factors(ctx, bad)


@pytest.mark.parametrize("m", [7, 70])
def test_sigma_bf16_with_fp32_coulomb(ctx, mol0, oracle0, m):
    # BF16 exchange with the Coulomb term from the FP32 copy of T_ia (bf16_coulomb_fp32): within the
    # BF16 bar, and its Coulomb part equal to the FP32 path's (the exchange-free variant isolates it)
    import paper_2603_29257_amd as P
    F = _gpu_factors(ctx, mol0, precision=P.BF16, bf16_coulomb_fp32=True)
    X = synth.random_trial_vectors(m, F.nocc, F.nvir, 23)
    ref = R.sigma(oracle0, X)
    Xd = torch.tensor(X, dtype=torch.float32, device=ctx.device)
    got = ctx.sigma(F, Xd).cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _print(f"sigma bf16 + FP32 Coulomb m={m} max rel err {err:.3e}")
    assert err <= BF16_SIGMA_TOL
    F.free()
    Fb = _gpu_factors(ctx, mol0, precision=P.BF16, bf16_coulomb_fp32=True, c_x=0.0, beta=0.0)
    Ff = _gpu_factors(ctx, mol0, precision=P.FP32, c_x=0.0, beta=0.0)
    a, b = ctx.sigma(Fb, Xd).cpu().numpy(), ctx.sigma(Ff, Xd).cpu().numpy()
    assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max()
    Fb.free()
    Ff.free()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_davidson_olsen_energies_config0(ctx, mol0, oracle0, prec):
    # Olsen's correction vectors (RISP_DAV_OLSEN) reach the same eigenpairs
    import paper_2603_29257_amd as P
    w, _ = R.lowest_eigh(R.dense_A(oracle0), 5)
    F = _gpu_factors(ctx, mol0, precision=P.PRECISIONS[prec])
    e, _, info = ctx.davidson(F, 5, tol=1e-5, olsen=True)
    _print(f"davidson {prec} with Olsen corrections: iters {info.iters}+{info.correction_iters}, "
           f"max |dE| {np.abs(e - w).max():.3e}")
    assert info.converged
    assert np.abs(e - w).max() <= (1e-6 if prec == "fp32" else 2e-5)
    F.free()


def test_davidson_bf16_correction_basis_both_ways(ctx, mol0, oracle0):
    # the BF16 correction pass with BF16-valued basis vectors (the default: two split products in the
    # first exchange contraction, Rayleigh-Ritz with the basis overlap) and with FP32 basis vectors
    # (RISP_DAV_FP32_BASIS): both reach the oracle's energies and agree with each other
    import paper_2603_29257_amd as P
    w, _ = R.lowest_eigh(R.dense_A(oracle0), 5)
    F = _gpu_factors(ctx, mol0, precision=P.BF16)
    ea, _, ia = ctx.davidson(F, 5, tol=1e-5)
    eb, _, ib = ctx.davidson(F, 5, tol=1e-5, fp32_basis=True)
    _print(f"bf16 correction basis: BF16-valued {ia.correction_iters} steps, FP32 {ib.correction_iters} steps, "
           f"|dE| {np.abs(ea - w).max():.2e} / {np.abs(eb - w).max():.2e}")
    assert ia.converged and ib.converged
    assert np.abs(ea - w).max() <= 2e-5 and np.abs(eb - w).max() <= 2e-5
    assert np.abs(ea - eb).max() <= 1e-6
    F.free()
