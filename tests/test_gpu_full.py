"""Full TDDFT-risp on the GPU (risp_sigma_full, risp_davidson_full through the C ABI) against the
FP64 oracle (oracle/full.py): the (A + B) and (A - B) products element by element, the excitation
energies and the pair equations of the returned amplitudes."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import full as FU
from oracle import risp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD300 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chainring300_oracle.json")


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


def _oracle(mol, window):
    prm = R.Params(window_ev=window)
    F = R.build_factors(mol, prm)
    return F, FU.exchange_ia_factor(mol, prm)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 2e-6)])
@pytest.mark.parametrize("window", [40.0, 10.0])
def test_sigma_full_matches_oracle(ctx, mol0, prec, tol, window):
    import paper_2603_29257_amd as P
    print(f"full TDDFT products: 20 atoms, {prec}, window {window} eV", flush=True)
    Fo, Xo = _oracle(mol0, window)
    F = ctx.build_factors(P.System(mol0), P.Params(precision=P.PRECISIONS[prec], window_ev=window, full_tddft=True))
    dt = torch.float64 if prec == "fp64" else torch.float32
    V = synth.random_trial_vectors(7, mol0.nocc, mol0.nvir, 17)
    Pg, Mg = ctx.sigma_full(F, torch.tensor(V, dtype=dt, device=ctx.device))
    Vin = V.astype(np.float32 if prec == "fp32" else np.float64).astype(np.float64)  # what the GPU reads
    Po, Mo = FU.sigma_pm(Fo, Xo, Vin)
    for got, want in ((Pg, Po), (Mg, Mo)):
        err = np.abs(got.double().cpu().numpy() - want).max() / np.abs(want).max()
        print(f"  max rel err {err:.2e}", flush=True)
        assert err <= tol
    F.free()


@pytest.mark.parametrize("prec,tol_e,tol_r", [("fp64", 1e-6, 1e-6), ("fp32", 1e-6, 1e-5)])
def test_davidson_full_energies_config0(ctx, mol0, prec, tol_e, tol_r):
    import paper_2603_29257_amd as P
    n = 5
    Fo, Xo = _oracle(mol0, 40.0)
    ApB, AmB = FU.dense_ApB_AmB(Fo, Xo)
    om_ref, _, _ = FU.full_eigh(ApB, AmB, n)
    F = ctx.build_factors(P.System(mol0), P.Params(precision=P.PRECISIONS[prec], full_tddft=True))
    om, xp, xm, info = ctx.davidson_full(F, n, tol=tol_r)
    e_tda, _, _ = ctx.davidson(F, n, tol=tol_r, want_vectors=False)
    F.free()
    print(f"  {prec}: full {om}, ref {om_ref}, {info.iters} iterations, {info.sigma_vectors} product vectors",
          flush=True)
    assert info.converged
    assert np.abs(om - om_ref).max() <= tol_e
    assert np.all(om <= e_tda + 1e-8)  # below the TDA energies, as the oracle's pins show
    xp, xm = xp.astype(np.float64), xm.astype(np.float64)
    for k in range(n):
        assert abs(xp[k] @ xm[k] - 1.0) <= 1e-5
        r1 = np.linalg.norm(ApB @ xp[k] - om[k] * xm[k])
        r2 = np.linalg.norm(AmB @ xm[k] - om[k] * xp[k])
        assert max(r1, r2) <= 10 * tol_r + 1e-6  # FP32-stored amplitudes round at 6e-8


def test_full_factors_rejected_for_bf16(ctx, mol0):
    import paper_2603_29257_amd as P
    with pytest.raises(P.RispError):
        ctx.build_factors(P.System(mol0), P.Params(precision=P.BF16, full_tddft=True))


@pytest.mark.skipif(not os.path.exists(GOLD300), reason="oracle reference energies not generated")
def test_davidson_full_300_atoms_below_tda(ctx):
    # 300 atoms, FP32: converges, and each full-TDDFT energy lies below the oracle's TDA energy of the
    # same state (the bound the oracle pins show)
    import paper_2603_29257_amd as P
    mol = synth.config_system("chainring300")
    gold = json.load(open(GOLD300))
    F = ctx.build_factors(P.System(mol), P.Params(precision=P.FP32, full_tddft=True))
    om, xp, xm, info = ctx.davidson_full(F, 15, tol=1e-5, want_vectors=False)
    F.free()
    ref = np.array(gold["energies_ha"])[:15]
    print(f"  300 atoms full TDDFT: {info.iters} iterations, max shift below TDA {np.max(ref - om):.3e} Ha", flush=True)
    assert info.converged
    assert np.all(om <= ref + 1e-6)
