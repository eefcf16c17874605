"""Full-size parity on the 300-atom molecule, in the configuration the benchmark times.

The oracle cannot run the whole solve inside a test, so its FP64 energies come from
tests/golden/chainring300_oracle.json (written by tests/golden/make_golden.py, oracle only). The
sigma products are checked on sampled outputs against properties that hold at any size.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chainring300_oracle.json")


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    mol = synth.config_system("chainring300")
    ctx = P.Context(0)
    yield mol, ctx, P.System(mol)
    ctx.close()


def test_sigma_bilinear_and_precision_agreement(big):
    # y^T A x = x^T A y (A symmetric) at full size, and BF16 products within their stated bound of FP32
    mol, ctx, sysc = big
    import paper_2603_29257_amd as P
    F32 = ctx.build_factors(sysc, P.Params(precision=P.FP32))
    FB = ctx.build_factors(sysc, P.Params(precision=P.BF16))
    X = torch.tensor(synth.random_trial_vectors(30, F32.nocc, F32.nvir, 7), dtype=torch.float32,
                     device=ctx.device)
    Y = torch.tensor(synth.random_trial_vectors(30, F32.nocc, F32.nvir, 8), dtype=torch.float32,
                     device=ctx.device)
    sx, sy = ctx.sigma(F32, X).double(), ctx.sigma(F32, Y).double()
    a = (Y.double() * sx).sum(dim=(1, 2))
    b = (X.double() * sy).sum(dim=(1, 2))
    assert torch.max(torch.abs(a - b) / torch.abs(a)).item() <= 1e-5
    sb = ctx.sigma(FB, X).double()
    rel = ((sb - sx).flatten(1).norm(dim=1) / sx.flatten(1).norm(dim=1)).max().item()
    print(f"BF16 vs FP32 sigma, 300 atoms, relative norm error {rel:.3e}", flush=True)
    assert rel <= 1e-3
    F32.free()
    FB.free()


@pytest.mark.skipif(not os.path.exists(GOLD), reason="oracle reference energies not generated")
@pytest.mark.parametrize("prec,tol_e", [("fp32", 1e-6), ("bf16", 2e-5)])
def test_energies_vs_oracle_300_atoms(big, prec, tol_e):
    mol, ctx, sysc = big
    import paper_2603_29257_amd as P
    gold = json.load(open(GOLD))
    ref = np.array(gold["energies_ha"])
    F = ctx.build_factors(sysc, P.Params(precision=P.PRECISIONS[prec]))
    d = F.desc
    assert (d.npair, d.nocc_k, d.nvir_k) == (gold["npair"], gold["nocc_k"], gold["nvir_k"])
    e, _, info = ctx.davidson(F, len(ref), tol=1e-5, want_vectors=False)
    err = np.abs(e - ref)
    print(f"{prec}: per-state |E - E_oracle| max {err.max():.3e} Ha, iterations {info.iters}+"
          f"{info.correction_iters}", flush=True)
    assert info.converged
    assert err.max() <= tol_e
    F.free()


def test_sigma_ao_route_300_atoms(big):
    # the AO-density Coulomb route against the stored-factor route at full size (FP32 exchange and
    # X / sigma in both; the AO Coulomb term is FP64)
    mol, ctx, sysc = big
    import paper_2603_29257_amd as P
    Fm = ctx.build_factors(sysc, P.Params(precision=P.FP32))
    Fa = ctx.build_factors(sysc, P.Params(precision=P.FP32, j_mode=P.J_AO_DIRECT))
    X = torch.tensor(synth.random_trial_vectors(4, Fm.nocc, Fm.nvir, 19), dtype=torch.float32, device=ctx.device)
    a = ctx.sigma(Fm, X).double()
    b = ctx.sigma(Fa, X).double()
    rel = ((b - a).flatten(1).norm(dim=1) / a.flatten(1).norm(dim=1)).max().item()
    print(f"AO vs stored Coulomb route, 300 atoms, relative norm difference {rel:.3e}; "
          f"factor bytes {Fa.desc.bytes} vs {Fm.desc.bytes}", flush=True)
    assert rel <= 1e-5
    Fm.free()
    Fa.free()
