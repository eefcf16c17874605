"""The allocation-free sigma entry point (risp_sigma_noalloc) against risp_sigma, through the C ABI.

Two calls in a row on one device, the second with a smaller molecule and fewer vectors, so the
second runs over the first one's leftovers in the shared scratch array; each result must match
risp_sigma's on the same inputs to the parity bars (FP64 1e-12, FP32 2e-6, BF16 1e-3 of the largest
element: the two differ only in the number of auxiliary functions per exchange chunk, i.e. in the
FP32/FP64 accumulation order). Sizes past the scratch array are rejected with RISP_E_SHAPE.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32": 2e-6, "bf16": 1e-3}


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


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_noalloc_sigma_matches_sigma_two_calls(ctx, prec):
    import paper_2603_29257_amd as P
    cases = [(synth.make_chain_ring(100, 100), 30), (synth.make_config0(), 7)]  # second call smaller
    for mol, m in cases:
        _print(f"noalloc sigma: {mol.natm} atoms, {prec}, m={m}")
        F = ctx.build_factors(P.System(mol), P.Params(precision=P.PRECISIONS[prec]))
        dt = torch.float64 if prec == "fp64" else torch.float32
        X = torch.tensor(synth.random_trial_vectors(m, mol.nocc, mol.nvir, 11), dtype=dt, device=ctx.device)
        want = ctx.sigma(F, X)
        out = torch.full_like(X, float("nan"))
        got = ctx.sigma(F, X, out=out, noalloc=True)
        torch.cuda.synchronize()
        w, g = want.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(g).all()
        err = np.abs(g - w).max() / np.abs(w).max()
        _print(f"  max |noalloc - sigma| / max|sigma| = {err:.2e}")
        assert err <= TOL[prec], err
        F.free()


def test_noalloc_rejects_sizes_beyond_the_scratch(ctx):
    import paper_2603_29257_amd as P
    mol = synth.make_chain_ring(300, 300)
    _print("noalloc sigma: 300 atoms, bf16, m=64 (beyond the scratch array)")
    F = ctx.build_factors(P.System(mol), P.Params(precision=P.BF16))
    X = torch.zeros((64, mol.nocc, mol.nvir), dtype=torch.float32, device=ctx.device)
    out = torch.zeros_like(X)
    with pytest.raises(P.RispError) as e:
        ctx.sigma(F, X, out=out, noalloc=True)
    from paper_2603_29257_amd import abi
    assert e.value.code == abi.RISP_E_SHAPE and "scratch" in str(e.value)
    # the bench block of 30 vectors fits, and matches risp_sigma
    X = torch.tensor(synth.random_trial_vectors(30, mol.nocc, mol.nvir, 5), dtype=torch.float32, device=ctx.device)
    want = ctx.sigma(F, X)
    got = ctx.sigma(F, X, out=torch.empty_like(X), noalloc=True)
    torch.cuda.synchronize()
    w, g = want.cpu().numpy(), got.cpu().numpy()
    err = np.abs(g - w).max() / np.abs(w).max()
    _print(f"  300 atoms, 30 vectors: max |noalloc - sigma| / max|sigma| = {err:.2e}")
    assert err <= TOL["bf16"]
    F.free()
