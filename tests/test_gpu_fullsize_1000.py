"""Full-size parity on the 1000-atom molecule, in the launch configuration the benchmark times.

The FP64 oracle cannot form this molecule's factors (the FP64 T_ia alone is 170 GB), so
tests/golden/chainring1000_sigma_rows.json holds sigma = A X for a seeded block of 30 trial vectors
at 64 sampled rows (i, a), computed by the oracle straight from the integrals
(oracle.risp.sigma_rows, written by tests/golden/make_sigma_rows_golden.py; no GPU value enters
it). The rows include both sides of the 40 eV window edge and the corners of the (i, a) range. The
GPU's 30-vector sigma block is compared with it element by element, for the BF16 and the plain FP32
factors, together with the screened pair count and the window sizes.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chainring1000_sigma_rows.json")

# Bars relative to the largest sampled element (the same bars as the small-case parity tests):
# FP32 factors 2e-6; BF16 factors 1e-3 (ten times the measured BF16 product error, so a wrong
# power-of-two scale on one auxiliary slice fails it).
TOL = {"fp32": 2e-6, "bf16": 1e-3}


@pytest.fixture(scope="module")
def c2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLD):
        pytest.skip("1000-atom oracle reference not generated")
    import paper_2603_29257_amd as P
    print("generating chainring1000", flush=True)
    mol = synth.config_system("chainring1000")
    ctx = P.Context(0)
    yield mol, ctx, P.System(mol), json.load(open(GOLD))
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_sigma_rows_vs_oracle_1000_atoms(c2, prec):
    mol, ctx, sysc, gold = c2
    import paper_2603_29257_amd as P
    print(f"1000 atoms: building {prec} factors", flush=True)
    F = ctx.build_factors(sysc, P.Params(precision=P.PRECISIONS[prec]))
    d = F.desc
    assert (d.npair, d.nocc_k, d.nvir_k) == (gold["npair"], gold["nocc_k"], gold["nvir_k"])
    assert (d.nocc, d.nvir) == (gold["nocc"], gold["nvir"])
    m = len(gold["sigma"])
    X = torch.tensor(synth.random_trial_vectors(m, d.nocc, d.nvir, gold["seed"]), dtype=torch.float32,
                     device=ctx.device)
    rows = torch.tensor(gold["rows"], device=ctx.device)
    S = ctx.sigma(F, X).reshape(m, -1)[:, rows].double().cpu().numpy()
    want = np.array(gold["sigma"])
    err = np.abs(S - want).max() / np.abs(want).max()
    print(f"1000 atoms, {prec}: max |sigma - oracle| / max |oracle| over {want.size} sampled elements = {err:.2e}",
          flush=True)
    assert err <= TOL[prec]
    F.free()
