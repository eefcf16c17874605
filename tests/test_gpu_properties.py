"""Transition properties and spectra on the GPU (risp_properties, risp_spectrum through the C ABI)
against the FP64 oracle (oracle/properties.py) on the same inputs."""
import numpy as np
import pytest

import synth
from oracle import properties as PR
from oracle import risp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("name,n", [("grid20", 5), ("chainring100", 16)])
def test_properties_match_oracle(ctx, name, n):
    import paper_2603_29257_amd as P
    mol = synth.config_system(name)
    print(f"properties: {name}, {n} states", flush=True)
    X = synth.random_trial_vectors(n, mol.nocc, mol.nvir, 31, dtype=np.float32)
    omega = np.linspace(0.18, 0.31, n)
    origin = mol.coords.mean(axis=0)
    Xd = torch.tensor(X, device=ctx.device)
    mu, m, f, Rr = ctx.properties(P.System(mol), omega, Xd, origin)
    mu0, m0, f0, R0 = PR.properties(mol, omega, X.astype(np.float64), origin)
    errs = (_rel(mu, mu0), _rel(m, m0), _rel(f, f0), _rel(Rr, R0))
    print(f"  rel errors mu {errs[0]:.2e} m {errs[1]:.2e} f {errs[2]:.2e} R {errs[3]:.2e}", flush=True)
    # FP64 integrals and transforms on both sides; the bar leaves room for the conditioning of
    # C = S^-1/2 Q (the transforms cancel about three digits, as in the factor tests)
    assert max(errs) <= 1e-9


def test_properties_of_converged_states_and_spectrum(ctx):
    # the states of the 20-atom molecule (FP64 path), their strengths against the oracle's for the
    # same vectors, and the broadened UV-vis and ECD spectra on a grid
    import paper_2603_29257_amd as P
    mol = synth.make_config0()
    F = ctx.build_factors(P.System(mol), P.Params(precision=P.FP64))
    e, vec, info = ctx.davidson(F, 5, tol=1e-6)
    F.free()
    X = np.asarray(vec, dtype=np.float32).reshape(5, mol.nocc, mol.nvir)
    Xd = torch.tensor(X, device=ctx.device)
    mu, m, f, Rr = ctx.properties(P.System(mol), e, Xd)
    mu0, m0, f0, R0 = PR.properties(mol, e, X.astype(np.float64))
    assert _rel(f, f0) <= 1e-9 and _rel(Rr, R0) <= 1e-9
    g = 0.05 / R.HARTREE_TO_EV
    e0, de, npts = 0.15, 1e-4, 2001
    grid = e0 + de * np.arange(npts)
    for s, s0 in ((f, f0), (Rr, R0)):
        got = ctx.spectrum(e, s, g, e0, de, npts)
        want = PR.spectrum(grid, e, s0, g)
        assert _rel(got, want) <= 1e-9
    print(f"  f {np.round(f, 6)} R {R0}", flush=True)
