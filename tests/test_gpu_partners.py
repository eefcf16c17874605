"""The build's first MO transform over per-atom partner lists of the kept shell pairs against the same
transform over dense (mu nu|P) slabs (Params.dense_transform), through the C ABI: every stored factor
element by element in FP64 (the two differ only in the order of the nonzero terms of each sum), on
a molecule where screening removes nothing (20 atoms), on the 300-atom molecule with orthogonal MO
coefficients (most shell pairs screened out), and with the shells listed in an order that interleaves
atoms, so that every shell forms its own group; there the factors must also equal those of the
original order."""
import dataclasses

import numpy as np
import pytest

import synth

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


def _factors(ctx, mol, dense, **kw):
    import paper_2603_29257_amd as P
    F = ctx.build_factors(P.System(mol), P.Params(precision=P.FP64, dense_transform=dense, **kw))
    out = {k: F.tensor(k).double().cpu().numpy() for k in ("t_ia", "t_ij", "t_ab", "diag_a")}
    out["npair"] = F.desc.npair
    F.free()
    return out


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _compare(a, b, tol):
    assert a["npair"] == b["npair"]
    for k in ("t_ia", "t_ij", "t_ab", "diag_a"):
        err = _rel(a[k], b[k])
        print(f"  {k}: max rel diff {err:.2e}", flush=True)
        assert err <= tol, k


@pytest.mark.parametrize("window", [40.0, 10.0])
def test_partner_transform_equals_dense_20_atoms(ctx, window):
    print(f"partner vs dense transform: 20 atoms, window {window} eV", flush=True)
    mol = synth.make_config0()
    _compare(_factors(ctx, mol, False, window_ev=window), _factors(ctx, mol, True, window_ev=window), 1e-12)


def test_partner_transform_equals_dense_300_atoms(ctx):
    # MO coefficients replaced by a seeded orthogonal matrix: with the molecule's own C = S^-1/2 Q the
    # transforms cancel heavily (cond(S) ~ 1e5) and rounding alone differs at ~4e-10 of the largest
    # element between the two summation orders; with |C| <= 1 it stays below ~3e-13 (T_ia, through
    # the Coulomb metric) and ~1e-14 (T_ij, T_ab), so a misplaced or dropped integral block of any
    # weight above the screening threshold's scale shows above the bar
    print("partner vs dense transform: 300 atoms", flush=True)
    mol = _orthogonal(synth.config_system("chainring300"), 300)
    a, b = _factors(ctx, mol, False), _factors(ctx, mol, True)
    nsh = len(mol.shells)
    assert a["npair"] < 0.5 * (nsh * (nsh + 1) // 2)  # screening is active
    _compare(a, b, 1e-12)


def _orthogonal(mol, seed):
    """The molecule with its MO coefficients replaced by a seeded orthogonal matrix (|C| <= 1)."""
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(mol.nao, mol.nmo)))
    return dataclasses.replace(mol, mo_coeff=np.ascontiguousarray(q * np.sign(np.diag(r))))


def _interleaved(mol):
    """The same molecule with its shells reordered so that consecutive shells sit on different atoms
    (round robin over the atoms), the MO coefficient rows permuted to match."""
    sizes = [1 if s[1] == 0 else 3 for s in mol.shells]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    by_atom = {}
    for k, s in enumerate(mol.shells):
        by_atom.setdefault(s[0], []).append(k)
    order, depth = [], 0
    while len(order) < len(mol.shells):
        for at in sorted(by_atom):
            if depth < len(by_atom[at]):
                order.append(by_atom[at][depth])
        depth += 1
    rows = np.concatenate([np.arange(offs[k], offs[k + 1]) for k in order])
    return dataclasses.replace(mol, shells=[mol.shells[k] for k in order],
                               mo_coeff=np.ascontiguousarray(mol.mo_coeff[rows]))


def test_partner_transform_with_interleaved_shells(ctx):
    print("partner vs dense transform: 20 atoms, shells interleaved over atoms", flush=True)
    # orthogonal C as at 300 atoms: groups of single shells shorten the partner lists of the tight
    # shells, so the K slices differ from the dense order and rounding is all that may differ
    mol = _orthogonal(synth.make_config0(), 20)
    mix = _interleaved(mol)
    assert all(mix.shells[k][0] != mix.shells[k + 1][0] for k in range(len(mix.shells) - 1))
    a, b = _factors(ctx, mix, False), _factors(ctx, mix, True)
    _compare(a, b, 1e-12)
    # AO order does not change the factors (C rows follow the functions)
    _compare(a, _factors(ctx, mol, False), 1e-12)
