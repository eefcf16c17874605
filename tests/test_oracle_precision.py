"""Why the factor build runs in FP64: emulated precision of the MO transforms (oracle arithmetic).

On the 20-atom molecule the MO coefficients C = S^-1/2 Q (cond(S) ~ 3e5) make the transform of the
three-centre integrals cancel heavily. Rounding the transform inputs and arithmetic to FP32 moves the
lowest excitation energies by ~1e-4 Ha, far beyond the 1e-6 Ha bar, while an FP64 transform whose
result is stored in FP32 stays ~1e-8 Ha away; storing FP64-built factors in BF16 costs ~1e-4 Ha, the
error the FP32 correction pass must remove.
"""
import copy

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import integrals as I
from oracle import risp as R


def _bf16(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def setup():
    mol = synth.make_config0()
    prm = R.Params()
    F = R.build_factors(mol, prm)
    w = np.linalg.eigvalsh(R.dense_A(F))[:5]
    auxJ, auxK = R.select_aux(mol.Z, mol.aux_radius)
    V3 = I.int3c(mol.coords, mol.shells, auxJ)
    V2 = I.int2c(mol.coords, auxJ)
    V3x = 0.22 * I.int3c(mol.coords, mol.shells, auxK) + 0.78 * I.int3c(mol.coords, mol.shells, auxK, 0.2)
    V2x = 0.22 * I.int2c(mol.coords, auxK) + 0.78 * I.int2c(mol.coords, auxK, 0.2)
    return mol, F, w, (V3, V2, V3x, V2x)


def _energies(mol, F, ints, build):
    V3, V2, V3x, V2x = ints
    C, o = mol.mo_coeff, mol.nocc
    G = copy.deepcopy(F)
    G.B_ia = build(V3, V2, C[:, :o], C[:, o:])
    CoK, CvK = C[:, :o][:, F.occK], C[:, o:][:, F.virK]
    G.Bx_ij = build(V3x, V2x, CoK, CoK)
    G.Bx_ab = build(V3x, V2x, CvK, CvK)
    return np.linalg.eigvalsh(R.dense_A(G))[:5]


def fp32_transform(V3, V2, Cl, Cr):
    L = np.linalg.cholesky(V2)
    T = np.einsum("mi,mnP,na->Pia", Cl.astype(np.float32), V3.astype(np.float32), Cr.astype(np.float32))
    T = T.astype(np.float64)
    B = sla.solve_triangular(L, T.reshape(T.shape[0], -1), lower=True).reshape(T.shape)
    return B.astype(np.float32).astype(np.float64)


def fp64_transform_fp32_store(V3, V2, Cl, Cr):
    L = np.linalg.cholesky(V2)
    T = np.einsum("mi,mnP,na->Pia", Cl, V3, Cr)
    B = sla.solve_triangular(L, T.reshape(T.shape[0], -1), lower=True).reshape(T.shape)
    return B.astype(np.float32).astype(np.float64)


def test_fp32_transform_misses_the_bar(setup):
    mol, F, w, ints = setup
    err = np.abs(_energies(mol, F, ints, fp32_transform) - w).max()
    assert err > 1e-5


def test_fp64_transform_with_fp32_storage_meets_the_bar(setup):
    mol, F, w, ints = setup
    err = np.abs(_energies(mol, F, ints, fp64_transform_fp32_store) - w).max()
    assert err < 1e-7


def test_bf16_storage_needs_correction(setup):
    mol, F, w, _ = setup
    G = copy.deepcopy(F)
    G.B_ia, G.Bx_ij, G.Bx_ab = _bf16(F.B_ia), _bf16(F.Bx_ij), _bf16(F.Bx_ab)
    err = np.abs(np.linalg.eigvalsh(R.dense_A(G))[:5] - w).max()
    assert 2e-5 < err < 1e-2
