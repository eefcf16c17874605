"""The AO-density Coulomb route (RISP_J_AO_DIRECT) on the 3000-atom chain-and-ring molecule (nao
22200): integrals regenerated in the packed layout over the kept pairs, so no [nao][nao] integral
slab is formed. Exchange off (the 40 eV window keeps T_ab far beyond one device at this size), FP64
throughout; checks on two seeded trial vectors that the Coulomb part J = (sigma - (e_a - e_i) X) / 2
is symmetric (x1.J x0 = x0.J x1) and positive (x.J x > 0), the properties that hold at any size.

The molecule takes the seeded generator's geometry, basis and overlap; S^-1/2 and the orthogonal
factor of C = S^-1/2 Q are formed on the GPU (the host's dense eigensolver needs minutes at this
size), so C differs from the host generator's by rounding."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _molecule_3000():
    from synth import molecule as M
    n_atoms, seed = 3000, 3000
    g_geo, g_h, g_q, g_e = M._streams(seed)
    n_c = int(round(0.6 * n_atoms))
    radius = (3.0 * n_atoms / (4.0 * math.pi * 0.1)) ** (1.0 / 3.0)
    c_ang = M._chain_ring_carbons(n_c, radius, g_geo)
    c_ang = c_ang + g_geo.uniform(-0.1, 0.1, size=c_ang.shape)
    h_ang = M._place_hydrogens(c_ang, n_atoms - n_c, g_h)
    coords = np.vstack([c_ang, h_ang]) * M.ANGSTROM_TO_BOHR
    Z = np.array([6] * len(c_ang) + [1] * len(h_ang), dtype=np.int32)
    shells = M._shells_for(Z)
    nao, nocc = M._nao(shells), (5 * len(c_ang)) // 2
    dev = torch.device("cuda:0")
    S = torch.tensor(M._overlap(coords, shells), device=dev)
    w, U = torch.linalg.eigh(S)
    del S
    smh = (U / torch.sqrt(w)[None, :]) @ U.T
    del U
    Q, R = torch.linalg.qr(torch.tensor(g_q.normal(size=(nao, nao)), device=dev))
    C = (smh @ (Q * torch.sign(torch.diagonal(R))[None, :])).cpu().numpy()
    del smh, Q, R
    torch.cuda.empty_cache()
    eo = np.sort(g_e.uniform(-0.8, -0.2, size=nocc))
    ev = np.sort(g_e.uniform(0.05, 2.0, size=nao - nocc))
    rad = np.array([M.COVALENT_RADIUS_ANGSTROM[int(z)] for z in Z]) * M.ANGSTROM_TO_BOHR
    return M.Molecule(coords=coords, Z=Z, shells=shells, aux_radius=rad, nao=nao, nocc=nocc,
                      mo_coeff=np.ascontiguousarray(C), mo_energy=np.concatenate([eo, ev]),
                      cond_S=float(w[-1] / w[0]), seed=seed, name="chainring3000")


def test_ao_route_coulomb_3000_atoms():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    import synth
    print("AO route, 3000 atoms: building the molecule", flush=True)
    mol = _molecule_3000()
    assert mol.nao == 22200  # beyond one dense FP64 integral slab of 2 GiB per auxiliary function
    ctx = P.Context(0)
    F = ctx.build_factors(P.System(mol), P.Params(precision=P.FP64, j_mode=P.J_AO_DIRECT, c_x=0.0, beta=0.0))
    d = F.desc
    print(f"  factors: npair {d.npair}, {d.bytes / 1e9:.2f} GB", flush=True)
    X = torch.tensor(synth.random_trial_vectors(2, d.nocc, d.nvir, 3000), dtype=torch.float64, device=ctx.device)
    de = torch.tensor(-np.subtract.outer(mol.mo_energy[:d.nocc], mol.mo_energy[d.nocc:]), device=ctx.device)
    J = []
    for k in range(2):
        s = ctx.sigma(F, X[k:k + 1])
        J.append((s[0] - de * X[k]) / 2.0)
        print(f"  sigma vector {k} done", flush=True)
    a, b = float((X[1] * J[0]).sum()), float((X[0] * J[1]).sum())
    p0, p1 = float((X[0] * J[0]).sum()), float((X[1] * J[1]).sum())
    print(f"  x1.J x0 {a:.12e}, x0.J x1 {b:.12e}, x.J x {p0:.6e} {p1:.6e}", flush=True)
    # FP64 rounding, amplified by the cancellation in D = C_occ X C_vir^T with C = S^-1/2 Q
    # (cond(S) = 2.9e6 here): measured 5.8e-10
    assert abs(a - b) <= 1e-8 * max(abs(a), abs(b))
    assert p0 > 0.0 and p1 > 0.0
    F.free()
    ctx.close()
