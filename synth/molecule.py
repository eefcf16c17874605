"""Synthetic molecules shaped like the paper's organic workloads (carbon skeleton + hydrogens).

Recipe (stated once, used by the oracle, the tests and the benchmark):

* Random streams: ``numpy.random.default_rng`` over ``SeedSequence(seed).spawn(4)`` giving separate
  streams for geometry, hydrogen placement, the Haar-orthogonal matrix Q and orbital energies.
* 20-atom molecule: 12 C on a 3x2x2 grid of 1.4 A spacing with U(+-0.1 A) jitter per coordinate,
  then 8 H, each on a distinct random C at 1.09 A in a uniform random direction; a direction is
  redrawn while the H would sit closer than 1.0 A to any other atom.
* Larger molecules ("chain and ring"): N_C = round(0.6 N) carbons, N_H = N - N_C hydrogens. The carbon
  skeleton grows as a self-avoiding walk of units, each a 2-C linker followed by a hexagon (1.4 A
  bonds, 120 degree angles, random dihedrals), confined to a sphere sized for an organic density of
  0.1 atoms/A^3; non-bonded C-C distances stay >= 2.5 A. A remainder shorter than one unit is a
  terminal zig-zag chain. The sphere grows by 3% whenever the walk jams. Jitter and H placement as above.
* AO basis: uncontracted normalised primitives with even-tempered exponents 0.15*3^k bohr^-2.
  C: s(k=0,1,2), p(k=0,1); H: s(k=0,1), p(k=0). Order: atom, shell as listed, then x, y, z.
* MOs: C = S^-1/2 Q with Q Haar-orthogonal (QR of a Gaussian matrix with the sign of diag(R) fixed).
  eps_occ ~ U[-0.8,-0.2] Ha and eps_vir ~ U[0.05, 2.0] Ha, each sorted ascending; nocc = floor(5 N_C/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ANGSTROM_TO_BOHR = 1.0 / 0.529177210903  # CODATA 2018 Bohr radius
HARTREE_TO_EV = 27.211386245988  # CODATA 2018

# even-tempered AO exponents (bohr^-2) per element: list of (l, exponent)
AO_EXPONENTS = {
    6: [(0, 0.15), (0, 0.45), (0, 1.35), (1, 0.15), (1, 0.45)],
    1: [(0, 0.15), (0, 0.45), (1, 0.15)],
}
# covalent radii (A) used as the auxiliary-basis radius R_A of each element
COVALENT_RADIUS_ANGSTROM = {6: 0.76, 1: 0.31}


@dataclass
class Molecule:
    coords: np.ndarray  # [natm, 3] bohr
    Z: np.ndarray  # [natm] int32
    shells: list  # [(atom, l, exponent, coef)] ; coef multiplies the normalised primitive
    aux_radius: np.ndarray  # [natm] bohr
    nao: int
    nocc: int
    mo_coeff: np.ndarray = field(repr=False)  # [nao, nmo]
    mo_energy: np.ndarray = field(repr=False)  # [nmo]
    cond_S: float = 0.0
    seed: int = 0
    name: str = ""

    @property
    def nmo(self):
        return self.mo_coeff.shape[1]

    @property
    def nvir(self):
        return self.nmo - self.nocc

    @property
    def natm(self):
        return len(self.Z)


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def _unit(v):
    return v / np.linalg.norm(v)


def _random_direction(rng):
    while True:
        v = rng.normal(size=3)
        n = np.linalg.norm(v)
        if n > 1e-8:
            return v / n


def _perp(u, rng):
    """A random unit vector perpendicular to unit vector u."""
    while True:
        v = rng.normal(size=3)
        v -= u * np.dot(u, v)
        n = np.linalg.norm(v)
        if n > 1e-6:
            return v / n


def _bond_dir(prev_dir, rng, angle_deg=120.0):
    """Direction of the next bond making `angle_deg` with the previous bond, random dihedral.

    prev_dir points from the previous atom to the current one; the returned direction points from
    the current atom to the next one, so the bond angle (prev, cur, next) equals angle_deg.
    """
    t = math.radians(180.0 - angle_deg)
    w = _perp(prev_dir, rng)
    return math.cos(t) * prev_dir + math.sin(t) * w


def _place_hydrogens(C_xyz, n_h, rng):
    """Put n_h hydrogens on distinct random carbons at 1.09 A, redrawing directions closer than 1.0 A."""
    nC = len(C_xyz)
    hosts = rng.choice(nC, size=n_h, replace=False)
    placed = list(C_xyz)
    H = []
    for h in hosts:
        for _ in range(10000):
            pos = C_xyz[h] + 1.09 * _random_direction(rng)
            d = np.linalg.norm(np.asarray(placed) - pos, axis=1)
            if np.all(d >= 1.0):
                break
        else:  # pragma: no cover - dense packing never reaches this at organic density
            raise RuntimeError("could not place hydrogen")
        placed.append(pos)
        H.append(pos)
    return np.asarray(H).reshape(-1, 3)


def _grid_carbons(rng):
    g = np.array([[i, j, k] for i in range(3) for j in range(2) for k in range(2)], dtype=float) * 1.4
    g -= g.mean(axis=0)
    return g + rng.uniform(-0.1, 0.1, size=g.shape)


class _Skeleton:
    """Self-avoiding carbon walk built from linker + hexagon units inside a sphere."""

    def __init__(self, radius, rng):
        self.R = radius
        self.rng = rng
        self.xyz = np.zeros((0, 3))
        self.nbr: list[set] = []
        self.ring_center: dict[int, np.ndarray] = {}  # ring atom -> centre of its hexagon
        self.sites: list[int] = []  # atoms where a new bond may attach, most recent first

    def _violates(self, new_xyz, new_bonds):
        """True if any new atom leaves the sphere or comes within 2.5 A of a non-bonded atom."""
        n_old = len(self.xyz)
        if np.any(np.linalg.norm(new_xyz, axis=1) > self.R):
            return True
        extra: dict[int, set] = {}  # tentative bonds, without copying the whole neighbour list
        for a, b in new_bonds:
            extra.setdefault(a, set()).add(b)
            extra.setdefault(b, set()).add(a)

        def nb(t):
            base = self.nbr[t] if t < n_old else set()
            return base | extra.get(t, set())

        allxyz = np.vstack([self.xyz, new_xyz]) if n_old else new_xyz
        for k in range(len(new_xyz)):
            idx = n_old + k
            if idx == 0:
                continue
            d = np.linalg.norm(allxyz[:idx] - allxyz[idx], axis=1)
            close = np.nonzero(d < 2.5)[0]
            if len(close) == 0:
                continue
            excl = {idx} | nb(idx)  # graph distance <= 2 is bonded geometry, not a clash
            for q in list(nb(idx)):
                excl |= nb(q)
            if any(int(t) not in excl for t in close):
                return True
        return False

    def _commit(self, new_xyz, new_bonds):
        n_old = len(self.xyz)
        self.xyz = np.vstack([self.xyz, new_xyz]) if n_old else np.asarray(new_xyz)
        self.nbr += [set() for _ in range(len(new_xyz))]
        for a, b in new_bonds:
            self.nbr[a].add(b)
            self.nbr[b].add(a)

    @staticmethod
    def _hexagon(center, u, v):
        """Hexagon of side 1.4 A in the plane (u, v); vertex 0 at center - 1.4 u."""
        ang = np.arange(6) * (math.pi / 3.0)
        return center + 1.4 * (-np.cos(ang)[:, None] * u + np.sin(ang)[:, None] * v)

    def _add_ring_sites(self, ring_idx, center):
        for k in ring_idx:
            self.ring_center[k] = center
        order = [3, 2, 4, 1, 5, 0]  # para to the attachment first
        self.sites = [ring_idx[k] for k in order] + self.sites

    def first_ring(self):
        u = _random_direction(self.rng)
        v = _perp(u, self.rng)
        ring = self._hexagon(np.zeros(3), u, v)
        self._commit(ring, [(k, (k + 1) % 6) for k in range(6)])
        self._add_ring_sites(list(range(6)), np.zeros(3))

    def out_direction(self, a):
        """Bond direction leaving atom a at 120 degrees to its existing bonds (random dihedral)."""
        if a in self.ring_center:
            return _unit(self.xyz[a] - self.ring_center[a])
        (q,) = tuple(self.nbr[a])
        return _bond_dir(_unit(self.xyz[a] - self.xyz[q]), self.rng)

    def is_free(self, a):
        return len(self.nbr[a]) < (3 if a in self.ring_center else 2)

    def try_unit(self, site):
        """Attach a 2-C linker and a hexagon at atom `site`."""
        n0 = len(self.xyz)
        out_dir = self.out_direction(site)
        L1 = self.xyz[site] + 1.4 * out_dir
        d2 = _bond_dir(out_dir, self.rng)
        L2 = L1 + 1.4 * d2
        w = _bond_dir(d2, self.rng)
        center = L2 + 2.8 * w
        ring = self._hexagon(center, w, _perp(w, self.rng))  # vertex 0 bonded to L2
        new = np.vstack([L1, L2, ring])
        bonds = [(site, n0), (n0, n0 + 1), (n0 + 1, n0 + 2)]
        bonds += [(n0 + 2 + k, n0 + 2 + (k + 1) % 6) for k in range(6)]
        if self._violates(new, bonds):
            return False
        self._commit(new, bonds)
        self._add_ring_sites(list(range(n0 + 2, n0 + 8)), center)
        return True

    def try_chain_atom(self, site):
        n0 = len(self.xyz)
        p = self.xyz[site] + 1.4 * self.out_direction(site)
        if self._violates(p[None, :], [(site, n0)]):
            return False
        self._commit(p[None, :], [(site, n0)])
        self.sites = [n0] + self.sites
        return True


def _chain_ring_carbons(n_c, radius, rng):
    while True:
        sk = _Skeleton(radius, rng)
        sk.first_ring()
        stuck = False
        while len(sk.xyz) < n_c:
            unit = (n_c - len(sk.xyz)) >= 8
            ok = False
            free = [a for a in sk.sites if sk.is_free(a)][:16]
            for a in free:
                for _ in range(6):
                    ok = sk.try_unit(a) if unit else sk.try_chain_atom(a)
                    if ok:
                        break
                if ok:
                    break
            if not ok:
                stuck = True
                break
        if not stuck:
            return sk.xyz
        radius *= 1.03  # the walk jammed: grow the sphere and start again


def _overlap(coords, shells):
    """AO overlap matrix of normalised primitive s/p Cartesian Gaussians (generator-only use)."""
    funcs = []  # (center, alpha, cart exponent tuple, norm)
    for (atom, l, alpha, coef) in shells:
        ns = (2.0 * alpha / math.pi) ** 0.75
        if l == 0:
            funcs.append((coords[atom], alpha, (0, 0, 0), coef * ns))
        else:
            for c in range(3):
                e = [0, 0, 0]
                e[c] = 1
                funcs.append((coords[atom], alpha, tuple(e), coef * ns * 2.0 * math.sqrt(alpha)))
    n = len(funcs)
    cen = np.array([f[0] for f in funcs])
    al = np.array([f[1] for f in funcs])
    ex = np.array([f[2] for f in funcs])
    nm = np.array([f[3] for f in funcs])
    p = al[:, None] + al[None, :]
    mu = al[:, None] * al[None, :] / p
    AB = cen[:, None, :] - cen[None, :, :]
    K = np.exp(-mu * np.sum(AB * AB, axis=2)) * (math.pi / p) ** 1.5
    P = (al[:, None, None] * cen[:, None, :] + al[None, :, None] * cen[None, :, :]) / p[:, :, None]
    S = K.copy()
    for d in range(3):
        ia = ex[:, d][:, None]
        ib = ex[:, d][None, :]
        PA = P[:, :, d] - cen[:, None, d]
        PB = P[:, :, d] - cen[None, :, d]
        # 1D factor for exponents (ia, ib) in {0,1}
        f = np.where((ia == 0) & (ib == 0), 1.0,
             np.where((ia == 1) & (ib == 0), PA,
              np.where((ia == 0) & (ib == 1), PB, PA * PB + 0.5 / p)))
        S *= f
    S *= nm[:, None] * nm[None, :]
    assert S.shape == (n, n)
    return 0.5 * (S + S.T)


def _shells_for(Z):
    shells = []
    for a, z in enumerate(Z):
        for (l, e) in AO_EXPONENTS[int(z)]:
            shells.append((a, l, e, 1.0))
    return shells


def _nao(shells):
    return sum(1 if l == 0 else 3 for (_, l, _, _) in shells)


def make_system(C_ang, H_ang, rng_q, rng_e, seed, name="") -> Molecule:
    coords = np.vstack([C_ang, H_ang]) * ANGSTROM_TO_BOHR
    Z = np.array([6] * len(C_ang) + [1] * len(H_ang), dtype=np.int32)
    shells = _shells_for(Z)
    nao = _nao(shells)
    nocc = (5 * len(C_ang)) // 2
    S = _overlap(coords, shells)
    w, U = np.linalg.eigh(S)
    cond = float(w[-1] / w[0])
    S_mhalf = (U / np.sqrt(w)) @ U.T
    G = rng_q.normal(size=(nao, nao))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))[None, :]
    C = S_mhalf @ Q
    eo = np.sort(rng_e.uniform(-0.8, -0.2, size=nocc))
    ev = np.sort(rng_e.uniform(0.05, 2.0, size=nao - nocc))
    radius = np.array([COVALENT_RADIUS_ANGSTROM[int(z)] for z in Z]) * ANGSTROM_TO_BOHR
    return Molecule(coords=coords, Z=Z, shells=shells, aux_radius=radius, nao=nao, nocc=nocc,
                    mo_coeff=np.ascontiguousarray(C), mo_energy=np.concatenate([eo, ev]),
                    cond_S=cond, seed=seed, name=name)


def make_config0(seed: int = 20) -> Molecule:
    """20-atom molecule: 12 C on a jittered 3x2x2 grid plus 8 H."""
    g_geo, g_h, g_q, g_e = _streams(seed)
    C = _grid_carbons(g_geo)
    H = _place_hydrogens(C, 8, g_h)
    return make_system(C, H, g_q, g_e, seed, name="grid20")


def make_chain_ring(n_atoms: int, seed: int) -> Molecule:
    """Chain-and-ring molecule with round(0.6 N) carbons and the rest hydrogens."""
    g_geo, g_h, g_q, g_e = _streams(seed)
    n_c = int(round(0.6 * n_atoms))
    n_h = n_atoms - n_c
    radius = (3.0 * n_atoms / (4.0 * math.pi * 0.1)) ** (1.0 / 3.0)
    C = _chain_ring_carbons(n_c, radius, g_geo)
    C = C + g_geo.uniform(-0.1, 0.1, size=C.shape)
    H = _place_hydrogens(C, n_h, g_h)
    return make_system(C, H, g_q, g_e, seed, name=f"chainring{n_atoms}")


def config_system(name: str) -> Molecule:
    """Named workloads: 'grid20' (20 atoms), 'chainring300', 'chainring1000', 'chainring3000',
    or 'tiny<N>' chain-ring molecules of N atoms (seed N) for small tests."""
    if name == "grid20":
        return make_config0(20)
    if name.startswith("chainring"):
        n = int(name[len("chainring"):])
        return make_chain_ring(n, n)
    raise KeyError(name)


def random_trial_vectors(m: int, nocc: int, nvir: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded trial-vector block X [m][nocc][nvir] with unit-norm rows (normal entries)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, m, nocc, nvir]))
    X = rng.normal(size=(m, nocc * nvir))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return X.reshape(m, nocc, nvir).astype(dtype)
