"""McMurchie-Davidson integrals over primitive Cartesian Gaussians (oracle, FP64).

Test infrastructure only: imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark, never by the HIP path.

Basis functions are uncontracted primitives g(r) = coef * N * x_A^lx y_A^ly z_A^lz exp(-alpha r_A^2),
the form of the auxiliary functions of eq. gr (and of the synthetic AO basis). N normalises the
primitive: N_s = (2 alpha/pi)^(3/4) and N_p = 2 sqrt(alpha) N_s for each Cartesian p component.

Two-electron integrals follow the Hermite-Gaussian route (McMurchie & Davidson 1978; Helgaker,
Jorgensen & Olsen, "Molecular Electronic-Structure Theory", ch. 9):

  (ab|c) = 2 pi^(5/2) / (p q sqrt(p+q)) * sum_tuv E^ab_tuv sum_tau,nu,phi (-1)^(tau+nu+phi)
           E^c_(tau nu phi) R_(t+tau, u+nu, v+phi)(alpha, R_PQ)

with p = a + b, q the exponent of c, alpha = p q / (p + q), E the Hermite expansion coefficients
and R the Hermite Coulomb integrals built from the Boys function F_n.

The attenuated operator erf(w r)/r is the Coulomb potential of a normalised Gaussian of exponent w^2,
so convolving it with the Gaussian distribution of exponent alpha gives a distribution of exponent
alpha' = alpha w^2/(alpha + w^2): R is evaluated with alpha' in place of alpha and the prefactor is
multiplied by sqrt(alpha'/alpha). This operator appears in the range-separated exchange operator
(eq. RSH and eq. K_mia_RSH).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import gamma, gammainc


# ----------------------------------------------------------------------------------------------
# Boys function
# ----------------------------------------------------------------------------------------------
def boys(n: int, T):
    """F_n(T) = int_0^1 t^(2n) exp(-T t^2) dt, via the regularised lower incomplete gamma function.

    F_n(T) = Gamma(n+1/2) P(n+1/2, T) / (2 T^(n+1/2)); for T below 1e-12 the Taylor series
    sum_k (-T)^k / (k! (2n+2k+1)) is used (four terms are exact to double precision there).
    """
    T = np.asarray(T, dtype=np.float64)
    out = np.empty_like(T)
    small = T < 1e-12
    a = n + 0.5
    Ts = np.where(small, 1.0, T)
    out[...] = gamma(a) * gammainc(a, Ts) / (2.0 * Ts ** a)
    if np.any(small):
        t = T[small]
        s = np.zeros_like(t)
        fact = 1.0
        for k in range(4):
            if k:
                fact *= k
            s += (-t) ** k / (fact * (2 * n + 2 * k + 1))
        out[small] = s
    return out


# ----------------------------------------------------------------------------------------------
# Basis functions
# ----------------------------------------------------------------------------------------------
def cart_components(l: int):
    """Cartesian exponent triples of angular momentum l in the order x, y, z (for p)."""
    if l == 0:
        return [(0, 0, 0)]
    if l == 1:
        return [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    raise ValueError("only s and p shells are used by the method")


def primitive_norm(alpha, comp):
    """Normalisation of x^lx y^ly z^lz exp(-alpha r^2) for l <= 1."""
    ns = (2.0 * np.asarray(alpha) / math.pi) ** 0.75
    if sum(comp) == 0:
        return ns
    return ns * 2.0 * np.sqrt(alpha)


def shell_offsets(shells):
    """First function index of each shell and the total number of functions."""
    off = []
    n = 0
    for (_, l, _, _) in shells:
        off.append(n)
        n += len(cart_components(l))
    return off, n


# ----------------------------------------------------------------------------------------------
# Hermite expansion coefficients and Hermite Coulomb integrals
# ----------------------------------------------------------------------------------------------
def hermite_E(i: int, j: int, XPA, XPB, p):
    """Hermite expansion coefficients E^{ij}_t (t = 0..i+j) of one Cartesian direction.

    x_A^i x_B^j exp(-a x_A^2 - b x_B^2) = K sum_t E^{ij}_t Lambda_t(x_P); the Gaussian prefactor K is
    applied by the caller, so E^{00}_0 = 1 here. Recurrences:
      E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}
      E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}
    Returns a list indexed by t of arrays broadcast like XPA.
    """
    XPA = np.asarray(XPA, dtype=np.float64)
    one = np.ones_like(XPA)
    inv2p = 0.5 / np.asarray(p, dtype=np.float64)

    @lru_cache(maxsize=None)
    def E(ii, jj, t):
        if t < 0 or t > ii + jj:
            return 0.0 * one
        if ii == 0 and jj == 0:
            return one
        if ii > 0:
            return inv2p * E(ii - 1, jj, t - 1) + XPA * E(ii - 1, jj, t) + (t + 1) * E(ii - 1, jj, t + 1)
        return inv2p * E(ii, jj - 1, t - 1) + XPB * E(ii, jj - 1, t) + (t + 1) * E(ii, jj - 1, t + 1)

    return [E(i, j, t) for t in range(i + j + 1)]


def hermite_R(L: int, alpha, PQ):
    """Hermite Coulomb integrals R_tuv = R^0_tuv for t+u+v <= L.

    R^n_000 = (-2 alpha)^n F_n(alpha |PQ|^2);
    R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_PQ R^{n+1}_{t,u,v} (and likewise for u, v).
    PQ has shape [..., 3]. Returns a dict (t, u, v) -> array.
    """
    alpha = np.asarray(alpha, dtype=np.float64)
    X, Y, Z = PQ[..., 0], PQ[..., 1], PQ[..., 2]
    T = alpha * (X * X + Y * Y + Z * Z)
    base = [(-2.0 * alpha) ** n * boys(n, T) for n in range(L + 1)]

    @lru_cache(maxsize=None)
    def R(n, t, u, v):
        if t < 0 or u < 0 or v < 0:
            return 0.0
        if t == 0 and u == 0 and v == 0:
            return base[n]
        if t > 0:
            return (t - 1) * R(n + 1, t - 2, u, v) + X * R(n + 1, t - 1, u, v)
        if u > 0:
            return (u - 1) * R(n + 1, t, u - 2, v) + Y * R(n + 1, t, u - 1, v)
        return (v - 1) * R(n + 1, t, u, v - 2) + Z * R(n + 1, t, u, v - 1)

    return {(t, u, v): R(0, t, u, v) for t in range(L + 1) for u in range(L + 1 - t)
            for v in range(L + 1 - t - u)}


def _operator_alpha(alpha, omega):
    """Effective exponent and prefactor scale for 1/r (omega None) or erf(omega r)/r."""
    if omega is None:
        return alpha, 1.0
    w2 = omega * omega
    a_eff = alpha * w2 / (alpha + w2)
    return a_eff, np.sqrt(a_eff / alpha)


# ----------------------------------------------------------------------------------------------
# Integral drivers
# ----------------------------------------------------------------------------------------------
def _pair_E(compA, compB, A, B, a, b):
    """Per-direction Hermite coefficients of the product of components compA at A and compB at B."""
    p = a + b
    P = (a[..., None] * A + b[..., None] * B) / p[..., None]
    Es = [hermite_E(compA[d], compB[d], P[..., d] - A[..., d], P[..., d] - B[..., d], p) for d in range(3)]
    return Es, P, p


def _one_E(comp, C, c):
    """Hermite coefficients of a single Cartesian Gaussian (its own product centre, X_PA = 0)."""
    zero = np.zeros(np.shape(c))
    return [hermite_E(comp[d], 0, zero, zero, c) for d in range(3)]


def _contract(EA, EB, R, sign_b=True):
    """sum_tuv EA_tuv sum_(tau nu phi) (-1)^(tau+nu+phi) EB_(tau nu phi) R_(t+tau, u+nu, v+phi)."""
    out = 0.0
    for t, ex in enumerate(EA[0]):
        for u, ey in enumerate(EA[1]):
            for v, ez in enumerate(EA[2]):
                eA = ex * ey * ez
                acc = 0.0
                for tt, fx in enumerate(EB[0]):
                    for uu, fy in enumerate(EB[1]):
                        for vv, fz in enumerate(EB[2]):
                            s = (-1.0) ** (tt + uu + vv) if sign_b else 1.0
                            acc = acc + s * fx * fy * fz * R[(t + tt, u + uu, v + vv)]
                eA_acc = eA * acc
                out = out + eA_acc
    return out


def _shell_arrays(coords, shells, idx):
    sh = [shells[k] for k in idx]
    cen = np.array([coords[s[0]] for s in sh], dtype=np.float64).reshape(-1, 3)
    ex = np.array([s[2] for s in sh], dtype=np.float64)
    cf = np.array([s[3] for s in sh], dtype=np.float64)
    return cen, ex, cf


def int3c(coords, shells, aux_shells, omega=None, pair_keep=None, aux_idx=None, batch=400000):
    """Three-centre integrals (mu nu | P) as an array [nao, nao, naux_selected].

    omega None: Coulomb 1/r; otherwise erf(omega r)/r. pair_keep: optional boolean [nshell, nshell]
    mask of kept shell pairs (dropped pairs give exact zeros). aux_idx: optional list of auxiliary
    shell indices to evaluate (in that order); default all.
    """
    coords = np.asarray(coords, dtype=np.float64)
    off, nao = shell_offsets(shells)
    if aux_idx is None:
        aux_idx = list(range(len(aux_shells)))
    aux_sel = [aux_shells[k] for k in aux_idx]
    aoff, naux = shell_offsets(aux_sel)
    out = np.zeros((nao, nao, naux))
    nsh = len(shells)
    ls = np.array([s[1] for s in shells])
    lc_all = np.array([s[1] for s in aux_sel])
    for la in (0, 1):
        for lb in (0, 1):
            SA = np.nonzero(ls == la)[0]
            SB = np.nonzero(ls == lb)[0]
            if len(SA) == 0 or len(SB) == 0:
                continue
            pa, pb = np.meshgrid(SA, SB, indexing="ij")
            pa = pa.ravel()
            pb = pb.ravel()
            if pair_keep is not None:
                m = pair_keep[pa, pb]
                pa, pb = pa[m], pb[m]
            for lc in (0, 1):
                SC = np.nonzero(lc_all == lc)[0]
                if len(SC) == 0 or len(pa) == 0:
                    continue
                step = max(1, batch // len(SC))
                for s0 in range(0, len(pa), step):
                    _int3c_block(coords, shells, aux_sel, off, aoff, pa[s0:s0 + step], pb[s0:s0 + step],
                                 SC, la, lb, lc, omega, out)
    assert nsh == len(off)
    return out


def _int3c_block(coords, shells, aux_sel, off, aoff, pa, pb, SC, la, lb, lc, omega, out):
    A, a, ca = _shell_arrays(coords, shells, pa)
    B, b, cb = _shell_arrays(coords, shells, pb)
    C, c, cc = _shell_arrays(coords, aux_sel, SC)
    shape = (len(pa), len(SC))  # every pair with every auxiliary shell
    A = np.broadcast_to(A[:, None, :], shape + (3,))
    B = np.broadcast_to(B[:, None, :], shape + (3,))
    C = np.broadcast_to(C[None, :, :], shape + (3,))
    a = np.broadcast_to(a[:, None], shape)
    b = np.broadcast_to(b[:, None], shape)
    c = np.broadcast_to(c[None, :], shape)
    p = a + b
    mu = a * b / p
    AB = A - B
    K = np.exp(-mu * np.sum(AB * AB, axis=-1))
    P = (a[..., None] * A + b[..., None] * B) / p[..., None]
    alpha = p * c / (p + c)
    a_eff, scale = _operator_alpha(alpha, omega)
    pref = 2.0 * math.pi ** 2.5 / (p * c * np.sqrt(p + c)) * K * scale
    R = hermite_R(la + lb + lc, a_eff, P - C)
    rows0 = np.array(off)[pa]
    cols0 = np.array(off)[pb]
    aux0 = np.array(aoff)[SC]
    for ia, compA in enumerate(cart_components(la)):
        for ib, compB in enumerate(cart_components(lb)):
            Es = [hermite_E(compA[d], compB[d], P[..., d] - A[..., d], P[..., d] - B[..., d], p) for d in range(3)]
            nab = primitive_norm(a, compA) * primitive_norm(b, compB)
            for ic, compC in enumerate(cart_components(lc)):
                Ec = _one_E(compC, None, c)
                val = pref * _contract(Es, Ec, R) * nab * primitive_norm(c, compC)
                val = val * ca[:, None] * cb[:, None] * cc[None, :]
                out[(rows0 + ia)[:, None], (cols0 + ib)[:, None], (aux0 + ic)[None, :]] = val


def int2c(coords, aux_shells, omega=None):
    """Two-centre integrals (P|Q) over the given shells: 1/r (omega None) or erf(omega r)/r."""
    coords = np.asarray(coords, dtype=np.float64)
    off, n = shell_offsets(aux_shells)
    out = np.zeros((n, n))
    ls = np.array([s[1] for s in aux_shells])
    for lp in (0, 1):
        for lq in (0, 1):
            SP = np.nonzero(ls == lp)[0]
            SQ = np.nonzero(ls == lq)[0]
            if len(SP) == 0 or len(SQ) == 0:
                continue
            Pc, pe, pc = _shell_arrays(coords, aux_shells, SP)
            Qc, qe, qc = _shell_arrays(coords, aux_shells, SQ)
            Pc = Pc[:, None, :]
            Qc = Qc[None, :, :]
            p = pe[:, None] * np.ones((1, len(SQ)))
            q = qe[None, :] * np.ones((len(SP), 1))
            alpha = p * q / (p + q)
            a_eff, scale = _operator_alpha(alpha, omega)
            pref = 2.0 * math.pi ** 2.5 / (p * q * np.sqrt(p + q)) * scale
            R = hermite_R(lp + lq, a_eff, np.broadcast_to(Pc - Qc, p.shape + (3,)))
            for ip, cP in enumerate(cart_components(lp)):
                EP = _one_E(cP, None, p)
                for iq, cQ in enumerate(cart_components(lq)):
                    EQ = _one_E(cQ, None, q)
                    val = pref * _contract(EP, EQ, R) * primitive_norm(p, cP) * primitive_norm(q, cQ)
                    val = val * pc[:, None] * qc[None, :]
                    rows = np.array(off)[SP] + ip
                    cols = np.array(off)[SQ] + iq
                    out[rows[:, None], cols[None, :]] = val
    return out


def schwarz_diag(coords, shells):
    """Q_AB = max over functions mu in A, nu in B of sqrt((mu nu|mu nu)), for all shell pairs.

    The 4-centre integral of a product distribution with itself has R_PQ = 0, so only F_n(0) =
    1/(2n+1) enters: (ab|ab) = 2 pi^(5/2)/(p^2 sqrt(2p)) sum E^ab (-1)^. E^ab R(p/2, 0).
    Returns [nshell, nshell] (symmetric).
    """
    coords = np.asarray(coords, dtype=np.float64)
    nsh = len(shells)
    Q = np.zeros((nsh, nsh))
    ls = np.array([s[1] for s in shells])
    for la in (0, 1):
        for lb in (0, 1):
            SA = np.nonzero(ls == la)[0]
            SB = np.nonzero(ls == lb)[0]
            if len(SA) == 0 or len(SB) == 0:
                continue
            pa, pb = np.meshgrid(SA, SB, indexing="ij")
            pa = pa.ravel()
            pb = pb.ravel()
            A, a, ca = _shell_arrays(coords, shells, pa)
            B, b, cb = _shell_arrays(coords, shells, pb)
            p = a + b
            mu = a * b / p
            AB = A - B
            K = np.exp(-mu * np.sum(AB * AB, axis=-1))
            P = (a[:, None] * A + b[:, None] * B) / p[:, None]
            pref = 2.0 * math.pi ** 2.5 / (p * p * np.sqrt(2.0 * p)) * K * K
            R = hermite_R(2 * (la + lb), p / 2.0, np.zeros(p.shape + (3,)))
            best = np.zeros(len(pa))
            for compA in cart_components(la):
                for compB in cart_components(lb):
                    Es = [hermite_E(compA[d], compB[d], P[:, d] - A[:, d], P[:, d] - B[:, d], p) for d in range(3)]
                    n2 = (primitive_norm(a, compA) * primitive_norm(b, compB) * ca * cb) ** 2
                    v = pref * _contract(Es, Es, R) * n2
                    best = np.maximum(best, np.sqrt(np.maximum(v, 0.0)))
            Q[pa, pb] = best
    return Q
