"""Numerical-quadrature pins for the oracle integrals (independent of the Hermite-Gaussian code).

* The electrostatic potential of a normalised primitive s Gaussian of exponent g at C is
  V_s(r) = N (pi/g)^(3/2) erf(sqrt(g) d)/d with d = |r - C|; a p_k Gaussian (r_k - C_k) e^{-g d^2}
  equals (1/2g) d/dC_k of the s Gaussian, so its potential is (1/2g) d/dC_k of the s potential.
  For erf(w r)/r the potential of a Gaussian of exponent g is that of exponent g w^2/(g + w^2).
* (mu nu|P) = int mu(r) nu(r) V_P(r) d^3r is then a smooth 3-D integral done with a product
  Gauss-Hermite rule centred on the Gaussian product centre of mu nu.
* The self-repulsion (mu nu|mu nu) is done in Fourier space:
  (rho|rho) = 1/(2 pi^2) int_0^inf dk int dOmega |rho^(k)|^2, with rho^ the analytic transform.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.hermite import hermgauss
from numpy.polynomial.legendre import leggauss
from scipy.special import erf


def norm(alpha, l):
    ns = (2.0 * alpha / math.pi) ** 0.75
    return ns if l == 0 else ns * 2.0 * math.sqrt(alpha)


def functions(coords, shells):
    """Expand shells into (centre, exponent, cartesian exponent triple, normalisation * coef)."""
    out = []
    for (atom, l, e, cf) in shells:
        comps = [(0, 0, 0)] if l == 0 else [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
        for c in comps:
            out.append((np.asarray(coords[atom], float), e, c, cf * norm(e, l)))
    return out


def potential(r, C, g, comp, nrm, omega=None):
    """Potential at points r [...,3] of nrm * (r-C)^comp exp(-g |r-C|^2) (l <= 1)."""
    ge = g if omega is None else g * omega * omega / (g + omega * omega)
    d = r - C
    R = np.sqrt(np.sum(d * d, axis=-1))
    R = np.maximum(R, 1e-300)
    pref = nrm * (math.pi / g) ** 1.5
    f = erf(math.sqrt(ge) * R) / R
    if sum(comp) == 0:
        return pref * f
    fp = (2.0 * math.sqrt(ge) / math.sqrt(math.pi)) * np.exp(-ge * R * R) / R - erf(math.sqrt(ge) * R) / (R * R)
    k = comp.index(1)
    return pref / (2.0 * g) * fp * (C[k] - r[..., k]) / R


def gh_grid(center, p, n):
    """Product Gauss-Hermite nodes/weights for int f(r) exp(-p |r-center|^2) d^3 r."""
    x, w = hermgauss(n)
    s = 1.0 / math.sqrt(p)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1) * s + center
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * s ** 3
    return X, W


def int3c_quad(coords, shells, aux, omega=None, n=48):
    fa = functions(coords, shells)
    fx = functions(coords, aux)
    out = np.zeros((len(fa), len(fa), len(fx)))
    for i, (A, a, ca, na) in enumerate(fa):
        for j, (B, b, cb, nb) in enumerate(fa):
            p = a + b
            P = (a * A + b * B) / p
            K = math.exp(-a * b / p * float(np.sum((A - B) ** 2)))
            X, W = gh_grid(P, p, n)
            poly = np.ones(X.shape[:-1])
            for d in range(3):
                poly *= (X[..., d] - A[d]) ** ca[d] * (X[..., d] - B[d]) ** cb[d]
            for k, (C, g, cc, nc) in enumerate(fx):
                out[i, j, k] = np.sum(W * K * na * nb * poly * potential(X, C, g, cc, nc, omega))
    return out


def int2c_quad(coords, aux, omega=None, n=48):
    fx = functions(coords, aux)
    out = np.zeros((len(fx), len(fx)))
    for i, (A, a, ca, na) in enumerate(fx):
        X, W = gh_grid(A, a, n)
        poly = np.ones(X.shape[:-1])
        for d in range(3):
            poly *= (X[..., d] - A[d]) ** ca[d]
        for k, (C, g, cc, nc) in enumerate(fx):
            out[i, k] = np.sum(W * na * poly * potential(X, C, g, cc, nc, omega))
    return out


def _ft_poly_1d(nA, nB, PA, PB, p, k):
    """Fourier transform factor of (x-A)^nA (x-B)^nB exp(-p (x-P)^2), without the Gaussian part.

    With u = x - P: (x-A) = u + PA and (x-B) = u + PB where PA = P - A, PB = P - B; the transform of
    u^n exp(-p u^2) over exp(-i k u) is (1, -i k/(2p), 1/(2p) - k^2/(4p^2)) x sqrt(pi/p) exp(-k^2/4p)
    for n = 0, 1, 2.
    """
    m = [1.0 + 0j, -1j * k / (2 * p), 1.0 / (2 * p) - k * k / (4 * p * p)]
    # expand (u + PA)^nA (u + PB)^nB
    coef = {0: 1.0}
    for (n, s) in ((nA, PA), (nB, PB)):
        for _ in range(n):
            new = {}
            for deg, c in coef.items():
                new[deg + 1] = new.get(deg + 1, 0.0) + c
                new[deg] = new.get(deg, 0.0) + c * s
            coef = new
    return sum(c * m[deg] for deg, c in coef.items())


def self_repulsion_kspace(fA, fB, nrad=200):
    """(mu nu|mu nu) for two primitive functions by Fourier-space quadrature."""
    (A, a, ca, na), (B, b, cb, nb) = fA, fB
    p = a + b
    P = (a * A + b * B) / p
    K = math.exp(-a * b / p * float(np.sum((A - B) ** 2)))
    PA, PB = P - A, P - B
    # angular grid: Gauss-Legendre in cos(theta) x uniform phi (exact for these polynomials)
    ct, wt = leggauss(16)
    nphi = 32
    phi = np.arange(nphi) * 2 * math.pi / nphi
    st = np.sqrt(1 - ct * ct)
    dirs = np.stack([st[:, None] * np.cos(phi)[None, :], st[:, None] * np.sin(phi)[None, :],
                     np.broadcast_to(ct[:, None], (16, nphi))], -1).reshape(-1, 3)
    wang = (wt[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).ravel()
    # radial: Gauss-Legendre on [0, kmax], the integrand decays like exp(-k^2/(2p))
    kmax = math.sqrt(2 * p * 80.0)
    xr, wr = leggauss(nrad)
    kk = 0.5 * kmax * (xr + 1)
    wk = 0.5 * kmax * wr
    total = 0.0
    for k, w in zip(kk, wk):
        kv = k * dirs
        f = np.ones(len(dirs), dtype=complex)
        for d in range(3):
            f *= _ft_poly_1d(ca[d], cb[d], PA[d], PB[d], p, kv[:, d])
        g = (math.pi / p) ** 3 * math.exp(-k * k / (2 * p))
        total += w * np.sum(wang * np.abs(f) ** 2) * g
    return (K * na * nb) ** 2 * total / (2 * math.pi ** 2)
