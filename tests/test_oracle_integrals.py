"""Pins of the oracle integrals against mathematics that does not use the Hermite-Gaussian code.

Boys function: closed form of F_0 and direct numerical quadrature of its defining integral.
Three- and two-centre integrals (1/r and erf(w r)/r): 3-D quadrature against the analytic potential
of the auxiliary Gaussian. Diagonal four-centre integrals: Fourier-space quadrature.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erf

from oracle import integrals as I
from tests import quadrature as Q

COORDS = np.array([[0.0, 0.0, 0.0], [0.9, -0.4, 1.3], [-1.1, 0.7, 0.4]])
SHELLS = [(0, 0, 0.45, 1.0), (0, 1, 0.6, 1.0), (1, 0, 0.3, 1.0), (1, 1, 0.8, 1.0), (2, 0, 1.2, 0.7)]
AUX = [(0, 0, 0.25, 1.0), (1, 1, 0.35, 1.0), (2, 1, 0.5, 1.3), (2, 0, 0.15, 1.0)]


@pytest.mark.parametrize("T", [1e-9, 1e-4, 0.3, 1.0, 7.5, 25.0, 80.0, 400.0])
def test_boys_F0_closed_form(T):
    ref = 0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T))
    assert abs(I.boys(0, T) - ref) <= 5e-15 * ref


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("T", [0.0, 1e-13, 1e-6, 0.05, 1.0, 3.3, 12.0, 40.0])
def test_boys_quadrature(n, T):
    ref, err = quad(lambda t: t ** (2 * n) * math.exp(-T * t * t), 0.0, 1.0, epsabs=1e-16, epsrel=1e-14)
    got = float(I.boys(n, T))
    assert abs(got - ref) <= 2e-14 * ref


def test_boys_zero_limit():
    for n in range(6):
        assert I.boys(n, 0.0) == pytest.approx(1.0 / (2 * n + 1), rel=1e-15)


@pytest.mark.parametrize("omega", [None, 0.2, 1.7])
def test_int3c_against_quadrature(omega):
    got = I.int3c(COORDS, SHELLS, AUX, omega)
    ref = Q.int3c_quad(COORDS, SHELLS, AUX, omega, n=40)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-11 * scale


@pytest.mark.parametrize("omega", [None, 0.2, 1.7])
def test_int2c_against_quadrature(omega):
    got = I.int2c(COORDS, AUX, omega)
    ref = Q.int2c_quad(COORDS, AUX, omega, n=48)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_int3c_permutation_symmetry():
    V = I.int3c(COORDS, SHELLS, AUX)
    assert np.abs(V - V.transpose(1, 0, 2)).max() <= 1e-15 * np.abs(V).max()
    W = I.int3c(COORDS, SHELLS, AUX, 0.3)
    assert np.abs(W - W.transpose(1, 0, 2)).max() <= 1e-15 * np.abs(W).max()


def test_erf_operator_limits():
    plain = I.int3c(COORDS, SHELLS, AUX)
    big = I.int3c(COORDS, SHELLS, AUX, 1e6)  # erf(w r) -> 1
    assert np.abs(big - plain).max() <= 1e-9 * np.abs(plain).max()
    small = I.int3c(COORDS, SHELLS, AUX, 1e-4)  # erf(w r)/r -> 2w/sqrt(pi): integrals scale with w
    assert np.abs(small).max() <= 1e-3 * np.abs(plain).max()
    m2 = I.int2c(COORDS, AUX, 1e6)
    assert np.abs(m2 - I.int2c(COORDS, AUX)).max() <= 1e-9 * np.abs(m2).max()


def test_translation_invariance():
    shift = np.array([3.1, -2.2, 0.7])
    a = I.int3c(COORDS, SHELLS, AUX, 0.4)
    b = I.int3c(COORDS + shift, SHELLS, AUX, 0.4)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_metric_positive_definite():
    for om in (None, 0.2):
        w = np.linalg.eigvalsh(I.int2c(COORDS, AUX, om))
        assert w.min() > 0


def test_schwarz_diag_against_kspace():
    Qab = I.schwarz_diag(COORDS, SHELLS)
    funcs = Q.functions(COORDS, SHELLS)
    off, _ = I.shell_offsets(SHELLS)
    for A in range(len(SHELLS)):
        for B in range(A + 1):
            nA = 1 if SHELLS[A][1] == 0 else 3
            nB = 1 if SHELLS[B][1] == 0 else 3
            best = 0.0
            for i in range(nA):
                for j in range(nB):
                    v = Q.self_repulsion_kspace(funcs[off[A] + i], funcs[off[B] + j])
                    best = max(best, math.sqrt(v))
            assert Qab[A, B] == pytest.approx(best, rel=1e-11)
            assert Qab[B, A] == pytest.approx(best, rel=1e-11)


def test_schwarz_bounds_3c():
    """Cauchy-Schwarz: |(mu nu|P)| <= sqrt((mu nu|mu nu)) sqrt((P|P))."""
    V = I.int3c(COORDS, SHELLS, AUX)
    qP = np.sqrt(np.diag(I.int2c(COORDS, AUX)))
    Qab = I.schwarz_diag(COORDS, SHELLS)
    off, nao = I.shell_offsets(SHELLS)
    sh_of = np.repeat(np.arange(len(SHELLS)), [1 if s[1] == 0 else 3 for s in SHELLS])
    bound = Qab[sh_of][:, sh_of][:, :, None] * qP[None, None, :]
    assert np.all(np.abs(V) <= bound * (1 + 1e-12))
