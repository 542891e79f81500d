"""Pins of the oracle's angular and radial building blocks.

Each check compares the oracle with something it does not share code with:
scipy's spherical harmonics and Bessel functions, sympy's Wigner-3j symbols,
closed forms, or an independent quadrature.
"""

import numpy as np
import pytest
from scipy.special import sph_harm_y, spherical_jn, spherical_yn

import oracle


def _l_of(L):
    return int(np.floor(np.sqrt(L) + 1e-9))


def _real_from_scipy(lmax, r):
    """Real harmonics without the Condon-Shortley factor, from scipy's complex
    Y_l^m (which carries it): Y_{l,+m} = sqrt2 (-1)^m Re Y_l^m,
    Y_{l,-m} = sqrt2 (-1)^m Im Y_l^m."""
    x, y, z = r
    rr = np.linalg.norm(r)
    th = np.arccos(z / rr)
    ph = np.arctan2(y, x)
    out = np.zeros((lmax + 1) ** 2)
    for l in range(lmax + 1):
        out[l * l + l] = sph_harm_y(l, 0, th, ph).real
        for m in range(1, l + 1):
            c = sph_harm_y(l, m, th, ph)
            out[l * l + l + m] = np.sqrt(2) * (-1) ** m * c.real
            out[l * l + l - m] = np.sqrt(2) * (-1) ** m * c.imag
    return out


@pytest.mark.parametrize("seed", range(4))
def test_ylm_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    for _ in range(10):
        r = rng.normal(size=3) * rng.uniform(0.1, 20)
        np.testing.assert_allclose(oracle.ylm(8, r), _real_from_scipy(8, r), rtol=0, atol=2e-13)


def test_ylm_orthonormal_independent_quadrature():
    # numpy's Gauss-Legendre (not the oracle's) x a uniform phi rule
    lmax = 6
    x, w = np.polynomial.legendre.leggauss(20)
    nph = 30
    G = np.zeros(((lmax + 1) ** 2,) * 2)
    for xi, wi in zip(x, w):
        st = np.sqrt(1 - xi * xi)
        for b in range(nph):
            ph = 2 * np.pi * b / nph
            Y = oracle.ylm(lmax, [st * np.cos(ph), st * np.sin(ph), xi])
            G += wi * 2 * np.pi / nph * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-14)


def _real_gaunt_from_sympy(lmax):
    """Real Gaunt table from sympy's complex Gaunt coefficients (a closed form
    in Wigner 3j symbols) and the unitary map between real (no Condon-Shortley
    factor) and complex harmonics."""
    from sympy.physics.wigner import gaunt as cgaunt

    def U(l):
        # Y^R_{l,m} = sum_mu U[m, mu] Y_l^mu (complex Y with Condon-Shortley factor)
        u = np.zeros((2 * l + 1, 2 * l + 1), complex)
        s2 = 1 / np.sqrt(2)
        for m in range(-l, l + 1):
            if m == 0:
                u[l, l] = 1
            elif m > 0:
                u[l + m, l + m] = (-1) ** m * s2
                u[l + m, l - m] = s2
            else:
                am = -m
                u[l + m, l + am] = (-1) ** am * s2 / 1j
                u[l + m, l - am] = -s2 / 1j
        return u

    kk = (lmax + 1) ** 2
    kk2 = (2 * lmax + 1) ** 2
    C = np.zeros((kk, kk, kk2))
    cache = {}
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for l3 in range(abs(l1 - l2), l1 + l2 + 1, 2):
                T = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
                for m1 in range(-l1, l1 + 1):
                    for m2 in range(-l2, l2 + 1):
                        m3 = -m1 - m2
                        if abs(m3) <= l3:
                            key = (l1, l2, l3, m1, m2, m3)
                            if key not in cache:
                                cache[key] = float(cgaunt(l1, l2, l3, m1, m2, m3))
                            T[l1 + m1, l2 + m2, l3 + m3] = cache[key]
                R = np.einsum("ai,bj,ck,ijk->abc", U(l1), U(l2), U(l3), T).real
                for a in range(2 * l1 + 1):
                    for b in range(2 * l2 + 1):
                        for c in range(2 * l3 + 1):
                            C[l1 * l1 + a, l2 * l2 + b, l3 * l3 + c] = R[a, b, c]
    return C


@pytest.mark.parametrize("lmax,nnz", [(3, 708), (4, 2229)])
def test_gaunt_matches_wigner3j(lmax, nnz):
    C, n = oracle.gaunt(lmax)
    ref = _real_gaunt_from_sympy(lmax)
    np.testing.assert_allclose(C, ref, rtol=0, atol=2e-15)
    assert n == nnz == int(np.count_nonzero(np.abs(ref) > 1e-12))


def test_gaunt_special_cases_and_symmetry():
    lmax = 4
    C, _ = oracle.gaunt(lmax)
    kk = (lmax + 1) ** 2
    # C^{L''}_{00, L'} = delta_{L' L''} / sqrt(4 pi)
    np.testing.assert_allclose(C[0, :, :kk], np.eye(kk) / np.sqrt(4 * np.pi), atol=1e-15)
    # full index symmetry over the common range
    sub = C[:, :, :kk]
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1)]:
        np.testing.assert_allclose(sub, sub.transpose(perm), atol=1e-15)


def _h_scipy(l, z):
    return spherical_jn(l, z) + 1j * spherical_yn(l, z)


@pytest.mark.parametrize("z", [3.5 + 0.02j, 7.0 + 1.3j, 12.0 + 0.5j, 4.2 + 4.0j, 20.0 + 0.01j])
def test_hankel_matches_scipy_and_closed_forms(z):
    h = oracle.hankel(8, z)
    for l in range(9):
        ref = _h_scipy(l, z)
        # scipy forms j + i y, whose terms grow like e^{Im z} while h decays
        # like e^{-Im z}: its own error scales with |j| + |y|.
        scale = abs(spherical_jn(l, z)) + abs(spherical_yn(l, z))
        assert abs(h[l] - ref) <= 1e-14 * scale
    assert abs(h[0] - np.exp(1j * z) / (1j * z)) <= 1e-15 * abs(h[0])
    assert abs(h[1] + np.exp(1j * z) * (1 / z + 1j / z ** 2)) <= 1e-15 * abs(h[1])
    for l in range(1, 8):  # h_{l+1} = (2l+1)/z h_l - h_{l-1}
        assert abs(h[l + 1] - ((2 * l + 1) / z * h[l] - h[l - 1])) <= 1e-12 * abs(h[l + 1])
