"""Pins for the oracle's quadrature rules (rule exactness and positivity).

The paper only says "fourth-order Gaussian quadrature" for P1 FEM and BEM
(Sec. 3, computational framework paragraph); the oracle reads this as the
symmetric 6-point degree-4 triangle rule and a 27-point degree-5 conical
product rule on tetrahedra.  Exactness is checked against the closed-form
simplex moments  int lambda^alpha = alpha! d! / (|alpha| + d)!  (normalised).
"""
import itertools
import math

import numpy as np
import pytest

import oracle


def simplex_mean(alpha):
    d = len(alpha) - 1
    num = math.prod(math.factorial(a) for a in alpha) * math.factorial(d)
    return num / math.factorial(sum(alpha) + d)


def test_tri6_exact_to_degree_4_and_positive():
    b, w = oracle.rule_tri6()
    assert np.all(w > 0)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(b.sum(1), 1.0, atol=1e-15)
    for deg in range(5):
        for a in itertools.product(range(deg + 1), repeat=3):
            if sum(a) != deg:
                continue
            q = np.sum(w * np.prod(b ** np.array(a), axis=1))
            assert abs(q - simplex_mean(a)) < 1e-15, a
    # not exact at degree 6 (it is a degree-4 rule, not something stronger)
    q6 = np.sum(w * b[:, 0] ** 6)
    assert abs(q6 - simplex_mean((6, 0, 0))) > 1e-6


def test_tri6_matches_published_values():
    # Dunavant (1985), degree 4: orbits (a, a, 1-2a) with a = 0.445948490915965,
    # weight 0.223381589678011, and a = 0.091576213509771, weight 0.109951743655322.
    b, w = oracle.rule_tri6()
    # the repeated barycentric of each point is the orbit parameter a
    a = np.array([np.median(pt) for pt in b])
    order = np.argsort(a)
    assert np.allclose(a[order], [0.091576213509771] * 3 + [0.445948490915965] * 3, atol=1e-14)
    assert np.allclose(w[order], [0.109951743655322] * 3 + [0.223381589678011] * 3, atol=1e-14)


def test_tet27_exact_to_degree_5_and_positive():
    b, w = oracle.rule_tet27()
    assert b.shape == (27, 4)
    assert np.all(w > 0)
    assert abs(w.sum() - 1.0) < 1e-14
    assert np.all(b > 0)
    for deg in range(6):
        for a in itertools.product(range(deg + 1), repeat=4):
            if sum(a) != deg:
                continue
            q = np.sum(w * np.prod(b ** np.array(a), axis=1))
            assert abs(q - simplex_mean(a)) < 2e-15, a


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12])
def test_gauss_legendre01(n):
    x, w = oracle.rule_gauss01(n)
    assert np.all((x > 0) & (x < 1)) and np.all(w > 0)
    for k in range(2 * n):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
    ref_x, ref_w = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, (ref_x + 1) / 2, atol=1e-14)
    assert np.allclose(w, ref_w / 2, atol=1e-14)


@pytest.mark.parametrize("m", [2, 4, 7])
def test_collapsed_triangle_rule(m):
    b, w = oracle.rule_tri_collapsed(m)
    for deg in range(2 * m - 1):
        for a in itertools.product(range(deg + 1), repeat=3):
            if sum(a) == deg:
                q = np.sum(w * np.prod(b ** np.array(a), axis=1))
                assert abs(q - simplex_mean(a)) < 1e-14
