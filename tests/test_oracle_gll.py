"""Pins for the GLL reference element (oracle/gll.py) against closed forms.

The paper uses nodal Lagrange P^p spectral elements (Sec. 3.1); the GLL
family and its collocated quadrature are the reading adopted (textbook
spectral-element values below are exact closed forms, not oracle output).
"""

import math

import numpy as np
import pytest

from oracle.gll import gll, lagrange_eval


def test_p4_closed_form():
    x, w, _ = gll(4)
    r = math.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


def test_p2_p3_closed_form():
    x, w, _ = gll(2)
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w, _ = gll(3)
    r = 1 / math.sqrt(5)
    np.testing.assert_allclose(x, [-1, -r, r, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


def test_p5_p6_tabulated():
    x, _, _ = gll(5)
    np.testing.assert_allclose(x[3:], [0.2852315164806451, 0.7650553239294647, 1.0], atol=1e-13)
    x, _, _ = gll(6)
    np.testing.assert_allclose(x[3:], [0.0, 0.4688487934707142, 0.8302238962785670, 1.0], atol=1e-13)


@pytest.mark.parametrize("p", range(1, 11))
def test_quadrature_and_derivative(p):
    x, w, D = gll(p)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.all(np.diff(x) > 0) and np.all(w > 0)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    # D annihilates constants and differentiates every polynomial of degree <= p exactly
    assert np.abs(D @ np.ones(p + 1)).max() < 1e-12 * p * p
    for k in range(1, p + 1):
        np.testing.assert_allclose(D @ x ** k, k * x ** (k - 1), atol=1e-12 * p * p)
    # collocated quadrature exact to degree 2p-1 ...
    for k in range(0, 2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-13
    # ... and not beyond (it is Lobatto, not Gauss)
    assert abs(w @ x ** (2 * p) - 2.0 / (2 * p + 1)) > 1e-6


def test_lagrange_interpolation():
    p = 5
    x, _, _ = gll(p)
    L = lagrange_eval(p, x)
    np.testing.assert_allclose(L, np.eye(p + 1), atol=1e-14)
    xq = np.linspace(-1, 1, 17)
    np.testing.assert_allclose(lagrange_eval(p, xq) @ (x ** 3 - 2 * x), xq ** 3 - 2 * xq, atol=1e-13)
