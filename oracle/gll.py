"""Gauss-Lobatto-Legendre reference element.

The paper discretises with C0 nodal Lagrange polynomials of degree p
(Sec. 3.1, spectral elements after the Karniadakis-Sherwin textbook it
cites).  The node family and the quadrature are not stated; the reading used
throughout is the classical spectral-element one: GLL nodes, with collocated
(p+1)-point GLL quadrature (exact to degree 2p-1).

Formulas (textbook):
* nodes: +-1 and the roots of P_p'; equivalently the roots of
  g(x) = x P_p(x) - P_{p-1}(x), whose derivative is (p+1) P_p(x);
* weights: w_i = 2 / (p (p+1) P_p(x_i)^2);
* derivative matrix D_ij = l_j'(x_i):
  D_ij = P_p(x_i) / (P_p(x_j) (x_i - x_j)) for i != j,
  D_00 = -p(p+1)/4, D_pp = p(p+1)/4, other diagonal entries 0.
"""

from __future__ import annotations

import functools

import numpy as np


def legendre(p: int, x):
    """(P_p(x), P_{p-1}(x)) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if p == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for n in range(1, p):
        p0, p1 = p1, ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
    return p1, p0


@functools.lru_cache(maxsize=None)
def gll(p: int):
    """Return (nodes, weights, D) for degree p >= 1 (ascending nodes)."""
    if p < 1:
        raise ValueError("p >= 1")
    n1 = p + 1
    # Chebyshev-Gauss-Lobatto starting guesses
    x = -np.cos(np.pi * np.arange(n1) / p)
    for _ in range(100):
        pp, pm = legendre(p, x)
        dx = (x * pp - pm) / ((p + 1) * pp)
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    pp, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * pp ** 2)
    D = np.zeros((n1, n1))
    for i in range(n1):
        for j in range(n1):
            if i != j:
                D[i, j] = pp[i] / (pp[j] * (x[i] - x[j]))
    D[0, 0] = -p * (p + 1) / 4.0
    D[p, p] = p * (p + 1) / 4.0
    x.setflags(write=False)
    w.setflags(write=False)
    D.setflags(write=False)
    return x, w, D


def lagrange_eval(p: int, xq):
    """Values of the p+1 GLL Lagrange polynomials at points xq: [len(xq), p+1]."""
    x, _, _ = gll(p)
    xq = np.atleast_1d(np.asarray(xq, dtype=np.float64))
    L = np.ones((len(xq), p + 1))
    for j in range(p + 1):
        for m in range(p + 1):
            if m != j:
                L[:, j] *= (xq - x[m]) / (x[j] - x[m])
    return L
