"""Modal filter of free-surface fields (paper Sec. 3.2, "Temporal discretization and modal
filtering").  Oracle: test infrastructure only, not part of the product path.

The paper filters a free-surface quantity element by element: nodal values g on an element are
mapped to modal coefficients with the inverse of a Vandermonde matrix, the highest modes are
damped by a filter matrix, and the result is mapped back with the Vandermonde matrix.  It works on
triangles with a modal basis on the reference triangle; the surface elements here are quads (3D)
or intervals (2D), so:

* modal basis: tensor products of orthonormal Legendre polynomials,
  psi_nm(r, s) = Pt_n(s) Pt_m(r), Pt_n = sqrt((2n + 1)/2) P_n, 0 <= n, m <= p;
* Vandermonde: V[(j, i), (n, m)] = psi_nm(x_i, x_j) at the GLL nodes (i along xi, fastest);
* filter matrix: diagonal, F = diag(sigma(n) sigma(m)) with the exponential filter of the
  filtering reference the paper cites (Hesthaven & Warburton):
  sigma(n) = 1 for n <= N_c, exp(-alpha ((n - N_c)/(p - N_c))^s) for n > N_c
  (cutoff N_c, strength alpha, order s; the paper leaves the parameters to its source);
* continuity: a node shared by several surface elements receives the average of the
  element results (each element's filter reproduces every polynomial of degree <= N_c, and so
  does the average, so continuous fields of that degree are left unchanged).

"parity pinned" by tests/test_oracle_filter.py: numpy's own Legendre series (single-element
meshes), polynomial invariance on multi-element meshes, identity limits.
"""

from __future__ import annotations

import numpy as np

from .gll import gll, legendre


def legendre_orthonormal(n: int, x):
    """Pt_n(x) = sqrt((2n+1)/2) P_n(x)."""
    return np.sqrt((2 * n + 1) / 2.0) * legendre(n, x)[0]


def vandermonde_1d(p: int):
    """V[i, n] = Pt_n(x_i) at the p+1 GLL nodes: [p+1, p+1]."""
    x, _, _ = gll(p)
    return np.stack([legendre_orthonormal(n, x) for n in range(p + 1)], axis=1)


def sigma(p: int, cutoff: int, alpha: float, order: int):
    """Exponential filter factors sigma(n), n = 0..p."""
    s = np.ones(p + 1)
    for n in range(cutoff + 1, p + 1):
        s[n] = np.exp(-alpha * ((n - cutoff) / (p - cutoff)) ** order)
    return s


def element_operators(dim: int, p: int, cutoff: int, alpha: float, order: int):
    """(V, diag of F) for one surface element (tensor product in 3D)."""
    V1 = vandermonde_1d(p)
    s1 = sigma(p, cutoff, alpha, order)
    if dim == 2:
        return V1, s1
    # local node (j, i) -> row j*(p+1)+i; mode (n, m) -> column n*(p+1)+m (n along eta)
    return np.kron(V1, V1), np.kron(s1, s1)


def modal_filter(mesh, f, cutoff: int, alpha: float, order: int):
    """Filtered copy of the surface field f[n_s] (the three maps of Sec. 3.2, then averaging)."""
    if not (0 <= cutoff < mesh.p):
        raise ValueError("filter cutoff must satisfy 0 <= cutoff < p")
    V, Fd = element_operators(mesh.dim, mesh.p, cutoff, alpha, order)
    f = np.asarray(f)
    nodes = mesh.eh_nodes
    acc = np.zeros(mesh.n_s, dtype=np.result_type(f.dtype, np.float64))
    mult = np.zeros(mesh.n_s)
    for e in range(mesh.n_eh):
        g = f[nodes[e]]
        g_hat = np.linalg.solve(V, g)          # modal coefficients
        g_hat_f = Fd * g_hat                   # damp the highest modes
        g_f = V @ g_hat_f                      # back to nodal values
        np.add.at(acc, nodes[e], g_f)
        np.add.at(mult, nodes[e], 1.0)
    return acc / mult
