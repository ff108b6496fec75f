"""The Laplace operator of the weak form a[phi; nu] = <grad phi, grad nu>_Omega (paper Eq. 4).

Two independent routes:

* R1 ``assemble_dense``: element matrices from explicit reference-gradient
  tables, K_e = sum_ab B_a^T diag(G_ab) B_b, added into a dense global matrix.
* R2 ``apply``: the plain sum-factorised matrix-free product: gradients by
  one-dimensional D contractions, the per-point G multiply, transposed D
  contractions, then a scatter-add over the global numbering.

With natural (homogeneous Neumann) boundaries on the bottom, walls and
bodies (Eq. 1), and periodicity carried entirely by the numbering, the
assembled operator is the full Neumann matrix; the free-surface Dirichlet
rows are handled in ``solve``.  ``neumann_load`` integrates prescribed flux
data (grad phi . n) over the bottom and the tagged side faces.
"""

from __future__ import annotations

import numpy as np

from .gll import gll
from .geometry import dof_map, dref, element_coords, jacobian, ref_axes


def grad_tables(mesh):
    """B[a][q, n] = d l_n / d xi_a at element node q (flat (k, j, i) order)."""
    _, _, D = gll(mesh.p)
    I = np.eye(mesh.p + 1)
    if mesh.dim == 3:
        return [np.kron(np.kron(I, I), D), np.kron(np.kron(I, D), I), np.kron(np.kron(D, I), I)]
    return [np.kron(I, D), np.kron(D, I)]


def element_matrices(mesh, G):
    """K[e] = sum_ab B_a^T diag(G_ab) B_b for every element."""
    B = grad_tables(mesh)
    d = mesh.dim
    n_e = G.shape[0]
    Gf = G.reshape(n_e, -1, d, d)
    npt = Gf.shape[1]
    K = np.zeros((n_e, npt, npt), dtype=G.dtype)
    for a in range(d):
        for b in range(d):
            K += (B[a].T[None, :, :] * Gf[:, None, :, a, b]) @ B[b]
    return K


def assemble_dense(mesh, G):
    """R1: dense global stiffness matrix A (n_v x n_v)."""
    K = element_matrices(mesh, G)
    dofs = dof_map(mesh)
    A = np.zeros((mesh.n_v, mesh.n_v), dtype=G.dtype)
    for e in range(K.shape[0]):
        A[np.ix_(dofs[e], dofs[e])] += K[e]
    return A


def _scatter(mesh, dofs, ye):
    flat_idx = dofs.ravel()
    vals = ye.reshape(-1)
    if np.iscomplexobj(vals):
        return (np.bincount(flat_idx, weights=vals.real, minlength=mesh.n_v)
                + 1j * np.bincount(flat_idx, weights=vals.imag, minlength=mesh.n_v))
    return np.bincount(flat_idx, weights=vals, minlength=mesh.n_v)


def apply(mesh, G, x, dofs=None):
    """R2: y = A x by sum factorisation (no assembled matrix)."""
    _, _, D = gll(mesh.p)
    if dofs is None:
        dofs = dof_map(mesh)
    n1 = mesh.p + 1
    shape = (dofs.shape[0],) + (n1,) * mesh.dim
    u = np.asarray(x)[dofs].reshape(shape)
    axes = ref_axes(mesh.dim)
    grads = [dref(u, D, ax) for ax in axes]
    ye = 0
    for a, ax in enumerate(axes):
        va = sum(G[..., a, b] * grads[b] for b in range(mesh.dim))
        ye = ye + dref(va, D.T, ax)
    return _scatter(mesh, dofs, ye)


def diagonal(mesh, G, dofs=None):
    """diag(A) from the element matrices' diagonals (used by the Jacobi preconditioner); G and
    dofs may cover a subset of the elements (dof_map(mesh, cols=...)), as in apply."""
    B = grad_tables(mesh)
    d = mesh.dim
    Gf = G.reshape(G.shape[0], -1, d, d)
    de = 0
    for a in range(d):
        for b in range(d):
            de = de + np.einsum("qn,eq,qn->en", B[a], Gf[:, :, a, b], B[b])
    return _scatter(mesh, dof_map(mesh) if dofs is None else dofs, de)


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)


def face_area_vectors(mesh, J):
    """Outward area vectors n dS / (d ref) at the nodes of every Neumann face.

    Returns a list of (element ids, node-selector tuple, area vectors, face weights).
    Faces: the bottom of layer 0 everywhere, and side faces tagged wall/body.
    """
    _, w, _ = gll(mesh.p)
    p, nz = mesh.p, mesh.nz
    out = []
    cols = np.arange(mesh.n_eh)
    if mesh.dim == 3:
        e_bot = cols * nz
        Jb = J[e_bot, 0]                                   # [ne, j, i, 3, 3]
        nb = -_cross(Jb[..., :, 0], Jb[..., :, 1])
        out.append((e_bot, (0, slice(None), slice(None)), nb, w[:, None] * w[None, :]))
        side_defs = [
            (0, lambda Je: -_cross(Je[:, :, 0, :, :, 2], Je[:, :, 0, :, :, 0]), (slice(None), 0, slice(None))),
            (1, lambda Je: _cross(Je[:, :, :, p, :, 1], Je[:, :, :, p, :, 2]), (slice(None), slice(None), p)),
            (2, lambda Je: _cross(Je[:, :, p, :, :, 2], Je[:, :, p, :, :, 0]), (slice(None), p, slice(None))),
            (3, lambda Je: -_cross(Je[:, :, :, 0, :, 1], Je[:, :, :, 0, :, 2]), (slice(None), slice(None), 0)),
        ]
        for side, fn, sel in side_defs:
            cs = cols[mesh.eh_face_tag[:, side] != 0]
            if len(cs) == 0:
                continue
            es = (cs[:, None] * nz + np.arange(nz)[None, :]).ravel()
            nvec = fn(J[es])                               # [ne, k, (i|j), 3]
            out.append((es, sel, nvec, w[:, None] * w[None, :]))
        return out
    # 2D slice: J[e, k, i, a, b], a in (x, z), b in (xi, zeta)
    e_bot = cols * nz
    Jb = J[e_bot, 0]                                       # [ne, i, 2, 2]
    nb = np.stack([Jb[..., 1, 0], -Jb[..., 0, 0]], -1)
    out.append((e_bot, (0, slice(None)), nb, w))
    for side, sgn, ii in ((0, -1.0, 0), (1, 1.0, p)):
        cs = cols[mesh.eh_face_tag[:, side] != 0]
        if len(cs) == 0:
            continue
        es = (cs[:, None] * nz + np.arange(nz)[None, :]).ravel()
        Je = J[es][:, :, ii]                               # [ne, k, 2, 2]
        nvec = sgn * np.stack([Je[..., 1, 1], -Je[..., 0, 1]], -1)
        out.append((es, (slice(None), ii), nvec, w))
    return out


def neumann_load(mesh, eta, h, q):
    """f_i = sum over Neumann faces of int (q . n) l_i dS with nodal flux vectors q [dim, n_v]."""
    X = element_coords(mesh, eta, h)
    J = jacobian(mesh, X)
    dofs = dof_map(mesh)
    n1 = mesh.p + 1
    dofs_n = dofs.reshape((dofs.shape[0],) + (n1,) * mesh.dim)
    q = np.asarray(q)
    f = np.zeros(mesh.n_v, dtype=np.result_type(q, X))
    for es, sel, nvec, wf in face_area_vectors(mesh, J):
        idx = dofs_n[(es,) + sel]                          # [ne, ...face nodes]
        qn = sum(q[a][idx] * nvec[..., a] for a in range(mesh.dim))
        np.add.at(f, idx.ravel(), (qn * wf[None]).ravel())
    return f
