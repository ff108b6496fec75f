"""Laplace problem for the velocity potential (paper Eq. 1; Sec. 3.4 Steps 4.2-4.3).

Dirichlet data phi = phi_eta on the free surface (the top node level, which
is the paper's surface map m taken as a slice of the layer-major volume
vector), natural Neumann data on the bottom, walls and bodies.  With
S = surface nodes and I = the rest:

    phi_S = phi_s,   A_II phi_I = f_I - A_IS phi_s,

f the Neumann load (zero unless flux data are prescribed).  The paper solves
with CG (Sec. 4, solver settings); here a dense direct solve is used for tiny
meshes and Jacobi-preconditioned CG (bilinear inner products, so it is also
valid for complex-step perturbations) for larger ones.  Stopping rule (a
reading; the paper does not state the norm): unpreconditioned
||r||_2 <= rtol ||b||_2 with b = f_I - A_IS phi_s.
"""

from __future__ import annotations

import numpy as np

from . import operator as op


def surface_slice(mesh):
    top = mesh.p * mesh.nz
    return slice(top * mesh.n_s, (top + 1) * mesh.n_s)


def interior_mask(mesh):
    m = np.ones(mesh.n_v, dtype=bool)
    m[surface_slice(mesh)] = False
    return m


def solve_dense(mesh, A, phi_s, f=None):
    """Direct solve of the lifted system with an assembled matrix."""
    I = interior_mask(mesh)
    S = surface_slice(mesh)
    phi = np.zeros(mesh.n_v, dtype=np.result_type(A, phi_s))
    phi[S] = phi_s
    b = -A[np.ix_(I, ~I)] @ np.asarray(phi_s)
    if f is not None:
        b = b + f[I]
    phi[I] = np.linalg.solve(A[np.ix_(I, I)], b)
    return phi


def solve_cg(mesh, G, phi_s, f=None, x0=None, rtol=1e-13, max_iter=100000, dofs=None, return_info=False):
    """Jacobi-preconditioned CG on A_II with the matrix-free apply."""
    I = interior_mask(mesh)
    S = surface_slice(mesh)
    if dofs is None:
        from .geometry import dof_map
        dofs = dof_map(mesh)
    dt = np.result_type(G, phi_s)
    phi = np.zeros(mesh.n_v, dtype=dt)
    if x0 is not None:
        phi[:] = x0
    phi[S] = phi_s
    lift = np.zeros(mesh.n_v, dtype=dt)
    lift[S] = phi_s
    b = -op.apply(mesh, G, lift, dofs)
    if f is not None:
        b = b + f
    b[~I] = 0.0
    bnorm = np.sqrt(np.real(b @ np.conj(b)))
    dinv = np.zeros(mesh.n_v)
    d = op.diagonal(mesh, G)
    dinv[I] = 1.0 / d[I]
    r = b - op.apply(mesh, G, np.where(I, phi, 0.0), dofs)
    r[~I] = 0.0
    z = dinv * r
    pdir = z.copy()
    rz = r @ z
    it = 0
    while True:
        rn = np.sqrt(np.real(r @ np.conj(r)))
        if rn <= rtol * bnorm or bnorm == 0.0:
            break
        if it >= max_iter:
            raise RuntimeError(f"CG did not converge: ||r||/||b|| = {rn / bnorm:g} after {it} iterations")
        q = op.apply(mesh, G, pdir, dofs)
        q[~I] = 0.0
        pq = pdir @ q
        if np.real(pq) <= 0.0:
            raise RuntimeError("CG breakdown: p^T A p <= 0")
        alpha = rz / pq
        phi = phi + alpha * pdir
        r = r - alpha * q
        z = dinv * r
        rz_new = r @ z
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
        it += 1
    if return_info:
        return phi, dict(iters=it, rel_res=float(rn / bnorm) if bnorm else 0.0)
    return phi


def line_unknowns(mesh):
    """Volume indices of every vertical node line's unknowns: [n_s][p nz] (level-major
    numbering v n_s + n, levels 0 .. p nz - 1; the free-surface level is Dirichlet)."""
    nl = mesh.p * mesh.nz
    return np.arange(nl)[None, :] * mesh.n_s + np.arange(mesh.n_s)[:, None]


def line_blocks(mesh, A):
    """The vertical line blocks of A_II: for every horizontal node n, the principal submatrix of
    the assembled operator on the unknowns of its node line.  They form the block-diagonal part
    of A_II that a vertical line smoother inverts in place of the Jacobi diagonal (a multilevel
    preconditioner in the role of the paper's algebraic multigrid, Sec. 4 solver settings)."""
    idx = line_unknowns(mesh)
    return np.stack([A[np.ix_(ix, ix)] for ix in idx])


def line_solve(mesh, blocks, r):
    """z = B^-1 r with B the block-diagonal line part of A_II (dense solve per line); z is zero
    on the free-surface level."""
    idx = line_unknowns(mesh)
    z = np.zeros(mesh.n_v, dtype=np.result_type(blocks, r))
    for n, ix in enumerate(idx):
        z[ix] = np.linalg.solve(blocks[n], np.asarray(r)[ix])
    return z
