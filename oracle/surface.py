"""Free-surface quantities (paper Sec. 3.4 Steps 4.4-4.6; Eqs. 2-3 and 5).

Vertical velocity (Steps 4.4-4.5).  The paper recovers w = d phi / dz from
phi by "gradient recovery" without naming the method.  Reading: the L2
projection of the element-wise d phi/dz onto the continuous nodal space with
collocated (lumped) GLL mass, evaluated at the free-surface nodes:

    w_n = sum_e m_en (d phi/dz)_e(x_n) / sum_e m_en,   m_en = w_q det J_e(x_n),

over the top-layer elements e that contain surface node n.

Free-surface right-hand side (Step 4.6, Eqs. 2-3 in the weak form Eq. 5).
Reading: collocated GLL quadrature with the lumped surface mass, so each
element's pointwise integrand is averaged onto the node with weights
m^s_en = w_i w_j det J_h (horizontal measure of the surface mesh):

    E_k = -grad eta . grad phi_s + w (1 + |grad eta|^2)
    E_d = -g eta - 1/2 |grad phi_s|^2 + 1/2 w^2 (1 + |grad eta|^2)

with horizontal gradients taken element-wise and eta, phi_s, w nodal.
"""

from __future__ import annotations

import numpy as np

from .gll import gll, lagrange_eval
from .geometry import dof_map, dref, element_coords, horizontal_coords, jacobian, quad_weights, ref_axes


def _bincount(idx, vals, n):
    if np.iscomplexobj(vals):
        return np.bincount(idx, weights=vals.real, minlength=n) + 1j * np.bincount(idx, weights=vals.imag, minlength=n)
    return np.bincount(idx, weights=vals, minlength=n)


def w_surface(mesh, phi, eta, h, xh=None):
    """Recovered vertical velocity at the free-surface nodes: [n_s]."""
    p, nz, n1 = mesh.p, mesh.nz, mesh.p + 1
    _, _, D = gll(p)
    X = element_coords(mesh, eta, h, xh)
    e_top = np.arange(mesh.n_eh) * nz + (nz - 1)
    Jt = jacobian(mesh, X[e_top])[:, p]                      # [n_eh, (j,) i, d, d] at k = p
    dofs = dof_map(mesh)[e_top]
    u = np.asarray(phi)[dofs].reshape((mesh.n_eh,) + (n1,) * mesh.dim)
    grads = [dref(u, D, ax)[:, p] for ax in ref_axes(mesh.dim)]   # at k = p
    Ji = np.linalg.inv(Jt)
    d = mesh.dim
    dphidz = sum(Ji[..., b, d - 1] * grads[b] for b in range(d))
    m = quad_weights(mesh)[p][None] * np.linalg.det(Jt)
    hn = mesh.eh_nodes.ravel()
    num = _bincount(hn, (m * dphidz).ravel(), mesh.n_s)
    den = _bincount(hn, m.ravel(), mesh.n_s)
    return num / den


def surface_metrics(mesh, xh=None):
    """Per surface element: inverse transposed horizontal Jacobian and lumped weights m^s."""
    p, n1 = mesh.p, mesh.p + 1
    x, w, D = gll(p)
    if xh is None:
        xh = horizontal_coords(mesh)
    if mesh.dim == 2:
        xxi = xh[:, :, 0] @ D.T                                  # d x / d xi at node i
        return (1.0 / xxi)[..., None, None], w[None, :] * xxi
    Xh = xh.reshape(mesh.n_eh, n1, n1, 2)                         # (j, i)
    Jh = np.stack([dref(Xh, D, 2), dref(Xh, D, 1)], axis=-1)       # [e, j, i, a(x,y), b(xi,eta)]
    JhiT = np.swapaxes(np.linalg.inv(Jh), -1, -2)
    ms = (w[:, None] * w[None, :])[None] * np.linalg.det(Jh)
    return JhiT, ms


def horizontal_gradient(mesh, f, JhiT):
    """Element-wise horizontal gradient of a nodal surface field: [n_eh, (j,) i, dim-1]."""
    p, n1 = mesh.p, mesh.p + 1
    _, _, D = gll(p)
    fe = np.asarray(f)[mesh.eh_nodes]
    if mesh.dim == 2:
        fx = fe @ D.T
        return (JhiT[..., 0, 0] * fx)[..., None]
    fe = fe.reshape(mesh.n_eh, n1, n1)
    gref = np.stack([dref(fe, D, 2), dref(fe, D, 1)], axis=-1)
    return np.einsum("...ab,...b->...a", JhiT, gref)


def free_surface_rhs(mesh, eta, phi_s, w, g, xh=None, metrics=None):
    """(d eta/dt, d phi_s/dt) at the surface nodes from Eqs. 2-3 (lumped weak form)."""
    JhiT, ms = metrics if metrics is not None else surface_metrics(mesh, xh)
    ge = horizontal_gradient(mesh, eta, JhiT)
    gp = horizontal_gradient(mesh, phi_s, JhiT)
    shape = ge.shape[:-1]
    eta_e = np.asarray(eta)[mesh.eh_nodes].reshape(shape)
    w_e = np.asarray(w)[mesh.eh_nodes].reshape(shape)
    ee = (ge * ge).sum(-1)
    ep = (ge * gp).sum(-1)
    pp = (gp * gp).sum(-1)
    Ek = -ep + w_e * (1.0 + ee)
    Ed = -g * eta_e - 0.5 * pp + 0.5 * w_e * w_e * (1.0 + ee)
    hn = mesh.eh_nodes.ravel()
    den = _bincount(hn, ms.ravel(), mesh.n_s)
    return (_bincount(hn, (ms * Ek).ravel(), mesh.n_s) / den,
            _bincount(hn, (ms * Ed).ravel(), mesh.n_s) / den)


def surface_mass(mesh, xh=None):
    """Lumped surface mass per node: sum_e w_i w_j det J_h."""
    _, ms = surface_metrics(mesh, xh)
    return np.bincount(mesh.eh_nodes.ravel(), weights=ms.ravel(), minlength=mesh.n_s)


# ---------------------------------------------------------------------------------------------
# Consistent (over-integrated) free-surface right-hand side (Eq. 5 with the over-integration of
# Sec. 3.2).  Oracle: test infrastructure only.
#
# Eq. 5 asks for d eta/dt and d phi_s/dt in the surface space such that, for every test function
# nu, <d eta/dt, nu> = <E_k, nu> and <d phi_s/dt, nu> = <E_d, nu> over the (horizontal) surface
# mesh.  Reading: both sides are integrated with nq Gauss-Legendre points per direction (nq >=
# p + 1; larger nq over-integrates the nonlinear terms), so the left side is the consistent
# surface mass matrix M and the result is M^{-1} b.  eta, phi_s, w are the nodal (degree-p)
# fields; their values and horizontal gradients at the Gauss points come from the Lagrange basis
# and the isoparametric horizontal Jacobian there.
# ---------------------------------------------------------------------------------------------


def gauss_tables(p, nq):
    """(B, Bd, W): GLL-Lagrange values and derivatives at nq Gauss points, Gauss weights."""
    from numpy.polynomial import legendre as npleg
    xq, W = npleg.leggauss(nq)
    _, _, D = gll(p)
    B = lagrange_eval(p, xq)                 # [nq, n1]
    return B, B @ D, W                       # l_j' is degree p-1: interpolated exactly at GLL nodes


def surface_quadrature(mesh, nq, xh=None):
    """Per element and Gauss point: inverse transposed Jacobian, W det J, and the tables."""
    p, n1 = mesh.p, mesh.p + 1
    if nq < p + 1:
        raise ValueError("nq >= p + 1")
    if xh is None:
        xh = horizontal_coords(mesh)
    B, Bd, W = gauss_tables(p, nq)
    if mesh.dim == 2:
        xxi = xh[:, :, 0] @ Bd.T                                 # [e, q]
        return (1.0 / xxi)[..., None, None], W[None, :] * xxi, B, Bd
    Xh = xh.reshape(mesh.n_eh, n1, n1, 2)                        # (j, i)
    # d X / d xi and d X / d eta at (q_eta, q_xi)
    Xxi = np.einsum("qj,rk,ejka->eqra", B, Bd, Xh)
    Xet = np.einsum("qj,rk,ejka->eqra", Bd, B, Xh)
    Jq = np.stack([Xxi, Xet], axis=-1)                           # [e, qe, qx, a, b]
    AT = np.swapaxes(np.linalg.inv(Jq), -1, -2)
    wdet = (W[:, None] * W[None, :])[None] * np.linalg.det(Jq)
    return AT, wdet, B, Bd


def _at_points(mesh, f, B, Bd):
    """Values and reference derivatives of a nodal surface field at the Gauss points."""
    n1 = mesh.p + 1
    fe = np.asarray(f)[mesh.eh_nodes]
    if mesh.dim == 2:
        return fe @ B.T, (fe @ Bd.T,)
    fe = fe.reshape(mesh.n_eh, n1, n1)
    val = np.einsum("qj,rk,ejk->eqr", B, B, fe)
    dxi = np.einsum("qj,rk,ejk->eqr", B, Bd, fe)
    det_ = np.einsum("qj,rk,ejk->eqr", Bd, B, fe)
    return val, (dxi, det_)


def _grad(AT, dref_):
    return np.einsum("...ab,...b->...a", AT, np.stack(dref_, axis=-1))


def _project_rhs(mesh, integrand, B):
    """b_i = sum_q W_q det J_q l_i(x_q) integrand_q, assembled: [n_s]."""
    if mesh.dim == 2:
        be = integrand @ B
    else:
        be = np.einsum("qj,rk,eqr->ejk", B, B, integrand).reshape(mesh.n_eh, -1)
    return _bincount(mesh.eh_nodes.ravel(), be.ravel(), mesh.n_s)


def consistent_surface_mass(mesh, nq, xh=None):
    """Dense consistent surface mass matrix with nq Gauss points per direction: [n_s, n_s]."""
    _, wdet, B, _ = surface_quadrature(mesh, nq, xh)
    M = np.zeros((mesh.n_s, mesh.n_s))
    for e in range(mesh.n_eh):
        if mesh.dim == 2:
            Phi = B                                              # [q, i]
            Me = Phi.T @ (wdet[e][:, None] * Phi)
        else:
            Phi = np.einsum("qj,rk->qrjk", B, B).reshape(B.shape[0] ** 2, -1)
            Me = Phi.T @ (wdet[e].reshape(-1)[:, None] * Phi)
        nodes = mesh.eh_nodes[e]
        M[np.ix_(nodes, nodes)] += Me
    return M


def free_surface_rhs_consistent(mesh, eta, phi_s, w, g, nq, xh=None, quad=None, mass=None):
    """(d eta/dt, d phi_s/dt) = M^{-1} (<E_k, l_i>, <E_d, l_i>) with nq-point Gauss quadrature."""
    AT, wdet, B, Bd = quad if quad is not None else surface_quadrature(mesh, nq, xh)
    M = mass if mass is not None else consistent_surface_mass(mesh, nq, xh)
    eta_q, eta_d = _at_points(mesh, eta, B, Bd)
    _, phi_d = _at_points(mesh, phi_s, B, Bd)
    w_q, _ = _at_points(mesh, w, B, Bd)
    ge = _grad(AT, eta_d)
    gp = _grad(AT, phi_d)
    ee = (ge * ge).sum(-1)
    ep = (ge * gp).sum(-1)
    pp = (gp * gp).sum(-1)
    Ek = -ep + w_q * (1.0 + ee)
    Ed = -g * eta_q - 0.5 * pp + 0.5 * w_q * w_q * (1.0 + ee)
    bk = _project_rhs(mesh, wdet * Ek, B)
    bd = _project_rhs(mesh, wdet * Ed, B)
    return np.linalg.solve(M, bk), np.linalg.solve(M, bd)
