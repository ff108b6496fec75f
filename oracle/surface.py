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

from .gll import gll
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
