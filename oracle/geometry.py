"""Extruded, free-surface-following geometry (paper Sec. 3.1.2, Step 4.1).

The horizontal mesh is extruded into nz layers; each vertical line of nodes
is translated so that the column spans [-h, eta] (the paper moves each column
of points to follow eta, and treats bathymetry the same way).  Reading of the
unstated translation rule: sigma-linear, i.e. node level v sits at
    z = -h + sigma_v (eta + h),
with sigma_v = s_l + (s_{l+1} - s_l)(xi_k + 1)/2 for v = l p + k (layer
fractions s, uniform unless given).  Element coordinates are isoparametric
(degree p): horizontal coordinates at the GLL nodes come from a Gordon-Hall
(transfinite) map of the element's corners and (straight or circular) edges.

Per-point factors use collocated GLL quadrature:
    J = dX/dxi (D applied to the nodal coordinates),
    G = w_q det(J) J^{-1} J^{-T},   wdetJ = w_q det(J),
so that a[phi; nu] = sum_e sum_q grad_ref(nu)^T G grad_ref(phi).

Array conventions: elements are ordered e = column * nz + layer; local nodes
are (k, j, i) with i (xi) fastest; 2D slices drop j.  Reference-derivative
index order is (xi, eta, zeta) in 3D and (xi, zeta) in 2D.
"""

from __future__ import annotations

import numpy as np

from .gll import gll


def ref_axes(dim: int):
    """Array axes of (xi, [eta,] zeta) in a per-element nodal array [e, k, (j,) i, ...]."""
    return (3, 2, 1) if dim == 3 else (2, 1)


def dref(U, D, axis):
    """Apply the GLL derivative matrix along one array axis: sum_m D[a, m] U[.., m, ..]."""
    out = np.tensordot(D, U, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def _edge_points(a, b, arc, t):
    """Points of an element edge from corner a to corner b at parameters t in [-1, 1]."""
    s = (t + 1.0) / 2.0
    if arc is None or arc[2] == 0.0:
        return a[None, :] * (1.0 - s)[:, None] + b[None, :] * s[:, None]
    c = arc[:2]
    r = arc[2]
    ta = np.arctan2(a[1] - c[1], a[0] - c[0])
    tb = np.arctan2(b[1] - c[1], b[0] - c[0])
    d = tb - ta
    d = (d + np.pi) % (2 * np.pi) - np.pi
    th = ta + d * s
    return np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], -1)


def horizontal_coords(mesh):
    """Physical horizontal coordinates at the element GLL nodes: [n_eh, nh, dim-1]."""
    x, _, _ = gll(mesh.p)
    n1 = mesh.p + 1
    if mesh.dim == 2:
        xa = mesh.eh_corner[:, 0, 0][:, None]
        xb = mesh.eh_corner[:, 1, 0][:, None]
        return (xa + (xb - xa) * (x[None, :] + 1.0) / 2.0)[:, :, None]
    out = np.zeros((mesh.n_eh, n1 * n1, 2))
    XI = np.tile(x, n1)      # i fastest
    ET = np.repeat(x, n1)
    for e in range(mesh.n_eh):
        c = mesh.eh_corner[e]
        arcs = mesh.eh_arc[e] if mesh.eh_arc is not None else [None] * 4
        E0 = _edge_points(c[0], c[1], arcs[0], x)   # eta = -1, along xi
        E1 = _edge_points(c[1], c[2], arcs[1], x)   # xi = +1, along eta
        E2 = _edge_points(c[3], c[2], arcs[2], x)   # eta = +1, along xi
        E3 = _edge_points(c[0], c[3], arcs[3], x)   # xi = -1, along eta
        i = np.tile(np.arange(n1), n1)
        j = np.repeat(np.arange(n1), n1)
        xi, et = XI[:, None], ET[:, None]
        P = (0.5 * (1 - et) * E0[i] + 0.5 * (1 + et) * E2[i] + 0.5 * (1 - xi) * E3[j] + 0.5 * (1 + xi) * E1[j]
             - 0.25 * ((1 - xi) * (1 - et) * c[0] + (1 + xi) * (1 - et) * c[1]
                       + (1 + xi) * (1 + et) * c[2] + (1 - xi) * (1 + et) * c[3]))
        out[e] = P
    return out


def check_numbering(mesh, xh=None, tol=1e-10):
    """Every global horizontal node id must map to one physical point (mod periods)."""
    if xh is None:
        xh = horizontal_coords(mesh)
    ids = mesh.eh_nodes.ravel()
    pts = xh.reshape(-1, xh.shape[-1]).copy()
    for a, L in enumerate(mesh.period[: xh.shape[-1]]):
        if L:
            pts[:, a] = np.mod(pts[:, a], L)
            pts[:, a] = np.where(np.abs(pts[:, a] - L) < tol, 0.0, pts[:, a])
    ref = np.full((mesh.n_s, xh.shape[-1]), np.nan)
    ref[ids] = pts
    err = np.abs(ref[ids] - pts).max()
    if not np.isfinite(ref).all():
        raise ValueError("horizontal numbering leaves unused node ids")
    if err > tol:
        raise ValueError(f"horizontal numbering is geometrically inconsistent (max mismatch {err:g})")
    return ref


def node_coords(mesh):
    """Horizontal coordinates per global horizontal node: [n_s, dim-1] (periodic: first image)."""
    xh = horizontal_coords(mesh)
    out = np.full((mesh.n_s, mesh.dim - 1), np.nan)
    ids = mesh.eh_nodes.ravel()
    pts = xh.reshape(-1, mesh.dim - 1)
    # write in reverse so the first occurrence wins
    out[ids[::-1]] = pts[::-1]
    return out


def node_xy(mesh):
    """(x, y) arrays at the global horizontal nodes (y = 0 for slices)."""
    c = node_coords(mesh)
    if mesh.dim == 2:
        return c[:, 0], np.zeros(mesh.n_s)
    return c[:, 0], c[:, 1]


def sigma_levels(mesh):
    """Column fraction sigma_v in [0, 1] of every vertical node level v = 0 .. p*nz."""
    x, _, _ = gll(mesh.p)
    s = mesh.layer_fractions()
    sig = np.zeros(mesh.n_lev)
    for l in range(mesh.nz):
        for k in range(mesh.p + 1):
            sig[l * mesh.p + k] = s[l] + (s[l + 1] - s[l]) * (x[k] + 1.0) / 2.0
    return sig


def dof_map(mesh, cols=None):
    """Global volume index (layer-major: v * n_s + hn) of every element node: [n_e, n1^dim]."""
    p, n1, nz = mesh.p, mesh.p + 1, mesh.nz
    nodes = mesh.eh_nodes if cols is None else mesh.eh_nodes[np.asarray(cols)]
    n_eh = nodes.shape[0]
    k = np.arange(n1)
    nh = n1 * n1 if mesh.dim == 3 else n1
    hn = nodes.reshape(n_eh, 1, 1, nh).astype(np.int64)
    lev = (np.arange(nz)[None, :, None, None] * p + k[None, None, :, None])
    idx = lev * mesh.n_s + hn
    return idx.reshape(n_eh * nz, n1 * nh)


def element_coords(mesh, eta, h, xh=None, cols=None):
    """Nodal physical coordinates [n_e, n1, (n1,) n1, dim] for surface eta and depth h.

    ``cols`` restricts the result to the elements of the given columns (in that
    order, layers inside each column); ``xh`` must then be the full array.
    """
    if xh is None:
        xh = horizontal_coords(mesh)
    nodes = mesh.eh_nodes
    if cols is not None:
        cols = np.asarray(cols)
        xh = xh[cols]
        nodes = nodes[cols]
    p, n1, nz = mesh.p, mesh.p + 1, mesh.nz
    n_eh = nodes.shape[0]
    sig = sigma_levels(mesh)
    dt = np.result_type(eta, h, np.float64)
    eta_e = np.asarray(eta)[nodes]   # [n_eh, nh]
    h_e = np.asarray(h)[nodes]
    lev = (np.arange(nz)[:, None] * p + np.arange(n1)[None, :])   # [nz, n1]
    s = sig[lev]                                                  # [nz, n1]
    z = -h_e[:, None, None, :] + s[None, :, :, None] * (eta_e + h_e)[:, None, None, :]   # [n_eh, nz, k, nh]
    if mesh.dim == 3:
        X = np.zeros((n_eh, nz, n1, n1, n1, 3), dtype=dt)
        X[..., 0] = xh[:, None, None, :, 0].reshape(n_eh, 1, 1, n1, n1)
        X[..., 1] = xh[:, None, None, :, 1].reshape(n_eh, 1, 1, n1, n1)
        X[..., 2] = z.reshape(n_eh, nz, n1, n1, n1)
        return X.reshape(n_eh * nz, n1, n1, n1, 3)
    X = np.zeros((n_eh, nz, n1, n1, 2), dtype=dt)
    X[..., 0] = xh[:, None, None, :, 0]
    X[..., 1] = z
    return X.reshape(n_eh * nz, n1, n1, 2)


def jacobian(mesh, X):
    """J[..., a, b] = d X_a / d xi_b at every element node."""
    _, _, D = gll(mesh.p)
    cols = [dref(X, D, ax) for ax in ref_axes(mesh.dim)]
    return np.stack(cols, axis=-1)


def quad_weights(mesh):
    """Tensor GLL weights per element node, shaped like the nodal arrays [n1, (n1,) n1]."""
    _, w, _ = gll(mesh.p)
    if mesh.dim == 3:
        return w[:, None, None] * w[None, :, None] * w[None, None, :]
    return w[:, None] * w[None, :]


def factors(mesh, eta, h, xh=None, cols=None):
    """Return (G, wdetJ, J) with G[e, nodes..., a, b] = w det(J) (J^-1 J^-T)_ab."""
    X = element_coords(mesh, eta, h, xh, cols)
    J = jacobian(mesh, X)
    det = np.linalg.det(J)
    if np.any(np.real(det) <= 0.0):
        raise ValueError("non-positive Jacobian determinant (eta + h <= 0 or tangled mesh)")
    Ji = np.linalg.inv(J)
    wq = quad_weights(mesh)[None, ...]
    G = (wq * det)[..., None, None] * np.einsum("...ac,...bc->...ab", Ji, Ji)
    return G, wq * det, J
