"""Pins for the geometry (Sec. 3.1.2) and the Laplace operator (Eq. 4) of the oracle."""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import operator as op
from oracle import solve as sv
from workloads import configs, mesh as wm


def _wavy(mesh, seed=0, amp=0.3):
    x, y = geo.node_xy(mesh)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, 4)
    eta = amp * 0.5 * np.cos(a[0] * x + 0.3) * np.cos(a[1] * y)
    h = 1.0 + amp * 0.3 * np.sin(a[2] * x) * np.cos(a[3] * y + 0.2)
    return eta, h


def _small_meshes():
    return [
        wm.structured_slice(3, 0.0, 1.5, True, p=4, nz=2),
        wm.structured_slice(3, 0.0, 1.5, False, p=3, nz=2),
        wm.structured_box(3, 3, 0.0, 1.5, 0.0, 1.2, True, True, p=2, nz=2),
        wm.structured_box(3, 2, 0.0, 1.5, 0.0, 1.0, True, False, p=3, nz=2),
        wm.structured_box(2, 2, 0.0, 1.0, 0.0, 1.0, False, False, p=4, nz=1),
        wm.structured_box(2, 2, 0.0, 1.0, 0.0, 1.0, False, False, p=5, nz=1),
    ]


def test_flat_affine_G_closed_form():
    nx, ny, nz, p = 4, 3, 2, 3
    lx, ly, h0 = 2.0, 1.5, 0.8
    m = wm.structured_box(nx, ny, 0.0, lx, 0.0, ly, True, False, p=p, nz=nz)
    G, wdet, _ = geo.factors(m, np.zeros(m.n_s), np.full(m.n_s, h0))
    a, b, c = lx / nx / 2, ly / ny / 2, h0 / nz / 2
    wq = geo.quad_weights(m)
    np.testing.assert_allclose(G[..., 0, 0], np.broadcast_to(wq * b * c / a, G.shape[:-2]), rtol=1e-13)
    np.testing.assert_allclose(G[..., 1, 1], np.broadcast_to(wq * a * c / b, G.shape[:-2]), rtol=1e-13)
    np.testing.assert_allclose(G[..., 2, 2], np.broadcast_to(wq * a * b / c, G.shape[:-2]), rtol=1e-13)
    off = np.abs(G[..., 0, 1]).max() + np.abs(G[..., 0, 2]).max() + np.abs(G[..., 1, 2]).max()
    assert off < 1e-14
    assert abs(wdet.sum() - lx * ly * h0) < 1e-12


@pytest.mark.parametrize("mi", range(6))
def test_volume_equals_gll_column_integral(mi):
    m = _small_meshes()[mi]
    eta, h = _wavy(m, mi)
    _, wdet, _ = geo.factors(m, eta, h)
    from oracle.surface import surface_mass
    assert abs(wdet.sum() - surface_mass(m) @ (eta + h)) < 1e-12 * wdet.sum()


def test_cylinder_area():
    m = configs.c3().mesh
    _, wdet, _ = geo.factors(m, np.zeros(m.n_s), np.ones(m.n_s))
    area = 10.0 * 5.0 - math.pi * 0.25 ** 2
    assert abs(wdet.sum() - area) < 1e-7


def test_geometry_errors():
    m = wm.structured_slice(3, 0.0, 1.5, True, p=2, nz=1)
    h = np.ones(m.n_s)
    eta = np.zeros(m.n_s)
    eta[1] = -1.1
    with pytest.raises(ValueError):
        geo.factors(m, eta, h)


@pytest.mark.parametrize("mi", range(6))
def test_dense_equals_matrix_free(mi):
    m = _small_meshes()[mi]
    eta, h = _wavy(m, mi)
    G, _, _ = geo.factors(m, eta, h)
    A = op.assemble_dense(m, G)
    Amf = np.stack([op.apply(m, G, e) for e in np.eye(m.n_v)], axis=1)
    assert np.linalg.norm(A - Amf) <= 1e-13 * np.linalg.norm(A)
    # symmetric, annihilates constants, positive semidefinite; A_II is SPD
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(A @ np.ones(m.n_v)).max() <= 1e-13 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > -1e-12 * ev.max()
    I = sv.interior_mask(m)
    assert np.linalg.eigvalsh(A[np.ix_(I, I)]).min() > 1e-8 * ev.max()
    np.testing.assert_allclose(op.diagonal(m, G), np.diag(A), rtol=1e-13, atol=1e-14 * np.abs(A).max())


def _nodal_coords(m, eta, h):
    X = geo.element_coords(m, eta, h)
    Xn = np.zeros((m.n_v, m.dim))
    Xn[geo.dof_map(m).ravel()] = X.reshape(-1, m.dim)
    return Xn


def _patch(m, eta, h, fn, grad):
    Xn = _nodal_coords(m, eta, h)
    G, _, _ = geo.factors(m, eta, h)
    f = op.neumann_load(m, eta, h, grad(Xn))
    A = op.assemble_dense(m, G)
    ex = fn(Xn)
    phi = sv.solve_dense(m, A, ex[sv.surface_slice(m)], f)
    return np.abs(phi - ex).max()


def test_patch_quadratic_affine():
    m2 = wm.structured_slice(3, 0.0, 1.5, False, p=3, nz=2)
    z2 = (np.zeros(m2.n_s), np.ones(m2.n_s))
    assert _patch(m2, *z2, lambda X: X[:, 0] ** 2 - X[:, 1] ** 2, lambda X: np.stack([2 * X[:, 0], -2 * X[:, 1]])) < 1e-12
    assert _patch(m2, *z2, lambda X: X[:, 0] * X[:, 1], lambda X: np.stack([X[:, 1], X[:, 0]])) < 1e-12
    m3 = wm.structured_box(3, 2, 0.0, 1.5, 0.0, 1.0, False, False, p=2, nz=2)
    z3 = (np.zeros(m3.n_s), np.ones(m3.n_s))
    assert _patch(m3, *z3, lambda X: X[:, 0] ** 2 + X[:, 1] ** 2 - 2 * X[:, 2] ** 2,
                  lambda X: np.stack([2 * X[:, 0], 2 * X[:, 1], -4 * X[:, 2]])) < 1e-12
    assert _patch(m3, *z3, lambda X: X[:, 1] * X[:, 2], lambda X: np.stack([0 * X[:, 0], X[:, 2], X[:, 1]])) < 1e-12


def test_patch_linear_curvilinear():
    m2 = wm.structured_slice(3, 0.0, 1.5, False, p=4, nz=2)
    x, _ = geo.node_xy(m2)
    eta, h = 0.1 * np.cos(2 * x), 1 + 0.2 * np.sin(3 * x)
    c = (0.7, -1.3)
    assert _patch(m2, eta, h, lambda X: 0.3 + c[0] * X[:, 0] + c[1] * X[:, 1],
                  lambda X: np.stack([np.full(len(X), c[0]), np.full(len(X), c[1])])) < 1e-12
    m3 = wm.structured_box(3, 2, 0.0, 1.5, 0.0, 1.0, False, False, p=3, nz=2)
    x, y = geo.node_xy(m3)
    eta, h = 0.1 * np.cos(2 * x + y), 1 + 0.2 * np.sin(3 * x) * np.cos(y)
    c = (0.7, 0.4, -1.3)
    assert _patch(m3, eta, h, lambda X: 0.3 + X @ np.array(c),
                  lambda X: np.stack([np.full(len(X), ci) for ci in c])) < 1e-12


def test_patch_linear_cylinder_small():
    """Curved (arc) horizontal elements: exact with a flat surface; with a wavy surface the
    doubly curved map breaks the discrete metric identities of collocated GLL quadrature,
    so the linear field is reproduced only to quadrature accuracy, converging spectrally."""
    c = (0.7, 0.4, -1.3)
    fn = lambda X: 0.3 + X @ np.array(c)
    grad = lambda X: np.stack([np.full(len(X), ci) for ci in c])
    errs = []
    for p in (2, 3, 4, 5, 6):
        m = wm.cylinder_tank_mesh(p=p, nz=1, n_theta=8, n_rad=2, tank=(6.0, 4.0), spacing=1.0, hole_half=1.0)
        x, y = geo.node_xy(m)
        assert _patch(m, np.zeros(m.n_s), np.ones(m.n_s), fn, grad) < 1e-12
        errs.append(_patch(m, 0.05 * np.cos(x) * np.sin(y), 1.0 + 0.1 * np.cos(0.5 * x), fn, grad))
    assert all(e1 < e0 / 5 for e0, e1 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6


def test_column_subset_apply_and_diagonal():
    """The element-subset mode of apply and diagonal (G and dofs for some columns only, as the
    sampled full-size checks use it): at the nodes of a column whose neighbours are all in the
    subset, both equal the whole-mesh result; elsewhere they hold only the subset's share."""
    m = wm.structured_box(5, 4, 0.0, 2.0, 0.0, 1.6, True, False, p=3, nz=2)
    eta, h = _wavy(m, seed=3)
    xh = geo.horizontal_coords(m)
    Gf, _, _ = geo.factors(m, eta, h, xh)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(m.n_v)
    yf = op.apply(m, Gf, x)
    df = op.diagonal(m, Gf)
    nx, ny = 5, 4
    cx, cy = 2, 1
    nb = sorted({((cx + dx) % nx) + (cy + dy) * nx for dx in (-1, 0, 1) for dy in (-1, 0, 1)})
    G, _, _ = geo.factors(m, eta, h, xh, cols=nb)
    dofs = geo.dof_map(m, cols=nb)
    own = geo.dof_map(m, cols=[cx + cy * nx]).ravel()
    y = op.apply(m, G, x, dofs)
    d = op.diagonal(m, G, dofs)
    np.testing.assert_allclose(y[own], yf[own], rtol=0, atol=1e-13 * np.abs(yf).max())
    np.testing.assert_allclose(d[own], df[own], rtol=1e-13)
    # a node outside the subset's closure gets nothing, a corner of the subset only part of its sum
    outside = np.setdiff1d(np.arange(m.n_v), dofs.ravel())
    assert outside.size > 0 and np.all(d[outside] == 0.0)
    others = geo.dof_map(m, cols=[c for c in range(m.n_eh) if c not in nb]).ravel()
    rim = np.intersect1d(dofs.ravel(), others)   # nodes the subset shares with other columns
    assert rim.size > 0 and np.all(d[rim] < df[rim])
