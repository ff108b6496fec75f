"""Pins for the Laplace solve (Eq. 1) and w recovery: manufactured harmonic potentials."""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import operator as op
from oracle import solve as sv
from oracle import surface as sf
from workloads import mesh as wm


def _nodal(m, eta, h):
    X = geo.element_coords(m, eta, h)
    Xn = np.zeros((m.n_v, m.dim))
    Xn[geo.dof_map(m).ravel()] = X.reshape(-1, m.dim)
    return Xn


def _solve_manufactured_2d(p, nx=4, nz=2, k=math.pi, amp=0.1):
    m = wm.structured_slice(nx, 0.0, 2.0, True, p=p, nz=nz)
    x, _ = geo.node_xy(m)
    eta = amp * np.cos(k * x)
    h = np.ones(m.n_s)
    Xn = _nodal(m, eta, h)
    ex = np.cosh(k * (Xn[:, 1] + 1.0)) * np.cos(k * Xn[:, 0])     # harmonic, d/dz = 0 at z = -1
    G, _, _ = geo.factors(m, eta, h)
    phi = sv.solve_dense(m, op.assemble_dense(m, G), ex[sv.surface_slice(m)])
    return np.abs(phi - ex).max()


def test_p_convergence_2d():
    errs = [_solve_manufactured_2d(p) for p in range(2, 10)]
    assert errs[-1] < 1e-7
    # spectral: monotone decay, every two degrees gain more than a decade, > 5 decades overall
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))
    assert all(e2 < e0 / 10 for e0, e2 in zip(errs, errs[2:]))
    assert errs[0] / errs[-1] > 1e5


def test_p_convergence_3d_sloped_bottom():
    """e^{kz} cos(kx x) cos(ky y) with Neumann data grad(phi).n on a non-flat bottom."""
    errs = []
    for p in (2, 3, 4, 5, 6):
        m = wm.structured_box(3, 3, 0.0, 2.0, 0.0, 2.0, True, True, p=p, nz=1)
        x, y = geo.node_xy(m)
        kx = ky = math.pi
        kk = math.hypot(kx, ky)
        eta = 0.05 * np.cos(kx * x) * np.sin(ky * y)
        h = 0.5 + 0.05 * np.sin(kx * x)
        Xn = _nodal(m, eta, h)
        e = np.exp(kk * Xn[:, 2])
        ex = e * np.cos(kx * Xn[:, 0]) * np.cos(ky * Xn[:, 1])
        q = np.stack([-kx * e * np.sin(kx * Xn[:, 0]) * np.cos(ky * Xn[:, 1]),
                      -ky * e * np.cos(kx * Xn[:, 0]) * np.sin(ky * Xn[:, 1]),
                      kk * ex])
        G, _, _ = geo.factors(m, eta, h)
        f = op.neumann_load(m, eta, h, q)
        phi = sv.solve_dense(m, op.assemble_dense(m, G), ex[sv.surface_slice(m)], f)
        errs.append(np.abs(phi - ex).max())
    assert all(e1 < e0 / 2.5 for e0, e1 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-4


def test_dtn_spectral():
    """Flat bottom, phi_s = cos(kx): recovered w -> k tanh(kh) cos(kx) spectrally in p."""
    k = math.pi
    errs = []
    for p in range(2, 11):
        m = wm.structured_slice(8, 0.0, 2.0, True, p=p, nz=4)
        x, _ = geo.node_xy(m)
        eta, h = np.zeros(m.n_s), np.ones(m.n_s)
        G, _, _ = geo.factors(m, eta, h)
        phi = sv.solve_dense(m, op.assemble_dense(m, G), np.cos(k * x))
        w = sf.w_surface(m, phi, eta, h)
        errs.append(np.abs(w - k * math.tanh(k) * np.cos(k * x)).max())
    assert errs[-1] < 1e-11
    assert all(e1 < e0 / 3 for e0, e1 in zip(errs, errs[1:]))


def test_cg_matches_dense():
    m = wm.structured_box(3, 3, 0.0, 1.5, 0.0, 1.5, True, False, p=3, nz=2)
    x, y = geo.node_xy(m)
    eta = 0.1 * np.cos(2 * x) * np.cos(y)
    h = 1 + 0.1 * np.sin(x + y)
    phis = np.sin(3 * x) + 0.2 * y
    G, _, _ = geo.factors(m, eta, h)
    ref = sv.solve_dense(m, op.assemble_dense(m, G), phis)
    cg, info = sv.solve_cg(m, G, phis, rtol=1e-14, return_info=True)
    assert np.abs(cg - ref).max() < 1e-11 * np.abs(ref).max()
    assert info["iters"] > 5


def test_cg_max_iter_error():
    m = wm.structured_slice(3, 0.0, 1.5, True, p=3, nz=2)
    x, _ = geo.node_xy(m)
    G, _, _ = geo.factors(m, np.zeros(m.n_s), np.ones(m.n_s))
    with pytest.raises(RuntimeError):
        sv.solve_cg(m, G, np.cos(2 * x), rtol=1e-14, max_iter=1)


def test_w_exact_for_linear_fields_on_curved_mesh():
    m = wm.structured_box(3, 2, 0.0, 1.5, 0.0, 1.0, True, False, p=4, nz=2)
    x, y = geo.node_xy(m)
    eta, h = 0.1 * np.cos(2 * x + y), 1 + 0.2 * np.sin(3 * x) * np.cos(y)
    Xn = _nodal(m, eta, h)
    phi = 0.3 + 0.7 * Xn[:, 0] + 0.4 * Xn[:, 1] - 1.3 * Xn[:, 2]
    w = sf.w_surface(m, phi, eta, h)
    np.testing.assert_allclose(w, -1.3, atol=1e-12)
    m2 = wm.structured_slice(4, 0.0, 2.0, False, p=5, nz=3)
    x, _ = geo.node_xy(m2)
    eta, h = 0.1 * np.cos(2 * x), 1 + 0.2 * np.sin(x)
    Xn = _nodal(m2, eta, h)
    w = sf.w_surface(m2, 2.0 * Xn[:, 1] - 0.5 * Xn[:, 0], eta, h)
    np.testing.assert_allclose(w, 2.0, atol=1e-12)


def _line_case(dim, p, nz, seed=3):
    rng = np.random.default_rng(seed)
    if dim == 2:
        m = wm.structured_slice(4, 0.0, 2.0, True, p=p, nz=nz)
    else:
        m = wm.structured_box(3, 2, 0.0, 1.5, 0.0, 1.0, True, False, p=p, nz=nz)
    x, y = geo.node_xy(m)
    eta = 0.05 * np.cos(2.0 * x) + 0.02 * rng.standard_normal(m.n_s)
    h = 1.0 + 0.1 * np.sin(x + 0.3 * y)
    G, _, _ = geo.factors(m, eta, h)
    return m, op.assemble_dense(m, G)


@pytest.mark.parametrize("dim,p,nz", [(2, 3, 2), (2, 5, 3), (3, 2, 3), (3, 4, 2)])
def test_line_blocks_structure(dim, p, nz):
    """Each vertical line block is SPD and coupled only within element layers (half bandwidth p,
    nothing between levels of different layers); the blocks' traces add up to tr(A_II)."""
    m, A = _line_case(dim, p, nz)
    B = sv.line_blocks(m, A)
    nl = p * nz
    assert B.shape == (m.n_s, nl, nl)
    lev = np.arange(nl)
    same_layer = np.zeros((nl, nl), dtype=bool)       # both levels in one element layer
    for l in range(nz):
        inl = (lev >= l * p) & (lev <= l * p + p)
        same_layer |= inl[:, None] & inl[None, :]
    for b in B:
        np.testing.assert_allclose(b, b.T, atol=1e-14 * np.abs(b).max())
        assert np.linalg.eigvalsh(b).min() > 0.0
        assert np.all(b[~same_layer] == 0.0)
    I = sv.interior_mask(m)
    assert abs(np.trace(B, axis1=1, axis2=2).sum() - np.trace(A[np.ix_(I, I)])) < 1e-12 * np.trace(A)


@pytest.mark.parametrize("dim,p,nz", [(2, 4, 2), (3, 3, 2)])
def test_line_solve_recovers_a_single_line(dim, p, nz):
    """For x supported on the unknowns of one vertical line, (A x) on that line is B_n x_n, so the
    line solve returns x there exactly (up to rounding), whatever the couplings to other lines."""
    m, A = _line_case(dim, p, nz, seed=5)
    B = sv.line_blocks(m, A)
    idx = sv.line_unknowns(m)
    rng = np.random.default_rng(9)
    for n in (0, m.n_s // 2, m.n_s - 1):
        x = np.zeros(m.n_v)
        x[idx[n]] = rng.standard_normal(idx.shape[1])
        z = sv.line_solve(m, B, A @ x)
        np.testing.assert_allclose(z[idx[n]], x[idx[n]], rtol=0, atol=1e-11 * np.abs(x).max())
        assert np.all(z[sv.surface_slice(m)] == 0.0)


def test_line_block_closed_form_p1_flat_column():
    """p = 1, one flat walled column of half widths a, d and layer half thickness c: the line
    block is tridiagonal with off-diagonal -a d / (2 c) per layer (the zeta-zeta term
    sum_c D[c][0] D[c][1] w det J / c^2 with D = [[-1/2, 1/2], [-1/2, 1/2]], unit weights; the
    cross terms vanish on flat geometry)."""
    lx, ly, nz = 0.8, 0.5, 4
    m = wm.structured_box(1, 1, 0.0, lx, 0.0, ly, False, False, p=1, nz=nz)
    eta = np.zeros(m.n_s)
    h = np.full(m.n_s, 2.0)
    G, _, _ = geo.factors(m, eta, h)
    B = sv.line_blocks(m, op.assemble_dense(m, G))
    a, d, c = lx / 2, ly / 2, 2.0 / nz / 2
    for b in B:
        np.testing.assert_allclose(np.diag(b, 1), -a * d / (2 * c), rtol=1e-13)
        assert np.all(np.triu(b, 2) == 0.0)
