"""Pins for the oracle's modal filter (Sec. 3.2, modal filtering), checked against numpy's own
Legendre series routines and exact polynomial invariance; no GPU."""

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import filter as mf
from oracle import geometry as geo
from oracle import gll as og
from oracle import timestep as ts
from workloads import configs, mesh as wm


def _expected_sigma(p, cutoff, alpha, order):
    # the exponential filter evaluated directly at each mode index
    return np.array([1.0 if n <= cutoff else np.exp(-alpha * ((n - cutoff) / (p - cutoff)) ** order)
                     for n in range(p + 1)])


def test_sigma_special_values():
    s = mf.sigma(6, 3, 2.5, 4)
    assert np.all(s[:4] == 1.0)
    assert s[6] == pytest.approx(np.exp(-2.5), rel=1e-15)          # top mode: exp(-alpha)
    assert np.all(np.diff(s[3:]) < 0)                             # strictly damped above the cutoff
    np.testing.assert_allclose(s, _expected_sigma(6, 3, 2.5, 4), rtol=1e-15)


@pytest.mark.parametrize("p,cutoff,alpha,order", [(4, 2, 1.0, 2), (6, 3, 36.0, 8), (7, 0, 0.5, 1)])
def test_single_interval_equals_legendre_series(p, cutoff, alpha, order):
    """One wall-bounded interval: every node belongs to one element, so the filter is exactly
    the Legendre series with coefficients scaled by sigma (numpy's series evaluation)."""
    m = wm.structured_slice(1, 0.0, 3.0, False, p=p, nz=1)
    x, _ = geo.node_xy(m)
    xi = 2.0 * x / 3.0 - 1.0
    a = np.random.default_rng(p).standard_normal(p + 1)
    f = npleg.legval(xi, a)
    got = mf.modal_filter(m, f, cutoff, alpha, order)
    want = npleg.legval(xi, a * _expected_sigma(p, cutoff, alpha, order))
    np.testing.assert_allclose(got, want, atol=1e-13 * np.abs(a).sum())


@pytest.mark.parametrize("p,cutoff", [(3, 1), (5, 3)])
def test_single_quad_equals_tensor_legendre_series(p, cutoff):
    m = wm.structured_box(1, 1, 0.0, 2.0, 0.0, 1.5, False, False, p=p, nz=1)
    x, y = geo.node_xy(m)
    xi, et = x - 1.0, 2.0 * y / 1.5 - 1.0
    c = np.random.default_rng(11).standard_normal((p + 1, p + 1))   # c[m, n]: P_m(xi) P_n(eta)
    f = npleg.legval2d(xi, et, c)
    s = _expected_sigma(p, cutoff, 3.0, 2)
    got = mf.modal_filter(m, f, cutoff, 3.0, 2)
    want = npleg.legval2d(xi, et, c * s[:, None] * s[None, :])
    np.testing.assert_allclose(got, want, atol=1e-13 * np.abs(c).sum())


def test_two_intervals_shared_node_is_the_average():
    """Two wall-bounded intervals: nodal filter matrices built from numpy's Legendre
    Vandermonde; the shared node takes the mean of the two element results."""
    p, cutoff, alpha, order = 4, 1, 2.0, 2
    m = wm.structured_slice(2, 0.0, 2.0, False, p=p, nz=1)
    xg, _, _ = og.gll(p)
    L = npleg.legvander(xg, p)
    M = L @ np.diag(_expected_sigma(p, cutoff, alpha, order)) @ np.linalg.inv(L)
    f = np.random.default_rng(3).standard_normal(m.n_s)
    got = mf.modal_filter(m, f, cutoff, alpha, order)
    acc = np.zeros(m.n_s)
    cnt = np.zeros(m.n_s)
    for e in range(2):
        nodes = m.eh_nodes[e]
        acc[nodes] += M @ f[nodes]
        cnt[nodes] += 1
    np.testing.assert_allclose(got, acc / cnt, atol=1e-14)
    assert cnt.max() == 2 and cnt[m.eh_nodes[0][-1]] == 2


@pytest.mark.parametrize("kind", ["slice", "box_walls", "box_periodic_x"])
def test_low_degree_polynomials_unchanged(kind):
    """Each element's filter reproduces polynomials of degree <= cutoff, so the averaged
    global filter leaves continuous fields of that degree unchanged (affine meshes)."""
    p, cutoff = 5, 2
    if kind == "slice":
        m = wm.structured_slice(4, 0.0, 4.0, False, p=p, nz=1)
    elif kind == "box_walls":
        m = wm.structured_box(3, 2, 0.0, 3.0, 0.0, 2.0, False, False, p=p, nz=1)
    else:
        m = wm.structured_box(3, 2, 0.0, 3.0, 0.0, 2.0, True, False, p=p, nz=1)
    x, y = geo.node_xy(m)
    if kind == "box_periodic_x":
        f = 0.3 + 0.2 * y - 0.7 * y ** 2            # periodic in x: y-polynomial only
    else:
        f = 0.3 - 1.1 * x + 0.4 * x * x + (0.2 * y - 0.5 * x * y ** 2 if m.dim == 3 else 0.0)
    got = mf.modal_filter(m, f, cutoff, 20.0, 2)
    np.testing.assert_allclose(got, f, atol=1e-12)
    # a mode above the cutoff is damped
    g = np.cos(3.0 * np.pi * x)
    assert np.linalg.norm(mf.modal_filter(m, g, cutoff, 20.0, 2) - g) > 1e-3


def test_identity_limits_and_linearity():
    wl = configs.small_box(nx=4, ny=3, nz=1, p=4, periodic=(True, False))
    m = wl.mesh
    rng = np.random.default_rng(2)
    f, g = rng.standard_normal(m.n_s), rng.standard_normal(m.n_s)
    np.testing.assert_allclose(mf.modal_filter(m, f, 2, 0.0, 4), f, atol=1e-13)
    a = mf.modal_filter(m, 2.0 * f - 3.0 * g, 1, 5.0, 2)
    b = 2.0 * mf.modal_filter(m, f, 1, 5.0, 2) - 3.0 * mf.modal_filter(m, g, 1, 5.0, 2)
    np.testing.assert_allclose(a, b, atol=1e-12)
    with pytest.raises(ValueError):
        mf.modal_filter(m, f, 4, 1.0, 2)


def test_filtered_step_is_step_then_filter():
    """The filtered ERK4 step is the plain step followed by the filter of eta and phi_s; with
    alpha = 0 the filtered model reproduces the plain one."""
    wl = configs.small_slice(nx=5, nz=2, p=4, periodic=True)
    md = ts.Model(wl, solver="dense")
    eta, phi = md.initial_state()
    e0, p0 = md.rk4_step(eta, phi, 0.0, 0.02)
    mf_ = ts.Model(wl, solver="dense", modal_filter=(2, 4.0, 2))
    e1, p1 = mf_.rk4_step(eta, phi, 0.0, 0.02)
    np.testing.assert_allclose(e1, mf.modal_filter(wl.mesh, e0, 2, 4.0, 2), atol=1e-14)
    np.testing.assert_allclose(p1, mf.modal_filter(wl.mesh, p0, 2, 4.0, 2), atol=1e-14)
    m0 = ts.Model(wl, solver="dense", modal_filter=(2, 0.0, 2))
    e2, p2 = m0.rk4_step(eta, phi, 0.0, 0.02)
    np.testing.assert_allclose(e2, e0, atol=1e-14)
    np.testing.assert_allclose(p2, p0, atol=1e-14)
