"""Pins for the oracle's consistent, over-integrated free-surface RHS (Eq. 5 with the
over-integration of Sec. 3.2): numpy Legendre-series arithmetic on single elements (the exact
L2 projection), exactness for integrands inside the discrete space on multi-element meshes,
the surface area, and convergence to the pointwise Eqs. 2-3; no GPU."""

import numpy as np
import pytest
from numpy.polynomial import legendre as L

from oracle import geometry as geo
from oracle import surface as sf
from oracle import timestep as ts
from workloads import configs, mesh as wm

G = 9.81


def _nq_exact(p):
    # the degree of the integrand times the test function is at most 5p - 2
    return (5 * p - 1) // 2 + 1


def _trunc(c, p):
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros(p + 1)
    out[: min(len(c), p + 1)] = c[: p + 1]
    return out


@pytest.mark.parametrize("p", [2, 4, 6])
def test_single_interval_is_the_legendre_projection(p):
    """One wall-bounded interval [0, Lx]: d/dx = (2/Lx) d/dxi; the consistent RHS is the
    truncated Legendre series of the integrand (numpy series products)."""
    Lx = 1.7
    m = wm.structured_slice(1, 0.0, Lx, False, p=p, nz=1)
    x, _ = geo.node_xy(m)
    xi = 2.0 * x / Lx - 1.0
    rng = np.random.default_rng(p)
    ce, cp, cw = (0.3 * rng.standard_normal(p + 1) for _ in range(3))
    s = 2.0 / Lx
    ex = s * L.legder(ce)
    px = s * L.legder(cp)
    one_ee = L.legadd([1.0], L.legmul(ex, ex))
    Ek = L.legadd(-L.legmul(ex, px), L.legmul(cw, one_ee))
    Ed = L.legadd(L.legadd(-G * ce, -0.5 * L.legmul(px, px)), 0.5 * L.legmul(L.legmul(cw, cw), one_ee))
    ke, kd = sf.free_surface_rhs_consistent(m, L.legval(xi, ce), L.legval(xi, cp), L.legval(xi, cw), G,
                                            _nq_exact(p))
    np.testing.assert_allclose(ke, L.legval(xi, _trunc(Ek, p)), atol=1e-12)
    np.testing.assert_allclose(kd, L.legval(xi, _trunc(Ed, p)), atol=1e-11)


def _sep_eval(terms, p, xi, et):
    """Evaluate the projection onto Q_p of sum_t f_t(xi) g_t(eta) (Legendre series)."""
    C = np.zeros((p + 1, p + 1))
    for f, g in terms:
        C += np.outer(_trunc(f, p), _trunc(g, p))
    return L.legval2d(xi, et, C)


def test_single_quad_separable_fields_projection():
    """One quad [0, Lx] x [0, Ly]; eta = a(xi) b(eta), phi = c(xi) d(eta), w = e(xi) f(eta):
    every term of the integrands is separable and its projection onto Q_p is the product of the
    1D truncated series."""
    p, Lx, Ly = 3, 2.0, 1.5
    m = wm.structured_box(1, 1, 0.0, Lx, 0.0, Ly, False, False, p=p, nz=1)
    x, y = geo.node_xy(m)
    xi, et = 2.0 * x / Lx - 1.0, 2.0 * y / Ly - 1.0
    rng = np.random.default_rng(8)
    a, b, c, d, e, f = (0.4 * rng.standard_normal(p + 1) for _ in range(6))
    sx, sy = 2.0 / Lx, 2.0 / Ly
    da, db, dc, dd = (L.legder(v) for v in (a, b, c, d))
    mul = L.legmul
    # |grad eta|^2 = sx^2 a'^2 b^2 + sy^2 a^2 b'^2 ; grad eta . grad phi = sx^2 a'c' bd + sy^2 ac b'd'
    gee = [(sx * sx * mul(da, da), mul(b, b)), (sy * sy * mul(a, a), mul(db, db))]
    gep = [(sx * sx * mul(da, dc), mul(b, d)), (sy * sy * mul(a, c), mul(db, dd))]
    gpp = [(sx * sx * mul(dc, dc), mul(d, d)), (sy * sy * mul(c, c), mul(dd, dd))]
    Ek = [(-u, v) for u, v in gep] + [(e, f)] + [(mul(e, u), mul(f, v)) for u, v in gee]
    ww = (mul(e, e), mul(f, f))
    Ed = ([(-G * a, b)] + [(-0.5 * u, v) for u, v in gpp] + [(0.5 * ww[0], ww[1])]
          + [(0.5 * mul(ww[0], u), mul(ww[1], v)) for u, v in gee])
    ke, kd = sf.free_surface_rhs_consistent(
        m, L.legval(xi, a) * L.legval(et, b), L.legval(xi, c) * L.legval(et, d),
        L.legval(xi, e) * L.legval(et, f), G, _nq_exact(p))
    np.testing.assert_allclose(ke, _sep_eval(Ek, p, xi, et), atol=1e-12)
    np.testing.assert_allclose(kd, _sep_eval(Ed, p, xi, et), atol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_integrand_in_the_space_is_reproduced(dim):
    """Multi-element walled meshes: eta quadratic in x, phi linear in x, w linear in y make both
    integrands polynomials of degree <= 2 per direction, so for p >= 2 the projection returns
    the pointwise Eqs. 2-3 exactly (nonlinear terms included)."""
    p = 3
    if dim == 2:
        m = wm.structured_slice(4, 0.0, 3.0, False, p=p, nz=1)
    else:
        m = wm.structured_box(3, 2, 0.0, 3.0, 0.0, 2.0, False, False, p=p, nz=1)
    x, y = geo.node_xy(m)
    y = y if dim == 3 else np.zeros_like(x)
    eta = 0.05 + 0.1 * x - 0.03 * x * x
    phi = 0.2 - 0.4 * x
    w = 0.3 + 0.2 * y          # (y = 0 on the slice)
    ex = 0.1 - 0.06 * x
    px = -0.4
    Ek = -ex * px + w * (1.0 + ex * ex)
    Ed = -G * eta - 0.5 * px * px + 0.5 * w * w * (1.0 + ex * ex)
    ke, kd = sf.free_surface_rhs_consistent(m, eta, phi, w, G, 8)
    np.testing.assert_allclose(ke, Ek, atol=1e-12)
    np.testing.assert_allclose(kd, Ed, atol=1e-11)


def test_mass_totals_area():
    m = wm.structured_box(4, 3, 0.0, 2.0, 0.0, 1.5, True, False, p=4, nz=1)
    assert abs(sf.consistent_surface_mass(m, 6).sum() - 3.0) < 1e-12
    mc = wm.cylinder_tank_mesh(p=4, nz=1, n_theta=8, n_rad=2, tank=(6.0, 4.0), spacing=1.0, hole_half=1.0)
    xh = geo.horizontal_coords(mc)
    _, wdet_c, _, _ = sf.surface_quadrature(mc, 8, xh)
    _, ms = sf.surface_metrics(mc, xh)
    # the Gauss and the GLL rules integrate the same isoparametric area (to quadrature error)
    assert abs(wdet_c.sum() - ms.sum()) < 1e-6 * ms.sum()
    M = sf.consistent_surface_mass(mc, 8, xh)
    assert abs(M.sum() - wdet_c.sum()) < 1e-10 * wdet_c.sum()
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > 0.0


def test_converges_to_pointwise_equations():
    """Smooth periodic fields: the consistent RHS converges spectrally to Eqs. 2-3 at the nodes."""
    k = np.pi
    errs = []
    for p in (3, 5, 7):
        m = wm.structured_box(3, 3, 0.0, 2.0, 0.0, 2.0, True, True, p=p, nz=1)
        x, y = geo.node_xy(m)
        eta = 0.1 * np.sin(k * x) * np.cos(k * y)
        phi = 0.2 * np.cos(k * x + 0.3) * np.cos(k * y)
        w = 0.3 * np.sin(k * y + 0.1)
        ex, ey = 0.1 * k * np.cos(k * x) * np.cos(k * y), -0.1 * k * np.sin(k * x) * np.sin(k * y)
        px, py = -0.2 * k * np.sin(k * x + 0.3) * np.cos(k * y), -0.2 * k * np.cos(k * x + 0.3) * np.sin(k * y)
        ee = ex * ex + ey * ey
        Ek = -(ex * px + ey * py) + w * (1 + ee)
        Ed = -G * eta - 0.5 * (px * px + py * py) + 0.5 * w * w * (1 + ee)
        ke, kd = sf.free_surface_rhs_consistent(m, eta, phi, w, G, _nq_exact(p))
        errs.append(max(np.abs(ke - Ek).max(), np.abs(kd - Ed).max()))
    assert errs[1] < 0.1 * errs[0] and errs[2] < 0.1 * errs[1] and errs[2] < 1e-4


def test_model_with_consistent_rhs_reduces_to_linear_limit():
    """One step of the consistent model matches the lumped model to O(amplitude^2)."""
    wl = configs.small_slice(nx=5, nz=2, p=4, periodic=True)
    mc = ts.Model(wl, solver="dense", surface_quadrature=8)
    ml = ts.Model(wl, solver="dense")
    x, _ = geo.node_xy(wl.mesh)
    diffs = []
    for amp in (1e-2, 1e-3):
        eta = amp * np.cos(np.pi * x)
        phi = amp * np.sin(np.pi * x)
        e1, _ = mc.rk4_step(eta, phi, 0.0, 0.01)
        e2, _ = ml.rk4_step(eta, phi, 0.0, 0.01)
        diffs.append(np.abs(e1 - e2).max() / amp)
    # the linear terms (w, -g eta) lie in the space, so both forms share them exactly: the
    # difference is quadratic in the amplitude (relative difference linear in it)
    assert diffs[0] < 1e-4 and diffs[1] < 0.15 * diffs[0]
