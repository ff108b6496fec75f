"""Pins for the free-surface RHS (Eqs. 2-3), ERK4 (Sec. 3.2), relaxation (Sec. 3.3) and diagnostics."""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import operator as op
from oracle import solve as sv
from oracle import surface as sf
from oracle import timestep as ts
from workloads import configs, mesh as wm, waves


def _rk4_amp(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def test_rhs_degenerate_cases():
    m = wm.structured_box(3, 3, 0.0, 2.0, 0.0, 2.0, True, True, p=4, nz=1)
    x, y = geo.node_xy(m)
    eta = 0.1 * np.sin(np.pi * x) * np.cos(np.pi * y)
    w = 0.3 * np.cos(np.pi * x + 0.2)
    z = np.zeros(m.n_s)
    de, dp = sf.free_surface_rhs(m, z, z, w, 9.81)
    np.testing.assert_allclose(de, w, atol=1e-14)
    np.testing.assert_allclose(dp, 0.5 * w * w, atol=1e-14)
    de, dp = sf.free_surface_rhs(m, eta, z, z, 9.81)
    np.testing.assert_allclose(de, 0.0, atol=1e-14)
    np.testing.assert_allclose(dp, -9.81 * eta, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_rhs_pointwise_closed_form(dim):
    """Smooth prescribed eta, phi_s, w: the lumped RHS converges to Eqs. 2-3 pointwise."""
    k = np.pi
    errs = []
    for p in (3, 5, 7, 9):
        if dim == 3:
            m = wm.structured_box(3, 3, 0.0, 2.0, 0.0, 2.0, True, True, p=p, nz=1)
        else:
            m = wm.structured_slice(3, 0.0, 2.0, True, p=p, nz=1)
        x, y = geo.node_xy(m)
        eta = 0.2 * np.sin(k * x) * np.cos(k * y)
        ex = 0.2 * k * np.cos(k * x) * np.cos(k * y)
        ey = -0.2 * k * np.sin(k * x) * np.sin(k * y)
        ph = 0.5 * np.cos(k * (x + y))
        px = py = -0.5 * k * np.sin(k * (x + y))
        if dim == 2:
            ey = py = 0.0 * x
            eta = 0.2 * np.sin(k * x)
            ex = 0.2 * k * np.cos(k * x)
            ph = 0.5 * np.cos(k * x)
            px = -0.5 * k * np.sin(k * x)
        w = 0.4 * np.cos(k * x + 0.3)
        g = 9.81
        ee = ex * ex + ey * ey
        Ek = -(ex * px + ey * py) + w * (1 + ee)
        Ed = -g * eta - 0.5 * (px * px + py * py) + 0.5 * w * w * (1 + ee)
        de, dp = sf.free_surface_rhs(m, eta, ph, w, g)
        errs.append(max(np.abs(de - Ek).max(), np.abs(dp - Ed).max()))
    assert errs[-1] < 1e-6
    assert all(e1 < e0 / 5 for e0, e1 in zip(errs, errs[1:]))


def test_rk4_combination_linear_ode():
    """With the stage replaced by a linear ODE y' = L y, one step equals R(L dt) y exactly."""
    wl = configs.c1()
    md = ts.Model(wl, solver="dense")
    lam_e, lam_p = -0.7, 0.4

    def fake(eta, phi_s, h=None, phi_guess=None):
        return lam_e * eta, lam_p * phi_s, np.zeros(wl.mesh.n_v), None

    md.stage = fake
    eta0 = np.linspace(0.5, 1.5, wl.mesh.n_s)
    phi0 = np.linspace(-1.0, 2.0, wl.mesh.n_s)
    dt = 0.3
    e1, p1 = md.rk4_step(eta0, phi0, 0.0, dt)
    np.testing.assert_allclose(e1, _rk4_amp(lam_e * dt) * eta0, rtol=1e-15)
    np.testing.assert_allclose(p1, _rk4_amp(lam_p * dt) * phi0, rtol=1e-15)


def test_relaxation_limits():
    wl = configs.c4(nx=8, ny=2, nz=1, p=2, nsteps=1)
    md = ts.Model(wl, solver="dense")
    cr, ec, es, pc, ps = md.relax
    eta = np.random.default_rng(0).standard_normal(wl.mesh.n_s)
    phi = np.random.default_rng(1).standard_normal(wl.mesh.n_s)
    t = 1.234
    e1, p1 = md.relax_apply(eta, phi, t)
    zero = cr == 0.0
    np.testing.assert_array_equal(e1[zero], eta[zero])
    one = cr >= 1.0 - 1e-15
    assert one.any() and zero.any()
    r = ts.ramp(t, wl.t_ramp)
    om = wl.relax_wave.omega
    x = md.x
    gen = x < 8.0 * 38.0 / 38.0
    target = np.where(gen, r * wl.relax_wave.eta(x, md.y, t), 0.0)
    np.testing.assert_allclose(e1[one], target[one], atol=1e-15)
    np.testing.assert_allclose(p1[one], np.where(gen, r * wl.relax_wave.phi(x, md.y, t), 0.0)[one], atol=1e-15)
    assert ts.ramp(0.0, 5.0) == 0.0 and ts.ramp(5.0, 5.0) == 1.0 and abs(ts.ramp(2.5, 5.0) - 0.5) < 1e-15


def _dtn_eigenvalue(wl):
    m = wl.mesh
    x, _ = geo.node_xy(m)
    k = wl.meta["k"]
    h = np.ones(m.n_s)
    G, _, _ = geo.factors(m, np.zeros(m.n_s), h)
    phi = sv.solve_dense(m, op.assemble_dense(m, G), np.cos(k * x))
    w = sf.w_surface(m, phi, np.zeros(m.n_s), h)
    # nodal cos(kx) is an eigenvector of the discrete DtN map only up to the non-uniform
    # GLL spacing (a few 1e-6 here); its Rayleigh quotient in the surface mass is the mode's
    # eigenvalue to second order in that defect
    ms = sf.surface_mass(m)
    c = np.cos(k * x)
    lam = (ms @ (c * w)) / (ms @ (c * c))
    assert np.abs(w - lam * c).max() < 1e-4 * lam
    return float(lam)


def test_c1_standing_wave_dispersion_and_energy():
    """C1: 32 ERK4 steps of a linear standing wave against the RK4/dispersion closed forms."""
    wl = configs.c1()
    md = ts.Model(wl, solver="dense")
    k, g, dt = wl.meta["k"], wl.g, wl.dt
    lam = _dtn_eigenvalue(wl)
    assert abs(lam / (k * math.tanh(k)) - 1) < 3e-3          # discretisation error of C1's DtN
    omega_h = math.sqrt(g * lam)
    R = _rk4_amp(1j * omega_h * dt)
    omega_rk = np.angle(R) / dt
    basis = np.cos(k * md.x)
    series = []

    def cb(n, t, eta, phi_s):
        series.append((t, (md.ms @ (eta * basis)) / (md.ms @ (basis * basis)), eta.copy(), phi_s.copy()))

    eta0, phi0 = md.initial_state()
    E0 = md.energy(eta0, phi0)
    M0 = md.mass(eta0)
    md.run(callback=cb)
    t = np.array([s[0] for s in series])
    zc = np.array([s[1] for s in series])
    # least-squares fit a cos(omega t): grid search + Newton-free refinement by scipy
    from scipy.optimize import least_squares
    fit = least_squares(lambda q: q[0] * np.cos(q[1] * t) - zc, [1e-3, omega_h], xtol=1e-15, ftol=1e-15)
    omega_fit = fit.x[1]
    assert abs(omega_fit - omega_rk) / omega_rk < 2e-5
    assert abs(omega_fit / wl.meta["omega"] - 1) < 2e-3
    # amplitude and energy decay follow |R(i theta)|^n
    assert abs(fit.x[0] / 1e-3 - 1) < 2e-5
    E1 = md.energy(series[-1][2], series[-1][3])
    assert abs(E1 / E0 - abs(R) ** 64) < 5e-6
    # mass: the initial mode has zero mean; drift stays at rounding level
    assert abs(md.mass(series[-1][2]) - M0) < 1e-12


def test_complex_step_matches_central_differences():
    """Complex-step directional derivative of a gauge loss vs central FD (small bar case)."""
    wl = configs.c4(nx=8, ny=2, nz=1, p=2, nsteps=3)
    md = ts.Model(wl, solver="dense")
    x = md.x
    P = ts.gauge_matrix(wl.mesh, [[10.0, 0.5], [21.0, 0.25]])
    eta0 = 0.01 * np.cos(2 * np.pi * x / 38.0 * 4)
    phi0 = 0.02 * np.sin(2 * np.pi * x / 38.0 * 4)
    h = md.h
    dt = 0.05
    obs = np.zeros((3, 2)) + 0.001
    rng = np.random.default_rng(3)
    dh = rng.standard_normal(wl.mesh.n_s) * 0.01
    de = rng.standard_normal(wl.mesh.n_s) * 0.001
    d_cs = ts.complex_step_derivative(md, P, obs, 3, dt, eta0, phi0, h, de, dh)
    eps = 1e-4
    Jp = ts.gauge_loss(md, P, obs, 3, dt, eta0 + eps * de, phi0, h + eps * dh)
    Jm = ts.gauge_loss(md, P, obs, 3, dt, eta0 - eps * de, phi0, h - eps * dh)
    d_fd = (Jp - Jm) / (2 * eps)
    assert abs(d_cs - d_fd) < 1e-7 * abs(d_fd) + 1e-18


def _dtn_matrix(md):
    """Discrete LPF Dirichlet-to-Neumann map S (w = S phi_s on the flat domain), column by column."""
    n = md.mesh.n_s
    flat = np.zeros(n)
    S = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        _, _, _, w = md.stage(flat, e)
        S[:, k] = w
    return S


def test_lpf_exact_eigenmode_follows_rk4_closed_form():
    """LPF on C1: started from an eigenvector v of the discrete DtN map (S v = lam v), the
    semi-discrete system is the 2x2 oscillator (eta, phi_s)' = [[0, lam], [-g, 0]] (eta, phi_s) on
    span(v), so N ERK4 steps equal the N-th power of the RK4 polynomial of dt times that matrix."""
    wl = configs.c1()
    md = ts.Model(wl, solver="dense", linear=True)
    S = _dtn_matrix(md)
    vals, vecs = np.linalg.eig(S)
    k = wl.meta["k"]
    target = k * math.tanh(k * wl.meta["h"])
    i = int(np.argmin(np.abs(vals - target)))
    lam, v = float(vals[i].real), np.real(vecs[:, i])
    assert abs(vals[i].imag) < 1e-10 * abs(lam)
    assert np.linalg.norm(S @ v - lam * v) < 1e-10 * np.linalg.norm(lam * v)
    assert abs(lam / target - 1) < 3e-3                      # spatial error of C1's DtN map
    g, dt, N = wl.g, wl.dt, 16
    L = dt * np.array([[0.0, lam], [-g, 0.0]])
    Pm = np.eye(2) + L + L @ L / 2 + L @ L @ L / 6 + L @ L @ L @ L / 24
    y = np.linalg.matrix_power(Pm, N) @ np.array([1e-3, 0.0])
    eta, phi = 1e-3 * v, np.zeros_like(v)
    t = 0.0
    for n in range(N):
        eta, phi = md.rk4_step(eta, phi, t, dt)
        t += dt
    assert np.linalg.norm(eta - y[0] * v) < 1e-11 * 1e-3 * np.linalg.norm(v)
    assert np.linalg.norm(phi - y[1] * v) < 1e-11 * abs(y[1]) * np.linalg.norm(v) + 1e-18


def test_lpf_linear_and_small_amplitude_limit():
    """LPF is linear (superposition to rounding); FNPF minus LPF shrinks quadratically with the
    amplitude (the neglected terms are products of two perturbation fields)."""
    wl = configs.small_box(nx=4, ny=3, nz=2, p=3, periodic=(True, False))
    lin = ts.Model(wl, solver="dense", linear=True)
    fnpf = ts.Model(wl, solver="dense")
    rng = np.random.default_rng(9)
    x = lin.x
    e1 = np.cos(2 * np.pi * x / 2.0)
    p1 = 0.3 * np.sin(2 * np.pi * x / 2.0)
    e2, p2 = 0.2 * rng.standard_normal(lin.mesh.n_s), 0.1 * rng.standard_normal(lin.mesh.n_s)

    def run(model, e, p, n=3, dt=0.02):
        t = 0.0
        for _ in range(n):
            e, p = model.rk4_step(e, p, t, dt)
            t += dt
        return e, p

    a = run(lin, e1, p1)
    b = run(lin, e2, p2)
    c = run(lin, 2.0 * e1 + e2, 2.0 * p1 + p2)
    assert np.abs(c[0] - (2 * a[0] + b[0])).max() < 1e-12 * np.abs(c[0]).max()
    assert np.abs(c[1] - (2 * a[1] + b[1])).max() < 1e-12 * np.abs(c[1]).max()
    diffs = []
    for amp in (1e-3, 2e-3):
        fl = run(lin, amp * e1, amp * p1)
        fn = run(fnpf, amp * e1, amp * p1)
        diffs.append(np.linalg.norm(fn[0] - fl[0]))
    assert 3.6 < diffs[1] / diffs[0] < 4.4


@pytest.mark.parametrize("dim,p", [(2, 3), (2, 5), (3, 2), (3, 4)])
def test_gauge_matrix_reproduces_polynomials(dim, p):
    """(P f)_g = f(point_g) for every field of degree <= p per direction (the element space on
    axis-aligned elements), at interior points, on element edges, at element corners and on the
    domain boundary; a transposed reference coordinate, a wrong node order or a wrong map to the
    reference element fails it because the x and y degrees differ."""
    rng = np.random.default_rng(11)
    if dim == 2:
        m = wm.structured_slice(4, 0.5, 3.7, False, p=p, nz=1)
        xs = np.concatenate([rng.uniform(0.5, 3.7, 6), [0.5, 3.7, 0.5 + 3.2 / 4, 0.5 + 2 * 3.2 / 4]])
        pts = xs[:, None]
        coef = rng.standard_normal(p + 1)

        def f(x, y):
            return sum(coef[a] * x ** a for a in range(p + 1))
    else:
        m = wm.structured_box(3, 2, -1.0, 2.0, 0.5, 1.7, False, False, p=p, nz=1)
        ex, ey = np.linspace(-1.0, 2.0, 4), np.linspace(0.5, 1.7, 3)
        pts = np.array([[rng.uniform(-1, 2), rng.uniform(0.5, 1.7)] for _ in range(6)]
                       + [[ex[1], rng.uniform(0.5, 1.7)], [rng.uniform(-1, 2), ey[1]],   # element edges
                          [ex[1], ey[1]], [ex[2], ey[1]],                                  # interior vertices
                          [-1.0, 0.5], [2.0, 1.7], [-1.0, rng.uniform(0.5, 1.7)]])         # boundary
        coef = rng.standard_normal((p + 1, p))

        def f(x, y):
            return sum(coef[a, b] * x ** a * y ** b for a in range(p + 1) for b in range(p))
    x, y = geo.node_xy(m)
    P = ts.gauge_matrix(m, pts)
    want = np.array([f(pt[0], pt[1] if dim == 3 else 0.0) for pt in pts])
    np.testing.assert_allclose(P @ f(x, y), want, rtol=0, atol=1e-11 * np.abs(want).max())
    # each row is a partition of unity over the nodes of one element
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-13)
    with pytest.raises(ValueError):
        ts.gauge_matrix(m, [[10.0] + ([0.0] if dim == 3 else [])])
