"""GPU parity of the consistent, over-integrated free-surface form (Eq. 5 with the
over-integration of Sec. 3.2) against the oracle: the RHS alone, the Chebyshev interval
claim, ERK4 steps, and the adjoints (complex step of the oracle).

Tolerances: the RHS at 1e-12 relative L2 (the Chebyshev length is set for a 1e-15 contraction;
quadrature sums of a few hundred terms); steps at the FP64 path's 1e-10 and the mixed path's
1e-8; adjoint identities at 1e-9.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import geometry as geo
from oracle import surface as sf
from oracle import timestep as ts
from paper_2506_09435_amd import fnpf
from workloads import configs, mesh as wm

EPS = 1e-30


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _mesh(name):
    if name == "slice_periodic":
        return wm.structured_slice(5, 0.0, 2.0, True, p=4, nz=2)
    if name == "slice_walls":
        return wm.structured_slice(4, 0.0, 2.0, False, p=5, nz=2)
    if name == "box_periodic":
        return wm.structured_box(4, 3, 0.0, 2.0, 0.0, 1.5, True, True, p=3, nz=2)
    if name == "box_mixed":
        return wm.structured_box(5, 3, 0.0, 2.0, 0.0, 1.5, True, False, p=4, nz=2)
    if name == "box_walls_p6":
        return wm.structured_box(3, 2, 0.0, 2.0, 0.0, 1.5, False, False, p=6, nz=2)
    if name == "cylinder":
        return wm.cylinder_tank_mesh(p=3, nz=2, n_theta=8, n_rad=2, tank=(6.0, 4.0), spacing=1.0, hole_half=1.0)
    if name == "cylinder_blocked":
        return wm.renumber_blocked(_mesh("cylinder"))
    raise KeyError(name)


MESHES = ["slice_periodic", "slice_walls", "box_periodic", "box_mixed", "box_walls_p6", "cylinder",
          "cylinder_blocked"]


def _fields(m, seed=3):
    x, y = geo.node_xy(m)
    rng = np.random.default_rng(seed)
    eta = 0.05 * np.cos(1.3 * x + 0.2) * np.cos(0.9 * y) + 0.002 * rng.standard_normal(m.n_s)
    phi = 0.1 * np.sin(1.1 * x + 0.7 * y) + 0.002 * rng.standard_normal(m.n_s)
    w = 0.2 * np.cos(0.8 * x - 0.4 * y) + 0.002 * rng.standard_normal(m.n_s)
    return eta, phi, w


@pytest.mark.parametrize("name", MESHES)
def test_consistent_rhs_parity_and_interval(name):
    m = _mesh(name)
    ctx = fnpf.Context(m, g=9.81)
    eta, phi, w = _fields(m)
    for nq in (m.p + 1, (5 * m.p - 1) // 2 + 1):
        ctx.set_surface_quadrature(nq)
        ke, kd = sf.free_surface_rhs_consistent(m, eta, phi, w, 9.81, nq)
        ge, gd = ctx.rhs(dev(eta), dev(phi), dev(w))
        assert rel(host(ge), ke) < 1e-12 and rel(host(gd), kd) < 1e-12
        info = ctx.surface_quadrature_info()
        assert info["nq"] == nq and 0 < info["iters"] <= 200
        # the Chebyshev interval contains the spectrum of M_L^{-1} M (oracle matrices)
        M = sf.consistent_surface_mass(m, nq)
        ml = sf.surface_mass(m)
        lam = np.linalg.eigvalsh(M / np.sqrt(ml)[:, None] / np.sqrt(ml)[None, :])
        assert info["lam_lo"] <= lam.min() * (1 + 1e-12) and lam.max() <= info["lam_hi"] * (1 + 1e-12)
    # back to the lumped form
    ctx.set_surface_quadrature(0)
    le, ld = sf.free_surface_rhs(m, eta, phi, w, 9.81)
    ge, gd = ctx.rhs(dev(eta), dev(phi), dev(w))
    assert rel(host(ge), le) < 1e-13 and rel(host(gd), ld) < 1e-13


def test_surface_quadrature_errors():
    m = _mesh("box_mixed")
    ctx = fnpf.Context(m, g=9.81)
    for nq in (m.p, 25, -1):
        with pytest.raises(fnpf.FnpfError) as ei:
            ctx.set_surface_quadrature(nq)
        assert ei.value.name == "ERR_ARG"
    assert ctx.surface_quadrature_info()["nq"] == 0


@pytest.mark.parametrize("name", ["slice", "box", "cylinder", "bar"])
@pytest.mark.parametrize("precision", [0, 1])
def test_consistent_rk4_steps_parity(name, precision):
    if name == "slice":
        wl = configs.small_slice(nx=5, nz=2, p=4, periodic=True)
    elif name == "box":
        wl = configs.small_box(nx=4, ny=3, nz=2, p=4, periodic=(True, False))
    elif name == "cylinder":
        wl = configs.small_box()
        wl.mesh = _mesh("cylinder")
        wl.depth = lambda x, y: 1.0 + 0.1 * np.cos(0.5 * np.asarray(x)) * np.sin(np.asarray(y))
        wl.eta0 = lambda x, y: 0.05 * np.cos(np.asarray(x)) * np.sin(np.asarray(y))
        wl.phi0 = lambda x, y: 0.1 * np.sin(np.asarray(x) + 0.3 * np.asarray(y))
    else:
        wl = configs.c4(nx=8, ny=2, nz=2, p=3, nsteps=3)
    nq = wl.mesh.p + 3
    md = ts.Model(wl, solver="dense", surface_quadrature=nq)
    x, y = geo.node_xy(wl.mesh)
    h = np.asarray(wl.depth(x, y), dtype=np.float64)
    rng = np.random.default_rng(4)
    eta = np.asarray(wl.eta0(x, y), dtype=np.float64) + 0.002 * rng.standard_normal(wl.mesh.n_s)
    phi = np.asarray(wl.phi0(x, y), dtype=np.float64)
    ctx = fnpf.Context(wl.mesh, g=wl.g)
    ra = wl.relaxation_arrays(x, y)
    if ra is not None:
        ctx.set_relaxation(*ra, omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    ctx.set_surface_quadrature(nq)
    e, p, dh = dev(eta), dev(phi), dev(h)
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-12, inner_rtol=1e-3)
    t = 0.1
    for n in range(3):
        eta, phi = md.rk4_step(eta, phi, t, 0.02)
        ctx.rk4_step(e, p, dh, t, 0.02, opts=opts)
        t += 0.02
    tol = 1e-10 if precision == 0 else 1e-8
    assert rel(host(e), eta) < tol and rel(host(p), phi) < tol


@pytest.mark.parametrize("name", ["slice_periodic", "box_mixed", "cylinder"])
def test_consistent_rhs_vjp(name):
    m = _mesh(name)
    ctx = fnpf.Context(m, g=9.81)
    nq = m.p + 2
    ctx.set_surface_quadrature(nq)
    eta, phi, w = _fields(m, seed=9)
    rng = np.random.default_rng(2)
    ve, vp, vw = (0.1 * rng.standard_normal(m.n_s) for _ in range(3))
    kbe, kbp = rng.standard_normal(m.n_s), rng.standard_normal(m.n_s)
    ke, kd = sf.free_surface_rhs_consistent(m, eta + 1j * EPS * ve, phi + 1j * EPS * vp, w + 1j * EPS * vw, 9.81,
                                            nq)
    lhs = kbe @ (ke.imag / EPS) + kbp @ (kd.imag / EPS)
    eb = dev(np.full(m.n_s, 0.5))
    pb, wb = torch.zeros_like(eb), torch.zeros_like(eb)
    ctx.rhs_vjp(dev(eta), dev(phi), dev(w), dev(kbe), dev(kbp), eb, pb, wb)
    rhs = (host(eb) - 0.5) @ ve + host(pb) @ vp + host(wb) @ vw
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("name", ["slice", "bar"])
def test_consistent_rk4_step_vjp(name):
    if name == "slice":
        wl = configs.small_slice(nx=5, nz=2, p=4, periodic=True)
    else:
        wl = configs.c4(nx=8, ny=2, nz=2, p=3, nsteps=1)
    m = wl.mesh
    nq = m.p + 2
    md = ts.Model(wl, solver="dense", surface_quadrature=nq)
    x, y = geo.node_xy(m)
    h = np.asarray(wl.depth(x, y), dtype=np.float64)
    rng = np.random.default_rng(19)
    eta = 0.01 * np.cos(2 * np.pi * x / 2.0) + 0.002 * rng.standard_normal(m.n_s)
    phis = 0.02 * np.sin(2 * np.pi * x / 2.0)
    ctx = fnpf.Context(m, g=wl.g)
    ra = wl.relaxation_arrays(x, y)
    if ra is not None:
        ctx.set_relaxation(*ra, omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    ctx.set_surface_quadrature(nq)
    t, dt = 0.37, 0.03
    ve, vp, vh = (rng.standard_normal(m.n_s) * s for s in (0.01, 0.1, 0.01))
    ybe, ybp = rng.standard_normal(m.n_s), rng.standard_normal(m.n_s)
    e1, p1 = md.rk4_step(eta + 1j * EPS * ve, phis + 1j * EPS * vp, t, dt, h=h + 1j * EPS * vh)
    lhs = ybe @ (e1.imag / EPS) + ybp @ (p1.imag / EPS)
    e, p = dev(eta), dev(phis)
    tape = ctx.new_tape()
    o = fnpf.default_opts(rtol=1e-13, check_every=10)
    ctx.rk4_step(e, p, dev(h), t, dt, opts=o, tape=tape)
    assert np.abs(host(e) - e1.real).max() < 1e-10 * np.abs(e1.real).max()
    eb, pb = dev(ybe), dev(ybp)
    hb = torch.zeros(m.n_s, dtype=torch.float64, device="cuda")
    ctx.rk4_step_vjp(dev(h), t, dt, tape, eb, pb, hb, opts=o)
    rhs = host(eb) @ ve + host(pb) @ vp + host(hb) @ vh
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
