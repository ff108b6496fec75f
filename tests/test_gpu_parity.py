"""GPU parity of every step of the path against the FP64 oracle (same seeded inputs).

Tolerances: the FP64 path to 1e-10 relative L2 (single kernels to ~1e-13), the mixed
FP32/FP64 path to 1e-8, as required of the two paths; FP32 applies alone are compared at
the FP32 rounding level.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import geometry as geo
from oracle import operator as op
from oracle import solve as sv
from oracle import surface as sf
from oracle import timestep as ts
from paper_2506_09435_amd import fnpf
from workloads import configs, mesh as wm


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(name):
    if name == "slice_periodic":
        return configs.small_slice(nx=5, nz=3, p=4, periodic=True)
    if name == "slice_walls":
        return configs.small_slice(nx=4, nz=2, p=5, periodic=False)
    if name == "box_periodic":
        return configs.small_box(nx=4, ny=3, nz=2, p=3, periodic=(True, True))
    if name == "box_mixed":
        return configs.small_box(nx=5, ny=3, nz=3, p=4, periodic=(True, False))
    if name == "box_walls_p6":
        return configs.small_box(nx=3, ny=2, nz=2, p=6, periodic=(False, False))
    if name == "box_one_layer_p6":
        # one element layer (the surface level is the first layer's top), tiles of five columns
        # spanning two rows of seven, periodic in x
        return configs.small_box(nx=7, ny=2, nz=1, p=6, periodic=(True, False))
    if name == "slice_one_layer":
        return configs.small_slice(nx=6, nz=1, p=6, periodic=False)
    if name == "cylinder":
        wl = configs.small_box()
        m = wm.cylinder_tank_mesh(p=3, nz=2, n_theta=8, n_rad=2, tank=(6.0, 4.0), spacing=1.0, hole_half=1.0)
        wl.mesh = m
        wl.depth = lambda x, y: 1.0 + 0.1 * np.cos(0.5 * np.asarray(x)) * np.sin(np.asarray(y))
        wl.eta0 = lambda x, y: 0.05 * np.cos(np.asarray(x)) * np.sin(np.asarray(y))
        wl.phi0 = lambda x, y: 0.1 * np.sin(np.asarray(x) + 0.3 * np.asarray(y))
        return wl
    if name.endswith("_blocked"):
        wl = _case(name[: -len("_blocked")])
        wl.mesh = wm.renumber_blocked(wl.mesh)
        return wl
    if name.endswith("_sharedfirst"):
        wl = _case(name[: -len("_sharedfirst")])
        wl.mesh = wm.renumber_blocked(wl.mesh, shared_first=True)
        return wl
    raise KeyError(name)


CASES = ["slice_periodic", "slice_walls", "box_periodic", "box_mixed", "box_walls_p6", "cylinder",
         "box_mixed_blocked", "cylinder_blocked", "box_walls_p6_sharedfirst", "cylinder_sharedfirst",
         "box_one_layer_p6_sharedfirst", "slice_one_layer"]


class Pair:
    """The same workload on both sides: oracle arrays and a library context."""

    def __init__(self, wl, fp32=False, variant=0):
        self.wl = wl
        self.m = wl.mesh
        self.xh = geo.horizontal_coords(self.m)
        self.x, self.y = geo.node_xy(self.m)
        self.h = np.asarray(wl.depth(self.x, self.y), dtype=np.float64)
        self.eta = np.asarray(wl.eta0(self.x, self.y), dtype=np.float64)
        self.phis = np.asarray(wl.phi0(self.x, self.y), dtype=np.float64)
        self.ctx = fnpf.Context(self.m, g=wl.g)
        if variant:
            self.ctx.set_apply_variant(variant)
        if fp32:
            self.ctx.enable_fp32()
        self.d_h, self.d_eta, self.d_phis = dev(self.h), dev(self.eta), dev(self.phis)

    def oracle_factors(self):
        return geo.factors(self.m, self.eta, self.h, self.xh)


@pytest.mark.parametrize("name", CASES)
def test_node_coords(name):
    pr = Pair(_case(name))
    xy = pr.ctx.node_coords()
    ref = geo.node_coords(pr.m)
    assert np.abs(xy - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("name", CASES)
def test_geometry_parity(name, variant):
    pr = Pair(_case(name), fp32=True, variant=variant)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    G, diag = pr.ctx.export_geometry(fnpf.F64)
    G32, _ = pr.ctx.export_geometry(fnpf.F32)
    Go, _, _ = pr.oracle_factors()
    d = pr.m.dim
    comps = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)] if d == 3 else [(0, 0), (0, 1), (1, 1)]
    Gor = np.stack([Go[..., a, b].reshape(Go.shape[0], -1) for a, b in comps], axis=1)
    scale = np.abs(Gor).max()
    assert np.abs(host(G) - Gor).max() < 1e-13 * scale
    assert np.abs(host(G32) - Gor).max() < 1e-6 * scale
    dref = op.diagonal(pr.m, Go)
    assert np.abs(host(diag) - dref).max() < 1e-13 * np.abs(dref).max()


@pytest.mark.parametrize("variant", [0, 6, 7])
@pytest.mark.parametrize("name", ["slice_periodic", "box_periodic", "cylinder", "box_mixed_blocked"])
def test_apply_equals_dense_matrix(name, variant):
    pr = Pair(_case(name), variant=variant)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    Go, _, _ = pr.oracle_factors()
    A = op.assemble_dense(pr.m, Go)
    n = pr.m.n_v
    E = torch.eye(n, dtype=torch.float64, device="cuda")
    cols = [pr.ctx.laplace_apply(E[k].contiguous()) for k in range(n)]
    Ag = host(torch.stack(cols, dim=1))
    assert np.linalg.norm(Ag - A) <= 1e-13 * np.linalg.norm(A)
    assert np.abs(Ag @ np.ones(n)).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("variant", [0, 1, 6, 7])
@pytest.mark.parametrize("name", CASES)
def test_apply_random_fp64_fp32(name, variant):
    pr = Pair(_case(name), fp32=True, variant=variant)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    Go, _, _ = pr.oracle_factors()
    rng = np.random.default_rng(11)
    xv = rng.standard_normal(pr.m.n_v)
    yo = op.apply(pr.m, Go, xv)
    y = host(pr.ctx.laplace_apply(dev(xv)))
    assert rel(y, yo) < 1e-13
    ym = host(pr.ctx.laplace_apply(dev(xv), mask_dirichlet=True))
    top = sv.surface_slice(pr.m)
    assert np.all(ym[top] == 0.0)
    assert rel(ym[: top.start], yo[: top.start]) < 1e-13
    y32 = host(pr.ctx.laplace_apply(dev(xv).float()))
    assert rel(y32, yo) < 2e-6


@pytest.mark.parametrize("name", ["slice_walls", "box_walls_p6", "box_mixed", "cylinder"])
def test_neumann_load_parity(name):
    pr = Pair(_case(name))
    pr.ctx.geom(pr.d_eta, pr.d_h)
    X = geo.element_coords(pr.m, pr.eta, pr.h, pr.xh)
    Xn = np.zeros((pr.m.n_v, pr.m.dim))
    Xn[geo.dof_map(pr.m).ravel()] = X.reshape(-1, pr.m.dim)
    q = np.stack([np.sin(Xn[:, 0] + 0.3 * Xn[:, -1]) + 0.2 * a for a in range(pr.m.dim)])
    fo = op.neumann_load(pr.m, pr.eta, pr.h, q)
    f = host(pr.ctx.neumann_load(dev(q)))
    assert np.abs(f - fo).max() < 1e-13 * np.abs(fo).max()


@pytest.mark.parametrize("variant", [0, 6, 7])
@pytest.mark.parametrize("name", CASES)
def test_solve_w_rhs_parity(name, variant):
    pr = Pair(_case(name), fp32=True, variant=variant)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    Go, _, _ = pr.oracle_factors()
    A = op.assemble_dense(pr.m, Go)
    phio = sv.solve_dense(pr.m, A, pr.phis)
    phi, info = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-13, check_every=7))
    assert info["status"] == "OK" and info["rel_res"] <= 1e-13
    assert rel(host(phi), phio) < 1e-10
    # mixed FP32 inner / FP64 outer to a 1e-11 FP64 residual
    phim, infom = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(precision=1, rtol=1e-11, inner_rtol=1e-3))
    assert infom["status"] == "OK" and infom["outer_iters"] >= 2
    assert rel(host(phim), phio) < 1e-8
    # Steps 4.4-4.6 on the oracle's potential
    wo = sf.w_surface(pr.m, phio, pr.eta, pr.h, pr.xh)
    w = host(pr.ctx.w_surface(dev(phio)))
    assert rel(w, wo) < 1e-12
    deo, dpo = sf.free_surface_rhs(pr.m, pr.eta, pr.phis, wo, pr.wl.g, xh=pr.xh)
    de, dp = pr.ctx.rhs(pr.d_eta, pr.d_phis, dev(wo))
    assert rel(host(de), deo) < 1e-12 and rel(host(dp), dpo) < 1e-12


@pytest.mark.parametrize("name", ["slice_periodic", "box_mixed", "cylinder", "box_one_layer_p6_sharedfirst"])
@pytest.mark.parametrize("precision", [0, 1])
def test_rk4_step_parity(name, precision):
    wl = _case(name)
    pr = Pair(wl, fp32=precision == 1)
    md = ts.Model(wl, solver="dense")
    dt = 0.02
    e1, p1 = md.rk4_step(pr.eta, pr.phis, 0.0, dt)
    e, p = pr.d_eta.clone(), pr.d_phis.clone()
    tape = pr.ctx.new_tape()
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-12, inner_rtol=1e-3)
    infos = pr.ctx.rk4_step(e, p, pr.d_h, 0.0, dt, opts=opts, tape=tape)
    tol = 1e-10 if precision == 0 else 1e-8
    assert rel(host(e), e1) < tol and rel(host(p), p1) < tol
    assert all(i["rel_res"] <= opts.rtol for i in infos)
    # the first stage's potential is the oracle's solve at the initial state
    phi0 = sv.solve_dense(pr.m, op.assemble_dense(pr.m, pr.oracle_factors()[0]), pr.phis)
    assert rel(host(tape[: pr.m.n_v]), phi0) < tol


def test_rk4_relaxation_parity():
    wl = configs.c4(nx=8, ny=2, nz=2, p=3, nsteps=3)
    pr = Pair(wl)
    ra = wl.relaxation_arrays(pr.x, pr.y)
    pr.ctx.set_relaxation(*ra, omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    md = ts.Model(wl, solver="dense")
    rng = np.random.default_rng(5)
    eta = 0.01 * np.cos(2 * np.pi * pr.x / 9.5) + 0.001 * rng.standard_normal(pr.m.n_s)
    phi = 0.02 * np.sin(2 * np.pi * pr.x / 9.5)
    e, p = dev(eta), dev(phi)
    t = 0.3
    for n in range(3):
        eta, phi = md.rk4_step(eta, phi, t, wl.dt)
        pr.ctx.rk4_step(e, p, pr.d_h, t, wl.dt, opts=fnpf.default_opts(rtol=1e-13))
        t += wl.dt
    assert rel(host(e), eta) < 1e-10 and rel(host(p), phi) < 1e-10


@pytest.mark.parametrize("name", ["slice_periodic", "box_mixed", "cylinder"])
@pytest.mark.parametrize("precision", [0, 1])
def test_lpf_rk4_steps_parity(name, precision):
    """Linear potential flow: three ERK4 steps against the oracle's linear model."""
    wl = _case(name)
    pr = Pair(wl, fp32=precision == 1)
    pr.ctx.set_linear(True)
    md = ts.Model(wl, solver="dense", linear=True)
    dt = 0.02
    eta, phi = pr.eta, pr.phis
    e, p = pr.d_eta.clone(), pr.d_phis.clone()
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-12, inner_rtol=1e-3)
    t = 0.0
    for n in range(3):
        eta, phi = md.rk4_step(eta, phi, t, dt)
        infos = pr.ctx.rk4_step(e, p, pr.d_h, t, dt, opts=opts)
        assert all(i["rel_res"] <= opts.rtol for i in infos)
        t += dt
    tol = 1e-10 if precision == 0 else 1e-8
    assert rel(host(e), eta) < tol and rel(host(p), phi) < tol
    # the linear and the nonlinear models differ at this amplitude
    en, _ = ts.Model(wl, solver="dense").rk4_step(pr.eta, pr.phis, 0.0, dt)
    e1, _ = md.rk4_step(pr.eta, pr.phis, 0.0, dt)
    assert rel(e1, en) > 1e-6


def test_lpf_flat_geometry_cache():
    """The flat geometry is kept across linear steps and rebuilt when another call replaced the
    geometry or after fnpf_set_linear (here after an in-place change of the depth)."""
    wl = _case("box_mixed")
    pr = Pair(wl)
    pr.ctx.set_linear(True)
    md = ts.Model(wl, solver="dense", linear=True)
    dt = 0.02
    opts = fnpf.default_opts(rtol=1e-13)
    eta, phi = pr.eta, pr.phis
    e, p = pr.d_eta.clone(), pr.d_phis.clone()
    t = 0.0
    for n in range(2):
        eta, phi = md.rk4_step(eta, phi, t, dt)
        pr.ctx.rk4_step(e, p, pr.d_h, t, dt, opts=opts)
        t += dt
    assert rel(host(e), eta) < 1e-10
    # a geometry from another call in between: the next linear step rebuilds the flat one
    pr.ctx.geom(e, pr.d_h)
    eta, phi = md.rk4_step(eta, phi, t, dt)
    pr.ctx.rk4_step(e, p, pr.d_h, t, dt, opts=opts)
    t += dt
    assert rel(host(e), eta) < 1e-10 and rel(host(p), phi) < 1e-10
    # the depth changed in place (same array): fnpf_set_linear drops the cached geometry
    h2 = pr.h * 1.1
    pr.d_h.copy_(dev(h2))
    pr.ctx.set_linear(True)
    eta, phi = md.rk4_step(eta, phi, t, dt, h=h2)
    pr.ctx.rk4_step(e, p, pr.d_h, t, dt, opts=opts)
    assert rel(host(e), eta) < 1e-10 and rel(host(p), phi) < 1e-10


def test_lpf_rhs_and_relaxation_parity():
    """Linear RHS is (w, -g eta) pointwise; LPF steps with relaxation zones match the oracle."""
    wl = configs.c4(nx=8, ny=2, nz=2, p=3, nsteps=3)
    pr = Pair(wl)
    pr.ctx.set_linear(True)
    rng = np.random.default_rng(8)
    eta = 0.01 * np.cos(2 * np.pi * pr.x / 9.5) + 0.001 * rng.standard_normal(pr.m.n_s)
    phi = 0.02 * np.sin(2 * np.pi * pr.x / 9.5)
    w = rng.standard_normal(pr.m.n_s)
    de, dp = pr.ctx.rhs(dev(eta), dev(phi), dev(w))
    assert rel(host(de), w) < 1e-14 and rel(host(dp), -wl.g * eta) < 1e-14
    ra = wl.relaxation_arrays(pr.x, pr.y)
    pr.ctx.set_relaxation(*ra, omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    md = ts.Model(wl, solver="dense", linear=True)
    e, p = dev(eta), dev(phi)
    t = 0.3
    for n in range(3):
        eta, phi = md.rk4_step(eta, phi, t, wl.dt)
        pr.ctx.rk4_step(e, p, pr.d_h, t, wl.dt, opts=fnpf.default_opts(rtol=1e-13))
        t += wl.dt
    assert rel(host(e), eta) < 1e-10 and rel(host(p), phi) < 1e-10
    # switching back restores the nonlinear model
    pr.ctx.set_linear(False)
    md_nl = ts.Model(wl, solver="dense")
    e2, p2 = md_nl.rk4_step(eta, phi, t, wl.dt)
    pr.ctx.rk4_step(e, p, pr.d_h, t, wl.dt, opts=fnpf.default_opts(rtol=1e-13))
    assert rel(host(e), e2) < 1e-10 and rel(host(p), p2) < 1e-10


@pytest.mark.parametrize("precond", [1, 2])
def test_c1_full_run(precond):
    """C1: 32 ERK4 steps (one period) of the standing wave; FP64 path vs the oracle (solves at
    rtol 1e-13: 128 solves whose errors accumulate in the state)."""
    wl = configs.c1()
    pr = Pair(wl)
    md = ts.Model(wl, solver="dense")
    eo, po = md.run()
    e, p = pr.d_eta.clone(), pr.d_phis.clone()
    opts = fnpf.default_opts(rtol=1e-13, precond=precond)
    t = 0.0
    for n in range(wl.nsteps):
        pr.ctx.rk4_step(e, p, pr.d_h, t, wl.dt, opts=opts)
        t += wl.dt
    assert rel(host(e), eo) < 1e-10
    assert rel(host(p), po) < 1e-10


def test_c2_full_size_apply_and_solve():
    """C2 (840,000 DoF): apply parity everywhere; the solve satisfies the oracle's equations."""
    wl = configs.c2()
    pr = Pair(wl, fp32=True)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    Go, _, _ = pr.oracle_factors()
    rng = np.random.default_rng(2)
    xv = rng.standard_normal(pr.m.n_v)
    yo = op.apply(pr.m, Go, xv)
    assert rel(host(pr.ctx.laplace_apply(dev(xv))), yo) < 1e-13
    assert rel(host(pr.ctx.laplace_apply(dev(xv).float())), yo) < 2e-6
    for v in (1, 6, 7):
        other = Pair(wl, fp32=True, variant=v)
        other.ctx.geom(other.d_eta, other.d_h)
        assert rel(host(other.ctx.laplace_apply(dev(xv))), yo) < 1e-13
        assert rel(host(other.ctx.laplace_apply(dev(xv).float())), yo) < 2e-6
        del other
    for precision, rtol in ((0, 1e-10), (1, 1e-10)):
        phi, info = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(precision=precision, rtol=rtol))
        assert info["status"] == "OK"
        ph = host(phi)
        lift = np.zeros(pr.m.n_v)
        lift[sv.surface_slice(pr.m)] = pr.phis
        b = -op.apply(pr.m, Go, lift)
        r = -op.apply(pr.m, Go, ph)
        I = sv.interior_mask(pr.m)
        assert np.linalg.norm(r[I]) <= 1.05 * rtol * np.linalg.norm(b[I])
        assert np.all(ph[sv.surface_slice(pr.m)] == pr.phis)
        wo = sf.w_surface(pr.m, ph, pr.eta, pr.h, pr.xh)
        assert rel(host(pr.ctx.w_surface(phi)), wo) < 1e-12


@pytest.mark.parametrize("variant", [0, 6, 7])
def test_c5_sampled_apply(variant):
    """C5 (43,675,392 DoF): apply parity at the nodes of sampled columns (oracle on their
    neighbourhood); with the default schedule also the FP32 apply and the assembled diagonal."""
    wl = configs.c5()
    m = wl.mesh
    ctx = fnpf.Context(m, g=wl.g)
    ctx.set_apply_variant(variant)
    x, y = ctx.node_xy()
    h = np.asarray(wl.depth(x, y))
    eta = np.asarray(wl.eta0(x, y))
    ctx.geom(dev(eta), dev(h))
    rng = np.random.default_rng(4)
    xv = torch.randn(m.n_v, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(4))
    y_gpu = host(ctx.laplace_apply(xv))
    xv_h = host(xv)
    if variant == 0:
        # the FP32 apply at the same columns, and the assembled diagonal (by default kept only
        # where the face pass completes it: the export recomputes it whole)
        ctx.enable_fp32()
        ctx.geom(dev(eta), dev(h))
        y32 = host(ctx.laplace_apply(xv.float()))
        diag = host(ctx.export_geometry(fnpf.F64)[1])
    nx, ny = m.extra["nx"], m.extra["ny"]
    samples = [(0, 0), (nx - 1, ny - 1), (nx // 2, ny // 2), (17, 101), (200, 3)]
    xh_all = None
    for (cx, cy) in samples:
        nb = sorted({((cx + dx) % nx) + ((cy + dy) % ny) * nx for dx in (-1, 0, 1) for dy in (-1, 0, 1)
                     if 0 <= cx + dx < nx})
        if xh_all is None:
            xh_all = geo.horizontal_coords(m)
        G, _, _ = geo.factors(m, eta, h, xh_all, cols=nb)
        dofs = geo.dof_map(m, cols=nb)
        yo = op.apply(m, G, xv_h, dofs)
        own = geo.dof_map(m, cols=[cx + cy * nx]).ravel()
        # p = 6 contractions of strongly anisotropic factors (aspect ratio ~ 5): rounding order
        # differences between the two sums reach a few 1e-13
        assert rel(y_gpu[own], yo[own]) < 2e-12
        if variant == 0:
            assert rel(y32[own], yo[own]) < 2e-6
            do = op.diagonal(m, G, dofs)
            # sums over up to eight elements in another order, of terms the anisotropic factors
            # make up to two orders of magnitude apart: measured 7e-13 of the largest entry
            assert np.abs(diag[own] - do[own]).max() < 2e-12 * np.abs(do[own]).max()


def test_error_paths():
    wl = configs.small_box(nx=3, ny=3, nz=2, p=2, periodic=(True, True))
    pr = Pair(wl)
    with pytest.raises(fnpf.FnpfError) as ei:
        pr.ctx.laplace_apply(pr.d_h.new_zeros(pr.m.n_v))
    assert ei.value.name == "ERR_STATE"
    pr.ctx.geom(pr.d_eta, pr.d_h)
    _, info = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-14, max_iter=1, check_every=1),
                           raise_on_error=False)
    assert info["status"] == "ERR_NOCONV" and info["iters"] == 1 and info["rel_res"] > 1e-14
    bad = pr.eta.copy()
    bad[3] = -pr.h[3] - 0.1
    pr.ctx.geom(dev(bad), pr.d_h)
    _, info = pr.ctx.solve(pr.d_phis, raise_on_error=False)
    assert info["status"] == "ERR_GEOM"
    with pytest.raises(fnpf.FnpfError):
        pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(precond=3))
    with pytest.raises(fnpf.FnpfError):
        pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(precond=2, cheb_degree=0))
    # the removed measurement schedules (2..5) and unknown variants are rejected
    for v in (-1, 2, 3, 4, 5, 8):
        with pytest.raises(fnpf.FnpfError) as ei:
            pr.ctx.set_apply_variant(v)
        assert ei.value.name == "ERR_ARG"
    # the binding checks sizes, dtypes and devices before the library sees a pointer
    pr.ctx.geom(pr.d_eta, pr.d_h)
    x = pr.d_h.new_zeros(pr.m.n_v)
    with pytest.raises(ValueError):
        pr.ctx.laplace_apply(x[:-1])
    with pytest.raises(ValueError):
        pr.ctx.laplace_apply(x, y=x.new_zeros(pr.m.n_v - 1))
    with pytest.raises(ValueError):
        pr.ctx.w_surface(x, w=x.new_zeros(pr.m.n_s + 1))
    with pytest.raises(ValueError):
        pr.ctx.rk4_step(pr.d_eta.clone(), pr.d_phis.clone(), pr.d_h[:-1], 0.0, 0.01)
    with pytest.raises(ValueError):
        pr.ctx.rk4_step(pr.d_eta.clone(), pr.d_phis.clone(), pr.d_h, 0.0, 0.01,
                        tape=x.new_zeros(4 * pr.ctx.tape_record - 1))
    with pytest.raises(ValueError):
        pr.ctx.geom(pr.d_eta.cpu(), pr.d_h)
    with pytest.raises(TypeError):
        pr.ctx.laplace_apply(x.half())


def test_bitwise_repeatable():
    wl = configs.small_box(nx=4, ny=4, nz=2, p=4, periodic=(True, True))
    pr = Pair(wl)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    a, _ = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-12, check_every=3))
    b, _ = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-12, check_every=11))
    assert torch.equal(a, b)


@pytest.mark.parametrize("precond", [0, 2])
@pytest.mark.parametrize("name", ["slice_walls", "box_mixed", "box_walls_p6", "cylinder", "cylinder_blocked"])
def test_solve_preconditioners(name, precond):
    """No preconditioner and the p-multigrid V-cycle reach the oracle's solution like Jacobi does."""
    pr = Pair(_case(name), fp32=True)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    Go, _, _ = pr.oracle_factors()
    phio = sv.solve_dense(pr.m, op.assemble_dense(pr.m, Go), pr.phis)
    phi, info = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-13, check_every=5, precond=precond))
    assert info["status"] == "OK" and info["rel_res"] <= 1e-13
    assert rel(host(phi), phio) < 1e-10
    _, info_j = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-13, check_every=5, precond=1))
    if precond == 2 and pr.m.p >= 3:
        assert info["iters"] < info_j["iters"]
    phim, infom = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(precision=1, rtol=1e-11, inner_rtol=1e-3,
                                                                  precond=precond))
    assert infom["status"] == "OK"
    assert rel(host(phim), phio) < 1e-8


@pytest.mark.parametrize("name", ["box_periodic", "box_walls_p6", "cylinder"])
def test_multigrid_eigenvalue_estimate(name):
    """The estimate of the largest eigenvalue of D^-1 A that sets the Chebyshev smoothing
    intervals: on the fine level it lies within 3% below the exact value of the oracle's
    assembled matrix (Lanczos on first use, power iterations from its Ritz vector after a
    geometry update), in both precisions; every level has a positive estimate.  The smoother
    stops being a contraction for eigenvalues above (1 + 1/24) x 1.1 x the estimate, so an
    estimate 1.146x short makes the V-cycle indefinite."""
    pr = Pair(_case(name), fp32=True)
    I = sv.interior_mask(pr.m)

    def lam_true(eta):
        Go, _, _ = geo.factors(pr.m, eta, pr.h, pr.xh)
        A = op.assemble_dense(pr.m, Go)[np.ix_(I, I)]
        s = 1.0 / np.sqrt(np.diag(A))
        return np.linalg.eigvalsh(A * s[:, None] * s[None, :]).max()

    for k, eta in enumerate((pr.eta, 1.5 * pr.eta)):
        pr.ctx.geom(dev(eta), pr.d_h)
        for precision in (0, 1):
            o = fnpf.default_opts(precision=precision, rtol=1e-10, inner_rtol=1e-3, precond=2)
            _, info = pr.ctx.solve(pr.d_phis, opts=o)
            assert info["status"] == "OK"
        mi = pr.ctx.multigrid_info()
        lt = lam_true(eta)
        assert mi["levels"] == (3 if pr.m.p == 6 else 2)
        assert 0.97 * lt <= mi["lam64"][0] <= lt * (1 + 1e-9), (k, mi, lt)
        assert 0.97 * lt <= mi["lam32"][0] <= lt * (1 + 1e-5), (k, mi, lt)
        assert all(x > 0 for x in mi["lam64"] + mi["lam32"])


@pytest.mark.parametrize("precision", [0, 1])
def test_rk4_step_multigrid(precision):
    """ERK4 steps with the p-multigrid preconditioner (geometry refreshed every stage)."""
    wl = _case("box_walls_p6")
    pr = Pair(wl, fp32=precision == 1)
    md = ts.Model(wl, solver="dense")
    dt = 0.02
    e1, p1 = md.rk4_step(pr.eta, pr.phis, 0.0, dt)
    e2, p2 = md.rk4_step(e1, p1, dt, dt)
    e, p = pr.d_eta.clone(), pr.d_phis.clone()
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-12, inner_rtol=1e-3,
                             precond=2)
    pr.ctx.rk4_step(e, p, pr.d_h, 0.0, dt, opts=opts)
    infos = pr.ctx.rk4_step(e, p, pr.d_h, dt, dt, opts=opts)
    tol = 1e-10 if precision == 0 else 1e-8
    assert rel(host(e), e2) < tol and rel(host(p), p2) < tol
    assert all(i["rel_res"] <= opts.rtol for i in infos)


def test_warm_start_extrapolation_c2():
    """C2 full size, 7 ERK4 steps: initial guesses extrapolated in time with polynomials of degree
    0 (none) to 4 from the previous steps reach the same states to the solve tolerance; each degree
    repeats the iterations of the one below until its longer history exists; and, with their
    histories in place, the quadratic guess needs fewer CG iterations than the linear one or none,
    and the quartic one no more than the quadratic.  (The previous stage's potential, used without
    extrapolation, is already a second-order guess for the first and third stages, so the linear
    extrapolation need not beat it.)"""
    wl = configs.c2()
    out, iters = {}, {}
    for ex in (0, 1, 2, 3, 4):
        pr = Pair(wl)   # a fresh context each: the multigrid eigenvalue estimates carry over otherwise
        e, p = pr.d_eta.clone(), pr.d_phis.clone()
        opts = fnpf.default_opts(rtol=1e-10, extrapolate=ex)
        its = []
        for n in range(7):
            infos = pr.ctx.rk4_step(e, p, pr.d_h, n * wl.dt, wl.dt, opts=opts)
            its.append(sum(i["iters"] for i in infos))
        out[ex], iters[ex] = (host(e), host(p)), its
    for ex in (1, 2, 3, 4):
        assert rel(out[ex][0], out[0][0]) < 1e-8 and rel(out[ex][1], out[0][1]) < 1e-8
        # degree ex needs ex + 1 past steps: the first ex + 1 steps repeat degree ex - 1
        assert iters[ex][: ex + 1] == iters[ex - 1][: ex + 1], iters
    assert all(iters[2][n] < min(iters[1][n], iters[0][n]) for n in (5, 6)), iters
    assert all(iters[4][n] <= iters[2][n] for n in (5, 6)), iters


def test_extrapolation_degree_changes_within_a_run():
    """Changing opts.extrapolate between steps of one context (4, then 2, 0, 3 and 1, and a
    different dt in between) restarts the history each time and keeps every state within the
    solve tolerance of a run without extrapolation."""
    wl = _case("box_mixed")
    runs = {}
    for plan in ("mixed", "none"):
        pr = Pair(wl)
        e, p = pr.d_eta.clone(), pr.d_phis.clone()
        t, states = 0.0, []
        for ex, dt, n in ((4, 0.02, 6), (2, 0.02, 3), (0, 0.02, 2), (3, 0.01, 5), (1, 0.02, 3)):
            o = fnpf.default_opts(rtol=1e-12, extrapolate=ex if plan == "mixed" else 0)
            for _ in range(n):
                infos = pr.ctx.rk4_step(e, p, pr.d_h, t, dt, opts=o)
                assert all(i["rel_res"] <= 1e-12 for i in infos)
                t += dt
            states.append((host(e), host(p)))
        runs[plan] = states
    for (ea, pa), (eb, pb) in zip(runs["mixed"], runs["none"]):
        assert rel(ea, eb) < 1e-9 and rel(pa, pb) < 1e-9


def test_multigrid_repeatable_and_c2():
    """C2 full size: the multigrid solve is bitwise repeatable and satisfies the oracle's residual."""
    wl = configs.c2()
    pr = Pair(wl, fp32=True)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    o = fnpf.default_opts(rtol=1e-10, precond=2, check_every=3)
    a, ia = pr.ctx.solve(pr.d_phis, opts=o)
    b, ib = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-10, precond=2, check_every=7))
    assert torch.equal(a, b) and ia["iters"] == ib["iters"]
    _, ij = pr.ctx.solve(pr.d_phis, opts=fnpf.default_opts(rtol=1e-10, precond=1))
    assert ia["iters"] * 4 < ij["iters"]
    Go, _, _ = pr.oracle_factors()
    lift = np.zeros(pr.m.n_v)
    lift[sv.surface_slice(pr.m)] = pr.phis
    bvec = -op.apply(pr.m, Go, lift)
    r = -op.apply(pr.m, Go, host(a))
    I = sv.interior_mask(pr.m)
    assert np.linalg.norm(r[I]) <= 1.05e-10 * np.linalg.norm(bvec[I])


def test_c2_fifty_steps_fp64_vs_mixed_and_invariants():
    """C2 full size (840,000 DoF), 50 ERK4 steps at rtol 1e-8 in FP64 and in mixed precision:
    the two trajectories agree to the solver tolerance, and the discrete mass (lumped surface mass
    times eta) and energy (kinetic phi.A phi / 2 plus potential g m.eta^2 / 2) stay constant to
    the solver tolerance and the time-discretisation error of ERK4 at T/64 (the periodic
    flat-bottom domain conserves both)."""
    wl = configs.c2()
    pr = Pair(wl, fp32=True)
    ms = sf.surface_mass(pr.m, pr.xh)

    def energy(e, p):
        pr.ctx.geom(e, pr.d_h)
        phi, info = pr.ctx.solve(p, opts=fnpf.default_opts(rtol=1e-12))
        assert info["status"] == "OK"
        kin = 0.5 * float(torch.dot(phi, pr.ctx.laplace_apply(phi)))
        eh = host(e)
        return kin + 0.5 * wl.g * float(ms @ (eh * eh))

    out = {}
    for precision in (0, 1):
        e, p = pr.d_eta.clone(), pr.d_phis.clone()
        pr.ctx.set_warm_start(None)
        opts = fnpf.default_opts(precision=precision, rtol=1e-8, inner_rtol=1e-4)
        t = 0.0
        for n in range(50):
            pr.ctx.rk4_step(e, p, pr.d_h, t, wl.dt, opts=opts)
            t += wl.dt
        out[precision] = (host(e), host(p), e, p)
    e64, p64 = out[0][0], out[0][1]
    assert rel(out[1][0], e64) < 1e-6 and rel(out[1][1], p64) < 1e-6
    # mass: d/dt sum(m eta) is the surface flux of the solved potential.  A annihilates constants,
    # so the total flux is minus the sum of the solve residual over the unknowns, at most
    # sqrt(n_I) ||r|| <= sqrt(n_I) rtol ||b|| per stage: zero only up to the solve tolerance, with a
    # constant that depends on how coherent the final residual is (measured: 2e-7 of
    # sum(m |eta|) ~ 1.3 at rtol 1e-8 with the multigrid CG).  An error in the kinematic condition
    # or the w recovery moves it by ~1e-2.
    m0, m1 = ms @ pr.eta, ms @ e64
    assert abs(m1 - m0) < 1e-6 * (ms @ np.abs(pr.eta))
    E0 = energy(pr.d_eta, pr.d_phis)
    E1 = energy(out[0][2], out[0][3])
    assert abs(E1 - E0) < 1e-6 * E0


def test_c5_twenty_steps_fp64_vs_mixed():
    """C5 full size (43.7 M DoF), 20 ERK4 steps at rtol 1e-8 in FP64 and in mixed precision (the
    benchmark's solver settings): every stage converges, the two trajectories agree to the solver
    tolerance, and the state stays finite and bounded."""
    wl = configs.c5()
    s = fnpf.setup_workload(wl, fp32=True)
    out = {}
    for precision in (0, 1):
        e, p = s.eta0.clone(), s.phi0.clone()
        s.ctx.set_warm_start(None)
        opts = fnpf.default_opts(precision=precision, rtol=1e-8, check_every=5)
        t = 0.0
        for n in range(20):
            infos = s.ctx.rk4_step(e, p, s.h, t, wl.dt, opts=opts)
            assert all(i["rel_res"] <= 1e-8 for i in infos), (precision, n, infos)
            t += wl.dt
        out[precision] = (host(e), host(p))
    assert rel(out[1][0], out[0][0]) < 1e-6 and rel(out[1][1], out[0][1]) < 1e-6
    e0 = host(s.eta0)
    assert np.all(np.isfinite(out[0][0])) and np.abs(out[0][0]).max() < 10 * np.abs(e0).max()


def test_c3_full_size_cylinder():
    """C3 (cylinder in a tank, 771,528 DoF, unstructured O-grid + jittered block, relaxation zones):
    apply parity everywhere, multigrid solves that satisfy the oracle's equations, w parity, and
    ERK4 steps with relaxation whose FP64 and mixed results agree."""
    wl = configs.c3()
    pr = Pair(wl, fp32=True)
    pr.ctx.geom(pr.d_eta, pr.d_h)
    Go, _, _ = pr.oracle_factors()
    rng = np.random.default_rng(3)
    xv = rng.standard_normal(pr.m.n_v)
    yo = op.apply(pr.m, Go, xv)
    # curved (arc) and jittered elements: the factors vary inside every element and the two sides
    # form them in different orders, so the sums differ by a few 1e-13
    assert rel(host(pr.ctx.laplace_apply(dev(xv))), yo) < 1e-12
    assert rel(host(pr.ctx.laplace_apply(dev(xv).float())), yo) < 2e-6
    # a wavy state so the solve is not trivial
    eta = 0.02 * np.cos(pr.x) * np.sin(0.7 * pr.y)
    phis = 0.05 * np.sin(pr.x + 0.2 * pr.y)
    pr.ctx.geom(dev(eta), pr.d_h)
    G2, _, _ = geo.factors(pr.m, eta, pr.h, pr.xh)
    lift = np.zeros(pr.m.n_v)
    lift[sv.surface_slice(pr.m)] = phis
    b = -op.apply(pr.m, G2, lift)
    I = sv.interior_mask(pr.m)
    for precision in (0, 1):
        phi, info = pr.ctx.solve(dev(phis), opts=fnpf.default_opts(precision=precision, rtol=1e-10))
        assert info["status"] == "OK" and info["iters"] < 120
        r = -op.apply(pr.m, G2, host(phi))
        assert np.linalg.norm(r[I]) <= 1.05e-10 * np.linalg.norm(b[I])
    wo = sf.w_surface(pr.m, host(phi), eta, pr.h, pr.xh)
    assert rel(host(pr.ctx.w_surface(phi)), wo) < 1e-12
    x, y = pr.ctx.node_xy()
    ra = wl.relaxation_arrays(x, y)
    pr.ctx.set_relaxation(*ra, omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    res = []
    for precision in (0, 1):
        e, p = dev(eta), dev(phis)
        o = fnpf.default_opts(precision=precision, rtol=1e-11, inner_rtol=1e-3)
        for n in range(3):
            pr.ctx.rk4_step(e, p, pr.d_h, n * wl.dt, wl.dt, opts=o)
        res.append((host(e), host(p)))
    assert rel(res[1][0], res[0][0]) < 1e-8 and rel(res[1][1], res[0][1]) < 1e-8


@pytest.mark.parametrize("precond", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_eager(precision, precond):
    """Iteration chunks replayed as HIP graphs give bitwise the eager result, replay after replay,
    with eager work (geometry, RHS, surface kernels, host checks) between the replays."""
    wl = _case("box_walls_p6")
    pe, pg = Pair(wl, fp32=True), Pair(wl, fp32=True)
    kw = dict(precision=precision, precond=precond, rtol=1e-12, inner_rtol=1e-3, check_every=3)
    oe, og = fnpf.default_opts(use_graph=0, **kw), fnpf.default_opts(use_graph=1, **kw)
    ee, phe = pe.d_eta.clone(), pe.d_phis.clone()
    eg, phg = pg.d_eta.clone(), pg.d_phis.clone()
    t, dt = 0.0, 0.02
    for n in range(4):
        ie = pe.ctx.rk4_step(ee, phe, pe.d_h, t, dt, opts=oe)
        ig = pg.ctx.rk4_step(eg, phg, pg.d_h, t, dt, opts=og)
        torch.cuda.synchronize()
        assert torch.equal(ee, eg) and torch.equal(phe, phg), f"step {n}"
        assert [i["iters"] for i in ie] == [i["iters"] for i in ig]
        t += dt
    # fnpf_solve into caller tensors: a new solution pointer captures a new graph
    for k in range(3):
        xe = torch.zeros(pe.m.n_v, dtype=torch.float64, device="cuda")
        xg = torch.zeros(pg.m.n_v, dtype=torch.float64, device="cuda")
        pe.ctx.geom(ee, pe.d_h)
        pg.ctx.geom(eg, pg.d_h)
        _, a = pe.ctx.solve(phe, phi=xe, opts=oe)
        _, b = pg.ctx.solve(phg, phi=xg, opts=og)
        assert torch.equal(xe, xg) and a["iters"] == b["iters"], f"solve {k}"
