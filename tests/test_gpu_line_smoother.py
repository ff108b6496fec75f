"""The vertical line smoother of the p-multigrid preconditioner (opts.line_smoother = 1).

* fnpf_line_smoother_apply against the oracle's block solve with the line blocks of its assembled
  operator (oracle.solve.line_blocks / line_solve), FP64 at rounding level and FP32 within the
  blocks' condition number times the FP32 unit roundoff;
* the Laplace solve with line smoothing against the oracle's dense solve (FP64 path 1e-10,
  mixed path 1e-8) on every mesh family and degree range, and one ERK4 step;
* on thin layers (strong vertical coupling) the line smoother needs fewer CG iterations than
  point smoothing.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import geometry as geo
from oracle import operator as op
from oracle import solve as sv
from oracle import timestep as ts
from paper_2506_09435_amd import fnpf
from workloads import configs, mesh as wm


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _case(name):
    if name == "slice":
        return configs.small_slice(nx=5, nz=3, p=4, periodic=True)
    if name == "box":
        return configs.small_box(nx=4, ny=3, nz=2, p=3, periodic=(True, True))
    if name == "box_walls_p6":
        return configs.small_box(nx=3, ny=2, nz=2, p=6, periodic=(False, False))
    if name == "box_p1":
        return configs.small_box(nx=4, ny=3, nz=3, p=1, periodic=(True, False))
    if name == "box_p8":
        return configs.small_box(nx=3, ny=3, nz=1, p=8, periodic=(True, False))
    if name == "cylinder":
        wl = configs.small_box()
        wl.mesh = wm.cylinder_tank_mesh(p=3, nz=2, n_theta=8, n_rad=2, tank=(6.0, 4.0), spacing=1.0, hole_half=1.0)
        wl.depth = lambda x, y: 1.0 + 0.1 * np.cos(0.5 * np.asarray(x)) * np.sin(np.asarray(y))
        wl.eta0 = lambda x, y: 0.05 * np.cos(np.asarray(x)) * np.sin(np.asarray(y))
        wl.phi0 = lambda x, y: 0.1 * np.sin(np.asarray(x) + 0.3 * np.asarray(y))
        return wl
    if name == "thin":
        # shallow, finely layered box: the vertical coupling dominates
        wl = configs.small_box(nx=4, ny=3, nz=4, p=3, periodic=(True, False), lx=6.0, ly=4.5)
        wl.depth = lambda x, y: 0.15 + 0.02 * np.cos(np.asarray(x))
        wl.eta0 = lambda x, y: 0.005 * np.cos(np.asarray(x)) * np.cos(0.5 * np.asarray(y))
        return wl
    raise KeyError(name)


CASES = ["slice", "box", "box_walls_p6", "box_p1", "box_p8", "cylinder", "thin"]


def _setup(name):
    wl = _case(name)
    m = wl.mesh
    x, y = geo.node_xy(m)
    h = np.asarray(wl.depth(x, y), dtype=np.float64)
    eta = np.asarray(wl.eta0(x, y), dtype=np.float64)
    phis = np.asarray(wl.phi0(x, y), dtype=np.float64)
    G, _, _ = geo.factors(m, eta, h)
    return wl, m, h, eta, phis, op.assemble_dense(m, G)


@pytest.mark.parametrize("name", CASES)
def test_line_block_solve_matches_oracle(name):
    wl, m, h, eta, phis, A = _setup(name)
    ctx = fnpf.Context(m, g=wl.g)
    ctx.enable_fp32()
    ctx.geom(dev(eta), dev(h))
    B = sv.line_blocks(m, A)
    r = np.random.default_rng(1).standard_normal(m.n_v)
    zo = sv.line_solve(m, B, r)
    z = host(ctx.line_smoother_apply(dev(r)))
    assert rel(z, zo) < 1e-12
    assert np.all(z[sv.surface_slice(m)] == 0.0)
    kappa = max(np.linalg.cond(b) for b in B)
    z32 = host(ctx.line_smoother_apply(dev(r).float()))
    assert rel(z32, zo) < 50 * kappa * 6e-8, (kappa, rel(z32, zo))


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_solve_with_line_smoother(name, precision):
    wl, m, h, eta, phis, A = _setup(name)
    ctx = fnpf.Context(m, g=wl.g)
    if precision == 1:
        ctx.enable_fp32()
    ctx.geom(dev(eta), dev(h))
    phio = sv.solve_dense(m, A, phis)
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-11, line_smoother=1,
                             check_every=5)
    phi, info = ctx.solve(dev(phis), opts=opts)
    assert info["status"] == "OK", info
    assert rel(host(phi), phio) < (1e-10 if precision == 0 else 1e-8)


@pytest.mark.parametrize("precision", [0, 1])
def test_rk4_step_with_line_smoother(precision):
    wl = configs.small_box(nx=4, ny=3, nz=2, p=4, periodic=(True, False))
    m = wl.mesh
    md = ts.Model(wl, solver="dense")
    eta, phis = md.initial_state()
    e1, p1 = md.rk4_step(eta, phis, 0.0, 0.02)
    ctx = fnpf.Context(m, g=wl.g)
    x, y = geo.node_xy(m)
    e, p = dev(eta), dev(phis)
    opts = fnpf.default_opts(precision=precision, rtol=1e-13 if precision == 0 else 1e-12, inner_rtol=1e-3,
                             line_smoother=1)
    ctx.rk4_step(e, p, dev(np.asarray(wl.depth(x, y), dtype=np.float64)), 0.0, 0.02, opts=opts)
    tol = 1e-10 if precision == 0 else 1e-8
    assert rel(host(e), e1) < tol and rel(host(p), p1) < tol


def test_line_smoother_fewer_iterations_on_thin_layers():
    wl, m, h, eta, phis, A = _setup("thin")
    ctx = fnpf.Context(m, g=wl.g)
    ctx.geom(dev(eta), dev(h))
    its = {}
    for line in (0, 1):
        _, info = ctx.solve(dev(phis), opts=fnpf.default_opts(rtol=1e-10, line_smoother=line, check_every=1))
        its[line] = info["iters"]
    print("iterations point / line:", its)
    assert its[1] < its[0], its
