"""Degenerate inputs of the per-stage path (Sec. 3.4 Steps 4.1-4.7), whose answers are exact:

* zero surface data: the Laplace solve (Eq. 1 with phi = 0 on the surface, no Neumann data) has
  the zero solution, reached with no iterations, by every preconditioner and precision;
* a constant surface potential over walls: A annihilates constants, so the harmonic extension is
  that constant everywhere (to the solver tolerance);
* still water: eta = 0, phi_s = 0 is a fixed point of the ERK4 step (Eqs. 2-3 vanish), bit for bit.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_09435_amd import fnpf
from workloads import configs


def _setup(name):
    if name == "slice":
        wl = configs.small_slice(nx=4, nz=2, p=5, periodic=False)
    elif name == "box":
        wl = configs.small_box(nx=4, ny=3, nz=2, p=4, periodic=(False, True))
    else:
        wl = configs.small_box(nx=3, ny=2, nz=2, p=6, periodic=(False, False))
    return wl, fnpf.setup_workload(wl, fp32=True)


@pytest.mark.parametrize("name", ["slice", "box", "box_p6"])
@pytest.mark.parametrize("precond,precision", [(0, 0), (1, 0), (2, 0), (1, 1), (2, 1)])
def test_zero_surface_data_gives_zero_potential(name, precond, precision):
    wl, s = _setup(name)
    s.ctx.geom(s.eta0, s.h)
    zero = torch.zeros(s.ctx.n_s, dtype=torch.float64, device="cuda")
    phi, info = s.ctx.solve(zero, opts=fnpf.default_opts(precond=precond, precision=precision, rtol=1e-12))
    assert info["status"] == "OK" and info["iters"] == 0
    assert float(phi.abs().max()) == 0.0


@pytest.mark.parametrize("name", ["slice", "box", "box_p6"])
@pytest.mark.parametrize("precond", [1, 2])
def test_constant_surface_potential_extends_as_the_constant(name, precond):
    wl, s = _setup(name)
    s.ctx.geom(s.eta0, s.h)
    c = 0.37
    phis = torch.full((s.ctx.n_s,), c, dtype=torch.float64, device="cuda")
    phi, info = s.ctx.solve(phis, opts=fnpf.default_opts(precond=precond, rtol=1e-13))
    assert info["status"] == "OK"
    assert float((phi - c).abs().max()) <= 1e-10 * c
    # and the vertical velocity it implies at the surface is zero
    w = s.ctx.w_surface(phi)
    assert float(w.abs().max()) <= 1e-9


@pytest.mark.parametrize("name", ["slice", "box", "box_p6"])
@pytest.mark.parametrize("precision", [0, 1])
def test_still_water_is_a_fixed_point(name, precision):
    wl, s = _setup(name)
    e = torch.zeros(s.ctx.n_s, dtype=torch.float64, device="cuda")
    p = torch.zeros_like(e)
    for n in range(3):
        s.ctx.rk4_step(e, p, s.h, n * 0.02, 0.02, opts=fnpf.default_opts(precision=precision, rtol=1e-12))
    assert float(e.abs().max()) == 0.0 and float(p.abs().max()) == 0.0
