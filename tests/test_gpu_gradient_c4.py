"""Adjoint gradient of the C4 twin experiment at its configured size, against central finite
differences of the library's own FP64 forward.

C4: submerged bar, 64 x 16 x 4 hexes, p = 5 (546,021 DoF), relaxation zones, 200 ERK4 steps of
T/64 from the incident linear wave over the flume, loss = 1/2 sum over steps and 8 gauges of the
squared misfit to observations from the perturbed bathymetry c_true; gradient with respect to the
64 bathymetry control points and the initial elevation.  Forward and adjoint in FP64 at rtol 1e-12.
Checked: five seeded control directions and one smooth initial-elevation direction, central
differences with eps = 1e-4, relative agreement <= 1e-5 (one test per direction, each two
rollouts, sharing the module's adjoint gradient); and the gradient of the mixed forward (FP32
inner solves) with FP64 adjoint solves against the FP64 gradient.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_09435_amd import fnpf
from paper_2506_09435_amd.autograd import gauge_matrix, rollout
from workloads import configs, waves

FD_BAR = 1e-5


class _C4:
    """The C4 twin experiment: context, controls, observations and the FP64 adjoint gradient."""

    def __init__(self):
        wl = configs.c4()
        m = wl.mesh
        self.wl, self.N, self.dt = wl, wl.nsteps, wl.dt
        assert (m.n_eh, m.nz, m.p, m.n_v, self.N) == (64 * 16, 4, 5, 546021, 200)
        self.fctx = fnpf.Context(m, g=wl.g)
        self.x, y = self.fctx.node_xy()
        self.fctx.set_relaxation(*wl.relaxation_arrays(self.x, y), omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
        self.c0 = wl.meta["c0"]
        self.B = torch.tensor(waves.piecewise_linear_matrix(self.x, wl.meta["xc"]), device="cuda")
        self.P = gauge_matrix(self.fctx, wl.meta["gauges"])
        self.eta_in = torch.tensor(wl.relax_wave.eta(self.x, y, 0.0), device="cuda")
        self.phi_in = torch.tensor(wl.relax_wave.phi(self.x, y, 0.0), device="cuda")
        self.o64 = fnpf.default_opts(rtol=1e-12, precond=1, check_every=25)
        with torch.no_grad():
            c_true = torch.tensor(wl.meta["c_true"], device="cuda")
            self.obs = rollout(self.fctx, self.eta_in, self.phi_in, self.B @ c_true, 0.0, self.dt, self.N,
                               opts=self.o64) @ self.P.T
        c = torch.tensor(self.c0, device="cuda", requires_grad=True)
        e0 = self.eta_in.clone().requires_grad_(True)
        self.loss(c, e0, self.o64).backward()
        self.gc, self.ge = c.grad.clone(), e0.grad.clone()

    def loss(self, c, e0, opts, adj_opts=None):
        traj = rollout(self.fctx, e0, self.phi_in, self.B @ c, 0.0, self.dt, self.N, opts=opts, adj_opts=adj_opts)
        return 0.5 * ((traj @ self.P.T - self.obs) ** 2).sum()

    def direction(self, k):
        g = np.random.default_rng(self.wl.meta["fd_seed"] + k)
        if k < 5:
            vc = torch.tensor(g.standard_normal(len(self.c0)) * 0.01, device="cuda")
            ve = torch.zeros_like(self.eta_in)
        else:
            # smooth initial-elevation direction: seeded long-wave modes along the flume
            kx = 2 * np.pi * np.arange(1, 5) / 38.0
            amp, ph = g.standard_normal(4), g.uniform(0, 2 * np.pi, 4)
            vc = torch.zeros(len(self.c0), dtype=torch.float64, device="cuda")
            ve = torch.tensor(1e-3 * (amp[None, :] * np.cos(kx[None, :] * self.x[:, None] + ph[None, :])).sum(1),
                              device="cuda")
        return vc, ve


@pytest.fixture(scope="module")
def c4():
    return _C4()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", range(6))
def test_c4_config_size_gradient_vs_central_differences(c4, k):
    vc, ve = c4.direction(k)
    d_adj = float(c4.gc @ vc + c4.ge @ ve)
    eps = 1e-4
    c = torch.tensor(c4.c0, device="cuda")
    with torch.no_grad():
        jp = float(c4.loss(c + eps * vc, c4.eta_in + eps * ve, c4.o64))
        jm = float(c4.loss(c - eps * vc, c4.eta_in - eps * ve, c4.o64))
    d_fd = (jp - jm) / (2 * eps)
    rel = abs(d_adj - d_fd) / abs(d_fd)
    print(f"direction {k}: adjoint {d_adj:.10e} fd {d_fd:.10e} rel {rel:.2e}", flush=True)
    assert rel <= FD_BAR, rel


@pytest.mark.timeout(600)
def test_c4_mixed_forward_gradient_matches_fp64(c4):
    # mixed forward (FP32 inner solves, FP64 defect correction) with FP64 adjoint solves
    om = fnpf.default_opts(rtol=1e-12, precond=1, precision=1, inner_rtol=1e-4, check_every=25)
    cm = torch.tensor(c4.c0, device="cuda", requires_grad=True)
    em = c4.eta_in.clone().requires_grad_(True)
    c4.loss(cm, em, om, adj_opts=c4.o64).backward()
    agree = float(torch.linalg.norm(torch.cat([cm.grad - c4.gc, em.grad - c4.ge])) /
                  torch.linalg.norm(torch.cat([c4.gc, c4.ge])))
    print(f"mixed-forward / FP64-adjoint gradient vs FP64: relative difference {agree:.2e}", flush=True)
    assert agree <= 1e-6, agree
