"""Adjoint gradient of the C4 twin experiment at its configured size, against central finite
differences of the library's own FP64 forward.

C4: submerged bar, 64 x 16 x 4 hexes, p = 5 (546,021 DoF), relaxation zones, 200 ERK4 steps of
T/64 from the incident linear wave over the flume, loss = 1/2 sum over steps and 8 gauges of the
squared misfit to observations from the perturbed bathymetry c_true; gradient with respect to the
64 bathymetry control points and the initial elevation.  Forward and adjoint in FP64 at rtol 1e-12.
Checked: five seeded control directions and one smooth initial-elevation direction, central
differences with eps = 1e-4, relative agreement <= 1e-5; and the gradient of the mixed forward
(FP32 inner solves) with FP64 adjoint solves against the FP64 gradient.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_09435_amd import fnpf
from paper_2506_09435_amd.autograd import gauge_matrix, rollout
from workloads import configs, waves

FD_BAR = 1e-5


@pytest.mark.timeout(1200)
def test_c4_config_size_gradient_vs_central_differences():
    wl = configs.c4()
    m, N, dt = wl.mesh, wl.nsteps, wl.dt
    assert (m.n_eh, m.nz, m.p, m.n_v, N) == (64 * 16, 4, 5, 546021, 200)
    fctx = fnpf.Context(m, g=wl.g)
    x, y = fctx.node_xy()
    fctx.set_relaxation(*wl.relaxation_arrays(x, y), omega=wl.relax_wave.omega, t_ramp=wl.t_ramp)
    xc, c0 = wl.meta["xc"], wl.meta["c0"]
    B = torch.tensor(waves.piecewise_linear_matrix(x, xc), device="cuda")
    P = gauge_matrix(fctx, wl.meta["gauges"])
    eta_in = torch.tensor(wl.relax_wave.eta(x, y, 0.0), device="cuda")
    phi_in = torch.tensor(wl.relax_wave.phi(x, y, 0.0), device="cuda")
    o64 = fnpf.default_opts(rtol=1e-12, precond=1, check_every=25)
    with torch.no_grad():
        obs = rollout(fctx, eta_in, phi_in, B @ torch.tensor(wl.meta["c_true"], device="cuda"), 0.0, dt, N,
                      opts=o64) @ P.T

    def loss(c, e0, opts, adj_opts=None):
        traj = rollout(fctx, e0, phi_in, B @ c, 0.0, dt, N, opts=opts, adj_opts=adj_opts)
        return 0.5 * ((traj @ P.T - obs) ** 2).sum()

    c = torch.tensor(c0, device="cuda", requires_grad=True)
    e0 = eta_in.clone().requires_grad_(True)
    loss(c, e0, o64).backward()
    gc, ge = c.grad.clone(), e0.grad.clone()
    rels = []
    for k in range(6):
        g = np.random.default_rng(wl.meta["fd_seed"] + k)
        if k < 5:
            vc = torch.tensor(g.standard_normal(len(c0)) * 0.01, device="cuda")
            ve = torch.zeros_like(eta_in)
        else:
            # smooth initial-elevation direction: seeded long-wave modes along the flume
            kx = 2 * np.pi * np.arange(1, 5) / 38.0
            amp, ph = g.standard_normal(4), g.uniform(0, 2 * np.pi, 4)
            vc = torch.zeros_like(c.detach())
            ve = torch.tensor(1e-3 * (amp[None, :] * np.cos(kx[None, :] * x[:, None] + ph[None, :])).sum(1),
                              device="cuda")
        d_adj = float(gc @ vc + ge @ ve)
        eps = 1e-4
        with torch.no_grad():
            jp = float(loss(c.detach() + eps * vc, e0.detach() + eps * ve, o64))
            jm = float(loss(c.detach() - eps * vc, e0.detach() - eps * ve, o64))
        d_fd = (jp - jm) / (2 * eps)
        rels.append(abs(d_adj - d_fd) / abs(d_fd))
        print(f"direction {k}: adjoint {d_adj:.10e} fd {d_fd:.10e} rel {rels[-1]:.2e}", flush=True)
    assert max(rels) <= FD_BAR, rels
    # mixed forward (FP32 inner solves, FP64 defect correction) with FP64 adjoint solves
    om = fnpf.default_opts(rtol=1e-12, precond=1, precision=1, inner_rtol=1e-4, check_every=25)
    cm = torch.tensor(c0, device="cuda", requires_grad=True)
    em = eta_in.clone().requires_grad_(True)
    loss(cm, em, om, adj_opts=o64).backward()
    agree = float(torch.linalg.norm(torch.cat([cm.grad - gc, em.grad - ge])) /
                  torch.linalg.norm(torch.cat([gc, ge])))
    print(f"mixed-forward / FP64-adjoint gradient vs FP64: relative difference {agree:.2e}", flush=True)
    assert agree <= 1e-6, agree
