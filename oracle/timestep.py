"""Time integration around the Laplace solve (paper Sec. 3.2-3.4).

* ERK4 (classic 4-stage, 4th order) with constant dt on (eta, phi_s)
  (Sec. 3.2).  Each stage runs Steps 4.1-4.6: mesh update (geometry from
  eta), Dirichlet lift, Laplace solve, w recovery, free-surface RHS.
* Relaxation after every full step (Sec. 3.3, Step 4.7):
  f <- (1 - C_r) f + C_r f_true, f in {eta, phi_s}; f_true is the incident
  linear wave in the generation zone (ramped in over five periods) and zero
  in the absorption zone.  Reading of the unstated shapes:
  C_r(s) = (1 - cos(pi s))/2 with s the normalised depth into the zone, and
  ramp(t) = (1 - cos(pi t / t_ramp))/2 for t < t_ramp, 1 afterwards.
* Diagnostics: mass sum_n m^s_n eta_n and energy
  1/2 phi^T A phi + 1/2 g sum_n m^s_n eta_n^2 (Zakharov Hamiltonian form).
* Complex-step directional derivatives: every step is complex-analytic, so
  running with eta0 + i e v, h + i e u (e = 1e-30) gives Im(J)/e as the exact
  directional derivative of a real loss J, independent of any adjoint code.
"""

from __future__ import annotations

import math

import numpy as np

from . import geometry as geo
from . import operator as op
from . import solve as sv
from . import surface as sf
from . import filter as mfl
from .gll import gll, lagrange_eval

RK4_C = (0.0, 0.5, 0.5, 1.0)
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


def ramp(t, t_ramp):
    if t_ramp <= 0.0 or t >= t_ramp:
        return 1.0
    return 0.5 * (1.0 - math.cos(math.pi * t / t_ramp))


class Model:
    """FNPF model on one extruded mesh (oracle).

    ``solver``: "dense" (assembled matrix, direct solve; tiny meshes) or "cg"
    (Jacobi-PCG on the matrix-free apply, warm-started from the last stage).
    ``linear``: the linear potential-flow (LPF) model the paper runs beside FNPF (Sec. 2.1
    remark, Sec. 4.1.2): the free surface stays at z = 0, so the Laplace domain is the fixed
    column [-h, 0], and the kinematic and dynamic conditions (Eqs. 2-3) keep only their
    linear terms, d eta/dt = w and d phi_s/dt = -g eta.
    ``modal_filter``: None, or (cutoff, alpha, order) of the modal filter of Sec. 3.2
    (oracle/filter.py), applied to eta and phi_s after every full step (after relaxation).
    ``surface_quadrature``: None (lumped GLL collocation of Eq. 5), or nq >= p + 1: the
    consistent form of Eq. 5 with nq Gauss points per direction (over-integration, Sec. 3.2).
    """

    def __init__(self, workload, solver="dense", rtol=1e-13, linear=False, modal_filter=None,
                 surface_quadrature=None):
        self.wl = workload
        self.linear = linear
        self.modal_filter = modal_filter
        self.nq = surface_quadrature
        self.mesh = workload.mesh
        self.g = workload.g
        self.solver = solver
        self.rtol = rtol
        self.xh = geo.horizontal_coords(self.mesh)
        geo.check_numbering(self.mesh, self.xh)
        self.x, self.y = geo.node_xy(self.mesh)
        self.h = np.asarray(workload.depth(self.x, self.y), dtype=np.float64)
        self.metrics = sf.surface_metrics(self.mesh, self.xh)
        if self.nq:
            self.quad = sf.surface_quadrature(self.mesh, self.nq, self.xh)
            self.mass_c = sf.consistent_surface_mass(self.mesh, self.nq, self.xh)
        self.ms = np.bincount(self.mesh.eh_nodes.ravel(), weights=self.metrics[1].ravel(), minlength=self.mesh.n_s)
        self.dofs = geo.dof_map(self.mesh)
        ra = workload.relaxation_arrays(self.x, self.y)
        self.relax = ra
        self.omega_relax = workload.relax_wave.omega if workload.relax_wave is not None else 0.0
        self.t_ramp = workload.t_ramp
        self.phi = None          # warm start (last stage's volume potential)
        self.last_iters = []

    def initial_state(self):
        return (np.asarray(self.wl.eta0(self.x, self.y), dtype=np.float64),
                np.asarray(self.wl.phi0(self.x, self.y), dtype=np.float64))

    # -- Steps 4.1-4.3 --------------------------------------------------------
    def laplace(self, eta, phi_s, h=None, phi_guess=None):
        h = self.h if h is None else h
        G, _, _ = geo.factors(self.mesh, eta, h, self.xh)
        if self.solver == "dense":
            A = op.assemble_dense(self.mesh, G)
            return sv.solve_dense(self.mesh, A, phi_s)
        phi, info = sv.solve_cg(self.mesh, G, phi_s, x0=phi_guess, rtol=self.rtol, dofs=self.dofs,
                                return_info=True)
        self.last_iters.append(info["iters"])
        return phi

    # -- one RK stage (Steps 4.1-4.6) -----------------------------------------
    def stage(self, eta, phi_s, h=None, phi_guess=None):
        h = self.h if h is None else h
        if self.linear:
            flat = np.zeros_like(np.asarray(eta))
            phi = self.laplace(flat, phi_s, h, phi_guess)
            w = sf.w_surface(self.mesh, phi, flat, h, self.xh)
            return w, -self.g * np.asarray(eta), phi, w
        phi = self.laplace(eta, phi_s, h, phi_guess)
        w = sf.w_surface(self.mesh, phi, eta, h, self.xh)
        if self.nq:
            deta, dphi = sf.free_surface_rhs_consistent(self.mesh, eta, phi_s, w, self.g, self.nq,
                                                        quad=self.quad, mass=self.mass_c)
        else:
            deta, dphi = sf.free_surface_rhs(self.mesh, eta, phi_s, w, self.g, metrics=self.metrics)
        return deta, dphi, phi, w

    def relax_apply(self, eta, phi_s, t):
        if self.relax is None:
            return eta, phi_s
        cr, ec, es, pc, ps = self.relax
        r = ramp(t, self.t_ramp)
        c, s = math.cos(self.omega_relax * t), math.sin(self.omega_relax * t)
        eta_t = r * (ec * c + es * s)
        phi_t = r * (pc * c + ps * s)
        return (1.0 - cr) * eta + cr * eta_t, (1.0 - cr) * phi_s + cr * phi_t

    def rk4_step(self, eta, phi_s, t, dt, h=None, tape=None):
        """One ERK4 step followed by relaxation at t + dt."""
        h = self.h if h is None else h
        acc_e = 0.0
        acc_p = 0.0
        ke = kp = None
        for s in range(4):
            if s == 0:
                ye, yp = eta, phi_s
            else:
                ye = eta + RK4_C[s] * dt * ke
                yp = phi_s + RK4_C[s] * dt * kp
            guess = None if self.phi is None else self.phi
            ke, kp, phi, _ = self.stage(ye, yp, h, guess)
            if np.isrealobj(phi):
                self.phi = phi
            if tape is not None:
                tape.append(phi)
            acc_e = acc_e + RK4_B[s] * dt * ke
            acc_p = acc_p + RK4_B[s] * dt * kp
        eta1, phi1 = self.relax_apply(eta + acc_e, phi_s + acc_p, t + dt)
        if self.modal_filter is not None:
            eta1 = mfl.modal_filter(self.mesh, eta1, *self.modal_filter)
            phi1 = mfl.modal_filter(self.mesh, phi1, *self.modal_filter)
        return eta1, phi1

    def run(self, nsteps=None, dt=None, eta=None, phi_s=None, h=None, callback=None):
        nsteps = self.wl.nsteps if nsteps is None else nsteps
        dt = self.wl.dt if dt is None else dt
        if eta is None:
            eta, phi_s = self.initial_state()
        t = 0.0
        if callback is not None:
            callback(0, t, eta, phi_s)
        for n in range(nsteps):
            eta, phi_s = self.rk4_step(eta, phi_s, t, dt, h)
            t += dt
            if callback is not None:
                callback(n + 1, t, eta, phi_s)
        return eta, phi_s

    # -- diagnostics ------------------------------------------------------------
    def mass(self, eta):
        return float(self.ms @ eta)

    def energy(self, eta, phi_s, h=None):
        h = self.h if h is None else h
        G, _, _ = geo.factors(self.mesh, eta, h, self.xh)
        phi = self.laplace(eta, phi_s, h)
        kin = 0.5 * phi @ op.apply(self.mesh, G, phi, self.dofs)
        pot = 0.5 * self.g * (self.ms @ (eta * eta))
        return float(np.real(kin + pot))


def gauge_matrix(mesh, points, xh=None):
    """Surface Lagrange interpolation P with (P f)_g = f(point_g) (axis-aligned quads / intervals)."""
    p, n1 = mesh.p, mesh.p + 1
    if xh is None:
        xh = geo.horizontal_coords(mesh)
    P = np.zeros((len(points), mesh.n_s))
    for g, pt in enumerate(points):
        pt = np.atleast_1d(pt)
        for e in range(mesh.n_eh):
            c = mesh.eh_corner[e]
            lo = c.min(0)
            hi = c.max(0)
            if np.all(pt >= lo - 1e-12) and np.all(pt <= hi + 1e-12):
                ref = 2.0 * (pt - lo) / (hi - lo) - 1.0
                Li = lagrange_eval(p, ref[0])[0]
                if mesh.dim == 3:
                    Lj = lagrange_eval(p, ref[1])[0]
                    wts = (Lj[:, None] * Li[None, :]).ravel()
                else:
                    wts = Li
                P[g, :] = 0.0
                np.add.at(P[g], mesh.eh_nodes[e], wts)
                break
        else:
            raise ValueError(f"gauge {pt} outside the mesh")
    return P


def gauge_loss(model, P, obs, nsteps, dt, eta0, phi0, h):
    """J = 1/2 sum_n sum_g (P eta^n - d^n_g)^2 over steps n = 1..nsteps."""
    eta, phi_s = eta0, phi0
    t = 0.0
    J = 0.0
    for n in range(nsteps):
        eta, phi_s = model.rk4_step(eta, phi_s, t, dt, h)
        t += dt
        r = P @ eta - obs[n]
        J = J + 0.5 * (r @ r)
    return J


def gauge_series(model, P, nsteps, dt, eta0, phi0, h):
    eta, phi_s = eta0, phi0
    t = 0.0
    out = []
    for n in range(nsteps):
        eta, phi_s = model.rk4_step(eta, phi_s, t, dt, h)
        t += dt
        out.append(P @ eta)
    return np.array(out)


def complex_step_derivative(model, P, obs, nsteps, dt, eta0, phi0, h, d_eta0, d_h, eps=1e-30):
    """Directional derivative dJ[d_eta0, d_h] by the complex step."""
    saved = model.phi
    model.phi = None
    Jc = gauge_loss(model, P, obs, nsteps, dt, eta0 + 1j * eps * d_eta0, phi0.astype(np.complex128),
                    h + 1j * eps * d_h)
    model.phi = saved
    return float(np.imag(Jc) / eps)
