"""Named synthetic workloads.

C1  2D vertical slice, linear standing wave, periodic L=2, h=1 (kh=pi), 8x2 elements, p=4.
C2  3D periodic 40x40x4 hexes, p=5, h=1, kh=1, a=0.05/k, linear-theory surface potential.
C3  Bottom-mounted cylinder R=0.25 in a 10x5 tank (O-grid 48x24 + jittered Cartesian block), 4 layers, p=4.
C4  Submerged bar 38x1, 64x16x4 hexes, p=5, wave T=2.02 s, H=0.02 m, 8 gauges, 64 bathymetry controls.
C5  256x128x6 hexes, p=6, periodic in y, walls in x, Fourier bathymetry, JONSWAP sea (128 components).
P1  The paper's profiling shape as hexes: periodic 64x64x4, p=4 (1,114,112 DoF, Table 2 mesh 1).

Only input data lives here; see each field's docstring in ``Workload``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .mesh import HexMesh, cylinder_tank_mesh, renumber_blocked, structured_box, structured_slice
from . import waves

G_STD = 9.81


def _zero(x, y):
    return np.zeros_like(np.asarray(x, dtype=np.float64))


@dataclass
class Workload:
    name: str
    mesh: HexMesh
    g: float
    dt: float
    nsteps: int
    eta0: Callable            # (x, y) -> initial surface elevation
    phi0: Callable            # (x, y) -> initial surface potential
    depth: Callable           # (x, y) -> still-water depth h
    rtol: float = 1e-8
    relax_cr: Optional[Callable] = None     # (x, y) -> relaxation weight C_r in [0, 1]
    relax_gen: Optional[Callable] = None    # (x, y) -> True inside the generation zone
    relax_wave: Optional[object] = None     # LinearWave prescribed in the generation zone
    t_ramp: float = 0.0                     # generation ramp duration (five periods)
    meta: dict = field(default_factory=dict)

    def relaxation_arrays(self, x, y):
        """(C_r, eta_c, eta_s, phi_c, phi_s) at the given nodes, or None."""
        if self.relax_cr is None:
            return None
        cr = self.relax_cr(x, y)
        gen = self.relax_gen(x, y).astype(np.float64)
        ec, es, pc, ps = self.relax_wave.split(x, y)
        return cr, gen * ec, gen * es, gen * pc, gen * ps


def parity_start(wl: Workload):
    """(t0, eta0, phi0) of the full-size two-step parity runs.  C2 starts from its own wave at
    t = 0; the tanks with relaxation zones (C3, C4) start from their incident linear wave over the
    whole domain at t = t_ramp, when generation is fully ramped in, so that every stage solves a
    nonzero problem and both zones act on the state."""
    if wl.relax_wave is None:
        return 0.0, wl.eta0, wl.phi0
    t0, wave = wl.t_ramp, wl.relax_wave
    return t0, (lambda x, y: wave.eta(x, y, t0)), (lambda x, y: wave.phi(x, y, t0))


def c1() -> Workload:
    g = G_STD
    k, h = math.pi, 1.0
    mesh = structured_slice(8, 0.0, 2.0, True, p=4, nz=2, name="C1")
    omega = waves.frequency(k, h, g)
    period = 2 * math.pi / omega
    return Workload(name="C1", mesh=mesh, g=g, dt=period / 32, nsteps=32,
                    eta0=lambda x, y: 1e-3 * np.cos(math.pi * np.asarray(x)), phi0=_zero,
                    depth=lambda x, y: np.ones_like(np.asarray(x, dtype=np.float64)), rtol=1e-12,
                    meta=dict(k=k, h=h, omega=omega, period=period, amp=1e-3))


def c2(n: int = 40, nz: int = 4, p: int = 5) -> Workload:
    g = G_STD
    k, h = 1.0, 1.0
    a = 0.05 / k
    L = 2 * math.pi / k
    mesh = renumber_blocked(structured_box(n, n, 0.0, L, 0.0, L, True, True, p=p, nz=nz, name="C2"),
                            shared_first=True)
    omega = waves.frequency(k, h, g)
    period = 2 * math.pi / omega
    wave = waves.LinearWave(a, k, 0.0, omega, g)
    return Workload(name="C2", mesh=mesh, g=g, dt=period / 64, nsteps=50,
                    eta0=lambda x, y: wave.eta(x, y), phi0=lambda x, y: wave.phi(x, y),
                    depth=lambda x, y: np.ones_like(np.asarray(x, dtype=np.float64)), rtol=1e-8,
                    meta=dict(k=k, h=h, a=a, omega=omega, period=period))


def c3(p: int = 4, nz: int = 4, seed: int = 0) -> Workload:
    g = G_STD
    h = 1.0
    k = 1.0 / h
    L = 2 * math.pi / k
    H = 0.02 * L
    mesh = renumber_blocked(cylinder_tank_mesh(p=p, nz=nz, seed=seed), shared_first=True)
    omega = waves.frequency(k, h, g)
    period = 2 * math.pi / omega
    wave = waves.LinearWave(H / 2, k, 0.0, omega, g)
    lx = mesh.extra["tank"][0]

    def cr(x, y):
        x = np.asarray(x, dtype=np.float64)
        return np.maximum(waves.relax_weight((2.0 - x) / 2.0) * (x < 2.0),
                          waves.relax_weight((x - (lx - 2.0)) / 2.0) * (x > lx - 2.0))

    return Workload(name="C3", mesh=mesh, g=g, dt=period / 80, nsteps=50, eta0=_zero, phi0=_zero,
                    depth=lambda x, y: np.full_like(np.asarray(x, dtype=np.float64), h), rtol=1e-8,
                    relax_cr=cr, relax_gen=lambda x, y: np.asarray(x) < 2.0, relax_wave=wave,
                    t_ramp=5 * period, meta=dict(k=k, h=h, H=H, omega=omega, period=period))


BAR_GAUGES_X = (10.0, 13.0, 16.0, 19.0, 21.0, 23.0, 26.0, 29.0)


def c4(nx: int = 64, ny: int = 16, nz: int = 4, p: int = 5, nsteps: int = 200, lx: float = 38.0,
       ly: float = 1.0, n_ctrl: int = 64) -> Workload:
    g = G_STD
    period = 2.02
    H = 0.02
    omega = 2 * math.pi / period
    h_deep = 0.4
    k = waves.wavenumber(omega, h_deep, g)
    mesh = renumber_blocked(structured_box(nx, ny, 0.0, lx, 0.0, ly, False, False, p=p, nz=nz, name="C4"),
                            shared_first=True)
    xc = waves.control_points(lx, n_ctrl)
    c0 = waves.bar_profile(xc)
    wave = waves.LinearWave(H / 2, k, 0.0, omega, g)
    gen_w, abs_w = 8.0 * lx / 38.0, 8.0 * lx / 38.0

    def depth(x, y, c=c0):
        return waves.piecewise_linear_matrix(np.asarray(x).ravel(), xc) @ c

    def cr(x, y):
        x = np.asarray(x, dtype=np.float64)
        return np.maximum(waves.relax_weight((gen_w - x) / gen_w) * (x < gen_w),
                          waves.relax_weight((x - (lx - abs_w)) / abs_w) * (x > lx - abs_w))

    rng = np.random.default_rng(1)
    c_true = c0 + 0.01 * rng.standard_normal(n_ctrl)
    gauges = np.array([[gx * lx / 38.0, 0.5 * ly] for gx in BAR_GAUGES_X])
    return Workload(name="C4", mesh=mesh, g=g, dt=period / 64, nsteps=nsteps, eta0=_zero, phi0=_zero,
                    depth=depth, rtol=1e-8, relax_cr=cr, relax_gen=lambda x, y: np.asarray(x) < gen_w,
                    relax_wave=wave, t_ramp=5 * period,
                    meta=dict(k=k, h=h_deep, H=H, omega=omega, period=period, xc=xc, c0=c0, c_true=c_true,
                              gauges=gauges, fd_seed=3))


def c5(nx: int = 256, ny: int = 128, nz: int = 6, p: int = 6, nsteps: int = 20) -> Workload:
    g = G_STD
    kp, h_mean = 2.0, 1.0
    lp = 2 * math.pi / kp
    lx, ly = 32 * lp * nx / 256, 16 * lp * ny / 128
    mesh = renumber_blocked(structured_box(nx, ny, 0.0, lx, 0.0, ly, False, True, p=p, nz=nz, name="C5"),
                            shared_first=True)
    omega_p = waves.frequency(kp, h_mean, g)
    tp = 2 * math.pi / omega_p
    bathy = waves.FourierBathymetry(lx, ly, h0=1.0, rel=0.2, seed=2)
    amp, w, ph = waves.jonswap_components(0.03 * lp, omega_p, 128, seed=4)
    sea = waves.IrregularSea(amp, w, ph, h_mean, g)
    return Workload(name="C5", mesh=mesh, g=g, dt=tp / 32, nsteps=nsteps, eta0=sea.eta, phi0=sea.phi,
                    depth=bathy, rtol=1e-8, meta=dict(kp=kp, omega_p=omega_p, period=tp, lp=lp))


def p1() -> Workload:
    g = G_STD
    L, h = 1.0, 1.0
    k = 2 * math.pi / L
    mesh = renumber_blocked(structured_box(64, 64, 0.0, L, 0.0, L, True, True, p=4, nz=4, name="P1"), shared_first=True)
    omega = waves.frequency(k, h, g)
    period = 2 * math.pi / omega
    wave = waves.LinearWave(0.01 / k, k, 0.0, omega, g)
    return Workload(name="P1", mesh=mesh, g=g, dt=period / 32, nsteps=10, eta0=wave.eta, phi0=wave.phi,
                    depth=lambda x, y: np.ones_like(np.asarray(x, dtype=np.float64)), rtol=1e-8,
                    meta=dict(k=k, h=h, omega=omega, period=period))


def small_box(nx=4, ny=3, nz=2, p=3, periodic=(True, False), seed=7, wavy=0.05, lx=2.0, ly=1.5,
              name="small") -> Workload:
    """Small 3D case with a seeded wavy surface and bottom (parity tests)."""
    g = G_STD
    mesh = structured_box(nx, ny, 0.0, lx, 0.0, ly, periodic[0], periodic[1], p=p, nz=nz, name=name)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 4)
    kx, ky = 2 * math.pi / lx, 2 * math.pi / ly

    def eta(x, y):
        return wavy * (np.cos(kx * np.asarray(x) + ph[0]) * np.cos(ky * np.asarray(y) + ph[1]))

    def phi(x, y):
        return 0.3 * np.sin(kx * np.asarray(x) + ph[2]) + 0.1 * np.cos(ky * np.asarray(y) + ph[3])

    def depth(x, y):
        return 1.0 + 0.1 * np.sin(kx * np.asarray(x) + ph[1]) * np.cos(ky * np.asarray(y))

    return Workload(name=name, mesh=mesh, g=g, dt=0.02, nsteps=2, eta0=eta, phi0=phi, depth=depth, rtol=1e-12)


def small_slice(nx=5, nz=3, p=4, periodic=True, seed=5, wavy=0.05, lx=2.0, name="small_slice") -> Workload:
    g = G_STD
    mesh = structured_slice(nx, 0.0, lx, periodic, p=p, nz=nz, name=name)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 3)
    kx = 2 * math.pi / lx
    return Workload(name=name, mesh=mesh, g=g, dt=0.02, nsteps=2,
                    eta0=lambda x, y: wavy * np.cos(kx * np.asarray(x) + ph[0]),
                    phi0=lambda x, y: 0.2 * np.sin(kx * np.asarray(x) + ph[1]),
                    depth=lambda x, y: 1.0 + 0.1 * np.cos(kx * np.asarray(x) + ph[2]), rtol=1e-12)


ALL = dict(C1=c1, C2=c2, C3=c3, C4=c4, C5=c5, P1=p1)
