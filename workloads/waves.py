"""Analytic wave and bathymetry data for the synthetic workloads.

Linear (small-amplitude) wave theory provides the initial and incident wave
fields (paper Sec. 3.3: initialisation from linear theory given kh); the
JONSWAP-type spectrum and the seeded Fourier bathymetry are synthetic stand-ins
for the paper's irregular-sea and variable-depth cases.  Every function is
evaluated by the caller at its own node coordinates.
"""

from __future__ import annotations

import math

import numpy as np


def wavenumber(omega: float, h: float, g: float) -> float:
    """Solve omega^2 = g k tanh(k h) for k > 0 (Newton from the deep-water guess)."""
    k = max(omega * omega / g, omega / math.sqrt(g * h))
    for _ in range(100):
        t = math.tanh(k * h)
        f = g * k * t - omega * omega
        df = g * t + g * k * h * (1.0 - t * t)
        dk = f / df
        k -= dk
        if abs(dk) < 1e-15 * k:
            break
    return k


def frequency(k: float, h: float, g: float) -> float:
    return math.sqrt(g * k * math.tanh(k * h))


class LinearWave:
    """eta = a cos(kx x + ky y - omega t + th), phi_s = (g a/omega) sin(...) at z = 0."""

    def __init__(self, a, kx, ky, omega, g, th=0.0):
        self.a, self.kx, self.ky, self.omega, self.g, self.th = a, kx, ky, omega, g, th

    def arg(self, x, y, t):
        return self.kx * x + self.ky * y - self.omega * t + self.th

    def eta(self, x, y, t=0.0):
        return self.a * np.cos(self.arg(x, y, t))

    def phi(self, x, y, t=0.0):
        return self.g * self.a / self.omega * np.sin(self.arg(x, y, t))

    def split(self, x, y):
        """(eta_c, eta_s, phi_c, phi_s) with f(t) = f_c cos(omega t) + f_s sin(omega t)."""
        s0 = self.kx * x + self.ky * y + self.th
        c, s = np.cos(s0), np.sin(s0)
        amp_phi = self.g * self.a / self.omega
        # cos(s0 - wt) = cos s0 cos wt + sin s0 sin wt ; sin(s0 - wt) = sin s0 cos wt - cos s0 sin wt
        return self.a * c, self.a * s, amp_phi * s, -amp_phi * c


def relax_weight(s):
    """Smooth 0 -> 1 relaxation weight 0.5 (1 - cos(pi s)) for s in [0, 1]."""
    s = np.clip(s, 0.0, 1.0)
    return 0.5 * (1.0 - np.cos(np.pi * s))


def jonswap_components(hs: float, omega_p: float, n: int, seed: int, gamma: float = 3.3,
                       wmin: float = 0.6, wmax: float = 2.0):
    """Amplitudes, frequencies and phases of a JONSWAP-like long-crested sea.

    S(w) ~ w^-5 exp(-1.25 (wp/w)^4) gamma^exp(-(w-wp)^2 / (2 sigma^2 wp^2)),
    sigma = 0.07 (w <= wp) or 0.09, scaled so that 4 sqrt(m0) = hs; n components
    uniformly spaced in [wmin, wmax] * wp with seeded phases.
    """
    rng = np.random.default_rng(seed)
    w = np.linspace(wmin * omega_p, wmax * omega_p, n)
    dw = w[1] - w[0]
    sig = np.where(w <= omega_p, 0.07, 0.09)
    shape = w ** -5 * np.exp(-1.25 * (omega_p / w) ** 4) * gamma ** np.exp(-((w - omega_p) ** 2) / (2 * sig ** 2 * omega_p ** 2))
    m0 = np.sum(shape) * dw
    scale = (hs / 4.0) ** 2 / m0
    amp = np.sqrt(2.0 * scale * shape * dw)
    phase = rng.uniform(0.0, 2.0 * np.pi, n)
    return amp, w, phase


class IrregularSea:
    """Superposition of long-crested linear components travelling in +x."""

    def __init__(self, amp, omega, phase, h_mean, g):
        self.amp = np.asarray(amp)
        self.omega = np.asarray(omega)
        self.phase = np.asarray(phase)
        self.k = np.array([wavenumber(w, h_mean, g) for w in self.omega])
        self.g = g

    def eta(self, x, y, t=0.0):
        x = np.asarray(x)
        arg = self.k[:, None] * x.reshape(1, -1) - self.omega[:, None] * t + self.phase[:, None]
        return (self.amp[:, None] * np.cos(arg)).sum(0).reshape(x.shape)

    def phi(self, x, y, t=0.0):
        x = np.asarray(x)
        arg = self.k[:, None] * x.reshape(1, -1) - self.omega[:, None] * t + self.phase[:, None]
        c = self.g * self.amp / self.omega
        return (c[:, None] * np.sin(arg)).sum(0).reshape(x.shape)


class FourierBathymetry:
    """h = h0 + rel * S / max|S|, S a sum of seeded Fourier modes, periodic in y.

    max|S| is taken on a fixed 1024 x 512 sampling grid of the domain so that h
    does not depend on the discretisation that later samples it.
    """

    def __init__(self, lx, ly, h0=1.0, rel=0.2, n_modes=16, mx_max=8, my_max=4, seed=2):
        rng = np.random.default_rng(seed)
        modes = []
        while len(modes) < n_modes:
            mx = int(rng.integers(0, mx_max + 1))
            my = int(rng.integers(0, my_max + 1))
            if mx == 0 and my == 0:
                continue
            modes.append((mx, my, float(rng.uniform(0.0, 2.0 * np.pi))))
        self.modes = modes
        self.lx, self.ly, self.h0, self.rel = lx, ly, h0, rel
        xs = np.linspace(0.0, lx, 1024)
        ys = np.linspace(0.0, ly, 512)
        X, Y = np.meshgrid(xs, ys, indexing="ij")
        self.smax = float(np.max(np.abs(self._s(X, Y))))

    def _s(self, x, y):
        s = np.zeros_like(np.asarray(x, dtype=np.float64))
        for mx, my, th in self.modes:
            s = s + np.cos(2 * np.pi * mx * x / self.lx + 2 * np.pi * my * y / self.ly + th)
        return s

    def __call__(self, x, y):
        return self.h0 + self.rel * self._s(x, y) / self.smax


def bar_profile(x, h_deep=0.4, h_crest=0.1, x_up=14.0, x_crest0=20.0, x_crest1=22.0, x_down=25.0):
    """Trapezoidal submerged bar: 1:20 rise over [14, 20], crest to 22, 1:10 fall to 25."""
    x = np.asarray(x, dtype=np.float64)
    h = np.full_like(x, h_deep)
    up = (x > x_up) & (x < x_crest0)
    h[up] = h_deep - (x[up] - x_up) * (h_deep - h_crest) / (x_crest0 - x_up)
    h[(x >= x_crest0) & (x <= x_crest1)] = h_crest
    dn = (x > x_crest1) & (x < x_down)
    h[dn] = h_crest + (x[dn] - x_crest1) * (h_deep - h_crest) / (x_down - x_crest1)
    return h


def control_points(lx: float, n: int = 64):
    return np.arange(n) * lx / (n - 1)


def piecewise_linear_matrix(xq, xc):
    """Matrix B with (B c)(xq) = piecewise-linear interpolation of c at knots xc."""
    xq = np.asarray(xq, dtype=np.float64).ravel()
    n = len(xc)
    idx = np.clip(np.searchsorted(xc, xq, side="right") - 1, 0, n - 2)
    t = (xq - xc[idx]) / (xc[idx + 1] - xc[idx])
    B = np.zeros((len(xq), n))
    B[np.arange(len(xq)), idx] = 1.0 - t
    B[np.arange(len(xq)), idx + 1] = t
    return B
