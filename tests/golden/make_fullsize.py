"""Write tests/golden/fullsize_<C>.npz: two ERK4 steps of the oracle on the full-size C2, C3 and
C4 meshes (Sec. 3.4 Steps 4.1-4.7 per stage, Sec. 3.2 ERK4, Sec. 3.3 relaxation after each step).

The oracle runs its Jacobi-PCG to a relative residual of 1e-14 (tighter than the 1e-13 of the
oracle's default, so that the stored states are limited by rounding rather than by the stopping
rule), warm-starting each stage from the previous stage's potential.  Start states and times come
from workloads.configs.parity_start.  Stored per workload:

  t0, dt, rtol                      start time, step, oracle tolerance
  eta1, phis1, eta2, phis2          surface elevation and potential after steps 1 and 2 [n_s]
  w0                                recovered vertical surface velocity of the first stage [n_s]
  phi0_idx, phi0_val, phi0_norm     first-stage volume potential at 8192 seeded node indices,
                                    and its full 2-norm
  iters                             oracle CG iterations per stage solve

This script calls only oracle/ and workloads/.  Usage (takes tens of minutes per workload):
    python tests/golden/make_fullsize.py C2 C3 C4
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import timestep as ts          # noqa: E402
from workloads import configs              # noqa: E402

RTOL = 1e-14
N_SAMPLE = 8192


def make(name: str) -> str:
    wl = configs.ALL[name]()
    t0, fe, fp = configs.parity_start(wl)
    md = ts.Model(wl, solver="cg", rtol=RTOL)
    eta0 = np.asarray(fe(md.x, md.y), dtype=np.float64)
    phis0 = np.asarray(fp(md.x, md.y), dtype=np.float64)
    dt = wl.dt
    t = time.time()
    _, _, phi0, w0 = md.stage(eta0, phis0)
    print(f"[{name}] first stage: {md.last_iters} iterations, {time.time() - t:.0f} s", flush=True)
    md.phi = None
    md.last_iters = []
    e1, p1 = md.rk4_step(eta0, phis0, t0, dt)
    print(f"[{name}] step 1: {md.last_iters} iterations, {time.time() - t:.0f} s", flush=True)
    e2, p2 = md.rk4_step(e1, p1, t0 + dt, dt)
    print(f"[{name}] step 2: {md.last_iters} iterations, {time.time() - t:.0f} s", flush=True)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(wl.mesh.n_v, size=min(N_SAMPLE, wl.mesh.n_v), replace=False)).astype(np.int64)
    out = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(out, t0=t0, dt=dt, rtol=RTOL, eta1=e1, phis1=p1, eta2=e2, phis2=p2, w0=w0,
                        phi0_idx=idx, phi0_val=phi0[idx], phi0_norm=np.linalg.norm(phi0),
                        iters=np.array(md.last_iters, dtype=np.int64))
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["C2", "C3", "C4"]:
        print(make(nm), flush=True)
