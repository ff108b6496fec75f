"""torch.autograd.Function over N ERK4 steps of the library, with sqrt(N) step checkpointing.

Forward: N calls of fnpf_rk4_step from (eta0, phi0) with depth h; returns the surface
elevation after every step, traj[n] = eta^{n+1} (shape [N, n_s]).  It keeps either the tape of
every step (fnpf_rk4_step tape: stage potentials and stage states; 4 (n_v + 2 n_s) doubles per
step), when checkpoint_every is 0 or, by default, when all N tapes take at most a quarter of the
free device memory; or only the state at every S-th step (S = checkpoint_every, by default
ceil(sqrt(N))).

Backward: fnpf_rk4_step_vjp runs each step's stages in reverse (adjoint solves with the same SPD
operator, geometry VJP) from its tape, the steps in reverse order; with checkpoints, each segment
is first recomputed from its checkpoint with tapes.  The adjoint of the trajectory enters as
ybar_eta += dL/d eta^{n}.  Gradients are returned for eta0, phi0 and h.

All numerical work is in the HIP library; this module orders the calls.
"""

from __future__ import annotations

import math

import torch

from . import fnpf


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(actx, eta0, phi0, h, fctx, t0, dt, nsteps, opts, adj_opts, every):
        e = eta0.detach().clone().contiguous()
        p = phi0.detach().clone().contiguous()
        hd = h.detach().contiguous()
        taping = any(actx.needs_input_grad[:3])     # False: neither tapes nor checkpoints
        if taping and every is None:
            need = nsteps * 4 * fctx.tape_record * 8
            free, _ = torch.cuda.mem_get_info(e.device)
            every = 0 if need <= free // 4 else max(1, int(math.ceil(math.sqrt(nsteps))))
        if taping and every > 0:
            every = min(every, max(nsteps, 1))      # one segment from step 0 at most
        traj = torch.empty((nsteps, fctx.n_s), dtype=torch.float64, device=e.device)
        checkpoints, tapes = {}, []
        fctx.set_warm_start(None)
        if getattr(fctx, "linear", False):
            fctx.set_linear(True)       # the depth may have changed in place since the last call
        t = t0
        for n in range(nsteps):
            tape = None
            if taping and every == 0:
                tape = fctx.new_tape()
                tapes.append((tape, t))
            elif taping and n % every == 0:
                checkpoints[n] = (e.clone(), p.clone(), t)
            fctx.rk4_step(e, p, hd, t, dt, opts=opts, tape=tape)
            traj[n] = e
            t = t0 + (n + 1) * dt
        actx.fctx, actx.dt, actx.nsteps, actx.opts, actx.adj_opts, actx.every = fctx, dt, nsteps, opts, adj_opts, every
        if taping and every > 0 and nsteps > 0 and 0 not in checkpoints:
            raise RuntimeError("rollout: step 0 was not checkpointed")
        actx.checkpoints, actx.tapes = checkpoints, tapes
        actx.save_for_backward(hd)
        return traj

    @staticmethod
    def backward(actx, gtraj):
        (hd,) = actx.saved_tensors
        fctx, dt, N, every = actx.fctx, actx.dt, actx.nsteps, actx.every
        gtraj = gtraj.contiguous()
        eb = torch.zeros(fctx.n_s, dtype=torch.float64, device=hd.device)
        pb = torch.zeros_like(eb)
        hb = torch.zeros_like(eb)
        if every == 0:
            for k in range(N - 1, -1, -1):
                eb += gtraj[k]
                tape, tk = actx.tapes[k]
                fctx.rk4_step_vjp(hd, tk, dt, tape, eb, pb, hb, opts=actx.adj_opts)
            actx.tapes = None
            return eb, pb, hb, None, None, None, None, None, None, None
        starts = sorted(actx.checkpoints)
        for s0 in reversed(starts):
            s1 = min(s0 + every, N)
            e, p, t = actx.checkpoints[s0]
            e, p = e.clone(), p.clone()
            fctx.set_warm_start(None)
            tapes, times = [], []
            for n in range(s0, s1):
                tape = fctx.new_tape()
                times.append(t)
                fctx.rk4_step(e, p, hd, t, dt, opts=actx.opts, tape=tape)
                tapes.append(tape)
                t = t + dt
            for k in range(s1 - 1, s0 - 1, -1):
                eb += gtraj[k]
                fctx.rk4_step_vjp(hd, times[k - s0], dt, tapes[k - s0], eb, pb, hb, opts=actx.adj_opts)
            del tapes
        return eb, pb, hb, None, None, None, None, None, None, None


def rollout(fctx, eta0, phi0, h, t0, dt, nsteps, opts=None, adj_opts=None, checkpoint_every=None):
    """Differentiable trajectory eta^1..eta^N ([N, n_s]) of N ERK4 steps.

    checkpoint_every: None chooses (every tape when they fit in a quarter of the free device
    memory, else sqrt(N) checkpoints); 0 keeps every tape; k > 0 keeps the state every k steps
    (k >= N: one checkpoint at step 0, the whole rollout recomputed in the backward)."""
    if checkpoint_every is not None and int(checkpoint_every) < 0:
        raise ValueError(f"checkpoint_every must be None or >= 0, got {checkpoint_every}")
    opts = opts if opts is not None else fnpf.default_opts()
    adj_opts = adj_opts if adj_opts is not None else opts
    return _Rollout.apply(eta0, phi0, h, fctx, float(t0), float(dt), int(nsteps), opts, adj_opts,
                          None if checkpoint_every is None else int(checkpoint_every))


def gauge_matrix(fctx, points):
    """Dense [n_gauges, n_s] observation matrix P with (P f)_g = f(point_g): the library's
    Lagrange weights (fnpf_surface_interp_weights) placed in a device tensor."""
    node, w = fctx.surface_interp_weights(points)
    P = torch.zeros((node.shape[0], fctx.n_s), dtype=torch.float64, device=fctx.device)
    rows = torch.arange(node.shape[0], device=fctx.device).repeat_interleave(node.shape[1])
    P[rows, torch.as_tensor(node.ravel(), dtype=torch.int64, device=fctx.device)] = torch.as_tensor(
        w.ravel(), dtype=torch.float64, device=fctx.device)
    return P
