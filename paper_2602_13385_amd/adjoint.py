"""Differentiable SCF trajectories: a torch.autograd.Function over scf_step and
scf_step_adjoint with recomputation from checkpoints.

The forward pass integrates nsteps leapfrog steps in segments of `checkpoint`
steps, keeping each segment's starting state (particles on the device, frame
centre on the host) and the force weights of every kick (one row of
(nmax + 1)(lmax + 1)^2 values per step, scf_step_keep_weights).  The backward
pass walks the segments in reverse; scf_step_adjoint recomputes a segment's
positions on the device from its checkpoint and the kept weights (no
coefficient passes) and returns the cotangents of its starting state, its
starting centre and the host-potential parameters.  Differentiable inputs: the initial particle state,
the host parameters p[] of every component, and the initial centre (R0, V0).

The stream-track loss of the adjoint workload (escapers' distance to a target
track, escaper set and nearest track points frozen at the base trajectory)
is provided as plain torch arithmetic on the trajectory's outputs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import scf


class SCFTrajectory(torch.autograd.Function):
    """outputs (state_T (6, n) device, centre_T (6,) double CPU) of
    (state_0 (6, n) device, theta (ncomp, 3) double CPU, centre_0 (6,) double CPU)."""

    @staticmethod
    def forward(ctx, state0, theta, centre0, plan, m, kinds, G, dt, nsteps, checkpoint):
        n = state0.shape[1]
        host = None
        if kinds:
            host = (list(zip(kinds, theta.detach().cpu().numpy().tolist())), G)
        st = [state0[i].detach().clone().contiguous() for i in range(6)]
        cen = centre0.detach().cpu().numpy().astype(np.float64)
        wsz = plan.weights_size
        # row j: the force weights of the kick at step j (a segment's first row
        # is rewritten, with the same values, by the next segment's start-up)
        hist = torch.empty((nsteps + 1) * wsz, dtype=st[0].dtype, device=st[0].device)
        segs = []
        done = 0
        while done < nsteps:
            k = min(checkpoint, nsteps - done)
            segs.append((torch.stack([t.clone() for t in st]), cen.copy(), k, done))
            cen, _ = plan.step(st, m, dt, k, host=host, centre=cen, w_hist=hist[done * wsz:])
            done += k
        ctx.plan, ctx.m, ctx.host, ctx.dt, ctx.segs = plan, m, host, dt, segs
        ctx.hist, ctx.wsz = hist, wsz
        ctx.ncomp = theta.shape[0]
        out = torch.stack(st)
        del n
        return out, torch.as_tensor(cen, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g_state, g_centre):
        plan = ctx.plan
        if g_state is None:
            g_state = torch.zeros_like(ctx.segs[0][0]) if ctx.segs else None
        lam = [g_state[i].detach().clone().contiguous() for i in range(6)]
        lc = (g_centre.detach().cpu().numpy().astype(np.float64) if g_centre is not None
              else np.zeros(6))
        gtheta = np.zeros((ctx.ncomp, 3))
        for st0, cen0, k, start in reversed(ctx.segs):
            st0l = [st0[i].contiguous() for i in range(6)]
            lc, gh = plan.step_adjoint(st0l, ctx.m, ctx.dt, k, lam, lc, host=ctx.host,
                                       centre0=cen0, w_hist=ctx.hist[start * ctx.wsz:])
            if gh.size:
                gtheta += gh
        return (torch.stack(lam), torch.as_tensor(gtheta, dtype=torch.float64),
                torch.as_tensor(lc, dtype=torch.float64), None, None, None, None, None, None, None)


def trajectory(plan, state0, m, theta, centre0, kinds, dt, nsteps, checkpoint=100, G=1.0):
    """Differentiable wrapper: see SCFTrajectory."""
    return SCFTrajectory.apply(state0, theta, centre0, plan, m, list(kinds), G, dt, nsteps,
                               checkpoint)


def escaped_mask(plan, state, m):
    """Escapers in the cluster frame, 1/2 |v|^2 + psi_SCF(x) >= 0 (not
    differentiated): the library's bound test (scf_select)."""
    with torch.no_grad():
        return plan.escaped([state[i].contiguous() for i in range(6)], m)


def nearest_track_points(state, centre, track, mask):
    """Index of the nearest track point for every escaper (frozen)."""
    with torch.no_grad():
        pos = (state[:3].double().T + torch.as_tensor(centre[:3], device=state.device,
                                                       dtype=torch.float64))
        tr = torch.as_tensor(track, device=state.device, dtype=torch.float64)
        sel = pos[mask]
        if sel.shape[0] == 0:
            return torch.zeros(0, dtype=torch.long, device=state.device)
        d = torch.cdist(sel, tr)
        return d.argmin(dim=1)


def track_loss(state, centre, track, mask, idx):
    """L = sum over escapers of |R + x_i - t_j(i)|^2 (mask and idx frozen)."""
    tr = torch.as_tensor(track, device=state.device, dtype=torch.float64)
    R = centre[:3].to(state.device)
    pos = state[:3].double().T + R
    d = pos[mask] - tr[idx]
    return (d * d).sum()
