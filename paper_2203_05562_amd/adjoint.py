"""Differentiable column runs: a torch.autograd.Function over ulppm_step with
checkpoints every k steps and recomputation between them, reversed by the
library's hand-written adjoint (ulppm_adjoint_step, ulppm_adjoint_init).

The differentiable inputs are the critical-state parameters theta = (M,
lambda~, kappa~, eta) of Section 3.2.1, the suction field s (constant in time)
and the initial velocity v0; the output is the displacement u^N after N
explicit steps (Algorithm 2) from the initial conditions that ulppm_init_state
builds.  Families and sub-horizons are frozen per step in the reverse sweep,
so the gradient is that of the piecewise-smooth map on the forward run's sets.

Memory: one point state per checkpoint (and the final state) plus k states
of the segment being reversed (about 190 bytes per point each), all on the
device.  Each reverse step is handed the recomputed state n+1 as well, so
the library rebuilds only positions and families instead of re-running the
step.

A mixed-precision forward is reversed about the mixed run's own states (the
recomputed segment is mixed as well, so it reproduces them), in FP64 by
default, or with reverse_precision = ULPPM_MIXED with the two
membership-matrix sweeps of each reverse step on FP32 matrix cores.
"""
from typing import Optional, Sequence

import numpy as np
import torch

from . import ulppm

THETA = ("M", "lam", "kap", "eta")


class _Clock:
    """Per-phase device time of the backward sweep (events on the current
    stream, which is the one the library was created on)."""

    def __init__(self, on: bool):
        self.on = on
        self.marks = {}

    def start(self, k):
        if self.on:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.marks.setdefault(k, []).append([e, None])

    def stop(self, k):
        if self.on:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.marks[k][-1][1] = e

    def totals(self):
        if not self.on:
            return None
        torch.cuda.synchronize()
        return {k: sum(a.elapsed_time(b) for a, b in v) for k, v in self.marks.items()}


class ColumnSpec:
    """Everything about a column run that is not differentiated: the
    as-built point data (positions, volumes, porosity, total stress, fixed
    base), the remaining material constants, the over-consolidation ratio,
    dt, the number of steps, the checkpoint interval and the forward
    precision.  Holds one library context with its adjoint scratch."""

    def __init__(self, col: dict, n_steps: int, checkpoint_every: int, dt: Optional[float] = None,
                 precision: int = ulppm.ULPPM_FP64, device="cuda", ctx: Optional["ulppm.Context"] = None,
                 history: int = ulppm.ULPPM_HISTORY_POINT, max_family: int = 0,
                 reverse_precision: int = ulppm.ULPPM_FP64):
        if n_steps < 0 or checkpoint_every < 1:
            raise ValueError("n_steps >= 0 and checkpoint_every >= 1 required")
        self.n = col["n"]
        self.params = dict(col["params"])
        self.ocr = float(col["params"]["ocr"])
        self.n_steps = int(n_steps)
        self.k = int(checkpoint_every)
        self.precision = precision
        self.reverse_precision = int(reverse_precision)
        self.history = int(history)
        self.device = torch.device(device)
        self.base = ulppm.column_state(col, device)        # pre-initialisation state
        self.ctx = ctx if ctx is not None else ulppm.Context(self.n, max_family=max_family)
        if self.history == ulppm.ULPPM_HISTORY_BOND:
            self.ctx.history_reserve()
        self.ctx.adjoint_reserve()
        if dt is None:
            S = self.base.clone()
            p = ulppm.make_params(self.params)
            self.ctx.init_state(S, p, self.ocr)
            dt = 0.5 * self.ctx.dt_crit(S, p)
        self.dt = float(dt)
        self.last_forward = None
        self.last_backward = None
        self.timing = False       # when set, backward records its phase times
        self.last_timing = None

    def theta0(self):
        return torch.tensor([self.params[k] for k in THETA], dtype=torch.float64)

    def params_for(self, theta, precision=None):
        d = dict(self.params)
        for k, v in zip(THETA, [float(t) for t in theta]):
            d[k] = v
        d["dt"] = self.dt
        d["history"] = self.history
        return ulppm.make_params(d, precision=self.precision if precision is None else precision)

    def initial_state(self, theta, s, v0):
        S = self.base.clone()
        S.t["s"].copy_(s)
        S.t["v"].copy_(v0.t())
        self.ctx.init_state(S, self.params_for(theta), self.ocr)
        return S


class ColumnRun(torch.autograd.Function):
    """u^N = ColumnRun.apply(theta, s, v0, spec): theta (4,) float64 on any
    device, s (n,) and v0 (n, 3) float64 on the spec's device.  Returns u^N as
    an (n, 3) float64 device tensor.  Backward: per segment from the last,
    recompute the segment's states from its checkpoint, then reverse its steps
    one by one; finally reverse the initial conditions.  With the history on
    the bonds each checkpoint also keeps the bond states and their families,
    a recomputed segment starts from them, and the reverse carries their
    adjoints from step to step."""

    @staticmethod
    def forward(ctx, theta, s, v0, spec):
        th = theta.detach().cpu()
        S = spec.initial_state(th, s.detach(), v0.detach())
        p = spec.params_for(th)
        bond = spec.history == ulppm.ULPPM_HISTORY_BOND
        ckpts = [S.snapshot()]
        hists = [None]                                     # init_state leaves no bond states
        reps = []
        done = 0
        while done < spec.n_steps:
            m = min(spec.k, spec.n_steps - done)
            reps.append(spec.ctx.step(S, p, m))
            done += m
            ckpts.append(S.snapshot())
            hists.append(spec.ctx.history_export() if bond else None)
        ctx.spec = spec
        ctx.theta = th
        ctx.ckpts = ckpts
        ctx.hists = hists
        ctx.theta_device = theta.device
        spec.last_forward = reps
        return S.t["u"].t().clone()

    @staticmethod
    def backward(ctx, gu):
        spec = ctx.spec
        p = spec.params_for(ctx.theta)
        p64 = spec.params_for(ctx.theta, precision=spec.reverse_precision)
        lam = ulppm.DeviceState(spec.n, spec.device)
        lam.t["u"].copy_(gu.t())
        tb = torch.zeros(4, dtype=torch.float64, device=spec.device)
        reps = []
        clock = _Clock(spec.timing)
        bond = spec.history == ulppm.ULPPM_HISTORY_BOND
        hbar = None
        if bond and spec.n_steps > 0:                      # nothing depends on the final bond states
            hbar = torch.zeros_like(ctx.hists[-1][2])
        starts = list(range(0, spec.n_steps, spec.k))
        for seg in range(len(starts) - 1, -1, -1):
            m = min(spec.k, spec.n_steps - starts[seg])
            clock.start("recompute")
            states = [ctx.ckpts[seg]]
            hists = [ctx.hists[seg]]
            S = ctx.ckpts[seg].snapshot()
            if bond:
                spec.ctx.history_import(ctx.hists[seg])
            for _ in range(m - 1):
                spec.ctx.step(S, p, 1)
                states.append(S.snapshot())
                if bond:
                    hists.append(spec.ctx.history_export())
            clock.stop("recompute")
            clock.start("reverse")
            states.append(ctx.ckpts[seg + 1])
            for n in range(m - 1, -1, -1):
                if bond:
                    hbar, rep = spec.ctx.adjoint_step_bond_history(states[n], states[n + 1], p64, hists[n], hbar,
                                                                   lam, lam, tb)
                    reps.append(rep)
                else:
                    reps.append(spec.ctx.adjoint_step(states[n], p64, lam, lam, tb, S1=states[n + 1]))
            clock.stop("reverse")
            del states, S
        sbar = torch.empty(spec.n, dtype=torch.float64, device=spec.device)
        spec.ctx.adjoint_init(ctx.ckpts[0], p64, spec.ocr, lam, sbar, tb)
        spec.last_backward = reps
        spec.last_timing = clock.totals()
        gv = lam.t["v"].t().clone()
        return tb.to(ctx.theta_device), sbar, gv, None


def runout_settlement(u, x0, top: Sequence[int], axis, tau: float):
    """Objective of the differentiable column: a smooth maximum (scale tau)
    of the points' horizontal distances from the column axis, the final
    runout, plus the settlement of the initial top layer (its mean initial
    height minus its mean final height).  u, x0: (n, 3) tensors."""
    x = x0 + u
    ax = torch.as_tensor(np.asarray(axis, dtype=np.float64), device=x.device)
    r = torch.sqrt((x[:, 0] - ax[0]) ** 2 + (x[:, 1] - ax[1]) ** 2)
    runout = tau * torch.logsumexp(r / tau, dim=0)
    top = torch.as_tensor(np.asarray(top, dtype=np.int64), device=x.device)
    settle = x0[top, 2].mean() - x[top, 2].mean()
    return runout + settle
