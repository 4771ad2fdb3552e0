"""Parity of the history carried on the bonds (ULPPM_HISTORY_BOND) between
the HIP library and the CPU oracle.

Bars: the exported bond families bit-exact; point fields and bond states
within 1e-10 relative L2 over 200 steps in FP64, 1e-4 in mixed precision.
"""
import sys

import numpy as np
import pytest

from paper_2203_05562_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_05562_amd import ulppm
    ulppm.load_library()
    return ulppm


def rel_l2(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def history_pair(olib, gpu, dims=(8, 8, 16), seed=0, precision=None, vscale=0.0, max_family=0):
    col = inputs.make_column(inputs.CONFIGS["C0"], seed=seed, dims=dims)
    oprm = olib.make_params(col["params"])
    S = olib.init_column(col, oprm, col["params"]["ocr"])
    if vscale > 0:
        v = inputs.random_velocity(col["n"], seed + 100, vscale)
        v[col["fixed"] == 1] = 0.0
        S["v"][:] = v
    oprm.dt = 0.5 * olib.dt_crit(S, oprm)
    over = dict(history=gpu.ULPPM_HISTORY_BOND)
    if precision is not None:
        over["precision"] = precision
    gprm = gpu.make_params(olib.params_dict(oprm), **over)
    ctx = gpu.Context(col["n"], max_family=max_family)
    ctx.history_reserve()
    G = gpu.DeviceState.from_arrays(S)
    H = olib.BondHistory(col["n"], 200 * col["n"])
    return col, oprm, gprm, S, G, ctx, H


@pytest.mark.parametrize("nsteps,calls,max_family", [(1, 1, 0), (200, 1, 0), (200, 4, 0), (200, 1, 128)])
def test_bond_history_trajectory(olib, gpu, nsteps, calls, max_family):
    """200 steps of the 8 x 8 x 16 column with the history on the bonds, in
    one call or spread over several (the states persist in the context); a
    family capacity of 128 runs the bond kernel's three-wave instance."""
    say("bond history", nsteps, calls, max_family)
    col, oprm, gprm, S, G, ctx, H = history_pair(olib, gpu, seed=0, vscale=0.05, max_family=max_family)
    E = np.zeros(3)
    rc, E, st = olib.step_bond_history(S, oprm, H, nsteps, E)
    assert rc == 0
    rep = None
    for _ in range(calls):
        rep = ctx.step(G, gprm, nsteps // calls)
    Sg = G.to_arrays()
    errs = {k: rel_l2(Sg[k], S[k]) for k in ("u", "v", "a", "sig", "pc", "J")}
    row, colx, st_g = ctx.history_export()
    n = col["n"]
    assert np.array_equal(row.cpu().numpy()[:n + 1], H.row) and np.array_equal(colx.cpu().numpy(), H.col[:H.nb])
    e_st = rel_l2(st_g.cpu().numpy()[:, :7], H.st[:H.nb, :7])
    say(f"{nsteps} steps", {k: f"{v:.2e}" for k, v in errs.items()}, "bond states", f"{e_st:.2e}",
        "plastic", st["n_plastic"], rep["n_plastic"])
    assert all(v <= 1e-10 for v in errs.values()), errs
    assert e_st <= 1e-10


def test_bond_history_differs_from_point_history(olib, gpu):
    """The two history rules give different columns (the point rule resets
    every bond to the point mean each step); both match their oracle."""
    say("bond vs point history")
    col, oprm, gprm, S, G, ctx, H = history_pair(olib, gpu, seed=3)
    Sp = {k: v.copy() for k, v in S.items()}
    rc, _, _ = olib.step_bond_history(S, oprm, H, 100)
    assert rc == 0
    rc, _, _ = olib.step(Sp, oprm, 100)
    assert rc == 0
    ctx.step(G, gprm, 100)
    d = rel_l2(S["sig"], Sp["sig"])
    say("sigma bond vs point", d)
    assert d > 1e-3
    assert rel_l2(G.to_arrays()["sig"], S["sig"]) <= 1e-10


def test_bond_history_mixed(olib, gpu):
    say("bond history mixed")
    col, oprm, gprm, S, G, ctx, H = history_pair(olib, gpu, seed=1, precision=gpu.ULPPM_MIXED)
    rc, _, _ = olib.step_bond_history(S, oprm, H, 200)
    assert rc == 0
    ctx.step(G, gprm, 200)
    Sg = G.to_arrays()
    errs = {k: rel_l2(Sg[k], S[k]) for k in ("u", "v", "sig")}
    say("mixed", errs)
    assert all(v <= 1e-4 for v in errs.values()), errs


def test_bond_history_errors(olib, gpu):
    import torch
    col, oprm, gprm, S, G, ctx, H = history_pair(olib, gpu, dims=(6, 6, 6))
    ctx2 = gpu.Context(col["n"])
    with pytest.raises(gpu.UlppmError) as ei:          # not reserved
        ctx2.step(G, gprm, 1)
    assert ei.value.code == -1
    with pytest.raises(gpu.UlppmError) as ei:          # nothing held yet
        ctx.history_export()
    assert ei.value.code == -1
    ctx.adjoint_reserve()
    A1 = gpu.DeviceState.from_arrays(olib.empty_state(col["n"]))
    A0 = gpu.DeviceState.from_arrays(olib.empty_state(col["n"]))
    with pytest.raises(gpu.UlppmError) as ei:          # the bond history has its own reverse entry point
        ctx.adjoint_step(G, gprm, A1, A0, torch.zeros(4, dtype=torch.float64, device="cuda"))
    assert ei.value.code == -1
    ctx2.adjoint_reserve()                             # no bond states reserved: no scratch for the reverse
    hb = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.UlppmError) as ei:
        ctx2.adjoint_step_bond_history(G, G, gprm, None, hb, A1, A0, torch.zeros(4, dtype=torch.float64,
                                                                                 device="cuda"))
    assert ei.value.code == -1


FIELDS_ADJ = ("u", "uc", "v", "a", "vol", "phi", "J", "Sr", "mass", "s", "sig", "pc")


def test_bond_history_adjoint_matches_dual_numbers(olib, gpu):
    """Gradient of J = sum c . u^N through 8 plastic steps with the history on
    the bonds: the GPU reverse sweep (ulppm_adjoint_step_bond_history, the
    bond states' adjoints carried between steps through the families each
    step exported) dotted with directions in (M, lam, kap, eta), the initial
    velocity, stress, pre-consolidation and suction equals the oracle's
    directional derivatives with the history on the bonds (dual numbers)."""
    import torch
    say("bond history adjoint vs dual")
    nsteps = 8
    col = inputs.make_column(inputs.CONFIGS["C0"], seed=1, dims=(6, 6, 8))
    n = col["n"]
    oprm = olib.make_params(col["params"])
    S = olib.init_column(col, oprm, col["params"]["ocr"])
    oprm.dt = 0.5 * olib.dt_crit(S, oprm)
    rng = np.random.default_rng(2)
    fixed = col["fixed"] == 1
    S["v"][:] = rng.uniform(-0.05, 0.05, S["v"].shape)
    S["v"][fixed] = 0.0
    gprm = gpu.make_params(olib.params_dict(oprm), history=gpu.ULPPM_HISTORY_BOND)
    ctx = gpu.Context(n)
    ctx.history_reserve()
    ctx.adjoint_reserve()
    G = gpu.DeviceState.from_arrays(S)
    states, hists = [G.clone()], [None]
    for _ in range(nsteps):
        ctx.step(G, gprm, 1)
        states.append(G.clone())
        hists.append(ctx.history_export())
    c = rng.normal(size=(n, 3))
    lamN = {k: np.zeros_like(S[k]) for k in FIELDS_ADJ}
    lamN["u"] = c
    lam = gpu.DeviceState.from_arrays({**lamN, "x0": np.zeros((n, 3))})
    hbar = torch.zeros((hists[-1][1].shape[0], 8), dtype=torch.float64, device="cuda")
    th = torch.zeros(4, dtype=torch.float64, device="cuda")
    for k in range(nsteps - 1, -1, -1):
        out = gpu.DeviceState(n)
        hbar, _ = ctx.adjoint_step_bond_history(states[k], states[k + 1], gprm, hists[k], hbar, lam, out, th)
        lam = out
    assert hbar is None                              # the first step carried no bond states
    lam0 = lam.to_arrays()
    th = th.cpu().numpy()
    say("theta_bar", th)
    vin = rng.normal(size=(n, 3))
    vin[fixed] = 0.0
    dirs = {
        "M": (np.array([1.0, 0, 0, 0]), {}),
        "lam": (np.array([0, 1.0, 0, 0]), {}),
        "kap": (np.array([0, 0, 1.0, 0]), {}),
        "eta": (np.array([0, 0, 0, oprm.eta]), {}),
        "v0": (np.zeros(4), {"v": vin}),
        "sig0": (np.zeros(4), {"sig": rng.normal(size=(n, 6)) * 1e3}),
        "pc0": (np.zeros(4), {"pc": rng.normal(size=n) * 1e3}),
        "s": (np.zeros(4), {"s": np.full(n, 1e3)}),
    }
    for name, (dpar, dfields) in dirs.items():
        dS = olib.empty_state(n)
        for k, val in dfields.items():
            dS[k][:] = val
        S1 = olib.copy_state(S)
        H = olib.BondHistory(n, 200 * n)
        rc, _, st = olib.step_dual_bond_history(S1, dS, oprm, dpar, H, nsteps)
        assert rc == 0 and st["n_plastic"] > 0
        dJ = float(np.sum(c * dS["u"]))
        g = float(np.dot(th, dpar))
        for k, val in dfields.items():
            g += float(np.sum(lam0[k] * val))
        say(name, dJ, g)
        assert abs(g - dJ) <= 1e-7 * max(abs(dJ), 1e-300), (name, g, dJ)


def test_bond_history_checkpointed_gradient(olib, gpu):
    """The checkpointed differentiable column with the history on the bonds:
    checkpoints every 1, 4 (ragged last segment) and 10 steps give the same
    gradient (a recomputed segment starts from the bond states its checkpoint
    kept), and its initial-velocity gradient of J = sum c . u^N over 10 steps
    equals the oracle's directional derivative with the history on the bonds."""
    import torch
    from paper_2203_05562_amd import adjoint
    say("bond history, checkpointed gradient")
    col = inputs.make_column(inputs.CONFIGS["C0"], seed=1, dims=(6, 6, 8))
    n = col["n"]
    fixed = col["fixed"] == 1
    rng = np.random.default_rng(4)
    v0 = rng.uniform(-0.05, 0.05, (n, 3))
    v0[fixed] = 0.0
    oprm = olib.make_params(col["params"])
    S = olib.init_column(col, oprm, col["params"]["ocr"], v0)
    dt = 0.5 * olib.dt_crit(S, oprm)
    c = rng.normal(size=(n, 3))

    def grad(k):
        spec = adjoint.ColumnSpec(col, 10, k, dt=dt, history=gpu.ULPPM_HISTORY_BOND)
        theta = spec.theta0().requires_grad_(True)
        s = torch.tensor(col["suction"], dtype=torch.float64, device="cuda", requires_grad=True)
        v = torch.tensor(v0, dtype=torch.float64, device="cuda", requires_grad=True)
        u = adjoint.ColumnRun.apply(theta, s, v, spec)
        J = (u * torch.tensor(c, device="cuda")).sum()
        J.backward()
        return theta.grad.numpy().copy(), s.grad.cpu().numpy(), v.grad.cpu().numpy()

    ref = grad(1)
    for k in (4, 10):
        got = grad(k)
        say("k", k, got[0], ref[0])
        for a, b in zip(got, ref):
            assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    dv = rng.normal(size=(n, 3))
    dv[fixed] = 0.0
    dS = olib.empty_state(n)
    dS["v"][:] = dv
    oprm.dt = dt
    H = olib.BondHistory(n, 200 * n)
    rc, _, st = olib.step_dual_bond_history(olib.copy_state(S), dS, oprm, np.zeros(4), H, 10)
    assert rc == 0 and st["n_plastic"] > 0
    dJ = float(np.sum(c * dS["u"]))
    g = float(np.sum(ref[2] * dv))
    say("v0 direction", dJ, g)
    assert abs(g - dJ) <= 1e-7 * abs(dJ)
