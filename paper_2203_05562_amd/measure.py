"""Accuracy and cost measurements of the library on one GPU, each printing
one JSON line.

    python -m paper_2203_05562_amd.measure mixed-error [--config C2] [--at 100,500,1000]
        Mixed-precision run against the FP64 run of the same column from the
        same initial state: relative L2 errors of u, sigma and v at the given
        step counts, and the time per step of each.

    python -m paper_2203_05562_amd.measure adjoint-cost [--config C4] [--steps 50] [--every 25]
                                                        [--precision mixed]
        Checkpointed forward and backward of the differentiable column
        (objective: runout + settlement): time per forward step, per reverse
        step and their ratio.

    python -m paper_2203_05562_amd.measure adjoint-check [--config C3] [--steps 1000] [--every 50]
        Gradients of runout + settlement from the checkpointed adjoint against
        GPU central differences (h = 1e-6 relative) of u^N contracted with
        the objective's gradient, in (M, lam, kap, eta), uniform suction and
        a seeded initial-velocity direction, each marked valid only when the
        two perturbed runs visit the same family and sub-horizon counts.

    python -m paper_2203_05562_amd.measure copy [--mib 1024]
        One device-to-device copy of a known size (a float64 tensor), the
        reference that scales the HBM byte counters of a profiler run.
"""
import argparse
import json
import sys
import time


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def mixed_error(cfg_name: str, at):
    import torch
    from . import inputs, ulppm
    cfg = inputs.CONFIGS[cfg_name]
    col = inputs.make_column(cfg)
    n = col["n"]
    runs = {}
    for name, prec in (("fp64", ulppm.ULPPM_FP64), ("mixed", ulppm.ULPPM_MIXED)):
        G = ulppm.column_state(col, "cuda:0")
        prm = ulppm.make_params(col["params"], precision=prec)
        ctx = ulppm.Context(n)
        ctx.init_state(G, prm, col["params"]["ocr"])
        runs[name] = [G, prm, ctx, 0.0]
    dt = 0.5 * runs["fp64"][2].dt_crit(runs["fp64"][0], runs["fp64"][1])
    for r in runs.values():
        r[1].dt = dt
    out, done = [], 0
    for target in at:
        for name, r in runs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r[2].step(r[0], r[1], target - done)
            torch.cuda.synchronize()
            r[3] += time.perf_counter() - t0
        done = target
        a, b = runs["mixed"][0], runs["fp64"][0]
        row = dict(step=target, u_rel_l2=rel_l2(a["u"], b["u"]), sig_rel_l2=rel_l2(a["sig"], b["sig"]),
                   v_rel_l2=rel_l2(a["v"], b["v"]), pc_rel_l2=rel_l2(a["pc"], b["pc"]))
        log(row)
        out.append(row)
    return dict(kind="mixed-error", workload=f"{cfg_name}: {cfg.nx}x{cfg.ny}x{cfg.nz} column", points=n, dt=dt,
                errors=out, ms_per_step={k: 1e3 * r[3] / done for k, r in runs.items()},
                speedup=runs["fp64"][3] / runs["mixed"][3])


def adjoint_cost(cfg_name: str, steps: int, every: int, precision: str):
    import torch
    from . import adjoint, inputs, ulppm
    cfg = inputs.CONFIGS[cfg_name]
    col = inputs.make_column(cfg)
    prec = ulppm.ULPPM_MIXED if precision == "mixed" else ulppm.ULPPM_FP64
    spec = adjoint.ColumnSpec(col, steps, every, precision=prec)
    spec.timing = True
    w = inputs.runout_objective_weights(col["lattice"], col["dims"])
    theta = spec.theta0().requires_grad_(True)
    s = torch.tensor(col["suction"], dtype=torch.float64, device="cuda", requires_grad=True)
    v = torch.zeros((col["n"], 3), dtype=torch.float64, device="cuda", requires_grad=True)
    x0 = torch.tensor(col["x0"], dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    u = adjoint.ColumnRun.apply(theta, s, v, spec)
    ev[1].record()
    J = adjoint.runout_settlement(u, x0, w["top"], w["axis"], 0.1 * inputs.DX)
    J.backward()
    ev[2].record()
    torch.cuda.synchronize()
    fwd, bwd = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    t = spec.last_timing
    return dict(kind="adjoint-cost",
                workload=f"{cfg_name}: {cfg.nx}x{cfg.ny}x{cfg.nz} column, {steps} steps, checkpoint every {every}, "
                         f"{precision} forward, objective runout + settlement",
                points=col["n"], forward_ms=round(fwd, 2), backward_ms=round(bwd, 2),
                recompute_ms=round(t["recompute"], 2), reverse_ms=round(t["reverse"], 2),
                forward_ms_per_step=round(fwd / steps, 4), adjoint_ms_per_step=round(t["reverse"] / steps, 4),
                adjoint_to_forward_step=round(t["reverse"] / fwd, 3), backward_to_forward=round(bwd / fwd, 3),
                objective=float(J.detach()), grad_theta=[float(g) for g in theta.grad],
                grad_suction_sum=float(s.grad.sum()), grad_v0_norm=float(torch.linalg.vector_norm(v.grad)))


def adjoint_check(cfg_name: str, steps: int, every: int, precision: str = "fp64", vscale: float = 0.3,
                  seed: int = 5):
    import numpy as np
    import torch
    from . import adjoint, inputs, ulppm
    cfg = inputs.CONFIGS[cfg_name]
    col = inputs.make_column(cfg)
    n = col["n"]
    prec = ulppm.ULPPM_MIXED if precision == "mixed" else ulppm.ULPPM_FP64
    spec = adjoint.ColumnSpec(col, steps, every, precision=prec)
    w = inputs.runout_objective_weights(col["lattice"], col["dims"])
    tau = 0.1 * inputs.DX
    rng = np.random.default_rng(seed)
    fixed = torch.tensor(col["fixed"] == 1, device="cuda")
    v0 = torch.tensor(rng.uniform(-vscale, vscale, (n, 3)), dtype=torch.float64, device="cuda")
    v0[fixed] = 0.0
    x0 = torch.tensor(col["x0"], dtype=torch.float64, device="cuda")
    theta = spec.theta0().requires_grad_(True)
    s = torch.tensor(col["suction"], dtype=torch.float64, device="cuda", requires_grad=True)
    v = v0.clone().requires_grad_(True)
    t0 = time.perf_counter()
    u = adjoint.ColumnRun.apply(theta, s, v, spec)
    J = adjoint.runout_settlement(u, x0, w["top"], w["axis"], tau)
    J.backward()
    t_adj = time.perf_counter() - t0
    uu = u.detach().clone().requires_grad_(True)
    adjoint.runout_settlement(uu, x0, w["top"], w["axis"], tau).backward()
    gu = uu.grad

    def run(th, sv, vv):
        S = spec.initial_state(th, sv, vv)
        p = spec.params_for(th)
        bonds = tri = pl = 0
        done = 0
        while done < steps:
            m = min(every, steps - done)
            rep = spec.ctx.step(S, p, m)
            bonds += rep["n_bond_updates"]
            tri += rep["n_triples"]
            pl += rep["n_plastic"]
            done += m
        return S.t["u"].t().clone(), (bonds, tri, pl)

    th0 = spec.theta0()
    dv = torch.tensor(rng.normal(size=(n, 3)), dtype=torch.float64, device="cuda")
    dv[fixed] = 0.0
    s0 = s.detach()
    dirs = []
    for k, name in enumerate(("M", "lam", "kap", "eta")):
        e = torch.zeros(4, dtype=torch.float64)
        e[k] = 1.0
        dirs.append((name, 1e-6 * float(th0[k]), lambda h, e=e: (th0 + h * e, s0, v0), float(theta.grad[k])))
    sm = float(s0.mean())
    dirs.append(("suction", 1e-6 * sm, lambda h: (th0, s0 + h, v0), float(s.grad.sum())))
    dirs.append(("v0", 1e-6 * vscale, lambda h: (th0, s0, v0 + h * dv), float((v.grad * dv).sum())))
    rows = []
    for name, h, mk, g in dirs:
        up, cp = run(*mk(+h))
        um, cm = run(*mk(-h))
        fd = float((gu * (up - um)).sum()) / (2 * h)
        rel = abs(fd - g) / max(abs(g), 1e-300)
        # families and sub-horizons are the sets the gradient is taken on; a
        # bond that crosses the yield surface leaves the Perzyna update
        # continuous and is only counted
        rows.append(dict(direction=name, adjoint=g, fd=fd, rel_err=rel, sets_equal=cp[:2] == cm[:2],
                         plastic_count_change=abs(cp[2] - cm[2])))
        log(rows[-1])
    return dict(kind="adjoint-check", workload=f"{cfg_name}: {cfg.nx}x{cfg.ny}x{cfg.nz} column, {steps} steps, "
                                               f"checkpoint every {every}, {precision}",
                points=n, objective=float(J.detach()), seconds_forward_backward=round(t_adj, 2), checks=rows)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("mixed-error")
    a.add_argument("--config", default="C2")
    a.add_argument("--at", default="100,500,1000")
    b = sub.add_parser("adjoint-cost")
    b.add_argument("--config", default="C4")
    b.add_argument("--steps", type=int, default=50)
    b.add_argument("--every", type=int, default=25)
    b.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    d = sub.add_parser("adjoint-check")
    d.add_argument("--config", default="C3")
    d.add_argument("--steps", type=int, default=1000)
    d.add_argument("--every", type=int, default=50)
    d.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "measurements need a GPU"
    torch.cuda.set_device(0)
    if args.what == "copy":
        nbytes = args.mib << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out = dict(kind="copy", bytes_read=nbytes, bytes_written=nbytes)
    elif args.what == "adjoint-check":
        out = adjoint_check(args.config, args.steps, args.every, args.precision)
    elif args.what == "mixed-error":
        out = mixed_error(args.config, [int(x) for x in args.at.split(",")])
    else:
        out = adjoint_cost(args.config, args.steps, args.every, args.precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
