"""Accuracy and cost measurements of the library on one GPU, each printing
one JSON line.

    python -m paper_2203_05562_amd.measure mixed-error [--config C2] [--at 100,500,1000] [--no-floor]
        Mixed-precision run against the FP64 run of the same column from the
        same initial state: relative L2 errors of u, sigma and v at the given
        step counts, and the time per step of each; beside it the floor, an
        FP64 run from initial positions moved by one ulp against the same
        FP64 run.

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

    python -m paper_2203_05562_amd.measure uniaxial [--m 2,3] [--t-end 0.1] [--dt 3e-6]
        Dynamic uniaxial compression of an elastic bar (Section 4.1), standard
        correspondence against sub-horizons: the non-affine and checkerboard
        parts of the velocity field and the sigma_xx oscillation along the
        axis over time.

    python -m paper_2203_05562_amd.measure point-order [--configs C1,C4] [--warm 1000]
        Time per step and per phase with the points numbered in lattice order
        and in Morton order (the library processes points in id order).

    python -m paper_2203_05562_amd.measure copy [--mib 1024]
        One device-to-device copy of a known size (a float64 tensor), the
        reference that scales the HBM byte counters of a profiler run.

    python -m paper_2203_05562_amd.measure profile-summary --dir D [--kernel REGEX] [--skip-first]
        Reads the database a rocprofv3 run wrote under D (kernel dispatches
        of --kernel-trace, and/or the per-dispatch counters of --pmc) and
        prints it as a JSON line: per kernel name the calls and the average /
        min / max duration, and per counter the mean value per dispatch of
        the kernels matching REGEX (the first dispatch left out with
        --skip-first).  No GPU is used.
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


def mixed_error(cfg_name: str, at, floor: bool = True, max_family: int = 0):
    """Mixed precision against FP64 from the same initial state, and (floor)
    FP64 against FP64 from perturbed initial positions: moved by one FP64 ulp
    in every coordinate (seeded signs), and rounded to FP32.  The first shows
    the smooth sensitivity of the trajectory; the second also lets pairs near
    |x_k - x_j| = delta change sides, as the positions of a mixed run do, and
    so measures the floor that the discontinuous set decisions put under any
    run perturbed at FP32 size."""
    import numpy as np
    import torch
    from . import inputs, ulppm
    cfg = inputs.CONFIGS[cfg_name]
    col = inputs.make_column(cfg)
    n = col["n"]
    runs = {}
    names = [("fp64", ulppm.ULPPM_FP64), ("mixed", ulppm.ULPPM_MIXED)]
    if floor:
        names += [("fp64_ulp", ulppm.ULPPM_FP64), ("fp64_x0f32", ulppm.ULPPM_FP64)]
    for name, prec in names:
        c = col
        if name == "fp64_ulp":
            sgn = np.random.default_rng(cfg.seed + 1000).choice([-1.0, 1.0], col["x0"].shape)
            c = dict(col, x0=np.nextafter(col["x0"], col["x0"] + sgn))
        elif name == "fp64_x0f32":
            # the initial positions rounded to FP32: a perturbation of the size
            # that FP32 arithmetic makes, taken once at the start
            c = dict(col, x0=col["x0"].astype(np.float32).astype(np.float64))
        G = ulppm.column_state(c, "cuda:0")
        prm = ulppm.make_params(col["params"], precision=prec)
        ctx = ulppm.Context(n, max_family=max_family)
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
        b = runs["fp64"][0]
        row = dict(step=target)
        for name in runs:
            if name == "fp64":
                continue
            a = runs[name][0]
            row[name] = dict(u_rel_l2=rel_l2(a["u"], b["u"]), sig_rel_l2=rel_l2(a["sig"], b["sig"]),
                             v_rel_l2=rel_l2(a["v"], b["v"]), pc_rel_l2=rel_l2(a["pc"], b["pc"]))
        log(row)
        out.append(row)
    return dict(kind="mixed-error", workload=f"{cfg_name}: {cfg.nx}x{cfg.ny}x{cfg.nz} column", points=n, dt=dt,
                errors=out, ms_per_step={k: 1e3 * r[3] / done for k, r in runs.items()},
                speedup=runs["fp64"][3] / runs["mixed"][3])


def uniaxial(ms, t_end: float, dt: float, sample_every: int, dims=(40, 12, 12)):
    """Dynamic uniaxial compression (Section 4.1) of the elastic bar, with the
    standard correspondence model (Eqs. 12-14) and with the bond-associated
    sub-horizons, for each horizon ratio m.  Every `sample_every` steps:
    the RMS velocity, the part of the velocity field that no affine field
    A x + b explains (least squares over all points) and its checkerboard
    component sum_i (-1)^(ix+iy+iz) v_i / n, both relative to the RMS
    velocity, and the oscillation of sigma_xx along the bar's axis (RMS of its
    second difference over the mean |sigma_xx| of the axis points)."""
    import numpy as np
    import torch
    from . import inputs, ulppm
    out = []
    for m in ms:
        blk = inputs.make_uniaxial_block(m, dims)
        lat = blk["lattice"]
        nx, ny, nz = blk["dims"]
        sgn = torch.tensor((-1.0) ** lat.sum(axis=1), dtype=torch.float64, device="cuda")
        axis = np.nonzero((lat[:, 1] == ny // 2) & (lat[:, 2] == nz // 2))[0]
        axis = torch.tensor(axis[np.argsort(lat[axis, 0])], device="cuda")
        X = torch.tensor(np.concatenate([blk["x0"], np.ones((blk["n"], 1))], axis=1), device="cuda")
        for name, mode in (("standard", ulppm.ULPPM_FORCE_STANDARD), ("sub-horizon", ulppm.ULPPM_FORCE_CONJUGATE)):
            G = ulppm.column_state(blk, "cuda:0", v0=blk["v0"])
            prm = ulppm.make_params(blk["params"], force_mode=mode)
            ctx = ulppm.Context(blk["n"], max_family=0 if m > 2 else 64)
            ctx.init_state(G, prm, blk["params"]["ocr"])
            dtc = ctx.dt_crit(G, prm)
            prm.dt = dt
            nsteps = int(round(t_end / dt))
            rows, done = [], 0
            t0 = time.perf_counter()
            while done < nsteps:
                k = min(sample_every, nsteps - done)
                ctx.step(G, prm, k)
                done += k
                v = G["v"].t()
                vr = float(torch.sqrt((v * v).sum(1).mean()))
                coef = torch.linalg.lstsq(X, v).solution
                na = v - X @ coef
                cb = (sgn[:, None] * v).mean(0)
                sx = G["sig"][0][axis]
                d2 = sx[2:] - 2.0 * sx[1:-1] + sx[:-2]
                na_rms = float(torch.sqrt((na * na).sum(1).mean()))
                rows.append(dict(step=done, t=done * dt, v_rms=vr, nonaffine_rms=na_rms, nonaffine=na_rms / vr,
                                 checkerboard_abs=float(torch.linalg.vector_norm(cb)),
                                 checkerboard=float(torch.linalg.vector_norm(cb)) / vr,
                                 sigxx_osc=float(torch.sqrt((d2 * d2).mean()) / sx.abs().mean()),
                                 sigxx_axis_mean=float(sx.mean())))
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            log(dict(m=m, model=name, last=rows[-1], seconds=round(el, 2)))
            out.append(dict(m=m, model=name, delta=blk["params"]["delta"], dt=dt, dt_crit=dtc, steps=nsteps,
                            seconds=round(el, 2), samples=rows))
            del ctx, G
    return dict(kind="uniaxial", workload=f"uniaxial compression bar {dims[0]}x{dims[1]}x{dims[2]}, spacing "
                                          f"{inputs.UNIAXIAL['spacing']} m, u_x = {inputs.UNIAXIAL['u_total']} m "
                                          f"over {t_end} s", runs=out)


def point_order(cfgs, warm: int, steps: int):
    """Time per step and per phase of the same column with its points numbered
    in lattice order and in Morton order, after `warm` untimed steps (the
    late state of a collapse when warm is large), FP64 and mixed."""
    import torch
    from . import inputs, ulppm
    rows = []
    for cfg_name in cfgs:
        cfg = inputs.CONFIGS[cfg_name]
        w = warm if cfg.n_points < 1_000_000 else 0
        for order in ("lattice", "morton"):
            col = inputs.make_column(cfg, order=order)
            for prec in ("fp64", "mixed"):
                G = ulppm.column_state(col, "cuda:0")
                prm = ulppm.make_params(col["params"], precision=ulppm.ULPPM_MIXED if prec == "mixed" else 0)
                ctx = ulppm.Context(col["n"], max_family=128)
                ctx.init_state(G, prm, col["params"]["ocr"])
                prm.dt = 0.5 * ctx.dt_crit(G, prm)
                if w:
                    ctx.step(G, prm, w)
                torch.cuda.synchronize()
                prm.timing = 1
                s = torch.cuda.current_stream()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                rep = ctx.step(G, prm, steps)
                e1.record(s)
                torch.cuda.synchronize()
                ph = {k: round(rep[f"t_{k}_ms"] / steps, 4) for k in ("predict", "family", "kin", "bond", "gather")}
                rows.append(dict(config=cfg_name, order=order, precision=prec, after_steps=w,
                                 ms_per_step=round(e0.elapsed_time(e1) / steps, 4), phase_ms=ph))
                log(rows[-1])
                del ctx, G
                torch.cuda.empty_cache()
    return dict(kind="point-order", rows=rows)


def adjoint_cost(cfg_name: str, steps: int, every: int, precision: str, max_family: int = 0,
                 reverse: str = "fp64"):
    import torch
    from . import adjoint, inputs, ulppm
    cfg = inputs.CONFIGS[cfg_name]
    col = inputs.make_column(cfg)
    prec = ulppm.ULPPM_MIXED if precision == "mixed" else ulppm.ULPPM_FP64
    rprec = ulppm.ULPPM_MIXED if reverse == "mixed" else ulppm.ULPPM_FP64
    spec = adjoint.ColumnSpec(col, steps, every, precision=prec, max_family=max_family, reverse_precision=rprec)
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
                         f"{precision} forward, {reverse} reverse, objective runout + settlement",
                points=col["n"], max_family=max_family or 152, forward_ms=round(fwd, 2), backward_ms=round(bwd, 2),
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


def profile_summary(d: str, kernel: str, skip_first: bool):
    """Kernel durations and per-dispatch counters from the SQLite database
    (rocpd) that rocprofv3 writes by default under d."""
    import glob
    import os
    import re
    import sqlite3
    out = dict(kind="profile-summary", dir=os.path.basename(os.path.normpath(d)), kernels={}, counters={})
    rx = re.compile(kernel)
    per = {}
    for f in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
        con = sqlite3.connect(f)
        durs = {}
        for name, dur, did in con.execute("select name, duration, dispatch_id from kernels"):
            durs.setdefault(name, []).append((did, dur * 1e-6))
        for name, v in durs.items():
            ms = [x for _, x in sorted(v)]
            out["kernels"][name] = dict(calls=len(ms), total_ms=sum(ms), avg_ms=sum(ms) / len(ms), min_ms=min(ms),
                                        max_ms=max(ms))
        q = ("select kernel_name, counter_name, dispatch_id, value, vgpr_count, accum_vgpr_count, sgpr_count, "
             "lds_block_size, scratch_size from counters_collection")
        for kn, cn, did, val, vg, ag, sg, lds, scr in con.execute(q):
            if not rx.search(kn):
                continue
            e = per.setdefault((kn, cn), {}).setdefault(did, [0.0, (vg, ag, sg, lds, scr)])
            e[0] += val
    for (kn, cn), disp in per.items():
        ids = sorted(disp)
        if skip_first and len(ids) > 1:
            ids = ids[1:]
        vals = [disp[i][0] for i in ids]
        vg, ag, sg, lds, scr = disp[ids[0]][1]
        out["counters"].setdefault(kn, {})[cn] = dict(mean=sum(vals) / len(vals), dispatches=len(vals))
        out["counters"][kn]["_resources"] = dict(vgpr=vg, agpr=ag, sgpr=sg, lds=lds, scratch=scr)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("mixed-error")
    a.add_argument("--config", default="C2")
    a.add_argument("--at", default="100,500,1000")
    a.add_argument("--no-floor", action="store_true", help="skip the FP64 run from one-ulp moved positions")
    a.add_argument("--max-family", type=int, default=0)
    b = sub.add_parser("adjoint-cost")
    b.add_argument("--config", default="C4")
    b.add_argument("--steps", type=int, default=50)
    b.add_argument("--every", type=int, default=25)
    b.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    b.add_argument("--max-family", type=int, default=0, help="family capacity of the context (0: 152)")
    b.add_argument("--reverse", default="fp64", choices=["fp64", "mixed"],
                   help="precision of the reverse steps' membership-matrix sweeps")
    d = sub.add_parser("adjoint-check")
    d.add_argument("--config", default="C3")
    d.add_argument("--steps", type=int, default=1000)
    d.add_argument("--every", type=int, default=50)
    d.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    o = sub.add_parser("point-order")
    o.add_argument("--configs", default="C1,C4")
    o.add_argument("--warm", type=int, default=1000)
    o.add_argument("--steps", type=int, default=20)
    f = sub.add_parser("uniaxial")
    f.add_argument("--m", default="2,3")
    f.add_argument("--t-end", type=float, default=0.1)
    f.add_argument("--dt", type=float, default=3.0e-6)
    f.add_argument("--sample-every", type=int, default=1000)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    e = sub.add_parser("profile-summary")
    e.add_argument("--dir", required=True)
    e.add_argument("--kernel", default=".")
    e.add_argument("--skip-first", action="store_true")
    args = ap.parse_args(argv)
    if args.what == "profile-summary":
        print(json.dumps(profile_summary(args.dir, args.kernel, args.skip_first)), flush=True)
        return
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
    elif args.what == "point-order":
        out = point_order(args.configs.split(","), args.warm, args.steps)
    elif args.what == "uniaxial":
        out = uniaxial([int(v) for v in args.m.split(",")], args.t_end, args.dt, args.sample_every)
    elif args.what == "mixed-error":
        out = mixed_error(args.config, [int(x) for x in args.at.split(",")], not args.no_floor, args.max_family)
    else:
        out = adjoint_cost(args.config, args.steps, args.every, args.precision, args.max_family, args.reverse)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
