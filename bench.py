"""Throughput of the explicit UL-PPM step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C1] [--precision fp64|mixed]

A step is one whole explicit Newmark step through the C ABI (predictor,
family rebuild, bond kernel, gather/corrector, energies) on a seeded
synthetic soil column whose state is resident in HBM.  The metric is
bond-updates/s: directed bonds taken through one step, summed over the K
timed steps, divided by the wall time of those steps (HIP events on the
stream the library runs on).  Prints exactly one JSON line on stdout;
progress goes to stderr.

The roofline object describes the dominant kernel, k_bond_mx, bound by the
FP64 arithmetic rate (the vector and the matrix FP64 peaks are equal on
this chip): algorithmic flops per launch over its average launch duration,
measured with HIP events around every launch in the timed region.
Algorithmic flops per launch:
    8  per sub-horizon membership test           (sum_i |H_i|^2)
    43 per sub-horizon member                    (sum |S_ij|; 34 for the
       shape tensor, gradient and volume sums, 9 for the force-state sum)
    250 per bond                                 (inversion, gradient, trial
       stress, yield check, force state)
Newton iterations of the return map are not counted; the full-horizon sums
(34 flops per bond) run in the point-kinematics kernel before it.

Two more objects ride on the same line.  "mixed": the same workload in mixed
precision from the same initial state (FP32 sums, gathers and force states),
its throughput, speed-up and relative L2 errors of u, sigma and v against
the FP64 run after warmup + steps steps.  "adjoint": the checkpointed
differentiable column (24x24x48 by default, 1000 steps, checkpoint every 50),
time per forward step, per reverse step (ulppm_adjoint_step) and their ratio.
"contact": the same column standing free on a rigid substrate lattice
(Eqs. 91-93, the substrate one column width wider on every side), its
throughput and gather phase, the kernel that adds the contact forces.
"plane": the plane-strain column P1 (512 x 1024 points in the x-z plane,
families of ~28), its throughput and bond-kernel time.  "history": the
workload with the history carried on the bonds (ULPPM_HISTORY_BOND).
"eq51": the workload with the force state of Eq. 51 as printed.
"adjoint_large": the 128 x 128 x 256 column (4.2M points) with a mixed
forward of 25 steps and its checkpointed reverse, the reverse sweeps in
mixed precision: time per forward step, per reverse step and their ratio.
"full_run": the workload as defined, 2000 steps from rest for seeds 1, 2 and
3 (suction drawn per seed), with the energy balance of Eq. 69 checked after
every 100 steps: time per step over the run and in windows, candidate
rebuilds, plastic fraction, largest family and the final energy residual.

The roofline object also carries the HBM side of the same kernel:
achieved_gbs = traffic / average launch duration and hbm_frac = that over
8 TB/s, where traffic is the counter-measured byte count of the committed
profile (null when the kernel source changed since).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_TEST = 8.0
FLOPS_PER_MEMBER_SUMS = 34.0      # shape tensor, gradient numerator, volume (Eqs. 23, 25, 55, 57)
FLOPS_PER_MEMBER_CONJ = 9.0       # the conjugate force-state sum (pass 2)
FLOPS_PER_MEMBER = FLOPS_PER_MEMBER_SUMS + FLOPS_PER_MEMBER_CONJ
FLOPS_PER_BOND = 250.0
PEAK_FP64_VALU_TFLOPS = 78.6      # MI355X vector FP64 (and FP32 without packing)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    with open(os.path.join(ROOT, "paper_2203_05562_amd", "csrc", "ulppm.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(config, precision):
    """HBM bytes per k_bond launch from the committed counter summary, if it
    was taken on the current kernel source for this workload; else None."""
    path = os.path.join(ROOT, "profiles", "k_bond_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    key = f"{config}_{precision}"
    e = d.get(key)
    if not e or e.get("source_sha") != kernel_source_sha():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(cfg_name, steps, dt):
    """The oracle as it stands, on the host cores, for a bounded sample."""
    import numpy as np
    import oracle
    from paper_2203_05562_amd import inputs
    cfg = inputs.CONFIGS[cfg_name]
    col = inputs.make_column(cfg)
    prm = oracle.make_params(col["params"])
    t0 = time.time()
    S = oracle.init_column(col, prm, col["params"]["ocr"])
    log(f"[cpu] oracle initial state {time.time() - t0:.1f}s")
    prm.dt = dt
    t0 = time.perf_counter()
    rc, E, st = oracle.step(S, prm, steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    log(f"[cpu] oracle {steps} steps {el:.1f}s rc={rc} bonds={st['n_bonds']}")
    return dict(value=st["n_bonds"] / el, unit="bond-updates/s", cores=cores, kind="oracle",
                sample=f"{steps} full explicit steps of the {cfg.nx}x{cfg.ny}x{cfg.nz} column "
                       f"({col['n']} points, {st['n_bonds']} bond-updates) from its initial state",
                seconds=round(el, 3))


def run_column(ulppm, col, precision, warmup, steps, timed=True, contact=None, max_family=0, history=0,
               force_mode=0):
    """Initial conditions, dt = dt_c / 2, `warmup` untimed steps, then
    `steps` steps timed with HIP events on the library's stream.  `contact`
    attaches a substrate (Eqs. 91-93) first."""
    import torch
    G = ulppm.column_state(col, "cuda:0")
    prm = ulppm.make_params(col["params"], precision=precision, history=history, force_mode=force_mode)
    ctx = ulppm.Context(col["n"], max_family=max_family)
    if history:
        ctx.history_reserve()
    if contact:
        ctx.set_contact(contact)
    ctx.init_state(G, prm, col["params"]["ocr"])
    prm.dt = 0.5 * ctx.dt_crit(G, prm)
    if warmup:
        ctx.step(G, prm, warmup)
    torch.cuda.synchronize()
    prm.timing = 1 if timed else 0
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rep = ctx.step(G, prm, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del ctx
    return G, rep, ms, prm.dt


def full_run(ulppm, cfg_name, seeds, nsteps, chunk, max_family):
    """The workload as defined: `nsteps` steps from rest per seed, in calls of
    `chunk` steps with the energy balance of Eq. 69 checked after each call
    (from the first call's end, past step 40).  A family that outgrows
    `max_family` restarts the seed at the default capacity."""
    import torch
    from paper_2203_05562_amd import inputs
    cfg = inputs.CONFIGS[cfg_name]
    runs = []
    tot_bonds, tot_ms = 0, 0.0
    for seed in seeds:
        col = inputs.make_column(cfg, seed=seed)
        cap = max_family
        while True:
            G = ulppm.column_state(col, "cuda:0")
            prm = ulppm.make_params(col["params"], energy_check=1, energy_tol=1e-2, timing=1)
            ctx = ulppm.Context(col["n"], max_family=cap)
            ctx.init_state(G, prm, col["params"]["ocr"])
            prm.dt = 0.5 * ctx.dt_crit(G, prm)
            stream = torch.cuda.current_stream()
            chunks, status = [], "ok"
            try:
                for c in range(nsteps // chunk):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    rep = ctx.step(G, prm, chunk)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    chunks.append((e0.elapsed_time(e1), rep))
            except ulppm.UlppmError as e:
                if e.code == -2 and cap != 0:
                    log(f"[gpu] full run seed {seed}: families outgrew {cap}; restarting at the default capacity")
                    cap = 0
                    del ctx, G
                    continue
                status = str(e)
            break
        ms = [c[0] for c in chunks]
        reps = [c[1] for c in chunks]
        bonds = sum(r["n_bond_updates"] for r in reps)
        last = reps[-1] if reps else {}
        E = (last.get("W_int", 0.0), last.get("W_ext", 0.0), last.get("W_kin", 0.0))
        emax = max(abs(v) for v in E) or 1.0

        def window(k):
            return round(ms[k] / chunk, 4) if k < len(ms) else None

        done = len(ms) * chunk
        runs.append(dict(seed=seed, suction_kpa=round(col["suction_kpa"], 3), steps=done, status=status,
                         ms_per_step=round(sum(ms) / max(done, 1), 4),
                         window_ms_per_step={f"{k * chunk}-{(k + 1) * chunk}": window(k)
                                             for k in (0, nsteps // chunk // 2 - 1, nsteps // chunk - 1)},
                         bond_ms_per_step=round(sum(r["t_bond_ms"] for r in reps) / max(done, 1), 4),
                         bond_updates_per_s=bonds / (sum(ms) * 1e-3) if ms else None,
                         rebuilds=sum(r["n_rebuilds"] for r in reps),
                         plastic_fraction=sum(r["n_plastic"] for r in reps) / max(bonds, 1),
                         largest_family=max((r["max_family"] for r in reps), default=0),
                         max_family=cap or 152,
                         energy_residual=abs(E[0] + E[2] - E[1]) / emax, W=E))
        log(f"[gpu] full run: {runs[-1]}")
        tot_bonds += bonds
        tot_ms += sum(ms)
        del ctx, G
        torch.cuda.empty_cache()
    return dict(workload=f"{cfg_name}: {cfg.nx}x{cfg.ny}x{cfg.nz} column, {nsteps} steps from rest per seed, "
                         f"Eq. 69 checked every {chunk} steps", seeds=list(seeds),
                value=tot_bonds / (tot_ms * 1e-3) if tot_ms else None, unit="bond-updates/s", runs=runs)


def rel_l2(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="C1")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--cpu-steps", type=int, default=5,
                    help="full oracle steps of the workload timed on the host cores (about 10 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision companion run")
    ap.add_argument("--adjoint-config", default="C3", help="configuration of the adjoint cost line ('' skips it)")
    ap.add_argument("--adjoint-steps", type=int, default=1000)
    ap.add_argument("--adjoint-every", type=int, default=50)
    ap.add_argument("--adjoint-large-config", default="C4",
                    help="configuration of the large mixed-precision adjoint line ('' skips it)")
    ap.add_argument("--adjoint-large-steps", type=int, default=25)
    ap.add_argument("--adjoint-large-every", type=int, default=25)
    ap.add_argument("--no-contact", action="store_true", help="skip the substrate-contact companion run")
    ap.add_argument("--no-plane", action="store_true", help="skip the plane-strain companion run")
    ap.add_argument("--no-history", action="store_true", help="skip the bond-history companion run")
    ap.add_argument("--no-standard", action="store_true",
                    help="skip the companion run of the standard (full-horizon) correspondence model")
    ap.add_argument("--full-steps", type=int, default=2000,
                    help="steps per seed of the full-run companion (0 skips it)")
    ap.add_argument("--full-seeds", default="1,2,3")
    ap.add_argument("--no-eq51", action="store_true", help="skip the Eq. 51 companion run")
    ap.add_argument("--max-family", type=int, default=128,
                    help="family capacity of the main run's context (0: the library default, 152); a run whose "
                         "families outgrow it is repeated with the default")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_05562_amd import inputs, ulppm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = inputs.CONFIGS[args.config]
    col = inputs.make_column(cfg)
    n = col["n"]
    log(f"[gpu] {args.config}: {cfg.nx}x{cfg.ny}x{cfg.nz} = {n} points, suction {col['suction_kpa']:.2f} kPa")
    prec = ulppm.ULPPM_MIXED if args.precision == "mixed" else ulppm.ULPPM_FP64
    # A capacity of 128 members (the column's families hold at most ~120) leaves
    # LDS for five bond workgroups per CU; a family that outgrows it raises a
    # capacity error, and the run is repeated with the default capacity.
    max_family = args.max_family
    try:
        G, rep, ms, dt = run_column(ulppm, col, prec, args.warmup, args.steps, max_family=max_family)
    except ulppm.UlppmError as e:
        if e.code != -2 or max_family == 0:
            raise
        log(f"[gpu] families outgrew max_family={max_family}; repeating with the default capacity")
        max_family = 0
        G, rep, ms, dt = run_column(ulppm, col, prec, args.warmup, args.steps, max_family=max_family)
    log(f"[gpu] dt = {dt:.4e} s; timed {args.steps} steps after {args.warmup}: {ms:.1f} ms; report {rep}")
    bonds = rep["n_bond_updates"]
    value = bonds / (ms * 1e-3)
    launches = rep["timed_steps"]
    t_bond = rep["t_bond_ms"] / max(launches, 1) * 1e-3
    flops_per_launch = (FLOPS_PER_TEST * rep["n_tests"] + FLOPS_PER_MEMBER * rep["n_triples"] +
                        FLOPS_PER_BOND * bonds) / args.steps
    achieved = flops_per_launch / t_bond / 1e12
    traffic = measured_traffic(args.config, args.precision)
    gbs = traffic / t_bond / 1e9 if traffic else None
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_VALU_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP64_VALU_TFLOPS, 4), traffic=traffic,
                    kernel="k_bond_mx", avg_launch_ms=round(t_bond * 1e3, 4),
                    flops_per_launch=flops_per_launch,
                    flops_per_unit=dict(test=FLOPS_PER_TEST, member_sums=FLOPS_PER_MEMBER_SUMS,
                                        member_conjugate_sum=FLOPS_PER_MEMBER_CONJ, bond=FLOPS_PER_BOND),
                    frac_without_conjugate_sum=round(
                        (flops_per_launch - FLOPS_PER_MEMBER_CONJ * rep["n_triples"] / args.steps) / t_bond / 1e12
                        / PEAK_FP64_VALU_TFLOPS, 4),
                    achieved_gbs=round(gbs, 1) if gbs else None,
                    hbm_frac=round(gbs / PEAK_HBM_GBS, 4) if gbs else None)
    phases = {k: round(rep[f"t_{k}_ms"] / max(launches, 1), 4) for k in ("predict", "family", "kin", "bond", "gather")}
    out = dict(metric="bond-updates/s per Newmark step", value=value, unit="bond-updates/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f64" if args.precision == "fp64" else "f32+f64",
               data="synthetic",
               config=dict(workload=f"{args.config}: jittered soil column {cfg.nx}x{cfg.ny}x{cfg.nz}, "
                                    f"{args.precision}", points=n, bonds_per_step=bonds / args.steps,
                           max_family=max_family or 152, largest_family=rep["max_family"],
                           dt=dt, suction_kpa=col["suction_kpa"], seed=cfg.seed, precision=args.precision),
               roofline=roofline, phase_ms=phases)
    def run_cap(c, precision=prec, **kw):
        # the main run's family capacity, or the default where a family outgrows it
        try:
            return run_column(ulppm, c, precision, args.warmup, args.steps, max_family=max_family, **kw) + (max_family,)
        except ulppm.UlppmError as e:
            if e.code != -2 or max_family == 0:
                raise
            return run_column(ulppm, c, precision, args.warmup, args.steps, **kw) + (0,)

    if args.precision == "fp64" and not args.no_mixed:
        # the same run in mixed precision from the same initial state, at the same family capacity
        Gm, repm, msm, _, capm = run_cap(col, precision=ulppm.ULPPM_MIXED)
        vm = repm["n_bond_updates"] / (msm * 1e-3)
        lm = max(repm["timed_steps"], 1)
        out["mixed"] = dict(value=vm, ms_per_step=msm / args.steps, speedup=round(vm / value, 3),
                            max_family=capm or 152, steps_compared=args.warmup + args.steps,
                            u_rel_l2=rel_l2(Gm["u"], G["u"]), sig_rel_l2=rel_l2(Gm["sig"], G["sig"]),
                            v_rel_l2=rel_l2(Gm["v"], G["v"]),
                            phase_ms={k: round(repm[f"t_{k}_ms"] / lm, 4)
                                      for k in ("predict", "family", "kin", "bond", "gather")})
        log(f"[gpu] mixed: {out['mixed']}")
        del Gm
    del G
    torch.cuda.empty_cache()

    if not args.no_contact:
        colc = inputs.make_column(cfg, fixed_base=False)
        sub = inputs.make_substrate(colc)
        Gc, repc, msc, _, capc = run_cap(colc, contact=sub)
        vc = repc["n_bond_updates"] / (msc * 1e-3)
        lc = max(repc["timed_steps"], 1)
        out["contact"] = dict(value=vc, ms_per_step=msc / args.steps, max_family=capc or 152,
                              sites=int(sub["n"][0] * sub["n"][1] * sub["n"][2]), mu_f=sub["mu_f"],
                              delta_c=sub["delta_c"], cs=sub["cs"],
                              gather_ms=round(repc["t_gather_ms"] / lc, 4),
                              gather_ms_without=phases["gather"],
                              phase_ms={k: round(repc[f"t_{k}_ms"] / lc, 4)
                                        for k in ("predict", "family", "kin", "bond", "gather")},
                              rebuilds=repc["n_rebuilds"], largest_family=repc["max_family"])
        log(f"[gpu] contact: {out['contact']}")
        del Gc
        torch.cuda.empty_cache()
    if not args.no_plane:
        colp = inputs.make_column(inputs.CONFIGS["P1"])
        # plane families hold about 30 members: a context sized for at most 64
        # runs one wave per point, and 48 leaves LDS for twelve such
        # workgroups per CU (three waves per SIMD); 64 if a family outgrows 48
        capp = 48
        try:
            Gp, repp, msp, _ = run_column(ulppm, colp, prec, args.warmup, args.steps, max_family=capp)
        except ulppm.UlppmError as e:
            if e.code != -2:
                raise
            capp = 64
            Gp, repp, msp, _ = run_column(ulppm, colp, prec, args.warmup, args.steps, max_family=capp)
        lp = max(repp["timed_steps"], 1)
        out["plane"] = dict(workload="P1: plane-strain column 512x1024", points=colp["n"], max_family=capp,
                            value=repp["n_bond_updates"] / (msp * 1e-3), ms_per_step=msp / args.steps,
                            bonds_per_step=repp["n_bond_updates"] / args.steps,
                            phase_ms={k: round(repp[f"t_{k}_ms"] / lp, 4)
                                      for k in ("predict", "family", "kin", "bond", "gather")})
        log(f"[gpu] plane: {out['plane']}")
        del Gp
        torch.cuda.empty_cache()
    if not args.no_history:
        Gh, reph, msh, _, caph = run_cap(col, history=ulppm.ULPPM_HISTORY_BOND)
        lh = max(reph["timed_steps"], 1)
        out["history"] = dict(value=reph["n_bond_updates"] / (msh * 1e-3), ms_per_step=msh / args.steps,
                              max_family=caph or 152,
                              phase_ms={k: round(reph[f"t_{k}_ms"] / lh, 4)
                                        for k in ("predict", "family", "kin", "bond", "gather")})
        log(f"[gpu] history: {out['history']}")
        del Gh
        torch.cuda.empty_cache()
    if not args.no_standard:
        # the standard correspondence model (Eqs. 12-14): one full-horizon K_i^{-1} per point
        Gs, reps, mss, _ = run_column(ulppm, col, prec, args.warmup, args.steps, max_family=max_family,
                                      force_mode=ulppm.ULPPM_FORCE_STANDARD)
        ls = max(reps["timed_steps"], 1)
        out["standard"] = dict(value=reps["n_bond_updates"] / (mss * 1e-3), ms_per_step=mss / args.steps,
                               phase_ms={k: round(reps[f"t_{k}_ms"] / ls, 4)
                                         for k in ("predict", "family", "kin", "bond", "gather")})
        log(f"[gpu] standard: {out['standard']}")
        del Gs
        torch.cuda.empty_cache()
    if not args.no_eq51:
        # the force state of Eq. 51 as printed (stable over this short window from rest)
        Ge, repe, mse, _, cape = run_cap(col, force_mode=ulppm.ULPPM_FORCE_EQ51)
        le = max(repe["timed_steps"], 1)
        out["eq51"] = dict(value=repe["n_bond_updates"] / (mse * 1e-3), ms_per_step=mse / args.steps,
                           max_family=cape or 152,
                           phase_ms={k: round(repe[f"t_{k}_ms"] / le, 4)
                                     for k in ("predict", "family", "kin", "bond", "gather")})
        log(f"[gpu] eq51: {out['eq51']}")
        del Ge
        torch.cuda.empty_cache()
    if args.full_steps > 0 and args.precision == "fp64":
        out["full_run"] = full_run(ulppm, args.config, [int(v) for v in args.full_seeds.split(",")],
                                   args.full_steps, 100, max_family)
    if args.adjoint_config:
        from paper_2203_05562_amd.measure import adjoint_cost
        try:
            out["adjoint"] = adjoint_cost(args.adjoint_config, args.adjoint_steps, args.adjoint_every, "fp64",
                                          max_family)
        except ulppm.UlppmError as e:
            if e.code != -2 or max_family == 0:
                raise
            out["adjoint"] = adjoint_cost(args.adjoint_config, args.adjoint_steps, args.adjoint_every, "fp64")
        log(f"[gpu] adjoint: {out['adjoint']}")
    if args.adjoint_large_config:
        # the 4M-point column: mixed forward, reverse sweeps in mixed precision
        from paper_2203_05562_amd.measure import adjoint_cost
        torch.cuda.empty_cache()
        try:
            out["adjoint_large"] = adjoint_cost(args.adjoint_large_config, args.adjoint_large_steps,
                                                args.adjoint_large_every, "mixed", max_family, "mixed")
        except ulppm.UlppmError as e:
            if e.code != -2 or max_family == 0:
                raise
            out["adjoint_large"] = adjoint_cost(args.adjoint_large_config, args.adjoint_large_steps,
                                                args.adjoint_large_every, "mixed", 0, "mixed")
        log(f"[gpu] adjoint_large: {out['adjoint_large']}")
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_steps, dt)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
