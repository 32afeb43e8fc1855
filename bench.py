"""Benchmark: Barnes-Hut force path on one MI355X, 16M-particle ring.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 2^24-particle thin ring (r in [1.0, 1.2], z ~ N(0, 5e-4),
central unit mass, Keplerian velocities with 1e-4 dispersion), eps = 1e-4,
dt = 1e-3, tree and lists rebuilt every 4 steps with moments refreshed on
the other steps.  One benchmark step = one rebuild cycle = 4 kick-drift-kick
steps: keys, sort, tree, moments, groups, walk and lists once, moments three
more times, four force evaluations and the integration.

Before timing, theta is tuned per path so that the 99th percentile of the
relative self-gravity force error over 4096 sampled particles (against the
library's FP64 direct sum) is at most 1e-3:
  tuned: FP32 interactions on group-relative coordinates, groups <= 256,
         lists reused for 4 steps, persistent longest-first force kernel;
  plain: FP64 interactions, groups <= 64, lists rebuilt every step.
The JSON line reports the tuned path's interactions/s (whole job, inputs
resident in device memory) and, alongside, the plain path and the oracle.
The "collisions" object times the tuned path again with the collision branch
of Eq. (2) on: particle radius from an optical depth of 0.5 over the ring's
area, r_coll = 2 radii, contact time 32 steps, restitution 0.5.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 19          # 3 sub, 3 fma, rsqrt, 3 mul, 3 fma (fma = 2 flops)
PAPER_FLOPS_PER_INTERACTION = 31    # the paper's count for a particle-cell interaction
FP32_PEAK_TFLOPS = 157.3
TARGET_P99 = 1e-3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def p99_nearest_rank(e):
    """The 99th percentile by nearest rank: the ceil(0.99 n)-th smallest of n values."""
    e = np.asarray(e)
    return float(np.sort(e)[int(math.ceil(0.99 * e.size)) - 1])


def rel_err_p99(ctx, dev, targets, ref, n):
    import torch
    # potentials requested too: the tuning launches use the potential-computing
    # variant of the force kernel, so per-kernel profiles of the timed variant
    # hold only timed-configuration launches
    out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az", "pot")}
    ctx.forces([out])
    a = torch.stack([out["ax"][targets], out["ay"][targets], out["az"][targets]])
    r = torch.stack([ref["ax"], ref["ay"], ref["az"]])
    e = (torch.linalg.vector_norm(a - r, dim=0) / torch.linalg.vector_norm(r, dim=0)).cpu().numpy()
    return p99_nearest_rank(e), float(np.median(e))


def tune_theta(ctx, dev, targets, ref, n, lo=0.1, hi=1.0, iters=10):
    """Largest theta (on a 2^-iters grid of [lo, hi]) with p99 <= TARGET_P99."""
    def p99(th):
        ctx.set_params(theta=th)
        ctx.make_lists()
        return rel_err_p99(ctx, dev, targets, ref, n)
    e_hi = p99(hi)
    if e_hi[0] <= TARGET_P99:
        return hi, e_hi
    best = (lo, p99(lo))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        e = p99(mid)
        if e[0] <= TARGET_P99:
            lo, best = mid, (mid, e)
        else:
            hi = mid
    return best[0], best[1]


def error_run(bh, w, dev0, sample, p, n_evals):
    """Force error of a configuration along its own trajectory (untimed):
    the run starts like the timed one, and after each of its first n_evals
    force evaluations the accelerations of that evaluation (the central
    planet's exact term taken back out: self-gravity only) are compared on
    the sample with the FP64 direct sum at the same positions.  Returns the
    p99 (nearest rank) and the median of each evaluation; evaluation k uses
    lists built k mod rebuild_every evaluations earlier."""
    import torch
    dev = {k: v.clone() for k, v in dev0.items()}
    ctx = bh.Context(theta=p["theta"], eps=w.eps, central_mass=w.central_mass, precision=p["precision"],
                     n_group=p["n_group"], cyl_radius=p.get("cyl_radius", 0.0))
    judge = bh.Context(theta=0.5, eps=w.eps)
    tg = sample.cpu().numpy()
    ref = {k: torch.zeros(sample.numel(), dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    gmc = w.central_mass * 1.0
    out, med = [], []
    ctx.step([dev], w.dt, 0, p["rebuild_every"])
    for k in range(n_evals):
        if k:
            ctx.step_continue(w.dt, 1, p["rebuild_every"])
        judge.direct_sum(dev, sample, ref)
        torch.cuda.synchronize()
        acc = ctx.export("acc_sorted")
        inv = np.empty(acc.shape[0], np.int64)
        inv[ctx.export("perm").astype(np.int64)] = np.arange(acc.shape[0])
        a = acc[inv[tg], :3]
        pos = np.stack([dev[f][sample].cpu().numpy() for f in ("x", "y", "z")], 1)
        a = a + gmc * pos / (np.sum(pos * pos, 1) ** 1.5)[:, None]
        r = np.stack([ref[f].cpu().numpy() for f in ("ax", "ay", "az")], 1)
        e = np.linalg.norm(a - r, axis=1) / np.linalg.norm(r, axis=1)
        out.append(p99_nearest_rank(e))
        med.append(float(np.median(e)))
        del acc
    ctx.close()
    judge.close()
    del dev
    torch.cuda.empty_cache()
    return out, med


GROUP_SIZES = (128, 256, 512)
LEARNED_BAND = (0.03, 0.5)


def learned_path(bh, inputs, w, dev0, sample, ref, n, tuned, args):
    """The learned opening rule: trained on separate 1M-particle rings and a
    Plummer sphere (seeds 100-102) with the library's training kernels, then
    tau bisected to p99 <= 1e-3 on the benchmark ring."""
    import torch
    lo, hi = LEARNED_BAND
    kw = dict(criterion=bh.LEARNED, theta_min=lo, theta_max=hi, tau=1e-4)
    tr = bh.Context(theta=tuned["theta"], eps=w.eps, precision=bh.FP32_REL, n_group=tuned["n_group"], **kw)
    for sysm in (inputs.ring(1 << 20, 100, central_mass=1.0),
                 inputs.ring(1 << 20, 101, r_out=1.2, z_sigma=5e-4, central_mass=1.0),
                 inputs.plummer(1 << 19, 102)):
        tr.build_tree([bh.to_device(sysm)])
        tr.mlp_collect(max_groups=256, count_cap=65536)
    n_pairs = tr.mlp_dataset()[0].shape[0]
    mse = tr.mlp_train(iters=3000, batch=4096, seed=7)
    weights = tr.mlp_weights()
    tr.close()
    torch.cuda.empty_cache()
    log(f"[bench] learned: {n_pairs} training pairs, mse {mse:.3f}")
    ctx = bh.Context(theta=tuned["theta"], eps=w.eps, precision=bh.FP32_REL, n_group=tuned["n_group"], **kw)
    ctx.mlp_weights(set=weights)
    ctx.build_tree([dev0])

    def err(lt):
        ctx.set_params(tau=10.0 ** lt)
        ctx.make_lists()
        return rel_err_p99(ctx, dev0, sample, ref, n)

    a, b, best = -9.0, 1.0, None
    for _ in range(12):
        mid = 0.5 * (a + b)
        e = err(mid)
        if e[0] <= TARGET_P99:
            a, best = mid, (mid, e)
        else:
            b = mid
    ctx.close()
    torch.cuda.empty_cache()
    lt, e = best
    log(f"[bench] learned: tau=1e{lt:.3f} p99={e[0]:.3e}")
    p = dict(tuned)
    p.update(learned=dict(kw, tau=10.0 ** lt), weights=weights, p99=e[0], p50=e[1], training_pairs=n_pairs,
             training_mse=mse, tree="cartesian", cyl_radius=0.0)     # the learned rule is Cartesian only
    return p


def collision_params(w, tau_opt=0.5, steps_per_contact=32, restitution=0.5):
    """Collision radius, spring and dashpot for the benchmark ring: equal
    particles of radius a with N pi a^2 = tau_opt * ring area, r_coll = 2a;
    kappa, eta of the damped oscillator (the relative motion of a contact)
    that lasts steps_per_contact steps and returns `restitution` of the
    approach speed."""
    s = w.systems[0]
    r_cyl = np.hypot(s.x, s.y)
    area = math.pi * (r_cyl.max() ** 2 - r_cyl.min() ** 2)
    a = math.sqrt(tau_opt * area / (math.pi * s.n))
    t_c = steps_per_contact * w.dt
    wd = math.pi / t_c
    gamma = -math.log(restitution) / t_c
    return dict(r_coll=2.0 * a, kappa=wd * wd + gamma * gamma, eta=2.0 * gamma), dict(
        optical_depth=tau_opt, t_contact=t_c, restitution=restitution)


REUSE_INTERVALS = (1, 2, 4, 8, 16)


def reuse_study(bh, w, dev0, sample, n, n_group, steps, cyl_radius=0.0, theta_lo=0.05, theta_hi=0.2, iters=7):
    """Interaction-list reuse (persistent lists): for each rebuild interval R,
    the loosest theta whose force error stays within p99 <= 1e-3 at every
    list age 0..R-1 of a cycle (positions moved by the leapfrog, moments
    refreshed, the judge recomputed at each age), then the time per step of
    that configuration.  Returns one record per R."""
    import torch
    judge = bh.Context(theta=0.5, eps=w.eps)
    gmc = w.central_mass * 1.0

    def cycle_errors(theta, R):
        dev = {k: v.clone() for k, v in dev0.items()}
        ctx = bh.Context(theta=theta, eps=w.eps, central_mass=w.central_mass, precision=bh.FP32_REL,
                         n_group=n_group, cyl_radius=cyl_radius)
        big = 1 << 30                         # never rebuild inside the cycle
        ctx.step([dev], w.dt, 0, big)
        errs = []
        for age in range(R):
            if age:
                ctx.step_continue(w.dt, 1, big)
            ref = {k: torch.zeros(sample.numel(), dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
            judge.direct_sum(dev, sample, ref)
            out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az", "pot")}
            ctx.forces([out])
            x, y, z = dev["x"][sample], dev["y"][sample], dev["z"][sample]
            r3 = (x * x + y * y + z * z) ** 1.5
            a = torch.stack([out["ax"][sample] + gmc * x / r3, out["ay"][sample] + gmc * y / r3,
                             out["az"][sample] + gmc * z / r3])
            r = torch.stack([ref["ax"], ref["ay"], ref["az"]])
            e = (torch.linalg.vector_norm(a - r, dim=0) / torch.linalg.vector_norm(r, dim=0)).cpu().numpy()
            errs.append(p99_nearest_rank(e))
        inter = ctx.query()["interactions"]
        ctx.close()
        del dev
        return errs, inter

    out = []
    for R in REUSE_INTERVALS:
        lo, hi, best = theta_lo, theta_hi, None
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            errs, inter = cycle_errors(mid, R)
            if max(errs) <= TARGET_P99:
                lo, best = mid, (mid, errs, inter)
            else:
                hi = mid
        if best is None:
            errs, inter = cycle_errors(theta_lo, R)
            best = (theta_lo, errs, inter)
        th, errs, inter = best
        # time `steps` cycles of this configuration
        dev = {k: v.clone() for k, v in dev0.items()}
        ctx = bh.Context(theta=th, eps=w.eps, central_mass=w.central_mass, precision=bh.FP32_REL, n_group=n_group,
                         cyl_radius=cyl_radius)
        ctx.step([dev], w.dt, 0, R)
        ctx.step_continue(w.dt, R, R)
        torch.cuda.synchronize()
        n_leap = max(R, (steps * 4 // R) * R)
        t0 = time.perf_counter()
        ctx.step_continue(w.dt, n_leap, R)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stage_times()
        ctx.close()
        del dev
        torch.cuda.empty_cache()
        rec = dict(rebuild_every=R, theta=th, p99_by_age=errs, interactions_per_force_eval_at_build=inter,
                   s_per_step=wall / n_leap, leapfrog_steps_timed=n_leap,
                   rebuild_ms=st["keys_sort"] + st["tree"] + st["moments"] + st["groups"] + st["walk"],
                   force_ms=st["forces"])
        log(f"[bench] reuse R={R}: theta={th:.4f} max p99={max(errs):.3e} s/step={rec['s_per_step']:.4f}")
        out.append(rec)
    judge.close()
    return out


def force_source_digest():
    src = os.path.join(ROOT, "paper_1907_02289_amd", "csrc", "bh_force.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(workload, n_group, theta, tree):
    """HBM bytes per force-kernel launch from the committed rocprofv3 counter
    summaries (one record per configuration), or None when none was taken on
    this workload, configuration and force-kernel source."""
    path = os.path.join(ROOT, "profiles", "force_kernel_traffic.json")
    try:
        recs = json.load(open(path))
    except (OSError, ValueError):
        return None
    for rec in (recs if isinstance(recs, list) else [recs]):
        if (rec.get("kernel_source_sha256_16") == force_source_digest() and rec.get("workload") == workload
                and rec.get("n_group") == n_group and rec.get("theta") == theta
                and rec.get("tree", "cartesian") == tree):
            return rec.get("hbm_bytes_per_launch")
    return None


def copy_calibration():
    """A plain device copy of known size (1 GiB read, 1 GiB written), three
    times, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "repeats": 3}))


def cpu_baseline(system, theta, n_grp, eps, rebuild_every, cyl_radius=0.0, n_sample_groups=16384, seed=0):
    """The oracle on the host cores: full tree build of the same ring (in the
    tuned path's tree coordinates), then walk + forces for a random sample of
    groups; interactions of the sample over the time of the sample's work
    (build prorated to the sample's share of groups and to one force
    evaluation of its reuse cycle)."""
    import oracle
    t0 = time.perf_counter()
    if cyl_radius > 0.0:
        _, _, _, key = oracle.keys_cyl(system.x, system.y, system.z, cyl_radius)
    else:
        _, _, _, key = oracle.keys(system.x, system.y, system.z)
    perm = oracle.sort_perm(key)
    skey = key[perm]
    t = oracle.tree(skey, 8)
    xs, ys, zs, ms = (a[perm] for a in (system.x, system.y, system.z, system.m))
    mom = oracle.moments(t, xs, ys, zs, ms)
    g = oracle.groups(t, n_grp)
    gbox, _ = oracle.group_boxes(g, t, skey, xs, ys, zs)
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(g.size, min(n_sample_groups, g.size), replace=False))
    t1 = time.perf_counter()
    pc_off, pc, pp_off, pp = oracle.lists(gbox[sel], t, theta, oracle.CYL_PERIOD if cyl_radius > 0.0 else 0)
    oracle.forces(g[sel], t, xs, ys, zs, ms, mom, pc_off, pc, pp_off, pp, eps)
    t_sample = time.perf_counter() - t1
    cnt = t["count"].astype(np.int64)
    pp_len = np.array([cnt[pp[pp_off[k]:pp_off[k + 1]]].sum() for k in range(sel.size)])
    inter = int(np.sum(cnt[g[sel]] * (pp_len + np.diff(pc_off))))
    share = sel.size / g.size
    t_total = t_sample + t_build * share / rebuild_every
    return dict(value=inter / t_total, unit="interactions/s", cores=oracle.n_threads(), kind="oracle",
                sample=(f"16M ring, theta={theta:.4f}, n_grp={n_grp}, "
                        f"{'cylindrical' if cyl_radius > 0.0 else 'Cartesian'} tree: oracle tree build of all {system.n} "
                        f"particles ({t_build:.1f} s, prorated {share:.4f} of groups / {rebuild_every} steps) "
                        f"+ walk and FP64 forces of {sel.size} random groups ({t_sample:.2f} s, "
                        f"{inter} interactions)"),
                seconds=t_build + t_sample)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed rebuild cycles (4 leapfrog steps each)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=4)
    ap.add_argument("--n", type=int, default=None, help="particle count override (default 2^24)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use theta = 0.5 for both paths")
    ap.add_argument("--n-group", type=int, default=256)
    ap.add_argument("--tree", choices=("auto", "cartesian", "cylindrical"), default="auto",
                    help="tree coordinates of the tuned path (auto: whichever is faster at matched error)")
    ap.add_argument("--theta-tuned", type=float, default=None, help="skip tuning, use this theta (tuned path)")
    ap.add_argument("--theta-plain", type=float, default=None, help="skip tuning, use this theta (plain path)")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy")
    ap.add_argument("--no-collisions", action="store_true", help="skip timing the collision branch")
    ap.add_argument("--match-along-run", action="store_true",
                    help="match theta on the largest p99 over the force evaluations of the error run (see "
                         "--error-evals) instead of on the first one")
    ap.add_argument("--error-evals", type=int, default=None,
                    help="force evaluations of the untimed runs that report each path's error along its "
                         "trajectory (default: through the last timed evaluation of the tuned path; 0: skip)")
    ap.add_argument("--reuse-study", action="store_true",
                    help="only the list-reuse study: matched-error theta and time per step for each rebuild interval")
    ap.add_argument("--learned", action="store_true",
                    help="also train, tune and time the learned-criterion form (off by default: its training-pair "
                         "collection is kept off the GPU after an unexplained silent test run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: sharding the groups "
              f"over several GPUs is a design, not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_02289_amd import bh, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration()
        return
    w = inputs.workload(3, n=args.n)
    sysm = w.systems[0]
    n = sysm.n
    R = w.rebuild_every
    if args.error_evals is None:
        # the first evaluation, the warm-up cycles and the timed cycles
        args.error_evals = 1 + R * (args.warmup + args.steps)
    log(f"[bench] ring n={n} rebuild_every={R}")
    dev0 = bh.to_device(sysm)
    sample = torch.as_tensor(inputs.force_sample(n, 3).astype(np.int64), device="cuda")

    # ---- judge: FP64 direct sum on the sample (self-gravity only)
    judge = bh.Context(theta=0.5, eps=w.eps)
    ref = {k: torch.zeros(sample.numel(), dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    t = time.perf_counter()
    judge.direct_sum(dev0, sample, ref)
    torch.cuda.synchronize()
    log(f"[bench] direct-sum judge on {sample.numel()} targets: {time.perf_counter() - t:.2f} s")
    judge.close()

    if args.reuse_study:
        r_cyl = np.hypot(sysm.x, sysm.y)
        cyl = 0.5 * float(r_cyl.min() + r_cyl.max()) if args.tree == "cylindrical" else 0.0
        recs = reuse_study(bh, w, dev0, sample, n, args.n_group, args.steps, cyl_radius=cyl)
        best = min(recs, key=lambda r: r["s_per_step"])
        print(json.dumps({"metric": "list-reuse study: s/step at matched p99 rel force err 1e-3 per rebuild interval",
                          "config": {"workload": f"ring{n}", "n_group": args.n_group, "eps": w.eps, "dt": w.dt,
                                     "tree_coordinates": "cylindrical" if cyl else "cartesian", "cyl_radius": cyl},
                          "fastest_rebuild_every": best["rebuild_every"], "records": recs}), flush=True)
        return

    # ---- matched error: theta per path (and per group size for the tuned path)
    paths = {
        "tuned": dict(precision=bh.FP32_REL, n_group=args.n_group, rebuild_every=R),
        "plain": dict(precision=bh.FP64, n_group=64, rebuild_every=1),
    }
    fixed = {"tuned": args.theta_tuned, "plain": args.theta_plain}
    group_sizes = [args.n_group] if (args.no_tune or args.theta_tuned is not None) else list(GROUP_SIZES)
    # tree coordinates of the tuned path: Cartesian, or cylindrical around the
    # ring's mid radius (Sec. 4.3)
    r_cyl = np.hypot(sysm.x, sysm.y)
    cyl_ref = 0.5 * float(r_cyl.min() + r_cyl.max())
    coords = {"cartesian": 0.0, "cylindrical": cyl_ref}
    tree_choices = [args.tree] if args.tree != "auto" else list(coords)
    autotune = []
    for name, p in paths.items():
        best = None
        for ng, tc in ([(g, t) for t in tree_choices for g in group_sizes] if name == "tuned"
                       else [(p["n_group"], "cartesian")]):
            ctx = bh.Context(theta=0.5, eps=w.eps, precision=p["precision"], n_group=ng, cyl_radius=coords[tc])
            ctx.build_tree([dev0])
            if args.no_tune or fixed[name] is not None:
                th = fixed[name] if fixed[name] is not None else 0.5
                ctx.set_params(theta=th)
                ctx.make_lists()
                e = rel_err_p99(ctx, dev0, sample, ref, n)
            else:
                th, e = tune_theta(ctx, dev0, sample, ref, n)
            ctx.set_params(theta=th)
            ctx.make_lists()
            inter = ctx.query()["interactions"]
            ctx.close()
            cost = None
            if name == "tuned" and len(group_sizes) * len(tree_choices) > 1:
                # cost at this theta where the timed region starts: the wall time
                # per leapfrog step of one rebuild cycle after the same warm-up
                cdev = {k: v.clone() for k, v in dev0.items()}
                cc = bh.Context(theta=th, eps=w.eps, central_mass=w.central_mass, precision=p["precision"],
                                n_group=ng, cyl_radius=coords[tc])
                cc.step([cdev], w.dt, 0, R)
                for _ in range(args.warmup):
                    cc.step_continue(w.dt, R, R)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                cc.step_continue(w.dt, R, R)
                torch.cuda.synchronize()
                cost = (time.perf_counter() - t0) * 1e3 / R
                cc.close()
                del cdev
            log(f"[bench] {name} n_group={ng} {tc}: theta={th:.4f} p99={e[0]:.3e}"
                + (f" cost {cost:.2f} ms per step after warm-up" if cost is not None else ""))
            if name == "tuned":
                autotune.append({"n_group": ng, "tree": tc, "theta": th, "p99": e[0],
                                 "interactions_per_force_eval": inter,
                                 "ms_per_step_after_warmup": cost})
            if best is None or (cost is not None and cost < best[0]):
                best = (cost, ng, th, e, tc)
            torch.cuda.empty_cache()
        p["n_group"], p["theta"], (p["p99"], p["p50"]), p["tree"] = best[1], best[2], best[3], best[4]
        p["cyl_radius"] = coords[best[4]]

    # ---- optionally: theta matched on the whole run, bisected below the
    # first-evaluation value (the error grows as the ring evolves)
    if args.match_along_run and args.error_evals > 0:
        for name, p in paths.items():
            hi = p["theta"]
            lo, best = 0.5 * hi, None
            e = error_run(bh, w, dev0, sample, p, args.error_evals)
            if max(e[0]) <= TARGET_P99:
                best = (hi, e)
            else:
                for _ in range(6):
                    mid = 0.5 * (lo + hi)
                    e = error_run(bh, w, dev0, sample, dict(p, theta=mid), args.error_evals)
                    log(f"[bench] {name}: theta {mid:.4f}: max p99 along the run {max(e[0]):.3e}")
                    if max(e[0]) <= TARGET_P99:
                        lo, best = mid, (mid, e)
                    else:
                        hi = mid
                if best is None:
                    best = (lo, error_run(bh, w, dev0, sample, dict(p, theta=lo), args.error_evals))
            log(f"[bench] {name}: theta {p['theta']:.4f} matched at the first evaluation, {best[0]:.4f} over "
                f"{args.error_evals} (max p99 {max(best[1][0]):.3e})")
            p["theta_first_eval"] = p["theta"]
            p["theta"] = best[0]
            p["p99"], p["p50"] = best[1][0][0], best[1][1][0]

    # ---- timed runs
    def timed(p, steps, warmup, leap_per_step):
        dev = {k: v.clone() for k, v in dev0.items()}
        ctx = bh.Context(theta=p["theta"], eps=w.eps, central_mass=w.central_mass, precision=p["precision"],
                         n_group=p["n_group"], cyl_radius=p.get("cyl_radius", 0.0), **p.get("learned", {}),
                         **p.get("contact", {}))
        if "weights" in p:
            ctx.mlp_weights(set=p["weights"])
        ctx.step([dev], w.dt, 0, p["rebuild_every"])
        for _ in range(warmup):
            ctx.step_continue(w.dt, leap_per_step, p["rebuild_every"])
        torch.cuda.synchronize()
        ctx.force_timing(reset=True)
        q0 = ctx.query()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.step_continue(w.dt, leap_per_step, p["rebuild_every"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        q1 = ctx.query()
        fms, fl = ctx.force_timing(reset=True)
        res = dict(wall=wall, interactions=q1["interactions_evaluated"] - q0["interactions_evaluated"],
                   force_evals=q1["force_evaluations"] - q0["force_evaluations"],
                   builds=q1["tree_builds"] - q0["tree_builds"], force_ms=fms, force_launches=fl,
                   n_groups=q1["n_groups"], n_nodes=q1["n_nodes"], stages=ctx.stage_times())
        ctx.close()
        del dev
        torch.cuda.empty_cache()
        return res

    tu = timed(paths["tuned"], args.steps, args.warmup, R)
    log(f"[bench] tuned: {tu}")
    lr = None
    if args.learned:
        lp = learned_path(bh, inputs, w, dev0, sample, ref, n, paths["tuned"], args)
        lr = timed(lp, max(1, args.steps // 2), 1, R)
        log(f"[bench] learned: {lr}")
    pl = timed(paths["plain"], args.plain_steps, 1, 1)
    log(f"[bench] plain: {pl}")
    co = None
    if not args.no_collisions:
        cparams, cinfo = collision_params(w)
        co_steps = max(2, args.steps // 2)
        co = timed(dict(paths["tuned"], contact=cparams), co_steps, 1, R)
        log(f"[bench] collisions {cparams}: {co}")

    errs = {}
    if args.error_evals > 0:
        for name in ("tuned", "plain"):
            errs[name] = error_run(bh, w, dev0, sample, paths[name], args.error_evals)[0]
            log(f"[bench] {name} path p99 over {len(errs[name])} force evaluations: max {max(errs[name]):.3e}")

    leap_t = tu["wall"] / (args.steps * R)
    leap_p = pl["wall"] / args.plain_steps
    value = tu["interactions"] / tu["wall"]
    per_launch = tu["interactions"] / max(1, tu["force_evals"])
    avg_ms = tu["force_ms"] / max(1, tu["force_launches"])
    achieved = per_launch * FLOPS_PER_INTERACTION / (avg_ms * 1e-3) / 1e12
    workload = f"ring{n}_reuse{R}"

    out = {
        "metric": "interactions/s & s/step, 16M ring, p99 rel force err 1e-3: tuned vs plain GPU BH",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tu["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "n_particles": n, "theta_tuned": paths["tuned"]["theta"], "theta_plain": paths["plain"]["theta"],
            "eps": w.eps, "dt": w.dt, "rebuild_every": R, "n_group": paths["tuned"]["n_group"],
            "tree_coordinates": paths["tuned"]["tree"], "cyl_radius": paths["tuned"]["cyl_radius"],
            "step": f"one rebuild cycle = {R} KDK steps", "positions_and_integration": "f64",
            "theta_matched_on": (f"largest p99 over the first {args.error_evals} force evaluations"
                                 if "theta_first_eval" in paths["tuned"] else "first force evaluation"),
        },
        "s_per_leapfrog_step": leap_t,
        "interactions_per_force_eval": per_launch,
        "p99_rel_err": paths["tuned"]["p99"], "p50_rel_err": paths["tuned"]["p50"],
        "plain": {"s_per_step": leap_p, "interactions_per_s": pl["interactions"] / pl["wall"],
                  "p99_rel_err": paths["plain"]["p99"], "dtype": "f64", "n_group": 64, "rebuild_every": 1},
        "speedup_vs_plain_s_per_step": leap_p / leap_t,
        "group_size_autotune": autotune,
        "force_kernel_ms": avg_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic(workload, paths["tuned"]["n_group"], paths["tuned"]["theta"],
                                                 paths["tuned"]["tree"]),
                     "flops_per_interaction": FLOPS_PER_INTERACTION,
                     "frac_at_paper_31_flops": achieved * PAPER_FLOPS_PER_INTERACTION / FLOPS_PER_INTERACTION
                     / FP32_PEAK_TFLOPS},
        "stages_ms_last": tu["stages"],
    }
    for name in ("tuned", "plain"):
        if "theta_first_eval" in paths[name]:
            out["config"][f"theta_{name}_matched_at_first_eval"] = paths[name]["theta_first_eval"]
    if errs:
        # the error along each path's run (theta as matched above), per
        # evaluation and as the maximum over each of the tuned path's rebuild
        # cycles
        out["p99_along_run"] = {
            name: {"per_force_eval": e, "max_per_4_evals": [max(e[i:i + R]) for i in range(0, len(e), R)],
                   "max": max(e)} for name, e in errs.items()}
        out["p99_along_run"]["target"] = TARGET_P99
    if co is not None:
        c_launch = co["interactions"] / max(1, co["force_evals"])
        c_ms = co["force_ms"] / max(1, co["force_launches"])
        c_ach = c_launch * FLOPS_PER_INTERACTION / (c_ms * 1e-3) / 1e12
        out["collisions"] = dict(cparams, **cinfo, s_per_step=co["wall"] / (co_steps * R),
                                 interactions_per_s=co["interactions"] / co["wall"],
                                 interactions_per_force_eval=c_launch, force_kernel_ms=c_ms,
                                 force_kernel_ms_ratio_vs_gravity_only=c_ms / avg_ms,
                                 achieved_tflops_19=c_ach, frac=c_ach / FP32_PEAK_TFLOPS)
    if lr is not None:
        lps = lr["wall"] / (max(1, args.steps // 2) * R)
        out["learned"] = {"s_per_step": lps, "interactions_per_s": lr["interactions"] / lr["wall"],
                          "interactions_per_force_eval": lr["interactions"] / max(1, lr["force_evals"]),
                          "tau": lp["learned"]["tau"], "p99_rel_err": lp["p99"], "p50_rel_err": lp["p50"],
                          "training_pairs": lp["training_pairs"], "training_mse": lp["training_mse"],
                          "speedup_vs_plain_s_per_step": leap_p / lps,
                          "interactions_vs_geometric": (lr["interactions"] / max(1, lr["force_evals"])) / per_launch}
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sysm, paths["tuned"]["theta"], paths["tuned"]["n_group"], w.eps, R,
                                           paths["tuned"]["cyl_radius"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
