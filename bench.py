"""Benchmark: Barnes-Hut force path on one MI355X, 16M-particle ring.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 2^24-particle thin ring (r in [1.0, 1.2], z ~ N(0, 5e-4),
central unit mass, Keplerian velocities with 1e-4 dispersion), eps = 1e-4,
dt = 1e-3.  A benchmark step is one kick-drift-kick step: one force
evaluation with its share of tree and list builds.  The run starts with a
force evaluation at t = 0 (bh_step with no steps), then W warm-up steps,
then the K timed steps.

Matched error.  For each path the opening parameter is set to the loosest
value whose force error stays within p99 <= 1e-3 at EVERY force evaluation
of the run through the last timed one (the 99th percentile, nearest rank, of
|a - a_direct| / |a_direct| over 4096 sampled particles, self-gravity only,
against the library's FP64 direct sum at the same positions).  Each trial
value is a full untimed run from t = 0; the matched run's per-evaluation
errors are the ones reported.
  tuned:   FP32 interactions on group-relative coordinates; rebuild policy
           (lists reused until the drift monitor asks for a rebuild, at most
           4 or 16 steps, or rebuilt every 2 steps), group configuration
           (size, packed small siblings, tree on Cartesian or cylindrical
           coordinates) and force tile chosen by measured time per step at
           matched error; reuse steps replayed from a HIP graph;
  plain:   FP64 interactions, groups <= 64, lists rebuilt every step;
  learned: the tuned path (on a Cartesian tree) with the learned opening
           rule (network trained on the GPU by the library's kernels on
           separate rings and a Plummer sphere), its budget tau matched the
           same way.
The JSON line reports the tuned path's interactions/s (whole job, inputs
resident in device memory, timed window only) and, alongside, the plain and
learned paths on the same steps, the collision branch of Eq. (2), the
batched 64-Plummer-sphere workload, and the oracle on the host cores.
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
FP64_PEAK_TFLOPS = 78.6
TARGET_P99 = 1e-3
CYL_RADIUS = 1.1                    # mid radius of the benchmark ring (r in [1, 1.2])
# A candidate of the tuned path's autotuning replaces the incumbent (the first
# of its list) only when it is faster by more than this fraction: times differ
# by ~1-2% from one MI355X to another, and the choice should not follow that.
MARGIN = 0.02
# group configurations of the tuned path (group size, packed small siblings,
# tree on cylindrical coordinates around the ring's mid radius), each matched
# along the run and timed; the first is the one the rebuild policy is chosen on
GROUP_CONFIGS = ((384, True, True), (384, True, False), (256, True, True), (512, True, True), (256, True, False),
                 (512, True, False), (384, False, False))
REUSE_MAX = 16                      # longest list age of the tuned path
# drift monitor of the tuned path: rebuild when, at some tree level, nodes
# whose particles moved by more than their side relative to the node's centre
# of mass since the build hold more than 10% of the particles (on the 16M ring
# this keeps the largest p99 along a 101-evaluation run at that of lists
# rebuilt every step, with 39% of the builds)
DRIFT = dict(reuse_drift=1.0, reuse_frac=0.1)
# rebuild policies the tuned path chooses from by measured time at matched
# error (name, command-line key, parameters): the monitor guards the error of
# aged lists, its age cap trades the cost of builds against that of lists
# built for an older state of the ring
POLICIES = (("drift monitor, lists at most 4 steps old", "drift4", dict(rebuild_every=4, drift=DRIFT)),
            ("drift monitor, lists at most 16 steps old", "drift16", dict(rebuild_every=REUSE_MAX, drift=DRIFT)),
            ("every 2 steps", "every2", dict(rebuild_every=2)))
LEARNED_BAND = (0.03, 0.5)
THETA_FLOOR = 0.02


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def p99_nearest_rank(e):
    """The 99th percentile by nearest rank: the ceil(0.99 n)-th smallest of n values."""
    e = np.asarray(e)
    return float(np.sort(e)[int(math.ceil(0.99 * e.size)) - 1])


class Judge:
    """Force error of a context's last evaluation on the sample, on the
    device: the library's FP64 direct sum at the caller's current positions
    against the sampled accelerations (bh_sample_acc) with the central
    planet's exact term taken back out."""

    def __init__(self, bh, w, sample):
        import torch
        self.torch = torch
        self.ctx = bh.Context(theta=0.5, eps=w.eps)
        self.sample = sample
        self.gm = w.central_mass
        z = lambda: torch.zeros(sample.numel(), dtype=torch.float64, device="cuda")
        self.ref = {k: z() for k in ("ax", "ay", "az")}
        self.got = {k: z() for k in ("ax", "ay", "az")}
        self.k = int(math.ceil(0.99 * sample.numel()))

    def reference(self, dev):
        self.ctx.direct_sum(dev, self.sample, self.ref)

    def errors(self, ctx, dev, fresh_reference=True):
        torch = self.torch
        if fresh_reference:
            self.reference(dev)
        ctx.sample_acc(self.sample, self.got)
        x, y, z = (dev[f][self.sample] for f in ("x", "y", "z"))
        r3 = (x * x + y * y + z * z) ** 1.5
        a = torch.stack([self.got["ax"] + self.gm * x / r3, self.got["ay"] + self.gm * y / r3,
                         self.got["az"] + self.gm * z / r3])
        r = torch.stack([self.ref["ax"], self.ref["ay"], self.ref["az"]])
        e = torch.linalg.vector_norm(a - r, dim=0) / torch.linalg.vector_norm(r, dim=0)
        s = torch.sort(e).values
        return float(s[self.k - 1]), float(s[(s.numel() - 1) // 2])

    def close(self):
        self.ctx.close()


def make_ctx(bh, w, p):
    kw = dict(theta=p["theta"], eps=w.eps, central_mass=w.central_mass, precision=p["precision"],
              n_group=p["n_group"], cyl_radius=p.get("cyl_radius", 0.0), force_tile=p.get("force_tile", 0),
              pack_groups=p.get("pack_groups", False))
    kw.update(p.get("drift", {}))
    kw.update(p.get("learned", {}))
    kw.update(p.get("contact", {}))
    ctx = bh.Context(**kw)
    if "weights" in p:
        ctx.mlp_weights(set=p["weights"])
    return ctx


def error_run(bh, w, dev0, judge, p, n_evals, timed_from=None):
    """The run of configuration p from t = 0 through n_evals force
    evaluations (untimed): after each evaluation its sampled accelerations
    are judged against the direct sum.  Also returns the device time of each
    leapfrog step (HIP events around the step) from evaluation timed_from on,
    and the number of tree builds."""
    import torch
    dev = {k: v.clone() for k, v in dev0.items()}
    ctx = make_ctx(bh, w, p)
    ctx.step([dev], w.dt, 0, p["rebuild_every"])
    p99, p50, step_ms = [], [], []
    # per evaluation: force-kernel device time, interactions of the lists
    # used, group count; walk time of each tree build (evaluation index, ms)
    force_ms, inter, groups, walk_ms = [], [], [], []
    builds = 0

    def record(k):
        nonlocal builds
        e = judge.errors(ctx, dev)
        p99.append(e[0])
        p50.append(e[1])
        q, st = ctx.query(), ctx.stage_times()
        force_ms.append(st["forces"])
        inter.append(q["interactions"])
        groups.append(q["n_groups"])
        if q["tree_builds"] > builds:
            walk_ms.append((k, st["walk"]))
            builds = q["tree_builds"]

    record(0)
    for k in range(1, n_evals):
        ctx.step_continue(w.dt, 1, p["rebuild_every"])
        if timed_from is not None and k >= timed_from:
            step_ms.append(ctx.stage_times()["step"])
        record(k)
    q = ctx.query()
    ctx.close()
    del dev
    torch.cuda.empty_cache()
    return dict(p99=p99, p50=p50, max=max(p99), step_ms=step_ms, builds=q["tree_builds"],
                drift_rebuilds=q["drift_rebuilds"], interactions=q["interactions_evaluated"],
                force_ms=force_ms, inter=inter, groups=groups, walk_ms=walk_ms)


def first_eval_theta(bh, w, dev0, judge, p, lo=THETA_FLOOR, hi=1.0, iters=10):
    """Largest theta (on a 2^-iters grid of [lo, hi]) with p99 <= 1e-3 at the
    first force evaluation, fresh lists.  Raises if even lo misses."""
    ctx = make_ctx(bh, w, dict(p, theta=hi))
    ctx.build_tree([dev0])
    judge.reference(dev0)

    def p99(th):
        ctx.set_params(theta=th)
        ctx.make_lists()
        ctx.forces(None)
        return judge.errors(ctx, dev0, fresh_reference=False)[0]

    try:
        if p99(hi) <= TARGET_P99:
            return hi
        ok = None
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if p99(mid) <= TARGET_P99:
                lo = ok = mid
            else:
                hi = mid
        if ok is None:
            # every trial missed: the floor itself decides (small theta means
            # long lists: a failure to allocate them is a miss as well)
            try:
                missed = p99(lo) > TARGET_P99
            except bh.BHError:
                missed = True
            if missed:
                raise RuntimeError(f"theta {lo} misses p99 <= {TARGET_P99} at the first evaluation")
        return lo
    finally:
        ctx.close()


def first_eval_tau(bh, w, dev0, judge, p, lo=-10.0, hi=0.0, iters=12):
    """Largest tau (log10 on a 2^-iters grid of [lo, hi]) of the learned rule
    with p99 <= 1e-3 at the first force evaluation."""
    ctx = make_ctx(bh, w, p)
    ctx.build_tree([dev0])
    judge.reference(dev0)

    def p99(lt):
        ctx.set_params(tau=10.0 ** lt)
        ctx.make_lists()
        ctx.forces(None)
        return judge.errors(ctx, dev0, fresh_reference=False)[0]

    try:
        ok = None
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if p99(mid) <= TARGET_P99:
                lo = ok = mid
            else:
                hi = mid
        if ok is None and p99(lo) > TARGET_P99:
            raise RuntimeError(f"learned: tau 1e{lo} misses p99 <= {TARGET_P99} at the first evaluation")
        return 10.0 ** lo
    finally:
        ctx.close()


def match_along_run(name, run, x0, alpha, floor, max_runs=6, tol=0.015, guess=None):
    """Largest x <= x0 (theta, or the learned rule's tau) whose run keeps
    p99 <= 1e-3 at every evaluation; the error grows with x.  Starts at
    `guess` (default x0); secant steps on log(max p99) against log(x), a
    power law of exponent alpha (or, after two misses, of the slope between
    them) until two points bracket the target; at most
    max_runs runs.  Returns (x, run record); raises when no trial down to the
    floor meets the target."""
    seen = {}
    ok = bad = None
    x = min(guess, x0) if guess else x0
    for it in range(max_runs):
        r = run(x)
        seen[x] = r
        log(f"[bench] {name}: {x:.6g} -> max p99 along the run {r['max']:.4e} ({r['builds']} tree builds)")
        if r["max"] <= TARGET_P99:
            ok = x if ok is None else max(ok, x)
        else:
            bad = x if bad is None else min(bad, x)
        if ok is not None and bad is not None:
            if (bad - ok) / bad < tol:
                break
            m_ok, m_bad = seen[ok]["max"], seen[bad]["max"]
            slope = math.log(m_bad / m_ok) / math.log(bad / ok) if m_bad > m_ok else alpha
            xn = ok * (0.99 * TARGET_P99 / m_ok) ** (1.0 / max(slope, 0.25))
            x = min(max(xn, ok + 0.2 * (bad - ok)), bad - 0.2 * (bad - ok))
        elif ok is not None:
            if ok >= x0:
                break
            xn = min(x0, ok * (0.99 * TARGET_P99 / seen[ok]["max"]) ** (1.0 / alpha))
            if xn <= ok * (1.0 + tol):
                break
            x = xn
        else:
            # only misses so far: the power law through the two smallest
            # misses once there are two, else the assumed exponent
            slope = alpha
            miss = sorted(seen)[:2]
            if len(miss) == 2 and seen[miss[1]]["max"] > seen[miss[0]]["max"]:
                slope = max(0.25, math.log(seen[miss[1]]["max"] / seen[miss[0]]["max"]) / math.log(miss[1] / miss[0]))
            xn = bad * (0.97 * TARGET_P99 / seen[bad]["max"]) ** (1.0 / slope)
            if xn <= floor:
                if bad <= floor:
                    raise RuntimeError(f"{name}: p99 {seen[bad]['max']:.3e} > {TARGET_P99} at the floor {floor}")
                xn = floor
            x = xn
    if ok is None:
        raise RuntimeError(f"{name}: no setting within {max_runs} runs keeps p99 <= {TARGET_P99}")
    return ok, seen[ok]


def timed(bh, w, dev0, p, steps, warmup):
    """Wall time of `steps` leapfrog steps after `warmup` ones (from the same
    t = 0 start as the error runs), with HIP-event force-kernel times."""
    import torch
    dev = {k: v.clone() for k, v in dev0.items()}
    ctx = make_ctx(bh, w, p)
    ctx.step([dev], w.dt, 0, p["rebuild_every"])
    if warmup:
        ctx.step_continue(w.dt, warmup, p["rebuild_every"])
    torch.cuda.synchronize()
    ctx.force_timing(reset=True)
    q0 = ctx.query()
    t0 = time.perf_counter()
    ctx.step_continue(w.dt, steps, p["rebuild_every"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q1 = ctx.query()
    fms, fl = ctx.force_timing(reset=True)
    res = dict(wall=wall, interactions=q1["interactions_evaluated"] - q0["interactions_evaluated"],
               force_evals=q1["force_evaluations"] - q0["force_evaluations"],
               builds=q1["tree_builds"] - q0["tree_builds"], force_ms=fms, force_launches=fl,
               host_syncs=q1["host_syncs"] - q0["host_syncs"],
               n_groups=q1["n_groups"], n_nodes=q1["n_nodes"], stages=ctx.stage_times())
    ctx.close()
    del dev
    torch.cuda.empty_cache()
    return res


def train_learned(bh, inputs, w, n_group, theta, band=LEARNED_BAND):
    """The learned rule's network, trained by the library's kernels on pairs
    it collects from separate 1M-particle rings and a Plummer sphere
    (seeds 100-102, disjoint from the benchmark ring's); training pairs are
    the (group, node) pairs of the band."""
    import torch
    lo, hi = band
    tr = bh.Context(theta=theta, eps=w.eps, precision=bh.FP32_REL, n_group=n_group, criterion=bh.LEARNED,
                    theta_min=lo, theta_max=hi, tau=1e-4)
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
    return weights, n_pairs, mse


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


def batched_leg(bh, inputs, steps, pack=None):
    """The batched workload: 64 Plummer spheres (N log-uniform in [1e3,
    2e5]) in one context, one launch per stage, FP32, theta 0.6, eps 1e-2,
    rebuilt every step, group size and force tile autotuned by bh_autotune;
    `steps` leapfrog steps timed after one warm-up step.  pack=None times
    tree-node and packed groups and keeps the faster (the workload sets no
    error target; packing moves the error of a given theta by little)."""
    import torch
    if pack is None:
        runs = [batched_leg(bh, inputs, steps, pk) for pk in (False, True)]
        best = min(runs, key=lambda r: r["s_per_step"])
        best["s_per_step_by_packing"] = {("packed" if r["pack_groups"] else "tree-node groups"): r["s_per_step"]
                                         for r in runs}
        return best
    w2 = inputs.workload(2)
    devs = [bh.to_device(s) for s in w2.systems]
    n_tot = sum(s.n for s in w2.systems)
    ctx = bh.Context(theta=w2.theta, eps=w2.eps, precision=bh.FP32_REL, n_group=128, pack_groups=pack)
    ctx.build_tree(devs)
    chosen = ctx.autotune(candidates=(32, 64, 128, 256, 512), rebuild_every=1)
    tile = ctx.query()["force_tile"]
    ctx.close()
    ctx = bh.Context(theta=w2.theta, eps=w2.eps, precision=bh.FP32_REL, n_group=chosen, force_tile=tile,
                     pack_groups=pack)
    ctx.step(devs, w2.dt, 1, 1)
    torch.cuda.synchronize()
    ctx.force_timing(reset=True)
    q0 = ctx.query()
    t0 = time.perf_counter()
    ctx.step_continue(w2.dt, steps, 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q1 = ctx.query()
    fms, fl = ctx.force_timing(reset=True)
    st = ctx.stage_times()
    ctx.close()
    inter = q1["interactions_evaluated"] - q0["interactions_evaluated"]
    return dict(workload=f"plummer64_batched_{n_tot}", n_systems=len(w2.systems), n_particles=n_tot,
                theta=w2.theta, eps=w2.eps, dt=w2.dt, rebuild_every=1, n_group=chosen, pack_groups=pack,
                force_tile=tile, steps=steps,
                s_per_step=wall / steps, interactions_per_s=inter / wall,
                force_kernel_ms=fms / max(1, fl), force_share_of_step=fms / (wall * 1e3),
                interactions_per_step=inter / steps,
                host_syncs_per_step=(q1["host_syncs"] - q0["host_syncs"]) / steps,
                tree_builds_per_step=(q1["tree_builds"] - q0["tree_builds"]) / steps,
                stages_ms_last=st)


def force_source_digest():
    """Digest of the force kernel's source and of the walk's (which sets the
    order the kernel takes its groups in)."""
    h = hashlib.sha256()
    for f in ("bh_force.hip", "bh_walk.hip"):
        h.update(open(os.path.join(ROOT, "paper_1907_02289_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, n_group, theta):
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
                and rec.get("n_group") == n_group and abs(rec.get("theta", -1) - theta) <= 1e-12):
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


def cpu_baseline(system, theta, n_grp, eps, n_sample_groups=16384, seed=0, cyl_r=0.0, pack=False):
    """The oracle on the host cores, in the tuned path's tree and group
    configuration: full tree build of the same ring, then walk + forces for
    a random sample of groups; interactions of the sample over the time of
    the sample's work (the build prorated to the sample's share of groups)."""
    import oracle
    t0 = time.perf_counter()
    if cyl_r > 0.0:
        _, _, _, key = oracle.keys_cyl(system.x, system.y, system.z, cyl_r)
    else:
        _, _, _, key = oracle.keys(system.x, system.y, system.z)
    perm = oracle.sort_perm(key)
    skey = key[perm]
    t = oracle.tree(skey, 8)
    xs, ys, zs, ms = (a[perm] for a in (system.x, system.y, system.z, system.m))
    mom = oracle.moments(t, xs, ys, zs, ms)
    if pack:
        g, gbeg, gcnt = oracle.groups_packed(t, n_grp)
    else:
        g = oracle.groups(t, n_grp)
        gbeg, gcnt = t["begin"][g], t["count"][g]
    gbox, _ = oracle.group_boxes(np.arange(g.size, dtype=np.uint32), dict(begin=gbeg, count=gcnt), skey,
                                 xs, ys, zs)
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(g.size, min(n_sample_groups, g.size), replace=False))
    t1 = time.perf_counter()
    pc_off, pc, pp_off, pp = oracle.lists(gbox[sel], t, theta, oracle.CYL_PERIOD if cyl_r > 0.0 else 0)
    oracle.forces(g[sel], t, xs, ys, zs, ms, mom, pc_off, pc, pp_off, pp, eps, granges=(gbeg[sel], gcnt[sel]))
    t_sample = time.perf_counter() - t1
    cnt = t["count"].astype(np.int64)
    pp_len = np.array([cnt[pp[pp_off[k]:pp_off[k + 1]]].sum() for k in range(sel.size)])
    inter = int(np.sum(gcnt[sel].astype(np.int64) * (pp_len + np.diff(pc_off))))
    share = sel.size / g.size
    t_total = t_sample + t_build * share
    tree = f"cylindrical tree (r_ref {cyl_r:g})" if cyl_r > 0.0 else "Cartesian tree"
    return dict(value=inter / t_total, unit="interactions/s", cores=oracle.n_threads(), kind="oracle",
                sample=(f"16M ring at t = 0, theta={theta:.4f}, n_grp={n_grp}{', packed' if pack else ''}, "
                        f"{tree}: oracle tree build "
                        f"of all {system.n} particles ({t_build:.1f} s, prorated {share:.4f} of groups) + walk and "
                        f"FP64 forces of {sel.size} random groups ({t_sample:.2f} s, {inter} interactions)"),
                seconds=t_build + t_sample)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed leapfrog steps")
    ap.add_argument("--warmup", type=int, default=5, help="leapfrog steps before the timed ones")
    ap.add_argument("--n", type=int, default=None, help="particle count override (default 2^24)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--legs", default="tuned,plain,learned,collisions,batched",
                    help="comma-separated legs to run (tuned always runs, unless the batched leg runs alone)")
    ap.add_argument("--n-group", type=int, default=None, help="tuned path group size (default: autotuned)")
    ap.add_argument("--cyl", choices=("on", "off"), default=None,
                    help="tuned path: tree on cylindrical coordinates (default: autotuned)")
    ap.add_argument("--pack", choices=("on", "off"), default=None,
                    help="pack small sibling groups, tuned path or (with --legs batched alone) the batched "
                         "workload (default: autotuned)")
    ap.add_argument("--policy", choices=[pl[1] for pl in POLICIES], default=None,
                    help="tuned path rebuild policy: the drift monitor with lists at most 16 or 4 steps old, or "
                         "lists rebuilt every 2 steps (default: the fastest at matched error)")
    ap.add_argument("--tile", type=int, default=None, choices=(256, 512),
                    help="tuned path force tile (default: autotuned)")
    ap.add_argument("--theta-tuned", type=float, default=None, help="skip matching, use this theta (tuned path)")
    ap.add_argument("--theta-plain", type=float, default=None, help="skip matching, use this theta (plain path)")
    ap.add_argument("--tau-learned", type=float, default=None, help="skip matching, use this tau (learned path)")
    ap.add_argument("--learned-band", type=float, nargs=2, default=LEARNED_BAND, metavar=("LO", "HI"),
                    help="learned rule: the band of side/distance in which the network decides")
    ap.add_argument("--learned-budget", choices=("mean", "min"), default="mean",
                    help="the learned rule's budget scale A_g: mean or smallest |a| of a group's particles")
    ap.add_argument("--no-error-runs", action="store_true",
                    help="with fixed parameters: skip the untimed runs that report the error along the run")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy")
    ap.add_argument("--reuse-configs", default=None,
                    help="reuse study: comma-separated subset of R=1,R=2,R=4,R=8,R=16,drift, or drift:<kappa>:<frac>[:<cap>]; "
                         "a +pack suffix packs small sibling groups, +cyl builds cylindrical trees")
    ap.add_argument("--reuse-study", action="store_true",
                    help="only the list-reuse study: fixed rebuild intervals and the drift monitor, each matched "
                         "along the run, and their time per step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: sharding the groups "
              f"over several GPUs is a design, not implemented.", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    if legs != {"batched"}:
        legs |= {"tuned"}

    import torch
    from paper_1907_02289_amd import bh, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration()
        return
    w = inputs.workload(3, n=args.n)
    sysm = w.systems[0]
    n = sysm.n
    n_evals = 1 + args.warmup + args.steps
    log(f"[bench] ring n={n}, {args.warmup} warm-up + {args.steps} timed leapfrog steps ({n_evals} force evaluations)")
    dev0 = bh.to_device(sysm)
    sample = torch.as_tensor(inputs.force_sample(n, 3).astype(np.int64), device="cuda")
    judge = Judge(bh, w, sample)
    t = time.perf_counter()
    judge.reference(dev0)
    torch.cuda.synchronize()
    log(f"[bench] direct-sum judge on {sample.numel()} targets: {time.perf_counter() - t:.3f} s")

    if args.reuse_study:
        reuse_study(bh, w, dev0, judge, n, args)
        return
    if legs == {"batched"}:
        # the batched workload alone (for a profile of that leg)
        pack = None if args.pack is None else args.pack == "on"
        print(json.dumps({"batched": batched_leg(bh, inputs, args.steps, pack)}), flush=True)
        return

    paths = {}
    autotune = []
    fixed_run = args.no_error_runs

    # ---- tuned path: first the rebuild policy (drift monitor or a fixed
    # interval), each with its own theta matched along the run, by measured
    # time per step; then the group configuration (size, packing, Cartesian
    # or cylindrical tree), each matched along the run (the error at a given
    # theta moves with the group boxes and the tree) and timed; last the force
    # tile, a changed choice checked by an error run of its own
    gcands = [(ng, pk, cy) for ng, pk, cy in GROUP_CONFIGS
              if args.n_group in (None, ng) and args.pack in (None, "on" if pk else "off")
              and args.cyl in (None, "on" if cy else "off")]
    if not gcands:
        gcands = [(args.n_group or 384, args.pack == "on", args.cyl == "on")]
    policies = [pl for pl in POLICIES if args.policy in (None, pl[1])]
    base = r = None
    policy_autotune = []
    th0 = None
    for pname, pkey, pol in policies:
        cand = dict(precision=bh.FP32_REL, n_group=gcands[0][0], pack_groups=gcands[0][1],
                    cyl_radius=CYL_RADIUS if gcands[0][2] else 0.0,
                    force_tile=args.tile or 512, policy=pname, policy_key=pkey,
                    **{k: (dict(v) if isinstance(v, dict) else v) for k, v in pol.items()})
        rc = None
        if args.theta_tuned is not None:
            cand["theta"] = args.theta_tuned
        else:
            if th0 is None:
                th0 = first_eval_theta(bh, w, dev0, judge, cand)
            cand["theta_first_eval"] = th0
            cand["theta"], rc = match_along_run(
                f"tuned {pname} n_group={cand['n_group']} theta",
                lambda th: error_run(bh, w, dev0, judge, dict(cand, theta=th), n_evals, 1 + args.warmup),
                th0, 2.0, THETA_FLOOR, guess=base["theta"] if base else None)
        if len(policies) > 1:
            t = timed(bh, w, dev0, cand, args.steps, args.warmup)
            cost = t["wall"] / args.steps * 1e3
            policy_autotune.append(dict(policy=pname, theta=cand["theta"], ms_per_step=cost, builds=t["builds"]))
            log(f"[bench] tuned {pname}: theta={cand['theta']:.5f} {cost:.2f} ms/step, {t['builds']} builds")
            if base is not None and cost >= base_cost * (1.0 - MARGIN):
                continue
            base_cost = cost
        base, r = cand, rc
    best = None
    best_cart = None           # the fastest Cartesian candidate: the learned rule's geometric reference
    for ng, pk, cy in gcands if len(gcands) > 1 else []:
        p = dict(base, n_group=ng, pack_groups=pk, cyl_radius=CYL_RADIUS if cy else 0.0)
        rp = r if (ng, pk, p["cyl_radius"]) == (base["n_group"], base["pack_groups"], base["cyl_radius"]) else None
        label = f"n_group={ng}{' packed' if pk else ''}{' cylindrical' if cy else ''}"
        if rp is None and args.theta_tuned is None:
            p["theta"], rp = match_along_run(
                f"tuned {label} theta",
                lambda th: error_run(bh, w, dev0, judge, dict(p, theta=th), n_evals, 1 + args.warmup),
                base["theta_first_eval"], 2.0, THETA_FLOOR, guess=base["theta"])
        t = timed(bh, w, dev0, p, args.steps, args.warmup)
        cost = t["wall"] / args.steps * 1e3
        autotune.append(dict(n_group=ng, pack_groups=pk, cylindrical=cy, force_tile=p["force_tile"],
                             theta=p["theta"], ms_per_step=cost, max_p99=rp["max"] if rp else None))
        log(f"[bench] tuned {label} theta={p['theta']:.5f}: {cost:.2f} ms/step")
        if best is None or cost < best[0] * (1.0 - MARGIN):
            best = (cost, p, rp)
        if not cy and (best_cart is None or cost < best_cart[0]):
            best_cart = (cost, p)
    if best is not None:
        _, base, r = best
    p = base
    if not args.tile:
        q = dict(p, force_tile=256 if p["force_tile"] == 512 else 512)
        t0 = best[0] if best else timed(bh, w, dev0, p, args.steps, args.warmup)["wall"] / args.steps * 1e3
        t = timed(bh, w, dev0, q, args.steps, args.warmup)
        cost = t["wall"] / args.steps * 1e3
        autotune.append(dict(n_group=q["n_group"], pack_groups=q["pack_groups"], cylindrical=q["cyl_radius"] > 0,
                             force_tile=q["force_tile"], theta=q["theta"], ms_per_step=cost, max_p99=None))
        log(f"[bench] tuned tile={q['force_tile']}: {cost:.2f} ms/step (tile {p['force_tile']}: {t0:.2f})")
        if cost < t0 * (1.0 - MARGIN):
            p = q
    if r is None or p is not base:
        if not fixed_run:
            r2 = error_run(bh, w, dev0, judge, p, n_evals, 1 + args.warmup)
            if r is not None and r2["max"] > TARGET_P99:
                log(f"[bench] tile={p['force_tile']}: max p99 {r2['max']:.3e} misses; keeping tile {base['force_tile']}")
                p = base
            else:
                r = r2
    paths["tuned"] = dict(p, run=r)

    # ---- plain path: FP64, groups <= 64, rebuilt every step
    if "plain" in legs:
        p = dict(precision=bh.FP64, n_group=64, rebuild_every=1)
        if args.theta_plain is not None:
            p["theta"] = args.theta_plain
            r = None if fixed_run else error_run(bh, w, dev0, judge, p, n_evals)
        else:
            th0 = first_eval_theta(bh, w, dev0, judge, p)
            p["theta_first_eval"] = th0
            # first guess: the tuned path's ratio of along-the-run to first-evaluation theta
            tp = paths["tuned"]
            guess = th0 * tp["theta"] / tp["theta_first_eval"] if "theta_first_eval" in tp else None
            p["theta"], r = match_along_run(
                "plain theta", lambda th: error_run(bh, w, dev0, judge, dict(p, theta=th), n_evals), th0, 2.0,
                THETA_FLOOR, guess=guess)
        paths["plain"] = dict(p, run=r)

    # ---- learned opening rule on the tuned configuration (on a Cartesian
    # tree: the learned rule does not walk cylindrical ones; then the fastest
    # Cartesian candidate is its geometric reference, timed as well)
    geo_ref = None
    if "learned" in legs:
        tp = paths["tuned"]
        if tp.get("cyl_radius", 0.0) > 0.0:
            geo_ref = dict(best_cart[1]) if best_cart else dict(tp, cyl_radius=0.0)
            geo_ref.pop("run", None)
            paths["geometric_reference"] = dict(geo_ref, run=None)
        lbase = geo_ref or tp
        lo, hi = args.learned_band
        t = time.perf_counter()
        weights, n_pairs, mse = train_learned(bh, inputs, w, lbase["n_group"], lbase["theta"], (lo, hi))
        t_train = time.perf_counter() - t
        log(f"[bench] learned: {n_pairs} training pairs, mse {mse:.3f}, {t_train:.1f} s")
        p = dict(lbase, learned=dict(criterion=bh.LEARNED, theta_min=lo, theta_max=hi, tau=1e-4,
                                     budget_min=args.learned_budget == "min"), weights=weights)
        p.pop("run", None)
        if args.tau_learned is not None:
            p["learned"]["tau"] = args.tau_learned
            r = None if fixed_run else error_run(bh, w, dev0, judge, p, n_evals, 1 + args.warmup)
        else:
            def run_tau(tau):
                return error_run(bh, w, dev0, judge, dict(p, learned=dict(p["learned"], tau=tau)), n_evals,
                                 1 + args.warmup)
            tau0 = first_eval_tau(bh, w, dev0, judge, p)
            # first guess: the error grows along the run as it did for the
            # tuned path's theta; p99 goes about as tau^(1/2)
            grow = (tp["theta_first_eval"] / lbase["theta"]) ** 2 if "theta_first_eval" in tp else 1.0
            tau, r = match_along_run("learned tau", run_tau, tau0, 0.5, 1e-14, guess=tau0 / grow ** 2)
            p["learned"]["tau"] = tau
            p["tau_first_eval"] = tau0
        paths["learned"] = dict(p, run=r, training_pairs=n_pairs, training_mse=mse, training_s=t_train)

    # ---- timed runs (same start, warm-up and steps for every path)
    res = {}
    for name in ("tuned", "plain", "learned", "geometric_reference"):
        if name in paths:
            res[name] = timed(bh, w, dev0, paths[name], args.steps, args.warmup)
            log(f"[bench] {name}: {res[name]}")
    co = None
    if "collisions" in legs:
        cparams, cinfo = collision_params(w)
        co = timed(bh, w, dev0, dict(paths["tuned"], contact=cparams), args.steps, args.warmup)
        log(f"[bench] collisions {cparams}: {co}")
    bat = None
    if "batched" in legs:
        bat = batched_leg(bh, inputs, 20)
        log(f"[bench] batched: {bat}")
    judge.close()

    tu, tp = res["tuned"], paths["tuned"]
    value = tu["interactions"] / tu["wall"]
    per_launch = tu["interactions"] / max(1, tu["force_evals"])
    avg_ms = tu["force_ms"] / max(1, tu["force_launches"])
    achieved = per_launch * FLOPS_PER_INTERACTION / (avg_ms * 1e-3) / 1e12
    workload = f"ring{n}_kdk{args.warmup}+{args.steps}"

    def path_record(name):
        p, r, t = paths[name], paths[name]["run"], res[name]
        rec = dict(theta=p["theta"], n_group=p["n_group"], pack_groups=p.get("pack_groups", False),
                   tree="cylindrical, r_ref %g" % p["cyl_radius"] if p.get("cyl_radius", 0.0) > 0 else "cartesian",
                   force_tile=p.get("force_tile", 512),
                   s_per_step=t["wall"] / args.steps,
                   interactions_per_s=t["interactions"] / t["wall"],
                   interactions_per_force_eval=t["interactions"] / max(1, t["force_evals"]),
                   tree_builds_timed=t["builds"], host_syncs_timed=t["host_syncs"],
                   force_kernel_ms=t["force_ms"] / max(1, t["force_launches"]),
                   dtype="f64" if p["precision"] == bh.FP64 else "f32",
                   rebuild=(f"drift monitor {p['drift']}, at most every {p['rebuild_every']} steps" if "drift" in p
                            else f"every {p['rebuild_every']} steps"))
        if "theta_first_eval" in p:
            rec["theta_first_eval"] = p["theta_first_eval"]
        if r is not None:
            rec["p99_along_run"] = dict(per_force_eval=r["p99"], max=r["max"], p50_max=max(r["p50"]))
        return rec

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
            "workload": workload, "n_particles": n, "eps": w.eps, "dt": w.dt,
            "step": "one kick-drift-kick step (one force evaluation, tree and list builds as they fall)",
            "theta_tuned": tp["theta"], "n_group": tp["n_group"], "pack_groups": tp["pack_groups"],
            "tree": "cylindrical, r_ref %g" % tp["cyl_radius"] if tp.get("cyl_radius", 0.0) > 0 else "cartesian",
            "force_tile": tp["force_tile"],
            "rebuild": (f"drift monitor {tp['drift']}, at most every {tp['rebuild_every']} steps" if "drift" in tp
                        else f"every {tp['rebuild_every']} steps"), "positions_and_integration": "f64",
            "matched_error": (f"p99 <= {TARGET_P99} at every one of the {n_evals} force evaluations through the "
                              f"last timed one, for each path; theta bracket floor {THETA_FLOOR}"),
        },
        "s_per_step": tu["wall"] / args.steps,
        "interactions_per_force_eval": per_launch,
        "tree_builds_timed": tu["builds"],
        "tuned": path_record("tuned"),
        "group_size_autotune": autotune,
        "rebuild_policy_autotune": policy_autotune,
        "force_kernel_ms": avg_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic(workload, tp["n_group"], tp["theta"]),
                     "flops_per_interaction": FLOPS_PER_INTERACTION,
                     "frac_at_paper_31_flops": achieved * PAPER_FLOPS_PER_INTERACTION / FLOPS_PER_INTERACTION
                     / FP32_PEAK_TFLOPS},
        "stages_ms_last": tu["stages"],
        "reproduce_without_matching": (f"--steps {args.steps} --warmup {args.warmup} --n-group {tp['n_group']} "
                                       f"--pack {'on' if tp['pack_groups'] else 'off'} "
                                       f"--cyl {'on' if tp.get('cyl_radius', 0.0) > 0 else 'off'} "
                                       f"--tile {tp['force_tile']} --policy {tp['policy_key']} "
                                       f"--theta-tuned {tp['theta']!r}"
                                       + (f" --theta-plain {paths['plain']['theta']!r}" if "plain" in paths else "")
                                       + (f" --tau-learned {paths['learned']['learned']['tau']!r}"
                                          if "learned" in paths else "")),
    }
    if "plain" in paths:
        pr = path_record("plain")
        pl = res["plain"]
        pms = pl["force_ms"] / max(1, pl["force_launches"])
        pach = pr["interactions_per_force_eval"] * FLOPS_PER_INTERACTION / (pms * 1e-3) / 1e12
        pr["force_kernel_fp64_tflops_19"] = pach
        pr["force_kernel_frac_of_fp64_peak"] = pach / FP64_PEAK_TFLOPS
        out["plain"] = pr
        out["speedup_vs_plain_s_per_step"] = pr["s_per_step"] / out["s_per_step"]
    if "learned" in paths:
        lr = path_record("learned")
        lp = paths["learned"]
        lr.update(tau=lp["learned"]["tau"], tau_first_eval=lp.get("tau_first_eval"), band=list(args.learned_band),
                  budget="min" if lp["learned"]["budget_min"] else "mean",
                  training_pairs=lp["training_pairs"],
                  training_mse=lp["training_mse"], training_s=lp["training_s"],
                  interactions_vs_geometric=lr["interactions_per_force_eval"] / per_launch,
                  s_per_step_vs_geometric=lr["s_per_step"] / out["s_per_step"])
        if "geometric_reference" in res:
            gr = path_record("geometric_reference")
            lr.update(geometric_reference=gr,
                      interactions_vs_geometric=lr["interactions_per_force_eval"] / gr["interactions_per_force_eval"],
                      s_per_step_vs_geometric=lr["s_per_step"] / gr["s_per_step"])
        if "plain" in out:
            lr["speedup_vs_plain_s_per_step"] = out["plain"]["s_per_step"] / lr["s_per_step"]
        out["learned"] = lr
    if co is not None:
        c_launch = co["interactions"] / max(1, co["force_evals"])
        c_ms = co["force_ms"] / max(1, co["force_launches"])
        c_ach = c_launch * FLOPS_PER_INTERACTION / (c_ms * 1e-3) / 1e12
        out["collisions"] = dict(cparams, **cinfo, s_per_step=co["wall"] / args.steps,
                                 interactions_per_s=co["interactions"] / co["wall"],
                                 interactions_per_force_eval=c_launch, force_kernel_ms=c_ms,
                                 force_kernel_ms_ratio_vs_gravity_only=c_ms / avg_ms,
                                 achieved_tflops_19=c_ach, frac=c_ach / FP32_PEAK_TFLOPS)
    if bat is not None:
        out["batched"] = bat
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sysm, tp["theta"], tp["n_group"], w.eps, cyl_r=tp.get("cyl_radius", 0.0),
                                           pack=tp.get("pack_groups", False))
    print(json.dumps(out), flush=True)


REUSE_INTERVALS = (1, 2, 4, 8, 16)


def reuse_study(bh, w, dev0, judge, n, args):
    """Interaction-list reuse (persistent lists): for each fixed rebuild
    interval R and for the drift monitor, theta matched so that p99 <= 1e-3
    at every evaluation of a run of 1 + warmup + steps evaluations, and the
    device time per step over the last `steps` of them."""
    n_evals = 1 + args.warmup + args.steps
    ng = args.n_group or 256
    recs = []
    configs = [(f"R={R}", dict(rebuild_every=R)) for R in REUSE_INTERVALS]
    configs.append(("drift", dict(rebuild_every=REUSE_MAX, drift=dict(DRIFT))))
    if args.reuse_configs:
        # names from the list above, or drift:<reuse_drift>:<reuse_frac> for another monitor setting
        # suffixes: "+pack" packs small sibling groups, "+cyl" builds the tree
        # on cylindrical coordinates around the ring's mid radius
        chosen = []
        for name in args.reuse_configs.split(","):
            base, *suffix = name.split("+")
            if set(suffix) - {"pack", "cyl"}:
                raise SystemExit(f"unknown suffix in {name}")
            if base.startswith("drift:"):
                parts = base.split(":")[1:]
                k, f = float(parts[0]), float(parts[1])
                cap = int(parts[2]) if len(parts) > 2 else REUSE_MAX
                extra = dict(rebuild_every=cap, drift=dict(reuse_drift=k, reuse_frac=f))
            else:
                extra = next(dict(c[1]) for c in configs if c[0] == base)
            if "pack" in suffix:
                extra["pack_groups"] = True
            if "cyl" in suffix:
                extra["cyl_radius"] = CYL_RADIUS
            chosen.append((name, extra))
        configs = chosen
    th0 = None
    for name, extra in configs:
        p = dict(precision=bh.FP32_REL, n_group=ng, **extra)
        if th0 is None:
            th0 = first_eval_theta(bh, w, dev0, judge, p)
        # first guess: what lists rebuilt every step need over such a run
        # (the ring's own error growth), 0.83 of the first-evaluation value
        try:
            th, r = match_along_run(f"reuse {name} theta",
                                    lambda th: error_run(bh, w, dev0, judge, dict(p, theta=th), n_evals,
                                                         1 + args.warmup), th0, 2.0, THETA_FLOOR, max_runs=7,
                                    guess=0.83 * th0)
        except RuntimeError as e:
            # no theta down to the floor holds the target along this run
            log(f"[bench] reuse {name}: {e}")
            recs.append(dict(config=name, theta=None, unmatched=str(e)))
            continue
        ns = [1e6 * f / max(1, i) for f, i in zip(r["force_ms"], r["inter"])]
        rec = dict(config=name, theta=th, max_p99=r["max"], p99_per_force_eval=r["p99"],
                   device_ms_per_step=float(np.mean(r["step_ms"])), tree_builds=r["builds"],
                   interactions_per_force_eval=r["interactions"] / n_evals,
                   force_ns_per_interaction_per_eval=ns, groups_per_eval=r["groups"],
                   interactions_per_eval=r["inter"], walk_ms_per_build=r["walk_ms"])
        # force-kernel efficiency early (the bench's window) and late in the run
        early = slice(1 + args.warmup, min(n_evals, 1 + args.warmup + 20))
        late = slice(max(0, n_evals - 20), n_evals)
        for tag, sl in (("early", early), ("late", late)):
            rec[f"force_ns_per_interaction_{tag}"] = float(np.median(ns[sl]))
            rec[f"mean_group_size_{tag}"] = float(n / np.mean(r["groups"][sl]))
            wk = [m for k, m in r["walk_ms"] if sl.start <= k < sl.stop]
            rec[f"walk_ms_{tag}"] = float(np.mean(wk)) if wk else None
        log(f"[bench] reuse {name}: theta={th:.5f} max p99={r['max']:.3e} "
            f"{rec['device_ms_per_step']:.2f} ms/step, {r['builds']} builds; force ps/interaction "
            f"{1e3 * rec['force_ns_per_interaction_early']:.4f} early, "
            f"{1e3 * rec['force_ns_per_interaction_late']:.4f} late")
        recs.append(rec)
    fastest = min((r for r in recs if r["theta"] is not None), key=lambda r: r["device_ms_per_step"],
                  default=dict(config=None))
    print(json.dumps({"metric": "list-reuse study: device ms/step at p99 <= 1e-3 along the whole run",
                      "config": {"workload": f"ring{n}", "n_group": ng, "eps": w.eps, "dt": w.dt,
                                 "force_evaluations": n_evals, "timed_from": 1 + args.warmup},
                      "fastest": fastest["config"], "records": recs}), flush=True)


if __name__ == "__main__":
    main()
