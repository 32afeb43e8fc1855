"""Parity at the full sizes of the workloads, on sampled outputs: the 2^20
ring (FP32 interactions, groups <= 256) at t = 0 and along 10 steps rebuilt
every step; the 2^24 ring in the benchmark's launch configuration (FP32,
tree on cylindrical coordinates around r = 1.1, packed groups <= 384,
512-source tiles, theta 0.0865, the value matched along the benchmark's
run); the 64 batched Plummer spheres (2.2M particles,
autotuned group size, 20 steps).  Keys, permutation and node arrays are compared in
full; lists and forces for a random sample of groups, against the oracle
walking those groups and evaluating their lists in FP64."""
import sys

import numpy as np
import pytest

from bars import fp32_bars

import oracle
from paper_1907_02289_amd import inputs

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _subset_lists(pc_off, pc, pp_off, pp, sel):
    """CSR lists of the groups in sel (in that order)."""
    def take(off, ids):
        parts = [ids[off[g]:off[g + 1]] for g in sel]
        o = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
        return o, (np.concatenate(parts) if parts else np.zeros(0, np.uint32)).astype(np.uint32)
    a, b = take(pc_off, pc)
    c, d = take(pp_off, pp)
    return a, b, c, d


def _check(ctx, x, y, z, m, theta, eps, n_grp, n_sample_groups, seed, gx, gy, gz, central_mass=0.0,
           resorted=False, pack=False, cyl_r=0.0):
    """The oracle's full build of (x, y, z, m) against the context's keys,
    permutation, nodes, moments, groups and group boxes; the lists and FP32
    forces of a random sample of groups against the oracle walking those
    groups and evaluating their lists in FP64.  gx, gy, gz: the context's
    forces in sorted order.  resorted: the context's tree was rebuilt from its
    own sorted order during a step, so particles with equal keys keep that
    order rather than the caller's; the permutation is then checked to sort
    the keys, and the oracle takes the same order.  Returns the permutation and
    the sorted-order particle indices of the sampled groups."""
    _, _, _, key = oracle.keys_cyl(x, y, z, cyl_r) if cyl_r > 0 else oracle.keys(x, y, z)
    perm = oracle.sort_perm(key)
    skey = key[perm]
    np.testing.assert_array_equal(ctx.export("keys"), skey)
    gperm = ctx.export("perm").astype(np.int64)
    if resorted:
        assert np.array_equal(np.sort(gperm), np.arange(x.size))
        np.testing.assert_array_equal(key[gperm], skey)
        ties = int(np.sum(skey[1:] == skey[:-1]))
        _log(f"    {ties} equal-key neighbours; permutations differ at {int(np.sum(gperm != perm))} slots")
        perm = gperm
    else:
        np.testing.assert_array_equal(gperm, perm)
    t = oracle.tree(skey, 8)
    nodes = ctx.export("nodes")
    np.testing.assert_array_equal(nodes[:, 3], t["begin"])
    np.testing.assert_array_equal(nodes[:, 4], t["count"])
    np.testing.assert_array_equal(nodes[:, 2].astype(np.uint64), t["prefix"])
    xs, ys, zs, ms = (a[perm] for a in (x, y, z, m))
    mom = oracle.moments(t, xs, ys, zs, ms)
    if pack:
        g, gbeg, gcnt = oracle.groups_packed(t, n_grp)
    else:
        g = oracle.groups(t, n_grp)
        gbeg, gcnt = t["begin"][g], t["count"][g]
    groups = ctx.export("groups")
    np.testing.assert_array_equal(groups[:, 0], g)
    np.testing.assert_array_equal(groups[:, 1], gbeg)
    np.testing.assert_array_equal(groups[:, 2], gcnt)
    gbox, gcen = oracle.group_boxes(np.arange(g.size, dtype=np.uint32), dict(begin=gbeg, count=gcnt), skey,
                                    xs, ys, zs)
    box, cen = ctx.export_groups()
    np.testing.assert_array_equal(box, gbox)
    np.testing.assert_array_equal(cen, gcen)
    ns = min(n_sample_groups, g.size)
    sel = np.sort(np.random.default_rng(seed).choice(g.size, ns, replace=False))
    o_pc_off, o_pc, o_pp_off, o_pp = oracle.lists(gbox[sel], t, theta, oracle.CYL_PERIOD if cyl_r > 0 else 0)
    pc_off, pc, pp_off, pp = ctx.export("lists")
    a, b, c, d = _subset_lists(pc_off, pc, pp_off, pp, sel)
    np.testing.assert_array_equal(a, o_pc_off)
    np.testing.assert_array_equal(b, o_pc)
    np.testing.assert_array_equal(c, o_pp_off)
    np.testing.assert_array_equal(d, o_pp)
    ax, ay, az, _, _ = oracle.forces(g[sel], t, xs, ys, zs, ms, mom, o_pc_off, o_pc, o_pp_off, o_pp, eps,
                                     granges=(gbeg[sel], gcnt[sel]))
    if central_mass:
        oracle.central(xs, ys, zs, central_mass, 1.0, ax, ay, az)
    idx = np.concatenate([np.arange(b, b + c) for b, c in zip(gbeg[sel].astype(np.int64), gcnt[sel].astype(np.int64))])
    rel = np.sqrt((gx[idx] - ax[idx]) ** 2 + (gy[idx] - ay[idx]) ** 2 + (gz[idx] - az[idx]) ** 2) / \
        np.sqrt(ax[idx] ** 2 + ay[idx] ** 2 + az[idx] ** 2)
    _log(f"    {idx.size} particles: fp32 rel err median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e}")
    fp32_bars(rel, f"{idx.size} sampled particles")
    return perm, idx


def _run(n, seed, theta, eps, n_grp, n_sample_groups, r_out=1.1, z_sigma=1e-3, pack=False, tile=0, cyl_r=0.0):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02289_amd import bh
    s = inputs.ring(n, seed, r_out=r_out, z_sigma=z_sigma, central_mass=1.0)
    _log(f"[gpu] fullsize n={n} theta={theta} groups <= {n_grp}{' packed' if pack else ''}")
    ctx = bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=bh.FP32_REL, pack_groups=pack, force_tile=tile,
                     cyl_radius=cyl_r)
    dev = bh.to_device(s)
    ctx.build_tree([dev])
    ctx.make_lists()
    out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    torch.cuda.synchronize()
    perm = ctx.export("perm")
    gx, gy, gz = (out[k].cpu().numpy()[perm] for k in ("ax", "ay", "az"))
    _check(ctx, s.x, s.y, s.z, s.m, theta, eps, n_grp, n_sample_groups, seed, gx, gy, gz, pack=pack, cyl_r=cyl_r)
    ctx.close()


def test_ring_1m_fp32_groups256():
    _run(1 << 20, 1, 0.5, 1e-4, 256, 256)


@pytest.mark.slow
def test_ring_16m_benchmark_configuration():
    _run(1 << 24, 3, 0.08650261852548162, 1e-4, 384, 48, r_out=1.2, z_sigma=5e-4, pack=True, tile=512, cyl_r=1.1)


def test_ring_1m_ten_steps_rebuilt_every_step():
    """The 2^20 ring with its central mass, 10 KDK steps (dt 1e-3, theta 0.5,
    eps 1e-4, groups <= 256, FP32 interactions, tree and lists rebuilt every
    step).  After steps 1, 5 and 10 the state the library holds is checked
    against the oracle rebuilding everything from the current positions
    (sampled groups, as above, central mass included), and the force error
    against the oracle's FP64 direct sum on 4096 sampled particles is
    reported."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02289_amd import bh
    w = inputs.workload(1)
    s = w.systems[0]
    _log(f"[gpu] ring 2^20, {w.n_steps} steps rebuilt every step")
    ctx = bh.Context(theta=w.theta, eps=w.eps, n_group=w.n_grp, precision=bh.FP32_REL, central_mass=w.central_mass)
    dev = bh.to_device(s)
    ctx.step([dev], w.dt, 0, w.rebuild_every)
    tg = inputs.force_sample(s.n, 1).astype(np.int64)
    for k in range(1, w.n_steps + 1):
        ctx.step_continue(w.dt, 1, w.rebuild_every)
        if k not in (1, 5, w.n_steps):
            continue
        torch.cuda.synchronize()
        x, y, z = (dev[f].cpu().numpy() for f in ("x", "y", "z"))
        acc = ctx.export("acc_sorted")
        perm, _ = _check(ctx, x, y, z, s.m, w.theta, w.eps, w.n_grp, 64, k, acc[:, 0], acc[:, 1], acc[:, 2],
                         central_mass=w.central_mass, resorted=True)
        # approximation error on the sample: the library's forces in caller order
        # against the FP64 direct sum plus the central mass
        a = np.zeros((s.n, 3))
        a[perm] = acc[:, :3]
        dx, dy, dz, _ = oracle.direct(x, y, z, s.m, w.eps, targets=tg)
        oracle.central(x[tg], y[tg], z[tg], w.central_mass, 1.0, dx, dy, dz)
        ref = np.stack([dx, dy, dz], 1)
        e = np.linalg.norm(a[tg] - ref, axis=1) / np.linalg.norm(ref, axis=1)
        _log(f"    step {k}: force error vs direct sum on {tg.size} particles: median {np.median(e):.2e} "
             f"p99 {np.percentile(e, 99):.2e}")
        assert np.percentile(e, 99) <= 0.1       # a sanity bound: theta 0.5 is far from the matched-error setting
    ctx.close()


def test_batched_plummer_full_size():
    """The batched workload at full size: 64 Plummer spheres (2.2M particles,
    N log-uniform in [1e3, 2e5]) in one launch per stage, FP32, theta 0.6,
    eps 1e-2, group size from the library's autotuner, 20 KDK steps rebuilt
    every step.  The largest, a middle and the smallest system: integrated
    alone they end bit-identical to their part of the batch, and at t = 0
    their tree, lists and forces match the oracle (sampled groups)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02289_amd import bh
    w = inputs.workload(2)
    order = np.argsort([sy.n for sy in w.systems])
    pick = [int(order[-1]), int(order[32]), int(order[0])]
    _log(f"[gpu] batched 64 Plummer spheres, {sum(sy.n for sy in w.systems)} particles")
    dev = [bh.to_device(sy) for sy in w.systems]
    cb = bh.Context(theta=w.theta, eps=w.eps, n_group=0, precision=bh.FP32_REL)
    cb.build_tree(dev)
    g = cb.autotune((64, 128, 256), rebuild_every=w.rebuild_every)
    _log(f"    autotuned group size {g}")
    cb.step(dev, w.dt, w.n_steps, rebuild_every=w.rebuild_every)
    torch.cuda.synchronize()
    assert cb.query()["n_systems"] == 64
    for k in pick:
        sy = w.systems[k]
        one = bh.to_device(sy)
        c1 = bh.Context(theta=w.theta, eps=w.eps, n_group=g, precision=bh.FP32_REL)
        c1.build_tree([bh.to_device(sy)])
        c1.make_lists()
        out = {f: torch.zeros(sy.n, dtype=torch.float64, device="cuda") for f in ("ax", "ay", "az")}
        c1.forces([out])
        torch.cuda.synchronize()
        perm = c1.export("perm")
        gx, gy, gz = (out[f].cpu().numpy()[perm] for f in ("ax", "ay", "az"))
        _log(f"    system {k}: n={sy.n}")
        _check(c1, sy.x, sy.y, sy.z, sy.m, w.theta, w.eps, g, 64, k, gx, gy, gz)
        c1.step([one], w.dt, w.n_steps, rebuild_every=w.rebuild_every)
        torch.cuda.synchronize()
        for f in ("x", "y", "z", "vx", "vy", "vz"):
            assert torch.equal(one[f], dev[k][f]), (k, f)
        c1.close()
    cb.close()
