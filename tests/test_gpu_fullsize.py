"""Parity at the benchmark sizes, in the benchmark's launch configuration,
on sampled outputs: the 2^20 ring (FP32 interactions, groups <= 256) and the
2^24 ring (the benchmark workload, FP32, groups <= 256, theta 0.5 and the
tuned 0.1035).  Keys, permutation and node arrays are compared in full;
lists and forces for a random sample of groups, against the oracle walking
those groups and evaluating their lists in FP64."""
import sys

import numpy as np
import pytest

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


def _run(n, seed, theta, eps, n_grp, n_sample_groups, r_out=1.1, z_sigma=1e-3):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02289_amd import bh
    s = inputs.ring(n, seed, r_out=r_out, z_sigma=z_sigma, central_mass=1.0)
    _log(f"[gpu] fullsize n={n} theta={theta}")
    ctx = bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=bh.FP32_REL)
    dev = bh.to_device(s)
    ctx.build_tree([dev])
    ctx.make_lists()
    out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    torch.cuda.synchronize()
    # oracle: full build
    _, _, _, key = oracle.keys(s.x, s.y, s.z)
    perm = oracle.sort_perm(key)
    skey = key[perm]
    np.testing.assert_array_equal(ctx.export("keys"), skey)
    np.testing.assert_array_equal(ctx.export("perm"), perm)
    t = oracle.tree(skey, 8)
    nodes = ctx.export("nodes")
    np.testing.assert_array_equal(nodes[:, 3], t["begin"])
    np.testing.assert_array_equal(nodes[:, 4], t["count"])
    np.testing.assert_array_equal(nodes[:, 2].astype(np.uint64), t["prefix"])
    xs, ys, zs, ms = (a[perm] for a in (s.x, s.y, s.z, s.m))
    mom = oracle.moments(t, xs, ys, zs, ms)
    g = oracle.groups(t, n_grp)
    np.testing.assert_array_equal(ctx.export("groups")[:, 0], g)
    gbox, gcen = oracle.group_boxes(g, t, skey, xs, ys, zs)
    box, cen = ctx.export_groups()
    np.testing.assert_array_equal(box, gbox)
    np.testing.assert_array_equal(cen, gcen)
    sel = np.sort(np.random.default_rng(seed).choice(g.size, n_sample_groups, replace=False))
    o_pc_off, o_pc, o_pp_off, o_pp = oracle.lists(gbox[sel], t, theta)
    pc_off, pc, pp_off, pp = ctx.export("lists")
    a, b, c, d = _subset_lists(pc_off, pc, pp_off, pp, sel)
    np.testing.assert_array_equal(a, o_pc_off)
    np.testing.assert_array_equal(b, o_pc)
    np.testing.assert_array_equal(c, o_pp_off)
    np.testing.assert_array_equal(d, o_pp)
    ax, ay, az, _, _ = oracle.forces(g[sel], t, xs, ys, zs, ms, mom, o_pc_off, o_pc, o_pp_off, o_pp, eps)
    gx, gy, gz = (out[k].cpu().numpy()[perm] for k in ("ax", "ay", "az"))
    idx = np.concatenate([np.arange(t["begin"][v], t["begin"][v] + t["count"][v]) for v in g[sel]])
    rel = np.sqrt((gx[idx] - ax[idx]) ** 2 + (gy[idx] - ay[idx]) ** 2 + (gz[idx] - az[idx]) ** 2) / \
        np.sqrt(ax[idx] ** 2 + ay[idx] ** 2 + az[idx] ** 2)
    _log(f"    {idx.size} particles: fp32 rel err median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e}")
    assert np.median(rel) <= 1e-5
    ctx.close()


def test_ring_1m_fp32_groups256():
    _run(1 << 20, 1, 0.5, 1e-4, 256, 256)


@pytest.mark.slow
def test_ring_16m_benchmark_configuration():
    _run(1 << 24, 3, 0.103515625, 1e-4, 256, 48, r_out=1.2, z_sigma=5e-4)
