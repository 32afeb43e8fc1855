"""GPU parity of packed groups (BH_FLAG_PACK_GROUPS) against the oracle.

Packing merges runs of consecutive small sibling nodes into one group (an
option of this implementation; the paper's groups are tree nodes, Sec. 4.2
(3d)).  Bars as for unpacked groups: groups (first node, particle range),
group boxes, centres and lists bit-exact; FP64 forces within 1e-12 of the sum
of the terms' magnitudes; FP32 within the FP32 bars of the oracle on the same
lists.
"""
import math
import sys

import numpy as np
import pytest

from bars import fp32_bars

import oracle
from paper_1907_02289_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _clumpy(n, seed):
    """A ring with a tenth of its particles in five clumps of radius ~5e-3.
    The clumps are wider than the softening on purpose: in clumps much
    tighter than it, deep nodes are accepted so close to the particles that
    the rounding of their centres of mass (the GPU sums children level by
    level, the oracle sums particles in order; both within the FP64
    summation bound) alone moves a force by more than 1e-12 of the sum of
    its terms' magnitudes, and the FP64 bar would measure that order, not
    the force kernel."""
    s = inputs.ring(n, seed)
    rng = np.random.default_rng(seed + 1000)
    k = n // 10
    idx = rng.choice(n, k, replace=False)
    centres = rng.choice(n, 5, replace=False)
    which = centres[rng.integers(0, 5, k)]
    for a in (s.x, s.y, s.z):
        a[idx] = a[which] + rng.normal(0.0, 5e-3, k)
    return s


def _coincident():
    s = inputs.ring(600, 4)
    for a in (s.x, s.y, s.z):
        a[:40] = a[0]                    # a level-21 leaf of 40 > n_group points
    return s


CASES = [
    # name, system factory, theta, eps, n_leaf, n_grp
    ("clumpy20000_g64", lambda: _clumpy(20000, 3), 0.5, 1e-3, 8, 64),
    ("plummer5000_g256", lambda: inputs.plummer(5000, 7), 0.7, 1e-2, 8, 256),
    ("ring3001_g32", lambda: inputs.ring(3001, 5), 0.6, 1e-3, 8, 32),
    ("coincident40_g32", _coincident, 0.5, 1e-3, 8, 32),
    ("clumpy2000_leaf1_g16", lambda: _clumpy(2000, 9), 0.4, 1e-3, 1, 16),
    ("single_particle", lambda: inputs.ring(1, 2), 0.5, 1e-3, 8, 64),
]


def _build(torch, systems, theta, eps, n_leaf, n_grp, precision):
    from paper_1907_02289_amd import bh
    ctx = bh.Context(theta=theta, eps=eps, n_leaf=n_leaf, n_group=n_grp, precision=precision, pack_groups=True)
    dev = [bh.to_device(s) for s in systems]
    ctx.build_tree(dev)
    ctx.make_lists()
    return ctx, dev


def _compare(ctx, st):
    groups = ctx.export("groups")
    np.testing.assert_array_equal(groups[:, 0], st.gnode)
    np.testing.assert_array_equal(groups[:, 1], st.gbeg)
    np.testing.assert_array_equal(groups[:, 2], st.gcnt)
    box, cen = ctx.export_groups()
    np.testing.assert_array_equal(box, st.gbox)
    np.testing.assert_array_equal(cen, st.gcen)
    pc_off, pc, pp_off, pp = ctx.export("lists")
    np.testing.assert_array_equal(pc_off, st.pc_off)
    np.testing.assert_array_equal(pp_off, st.pp_off)
    np.testing.assert_array_equal(pc, st.pc)
    np.testing.assert_array_equal(pp, st.pp)
    assert ctx.query()["interactions"] == st.interactions()


@pytest.mark.parametrize("name,make,theta,eps,n_leaf,n_grp", CASES, ids=[c[0] for c in CASES])
def test_packed_structures_and_forces(torch_cuda, name, make, theta, eps, n_leaf, n_grp):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    s = make()
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, n_leaf, n_grp, pack=True)
    ax, ay, az, pot, mag = st.accel(s.x, s.y, s.z, s.m, eps)
    for prec in (bh.FP64, bh.FP32_REL):
        _log(f"[gpu] packed groups {name}, precision {prec}")
        ctx, dev = _build(torch, [s], theta, eps, n_leaf, n_grp, prec)
        _compare(ctx, st)
        out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
        ctx.forces([out])
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
        err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
        if prec == bh.FP64:
            assert np.all(err <= 1e-12 * mag + 1e-300), f"max err/mag {np.max(err / mag)}"
        elif s.n > 1:
            rel = err / np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
            _log(f"    fp32 rel err: median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}")
            fp32_bars(rel, name)
        ctx.close()


def test_packing_merges_groups(torch_cuda):
    """On the clumpy ring packing gives fewer groups than tree-node groups,
    and the unpacked context still equals the unpacked oracle."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] packed vs unpacked group counts, clumpy ring n=20000")
    s = _clumpy(20000, 3)
    st0 = oracle.BHState(s.x, s.y, s.z, s.m, 0.5, 8, 64)
    st1 = oracle.BHState(s.x, s.y, s.z, s.m, 0.5, 8, 64, pack=True)
    assert st1.gnode.size < st0.gnode.size
    ctx = bh.Context(theta=0.5, eps=1e-3, n_group=64)
    dev = bh.to_device(s)
    ctx.build_tree([dev])
    ctx.make_lists()
    assert ctx.query()["n_groups"] == st0.gnode.size
    np.testing.assert_array_equal(ctx.export("groups")[:, 0], st0.gnode)
    # switching packing on invalidates the tree: the next build packs
    ctx.set_params(flags=ctx.params.flags | bh.FLAG_PACK_GROUPS)
    with pytest.raises(bh.BHError):
        ctx.make_lists()
    ctx.build_tree([dev])
    ctx.make_lists()
    _compare(ctx, st1)
    ctx.close()


def test_packed_batched_systems(torch_cuda):
    """Several systems in one context: each system's packed groups and FP64
    forces equal the oracle run on that system alone (packs never span two
    systems)."""
    torch = torch_cuda
    _log("[gpu] packed groups, batched systems")
    systems = [_clumpy(3000, 31), inputs.plummer(4100, 32), inputs.ring(37, 33), inputs.plummer(900, 34)]
    theta, eps, n_grp = 0.6, 1e-2, 32
    ctx, dev = _build(torch, systems, theta, eps, 8, n_grp, 0)
    outs = [{k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")} for s in systems]
    ctx.forces(outs)
    torch.cuda.synchronize()
    groups = ctx.export("groups")
    nodes = ctx.export("nodes")
    off = np.concatenate([[0], np.cumsum([s.n for s in systems])])
    for k, s in enumerate(systems):
        st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp, pack=True)
        mine = groups[groups[:, 3] == k]
        np.testing.assert_array_equal(mine[:, 1] - off[k], st.gbeg)
        np.testing.assert_array_equal(mine[:, 2], st.gcnt)
        # first node of each pack: the same node of this system's tree
        sys_nodes = np.nonzero(nodes[:, 1] == k)[0]
        np.testing.assert_array_equal(np.searchsorted(sys_nodes, mine[:, 0]), st.gnode)
        ax, ay, az, _, mag = st.accel(s.x, s.y, s.z, s.m, eps)
        g = {q: v.cpu().numpy() for q, v in outs[k].items()}
        err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
        assert np.all(err <= 1e-12 * mag)
    ctx.close()


def _contact_params(t_c, e):
    """Spring and dashpot of a contact lasting t_c with restitution e."""
    wd = math.pi / t_c
    gamma = -math.log(e) / t_c
    return wd * wd + gamma * gamma, 2.0 * gamma


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_packed_groups_with_contacts(torch_cuda, precision):
    """The collision branch of Eq. (2) over packed groups of <= 384 (the
    bench's tuned configuration) against the oracle on the same packs."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] packed groups with contacts, ring n=20000 seed 31, precision {precision}")
    s = inputs.ring(20000, 31, v_disp=3e-3)
    theta, eps, n_grp, rc = 0.5, 1e-4, 384, 2e-3
    kappa, eta = _contact_params(0.02, 0.5)
    ctx = bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=precision, r_coll=rc, kappa=kappa, eta=eta,
                     pack_groups=True)
    ctx.build_tree([bh.to_device(s)])
    ctx.make_lists()
    out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    torch.cuda.synchronize()
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp, pack=True)
    _compare(ctx, st)
    ax, ay, az, _, mag = st.accel(s.x, s.y, s.z, s.m, eps, vel=(s.vx, s.vy, s.vz), contact=(rc, kappa, eta))
    nx, ny, nz, _, _ = st.accel(s.x, s.y, s.z, s.m, eps)
    moved = np.sqrt((nx - ax) ** 2 + (ny - ay) ** 2 + (nz - az) ** 2) > 1e-3 * mag
    assert moved.sum() > 50                       # the contact terms matter
    g = {k: v.cpu().numpy() for k, v in out.items()}
    err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
    if precision == 0:
        assert np.all(err <= 1e-12 * mag), f"max err/mag {np.max(err / mag)}"
    else:
        rel = err / np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
        _log(f"    fp32 rel err: median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}")
        fp32_bars(rel, "packed groups with contacts")
    ctx.close()


def test_packed_monitor_trajectory_matches_oracle(torch_cuda):
    """FP64 leapfrog over packed groups with the drift monitor choosing the
    rebuilds (lists at most 4 steps old, as in the bench's tuned
    configuration): the trajectory equals the oracle's with packed groups
    rebuilt before the same steps."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] packed groups, drift monitor trajectory: ring n=3000 seed 33, fp64, 12 steps of dt 2e-3")
    s = inputs.ring(3000, 33, central_mass=1.0, v_disp=3e-3)
    dt, n, cap = 2e-3, 12, 4
    dev = bh.to_device(s)
    ctx = bh.Context(theta=0.5, eps=1e-3, central_mass=1.0, n_group=128, precision=bh.FP64, reuse_drift=0.1,
                     reuse_frac=0.02, pack_groups=True)
    ctx.step([dev], dt, 0, cap)
    builds = []
    for k in range(n):
        b0 = ctx.query()["tree_builds"]
        ctx.step_continue(dt, 1, cap)
        if ctx.query()["tree_builds"] > b0:
            builds.append(k + 1)
    torch.cuda.synchronize()
    q = ctx.query()
    _log(f"    rebuilt before steps {builds} ({q['drift_rebuilds']} by the monitor)")
    assert 0 < q["drift_rebuilds"] and len(builds) < n
    ref = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, 1e-3, central_mass=1.0, theta=0.5,
                     n_grp=128, rebuild_at=set([0] + builds), pack=True)
    for k, f in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        assert np.max(np.abs(dev[f].cpu().numpy() - ref[k])) < 1e-10, f
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_packed_groups_on_cylindrical_tree(torch_cuda, precision):
    """Packing on a tree built in cylindrical coordinates (Sec. 4.3): packs,
    boxes, lists and forces against the oracle."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] packed groups, cylindrical tree, ring n=30000 seed 43, precision {precision}")
    s = inputs.ring(30000, 43, r_out=1.2, z_sigma=5e-4)
    r_ref, theta, eps, n_grp = 1.1, 0.4, 1e-4, 200
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp, cyl_r=r_ref, pack=True)
    assert st.gnode.size < oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp, cyl_r=r_ref).gnode.size
    ctx = bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=precision, cyl_radius=r_ref, pack_groups=True)
    ctx.build_tree([bh.to_device(s)])
    ctx.make_lists()
    _compare(ctx, st)
    out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    torch.cuda.synchronize()
    ax, ay, az, _, mag = st.accel(s.x, s.y, s.z, s.m, eps)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
    if precision == 0:
        assert np.all(err <= 1e-12 * mag), f"max err/mag {np.max(err / mag)}"
    else:
        fp32_bars(err / np.sqrt(ax ** 2 + ay ** 2 + az ** 2), "packed groups, cylindrical tree")
    ctx.close()
