"""GPU checks of the drift monitor of list-reusing steps (the rebuild
trigger for the persistent interaction list of Sec. 4.2):

- per-node drift measured in the moment refresh against the oracle's
  definition over the oracle's own tree, moments and leapfrog positions
  (leaves: the leaf form itself; parents: the recurrence), and the bound
  over every node's particles; the two trajectories agree to ~1e-10, so
  the drifts do to ~1e-9;
- the monitor's two limits are the fixed schedules, bit for bit: a threshold
  never reached gives the trajectory of rebuild_every alone, a zero threshold
  rebuilds before every force evaluation like rebuild_every = 1;
- in between, the trajectory with the rebuild steps the monitor chose
  matches the oracle's leapfrog rebuilt at the same steps (FP64, 1e-10)."""
import sys

import numpy as np
import pytest

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


def _tree(ctx):
    nodes = ctx.export("nodes")
    return dict(level=nodes[:, 0], begin=nodes[:, 3], count=nodes[:, 4], first_child=nodes[:, 5],
                n_child=nodes[:, 6])


def test_node_drift_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] drift values: ring n=20000 seed 31, fp64, 3 reusing steps of dt 0.02")
    s = inputs.ring(20000, 31, central_mass=1.0, v_disp=3e-3)
    theta, eps, n_grp, dt = 0.5, 1e-3, 64, 0.02
    # the oracle's side: its tree and moments at the build, its leapfrog
    # positions after each list-reusing step, its moments there
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp)
    t, perm = st.tree, st.perm
    ms = s.m[perm]

    def sorted_xyz(x, y, z):
        return np.stack([x[perm], y[perm], z[perm]], 1)

    def com(xyz):
        mo = oracle.moments(t, xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), ms)
        return np.stack([mo["cx"], mo["cy"], mo["cz"]], 1)

    x_b = sorted_xyz(s.x, s.y, s.z)
    c_b = com(x_b)
    traj = []
    oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, 3, eps, central_mass=1.0, theta=theta, n_grp=n_grp,
               rebuild_at={0}, trace=lambda k, x, y, z, *v: traj.append(sorted_xyz(x, y, z)))
    # the GPU's side
    dev = bh.to_device(s)
    big = 1 << 30
    ctx = bh.Context(theta=theta, eps=eps, central_mass=1.0, precision=bh.FP64, n_group=n_grp,
                     reuse_drift=1e30, reuse_frac=0.0)
    ctx.step([dev], dt, 0, big)
    gt = _tree(ctx)
    np.testing.assert_array_equal(gt["begin"], t["begin"])
    np.testing.assert_array_equal(gt["count"], t["count"])
    for k in range(3):
        ctx.step_continue(dt, 1, big)
        torch.cuda.synchronize()
        got = ctx.export("drift")
        x_n = traj[k]
        want, direct = oracle.node_drift(t, x_b, x_n, c_b, com(x_n))
        leaf = t["n_child"] == 0
        assert np.max(np.abs(got - want)) <= 1e-9, np.max(np.abs(got - want))
        assert np.all(got >= direct - 1e-9)
        assert np.max(want[leaf]) > 1e-6
        _log(f"    step {k + 1}: largest leaf drift {got[leaf].max():.3e}, root bound {got[0]:.3e}, "
             f"largest difference {np.max(np.abs(got - want)):.1e}")
    assert ctx.query()["tree_builds"] == 1
    ctx.close()


def _run(bh, s, dt, n, **kw):
    import torch
    dev = bh.to_device(s)
    ctx = bh.Context(theta=0.5, eps=1e-3, central_mass=1.0, n_group=64, **kw.pop("ctx"))
    rebuild_every = kw.pop("rebuild_every")
    ctx.step([dev], dt, 0, rebuild_every)
    builds = []
    for k in range(n):
        b0 = ctx.query()["tree_builds"]
        ctx.step_continue(dt, 1, rebuild_every)
        if ctx.query()["tree_builds"] > b0:
            builds.append(k + 1)
    torch.cuda.synchronize()
    out = {f: dev[f].cpu().numpy() for f in ("x", "y", "z", "vx", "vy", "vz")}
    q = ctx.query()
    ctx.close()
    return out, builds, q


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_monitor_limits_are_the_fixed_schedules(torch_cuda, precision):
    from paper_1907_02289_amd import bh
    _log(f"[gpu] drift limits, precision {precision}: ring n=8000 seed 32, 9 steps")
    s = inputs.ring(8000, 32, central_mass=1.0, v_disp=3e-3)
    dt, n = 0.01, 9
    fixed3, b3, _ = _run(bh, s, dt, n, rebuild_every=3, ctx=dict(precision=precision))
    never, bn, qn = _run(bh, s, dt, n, rebuild_every=3,
                         ctx=dict(precision=precision, reuse_drift=1e30, reuse_frac=0.0))
    assert bn == b3 == [3, 6, 9] and qn["drift_rebuilds"] == 0
    for f in fixed3:
        np.testing.assert_array_equal(never[f], fixed3[f])
    every, b1, _ = _run(bh, s, dt, n, rebuild_every=1, ctx=dict(precision=precision))
    always, ba, qa = _run(bh, s, dt, n, rebuild_every=1 << 20,
                          ctx=dict(precision=precision, reuse_drift=1e-300, reuse_frac=0.0))
    assert ba == b1 == list(range(1, n + 1)) and qa["drift_rebuilds"] == n
    for f in every:
        np.testing.assert_array_equal(always[f], every[f])


def test_monitor_trajectory_matches_oracle(torch_cuda):
    from paper_1907_02289_amd import bh
    _log("[gpu] drift monitor trajectory: ring n=3000 seed 33, fp64, 12 steps of dt 2e-3")
    s = inputs.ring(3000, 33, central_mass=1.0, v_disp=3e-3)
    dt, n = 2e-3, 12
    got, builds, q = _run(bh, s, dt, n, rebuild_every=1 << 20,
                          ctx=dict(precision=bh.FP64, reuse_drift=0.1, reuse_frac=0.02))
    _log(f"    rebuilt before steps {builds}")
    assert 0 < len(builds) < n and q["drift_rebuilds"] == len(builds)
    ref = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, 1e-3, central_mass=1.0, theta=0.5,
                     n_grp=64, rebuild_at=set([0] + builds))
    for k, f in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        assert np.max(np.abs(got[f] - ref[k])) < 1e-10, f
