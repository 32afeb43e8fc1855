"""GPU parity of the cylindrical tree coordinates (Sec. 4.3, Eq. (1)) through
the C ABI: keys, permutation, tree, groups, group boxes and lists bit-exact
against the oracle (the angle is built from correctly rounded operations on
both sides); FP64 forces within 1e-12 of the term sum, FP32 median relative
error <= 1e-5; FP64 trajectories within 1e-10."""
import sys

import numpy as np
import pytest

from bars import fp32_bars

import oracle
from paper_1907_02289_amd import inputs
from test_gpu_parity import _compare_structures

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


CASES = [
    # name, system factory, r_ref, theta, eps, n_grp
    ("ring20000_g64", lambda: inputs.ring(20000, 41), 1.05, 0.5, 1e-3, 64),
    ("ring3001_g32", lambda: inputs.ring(3001, 42), 1.05, 0.6, 1e-3, 32),
    ("wide_ring30000_g256", lambda: inputs.ring(30000, 43, r_out=1.2, z_sigma=5e-4), 1.1, 0.4, 1e-4, 256),
    ("ring5000_theta0", lambda: inputs.ring(5000, 44), 1.0, 0.0, 1e-3, 64),
]


@pytest.mark.parametrize("name,make,r_ref,theta,eps,n_grp", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_cylindrical_structures_and_forces(torch_cuda, name, make, r_ref, theta, eps, n_grp, precision):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] cylindrical {name} precision={precision}")
    s = make()
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp, cyl_r=r_ref)
    ctx = bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=precision, cyl_radius=r_ref)
    ctx.build_tree([bh.to_device(s)])
    ctx.make_lists()
    _compare_structures(ctx, st, s.n)
    box = ctx.export("root_box")[0]
    assert box[0] == -np.pi and box[1] == st.lo[1] and box[2] == st.lo[2]
    out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    torch.cuda.synchronize()
    ax, ay, az, pot, mag = st.accel(s.x, s.y, s.z, s.m, eps)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
    if precision == 0:
        assert np.all(err <= 1e-12 * mag), f"max err/mag {np.max(err / mag)}"
    else:
        rel = err / np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
        _log(f"    fp32 rel err: median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e}")
        fp32_bars(rel, name)
    ctx.close()


def test_cylindrical_batched_systems(torch_cuda):
    """Two rings of different radii in one context: each system's keys and
    lists equal the oracle's for that system alone."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] cylindrical batched")
    systems = [inputs.ring(7000, 45), inputs.ring(4000, 46, r_in=1.1, r_out=1.3)]
    ctx = bh.Context(theta=0.5, eps=1e-3, n_group=64, precision=bh.FP64, cyl_radius=1.1)
    ctx.build_tree([bh.to_device(s) for s in systems])
    ctx.make_lists()
    keys = ctx.export("keys")
    groups = ctx.export("groups")
    off = [0, systems[0].n, systems[0].n + systems[1].n]
    for k, s in enumerate(systems):
        st = oracle.BHState(s.x, s.y, s.z, s.m, 0.5, 8, 64, cyl_r=1.1)
        np.testing.assert_array_equal(keys[off[k]:off[k + 1]], st.skey)
        assert np.sum(groups[:, 3] == k) == st.gnode.size
    ctx.close()


def test_cylindrical_step_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] cylindrical step fp64")
    s = inputs.ring(3000, 47, central_mass=1.0)
    theta, eps, dt, n = 0.5, 1e-3, 1e-3, 7
    ref = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, eps, central_mass=1.0, theta=theta, n_grp=64,
                     rebuild_every=3, cyl_r=1.05)
    ctx = bh.Context(theta=theta, eps=eps, n_group=64, precision=bh.FP64, central_mass=1.0, cyl_radius=1.05)
    dev = bh.to_device(s)
    ctx.step([dev], dt, n, rebuild_every=3)
    torch.cuda.synchronize()
    for k, key in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        assert np.max(np.abs(dev[key].cpu().numpy() - ref[k])) < 1e-10, key
    ctx.close()


def test_cylindrical_rejections(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    s = inputs.ring(2000, 48)
    ctx = bh.Context(theta=0.5, eps=1e-3, cyl_radius=0.01)        # 2 pi 0.01 < radial extent 0.1
    with pytest.raises(bh.BHError) as e:
        ctx.build_tree([bh.to_device(s)])
    assert e.value.status == bh.BH_EINVAL
    ctx.close()
    with pytest.raises(bh.BHError) as e:
        bh.Context(theta=0.5, eps=1e-3, cyl_radius=1.0, criterion=bh.LEARNED)
    assert e.value.status == bh.BH_EINVAL


def test_changing_tree_coordinates_needs_a_new_tree(torch_cuda):
    """The tree is built in the coordinates cyl_radius selects, so changing it
    through bh_set_params invalidates the tree: bh_make_lists is BH_ESTATE
    until bh_build_tree, and the rebuilt tree and lists are then the oracle's
    cylindrical ones, bit-exact."""
    from paper_1907_02289_amd import bh
    _log("[gpu] cyl_radius change after a Cartesian build")
    s = inputs.ring(6000, 45)
    ctx = bh.Context(theta=0.5, eps=1e-3, n_group=64)
    ctx.build_tree([bh.to_device(s)])
    ctx.make_lists()
    ctx.set_params(cyl_radius=1.05)
    with pytest.raises(bh.BHError) as e:
        ctx.make_lists()
    assert e.value.status == bh.BH_ESTATE
    ctx.build_tree([bh.to_device(s)])
    ctx.make_lists()
    st = oracle.BHState(s.x, s.y, s.z, s.m, 0.5, 8, 64, cyl_r=1.05)
    _compare_structures(ctx, st, s.n)
    ctx.close()
