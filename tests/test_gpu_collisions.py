"""GPU parity of the collision branch of Eq. (2) (Sec. 5.1) through the C ABI.

Bars as for the gravity-only path: FP64 forces per particle within 1e-12 of
the sum of the magnitudes of the terms, FP32-relative forces with median
relative error <= 1e-5, the direct-sum judge within 1e-12 of the term sum,
and FP64 leapfrog trajectories within 1e-10 of the oracle's.  The contact
decision itself is taken in FP64 on both sides, so the set of contact pairs
is identical; each case checks that it has contacts.
"""
import math
import sys

import numpy as np
import pytest

from bars import fp32_bars
from scipy.spatial import cKDTree

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


def contact_params(t_c, e):
    """Spring and dashpot of a contact lasting t_c with restitution e."""
    wd = math.pi / t_c
    gamma = -math.log(e) / t_c
    return wd * wd + gamma * gamma, 2.0 * gamma


def _contact_ring(n, seed, v_disp=3e-3):
    s = inputs.ring(n, seed, v_disp=v_disp)
    return s


def _n_contacts(s, rc):
    pts = np.stack([s.x, s.y, s.z], 1)
    return len(cKDTree(pts).query_pairs(rc))


CASES = [
    # name, n, seed, theta, eps, n_grp, rc
    ("ring20000_g64", 20000, 31, 0.5, 1e-4, 64, 2e-3),
    ("ring3001_g32_ragged", 3001, 32, 0.6, 1e-4, 32, 6e-3),
    ("ring8000_eps0", 8000, 33, 0.5, 0.0, 64, 3e-3),
    ("ring20000_g300", 20000, 34, 0.4, 1e-4, 300, 2e-3),
]


def _ctx(theta, eps, n_grp, precision, rc, kappa, eta, central_mass=0.0, use_graphs=True):
    from paper_1907_02289_amd import bh
    return bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=precision, r_coll=rc, kappa=kappa, eta=eta,
                      central_mass=central_mass, use_graphs=use_graphs)


@pytest.mark.parametrize("name,n,seed,theta,eps,n_grp,rc", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_forces_with_contacts(torch_cuda, name, n, seed, theta, eps, n_grp, rc, precision):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] contacts {name} precision={precision}")
    s = _contact_ring(n, seed)
    assert _n_contacts(s, rc) > 50
    kappa, eta = contact_params(0.02, 0.5)
    ctx = _ctx(theta, eps, n_grp, precision, rc, kappa, eta)
    dev = bh.to_device(s)
    ctx.build_tree([dev])
    ctx.make_lists()
    out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az", "pot")}
    ctx.forces([out])
    torch.cuda.synchronize()
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp)
    pc_off, pc, pp_off, pp = ctx.export("lists")
    np.testing.assert_array_equal(pp, st.pp)
    np.testing.assert_array_equal(pc, st.pc)
    ax, ay, az, pot, mag = st.accel(s.x, s.y, s.z, s.m, eps, vel=(s.vx, s.vy, s.vz), contact=(rc, kappa, eta))
    g = {k: v.cpu().numpy() for k, v in out.items()}
    err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
    # the contact terms must matter: without them the answer is far off
    nx, ny, nz, _, _ = st.accel(s.x, s.y, s.z, s.m, eps)
    moved = np.sqrt((nx - ax) ** 2 + (ny - ay) ** 2 + (nz - az) ** 2) > 1e-3 * mag
    assert moved.sum() > 50
    if precision == 0:
        assert np.all(err <= 1e-12 * mag), f"max err/mag {np.max(err / mag)}"
        np.testing.assert_allclose(g["pot"], pot, rtol=1e-12)
    else:
        rel = err / np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
        relm = err[moved] / mag[moved]
        _log(f"    fp32 rel err: median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e} max {rel.max():.2e}; "
             f"particles in contact: max err/term sum {relm.max():.2e}")
        fp32_bars(rel, "all particles")
        assert np.median(relm) <= 1e-5 and relm.max() <= 1e-4, (np.median(relm), relm.max())
    ctx.close()


def test_direct_sum_judge_with_contacts(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] direct sum with contacts")
    s = _contact_ring(30000, 35)
    rc, eps = 2e-3, 1e-4
    kappa, eta = contact_params(0.02, 0.5)
    # targets: particles that have a contact, and random ones
    pairs = np.array(sorted(cKDTree(np.stack([s.x, s.y, s.z], 1)).query_pairs(rc)))
    rng = np.random.default_rng(2)
    tg = np.unique(np.concatenate([pairs[:200, 0], rng.choice(s.n, 200, replace=False)])).astype(np.int64)
    ctx = _ctx(0.5, eps, 64, 0, rc, kappa, eta)
    dev = bh.to_device(s)
    out = {k: torch.zeros(tg.size, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.direct_sum(dev, torch.as_tensor(tg, device="cuda"), out)
    torch.cuda.synchronize()
    ax, ay, az, _ = oracle.direct(s.x, s.y, s.z, s.m, eps, targets=tg, vel=(s.vx, s.vy, s.vz),
                                  contact=(rc, kappa, eta))
    # scale: the sum of term magnitudes (theta = 0 tree sum is the direct sum)
    _, _, _, _, mag, _ = oracle.bh_accel(s.x, s.y, s.z, s.m, 0.0, eps, vel=(s.vx, s.vy, s.vz),
                                         contact=(rc, kappa, eta))
    g = {k: v.cpu().numpy() for k, v in out.items()}
    err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
    assert np.all(err <= 1e-12 * mag[tg])
    ctx.close()


def test_step_fp64_with_contacts_matches_oracle(torch_cuda):
    """KDK with contacts and list reuse: the dashpot sees the velocities held
    at each force evaluation (half-kicked after a drift) on both sides."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] step fp64 with contacts")
    s = inputs.ring(4000, 36, central_mass=1.0, v_disp=3e-3)
    theta, eps, dt, n, rc = 0.5, 1e-4, 1e-3, 7, 4e-3
    kappa, eta = contact_params(0.02, 0.5)
    assert _n_contacts(s, rc) > 50
    ref = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, eps, central_mass=1.0, theta=theta, n_grp=64,
                     rebuild_every=3, contact=(rc, kappa, eta))
    nog = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, eps, central_mass=1.0, theta=theta, n_grp=64,
                     rebuild_every=3)
    assert np.max(np.abs(ref[3] - nog[3])) > 1e-6          # the contacts change the velocities
    ctx = _ctx(theta, eps, 64, 0, rc, kappa, eta, central_mass=1.0)
    dev = bh.to_device(s)
    ctx.step([dev], dt, n, rebuild_every=3)
    torch.cuda.synchronize()
    for k, key in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        got = dev[key].cpu().numpy()
        assert np.max(np.abs(got - ref[k])) < 1e-10, key
    ctx.close()


def test_step_fp32_with_contacts_graph_equals_eager(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] step fp32 with contacts, graph vs eager")
    s = inputs.ring(20000, 37, central_mass=1.0, v_disp=3e-3)
    kappa, eta = contact_params(0.02, 0.5)
    a, b = bh.to_device(s), bh.to_device(s)
    cg = _ctx(0.5, 1e-4, 128, 1, 2e-3, kappa, eta, central_mass=1.0, use_graphs=True)
    ce = _ctx(0.5, 1e-4, 128, 1, 2e-3, kappa, eta, central_mass=1.0, use_graphs=False)
    cg.step([a], 1e-3, 2, rebuild_every=4)
    ce.step([b], 1e-3, 2, rebuild_every=4)
    for k in range(6):
        cg.step_continue(1e-3, 1, rebuild_every=4)
        ce.step_continue(1e-3, 1, rebuild_every=4)
        torch.cuda.synchronize()
        for f in ("x", "y", "z", "vx", "vy", "vz"):
            assert torch.equal(a[f], b[f]), (k, f)
    cg.close()
    ce.close()


def test_contacts_need_velocities(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    s = inputs.ring(1000, 38)
    dev = bh.to_device(s)
    for k in ("vx", "vy", "vz"):
        dev.pop(k)
    ctx = _ctx(0.5, 1e-4, 64, 1, 1e-2, 1.0, 1.0)
    ctx.build_tree([dev])
    ctx.make_lists()
    out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    with pytest.raises(bh.BHError) as e:
        ctx.forces([out])
    assert e.value.status == bh.BH_EINVAL
    with pytest.raises(bh.BHError) as e:
        ctx.set_params(kappa=-1.0)
    assert e.value.status == bh.BH_EINVAL
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_contacts_with_cylindrical_tree_and_two_systems(torch_cuda, precision):
    """The collision branch, cylindrical tree coordinates and two systems in
    one context together: each system's forces against the oracle for that
    system alone, at the same bars as above."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] contacts + cylindrical + two systems, precision={precision}")
    systems = [inputs.ring(9000, 39, v_disp=3e-3), inputs.ring(5000, 40, r_in=1.1, r_out=1.3, v_disp=3e-3)]
    rc, eps, theta, n_grp, r_ref = 3e-3, 1e-4, 0.5, 64, 1.1
    kappa, eta = contact_params(0.02, 0.5)
    for s in systems:
        assert _n_contacts(s, rc) > 20
    ctx = bh.Context(theta=theta, eps=eps, n_group=n_grp, precision=precision, r_coll=rc, kappa=kappa, eta=eta,
                     cyl_radius=r_ref)
    dev = [bh.to_device(s) for s in systems]
    ctx.build_tree(dev)
    ctx.make_lists()
    outs = [{k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")} for s in systems]
    ctx.forces(outs)
    torch.cuda.synchronize()
    for s, out in zip(systems, outs):
        st = oracle.BHState(s.x, s.y, s.z, s.m, theta, 8, n_grp, cyl_r=r_ref)
        ax, ay, az, _, mag = st.accel(s.x, s.y, s.z, s.m, eps, vel=(s.vx, s.vy, s.vz), contact=(rc, kappa, eta))
        g = {k: v.cpu().numpy() for k, v in out.items()}
        err = np.sqrt((g["ax"] - ax) ** 2 + (g["ay"] - ay) ** 2 + (g["az"] - az) ** 2)
        if precision == 0:
            assert np.all(err <= 1e-12 * mag), f"max err/mag {np.max(err / mag)}"
        else:
            rel = err / np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
            _log(f"    n={s.n}: fp32 rel err median {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e}")
            fp32_bars(rel, f"n={s.n}")
    ctx.close()


def test_step_fp64_contacts_cylindrical_matches_oracle(torch_cuda):
    """KDK with contacts on a cylindrical tree, lists reused: within 1e-10 of
    the oracle's trajectory."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] step fp64, contacts + cylindrical")
    s = inputs.ring(4000, 38, central_mass=1.0, v_disp=3e-3)
    theta, eps, dt, n, rc = 0.5, 1e-4, 1e-3, 7, 4e-3
    kappa, eta = contact_params(0.02, 0.5)
    ref = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, eps, central_mass=1.0, theta=theta, n_grp=64,
                     rebuild_every=3, contact=(rc, kappa, eta), cyl_r=1.05)
    ctx = bh.Context(theta=theta, eps=eps, n_group=64, precision=0, r_coll=rc, kappa=kappa, eta=eta,
                     central_mass=1.0, cyl_radius=1.05)
    dev = bh.to_device(s)
    ctx.step([dev], dt, n, rebuild_every=3)
    torch.cuda.synchronize()
    for k, key in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        assert np.max(np.abs(dev[key].cpu().numpy() - ref[k])) < 1e-10, key
    ctx.close()
