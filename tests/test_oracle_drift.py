"""Pins for the oracle's drift of tree nodes since a build (the rebuild
monitor of list-reusing steps) and for its leapfrog with a given rebuild
schedule.

- rigid translation: every particle and every centre of mass moves alike,
  no node drifts;
- homologous expansion x -> p + (1 + a)(x - p): a particle moves by
  a (x - p) and a centre of mass by a (c - p), so the leaf form over any
  node is a * max |x_i - c| (closed form); the parents' recurrence bounds it
  from above (triangle inequality) and equals it at the leaves;
- random motion: the recurrence bounds the leaf form over every node;
- a rebuild schedule given as evaluation indices reproduces rebuild_every."""
import numpy as np

import oracle
from paper_1907_02289_amd import inputs


def _tree(n=3000, seed=4):
    s = inputs.ring(n, seed)
    st = oracle.BHState(s.x, s.y, s.z, s.m, 0.5, 8, 64)
    xs = np.stack([s.x, s.y, s.z], 1)[st.perm]
    ms = s.m[st.perm]
    return st.tree, xs, ms


def _com(t, xs, ms):
    mom = oracle.moments(t, xs[:, 0].copy(), xs[:, 1].copy(), xs[:, 2].copy(), ms)
    return np.stack([mom["cx"], mom["cy"], mom["cz"]], 1)


def test_rigid_translation_does_not_drift():
    t, xs, ms = _tree()
    u = np.array([3e-3, -2e-3, 5e-4])
    x1 = xs + u
    drift, direct = oracle.node_drift(t, xs, x1, _com(t, xs, ms), _com(t, x1, ms))
    assert drift.max() <= 1e-13 * np.linalg.norm(u) * 30


def test_homologous_expansion_closed_form():
    t, xs, ms = _tree()
    p, a = np.array([0.3, -0.2, 0.01]), 2.0 ** -7
    x1 = p + (1.0 + a) * (xs - p)
    c0 = _com(t, xs, ms)
    drift, direct = oracle.node_drift(t, xs, x1, c0, _com(t, x1, ms))
    want = np.array([a * np.linalg.norm(xs[b:b + c] - c0[v], axis=1).max()
                     for v, (b, c) in enumerate(zip(t["begin"], t["count"]))])
    np.testing.assert_allclose(direct, want, rtol=1e-9, atol=1e-15)
    leaf = t["n_child"] == 0
    np.testing.assert_array_equal(drift[leaf], direct[leaf])
    assert np.all(drift >= direct * (1 - 1e-12))
    # a parent's bound is strictly looser somewhere (children spread around it)
    assert np.any(drift[~leaf] > 1.01 * direct[~leaf])


def test_random_motion_bound():
    t, xs, ms = _tree(seed=6)
    x1 = xs + np.random.default_rng(6).normal(0, 1e-3, xs.shape)
    drift, direct = oracle.node_drift(t, xs, x1, _com(t, xs, ms), _com(t, x1, ms))
    leaf = t["n_child"] == 0
    np.testing.assert_array_equal(drift[leaf], direct[leaf])
    assert np.all(drift >= direct * (1 - 1e-12))
    single = t["count"] == 1
    assert np.all(drift[single] <= 1e-15)     # a single particle is its own centre of mass


def test_rebuild_schedule_reproduces_rebuild_every():
    s = inputs.ring(1500, 7, central_mass=1.0)
    kw = dict(dt=1e-3, n_steps=7, eps=1e-3, central_mass=1.0, theta=0.5, n_grp=64)
    a = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, rebuild_every=3, **kw)
    b = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, rebuild_at={0, 3, 6}, **kw)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    c = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, rebuild_at={0, 2, 6}, **kw)
    assert not np.array_equal(a[0], c[0])
