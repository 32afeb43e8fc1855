"""Pins for the oracle's packed groups (an option of this implementation: the
paper forms its groups from tree nodes, Sec. 4.2 (3d)).

Packing rule: below a node of more than n_grp particles, children are taken
in octant order; a child of at most n_grp particles joins the pack opened by
the previous child while the pack's count stays <= n_grp, else it opens a
new pack; a child of more than n_grp particles (split further, or a leaf of
coincident points) closes the open pack.

Checked against a hand-worked tree, and on real trees against the
invariants that fix the greedy packing: the packs partition the particles,
each is a run of consecutive small siblings under a node larger than n_grp
(or a single group node of the unpacked rule), each holds <= n_grp
particles unless it is one over-full leaf, and no pack could have taken the
first node of the next pack of the same run.
"""
import numpy as np
import pytest

import oracle
from paper_1907_02289_amd import inputs


def _tree_arrays(count, begin, first_child, n_child):
    return dict(count=np.asarray(count, np.uint32), begin=np.asarray(begin, np.uint32),
                first_child=np.asarray(first_child, np.uint32), n_child=np.asarray(n_child, np.uint8))


def test_packed_groups_worked_example():
    # root (34 particles) with children of 3, 5, 2, 6, 1, 9, 4, 4 particles;
    # the 9-particle child is split into leaves of 4 and 5.  n_grp = 8:
    # packs {3, 5} = 8, {2, 6} = 8, {1} (the 9 closes it), inside the 9:
    # {4} and {5} (4 + 5 > 8), then {4, 4} = 8.
    count = [34, 3, 5, 2, 6, 1, 9, 4, 4, 4, 5]
    begin = [0, 0, 3, 8, 10, 16, 17, 26, 30, 17, 21]
    first_child = [1, 0, 0, 0, 0, 0, 9, 0, 0, 0, 0]
    n_child = [8, 0, 0, 0, 0, 0, 2, 0, 0, 0, 0]
    g, b, c = oracle.groups_packed(_tree_arrays(count, begin, first_child, n_child), 8)
    assert g.tolist() == [1, 3, 5, 9, 10, 7]
    assert b.tolist() == [0, 8, 16, 17, 21, 26]
    assert c.tolist() == [8, 8, 1, 4, 5, 8]
    # the unpacked rule on the same tree: every child, and the two leaves
    assert oracle.groups(_tree_arrays(count, begin, first_child, n_child), 8).tolist() == \
        [1, 2, 3, 4, 5, 9, 10, 7, 8]


def test_packed_groups_overfull_leaf_closes_the_run():
    # children 2, 3, a leaf of 12 coincident points, 1, 2; n_grp = 8
    count = [20, 2, 3, 12, 1, 2]
    begin = [0, 0, 2, 5, 17, 18]
    first_child = [1, 0, 0, 0, 0, 0]
    n_child = [5, 0, 0, 0, 0, 0]
    g, b, c = oracle.groups_packed(_tree_arrays(count, begin, first_child, n_child), 8)
    assert g.tolist() == [1, 3, 4]
    assert b.tolist() == [0, 5, 17]
    assert c.tolist() == [5, 12, 3]


def test_packed_groups_small_root_and_leaf_root():
    # a root within n_grp is one group; so is a leaf root of any size
    t = _tree_arrays([5, 2, 3], [0, 0, 2], [1, 0, 0], [2, 0, 0])
    g, b, c = oracle.groups_packed(t, 8)
    assert (g.tolist(), b.tolist(), c.tolist()) == ([0], [0], [5])
    t = _tree_arrays([40], [0], [0], [0])
    g, b, c = oracle.groups_packed(t, 8)
    assert (g.tolist(), b.tolist(), c.tolist()) == ([0], [0], [40])


def _clumpy(n, seed):
    """A ring with a tenth of its particles in five clumps of radius ~5e-3:
    the nodes around a clump hold few particles each, as late in a
    fragmenting ring."""
    s = inputs.ring(n, seed)
    rng = np.random.default_rng(seed + 1000)
    k = n // 10
    idx = rng.choice(n, k, replace=False)
    centres = rng.choice(n, 5, replace=False)
    which = centres[rng.integers(0, 5, k)]
    for a in (s.x, s.y, s.z):
        a[idx] = a[which] + rng.normal(0.0, 5e-3, k)
    return s


@pytest.mark.parametrize("n,seed,n_leaf,n_grp", [(3000, 1, 8, 64), (5000, 2, 8, 256), (2000, 3, 1, 16),
                                                 (4000, 4, 8, 32)])
def test_packed_groups_invariants(n, seed, n_leaf, n_grp):
    s = _clumpy(n, seed)
    _, _, _, key = oracle.keys(s.x, s.y, s.z)
    t = oracle.tree(key[oracle.sort_perm(key)], n_leaf)
    g, b, c = oracle.groups_packed(t, n_grp)
    g0 = oracle.groups(t, n_grp)
    nn = t["begin"].size
    parent = np.full(nn, -1)
    for v in range(nn):
        parent[t["first_child"][v]:t["first_child"][v] + t["n_child"][v]] = v
    # partition of the sorted particles, in ascending order
    assert b[0] == 0 and np.all(b[1:] == b[:-1] + c[:-1]) and int(b[-1]) + int(c[-1]) == n
    # every pack is a run of consecutive nodes of the unpacked rule
    members = []
    pos = {int(v): k for k, v in enumerate(g0)}
    for k in range(g.size):
        j = pos[int(g[k])]
        run = [int(g0[j])]
        while sum(int(t["count"][u]) for u in run) < c[k]:
            j += 1
            run.append(int(g0[j]))
        assert sum(int(t["count"][u]) for u in run) == c[k]
        assert int(t["begin"][run[0]]) == b[k]
        if len(run) > 1:
            p = parent[run[0]]
            assert all(parent[u] == p for u in run)                 # siblings ...
            assert run == list(range(run[0], run[0] + len(run)))    # ... consecutive
            assert t["count"][p] > n_grp and c[k] <= n_grp
        elif c[k] > n_grp:
            assert t["n_child"][run[0]] == 0                        # an over-full leaf
        members.append(run)
    assert sorted(u for r in members for u in r) == sorted(g0.tolist())
    # greedy: the next pack's first node, a small consecutive sibling, did not fit
    for k in range(g.size - 1):
        u = members[k + 1][0]
        last = members[k][-1]
        if u == last + 1 and parent[u] == parent[last] and parent[u] >= 0 \
                and t["count"][u] <= n_grp and c[k] <= n_grp:
            assert c[k] + t["count"][u] > n_grp
    # packing merges: fewer groups here, never more
    assert g.size < g0.size


def test_packed_state_uses_pack_ranges():
    """BHState with packing: group boxes and interaction counts follow the
    packs' particle ranges."""
    s = _clumpy(3000, 7)
    st = oracle.BHState(s.x, s.y, s.z, s.m, 0.5, 8, 64, pack=True)
    _, _, q, _ = oracle.keys(s.x, s.y, s.z)
    qs = q[st.perm]
    for k in range(st.gnode.size):
        b, c = int(st.gbeg[k]), int(st.gcnt[k])
        assert list(st.gbox[k, :3]) == list(qs[b:b + c].min(0))
        assert list(st.gbox[k, 3:]) == list(qs[b:b + c].max(0) + 1)
    # forces over packed lists equal the direct sum at theta = 0
    st0 = oracle.BHState(s.x, s.y, s.z, s.m, 0.0, 8, 64, pack=True)
    ax, ay, az, _, mag = st0.accel(s.x, s.y, s.z, s.m, 1e-3)
    dx, dy, dz, _ = oracle.direct(s.x, s.y, s.z, s.m, 1e-3)
    scale = mag                                  # sum of the terms' magnitudes
    assert np.all(np.abs(ax - dx) <= 1e-12 * scale + 1e-300)
    assert np.all(np.abs(ay - dy) <= 1e-12 * scale + 1e-300)
    assert np.all(np.abs(az - dz) <= 1e-12 * scale + 1e-300)
