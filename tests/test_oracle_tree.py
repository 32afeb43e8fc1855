"""Pins for the oracle's keys, sort, tree, moments, groups and lists.

Each check compares the oracle with something other than itself: a string
bit interleave, the classic "most significant differing bit" Morton
comparison, numpy's lexsort, a set-based tree built from the split rule,
exact rational arithmetic, and invariants the structures must satisfy.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1907_02289_amd import inputs


def _grid_points(rng, n, S_exp=2):
    """Points with known grid coordinates: a box [0, 3]^3 (so S = 4) and
    x = (q + 1/2) * S / 2^21, exact in FP64."""
    q = rng.integers(0, 3 << 19, size=(n, 3))
    pts = (q + 0.5) * (2.0 ** S_exp) / 2.0 ** 21
    pts[0] = 0.0
    pts[1] = 3.0
    q[0] = 0
    q[1] = 3 << 19
    return pts, q


def _key_by_string(qx, qy, qz):
    s = "".join(f"{(qx >> k) & 1}{(qy >> k) & 1}{(qz >> k) & 1}" for k in range(20, -1, -1))
    return int(s, 2)


def _morton_less(a, b):
    """a before b in Morton order (x major within each triple), without keys."""
    best_d, best_x = -1, 0
    for d in range(3):
        x = int(a[d]) ^ int(b[d])
        # a later axis wins only with a strictly higher differing bit
        if x.bit_length() > best_x.bit_length():
            best_d, best_x = d, x
    if best_d < 0:
        return False
    return int(a[best_d]) < int(b[best_d])


def test_root_box_side():
    for w, S in [(3.0, 4.0), (4.0, 8.0), (0.75, 1.0), (1e-3, 2.0 ** -9), (0.0, 1.0)]:
        x = np.array([0.0, w]) + 5.0 if w else np.array([5.0])
        lo, S_got, q, k = oracle.keys(x, np.zeros_like(x), np.zeros_like(x))
        assert S_got == S
        assert lo[0] == 5.0


def test_keys_hand_placed():
    pts = np.array([[0.0, 0.0, 0.0], [2.5, 0.0, 2.5], [3.0, 3.0, 3.0], [0.0, 0.5, 0.0]])
    lo, S, q, k = oracle.keys(pts[:, 0], pts[:, 1], pts[:, 2])
    assert S == 4.0 and list(lo) == [0.0, 0.0, 0.0]
    assert k[0] == 0
    assert int(k[1]) >> 60 == 0b101                  # octant (1, 0, 1) at level 1
    assert int(k[3]) >> 54 == 0b000_000_010           # q_y = 2^18: y bit of the third triple
    assert list(q[2]) == [3 << 19] * 3
    assert int(k[2]) >> 57 == 0b111_111


def test_keys_grid_and_interleave():
    rng = np.random.default_rng(7)
    pts, qtrue = _grid_points(rng, 3000)
    lo, S, q, k = oracle.keys(pts[:, 0], pts[:, 1], pts[:, 2])
    assert S == 4.0
    np.testing.assert_array_equal(q, qtrue)
    for i in range(0, 3000, 7):
        assert int(k[i]) == _key_by_string(*map(int, qtrue[i]))
    # key order agrees with the Morton order computed without keys
    for _ in range(2000):
        i, j = rng.integers(0, 3000, 2)
        assert (int(k[i]) < int(k[j])) == _morton_less(qtrue[i], qtrue[j])


def test_keys_reject_nonfinite():
    x = np.array([0.0, np.nan, 1.0])
    with pytest.raises(ValueError):
        oracle.keys(x, x * 0, x * 0)


def test_sort_is_lexsort():
    rng = np.random.default_rng(3)
    key = rng.integers(0, 50, 5000).astype(np.uint64)        # many ties
    perm = oracle.sort_perm(key)
    np.testing.assert_array_equal(perm, np.lexsort((np.arange(5000), key)))


def _brute_tree(skey, n_leaf):
    """Nodes as (level, prefix, begin, count) from the split rule alone."""
    out = []
    frontier = [0]
    for lvl in range(22):
        nxt = []
        for p in frontier:
            sel = np.nonzero((skey >> np.uint64(3 * (21 - lvl))) == np.uint64(p))[0]
            out.append((lvl, p, int(sel[0]), int(sel.size)))
            if sel.size > n_leaf and lvl < 21:
                kids = np.unique(skey[sel] >> np.uint64(3 * (20 - lvl)))
                nxt.extend(int(c) for c in kids)
        frontier = sorted(nxt)
    return out


@pytest.mark.parametrize("n,n_leaf,seed", [(1, 8, 0), (8, 8, 1), (9, 8, 2), (700, 8, 3), (1500, 1, 4)])
def test_tree_against_split_rule(n, n_leaf, seed):
    s = inputs.ring(n, seed)
    _, _, _, key = oracle.keys(s.x, s.y, s.z)
    skey = np.sort(key)
    t = oracle.tree(skey, n_leaf)
    want = _brute_tree(skey, n_leaf)
    got = list(zip(t["level"].tolist(), t["prefix"].tolist(), t["begin"].tolist(), t["count"].tolist()))
    assert got == want
    # child links: children of v are exactly the next-level nodes extending v's prefix
    nn = len(got)
    for v in range(nn):
        kids = [u for u in range(nn) if t["level"][u] == t["level"][v] + 1
                and (int(t["prefix"][u]) >> 3) == int(t["prefix"][v])]
        assert t["n_child"][v] == len(kids)
        if kids:
            assert kids == list(range(t["first_child"][v], t["first_child"][v] + len(kids)))
            assert sum(int(t["count"][u]) for u in kids) == int(t["count"][v])
        else:
            assert t["count"][v] <= n_leaf or t["level"][v] == 21


def test_tree_coincident_points_stop_at_level_21():
    x = np.array([0.0] * 12 + [1.0])
    _, _, _, key = oracle.keys(x, x, x)
    t = oracle.tree(np.sort(key), 8)
    leaf = np.nonzero(t["n_child"] == 0)[0]
    big = [v for v in leaf if t["count"][v] == 12]
    assert len(big) == 1 and t["level"][big[0]] == 21


def test_moments_exact_on_dyadic_inputs():
    rng = np.random.default_rng(5)
    n = 1200
    x, y, z = (rng.integers(-1024, 1024, n) / 1024.0 for _ in range(3))
    m = 2.0 ** -rng.integers(3, 9, n).astype(float)
    _, _, _, key = oracle.keys(x, y, z)
    perm = oracle.sort_perm(key)
    xs, ys, zs, ms = x[perm], y[perm], z[perm], m[perm]
    t = oracle.tree(key[perm], 8)
    mom = oracle.moments(t, xs, ys, zs, ms)
    for v in range(0, t["begin"].size, 5):
        b, c = int(t["begin"][v]), int(t["count"][v])
        M = sum(Fraction(a) for a in ms[b:b + c])
        assert mom["M"][v] == float(M)
        for arr, key_ in ((xs, "cx"), (ys, "cy"), (zs, "cz")):
            S1 = sum(Fraction(mm) * Fraction(a) for mm, a in zip(ms[b:b + c], arr[b:b + c]))
            assert mom[key_][v] == float(S1 / M)


def _build(n, seed, n_leaf, n_grp, theta):
    s = inputs.ring(n, seed)
    _, _, _, key = oracle.keys(s.x, s.y, s.z)
    perm = oracle.sort_perm(key)
    skey = key[perm]
    t = oracle.tree(skey, n_leaf)
    xs, ys, zs = s.x[perm], s.y[perm], s.z[perm]
    g = oracle.groups(t, n_grp)
    gbox, gcen = oracle.group_boxes(g, t, skey, xs, ys, zs)
    lists = oracle.lists(gbox, t, theta)
    return s, perm, skey, t, g, gbox, gcen, lists


def test_groups_rule_and_cover():
    s, perm, skey, t, g, gbox, gcen, _ = _build(900, 11, 8, 32, 0.5)
    begin, count = t["begin"][g], t["count"][g]
    assert np.all(np.diff(begin.astype(np.int64)) > 0)
    assert begin[0] == 0 and int(begin[-1]) + int(count[-1]) == 900
    assert np.all(begin[1:] == begin[:-1] + count[:-1])               # disjoint cover
    parent = {}
    for v in range(t["begin"].size):
        for c in range(t["n_child"][v]):
            parent[int(t["first_child"][v]) + c] = v
    for v in g:
        assert count[list(g).index(v)] <= 32 or t["n_child"][v] == 0
        if v != 0:
            assert t["count"][parent[int(v)]] > 32
    # boxes hold every particle's grid coordinate; centre is the bbox midpoint
    _, _, q, _ = oracle.keys(s.x, s.y, s.z)
    qs = q[perm]
    for k, v in enumerate(g):
        b, c = int(t["begin"][v]), int(t["count"][v])
        assert list(gbox[k, :3]) == list(qs[b:b + c].min(0))
        assert list(gbox[k, 3:]) == list(qs[b:b + c].max(0) + 1)
        for d, a in enumerate((s.x[perm], s.y[perm], s.z[perm])):
            assert gcen[k, d] == 0.5 * (a[b:b + c].min() + a[b:b + c].max())


def _accept_exact(gb, lvl, pfx, theta):
    """Opening test in exact rationals from its geometric statement: the cell
    lies outside the group box and side / distance(cell centre, box) < theta."""
    side = 1 << (21 - lvl)
    corner = [0, 0, 0]
    for k in range(lvl):
        corner[0] |= ((pfx >> (3 * k + 2)) & 1) << k
        corner[1] |= ((pfx >> (3 * k + 1)) & 1) << k
        corner[2] |= ((pfx >> (3 * k)) & 1) << k
    corner = [c << (21 - lvl) for c in corner]
    outside = any(corner[a] + side <= gb[a] or corner[a] >= gb[3 + a] for a in range(3))
    d2 = Fraction(0)
    for a in range(3):
        c = Fraction(corner[a]) + Fraction(side, 2)
        nearest = min(max(c, Fraction(int(gb[a]))), Fraction(int(gb[3 + a])))
        d2 += (c - nearest) ** 2
    return outside and Fraction(side) ** 2 < Fraction(theta) ** 2 * d2


@pytest.mark.parametrize("theta", [0.25, 0.5, 0.75])
def test_lists_declarative(theta):
    n = 400
    s, perm, skey, t, g, gbox, gcen, (pc_off, pc, pp_off, pp) = _build(n, 21, 4, 16, theta)
    nn = t["begin"].size
    parent = np.full(nn, -1)
    for v in range(nn):
        for c in range(t["n_child"][v]):
            parent[t["first_child"][v] + c] = v
    for k in range(g.size):
        acc = [_accept_exact(gbox[k], int(t["level"][v]), int(t["prefix"][v]), theta) for v in range(nn)]

        def anc_accepted(v):
            u = parent[v]
            while u >= 0:
                if acc[u]:
                    return True
                u = parent[u]
            return False

        want_pc = [v for v in range(nn) if acc[v] and not anc_accepted(v)]
        want_pp = [v for v in range(nn) if t["n_child"][v] == 0 and not acc[v] and not anc_accepted(v)]
        assert pc[pc_off[k]:pc_off[k + 1]].tolist() == want_pc
        assert pp[pp_off[k]:pp_off[k + 1]].tolist() == want_pp


def test_lists_cover_every_particle_once():
    n = 3000
    s, perm, skey, t, g, gbox, gcen, (pc_off, pc, pp_off, pp) = _build(n, 5, 8, 64, 0.6)
    for k in range(g.size):
        cover = np.zeros(n, np.int64)
        for v in np.concatenate([pc[pc_off[k]:pc_off[k + 1]], pp[pp_off[k]:pp_off[k + 1]]]):
            cover[t["begin"][v]:t["begin"][v] + t["count"][v]] += 1
        assert np.all(cover == 1)


def test_lists_special_cases():
    # theta = 0: nothing is accepted, every leaf is in every particle list
    s, perm, skey, t, g, gbox, gcen, (pc_off, pc, pp_off, pp) = _build(500, 2, 8, 64, 0.0)
    leaves = np.nonzero(t["n_child"] == 0)[0]
    assert pc.size == 0
    for k in range(g.size):
        assert pp[pp_off[k]:pp_off[k + 1]].tolist() == leaves.tolist()
    # n <= n_leaf: one node, one group, one particle-list entry
    s, perm, skey, t, g, gbox, gcen, (pc_off, pc, pp_off, pp) = _build(8, 2, 8, 64, 0.5)
    assert t["begin"].size == 1 and g.tolist() == [0] and pp.tolist() == [0] and pc.size == 0
