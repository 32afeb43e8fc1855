"""ctypes front end of the C oracle plus the step drivers built on it.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function here
is a thin call into bh_oracle.c or plain numpy bookkeeping around it; the
arithmetic of the method lives in the C file.

Stages (Iwasawa et al. 2019, Sec. 4.2 step (3) and Sec. 5.1):
    keys -> sort -> tree -> moments -> groups -> lists -> forces
and the kick-drift-kick integrator of step (4), with the list-reuse rule of
Sec. 4.2: on a list-reusing step the tree topology, groups and lists are
kept and only the node moments are recomputed from the current positions.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

__all__ = [
    "lib", "keys", "sort_perm", "tree", "moments", "groups", "groups_packed", "group_boxes",
    "lists", "forces", "direct", "central", "bh_accel", "direct_accel",
    "kdk", "node_drift", "n_threads", "BHState", "lg2p", "node_qn", "box_ratio2", "features", "mlp_forward", "lists_learned",
    "label_ratio", "keys_cyl", "atan2", "CYL_PERIOD",
]

_lib = None


def lib():
    global _lib
    if _lib is None:
        src_m = os.path.getmtime(_build.SRC)
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < src_m:
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        L.orc_keys.argtypes = [i64, P, P, P, P, P, P, P]
        L.orc_keys.restype = C.c_int
        L.orc_sort.argtypes = [i64, P, P]
        L.orc_tree.argtypes = [i64, P, i32, i64, P, P, P, P, P, P]
        L.orc_tree.restype = i64
        L.orc_moments.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_groups.argtypes = [P, P, P, i32, i64, P]
        L.orc_groups.restype = i64
        L.orc_groups_packed.argtypes = [P, P, P, P, i32, i64, P, P, P]
        L.orc_groups_packed.restype = i64
        L.orc_group_boxes.argtypes = [i64, P, P, P, P, P, P, P, P, P]
        L.orc_lists.argtypes = [i64, P, P, P, P, P, dbl, P, P, P, P]
        L.orc_lists_p.argtypes = [i64, P, P, P, P, P, dbl, i64, P, P, P, P]
        L.orc_keys_cyl.argtypes = [i64, P, P, P, dbl, P, P, P, P]
        L.orc_keys_cyl.restype = C.c_int
        L.orc_atan2.argtypes = [dbl, dbl]
        L.orc_atan2.restype = dbl
        L.orc_forces.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, dbl, dbl, P, P, P, dbl, dbl,
                                 dbl, P, P, P, P, P]
        L.orc_direct.argtypes = [i64, P, P, P, P, dbl, dbl, i64, P, P, P, P, dbl, dbl, dbl, P, P, P, P]
        L.orc_central.argtypes = [i64, P, P, P, dbl, dbl, P, P, P]
        L.orc_threads.restype = C.c_int
        L.orc_lg2p.argtypes = [dbl]
        L.orc_lg2p.restype = dbl
        L.orc_node_qn.argtypes = [P, dbl, dbl]
        L.orc_node_qn.restype = C.c_float
        L.orc_features.argtypes = [P, dbl, dbl, C.c_float, P, dbl, dbl, P, P]
        L.orc_box_ratio2.argtypes = [P, C.c_int, C.c_uint64]
        L.orc_box_ratio2.restype = dbl
        L.orc_mlp_forward_batch.argtypes = [P, i64, P, P]
        L.orc_lists_learned.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, dbl, dbl, dbl, dbl, dbl, dbl,
                                        C.c_uint32, P, P, P, P]
        L.orc_label_ratio.argtypes = [C.c_uint32] * 4 + [P] * 6 + [dbl, dbl]
        L.orc_label_ratio.restype = dbl
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def n_threads() -> int:
    return int(lib().orc_threads())


def keys(x, y, z):
    """Root box and 63-bit keys.  Returns (lo[3], S, q[n,3] uint32, key uint64)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    lo = np.zeros(3)
    S = np.zeros(1)
    q = np.zeros((n, 3), np.uint32)
    k = np.zeros(n, np.uint64)
    rc = lib().orc_keys(n, _p(x), _p(y), _p(z), _p(lo), _p(S), _p(q), _p(k))
    if rc != 0:
        raise ValueError("oracle keys: non-finite coordinate or empty input")
    return lo, float(S[0]), q, k


CYL_PERIOD = 1 << 21      # grid units of one turn in phi (cylindrical tree coordinates)


def atan2(y, x):
    """The oracle's angle of (x, y), from correctly rounded operations only."""
    return float(lib().orc_atan2(float(y), float(x)))


def keys_cyl(x, y, z, r_ref):
    """Keys on cylindrical tree coordinates (phi, r, z) for a ring near radius
    r_ref: returns (lo[3] = (-pi, min r, min z), S = 2 pi r_ref, q[n,3], key)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    lo = np.zeros(3)
    S = np.zeros(1)
    q = np.zeros((n, 3), np.uint32)
    k = np.zeros(n, np.uint64)
    rc = lib().orc_keys_cyl(n, _p(x), _p(y), _p(z), float(r_ref), _p(lo), _p(S), _p(q), _p(k))
    if rc == -2:
        raise ValueError("oracle keys_cyl: radial or vertical extent exceeds 2 pi r_ref")
    if rc != 0:
        raise ValueError("oracle keys_cyl: non-finite coordinate, empty input or r_ref <= 0")
    return lo, float(S[0]), q, k


def sort_perm(key):
    key = np.ascontiguousarray(key, np.uint64)
    perm = np.zeros(key.size, np.uint32)
    lib().orc_sort(key.size, _p(key), _p(perm))
    return perm


def tree(skey, n_leaf):
    skey = np.ascontiguousarray(skey, np.uint64)
    n = skey.size
    cap = max(16, 2 * n + 64)
    a = dict(level=np.zeros(cap, np.uint8), prefix=np.zeros(cap, np.uint64),
             begin=np.zeros(cap, np.uint32), count=np.zeros(cap, np.uint32),
             first_child=np.zeros(cap, np.uint32), n_child=np.zeros(cap, np.uint8))
    nn = lib().orc_tree(n, _p(skey), int(n_leaf), cap, _p(a["level"]), _p(a["prefix"]),
                        _p(a["begin"]), _p(a["count"]), _p(a["first_child"]), _p(a["n_child"]))
    if nn < 0:
        raise RuntimeError("oracle tree: node capacity exceeded")
    return {k: v[:nn].copy() for k, v in a.items()}


def moments(t, xs, ys, zs, ms, with_q=False):
    nn = t["begin"].size
    M, cx, cy, cz = (np.zeros(nn) for _ in range(4))
    Q = np.zeros((nn, 6)) if with_q else None
    xs, ys, zs, ms = _f64(xs), _f64(ys), _f64(zs), _f64(ms)
    lib().orc_moments(nn, _p(t["begin"]), _p(t["count"]), _p(xs), _p(ys), _p(zs), _p(ms),
                      _p(M), _p(cx), _p(cy), _p(cz), _p(Q))
    out = dict(M=M, cx=cx, cy=cy, cz=cz)
    if with_q:
        out["Q"] = Q
    return out


def groups(t, n_grp):
    cap = t["begin"].size
    g = np.zeros(cap, np.uint32)
    ng = lib().orc_groups(_p(t["count"]), _p(t["first_child"]), _p(t["n_child"]), int(n_grp), cap, _p(g))
    if ng < 0:
        raise RuntimeError("oracle groups: capacity exceeded")
    return g[:ng].copy()


def groups_packed(t, n_grp):
    """Packed groups: (first node, particle begin, particle count) of each."""
    cap = t["begin"].size
    g, b, c = (np.zeros(cap, np.uint32) for _ in range(3))
    ng = lib().orc_groups_packed(_p(t["count"]), _p(t["begin"]), _p(t["first_child"]), _p(t["n_child"]),
                                 int(n_grp), cap, _p(g), _p(b), _p(c))
    if ng < 0:
        raise RuntimeError("oracle groups: capacity exceeded")
    return g[:ng].copy(), b[:ng].copy(), c[:ng].copy()


def group_boxes(gnode, t, skey, xs, ys, zs):
    ng = gnode.size
    gbox = np.zeros((ng, 6), np.int32)
    gcen = np.zeros((ng, 3))
    skey = np.ascontiguousarray(skey, np.uint64)
    xs, ys, zs = _f64(xs), _f64(ys), _f64(zs)
    lib().orc_group_boxes(ng, _p(gnode), _p(t["begin"]), _p(t["count"]), _p(skey),
                          _p(xs), _p(ys), _p(zs), _p(gbox), _p(gcen))
    return gbox, gcen


def lists(gbox, t, theta, period=0):
    """Interaction lists; period > 0 makes the first grid axis periodic."""
    gbox = np.ascontiguousarray(gbox, np.int32)
    ng = gbox.shape[0]
    pc_off = np.zeros(ng + 1, np.int64)
    pp_off = np.zeros(ng + 1, np.int64)
    L = lib()
    args = (_p(gbox), _p(t["level"]), _p(t["prefix"]), _p(t["first_child"]), _p(t["n_child"]),
            float(theta), int(period))
    L.orc_lists_p(ng, *args, _p(pc_off), _p(pp_off), None, None)
    pc = np.zeros(max(1, int(pc_off[-1])), np.uint32)
    pp = np.zeros(max(1, int(pp_off[-1])), np.uint32)
    L.orc_lists_p(ng, *args, _p(pc_off), _p(pp_off), _p(pc), _p(pp))
    return pc_off, pc[: pc_off[-1]].copy(), pp_off, pp[: pp_off[-1]].copy()


def _contact_args(contact, vel, n):
    """(vx, vy, vz, rc, kappa, eta) for the C calls; contact = (rc, kappa, eta)
    switches on the collision branch of Eq. (2) and then needs vel = (vx, vy, vz)."""
    if contact is None or contact[0] <= 0.0:
        return (None, None, None, 0.0, 0.0, 0.0), ()
    if vel is None:
        raise ValueError("the collision branch needs velocities")
    v = tuple(_f64(a) for a in vel)
    assert all(a.size == n for a in v)
    rc, kappa, eta = (float(a) for a in contact)
    return (_p(v[0]), _p(v[1]), _p(v[2]), rc, kappa, eta), v


def forces(gnode, t, xs, ys, zs, ms, mom, pc_off, pc, pp_off, pp, eps, G=1.0, vel=None, contact=None,
           granges=None):
    """Barnes-Hut sums over the lists (arrays in sorted order).  The groups
    are the particle ranges of the nodes gnode, or granges = (begin, count)
    of each group (packed groups).  contact = (rc, kappa, eta) adds the
    collision branch of Eq. (2) for particle sources, with vel = (vx, vy,
    vz) in sorted order."""
    n = xs.size
    ax, ay, az, pot, mag = (np.zeros(n) for _ in range(5))
    xs, ys, zs, ms = _f64(xs), _f64(ys), _f64(zs), _f64(ms)
    cargs, _keep = _contact_args(contact, vel, n)
    pc = np.ascontiguousarray(pc, np.uint32) if pc.size else np.zeros(1, np.uint32)
    pp = np.ascontiguousarray(pp, np.uint32) if pp.size else np.zeros(1, np.uint32)
    if granges is None:
        granges = (t["begin"][gnode], t["count"][gnode])
    gbeg, gcnt = (np.ascontiguousarray(a, np.uint32) for a in granges)
    lib().orc_forces(gbeg.size, _p(gbeg), _p(gcnt), _p(t["begin"]), _p(t["count"]),
                     _p(xs), _p(ys), _p(zs), _p(ms),
                     _p(mom["M"]), _p(mom["cx"]), _p(mom["cy"]), _p(mom["cz"]),
                     _p(pc_off), _p(pc), _p(pp_off), _p(pp), float(eps), float(G), *cargs,
                     _p(ax), _p(ay), _p(az), _p(pot), _p(mag))
    return ax, ay, az, pot, mag


def direct(x, y, z, m, eps, G=1.0, targets=None, vel=None, contact=None):
    """O(N * n_targets) direct sum; returns (ax, ay, az, pot) per target.
    contact = (rc, kappa, eta) with vel = (vx, vy, vz): Eq. (2) with both branches."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    tg = None if targets is None else np.ascontiguousarray(targets, np.int64)
    nt = x.size if tg is None else tg.size
    cargs, _keep = _contact_args(contact, vel, x.size)
    ax, ay, az, pot = (np.zeros(nt) for _ in range(4))
    lib().orc_direct(x.size, _p(x), _p(y), _p(z), _p(m), float(eps), float(G), nt, _p(tg), *cargs,
                     _p(ax), _p(ay), _p(az), _p(pot))
    return ax, ay, az, pot


def central(x, y, z, Mc, G, ax, ay, az):
    """Adds the external point mass at the origin to (ax, ay, az) in place."""
    lib().orc_central(x.size, _p(_f64(x)), _p(_f64(y)), _p(_f64(z)), float(Mc), float(G),
                      _p(ax), _p(ay), _p(az))


class BHState:
    """Tree, groups and lists of one build, kept for list-reusing steps."""

    def __init__(self, x, y, z, m, theta, n_leaf, n_grp, with_q=False, cyl_r=0.0, pack=False):
        if cyl_r > 0.0:
            self.lo, self.S, _, key = keys_cyl(x, y, z, cyl_r)
        else:
            self.lo, self.S, _, key = keys(x, y, z)
        self.perm = sort_perm(key)
        self.skey = key[self.perm]
        self.tree = tree(self.skey, n_leaf)
        xs, ys, zs, ms = (np.asarray(a)[self.perm] for a in (x, y, z, m))
        self.mom = moments(self.tree, xs, ys, zs, ms, with_q)
        if pack:
            self.gnode, self.gbeg, self.gcnt = groups_packed(self.tree, n_grp)
        else:
            self.gnode = groups(self.tree, n_grp)
            self.gbeg, self.gcnt = self.tree["begin"][self.gnode], self.tree["count"][self.gnode]
        # group boxes from each group's particle range (begin[id], count[id])
        self.gbox, self.gcen = group_boxes(np.arange(self.gnode.size, dtype=np.uint32),
                                           dict(begin=self.gbeg, count=self.gcnt), self.skey, xs, ys, zs)
        self.pc_off, self.pc, self.pp_off, self.pp = lists(self.gbox, self.tree, theta,
                                                           CYL_PERIOD if cyl_r > 0.0 else 0)

    def refresh(self, x, y, z, m):
        """List-reusing step: same topology, moments from the current positions."""
        xs, ys, zs, ms = (np.asarray(a)[self.perm] for a in (x, y, z, m))
        self.mom = moments(self.tree, xs, ys, zs, ms, "Q" in self.mom)

    def accel(self, x, y, z, m, eps, G=1.0, vel=None, contact=None):
        xs, ys, zs, ms = (np.asarray(a)[self.perm] for a in (x, y, z, m))
        vs = None if vel is None else tuple(np.asarray(a)[self.perm] for a in vel)
        ax, ay, az, pot, mag = forces(self.gnode, self.tree, xs, ys, zs, ms, self.mom,
                                      self.pc_off, self.pc, self.pp_off, self.pp, eps, G, vs, contact,
                                      granges=(self.gbeg, self.gcnt))
        out = [np.empty_like(ax) for _ in range(5)]
        for o, a in zip(out, (ax, ay, az, pot, mag)):
            o[self.perm] = a
        return tuple(out)

    def interactions(self):
        """Pairs evaluated: sum over groups of n_g * (particles in pp leaves + pc cells)."""
        cnt = self.tree["count"]
        ng = self.gcnt.astype(np.int64)
        pp_len = np.add.reduceat(cnt[self.pp].astype(np.int64), self.pp_off[:-1]) if self.pp.size else 0
        pp_len = np.where(np.diff(self.pp_off) > 0, pp_len, 0)
        pc_len = np.diff(self.pc_off)
        return int(np.sum(ng * (pp_len + pc_len)))


def bh_accel(x, y, z, m, theta, eps, n_leaf=8, n_grp=64, G=1.0, vel=None, contact=None, cyl_r=0.0):
    """Full Barnes-Hut force in caller order: (ax, ay, az, pot, magsum, state)."""
    st = BHState(x, y, z, m, theta, n_leaf, n_grp, cyl_r=cyl_r)
    return (*st.accel(x, y, z, m, eps, G, vel, contact), st)


def direct_accel(x, y, z, m, eps, G=1.0, vel=None, contact=None):
    ax, ay, az, pot = direct(x, y, z, m, eps, G, vel=vel, contact=contact)
    return ax, ay, az, pot


def kdk(x, y, z, vx, vy, vz, m, dt, n_steps, eps, G=1.0, central_mass=0.0,
        theta=None, n_leaf=8, n_grp=64, rebuild_every=1, contact=None, trace=None, cyl_r=0.0,
        rebuild_at=None, pack=False):
    """Kick-drift-kick leapfrog in FP64 (the integration step (4) of Sec. 4.2).

    theta=None uses the direct sum; otherwise Barnes-Hut with lists rebuilt
    every `rebuild_every` steps and moments refreshed on the other steps.
    contact = (rc, kappa, eta) adds the collision branch of Eq. (2); its
    dashpot sees the velocities held when the force is evaluated: the
    initial ones for the first evaluation, the half-kicked ones after each
    drift.  cyl_r > 0 builds the trees on cylindrical coordinates around
    that radius.  rebuild_at, if given, replaces rebuild_every: the set of
    force evaluations (0 = the first, k = the one ending step k) before which
    the tree and lists are built.  pack packs small sibling groups.  trace, if given, is called as
    trace(step, x, y, z, vx, vy, vz) after every completed step.  Returns new
    copies of (x, y, z, vx, vy, vz).
    """
    x, y, z, vx, vy, vz = (np.array(a, dtype=np.float64, copy=True) for a in (x, y, z, vx, vy, vz))
    m = _f64(m)
    state = None

    def acc(step):
        nonlocal state
        vel = (vx, vy, vz) if contact is not None else None
        if theta is None:
            ax, ay, az, _ = direct(x, y, z, m, eps, G, vel=vel, contact=contact)
        else:
            build = step % rebuild_every == 0 if rebuild_at is None else step in rebuild_at
            if state is None or build:
                state = BHState(x, y, z, m, theta, n_leaf, n_grp, cyl_r=cyl_r, pack=pack)
            else:
                state.refresh(x, y, z, m)
            ax, ay, az, _, _ = state.accel(x, y, z, m, eps, G, vel, contact)
        if central_mass:
            central(x, y, z, central_mass, G, ax, ay, az)
        return ax, ay, az

    ax, ay, az = acc(0)
    h = 0.5 * dt
    for k in range(n_steps):
        vx += h * ax
        vy += h * ay
        vz += h * az
        x += dt * vx
        y += dt * vy
        z += dt * vz
        ax, ay, az = acc(k + 1)
        vx += h * ax
        vy += h * ay
        vz += h * az
        if trace is not None:
            trace(k, x, y, z, vx, vy, vz)
    return x, y, z, vx, vy, vz


def node_drift(t, x_build, x_now, com_build, com_now):
    """Drift of every tree node since the build (the rebuild monitor of
    list-reusing steps; the paper reuses lists for a fixed number of steps,
    Sec. 4.2, this measures when the moved particles have left the build's
    geometry).  For a leaf: the largest distance by which one of its
    particles has moved relative to the leaf's centre of mass,
        max_i |(x_i - x_i^build) - (c - c^build)|;
    for a parent: the largest over its children of the child's drift plus
    the child's centre-of-mass motion relative to the parent's, a bound of
    the leaf form over the parent's particles.  x_*: (n, 3) positions in the
    tree's order; com_*: (n_nodes, 3) centres of mass.  Returns
    (drift, direct): direct is the leaf form over each node's particles."""
    x_build = np.asarray(x_build, np.float64)
    x_now = np.asarray(x_now, np.float64)
    dc = np.asarray(com_now, np.float64) - np.asarray(com_build, np.float64)
    nn = t["begin"].size
    drift = np.zeros(nn)
    direct = np.zeros(nn)
    for v in range(nn - 1, -1, -1):          # children have larger ids than their parents
        b, c = int(t["begin"][v]), int(t["count"][v])
        e = (x_now[b:b + c] - x_build[b:b + c]) - dc[v]
        direct[v] = np.sqrt(e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1] + e[:, 2] * e[:, 2]).max()
        if t["n_child"][v] == 0:
            drift[v] = direct[v]
        else:
            f = int(t["first_child"][v])
            ch = np.arange(f, f + int(t["n_child"][v]))
            q = dc[ch] - dc[v]
            drift[v] = (drift[ch] + np.sqrt(q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1] + q[:, 2] * q[:, 2])).max()
    return drift, direct


# ---------------------------------------------------------------------------
# Learned opening rule (an addition to the walk; see bh_oracle.c)
# ---------------------------------------------------------------------------
def lg2p(x):
    return float(lib().orc_lg2p(float(x)))


def node_qn(Q6, M, side):
    Q6 = np.ascontiguousarray(Q6, np.float64)
    return float(lib().orc_node_qn(_p(Q6), float(M), float(side)))


def box_ratio2(gbox, level, prefix):
    gbox = np.ascontiguousarray(gbox, np.int32)
    return float(lib().orc_box_ratio2(_p(gbox), int(level), int(prefix)))


def features(com, M, r2, qn, gcen, grad, Msys):
    """Four FP32 features and d^2 of a (group, node) pair (r2 = box_ratio2)."""
    com = np.ascontiguousarray(com, np.float64)
    gcen = np.ascontiguousarray(gcen, np.float64)
    f = np.zeros(4, np.float32)
    d2 = np.zeros(1)
    lib().orc_features(_p(com), float(M), float(r2), C.c_float(qn), _p(gcen), float(grad), float(Msys),
                       _p(f), _p(d2))
    return f, float(d2[0])


def mlp_forward(w, X):
    """FP32 network output for rows of X (n x 4), weights w (1259 floats)."""
    w = np.ascontiguousarray(w, np.float32)
    X = np.ascontiguousarray(X, np.float32).reshape(-1, 4)
    out = np.zeros(X.shape[0], np.float32)
    lib().orc_mlp_forward_batch(_p(w), X.shape[0], _p(X), _p(out))
    return out


def lists_learned(gbox, gcen, grad, gamin, t, com4, qn, w, S, theta, theta_min, theta_max, tau, G=1.0,
                  count_cap=65536):
    """Lists of one system's groups under the learned rule (CSR, ascending ids)."""
    gbox = np.ascontiguousarray(gbox, np.int32)
    gcen = np.ascontiguousarray(gcen, np.float64)
    grad = np.ascontiguousarray(grad, np.float64)
    gamin = np.ascontiguousarray(gamin, np.float64)
    com4 = np.ascontiguousarray(com4, np.float64)
    qn = np.ascontiguousarray(qn, np.float32)
    w = np.ascontiguousarray(w, np.float32)
    ng = gbox.shape[0]
    pc_off = np.zeros(ng + 1, np.int64)
    pp_off = np.zeros(ng + 1, np.int64)
    count = np.ascontiguousarray(t["count"], np.uint32)
    args = [_p(gbox), _p(gcen), _p(grad), _p(gamin), _p(t["level"]), _p(t["prefix"]), _p(count),
            _p(t["first_child"]), _p(t["n_child"]), _p(com4), _p(qn), _p(w), float(S), float(theta),
            float(theta_min), float(theta_max), float(tau), float(G), int(count_cap)]
    L = lib()
    L.orc_lists_learned(ng, *args, _p(pc_off), _p(pp_off), None, None)
    pc = np.zeros(max(1, int(pc_off[-1])), np.uint32)
    pp = np.zeros(max(1, int(pp_off[-1])), np.uint32)
    L.orc_lists_learned(ng, *args, _p(pc_off), _p(pp_off), _p(pc), _p(pp))
    return pc_off, pc[: pc_off[-1]].copy(), pp_off, pp[: pp_off[-1]].copy()


def label_ratio(gbeg, gcnt, cbeg, ccnt, xs, ys, zs, ms, com4, gcen, eps, G=1.0):
    xs, ys, zs, ms = _f64(xs), _f64(ys), _f64(zs), _f64(ms)
    com4 = np.ascontiguousarray(com4, np.float64)
    gcen = np.ascontiguousarray(gcen, np.float64)
    return float(lib().orc_label_ratio(int(gbeg), int(gcnt), int(cbeg), int(ccnt), _p(xs), _p(ys), _p(zs),
                                       _p(ms), _p(com4), _p(gcen), float(eps), float(G)))
