"""Inputs of the learned opening rule computed by the oracle alone (tree,
moments, second-moment norms, groups, group radii and error budgets), for
the GPU tests that compare the library's learned walk and training pairs
with the oracle's."""
import numpy as np

import oracle


def learned_inputs(s, theta, eps, n_grp, n_leaf=8, pack=False, budget_min=False):
    """Oracle state of system s with everything the learned rule reads:
    returns (state, dict(t, com4, qn, gbox, gcen, grad, gamin, S, xs, ys,
    zs, ms)).  The budget scale A_g is the mean (budget_min: the smallest)
    FP64 |a| of the group's particles under the geometric rule at theta."""
    st = oracle.BHState(s.x, s.y, s.z, s.m, theta, n_leaf, n_grp, with_q=True, pack=pack)
    t = st.tree
    xs, ys, zs, ms = (np.asarray(a, np.float64)[st.perm] for a in (s.x, s.y, s.z, s.m))
    ng = st.gnode.size
    grad = np.empty(ng)
    for g in range(ng):
        b, c = int(st.gbeg[g]), int(st.gcnt[g])
        ex = xs[b:b + c].max() - xs[b:b + c].min()
        ey = ys[b:b + c].max() - ys[b:b + c].min()
        ez = zs[b:b + c].max() - zs[b:b + c].min()
        grad[g] = 0.5 * np.sqrt(ex * ex + ey * ey + ez * ez)
    ax, ay, az, _, _ = st.accel(s.x, s.y, s.z, s.m, eps)
    amag = np.sqrt(ax * ax + ay * ay + az * az)[st.perm]
    red = np.min if budget_min else np.mean
    gamin = np.array([red(amag[int(b):int(b) + int(c)]) for b, c in zip(st.gbeg, st.gcnt)])
    mom = st.mom
    com4 = np.stack([mom["cx"], mom["cy"], mom["cz"], mom["M"]], 1)
    side = st.S * np.ldexp(1.0, -t["level"].astype(np.int64))
    qn = np.array([oracle.node_qn(mom["Q"][v], mom["M"][v], side[v]) for v in range(t["begin"].size)],
                  np.float32)
    return st, dict(t=t, com4=com4, qn=qn, gbox=st.gbox, gcen=st.gcen, grad=grad, gamin=gamin, S=st.S,
                    xs=xs, ys=ys, zs=zs, ms=ms)


def assert_fp32_close(got, want, what, min_exact=0.99, max_ulps=2):
    """FP32 values the GPU computed from its own FP64 moments against the
    oracle's from its moments.  The two moment sums round differently (by a
    few units of 2^-53), which can move an FP32 result across a rounding
    boundary: at least min_exact of the values must be identical and every
    value within max_ulps FP32 units of the last place."""
    got = np.asarray(got, np.float32)
    want = np.asarray(want, np.float32)
    assert got.shape == want.shape, what
    same = got == want
    ulp = np.spacing(np.maximum(np.abs(got), np.abs(want)).astype(np.float32))
    far = np.abs(got.astype(np.float64) - want.astype(np.float64)) > max_ulps * ulp.astype(np.float64)
    assert not far.any(), (what, int(far.sum()), got[far][:5], want[far][:5])
    assert same.mean() >= min_exact, (what, float(same.mean()))
