"""What the trained network gains, on the GPU, with a training set that the
CPU oracle gathers (so the library's own pair collection is not used here).

Training pairs: for a sample of groups of three training systems (two rings
and a Plummer sphere, seeds 100-102), the nodes that the oracle's walk
accepts at several opening angles across the band [theta_min, theta_max),
kept when their box ratio lies in the band and they hold at least two
particles; features and labels from the oracle's learned-rule functions
(the same definitions the library's collection computes).  The library then
trains the network on them with its own GPU kernels (bh_mlp_set_dataset,
bh_mlp_train).

On a held-out ring (seed 1), each form is tuned to p99 <= 1e-3 of the
relative force error against the FP64 direct sum: the learned rule with the
trained network, the same rule with the network replaced by a constant (the
training set's mean label), and the geometric rule.  The trained network
must need fewer interactions than the constant; against the geometric rule
(the method without it) it must stay within 0.8-1.25x of its interaction
count: on these rings it needs slightly more (about 1.05x), which the test
pins rather than hides.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1907_02289_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4
N_GRP = 128
TH_MIN, TH_MAX = 0.03, 0.5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_pairs(sysm, n_groups, n_pairs, seed):
    """(features, labels) of band pairs of one system, from the oracle alone."""
    st = oracle.BHState(sysm.x, sysm.y, sysm.z, sysm.m, 0.5, 8, N_GRP, with_q=True)
    t, mom = st.tree, st.mom
    xs, ys, zs, ms = (np.asarray(a)[st.perm] for a in (sysm.x, sysm.y, sysm.z, sysm.m))
    com4 = np.stack([mom["cx"], mom["cy"], mom["cz"], mom["M"]], 1)
    side = st.S * np.ldexp(1.0, -t["level"].astype(np.int64))
    qn = np.array([oracle.node_qn(mom["Q"][v], mom["M"][v], side[v]) for v in range(t["begin"].size)],
                  np.float32)
    gbeg, gcnt = t["begin"][st.gnode], t["count"][st.gnode]
    grad = np.empty(st.gnode.size)
    for g in range(st.gnode.size):
        sl = slice(int(gbeg[g]), int(gbeg[g] + gcnt[g]))
        ext = [a[sl].max() - a[sl].min() for a in (xs, ys, zs)]
        grad[g] = 0.5 * math.sqrt(ext[0] ** 2 + ext[1] ** 2 + ext[2] ** 2)
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(st.gnode.size, min(n_groups, st.gnode.size), replace=False))
    cand = set()
    for th in np.geomspace(TH_MIN, TH_MAX, 8)[:-1]:
        pc_off, pc, _, _ = oracle.lists(st.gbox[sel], t, float(th))
        for k, g in enumerate(sel):
            for v in pc[pc_off[k]:pc_off[k + 1]]:
                if t["count"][v] >= 2:
                    cand.add((int(g), int(v)))
    cand = sorted(cand)
    pick = rng.choice(len(cand), min(n_pairs, len(cand)), replace=False)
    X, Y = [], []
    Msys = mom["M"][0]
    for k in pick:
        g, v = cand[k]
        r2 = oracle.box_ratio2(st.gbox[g], int(t["level"][v]), int(t["prefix"][v]))
        if not (TH_MIN * TH_MIN <= r2 < TH_MAX * TH_MAX):
            continue
        f, _ = oracle.features(com4[v, :3], com4[v, 3], r2, qn[v], st.gcen[g], grad[g], Msys)
        r = oracle.label_ratio(gbeg[g], gcnt[g], t["begin"][v], t["count"][v], xs, ys, zs, ms, com4[v],
                               st.gcen[g], EPS)
        X.append(f)
        Y.append(np.float32(oracle.lg2p(r)))
    return np.array(X, np.float32), np.array(Y, np.float32)


def _p99(ctx, dev, targets, ref, n):
    import torch
    out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    a = torch.stack([out["ax"][targets], out["ay"][targets], out["az"][targets]])
    r = torch.stack([ref["ax"], ref["ay"], ref["az"]])
    e = (torch.linalg.vector_norm(a - r, dim=0) / torch.linalg.vector_norm(r, dim=0)).cpu().numpy()
    return float(np.sort(e)[int(math.ceil(0.99 * e.size)) - 1])


def _bisect(f, lo, hi, iters=14):
    """Largest x in [lo, hi] (to 2^-iters of the range) with f(x) <= 1e-3, f increasing."""
    best = None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if f(mid) <= 1e-3:
            lo, best = mid, mid
        else:
            hi = mid
    return best


def test_trained_network_beats_a_constant_at_matched_error(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    Xs, Ys = [], []
    for k, sysm in enumerate((inputs.ring(60000, 100, central_mass=1.0),
                              inputs.ring(60000, 101, r_out=1.2, z_sigma=5e-4),
                              inputs.plummer(30000, 102))):
        X, Y = _oracle_pairs(sysm, 64, 25000, 200 + k)
        _log(f"[gpu] learned gain: oracle training pairs of system {k}: {Y.size}")
        Xs.append(X)
        Ys.append(Y)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    kw = dict(eps=EPS, n_group=N_GRP, precision=bh.FP32_REL, criterion=bh.LEARNED, theta_min=TH_MIN,
              theta_max=TH_MAX)
    tr = bh.Context(theta=0.3, tau=1e-3, **kw)
    tr.mlp_set_dataset(X, Y)
    pairs, X2, Y2 = tr.mlp_dataset()
    np.testing.assert_array_equal(X2, X)
    np.testing.assert_array_equal(Y2, Y)
    assert not pairs.any()
    mse = tr.mlp_train(iters=3000, batch=4096, seed=7)
    _log(f"[gpu] learned gain: {Y.size} pairs, training mse {mse:.3f} (label variance {Y.var():.3f})")
    assert mse < Y.var()
    w = tr.mlp_weights()
    tr.close()
    w_const = np.zeros_like(w)
    w_const[1253:1257] = 1.0
    w_const[1257], w_const[1258] = w[1257], 1.0

    s = inputs.ring(400000, 1)
    dev = bh.to_device(s)
    tg = torch.as_tensor(inputs.force_sample(s.n, 1, 2048).astype(np.int64), device="cuda")
    ref = {k: torch.zeros(tg.numel(), dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    geo = bh.Context(theta=0.5, eps=EPS, n_group=N_GRP, precision=bh.FP32_REL)
    geo.direct_sum(dev, tg, ref)
    geo.build_tree([dev])

    def geo_err(th):
        geo.set_params(theta=th)
        geo.make_lists()
        return _p99(geo, dev, tg, ref, s.n)

    th = _bisect(geo_err, 0.02, 0.6)
    assert th is not None
    geo_err(th)
    n_geo = geo.query()["interactions"]
    geo.close()
    res = {}
    for name, weights in (("trained", w), ("constant", w_const)):
        lrn = bh.Context(theta=th, tau=1e-3, **kw)
        lrn.mlp_weights(set=weights)
        lrn.build_tree([dev])

        def lrn_err(lt):
            lrn.set_params(tau=10.0 ** lt)
            lrn.make_lists()
            return _p99(lrn, dev, tg, ref, s.n)

        lt = _bisect(lrn_err, -9.0, 1.0)
        assert lt is not None
        e = lrn_err(lt)
        res[name] = lrn.query()["interactions"]
        _log(f"    {name} network: tau=1e{lt:.2f} p99={e:.2e} {res[name]:.4g} interactions")
        lrn.close()
    _log(f"    geometric theta={th:.4f}: {n_geo:.4g} interactions; constant/trained "
         f"{res['constant'] / res['trained']:.3f}x, geometric/trained {n_geo / res['trained']:.3f}x")
    assert res["trained"] < res["constant"]
    # against the method without the network (the geometric rule at matched
    # error): measured 0.94-0.96x as many interactions as the trained rule
    # (the trained rule needs more); the bar pins that relation from both sides
    assert 0.8 <= n_geo / res["trained"] <= 1.25, n_geo / res["trained"]
