"""GPU tests of the learned opening rule (an addition to the paper's walk).

- training pairs: features and labels against the oracle computing them from
  its own tree, moments and groups for the pairs the GPU collected (the
  two sides' FP64 moment sums round differently, so a few FP32 results may
  sit one unit of the last place apart; nearly all are identical);
- the network: GPU forward bit-exact against the oracle's FP32 forward, GPU
  training gradient within 1e-4 of the FP64 oracle gradient;
- the learned walk with the weights the GPU trained: lists bit-exact against
  the oracle walking over its own tree, moments, node features and group
  data with those weights; FP64 forces on those lists within the FP64 bar;
- the gain: at matched p99 relative force error 1e-3 on a held-out ring the
  trained network needs fewer interactions than the same rule with a
  constant in its place; its ratio to the geometric rule is reported.
"""
import math
import sys

import numpy as np
import pytest

from learned_ref import assert_fp32_close, learned_inputs

import oracle
from oracle import mlp
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


def _lctx(theta=0.3, theta_min=0.05, theta_max=0.6, tau=1e-3, n_group=64, eps=1e-3):
    from paper_1907_02289_amd import bh
    return bh.Context(theta=theta, eps=eps, n_group=n_group, precision=bh.FP32_REL, criterion=bh.LEARNED,
                      theta_min=theta_min, theta_max=theta_max, tau=tau)


@pytest.fixture(scope="module")
def collected(torch_cuda):
    from paper_1907_02289_amd import bh
    _log("[gpu] learned: collect, ring n=20000 seed 21, n_group 64, band 0.05-0.6, max_groups 48, "
         "count_cap 4096")
    s = inputs.ring(20000, 21)
    ctx = _lctx()
    ctx.build_tree([bh.to_device(s)])
    ctx.mlp_collect(max_groups=48, count_cap=4096)
    pairs, X, Y = ctx.mlp_dataset()
    _log(f"    {pairs.shape[0]} pairs collected")
    yield s, ctx, pairs, X, Y
    ctx.close()


def test_features_and_labels_match_oracle(collected):
    s, ctx, pairs, X, Y = collected
    assert pairs.shape[0] > 1000
    st, L = learned_inputs(s, 0.3, 1e-3, 64)
    t, com4 = L["t"], L["com4"]
    # the GPU's tree and groups are the oracle's (bit-exact elsewhere): node and
    # group ids name the same objects on both sides
    nodes = ctx.export("nodes")
    np.testing.assert_array_equal(nodes[:, 3], t["begin"])
    np.testing.assert_array_equal(nodes[:, 4], t["count"])
    np.testing.assert_array_equal(ctx.export("groups")[:, 1], st.gbeg)
    assert_fp32_close(ctx.export("node_qn"), L["qn"], "second-moment norms", min_exact=0.999)
    Msys = com4[0, 3]
    sel = np.random.default_rng(0).choice(pairs.shape[0], 400, replace=False)
    f_want = np.zeros((sel.size, 4), np.float32)
    y_want = np.zeros(sel.size, np.float32)
    for j, k in enumerate(sel):
        g, v = int(pairs[k, 0]), int(pairs[k, 1])
        assert 2 <= t["count"][v] <= 4096
        r2 = oracle.box_ratio2(L["gbox"][g], int(t["level"][v]), int(t["prefix"][v]))
        f_want[j], _ = oracle.features(com4[v, :3], com4[v, 3], r2, L["qn"][v], L["gcen"][g], L["grad"][g], Msys)
        r = oracle.label_ratio(st.gbeg[g], st.gcnt[g], t["begin"][v], t["count"][v], L["xs"], L["ys"], L["zs"],
                               L["ms"], com4[v], L["gcen"][g], 1e-3)
        y_want[j] = np.float32(oracle.lg2p(r))
    assert_fp32_close(X[sel], f_want, "features")
    assert_fp32_close(Y[sel], y_want, "labels")


def test_network_forward_bit_exact_and_gradient(collected, torch_cuda):
    torch = torch_cuda
    s, ctx, pairs, X, Y = collected
    rng = np.random.default_rng(5)
    w = np.zeros(1259, np.float32)
    w[:1249] = rng.normal(0, 0.3, 1249)
    w[1249:1253] = X.mean(0)
    w[1253:1257] = 1.0 / (X.std(0) + 1e-6)
    w[1257], w[1258] = Y.mean(), Y.std()
    ctx.mlp_weights(set=w)
    Xd = torch.as_tensor(X, device="cuda")
    pred = ctx.mlp_predict(Xd).cpu().numpy()
    np.testing.assert_array_equal(pred, oracle.mlp_forward(w, X))
    B = 1024
    g, loss = ctx.mlp_gradient(Xd[:B], torch.as_tensor(Y[:B], device="cuda"))
    torch.cuda.synchronize()
    l64, g64 = mlp.loss_and_grad(w.astype(np.float64), X[:B], Y[:B])
    g = g.cpu().numpy()
    scale = np.abs(g64).max()
    assert np.max(np.abs(g - g64)) <= 1e-4 * scale, np.max(np.abs(g - g64)) / scale
    assert abs(float(loss.cpu()[0]) - l64) <= 1e-4 * l64


def test_learned_lists_bit_exact(collected, torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    s, ctx, pairs, X, Y = collected
    mse = ctx.mlp_train(iters=400, batch=1024, seed=3)
    _log(f"    training mse {mse:.3f} (label variance {Y.var():.3f})")
    w = ctx.mlp_weights()
    # the trained weights are a parameter of the rule, given to both sides; the
    # context runs its geometric budget pass in FP64 like the oracle
    c2 = bh.Context(theta=0.3, eps=1e-3, n_group=64, precision=bh.FP64, criterion=bh.LEARNED,
                    theta_min=0.05, theta_max=0.6, tau=3e-3)
    c2.mlp_weights(set=w)
    dev = bh.to_device(s)
    c2.build_tree([dev])
    c2.make_lists()
    out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    c2.forces([out])
    torch.cuda.synchronize()
    st, L = learned_inputs(s, 0.3, 1e-3, 64)
    want = oracle.lists_learned(L["gbox"], L["gcen"], L["grad"], L["gamin"], L["t"], L["com4"], L["qn"], w,
                                L["S"], theta=0.3, theta_min=0.05, theta_max=0.6, tau=3e-3)
    got = c2.export("lists")
    for a, b in zip(got, want):
        np.testing.assert_array_equal(a, b)
    # the rule did decide something in the band: lists differ from both geometric limits
    geo_min = oracle.lists(L["gbox"], L["t"], 0.05)
    assert got[1].size != geo_min[1].size
    # forces on the learned lists: the oracle's sums over its own lists and moments
    ax, ay, az, _, mag = oracle.forces(st.gnode, L["t"], L["xs"], L["ys"], L["zs"], L["ms"], st.mom,
                                       want[0], want[1], want[2], want[3], 1e-3, granges=(st.gbeg, st.gcnt))
    perm = st.perm
    gx, gy, gz = (out[k].cpu().numpy()[perm] for k in ("ax", "ay", "az"))
    err = np.sqrt((gx - ax) ** 2 + (gy - ay) ** 2 + (gz - az) ** 2)
    assert np.all(err <= 1e-12 * mag), f"max err/mag {np.max(err / mag)}"
    c2.close()


def _p99(ctx, dev, targets, ref, n):
    import torch
    out = {k: torch.zeros(n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    ctx.forces([out])
    a = torch.stack([out["ax"][targets], out["ay"][targets], out["az"][targets]])
    r = torch.stack([ref["ax"], ref["ay"], ref["az"]])
    e = (torch.linalg.vector_norm(a - r, dim=0) / torch.linalg.vector_norm(r, dim=0)).cpu().numpy()
    return float(np.sort(e)[int(math.ceil(0.99 * e.size)) - 1])


def test_learned_rule_gain_at_matched_error(torch_cuda):
    """Train on rings and Plummer spheres (seeds 100-102); on a held-out ring
    (seed 1) tune, each to p99 <= 1e-3 against the FP64 direct sum:
      - the geometric rule (theta),
      - the learned rule with the trained network (tau),
      - the same rule with the network replaced by a constant, the training
        set's mean label (tau).
    The trained network must need fewer interactions than the constant; the
    ratio to the geometric rule is reported (on this thin ring the geometric
    box-distance rule stays ahead: the per-node error keeps a scatter that the
    four features do not resolve)."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    eps = 1e-4
    tr = _lctx(eps=eps, n_group=128, theta_min=0.03, theta_max=0.5)
    for sysm in (inputs.ring(200000, 100, central_mass=1.0), inputs.ring(200000, 101, r_out=1.2, z_sigma=5e-4),
                 inputs.plummer(100000, 102)):
        tr.build_tree([bh.to_device(sysm)])
        tr.mlp_collect(max_groups=192, count_cap=65536)
    n_train = tr.mlp_dataset()[0].shape[0]
    mse = tr.mlp_train(iters=3000, batch=4096, seed=7)
    _log(f"[gpu] learned gain: {n_train} training pairs, mse {mse:.3f}")
    w = tr.mlp_weights()
    tr.close()
    w_const = np.zeros_like(w)
    w_const[1253:1257] = 1.0
    w_const[1257], w_const[1258] = w[1257], 1.0

    s = inputs.ring(400000, 1)
    dev = bh.to_device(s)
    tg = torch.as_tensor(inputs.force_sample(s.n, 1, 2048).astype(np.int64), device="cuda")
    ref = {k: torch.zeros(tg.numel(), dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    geo = bh.Context(theta=0.5, eps=eps, n_group=128, precision=bh.FP32_REL)
    geo.direct_sum(dev, tg, ref)
    geo.build_tree([dev])

    def bisect(f, lo, hi, iters=14):
        # largest x in [lo, hi] with f(x) <= 1e-3, f increasing in x
        best = None
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if f(mid) <= 1e-3:
                lo, best = mid, mid
            else:
                hi = mid
        return best

    def geo_err(th):
        geo.set_params(theta=th)
        geo.make_lists()
        return _p99(geo, dev, tg, ref, s.n)

    th = bisect(geo_err, 0.02, 0.6)
    geo_err(th)
    n_geo = geo.query()["interactions"]
    geo.close()
    res = {}
    for name, weights in (("trained", w), ("constant", w_const)):
        lrn = _lctx(eps=eps, n_group=128, theta=th, theta_min=0.03, theta_max=0.5)
        lrn.mlp_weights(set=weights)
        lrn.build_tree([dev])

        def lrn_err(lt):
            lrn.set_params(tau=10.0 ** lt)
            lrn.make_lists()
            return _p99(lrn, dev, tg, ref, s.n)

        lt = bisect(lrn_err, -9.0, 1.0)
        assert lt is not None
        e = lrn_err(lt)
        res[name] = lrn.query()["interactions"]
        _log(f"    {name} network: tau=1e{lt:.2f} p99={e:.2e} {res[name]:.4g} interactions")
        lrn.close()
    _log(f"    geometric theta={th:.4f}: {n_geo:.4g} interactions; trained/constant "
         f"{res['constant'] / res['trained']:.2f}x, geometric/trained {n_geo / res['trained']:.2f}x")
    assert res["trained"] < res["constant"]
    # against the method without the network (the geometric rule at matched
    # error): measured 0.94-0.96x as many interactions as the trained rule
    # (the trained rule needs more); the bar pins that relation from both sides
    assert 0.8 <= n_geo / res["trained"] <= 1.25, n_geo / res["trained"]
