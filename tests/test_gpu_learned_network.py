"""GPU checks of the learned opening rule that need no training-pair
collection: the network's inference and training-gradient kernels on
synthetic features, and the learned walk with fixed weights.

- forward: bit-exact against the oracle's FP32 forward (same fused
  multiply-add chains in the same order);
- gradient of the mean squared error: within 1e-4 of the FP64 oracle
  gradient (itself pinned by finite differences on the CPU), for full and
  ragged batches;
- learned walk: lists bit-exact against the oracle walking over its own
  tree, moments, node features and group data with the same weights, for
  tree-node and packed groups.
"""
import sys

import numpy as np
import pytest

from learned_ref import learned_inputs

import oracle
from oracle import mlp
from paper_1907_02289_amd import inputs

pytestmark = pytest.mark.gpu

NPARAM = 1259


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _synthetic(n, seed):
    """Features on the scale of the rule's lg2p features and a smooth target."""
    rng = np.random.default_rng(seed)
    X = np.stack([rng.normal(-6.0, 2.0, n), rng.normal(-3.0, 1.5, n), rng.normal(-12.0, 3.0, n),
                  rng.normal(-4.0, 1.0, n)], 1).astype(np.float32)
    Y = (0.8 * X[:, 0] + 0.3 * X[:, 1] - 0.1 * X[:, 3] + np.sin(X[:, 2]) + rng.normal(0, 0.1, n)).astype(np.float32)
    return X, Y


def _weights(X, Y, seed):
    rng = np.random.default_rng(seed)
    w = np.zeros(NPARAM, np.float32)
    w[:1249] = rng.normal(0, 0.3, 1249)
    w[1249:1253] = X.mean(0)
    w[1253:1257] = 1.0 / (X.std(0) + 1e-6)
    w[1257], w[1258] = Y.mean(), Y.std()
    return w


def test_network_forward_bit_exact(torch_cuda):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] learned network: forward")
    X, Y = _synthetic(5001, 1)
    w = _weights(X, Y, 2)
    ctx = bh.Context(theta=0.5, eps=1e-3, precision=bh.FP32_REL)
    ctx.mlp_weights(set=w)
    pred = ctx.mlp_predict(torch.as_tensor(X, device="cuda")).cpu().numpy()
    np.testing.assert_array_equal(pred, oracle.mlp_forward(w, X))
    ctx.close()


@pytest.mark.parametrize("batch", [1024, 777])
def test_network_gradient_matches_fp64(torch_cuda, batch):
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] learned network: gradient, batch {batch}")
    X, Y = _synthetic(batch, 3)
    w = _weights(X, Y, 4)
    ctx = bh.Context(theta=0.5, eps=1e-3, precision=bh.FP32_REL)
    ctx.mlp_weights(set=w)
    g, loss = ctx.mlp_gradient(torch.as_tensor(X, device="cuda"), torch.as_tensor(Y, device="cuda"))
    torch.cuda.synchronize()
    l64, g64 = mlp.loss_and_grad(w.astype(np.float64), X, Y)
    g = g.cpu().numpy()
    scale = np.abs(g64).max()
    assert np.max(np.abs(g - g64)) <= 1e-4 * scale, np.max(np.abs(g - g64)) / scale
    assert abs(float(loss.cpu()[0]) - l64) <= 1e-4 * l64
    ctx.close()


@pytest.mark.parametrize("pack", [False, True], ids=["tree_groups", "packed_groups"])
def test_learned_walk_with_fixed_weights(torch_cuda, pack):
    """Lists of the learned rule (band theta_min..theta_max, error budget tau)
    with hand-set weights: bit-exact against the oracle's learned walk over
    the oracle's own tree, moments, second-moment norms, groups and budgets.
    The context runs its geometric budget pass in FP64, so both budgets are
    FP64 sums of the same terms and agree to rounding, far inside anything
    that moves a decision."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    n_grp = 384 if pack else 64
    _log(f"[gpu] learned walk, fixed weights, ring n=20000 seed 51, groups <= {n_grp}{' packed' if pack else ''}")
    s = inputs.ring(20000, 51)
    X, Y = _synthetic(4096, 5)
    w = _weights(X, Y, 6)
    ctx = bh.Context(theta=0.3, eps=1e-3, n_group=n_grp, precision=bh.FP64, criterion=bh.LEARNED,
                     theta_min=0.05, theta_max=0.6, tau=3e-3, pack_groups=pack)
    ctx.mlp_weights(set=w)
    ctx.build_tree([bh.to_device(s)])
    ctx.make_lists()
    torch.cuda.synchronize()
    st, L = learned_inputs(s, 0.3, 1e-3, n_grp, pack=pack)
    want = oracle.lists_learned(L["gbox"], L["gcen"], L["grad"], L["gamin"], L["t"], L["com4"], L["qn"], w,
                                L["S"], theta=0.3, theta_min=0.05, theta_max=0.6, tau=3e-3)
    got = ctx.export("lists")
    for a, b in zip(got, want):
        np.testing.assert_array_equal(a, b)
    # the network did decide something inside the band: the lists differ from
    # both geometric limits
    lo = oracle.lists(L["gbox"], L["t"], 0.05)
    hi = oracle.lists(L["gbox"], L["t"], 0.6)
    assert got[1].size != lo[1].size and got[1].size != hi[1].size
    _log(f"    node-list entries: theta_max {hi[1].size}, learned {got[1].size}, theta_min {lo[1].size}")
    ctx.close()


def test_parameters_and_calls_without_weights(torch_cuda):
    """The network calls need weights: inference and gradient are BH_ESTATE
    until weights are set, then run.  Out-of-range band parameters of the
    learned rule are BH_EINVAL, and the context (and the binding's copy)
    keep the previous ones."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] learned network: calls without weights, parameter checks")
    ctx = bh.Context(theta=0.5, eps=1e-3, n_group=64, criterion=bh.LEARNED)
    X, Y = _synthetic(100, 9)
    Xd, Yd = torch.as_tensor(X, device="cuda"), torch.as_tensor(Y, device="cuda")
    for call in (lambda: ctx.mlp_predict(Xd), lambda: ctx.mlp_gradient(Xd, Yd)):
        with pytest.raises(bh.BHError) as e:
            call()
        assert e.value.status == bh.BH_ESTATE
    for bad in (dict(theta_min=-0.1), dict(theta_max=float("nan")), dict(tau=float("inf"))):
        with pytest.raises(bh.BHError) as e:
            ctx.set_params(**bad)
        assert e.value.status == bh.BH_EINVAL
        assert (ctx.params.theta_min, ctx.params.theta_max, ctx.params.tau) == (0.2, 1.0, 1e-3)
    ctx.set_params(theta_min=0.3)
    ctx.mlp_weights(set=_weights(X, Y, 10))
    pred = ctx.mlp_predict(Xd).cpu().numpy()
    assert np.isfinite(pred).all()
    ctx.close()


def test_training_on_a_supplied_set_without_a_tree(torch_cuda):
    """A context that never built a tree trains on a set given through
    bh_mlp_set_dataset (the training's epoch shuffle sorts with scratch that
    a tree build used to be the only one to allocate): the set reads back
    unchanged, and training brings the error well below the label variance."""
    from paper_1907_02289_amd import bh
    _log("[gpu] learned network: training on a supplied set, no tree")
    X, Y = _synthetic(6000, 11)
    ctx = bh.Context(theta=0.5, eps=1e-3, n_group=64, criterion=bh.LEARNED)
    ctx.mlp_set_dataset(X, Y)
    pairs, X2, Y2 = ctx.mlp_dataset()
    np.testing.assert_array_equal(X2, X)
    np.testing.assert_array_equal(Y2, Y)
    assert pairs.shape == (6000, 2) and not pairs.any()
    mse = ctx.mlp_train(iters=300, batch=1024, seed=1)
    _log(f"    mse {mse:.4f}, label variance {Y.var():.4f}")
    assert np.isfinite(mse) and mse < 0.5 * Y.var()
    ctx.close()


def _adam_numpy(w0, grads, lr, b1, b2, eps):
    """Adam as Kingma & Ba (2015) publish it, in FP64: biased first and
    second moment estimates, their bias corrections by 1 - beta^t, and the
    step lr * m_hat / (sqrt(v_hat) + eps)."""
    w = w0.astype(np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t, g in enumerate(grads, start=1):
        g = g.astype(np.float64)
        m = b1 * m + (1.0 - b1) * g
        v = b2 * v + (1.0 - b2) * g * g
        m_hat = m / (1.0 - b1 ** t)
        v_hat = v / (1.0 - b2 ** t)
        w = w - lr * m_hat / (np.sqrt(v_hat) + eps)
    return w


def test_adam_matches_published_update(torch_cuda):
    """Ten Adam steps of the library (bh_mlp_adam, the kernel bh_mlp_train
    applies after each batch) against the published update in numpy, from
    freshly installed weights (moments and step count start at zero):
    gradients of mixed signs and scales, some exactly zero; then a second
    installation restarts the step count."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log("[gpu] adam: 10 steps against the published update")
    rng = np.random.default_rng(8)
    X, Y = _synthetic(64, 8)
    w0 = _weights(X, Y, 8)
    grads = []
    for t in range(10):
        g = (rng.normal(0, 1, 1249) * 10.0 ** rng.uniform(-4, 1, 1249)).astype(np.float32)
        g[rng.choice(1249, 50, replace=False)] = 0.0
        grads.append(g)
    ctx = bh.Context(precision=bh.FP32_REL, criterion=bh.LEARNED)
    for lr, b1, b2, eps in ((1e-3, 0.9, 0.999, 1e-8), (3e-2, 0.8, 0.99, 1e-6)):
        ctx.mlp_weights(set=w0)
        for g in grads:
            ctx.mlp_adam(torch.as_tensor(g, device="cuda"), lr, b1, b2, eps)
        torch.cuda.synchronize()
        got = ctx.mlp_weights()
        want = _adam_numpy(w0[:1249], grads, lr, b1, b2, eps)
        err = np.max(np.abs(got[:1249].astype(np.float64) - want))
        _log(f"    lr={lr} beta=({b1}, {b2}) eps={eps}: max |w_gpu - w_ref| = {err:.2e}")
        assert err <= 1e-6, err
        np.testing.assert_array_equal(got[1249:], w0[1249:])     # normalisation untouched
        moved = np.abs(got[:1249].astype(np.float64) - w0[:1249])
        assert moved.max() > 5 * lr
    ctx.close()


@pytest.mark.parametrize("budget_min", [False, True], ids=["mean", "min"])
def test_group_budget_is_the_mean_or_smallest_acceleration(torch_cuda, budget_min):
    """The learned rule's budget scale A_g of each group, from the first
    geometric pass of a learned context, against |a| of the same forces
    computed by a geometric context (same tree, lists and kernel: the same
    accelerations bit for bit): the mean over the group's particles, or with
    BH_FLAG_BUDGET_MIN their smallest."""
    torch = torch_cuda
    from paper_1907_02289_amd import bh
    _log(f"[gpu] group budget ({'min' if budget_min else 'mean'}): ring n=12000 seed 51")
    s = inputs.ring(12000, 51)
    dev = bh.to_device(s)
    w = np.zeros(NPARAM, np.float32)
    w[1253:1257] = 1.0
    w[1258] = 1.0
    lc = bh.Context(theta=0.4, eps=1e-3, n_group=64, precision=bh.FP32_REL, criterion=bh.LEARNED,
                    theta_min=0.1, theta_max=0.6, tau=1e-3, budget_min=budget_min)
    lc.mlp_weights(set=w)
    lc.build_tree([dev])
    lc.make_lists()
    got = lc.export("group_extra")[:, 1]
    groups = lc.export("groups")
    gc = bh.Context(theta=0.4, eps=1e-3, n_group=64, precision=bh.FP32_REL)
    gc.build_tree([dev])
    gc.make_lists()
    out = {k: torch.zeros(s.n, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    gc.forces([out])
    torch.cuda.synchronize()
    perm = gc.export("perm").astype(np.int64)
    a = np.sqrt(sum(out[k].cpu().numpy() ** 2 for k in ("ax", "ay", "az")))[perm]
    want = np.array([(a[b:b + c].min() if budget_min else a[b:b + c].mean()) for b, c in groups[:, 1:3]])
    if budget_min:
        np.testing.assert_array_equal(got, want)
    else:
        np.testing.assert_allclose(got, want, rtol=1e-13)
    lc.close()
    gc.close()
