"""bh_direct_sum_static, the entry point that allocates nothing, against
bh_direct_sum (same kernels, context scratch grown on demand): bit-identical
results on two calls in a row, the second with a smaller system and fewer
targets, and the target limit rejected before any device work."""
import sys

import numpy as np
import pytest

from paper_1907_02289_amd import inputs

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_static_direct_sum_matches_allocating_one():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_02289_amd import bh
    ctx = bh.Context(theta=0.5, eps=1e-3)
    for n, nt, seed in ((200000, 4096, 41), (5000, 700, 42)):
        _log(f"[gpu] static direct sum: ring n={n}, {nt} targets, seed {seed}")
        s = inputs.ring(n, seed)
        dev = bh.to_device(s)
        tg = torch.as_tensor(np.sort(np.random.default_rng(seed).choice(n, nt, replace=False)), device="cuda")
        want = {k: torch.zeros(nt, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
        got = {k: torch.full((nt,), np.nan, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
        ctx.direct_sum(dev, tg, want)
        ctx.direct_sum_static(dev, tg, got)
        torch.cuda.synchronize()
        for k in ("ax", "ay", "az"):
            a, b = got[k].cpu().numpy(), want[k].cpu().numpy()
            assert np.all(np.isfinite(a))
            np.testing.assert_array_equal(a, b)
    # the limit: 4097 targets are refused, the context stays usable
    s = inputs.ring(3000, 43)
    dev = bh.to_device(s)
    tg = torch.arange(4097, dtype=torch.int64, device="cuda") % s.n
    out = {k: torch.zeros(4097, dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
    with pytest.raises(bh.BHError) as e:
        ctx.direct_sum_static(dev, tg, out)
    assert e.value.status == bh.BH_EINVAL
    ctx.close()
