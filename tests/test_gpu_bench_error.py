"""The benchmark's error along a run maps the library's sorted accelerations
back to the sampled particles and takes the central planet's term back out.
At t = 0 that must give the p99 the theta tuning measures directly on a
context without the planet (same lists, self-gravity only)."""
import sys
import types

import numpy as np
import pytest

from paper_1907_02289_amd import inputs

pytestmark = pytest.mark.gpu


def test_error_run_first_evaluation_matches_direct_measurement():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    from paper_1907_02289_amd import bh
    print("[gpu] bench error run vs direct measurement", flush=True)
    sys.stdout.flush()
    s = inputs.ring(20000, 5, central_mass=1.0)
    w = types.SimpleNamespace(eps=1e-4, dt=1e-3, central_mass=1.0)
    dev0 = bh.to_device(s)
    sample = torch.as_tensor(inputs.force_sample(s.n, 5, 1024).astype(np.int64), device="cuda")
    for prec in (bh.FP32_REL, bh.FP64):
        p = dict(theta=0.4, precision=prec, n_group=128, rebuild_every=4)
        p99, med = bench.error_run(bh, w, dev0, sample, p, 3)
        judge = bh.Context(theta=0.5, eps=w.eps)
        ref = {k: torch.zeros(sample.numel(), dtype=torch.float64, device="cuda") for k in ("ax", "ay", "az")}
        judge.direct_sum(dev0, sample, ref)
        ctx = bh.Context(theta=0.4, eps=w.eps, precision=prec, n_group=128)
        ctx.build_tree([dev0])
        ctx.make_lists()
        want, want_med = bench.rel_err_p99(ctx, dev0, sample, ref, s.n)
        ctx.close()
        judge.close()
        # FP64: the same sums up to the planet's term added and taken back;
        # FP32: the tuning runs the potential-computing kernel instance, whose
        # FP32 sums may round differently (a relative change of ~1e-7 in a
        # moves an error of ~1e-3 by ~1e-4 of itself).  A wrong mapping would
        # be off by orders of magnitude.
        tol = 1e-6 if prec == bh.FP64 else 1e-3
        assert len(p99) == 3 and all(np.isfinite(p99))
        assert abs(p99[0] - want) <= tol * want, (prec, p99[0], want)
        assert abs(med[0] - want_med) <= tol * want_med, (prec, med[0], want_med)
