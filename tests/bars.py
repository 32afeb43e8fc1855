"""Parity bars shared by the GPU tests.

FP32-relative forces against the oracle evaluating the same lists in FP64:
the relative error |a_gpu - a_oracle| / |a_oracle| per particle must have a
median <= 1e-5 (the bar the method's FP32 form is held to), a 99th
percentile (nearest rank) <= 1e-5 and a maximum <= 1e-4, so that a defect
confined to a minority of particles (one partial-chunk form, the search
fallback) cannot hide behind the median."""
import math

import numpy as np

FP32_MEDIAN, FP32_P99, FP32_MAX = 1e-5, 1e-5, 1e-4


def p99(e):
    e = np.sort(np.asarray(e, np.float64).ravel())
    return float(e[int(math.ceil(0.99 * e.size)) - 1])


def fp32_bars(rel, what=""):
    rel = np.asarray(rel, np.float64).ravel()
    med, q, mx = float(np.median(rel)), p99(rel), float(rel.max())
    assert med <= FP32_MEDIAN, f"{what}: median {med:.3e}"
    assert q <= FP32_P99, f"{what}: p99 {q:.3e}"
    assert mx <= FP32_MAX, f"{what}: max {mx:.3e}"
    return med, q, mx
