"""Pins for the oracle's forces and integrator.

Closed forms (two bodies, the regular N-gon ring, a circular Kepler orbit),
special cases (theta = 0 reduces Barnes-Hut to the direct sum), invariants
(momentum conservation of the pairwise sum, time reversibility of the
leapfrog) and the expected shrinking of the monopole error with theta.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1907_02289_amd import inputs


def _norm(ax, ay, az):
    return np.sqrt(ax * ax + ay * ay + az * az)


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_two_body_closed_form(eps):
    d, m1, m2, G = 0.3, 0.25, 0.75, 1.5
    x = np.array([0.1, 0.1 + d])
    y = np.array([-0.2, -0.2])
    z = np.array([0.05, 0.05])
    m = np.array([m1, m2])
    den = (d * d + eps * eps) ** 1.5
    want = np.array([G * m2 * d / den, -G * m1 * d / den])
    ax, ay, az, pot = oracle.direct(x, y, z, m, eps, G)
    np.testing.assert_allclose(ax, want, rtol=1e-15)
    assert np.all(ay == 0) and np.all(az == 0)
    if eps > 0:
        self_pot = -G * m / eps
        np.testing.assert_allclose(pot - self_pot, [-G * m2 / math.sqrt(d * d + eps * eps),
                                                    -G * m1 / math.sqrt(d * d + eps * eps)], rtol=1e-14)
    bax, bay, baz, _, _, _ = oracle.bh_accel(x, y, z, m, theta=0.5, eps=eps, G=G)
    np.testing.assert_allclose(bax, want, rtol=1e-15)


def _ngon_inward(N, R, m, eps, G=1.0):
    terms = []
    for k in range(1, N):
        s = math.sin(math.pi * k / N)
        dk = 2 * R * s
        terms.append(G * m * dk * s / (dk * dk + eps * eps) ** 1.5)
    return math.fsum(terms)


@pytest.mark.parametrize("N,eps", [(7, 0.0), (64, 1e-3), (301, 0.05)])
def test_regular_ngon_ring(N, eps):
    R = 1.3
    th = 2 * np.pi * np.arange(N) / N
    x, y, z = R * np.cos(th), R * np.sin(th), np.zeros(N)
    m = np.full(N, 1.0 / N)
    a = _ngon_inward(N, R, 1.0 / N, eps)
    ax, ay, az, _ = oracle.direct(x, y, z, m, eps)
    radial = -(ax * np.cos(th) + ay * np.sin(th))
    tang = -ax * np.sin(th) + ay * np.cos(th)
    np.testing.assert_allclose(radial, a, rtol=1e-13)
    assert np.max(np.abs(tang)) < 1e-13 * a
    # Barnes-Hut with theta = 0 opens everything: the same sum, reordered
    bax, bay, baz, _, _, _ = oracle.bh_accel(x, y, z, m, theta=0.0, eps=eps, n_leaf=4, n_grp=8)
    np.testing.assert_allclose(-(bax * np.cos(th) + bay * np.sin(th)), a, rtol=1e-13)


def test_theta_zero_equals_direct():
    s = inputs.ring(1500, 4)
    eps = 1e-3
    dax, day, daz, dpot = oracle.direct(s.x, s.y, s.z, s.m, eps)
    bax, bay, baz, bpot, mag, st = oracle.bh_accel(s.x, s.y, s.z, s.m, theta=0.0, eps=eps, n_grp=32)
    err = _norm(bax - dax, bay - day, baz - daz)
    assert np.all(err <= 1e-13 * mag)
    np.testing.assert_allclose(bpot, dpot, rtol=1e-13)
    assert st.pc.size == 0


def test_direct_sum_conserves_momentum():
    s = inputs.plummer(2000, 9)
    ax, ay, az, _ = oracle.direct(s.x, s.y, s.z, s.m, 1e-2)
    P = np.array([np.sum(s.m * ax), np.sum(s.m * ay), np.sum(s.m * az)])
    assert np.linalg.norm(P) <= 1e-14 * np.sum(s.m * _norm(ax, ay, az))


def test_monopole_error_shrinks_with_theta():
    s = inputs.ring(4096, 0)
    eps = 1e-3
    dax, day, daz, _ = oracle.direct(s.x, s.y, s.z, s.m, eps)
    dn = _norm(dax, day, daz)
    med = []
    for theta in (0.8, 0.4, 0.2):
        bax, bay, baz, _, _, _ = oracle.bh_accel(s.x, s.y, s.z, s.m, theta=theta, eps=eps)
        med.append(np.median(_norm(bax - dax, bay - day, baz - daz) / dn))
    assert med[0] > med[1] > med[2]
    assert med[1] < 0.5 * med[0] and med[2] < 0.5 * med[1]
    assert med[1] < 1e-3


def test_kepler_circular_orbit():
    # one test particle of negligible mass around a unit central mass
    x, y, z = np.array([1.0]), np.array([0.0]), np.array([0.0])
    vx, vy, vz = np.array([0.0]), np.array([1.0]), np.array([0.0])
    m = np.array([1e-300])
    n = 2000
    dt = 2 * math.pi / n
    x1, y1, z1, vx1, vy1, vz1 = oracle.kdk(x, y, z, vx, vy, vz, m, dt, n, eps=1e-3, central_mass=1.0)
    r = math.hypot(x1[0], y1[0])
    assert abs(r - 1.0) < 1e-5                       # radius held to O(dt^2)
    assert math.hypot(x1[0] - 1.0, y1[0]) < 1e-3      # back near the start after one period
    assert abs(vx1[0] * x1[0] + vy1[0] * y1[0]) < 1e-4


def test_kdk_time_reversible():
    s = inputs.plummer(256, 4)
    eps, dt, n = 0.05, 1.0 / 64, 40
    a = oracle.kdk(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, dt, n, eps)
    b = oracle.kdk(a[0], a[1], a[2], -a[3], -a[4], -a[5], s.m, dt, n, eps)
    for got, want in zip(b[:3], (s.x, s.y, s.z)):
        assert np.max(np.abs(got - want)) < 1e-11
    for got, want in zip(b[3:], (s.vx, s.vy, s.vz)):
        assert np.max(np.abs(-got - want)) < 1e-11


def _energy(x, y, z, vx, vy, vz, m, eps):
    _, _, _, pot = oracle.direct(x, y, z, m, eps)
    pot = pot + m / eps                                # drop each particle's self term
    return 0.5 * np.sum(m * (vx * vx + vy * vy + vz * vz)) + 0.5 * np.sum(m * pot)


def test_leapfrog_energy_drift_small():
    s = inputs.plummer(512, 6)
    eps, dt = 0.05, 1.0 / 128
    E0 = _energy(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m, eps)
    st = (s.x, s.y, s.z, s.vx, s.vy, s.vz)
    errs = []
    for _ in range(4):
        st = oracle.kdk(*st, s.m, dt, 64, eps)
        errs.append(abs(_energy(*st, s.m, eps) / E0 - 1.0))
    assert max(errs) < 2e-4


def test_bh_kdk_list_reuse_matches_rebuild_when_static():
    # particles at rest over tiny steps barely move: reused lists (moments
    # refreshed from the moved particles) give the rebuilt trajectory
    s = inputs.ring(2000, 8)
    zero = np.zeros(2000)
    kw = dict(eps=1e-3, theta=0.5)
    a = oracle.kdk(s.x, s.y, s.z, zero, zero, zero, s.m, 1e-4, 4, rebuild_every=1, **kw)
    b = oracle.kdk(s.x, s.y, s.z, zero, zero, zero, s.m, 1e-4, 4, rebuild_every=4, **kw)
    for u, v in zip(a, b):
        assert np.max(np.abs(u - v)) < 1e-15
    assert np.max(np.abs(a[0] - s.x)) > 0
