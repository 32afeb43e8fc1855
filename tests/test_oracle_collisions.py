"""Pins of the oracle's collision branch of Eq. (2) (Sec. 5.1) against facts
that do not come from its own formula:

- two bodies meeting head-on obey, inside the contact, the damped oscillator
  delta'' + eta delta' + kappa delta = 0 for the overlap delta = r - r_coll
  (the mass factors m_j/(m_i+m_j) and m_i/(m_i+m_j) add up to one in the
  relative motion).  Its closed form gives the coefficient of restitution
  e = exp(-gamma pi / omega_d) and the contact time pi / omega_d,
  gamma = eta/2, omega_d = sqrt(kappa - gamma^2); the oracle's leapfrog must
  reproduce both, for equal and unequal masses, and e = 1 when eta = 0;
- total momentum is conserved exactly (every pair term is antisymmetric once
  multiplied by the masses), which a swapped mass factor would break;
- the gravity part is continuous at r_coll and the reported potential is the
  integral of the reported force (a finite-difference check);
- with theta = 0 the tree sum is the direct sum, collisions included.
"""
import math

import numpy as np
import pytest

import oracle
from golden import paper_values
from paper_1907_02289_amd import inputs

# the paper's radial coefficient of restitution (Sec. 5.1)
E_PAPER = paper_values()["restitution_radial"]


def contact_params(t_c, e):
    """kappa, eta of the damped oscillator with contact time t_c and restitution e."""
    wd = math.pi / t_c
    gamma = -math.log(e) / t_c
    return wd * wd + gamma * gamma, 2.0 * gamma


def head_on(m1, m2, rc, kappa, eta, v_in, dt, G=0.0):
    """Two particles on the x axis approaching at relative speed v_in from a
    gap of rc/2; returns (relative speed after, contact time, momentum drift)."""
    x = np.array([0.0, 1.5 * rc])
    z0 = np.zeros(2)
    m = np.array([m1, m2])
    # centre-of-mass frame: total momentum zero
    vx = np.array([v_in * m2 / (m1 + m2), -v_in * m1 / (m1 + m2)])
    p0 = float(np.sum(m * vx))
    state = dict(inside=0, pmax=0.0)

    def trace(k, x_, y_, z_, vx_, vy_, vz_):
        if x_[1] - x_[0] <= rc:
            state["inside"] += 1
        state["pmax"] = max(state["pmax"], abs(float(np.sum(m * vx_)) - p0))

    t_total = 0.5 * rc / v_in * 2 + math.pi / math.sqrt(kappa) * 3
    n = int(t_total / dt) + 1
    xo, _, _, vxo, _, _ = oracle.kdk(x, z0.copy(), z0.copy(), vx, z0.copy(), z0.copy(), m, dt, n, 0.0, G=G,
                                     contact=(rc, kappa, eta), trace=trace)
    assert xo[1] - xo[0] > rc, "still in contact at the end"
    return (vxo[1] - vxo[0]) / v_in, state["inside"] * dt, state["pmax"]


@pytest.mark.parametrize("m1,m2", [(1.0, 1.0), (1.0, 3.0), (0.25, 2.0)])
def test_restitution_and_contact_time(m1, m2):
    rc, t_c, e = 1e-2, 1.0, E_PAPER
    kappa, eta = contact_params(t_c, e)
    e_num, tc_num, dp = head_on(m1, m2, rc, kappa, eta, v_in=1e-2, dt=5e-4)
    assert abs(e_num - e) <= 6e-4, e_num
    assert abs(tc_num - t_c) <= 4 * 5e-4, tc_num
    assert dp <= 1e-15 * (m1 + m2) * 1e-2 * 10


def test_elastic_contact_keeps_speed():
    rc, t_c = 1e-2, 0.5
    kappa = (math.pi / t_c) ** 2
    e_num, tc_num, _ = head_on(1.0, 2.0, rc, kappa, 0.0, v_in=2e-2, dt=2.5e-4)
    assert abs(e_num - 1.0) <= 1e-3
    assert abs(tc_num - t_c) <= 4 * 2.5e-4


def test_restitution_converges_with_step():
    # the leapfrog's error in e shrinks as dt does (the dashpot sees
    # half-kicked velocities): halving dt must at least halve it
    rc, kappa, eta = 1e-2, *contact_params(1.0, E_PAPER)
    errs = [abs(head_on(1.0, 1.0, rc, kappa, eta, 1e-2, dt)[0] - E_PAPER) for dt in (8e-3, 4e-3, 2e-3)]
    assert errs[1] <= 0.6 * errs[0] and errs[2] <= 0.6 * errs[1], errs


def _cluster(n, seed):
    """n particles in a small cube, so that many pairs overlap, with
    unequal masses and random velocities."""
    rng = np.random.default_rng(seed)
    x, y, z = (rng.uniform(0.0, 1.0, n) for _ in range(3))
    vx, vy, vz = (rng.normal(0.0, 1.0, n) for _ in range(3))
    m = rng.uniform(0.5, 2.0, n)
    return x, y, z, vx, vy, vz, m


def test_direct_sum_with_contacts_conserves_momentum():
    x, y, z, vx, vy, vz, m = _cluster(300, 3)
    contact = (0.12, 50.0, 3.0)
    ax, ay, az, _ = oracle.direct(x, y, z, m, 0.0, G=1.0, vel=(vx, vy, vz), contact=contact)
    # the cluster must have contacts for the check to mean anything
    d2 = (x[:, None] - x[None]) ** 2 + (y[:, None] - y[None]) ** 2 + (z[:, None] - z[None]) ** 2
    assert np.sum(d2 <= 0.12 ** 2) - 300 > 500
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) <= 1e-13 * np.sum(np.abs(m * a))


def test_gravity_part_continuous_and_potential_integrates_force():
    rc = 0.1
    for eps in (0.0, 0.03):
        # i at the origin, j on a ray; at rest, no spring or dashpot
        def at(r):
            x = np.array([0.0, r * 0.6])
            y = np.array([0.0, r * 0.8])
            z = np.zeros(2)
            m = np.array([1.0, 2.0])
            ax, ay, _, pot = oracle.direct(x, y, z, m, eps, G=1.0, targets=np.array([0]),
                                           vel=(z, z, z), contact=(rc, 0.0, 0.0))
            return math.hypot(ax[0], ay[0]), pot[0]

        a_in, p_in = at(rc * (1 - 1e-10))
        a_out, p_out = at(rc * (1 + 1e-10))
        assert abs(a_in - a_out) <= 1e-8 * a_out
        assert abs(p_in - p_out) <= 1e-8 * abs(p_out)
        # inside the contact sphere: |a| = -d(pot)/dr (central difference)
        for r in (0.3 * rc, 0.7 * rc):
            h = 1e-6 * rc
            dp = (at(r + h)[1] - at(r - h)[1]) / (2 * h)
            assert abs(dp - at(r)[0]) <= 1e-6 * at(r)[0]


def test_theta_zero_tree_equals_direct_with_contacts():
    s = inputs.ring(2000, 4, z_sigma=1e-3)
    rng = np.random.default_rng(9)
    vx, vy, vz = (rng.normal(0.0, 1e-3, s.n) for _ in range(3))
    contact = (3e-3, 1e3, 10.0)
    ax, ay, az, _, _, st = oracle.bh_accel(s.x, s.y, s.z, s.m, 0.0, 1e-4, vel=(vx, vy, vz), contact=contact)
    dx, dy, dz, _ = oracle.direct(s.x, s.y, s.z, s.m, 1e-4, vel=(vx, vy, vz), contact=contact)
    scale = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
    assert np.max(np.sqrt((ax - dx) ** 2 + (ay - dy) ** 2 + (az - dz) ** 2) / scale) <= 1e-11
    # without the branch the answer differs: the ring has contacts
    nx, _, _, _ = oracle.direct(s.x, s.y, s.z, s.m, 1e-4)
    assert np.max(np.abs(nx - dx) / scale) > 1e-3
