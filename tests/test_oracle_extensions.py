"""Pins of the oracle's extensions beyond the deterministic fine-box step:

* the accelerated-frame body force (Sec. 2: in the tracer's frame the flow
  w = u - v(t) obeys the Navier-Stokes equation with the extra force density
  -rho dv/dt), pinned by exact momentum balances in periodic boxes;
* thermal fluctuations of the LB-MD coupling the paper builds on (Sec. 1:
  Stokes friction of the beads; the fluctuating LB of the review it cites),
  pinned by the generator's published known-answer vectors, equipartition of
  every relaxed mode, the exact stationary variance of the bead's friction
  update and exact momentum conservation with noise.
"""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------- body force
def uniform_box(n, u0, coll=oracle.MRT, rho=None):
    ob = oracle.OracleBox((n, n, n), collision=coll, tau=0.8, tau_bulk=0.9, periodic_mask=7)
    ob.set_initial(np.broadcast_to(np.asarray(u0, dtype=float), (n, n, n, 3)).copy())
    if rho is not None:
        f = ob.pop()
        ob.set_populations(f * rho[None])
    return ob


@pytest.mark.parametrize("coll", [oracle.BGK, oracle.MRT])
def test_uniform_flow_decelerates_by_the_acceleration_each_step(coll):
    """A uniform state stays uniform and its momentum gains g = -rho a per
    step exactly: u(t_n) = u0 - n a."""
    u0 = np.array([2e-3, -1e-3, 5e-4])
    a = np.array([1e-5, 3e-5, -2e-5])
    ob = uniform_box(5, u0, coll)
    ob.set_body_force(np.tile(a, (2, 1)), t0=0, dt=100)
    assert ob.step(20) == 0
    _, u = ob.rho_u()
    assert np.abs(u - (u0 - 20 * a)).max() < 1e-15


def test_momentum_balance_uses_the_local_density_and_time_interpolation():
    """With a non-uniform density the total momentum changes by -a(t_n) sum rho
    per step (the local mass, not rho0), a linear in time between samples."""
    n = 6
    rng = np.random.default_rng(3)
    rho = 1.0 + 0.05 * rng.standard_normal((n, n, n))
    ob = uniform_box(n, [1e-3, 0, 0], rho=rho)
    a0, a1 = np.array([2e-5, -1e-5, 3e-5]), np.array([-4e-5, 2e-5, 1e-5])
    ob.set_body_force(np.stack([a0, a1]), t0=0, dt=4)
    f = ob.pop()
    c, _ = oracle.lattice()
    M = f.sum()
    P0 = np.einsum("ia,izyx->a", c, f)
    assert ob.step(4) == 0
    P1 = np.einsum("ia,izyx->a", c, ob.pop())
    want = -M * sum((1 - k / 4) * a0 + (k / 4) * a1 for k in range(4))
    # rounding of the momentum sums: ~eps sum |c f| < 1e-13 M; taking rho0
    # instead of the local density would be off by (M - N) |a| 4 = 5.6e-5
    assert np.abs(P1 - P0 - want).max() < 1e-13 * M
    assert abs(ob.pop().sum() - M) < 1e-12 * M
    # step 4 sits on the last sample; step 5 would need the one after it:
    # refused, never extrapolated
    assert ob.step(1) == 0
    assert ob.step(1) == oracle.ERR_ARG


def test_zero_acceleration_is_the_plain_step():
    rng = np.random.default_rng(5)
    u0 = 1e-3 * rng.standard_normal((7, 7, 7, 3))
    A = np.zeros((30, 9))
    runs = []
    for with_force in (False, True):
        ob = oracle.OracleBox((7, 7, 7), collision=oracle.MRT, tau=0.7, tau_bulk=0.7)
        ob.set_initial(u0)
        ob.set_boundary(oracle.BC_AFFINE, A)
        if with_force:
            ob.set_body_force(np.zeros((2, 3)), t0=0, dt=50)
        assert ob.step(20) == 0
        runs.append(ob.pop())
    assert np.array_equal(runs[0], runs[1])


# --------------------------------------------------- thermal fluctuations
def test_philox_known_answer_vectors():
    kat = json.load(open(os.path.join(HERE, "golden", "philox_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        want = [int(x, 16) for x in v["out"]]
        assert list(oracle.philox(ctr, key)) == want


def test_unit_uniform_is_symmetric_with_unit_variance():
    for u in (0, 1, 12345, 2 ** 31 - 1, 2 ** 31):
        assert oracle.unit_uniform(u) == -oracle.unit_uniform(2 ** 32 - 1 - u)
    assert abs(oracle.unit_uniform(0) + np.sqrt(3)) < 1e-9
    # variance of the map over a regular grid of 32-bit values: 1 - O(2^-20)
    us = np.arange(0, 2 ** 32, 4099, dtype=np.uint64)
    vals = np.array([oracle.unit_uniform(int(u)) for u in us[::97]])
    assert abs(vals.mean()) < 0.02 and abs(vals.var() - 1.0) < 0.05


def test_fluid_equipartition_of_every_mode():
    """Periodic box at kT: velocity variance kT/rho, density variance 3 kT rho
    and every relaxed mode at mu rho b_k (mu = 3 kT), each with the factor
    (1 - 1/N) of the conserved total where it applies."""
    n, kT = 6, 1e-4
    ob = oracle.OracleBox((n, n, n), collision=oracle.MRT, tau=0.8, tau_bulk=0.8, ghost_rate=1.0,
                          periodic_mask=7)
    assert ob.set_thermal(kT, seed=1234, box_index=3) == 0
    E, B = oracle.mrt_basis()
    assert ob.step(200) == 0
    acc_u, acc_r, acc_m, cnt = np.zeros(3), 0.0, np.zeros(19), 0
    for _ in range(1500):
        ob.step(1)
        rho, u = ob.rho_u()
        m = E @ ob.pop().reshape(19, -1)
        acc_u += (u.reshape(-1, 3) ** 2).mean(0)
        acc_r += ((rho - 1) ** 2).mean()
        acc_m += (m ** 2).mean(1)
        cnt += 1
    N = n ** 3
    assert np.abs(acc_u / cnt / (kT * (1 - 1 / N)) - 1).max() < 0.03
    assert abs(acc_r / cnt / (3 * kT * (1 - 1 / N)) - 1) < 0.03
    assert np.abs(acc_m[4:] / cnt / (3 * kT * B[4:]) - 1).max() < 0.03


def test_bead_friction_update_has_the_exact_stationary_variance():
    """The noisy exact friction update of one free bead in a fluid at rest is
    an Ornstein-Uhlenbeck process sampled exactly: its stationary velocity
    variance is kT/m whatever the substep."""
    kT, m, zeta, sub = 2e-4, 0.7, 5.0, 10
    rng = np.random.default_rng(7)
    pos, vel = np.zeros((1, 3)), np.zeros((1, 3))
    vs = []
    for step in range(6000):
        rnd = rng.uniform(-np.sqrt(3), np.sqrt(3), size=(sub, 1, 3))
        st, pos, vel, dp = oracle.chain_md_noise(pos, vel, np.zeros((1, 3)), kT, rnd, substeps=sub,
                                                 zeta=zeta, mass=m)
        assert st == 0
        # the friction impulse handed to the fluid is the bead's momentum change
        if step > 100:
            vs.append(vel[0].copy())
    v = np.array(vs)
    assert np.abs(v.var(axis=0) / (kT / m) - 1).max() < 0.05


def test_fluid_and_bead_momentum_conserved_with_noise():
    """Fluid noise acts on non-conserved modes only and the bead's noise
    impulse is spread back to the fluid: with the centre-of-mass pin off, the
    total momentum of fluid and bead is exact."""
    n = 7
    ob = oracle.OracleBox((n, n, n), collision=oracle.MRT, tau=0.8, tau_bulk=0.8, periodic_mask=7)
    ob.set_thermal(1e-4, seed=77, box_index=1)
    ob.add_chain(np.array([[2.3, 3.1, 4.7], [3.1, 3.4, 4.2]]), None, substeps=10, fix_com=False,
                 zeta=5.0, mass=0.5, anchor=[2.7, 3.25, 4.45])
    c, _ = oracle.lattice()

    def total():
        _, v = ob.beads()
        return np.einsum("ia,izyx->a", c, ob.pop()) + 0.5 * v.sum(0)

    P0 = total()
    assert ob.step(50) == 0
    assert np.abs(total() - P0).max() < 1e-13
