"""GPU parity of the extensions beyond the deterministic fine-box step:

* the accelerated-frame body force -rho dv/dt (Sec. 2), on walled row and
  tile boxes with chains (the force pass re-collides the chain nodes with it)
  and on periodic boxes;
* thermal fluctuations (fluctuating MRT and the beads' Langevin noise): the
  library and the oracle draw the same Philox4x32-10 numbers, so the runs are
  compared deterministically like the plain step -- any different draw would
  show as an O(1) error -- and, at a larger size, the GPU's fluid temperature
  against equipartition.
"""
import numpy as np
import pytest

import oracle
from lbcase import CHAIN_BOND, Case, ks_case
from paper_0809_4958_amd import inputs
from test_gpu_parity import STORE, check, compare, make_ctx

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_0809_4958_amd.lbm")


def say(*a):
    print(*a, flush=True)


def accel_history(n, rng, scale=2e-6, dt=7):
    """Tracer accelerations sampled every dt steps (lattice units)."""
    return (scale * rng.standard_normal((n // dt + 2, 3)), 0, dt)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_body_force_walled_box_with_chain(storage):
    steps = 120
    case = ks_case(30, steps, dt=20, res=9, tau=0.6, n_beads=10, f32_samples=storage != "f64")
    case.body = accel_history(steps, np.random.default_rng(2))
    case.reduce_every = 40
    say("case body force KS 30^3,", storage)
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    ctx = make_ctx(case, storage)
    ctx.step(steps)
    check(compare(ctx, ob, case, storage), storage, "body force walled")
    mm_o, mm_g = ob.mass_mom(), ctx.read(0, lbm.F_MASS_MOM)
    assert mm_o[0] == mm_g[0]
    ctx.close()


def test_body_force_periodic_and_mixed_fp64():
    rng = np.random.default_rng(4)
    dims = (14, 12, 13)
    pos, _ = inputs.chain_init(5, [6.5, 5.5, 6.0], rng)
    per = Case(dims, collision=oracle.MRT, tau=0.8, tau_bulk=0.9, ghost_rate=1.3, periodic_mask=7,
               u0=1e-3 * rng.standard_normal(dims[::-1] + (3,)),
               chains=[dict(pos=pos, vel=1e-3 * rng.standard_normal((5, 3)), fix_com=False,
                            anchor=[6.5, 5.5, 6.0])],
               body=accel_history(40, rng, 5e-6, 3), reduce_every=10)
    mixed = Case((12, 11, 9), collision=oracle.MRT, tau=0.8, tau_bulk=0.9, ghost_rate=1.3,
                 periodic_mask=5, bc=(oracle.BC_AFFINE, inputs.ou_strain(41, rng, 20.0, 1e-3), 0, 1, 0),
                 u0=1e-3 * rng.standard_normal((9, 11, 12, 3)), body=accel_history(40, rng, 5e-6, 5),
                 reduce_every=10, box_index=1)
    say("case body force periodic + mixed, fp64")
    ctx = lbm.Context([per.dims + (7,), mixed.dims + (5,)], collision=lbm.MRT, tau=0.8, tau_bulk=0.9,
                      ghost_rate=1.3, storage=0, reduce_every=10)
    per.add_to(ctx, 0)
    mixed.add_to(ctx, 1)
    ctx.step(40)
    for k, c in enumerate((per, mixed)):
        ob = c.oracle_box()
        assert ob.step(40) == 0
        check(compare(ctx, ob, c, "f64", box=k), "f64", f"body force box {k}")
    # stepping beyond the acceleration samples is refused on the host
    assert ctx.step_status(10) == lbm.ERR_ARG
    ctx.close()


@pytest.mark.parametrize("ghost", [1.0, 1.4])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_thermal_walled_box_with_chain(storage, ghost):
    steps = 80
    case = ks_case(26, steps, dt=20, res=9, tau=0.6, n_beads=8, f32_samples=storage != "f64")
    case.ghost_rate = ghost
    case.kT, case.seed = 2e-6, 0x1234_5678_9abc
    case.reduce_every = 40
    say("case thermal KS 26^3,", storage, "ghost", ghost)
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    ctx = make_ctx(case, storage)
    ctx.set_thermal(case.kT, case.seed)
    ctx.step(steps)
    check(compare(ctx, ob, case, storage), storage, f"thermal ghost {ghost}")
    ctx.close()


def test_thermal_two_boxes_fp64_and_argument_checks():
    """Counters carry the box index: the second box of a context draws its own
    numbers, matching an oracle box told that index."""
    rng = np.random.default_rng(12)
    dims = (10, 9, 11)
    cases = []
    for k in range(2):
        pos, _ = inputs.chain_init(4, [4.5, 4.0, 5.0], rng)
        cases.append(Case(dims, collision=oracle.MRT, tau=0.7, tau_bulk=0.7, periodic_mask=7,
                          u0=1e-3 * rng.standard_normal(dims[::-1] + (3,)),
                          chains=[dict(pos=pos, vel=None, fix_com=False, anchor=[4.5, 4.0, 5.0])],
                          kT=1e-5, seed=99, box_index=k))
    ctx = lbm.Context([dims + (7,)] * 2, collision=lbm.MRT, tau=0.7, tau_bulk=0.7, storage=0)
    for k, c in enumerate(cases):
        c.add_to(ctx, k)
    ctx.set_thermal(1e-5, 99)
    ctx.step(30)
    for k, c in enumerate(cases):
        ob = c.oracle_box()
        assert ob.step(30) == 0
        check(compare(ctx, ob, c, "f64", box=k), "f64", f"thermal periodic box {k}")
    with pytest.raises(lbm.LBError) as e:
        ctx.set_thermal(1e-5, 1)
    assert e.value.status == lbm.ERR_STATE
    bgk = lbm.Context([dims + (7,)], collision=lbm.BGK, tau=0.7, storage=0)
    with pytest.raises(lbm.LBError) as e:
        bgk.set_thermal(1e-5, 1)
    assert e.value.status == lbm.ERR_ARG
    bgk.close()
    ctx.close()


def test_thermal_equipartition_fp32_64cubed():
    """A 64^3 periodic FP32 box at kT = 1e-4 reaches its temperature: the
    velocity variance per component is kT / rho0 within 2 %, the density
    variance 3 kT rho0 within 2 %."""
    n, kT = 64, 1e-4
    ctx = lbm.Context([(n, n, n, 7)], collision=lbm.MRT, tau=0.8, tau_bulk=0.8, storage=1)
    ctx.set_thermal(kT, 2024)
    ctx.step(300)
    acc_u, acc_r, cnt = np.zeros(3), 0.0, 0
    for _ in range(6):
        ctx.step(20)
        rho = ctx.read(0, lbm.F_RHO)
        u = ctx.read(0, lbm.F_U)
        acc_u += (u.reshape(-1, 3) ** 2).mean(0)
        acc_r += ((rho - 1.0) ** 2).mean()
        cnt += 1
    ru = acc_u / cnt / kT
    rr = acc_r / cnt / (3 * kT)
    say("equipartition: <u^2>/(kT/rho)", ru, "<drho^2>/(3 kT rho)", rr)
    assert np.abs(ru - 1).max() < 0.02 and abs(rr - 1) < 0.02
    ctx.close()
