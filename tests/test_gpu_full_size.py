"""Parity at the full sizes of the workloads (GPU, and the oracle on the host).

* 128^3, FP32 compute and storage, MRT tau = 0.6, KS tracer boundary (17 x 17
  faces every 20 steps), one 64-bead chain: 50 steps against the oracle.
* The batched workload of the benchmark (256 KS boxes with edges from
  {32, 48, 64, 96}, FP16, one 32-bead chain each), in the benchmark's launch
  configuration (autotuned work list, graph-replayed steps): 40 steps, the
  first box of every edge length against the oracle run of that box.

Every comparison covers the whole interior (rel-L2 and per-node max-norm of u
and of the population deviations) and every bead.  The 512^3 large box and
the workloads' full lengths are compared in test_gpu_long_runs.py.
"""
import numpy as np
import pytest

import oracle
from lbcase import bead_errors, bead_mass, ks_case, max_rel, rel_l2

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_0809_4958_amd import lbm  # noqa: E402

STORE = {"f64": lbm.STORE_F64, "f32": lbm.STORE_F32, "f16": lbm.STORE_F16DEV}
TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}
TOL_MAX = {"f64": 1e-12, "f32": 1e-4, "f16": 4e-3}


def say(*a):
    print(*a, flush=True)


def run_gpu(case, storage, steps, **kw):
    ctx = lbm.Context([case.dims + (case.pmask,)], collision=case.collision, tau=case.tau,
                      tau_bulk=case.tau_bulk, ghost_rate=case.ghost_rate, storage=STORE[storage],
                      reduce_every=case.reduce_every, **kw)
    case.add_to(ctx, 0)
    ctx.step(steps)
    ctx.sync()
    return ctx


W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def field_errors(ctx, k, ob, chains=None, n_beads=0):
    """rel-L2 and per-node max-norm of u and of the population deviations over
    the whole interior, and the bead errors element by element."""
    m = ob.interior_mask()
    _, uo = ob.rho_u()
    ug = ctx.read(k, lbm.F_U)
    r = {"u": rel_l2(ug, uo, m), "u_max": max_rel(ug[m], uo[m])}
    umax = np.abs(uo[m]).max()
    del ug, uo
    fo = ob.pop()[:, m] - W[:, None]
    fg = ctx.read(k, lbm.F_POP)[:, m] - W[:, None]
    r.update(pop=rel_l2(fg, fo), pop_max=max_rel(fg, fo))
    del fo, fg
    if n_beads:
        p_o, v_o = ob.beads()
        r.update(bead_errors(ctx.read(k, lbm.F_BEAD_POS, n_beads=n_beads),
                             ctx.read(k, lbm.F_BEAD_VEL, n_beads=n_beads), p_o, v_o, chains, umax))
    return r


def check(r, storage, label):
    """rel-L2 fields against TOL_U, per-node max-norms (``*_max``) against
    TOL_MAX (derived in test_gpu_parity.py)."""
    say(label, {a: f"{v:.3e}" for a, v in r.items()})
    bad = {a: v for a, v in r.items()
           if not v < (TOL_MAX[storage] if a.endswith("_max") else TOL_U[storage])}
    assert not bad, f"{label}: over the bound: {bad}"


def test_128_fp32_ks_chain_50_steps():
    case = ks_case(128, 50, dt=20, res=17, n_beads=64, config_idx=1, box_idx=7)
    say("case 128^3 FP32 MRT, KS boundary, 64-bead chain, 50 steps")
    ob = case.oracle_box()
    assert ob.step(50) == 0
    ctx = run_gpu(case, "f32", 50)
    check(field_errors(ctx, 0, ob, case.chains, case.n_beads), "f32", "128^3 f32")
    ctx.close()


def test_batched_workload_in_bench_configuration():
    import bench
    steps, tau = 40, 0.6
    boxes = bench.batch_inputs(256, steps, tau)
    say("case batched workload, 256 boxes, FP16, autotuned, graph-replayed, 40 steps")
    ctx = bench.make_ctx(lbm, boxes, lbm.STORE_F16DEV, tau, reduce_every=20, graph_steps=20)
    ctx.autotune(2)
    ctx.step(steps)
    ctx.sync()
    for n in (32, 48, 64, 96):
        k = next(i for i, b in enumerate(boxes) if b["n"] == n)
        b = boxes[k]
        ob = oracle.OracleBox((n, n, n), collision=oracle.MRT, tau=tau, tau_bulk=tau, ghost_rate=1.0)
        ob.set_initial(b["u0"])
        ob.set_boundary(oracle.BC_SAMPLED, b["faces"].astype(np.float64), t0=0, dt=20, res=17)
        ob.add_chain(b["pos"], None, substeps=10, fix_com=True, zeta=5.0, mass=bead_mass(32),
                     fene_k=1.0, fene_r0=2.0, anchor=b["anchor"])
        assert ob.step(steps) == 0
        chains = [dict(pos=b["pos"], anchor=b["anchor"])]
        check(field_errors(ctx, k, ob, chains, 32), "f16", f"batch box {k} (edge {n})")
    ctx.close()
