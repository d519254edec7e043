"""Parity at the full sizes of the workloads (GPU, and the oracle on the host).

* 128^3, FP32 compute and storage, MRT tau = 0.6, KS tracer boundary (17 x 17
  faces every 20 steps), one 64-bead chain: 50 steps against the oracle.
* 512^3, FP16-deviation storage, 32 chains of 256 beads at seeded anchors,
  affine OU boundary, a divergence-free sine initial field: 3 steps against
  the oracle (its FP64 state needs about 65 GB of host memory); the box's
  population set is 5.1 GB, so every row offset beyond 4 GiB is exercised.
* The batched workload of the benchmark (256 KS boxes with edges from
  {32, 48, 64, 96}, FP16, one 32-bead chain each), in the benchmark's launch
  configuration (autotuned work list, graph-replayed steps): 40 steps, the
  first box of every edge length against the oracle run of that box.
"""
import numpy as np
import pytest

import oracle
from lbcase import CHAIN_BOND, Case, bead_mass, ks_case, rel_l2
from paper_0809_4958_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_0809_4958_amd import lbm  # noqa: E402

STORE = {"f64": lbm.STORE_F64, "f32": lbm.STORE_F32, "f16": lbm.STORE_F16DEV}
TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}


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


def bead_errors(ctx, ob, case):
    p_o, v_o = ob.beads()
    p_g = ctx.read(0, lbm.F_BEAD_POS, n_beads=case.n_beads)
    v_g = ctx.read(0, lbm.F_BEAD_VEL, n_beads=case.n_beads)
    anc = np.concatenate([np.broadcast_to(c["anchor"], (len(c["pos"]), 3)) for c in case.chains])
    p0 = np.concatenate([np.asarray(c["pos"]) for c in case.chains])
    ep = float(np.linalg.norm(p_g - p_o) / np.linalg.norm(p0 - anc))
    ev = float(np.linalg.norm(v_g - v_o) / (np.linalg.norm(v_o) + 1e-300))
    return ep, ev


def test_128_fp32_ks_chain_50_steps():
    case = ks_case(128, 50, dt=20, res=17, n_beads=64, config_idx=1, box_idx=7)
    say("case 128^3 FP32 MRT, KS boundary, 64-bead chain, 50 steps")
    ob = case.oracle_box()
    assert ob.step(50) == 0
    ctx = run_gpu(case, "f32", 50)
    m = ob.interior_mask()
    _, uo = ob.rho_u()
    eu = rel_l2(ctx.read(0, lbm.F_U), uo, m)
    ep, ev = bead_errors(ctx, ob, case)
    say(f"128^3 f32: u {eu:.3e}  bead pos {ep:.3e}  bead vel {ev:.3e}")
    assert eu < TOL_U["f32"] and ep < TOL_U["f32"] and ev < 1e-3
    ctx.close()


def test_512_fp16_32_chains_first_steps():
    n, steps = 512, 3
    A = inputs.ou_strain(steps + 1, inputs.rng(4, 0), corr_steps=500.0, rms=1e-3)
    g = inputs.rng(4, 2)
    anchors = inputs.anchors(32, n, g)
    chains = []
    for a in anchors:
        pos, vel = inputs.chain_init(256, a, g, bond=CHAIN_BOND)
        chains.append(dict(pos=pos, vel=vel, anchor=a))
    # divergence-free sine field: u_x(y), u_y(z), u_z(x)
    q = np.sin(2.0 * np.pi * np.arange(n) / (n - 1)) * 1e-3
    u0 = np.empty((n, n, n, 3))
    u0[..., 0] = q[None, :, None]
    u0[..., 1] = q[:, None, None]
    u0[..., 2] = q[None, None, :]
    case = Case((n, n, n), collision=oracle.MRT, tau=0.6, tau_bulk=0.6, ghost_rate=1.0,
                bc=(oracle.BC_AFFINE, A, 0, 1, 0), u0=u0, chains=chains)
    say("case 512^3 FP16 MRT, 32 x 256-bead chains, 3 steps (oracle: ~65 GB host memory)")
    ctx = run_gpu(case, "f16", steps)
    ug = ctx.read(0, lbm.F_U)
    ep_g = (ctx.read(0, lbm.F_BEAD_POS, n_beads=case.n_beads), ctx.read(0, lbm.F_BEAD_VEL, n_beads=case.n_beads))
    ctx.close()
    del u0
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    m = ob.interior_mask()
    _, uo = ob.rho_u()
    eu = rel_l2(ug, uo, m)
    p_o, v_o = ob.beads()
    anc = np.concatenate([np.broadcast_to(c["anchor"], (256, 3)) for c in chains])
    p0 = np.concatenate([c["pos"] for c in chains])
    ep = float(np.linalg.norm(ep_g[0] - p_o) / np.linalg.norm(p0 - anc))
    say(f"512^3 f16: u {eu:.3e}  bead pos {ep:.3e}")
    assert eu < TOL_U["f16"] and ep < TOL_U["f16"]


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
        _, uo = ob.rho_u()
        eu = rel_l2(ctx.read(k, lbm.F_U), uo, ob.interior_mask())
        say(f"batch box {k} (edge {n}): u {eu:.3e}")
        assert eu < TOL_U["f16"]
    ctx.close()
