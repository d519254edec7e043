"""Throughput of the step on the workloads other than the benchmark's batch.

One JSON line per run: ms per step, the fused kernel's average duration (HIP
device timestamps inside replayed graphs), MLUPS over interior nodes and the
fused kernel's algorithmic HBM rate against the 8 TB/s peak.  Run under
``rocprofv3 --kernel-trace --stats`` for the per-kernel tables in profiles/.

Workloads (MRT tau = 0.6, KS tracer boundary sampled on 17 x 17 faces every
20 steps, KS initial field, one or more FENE chains):

  batch-f32     the 256-box batch (edges from {32, 48, 64, 96}, one 32-bead
                chain each) with FP32 storage
  batch-f16-extended
                the batch with FP16 storage whose chains are random walks
                of bond 0.8 (spring constant 0.003) instead of collapsed
                coils: stencil boxes of 5-9 nodes per axis, the force pass's
                heavy case
  batch-f16-thermal
                the benchmark's batch (FP16 storage, one 32-bead chain per box)
                with thermal fluctuations (kT = 1e-5 in lattice units:
                fluctuating MRT and bead Langevin noise, Philox draws) and the
                accelerated-frame body force -rho dv/dt (a seeded tracer
                acceleration history per box, rms 1e-6 per step^2, sampled
                every 20 steps): the extended step kernels
  large-f16     512^3, FP16 storage, 32 chains of 256 beads (two buffers)
  large-f16-aa  the same on one buffer updated in place
  single-f32    128^3, FP32 storage, one 64-bead chain

  python -m paper_0809_4958_amd.rates WORKLOAD [--steps 200] [--warmup 20] [--graph-steps 100]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import inputs

TAU = 0.6
HBM_PEAK_GBS = 8000.0


def _chains_big(n, config_idx=4):
    g = inputs.rng(config_idx, 2)
    out = []
    for a in inputs.anchors(32, n, g):
        pos, _ = inputs.chain_init(256, a, g, bond=0.05)
        out.append((pos, np.asarray(a, dtype=np.float64)))
    return out


def build(lbm, workload, steps, graph_steps):
    """Context of a workload and its interior node count."""
    if workload in ("batch-f32", "batch-f16-extended", "batch-f16-thermal"):
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        if root not in sys.path:
            sys.path.insert(0, root)
        import bench
        boxes = bench.batch_inputs(256, steps, TAU)
        if workload == "batch-f32":
            ctx = bench.make_ctx(lbm, boxes, lbm.STORE_F32, TAU, reduce_every=100,
                                 graph_steps=graph_steps)
            return ctx, float(sum((b["n"] - 2) ** 3 for b in boxes)), True
        if workload == "batch-f16-thermal":
            ctx = bench.make_ctx(lbm, boxes, lbm.STORE_F16DEV, TAU, reduce_every=100,
                                 graph_steps=graph_steps)
            n_samples = steps // 20 + 2
            for k in range(len(boxes)):
                ctx.set_body_force(k, inputs.rng(7, k).standard_normal((n_samples, 3)) * 1e-6, t0=0, dt=20)
            ctx.set_thermal(1e-5, 2024)
            return ctx, float(sum((b["n"] - 2) ** 3 for b in boxes)), True
        ctx = lbm.Context([(b["n"],) * 3 for b in boxes], collision=lbm.MRT, tau=TAU, tau_bulk=TAU,
                          ghost_rate=1.0, storage=lbm.STORE_F16DEV, reduce_every=100,
                          torch_alloc=True, graph_steps=graph_steps)
        for k, b in enumerate(boxes):
            ctx.set_initial(k, b["u0"])
            ctx.set_boundary(k, lbm.BC_SAMPLED, b["faces"], t0=0, dt=20, res=b["faces"].shape[2])
            pos, _ = inputs.chain_init(len(b["pos"]), b["anchor"], inputs.rng(6, k), bond=0.8)
            ctx.couple_chain(k, pos, None, substeps=10, fix_com=True, zeta=5.0,
                             mass=bench.bead_mass(len(pos)), fene_k=0.003, fene_r0=2.0,
                             anchor=b["anchor"])
        return ctx, float(sum((b["n"] - 2) ** 3 for b in boxes)), True
    if workload in ("large-f16", "large-f16-aa"):
        n, storage, chains = 512, lbm.STORE_F16DEV, _chains_big(512)
        cidx = 4
    elif workload == "single-f32":
        n, storage = 128, lbm.STORE_F32
        xc = np.full(3, (n - 1) / 2.0)
        pos, _ = inputs.chain_init(64, xc, inputs.rng(1, 2), bond=0.05)
        chains, cidx = [(pos, xc)], 1
    else:
        raise SystemExit(f"unknown workload {workload}")
    aa = workload.endswith("-aa")
    units, u0, faces = inputs.ks_box_inputs(cidx, 0, n=n, tau=TAU, n_steps=steps, dt=20, res=17)
    ctx = lbm.Context([(n, n, n)], collision=lbm.MRT, tau=TAU, tau_bulk=TAU, ghost_rate=1.0,
                      storage=storage, reduce_every=100, torch_alloc=True, graph_steps=graph_steps,
                      streaming=lbm.STREAM_AA if aa else lbm.STREAM_AB)
    ctx.set_initial(0, u0)
    del u0
    ctx.set_boundary(0, lbm.BC_SAMPLED, faces.astype(np.float32), t0=0, dt=20, res=17)
    for pos, anchor in chains:
        ctx.couple_chain(0, pos, None, substeps=10, fix_com=True, zeta=5.0, mass=0.5 / len(pos),
                         fene_k=1.0, fene_r0=2.0, anchor=anchor)
    return ctx, float((n - 2) ** 3), not aa


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("workload")
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--graph-steps", type=int, default=100)
    args = p.parse_args(argv)
    import torch

    from . import lbm
    torch.cuda.set_device(0)
    ctx, interior, tunable = build(lbm, args.workload, args.warmup + args.steps, args.graph_steps)
    if tunable:
        ctx.autotune(3)
    ctx.step(args.warmup)
    ctx.sync()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    ctx.sync()
    elapsed = time.perf_counter() - t0
    tm = ctx.timing()
    status = ctx.sync_status()
    rec = ctx.read(0, lbm.F_MASS_MOM) if status == lbm.OK else None
    out = {"workload": args.workload, "steps": args.steps, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
           "status": int(status), "step_index": int(ctx.read(0, lbm.F_STEP, strict=False)[0]),
           "box0_mass_momentum_record": None if rec is None else [float(v) for v in rec],
           "mlups": round(interior * args.steps / elapsed / 1e6, 1), "k_lb_ms": round(tm[1], 4),
           "pre_lb_kernels_ms": round(tm[2], 4),
           "algorithmic_gbs": round(tm[3] / (tm[1] * 1e-3) / 1e9, 1),
           "frac_of_8tbs": round(tm[3] / (tm[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "launch": ctx.describe()}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
