#!/usr/bin/env python3
"""Throughput of the fine-box lattice-Boltzmann hot path on one MI355X.

Workload (default): the batched configuration -- 256 independent tracer
sub-boxes with edge lengths drawn from {32, 48, 64, 96}, each driven by its own
kinematic-simulation tracer boundary history (sampled faces, 17x17 corner-aligned
grid every 20 steps), each with one 32-bead FENE chain, D3Q19 MRT tau = 0.6,
FP32 compute with FP16-deviation population storage, all boxes advanced by one
fused launch per step, steps replayed from captured HIP graphs.  A step is one
pass of the whole path: x-face boundary velocities + chain kernel
(interpolation, MD substeps, spreading records) + fused collide/stream over
every box and boundary face + the mass/momentum check and finalisation.

Prints one JSON line: MLUPS over interior nodes; the HBM roofline of the fused
kernel (its average duration from device timestamps that the kernels record
inside the replayed graphs, the measured copy ceilings -- this library's copy
kernel and the runtime's hipMemcpyAsync -- and the HBM traffic of the committed
counter run when it was taken on the current kernel sources); the same boxes
run one by one as plain FP32 single-box contexts for the gain; and the oracle
leg: the FP64 oracle's own throughput on the host cores and the FP16 velocity
error of one box of the batch against it.

Windows.  The timed region is exactly --steps steps.  The mass/momentum check
runs every K steps, K the largest divisor of --steps up to 100, so the window
holds --steps / K check steps whatever the warmup; the steps are replayed from
HIP graphs whose length is a multiple of K dividing --steps, so every timed
step is graph-replayed (both recorded in the output).  The plain-FP32 leg
times 200 graph-replayed steps per box size after 20 warmup steps, and the
oracle-error leg runs the workload's full 5,000 steps on one box, whatever
--steps is.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS & % HBM roofline; batched FP16-store vs plain FP32 at ≤1e-3 rel err"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--boxes", type=int, default=256)
    p.add_argument("--storage", default="f16", choices=["f16", "f32"])
    p.add_argument("--graph-steps", type=int, default=100,
                   help="steps per captured HIP graph (0: plain stream launches)")
    p.add_argument("--no-baselines", action="store_true",
                   help="skip the plain-FP32 single-box and oracle legs")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-mib", type=int, default=1024, help="copy-probe size (0: skip)")
    p.add_argument("--no-tune", action="store_true",
                   help="skip the autotuner (default: tune item sizes and grid before timing)")
    p.add_argument("--tune-cache", default=None,
                   help="autotuner cache: if the file exists its launch shape is used and the "
                        "autotuner is skipped; otherwise the autotuner writes it")
    return p.parse_args()


def batch_inputs(n_boxes, n_steps, tau, dt=20, res=17, n_beads=32, config_idx=2, only=None):
    """Inputs of the batched workload; ``only`` lists the box indices to build
    (the rest are skipped; every box's inputs depend on its index alone)."""
    from paper_0809_4958_amd import inputs
    sizes = inputs.box_sizes(n_boxes, inputs.rng(config_idx, 3))
    boxes = []
    for b, n in enumerate(sizes):
        if only is not None and b not in only:
            continue
        units, u0, faces = inputs.ks_box_inputs(config_idx, b, n=int(n), tau=tau,
                                                n_steps=n_steps, dt=dt, res=res)
        xc = np.full(3, (n - 1) / 2.0)
        pos, _ = inputs.chain_init(n_beads, xc, np.random.Generator(np.random.PCG64(
            np.random.SeedSequence(entropy=inputs.ENTROPY, spawn_key=(config_idx, 2, b)))),
            bond=CHAIN_BOND)
        boxes.append(dict(n=int(n), u0=u0, faces=faces.astype(np.float32), pos=pos, anchor=xc,
                          index=b))
    return boxes


# random-walk bond length of the initial chains (lattice spacings): k b stays
# comparable to the friction force of the boundary-driven flow
CHAIN_BOND = 0.05


def bead_mass(n_beads):
    # whole chain weighs half a fluid node: keeps the explicit friction
    # exchange stable once the chain has collapsed (see the tests' fixture)
    return 0.5 / n_beads


def make_ctx(lbm, boxes, storage, tau, reduce_every=0, stream=None, graph_steps=0, tune_cache=None):
    ctx = lbm.Context([(b["n"],) * 3 for b in boxes], collision=lbm.MRT, tau=tau, tau_bulk=tau,
                      ghost_rate=1.0, storage=storage, reduce_every=reduce_every, stream=stream,
                      torch_alloc=True, graph_steps=graph_steps, tune_cache=tune_cache)
    for k, b in enumerate(boxes):
        ctx.set_initial(k, b["u0"])
        ctx.set_boundary(k, lbm.BC_SAMPLED, b["faces"], t0=0, dt=20, res=b["faces"].shape[2])
        ctx.couple_chain(k, b["pos"], None, substeps=10, fix_com=True, zeta=5.0,
                         mass=bead_mass(len(b["pos"])), fene_k=1.0, fene_r0=2.0,
                         anchor=b["anchor"])
    return ctx


def traffic_file(storage, n_boxes):
    return os.path.join(ROOT, "profiles", f"k_lb_batch{n_boxes}_{storage}_hbm_traffic.txt")


def committed_traffic(storage, n_boxes):
    """HBM bytes per k_lb launch from the committed counter summary, or None
    when it is missing or was taken on other kernel sources."""
    path = traffic_file(storage, n_boxes)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    from paper_0809_4958_amd.prof_summary import kernel_source_hash
    if vals.get("kernel_sources_sha1") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(ctx, steps, torch):
    """Exactly `steps` steps with per-step HIP events; returns (seconds, timing)."""
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = ctx.timing()
    ctx.set_timing(False)
    return elapsed, tm


def check_interval(steps, cap=100):
    """Steps between mass/momentum checks: the largest divisor of the timed
    step count not above ``cap``, so that every timed window holds whole check
    periods (steps / K check steps, whatever the warmup's phase)."""
    return max(d for d in range(1, min(cap, steps) + 1) if steps % d == 0)


def graph_length(steps, k, cap):
    """Steps per replayed HIP graph: the largest multiple of the check interval
    k that divides the timed step count and is at most max(cap, k), so the
    whole timed region is graph-replayed (lb_step replays a graph only while
    at least its length is left) and each graph holds its check steps."""
    best, m = k, k
    while m <= max(cap, k):
        if steps % m == 0:
            best = m
        m += k
    return best


# fixed windows of the side legs, independent of --steps
PLAIN_WARMUP, PLAIN_STEPS, PLAIN_GRAPH = 20, 200, 100
ORACLE_ERR_STEPS = 5000


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the batch of independent "
                                   "boxes would shard across GPUs without communication, which "
                                   "is described but not implemented"}))
        sys.exit(2)
    import torch
    from paper_0809_4958_amd import lbm

    torch.cuda.set_device(0)
    tau = 0.6
    total_steps = args.warmup + args.steps
    t_in = time.time()
    boxes = batch_inputs(args.boxes, total_steps, tau)
    t_in = time.time() - t_in
    print(json.dumps({"progress": "inputs ready", "seconds": round(t_in, 1)}), file=sys.stderr,
          flush=True)
    interior = float(sum((b["n"] - 2) ** 3 for b in boxes))
    storage = lbm.STORE_F16DEV if args.storage == "f16" else lbm.STORE_F32
    stream = torch.cuda.current_stream().cuda_stream
    copy_gbs = lbm.copy_probe(args.copy_mib << 20, 20) if args.copy_mib > 0 else None
    memcpy_gbs = lbm.memcpy_probe(4 << 30, 10) if args.copy_mib > 0 else None
    check_every = check_interval(args.steps)
    gs = graph_length(args.steps, check_every, args.graph_steps) if args.graph_steps > 0 else 0
    cached = bool(args.tune_cache) and os.path.exists(args.tune_cache)
    ctx = make_ctx(lbm, boxes, storage, tau, reduce_every=check_every, stream=stream,
                   graph_steps=gs, tune_cache=args.tune_cache)
    t_tune = time.time()
    if not args.no_tune and not cached:
        ctx.autotune(3)
    t_tune = time.time() - t_tune
    ctx.step(args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    # timed region: exactly K steps; device timestamps inside the replayed graphs
    elapsed, tm = time_steps(ctx, args.steps, torch)
    ms_step = elapsed * 1e3 / args.steps
    mlups = interior * args.steps / elapsed / 1e6
    lb_ms = tm[1]
    alg_bytes = tm[3]
    achieved = alg_bytes / (lb_ms * 1e-3) / 1e9
    traffic = committed_traffic(args.storage, args.boxes)
    checks = sum(1 for n in range(args.warmup, total_steps) if (n + 1) % check_every == 0)
    from paper_0809_4958_amd.prof_summary import kernel_source_hash
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"batched: {args.boxes} KS tracer boxes with edges from {{32,48,64,96}}, "
                         f"D3Q19 MRT tau=0.6, FP32 compute / "
                         f"{'FP16-deviation' if args.storage == 'f16' else 'FP32'} storage, "
                         "sampled 17x17 faces every 20 steps, one 32-bead FENE chain per box"),
            "boxes": args.boxes,
            "interior_nodes": int(interior),
            "storage": args.storage,
            "graph_steps": gs,
            "graph_replayed": gs > 0 and args.steps % gs == 0,
            "check_every": check_every,
            "check_steps_timed": checks,
            "autotuned": not args.no_tune and not cached,
            "tune_cache": args.tune_cache if cached else None,
            "autotune_s": round(t_tune, 2),
            "launch": ctx.describe(),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_lb (fused collide-stream + boundary faces)",
            "kernel_ms": round(lb_ms, 4),
            # x-face boundary velocities + chain kernel, per step
            "pre_lb_kernels_ms": round(tm[2], 4),
            "algorithmic_bytes_per_launch": alg_bytes,
            "copy_probe_gbs": None if copy_gbs is None else round(copy_gbs, 1),
            "memcpy_d2d_gbs": None if memcpy_gbs is None else round(memcpy_gbs, 1),
            "kernel_sources_sha1": kernel_source_hash(),
        },
        "input_generation_s": round(t_in, 1),
    }
    ctx.close()
    print(json.dumps({"progress": "timed region done", "mlups": out["value"],
                      "k_lb_ms": round(lb_ms, 4)}), file=sys.stderr, flush=True)

    if not args.no_baselines:
        # plain FP32: one single-box context per box size, each timed over a
        # fixed graph-replayed window; the batch's time is the sum over its boxes
        sizes = sorted({b["n"] for b in boxes})
        first = {n: next(b["index"] for b in boxes if b["n"] == n) for n in sizes}
        singles = batch_inputs(args.boxes, PLAIN_WARMUP + PLAIN_STEPS, tau, only=set(first.values()))
        per_size_ms = {}
        for b in singles:
            single = make_ctx(lbm, [b], lbm.STORE_F32, tau, reduce_every=100, stream=stream,
                              graph_steps=PLAIN_GRAPH)
            single.step(PLAIN_WARMUP)
            single.sync()
            t, _ = time_steps(single, PLAIN_STEPS, torch)
            per_size_ms[b["n"]] = t * 1e3 / PLAIN_STEPS
            single.close()
        plain_ms = sum(per_size_ms[b["n"]] for b in boxes)
        plain_mlups = interior / (plain_ms * 1e-3) / 1e6
        out["plain_fp32_single_box"] = {"mlups": round(plain_mlups, 1),
                                        "ms_per_step_all_boxes": round(plain_ms, 3),
                                        "ms_per_box_step": {str(k): round(v, 4)
                                                            for k, v in per_size_ms.items()},
                                        "window": f"{PLAIN_WARMUP} + {PLAIN_STEPS} steps, "
                                                  f"{PLAIN_GRAPH}-step graphs"}
        out["gain_vs_plain_fp32"] = round(mlups / plain_mlups, 2)
        print(json.dumps({"progress": "plain FP32 leg done"}), file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_leg(args, lbm, singles, tau, storage, stream, torch)
    print(json.dumps(out), flush=True)


def cpu_baseline_leg(args, lbm, sample_boxes, tau, storage, stream, torch):
    """The FP64 oracle on the host cores: its throughput on a bounded sample of
    the workload (one box of each edge), and the error of the GPU path's
    velocity on the first 32^3 box of the batch against it over the
    workload's full 5,000 steps."""
    import oracle
    sizes = [b["n"] for b in sample_boxes]
    lups = 0.0
    t1 = time.perf_counter()
    for bb in sample_boxes:
        n = bb["n"]
        o2 = oracle.OracleBox((n, n, n), collision=oracle.MRT, tau=tau, tau_bulk=tau)
        o2.set_initial(bb["u0"])
        o2.set_boundary(oracle.BC_SAMPLED, bb["faces"].astype(np.float64), t0=0, dt=20, res=17)
        o2.add_chain(bb["pos"], None, mass=bead_mass(32), anchor=bb["anchor"])
        k = 0
        ts = time.perf_counter()
        while (time.perf_counter() - ts < args.cpu_seconds / len(sample_boxes)
               and k + 5 <= PLAIN_WARMUP + PLAIN_STEPS):
            if o2.step(5) != 0:
                raise RuntimeError("oracle stopped with status %d" % o2.error()[0])
            k += 5
        lups += (n - 2) ** 3 * k
    t_cpu = time.perf_counter() - t1
    res = {"value": round(lups / t_cpu / 1e6, 2), "unit": "MLUPS",
           "cores": oracle.threads(), "kind": "oracle",
           "sample": (f"FP64 oracle, one box of each edge {sizes} from the batch, MRT + chain, "
                      f"about {args.cpu_seconds:.0f} s of stepping ({lups:.3g} lattice updates)")}
    # accuracy: the first 32^3 box of the batch, alone in a context of the
    # benchmarked storage (batched and single contexts are bitwise identical),
    # against the oracle over the workload's 5,000 steps
    k32 = next(b["index"] for b in sample_boxes if b["n"] == 32)
    b = batch_inputs(args.boxes, ORACLE_ERR_STEPS, tau, only={k32})[0]
    ob = oracle.OracleBox((32, 32, 32), collision=oracle.MRT, tau=tau, tau_bulk=tau, ghost_rate=1.0)
    ob.set_initial(b["u0"])
    ob.set_boundary(oracle.BC_SAMPLED, b["faces"].astype(np.float64), t0=0, dt=20, res=17)
    ob.add_chain(b["pos"], None, substeps=10, fix_com=True, zeta=5.0, mass=bead_mass(32),
                 fene_k=1.0, fene_r0=2.0, anchor=b["anchor"])
    t2 = time.perf_counter()
    st = ob.step(ORACLE_ERR_STEPS)
    t_or = time.perf_counter() - t2
    g = make_ctx(lbm, [b], storage, tau, reduce_every=100, stream=stream, graph_steps=100)
    g.step(ORACLE_ERR_STEPS)
    g.sync()
    torch.cuda.synchronize()
    _, uo = ob.rho_u()
    ug = g.read(0, lbm.F_U)
    g.close()
    m = ob.interior_mask()
    err = float(np.linalg.norm(ug[m] - uo[m]) / np.linalg.norm(uo[m]))
    err_max = float(np.abs(ug[m] - uo[m]).max() / np.abs(uo[m]).max())
    res["rel_err_u_vs_oracle"] = {"value": err, "max_norm": err_max, "storage": args.storage,
                                  "box": k32, "edge": 32, "steps": ORACLE_ERR_STEPS,
                                  "oracle_status": int(st), "oracle_seconds": round(t_or, 2)}
    return res


if __name__ == "__main__":
    main()
