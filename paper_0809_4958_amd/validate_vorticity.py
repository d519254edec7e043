"""Validation analogue of the paper's comparison of the fine box with the DNS
(Sec. 3, Figs. 1 and 2): the vorticity magnitude averaged over the whole box
((6 eta)^3 in the paper) and over a central (1.25 eta)^3 volume, for many
tracers, from the LB box driven only by its initial field and its boundary
history, against the field that drives it.

The paper's field is its DNS (not available); a kinematic-simulation (KS)
field stands in (paper_0809_4958_amd/inputs.py).  The setup follows Sec. 3:
a box of 121 nodes per edge spanning 6 eta (zoom 6 of a DNS with eta/Delta =
3.33), faces sampled on the 21 x 21 grid of DNS points every 0.05 tau_eta and
interpolated linearly in space and time, tau = 1 (nu = 1/6, Mach number
eta~ / (tau~_eta c_s) = 0.0144 against the paper's 0.0149).  The KS field is
not a solution of the Navier-Stokes equations, so the LB interior, which is,
departs from it inside the box: the differences are reported, with no pass
bar (the paper's DNS gives less than 5 %).

Every step of the LB and the vorticity runs in the HIP library; the analytic
KS vorticity is evaluated on the host from the field's modes.

  python -m paper_0809_4958_amd.validate_vorticity [--tracers 16] [--tau-eta 4]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs

CONFIG_IDX = 5          # seed stream of this validation run
N = 121                 # nodes per edge: (120 a)^3
WIDTH_ETA = 6.0         # box width in Kolmogorov lengths
TAU = 1.0
RES = 21                # DNS points per face edge
CENTRE_ETA = 1.25       # edge of the central control volume


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--tracers", type=int, default=16)
    p.add_argument("--tau-eta", type=float, default=4.0, help="run length in Kolmogorov times")
    p.add_argument("--samples-per-tau", type=int, default=5)
    p.add_argument("--storage", default="f32", choices=["f32", "f16"])
    p.add_argument("--out", default=None, help="write the summary (text) to this file")
    return p.parse_args(argv)


def main(argv=None):
    args = parse(argv)
    import torch

    from . import lbm
    torch.cuda.set_device(0)
    units = inputs.UnitMap(N, TAU, WIDTH_ETA)
    dt = int(round(0.05 * units.tau_eta))                 # face samples every 0.05 tau_eta
    every = int(round(units.tau_eta / args.samples_per_tau / dt)) * dt
    n_samples_out = int(round(args.tau_eta * args.samples_per_tau))
    steps = every * n_samples_out
    n_face = steps // dt + 1
    face_steps = np.arange(n_face) * dt
    t0 = time.time()
    boxes = []
    for b in range(args.tracers):
        ks, x0 = inputs.ks_tracer(CONFIG_IDX, b)
        tr = inputs.tracer_path(ks, x0, face_steps / units.tau_eta)
        u0 = inputs.initial_field(ks, tr, (N, N, N), units, 0)
        faces = inputs.face_samples(ks, tr, (N, N, N), units, RES, face_steps).astype(np.float32)
        boxes.append(dict(ks=ks, tr=tr, u0=u0, faces=faces))
    print(json.dumps({"progress": "inputs", "seconds": round(time.time() - t0, 1), "dt": dt,
                      "steps": steps, "tau_eta_steps": units.tau_eta}), flush=True)
    storage = lbm.STORE_F16DEV if args.storage == "f16" else lbm.STORE_F32
    ctx = lbm.Context([(N, N, N)] * len(boxes), collision=lbm.MRT, tau=TAU, tau_bulk=TAU,
                      ghost_rate=1.0, storage=storage, torch_alloc=True, graph_steps=every)
    for k, b in enumerate(boxes):
        ctx.set_initial(k, b.pop("u0"))
        ctx.set_boundary(k, lbm.BC_SAMPLED, b["faces"], t0=0, dt=dt, res=RES)
    # control volumes: every node with interior neighbours, and the central
    # (1.25 eta)^3 box
    c = (N - 1) // 2
    half = int(round(CENTRE_ETA * units.eta / 2))
    vols = [([2, 2, 2], [N - 3] * 3), ([c - half] * 3, [c + half] * 3)]
    axes_all = [(np.arange(2, N - 2) - c) / units.eta] * 3
    sl_c = slice(c - half - 2, c + half - 1)   # central volume inside the whole range
    lb_mean = np.zeros((n_samples_out + 1, len(boxes), 2))
    ks_mean = np.zeros_like(lb_mean)
    t_lb = 0.0
    for s in range(n_samples_out + 1):
        if s:
            t1 = time.time()
            ctx.step(every)
            ctx.sync()
            t_lb += time.time() - t1
        n_step = s * every
        fi = n_step // dt
        for k, b in enumerate(boxes):
            lb_mean[s, k] = ctx.vorticity(k, vols)
            w = b["ks"].grid_vorticity(b["tr"].pos[fi], float(b["tr"].times[fi]), axes_all)
            mag = np.linalg.norm(w, axis=-1) / units.tau_eta      # lattice units
            ks_mean[s, k] = [mag.mean(), mag[sl_c, sl_c, sl_c].mean()]
        print(json.dumps({"progress": "sample", "step": n_step,
                          "rel_diff_whole_mean": float(np.mean(np.abs(lb_mean[s, :, 0] / ks_mean[s, :, 0] - 1))),
                          "rel_diff_centre_mean": float(np.mean(np.abs(lb_mean[s, :, 1] / ks_mean[s, :, 1] - 1)))}),
              flush=True)
    ctx.close()
    rel = np.abs(lb_mean / ks_mean - 1.0)           # [time][tracer][volume]
    summary = {
        "workload": (f"{len(boxes)} KS tracer boxes, {N}^3 nodes spanning {WIDTH_ETA:g} eta, "
                     f"MRT tau={TAU:g}, {args.storage} storage, {RES}x{RES} faces every {dt} steps "
                     f"(0.05 tau_eta), {steps} steps ({steps / units.tau_eta:.2f} tau_eta)"),
        "mach": units.mach(),
        "lb_seconds": round(t_lb, 2),
        "mlups": round(len(boxes) * (N - 2) ** 3 * steps / max(t_lb, 1e-9) / 1e6, 1),
        "rel_diff_at_t0": {"whole": float(rel[0, :, 0].mean()), "centre": float(rel[0, :, 1].mean())},
        "rel_diff_tracer_time_mean": {"whole": float(rel[1:, :, 0].mean()),
                                      "centre": float(rel[1:, :, 1].mean())},
        "rel_diff_median": {"whole": float(np.median(rel[1:, :, 0])),
                            "centre": float(np.median(rel[1:, :, 1]))},
        "rel_diff_p90": {"whole": float(np.percentile(rel[1:, :, 0], 90)),
                         "centre": float(np.percentile(rel[1:, :, 1], 90))},
        "rel_diff_vs_time_whole": [round(float(v), 4) for v in rel[:, :, 0].mean(axis=1)],
        "rel_diff_vs_time_centre": [round(float(v), 4) for v in rel[:, :, 1].mean(axis=1)],
        "sample_steps": [s * every for s in range(n_samples_out + 1)],
    }
    print(json.dumps(summary), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write("# Vorticity validation analogue (Sec. 3, Figs. 1-2): LB box vs the KS field that drives it\n")
            fh.write("# command: python -m paper_0809_4958_amd.validate_vorticity " + " ".join(sys.argv[1:]) + "\n")
            for key, val in summary.items():
                fh.write(f"{key}: {json.dumps(val)}\n")
    return summary


if __name__ == "__main__":
    main()
