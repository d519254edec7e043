"""Train the learned boundary upsampler on the GPU and evaluate it.

Training data come from the plain method's input fields: for each KS tracer
trajectory, the coarse face samples (8 x 8 corner-aligned every 20 steps) and
the dense per-step 64 x 64 face field they should be mapped to
(``inputs.upsampler_samples``).  Every training step (forward, loss, backward,
Adam) runs in the library's kernels; this script only feeds batches.

Evaluation on held-out trajectories:
  * face field: relative L2 error of the learned field and of the plain
    interpolation (bilinear in space, linear in time) against the dense field;
  * downstream: a 64^3 box (D3Q19 MRT, tau = 0.6, FP32 storage) run three times
    from the same initial field, driven by the dense field (every step, every
    node), by the interpolation of the coarse samples, and by the learned
    field (LEARNED ring refilled every window); relative L2 error of the
    interior velocity of the latter two against the first.

Inference speed: one window of lbn_window_forward (6 faces x 20 steps of
64 x 64 fields from resident samples), timed with HIP events.

Usage:  python -m paper_0809_4958_amd.train_upsampler [--traj 2000] [--out PATH]
Prints one JSON line; writes the parameter vector (float32, .npy) to --out.

        python -m paper_0809_4958_amd.train_upsampler --speed
times only the kernels: window inference with the committed weights and
training iterations of batch 64 on 16 trajectories' samples (no training
run, nothing written).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(PKG))

from paper_0809_4958_amd import inputs, lbm, lbnet  # noqa: E402

CFG_LEARNED = 3
FLOPS_SAMPLE = 2.0 * 64 * 64 * 9 * (16 * 64 + 64 * 64 + 64 * 16)   # MFMA work per image, padded channels
WEIGHTS = os.path.join(PKG, "weights", "upsampler_r8.npy")
HELD_OUT_BASE = 5000


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) /
                 np.linalg.norm(np.asarray(b, np.float64)))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def train(net, c, th, truth, iters, batch, lr, seed=0, log_every=500):
    import torch
    g = np.random.Generator(np.random.PCG64(seed))
    cd, thd, trd = dev(c), dev(th), dev(truth)
    n = c.shape[0]
    hist = []
    for it in range(iters):
        idx = torch.from_numpy(g.choice(n, size=batch, replace=False)).cuda()
        want = it % log_every == 0 or it == iters - 1
        loss = net.train_step(cd[idx].contiguous(), thd[idx].contiguous(), trd[idx].contiguous(),
                              lr=lr * 0.1 ** (it / iters), want_loss=want)
        if want:
            hist.append((it, loss))
            print(json.dumps({"progress": "train", "iter": it, "loss": loss}), file=sys.stderr, flush=True)
    return hist


def face_fields(net, c, th, batch):
    """Learned fields and (from a zero network) the plain interpolation."""
    import torch
    out = torch.zeros((c.shape[0], 64, 64, 3), device="cuda")
    for i in range(0, c.shape[0], batch):
        net.forward(dev(c[i:i + batch]), dev(th[i:i + batch]), out[i:i + batch])
    plain = lbnet.Upsampler(coarse=c.shape[-1], max_batch=batch)
    plain.set_params(np.zeros(lbnet.PARAM_COUNT, np.float32))
    base = torch.zeros_like(out)
    for i in range(0, c.shape[0], batch):
        plain.forward(dev(c[i:i + batch]), dev(th[i:i + batch]), base[i:i + batch])
    torch.cuda.synchronize()
    plain.close()
    return out.cpu().numpy(), base.cpu().numpy()


def time_window_inference(net, traj, dt=20, R=8, reps=200):
    """Average time of one window of inference (lbn_window_forward: the 6 faces
    x dt per-step fields of one window, 6 dt images of 64 x 64) on resident
    samples, timed with HIP events on the network's stream."""
    import torch
    _, _, coarse = inputs.ks_box_inputs(CFG_LEARNED, traj, n=64, tau=0.6, n_steps=4 * dt, dt=dt, res=R)
    hist = dev(coarse)
    ring = torch.zeros((dt, 6, 64, 64, 3), device="cuda")
    for _ in range(5):
        net.window_forward(hist, 1, dt, ring)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.window_forward(hist, 1, dt, ring)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps, 6 * dt


def downstream(net, traj, n=64, tau=0.6, windows=3, dt=20, R=8):
    """Interior-velocity errors of the interpolated and the learned boundary
    against the dense boundary after `windows` windows of dt steps."""
    import torch
    steps = windows * dt
    _, u0, dense = inputs.ks_box_inputs(CFG_LEARNED, traj, n=n, tau=tau, n_steps=steps, dt=1, res=n)
    _, _, coarse = inputs.ks_box_inputs(CFG_LEARNED, traj, n=n, tau=tau, n_steps=steps + 2 * dt, dt=dt, res=R)
    stream = torch.cuda.current_stream().cuda_stream
    us = {}
    for mode in ("dense", "interp", "learned"):
        ctx = lbm.Context([(n, n, n)], collision=lbm.MRT, tau=tau, tau_bulk=tau, storage=lbm.STORE_F32,
                          stream=stream)
        ctx.set_initial(0, u0)
        if mode == "dense":
            ctx.set_boundary(0, lbm.BC_SAMPLED, dense.astype(np.float32), t0=0, dt=1, res=n)
            ctx.step(steps)
        elif mode == "interp":
            ctx.set_boundary(0, lbm.BC_SAMPLED, coarse.astype(np.float32), t0=0, dt=dt, res=R)
            ctx.step(steps)
        else:
            ring = torch.zeros((dt, 6, n, n, 3), device="cuda")
            hist = dev(coarse)
            ctx.set_boundary(0, lbm.BC_LEARNED, ring, t0=0, dt=1, res=n)
            for k in range(windows):
                net.window_forward(hist, k, dt, ring)      # same stream: ordered with the steps
                ctx.step(dt)
        ctx.sync()
        us[mode] = ctx.read(0, lbm.F_U)[1:-1, 1:-1, 1:-1]
        ctx.close()
    return rel_l2(us["interp"], us["dense"]), rel_l2(us["learned"], us["dense"])


def speed(args, iters=200):
    """Kernel speed: one inference window and training iterations."""
    import torch
    net = lbnet.Upsampler(coarse=8, max_batch=max(args.batch, 120))
    net.set_params(np.load(WEIGHTS))
    win_ms, win_images = time_window_inference(net, HELD_OUT_BASE)
    c, th, truth = inputs.upsampler_samples(CFG_LEARNED, range(16), windows=(0, 1), phases=(0, 10))
    b = args.batch
    cd, thd, trd = dev(c[:b]), dev(th[:b]), dev(truth[:b])
    for _ in range(10):
        net.loss_grad(cd, thd, trd, want_loss=False)
        net.adam_step(args.lr)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        net.loss_grad(cd, thd, trd, want_loss=False)
        net.adam_step(args.lr)
    e1.record()
    e1.synchronize()
    train_ms = e0.elapsed_time(e1) / iters
    fs = FLOPS_SAMPLE
    out = {"infer_window_ms": round(win_ms, 4), "infer_window_images": win_images,
           "infer_tflops_mfma": round(fs * win_images / (win_ms * 1e-3) / 1e12, 2),
           "infer_mfma_frac_of_bf16_dense_peak": round(fs * win_images / (win_ms * 1e-3) / 2.5e15, 4),
           "train_ms_per_iter": round(train_ms, 4), "train_batch": b,
           "train_tflops_mfma": round(3 * fs * b / (train_ms * 1e-3) / 1e12, 2)}
    print(json.dumps(out), flush=True)
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--traj", type=int, default=2000)
    ap.add_argument("--held-out", type=int, default=200)
    ap.add_argument("--iters", type=int, default=8000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--downstream", type=int, default=4, help="held-out boxes run downstream")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--speed", action="store_true", help="time the kernels only")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.speed:
        return speed(args)
    t0 = time.time()
    parts = []
    for a in range(0, args.traj, 250):
        parts.append(inputs.upsampler_samples(CFG_LEARNED, range(a, min(a + 250, args.traj)),
                                              windows=(0, 1), phases=(0, 10)))
        print(json.dumps({"progress": "data", "trajectories": min(a + 250, args.traj)}), file=sys.stderr,
              flush=True)
    c, th, truth = (np.concatenate([p[i] for p in parts]) for i in range(3))
    del parts
    ch, thh, trh = inputs.upsampler_samples(CFG_LEARNED, range(HELD_OUT_BASE, HELD_OUT_BASE + args.held_out),
                                            windows=(1,), phases=(5, 15))
    t_data = time.time() - t0
    print(json.dumps({"progress": "data", "train_samples": int(c.shape[0]), "seconds": round(t_data, 1)}),
          file=sys.stderr, flush=True)
    net = lbnet.Upsampler(coarse=8, max_batch=max(args.batch, 120))
    net.set_params(lbnet.init_params(0))
    torch.cuda.synchronize()
    t1 = time.time()
    hist = train(net, c, th, truth, args.iters, args.batch, args.lr)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    u_net, u_base = face_fields(net, ch, thh, 120)
    e_net, e_base = rel_l2(u_net, trh), rel_l2(u_base, trh)
    ds = [downstream(net, HELD_OUT_BASE + i) for i in range(args.downstream)]
    win_ms, win_images = time_window_inference(net, HELD_OUT_BASE)
    p = net.params()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, p)
    flops_sample = FLOPS_SAMPLE
    out = {
        "workload": "learned boundary upsampler, 8x8 coarse faces every 20 steps -> 64x64 per step",
        "train_trajectories": args.traj, "train_samples": int(c.shape[0]),
        "held_out_trajectories": args.held_out, "held_out_samples": int(ch.shape[0]),
        "iters": args.iters, "batch": args.batch, "lr": args.lr,
        "loss_first": hist[0][1], "loss_last": hist[-1][1],
        "face_rel_l2_learned": e_net, "face_rel_l2_interpolation": e_base,
        "face_gain": e_base / e_net,
        "downstream_interior_u_rel_l2_interpolation": [d[0] for d in ds],
        "downstream_interior_u_rel_l2_learned": [d[1] for d in ds],
        "train_seconds": round(t_train, 2), "data_seconds": round(t_data, 1),
        "train_ms_per_iter": round(t_train * 1e3 / args.iters, 3),
        "train_tflops_mfma": round(3.0 * flops_sample * args.batch * args.iters / t_train / 1e12, 2),
        "infer_window_ms": round(win_ms, 4),
        "infer_window_images": win_images,
        "infer_tflops_mfma": round(flops_sample * win_images / (win_ms * 1e-3) / 1e12, 2),
        "infer_mfma_frac_of_bf16_dense_peak": round(flops_sample * win_images / (win_ms * 1e-3) / 2.5e15, 4),
        "weights": os.path.relpath(args.out, os.path.dirname(PKG)),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
