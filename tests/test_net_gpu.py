"""GPU parity of the learned boundary upsampler against the FP64 oracle, its
training on the GPU, and the LEARNED boundary of the lattice-Boltzmann library.

Tolerances.  The oracle runs with bfloat16 rounding at the points where the
kernels store bfloat16 (``bf=True``), so the remaining differences come from
FP32 accumulation against FP64 (relative ~1e-6) and the rare bfloat16
rounding it flips (one ulp, 2^-8 relative, on a fraction ~2^-15 of the
values).  Element-wise these stay far below 2e-3 in relative L2; a wrong tap,
a transposed operand or a dropped term gives O(1).  Against the unrounded FP64
oracle the network output differs by the bfloat16 precision itself, stated
below as ~3e-2 relative on r.
"""
import numpy as np
import pytest

from lbcase import max_rel, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import net_oracle as no  # noqa: E402
from paper_0809_4958_amd import inputs, lbm, lbnet  # noqa: E402

CFG_LEARNED = 3   # seed stream of the learned-boundary workload


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module")
def samples():
    # one trajectory, window 1, phases 0 and 10: 12 samples of real KS faces
    return inputs.upsampler_samples(CFG_LEARNED, [1000], windows=(1,), phases=(0, 10))


def test_forward_matches_oracle(samples):
    c, th, truth = samples
    B = 6
    c, th = c[:B], th[:B]
    p = lbnet.init_params(1)
    # a non-trivial last layer (the initial one is zero)
    p[-(3 * 64 * 9 + 3):] = np.random.Generator(np.random.PCG64(21)).standard_normal(3 * 64 * 9 + 3) * 0.05
    net = lbnet.Upsampler(coarse=8, max_batch=16)
    net.set_params(p)
    out = torch.zeros((B, 64, 64, 3), device="cuda")
    say("case upsampler forward B=6")
    net.forward(dev(c), dev(th), out)
    torch.cuda.synchronize()
    fw = no.forward(p.astype(np.float64), c, th, bf=True)
    x0 = net.read_buffer(lbnet.BUF_LIFT, B)
    a1 = net.read_buffer(lbnet.BUF_A1, B)
    a2 = net.read_buffer(lbnet.BUF_A2, B)
    r = net.read_buffer(lbnet.BUF_R, B)
    chw = lambda a: a.transpose(0, 3, 1, 2)  # noqa: E731
    pairs = {"x0": (chw(x0[..., :15]), fw["x0"]), "a1": (chw(a1), fw["a1"]), "a2": (chw(a2), fw["a2"]),
             "r": (chw(r[..., :3]), fw["r"]), "u": (out.cpu().numpy(), fw["u"].transpose(0, 2, 3, 1))}
    e = {k: rel_l2(a, b) for k, (a, b) in pairs.items()}
    m = {k: max_rel(a, b) for k, (a, b) in pairs.items()}
    say("forward rel-L2 vs bf16-emulating oracle", e)
    say("forward max-norm (largest error over the field's largest value)", m)
    assert max(e.values()) < 2e-3
    # a bf16 activation can land one bf16 step (2^-8 of its value) away where
    # the FP32 sum and the oracle's FP64 sum round to neighbouring values
    # (measured 2.6e-3 for a1 and a2)
    assert max(m.values()) < 5e-3
    assert np.all(x0[..., 15:] == 0) and np.all(r[..., 3:] == 0)
    # the bfloat16 precision itself, against the unrounded FP64 network
    fw64 = no.forward(p.astype(np.float64), c, th, bf=False)
    e64 = rel_l2(chw(r[..., :3]), fw64["r"])
    say("r vs FP64 oracle", e64)
    assert e64 < 3e-2
    net.close()


def test_forward_is_independent_of_the_batch_split():
    """Layers 2 and 3 walk bands of image rows whose number depends on the
    batch (one band per image at 256 samples, two at 120, four at 64, sixteen
    at 12 or 1); every output comes from the same products in the same order
    whatever band computes it, so a sample's face field and layer-2
    activations are bitwise the same in any batch."""
    g = np.random.Generator(np.random.PCG64(5))
    N = 256
    c = (g.standard_normal((N, 4, 3, 8, 8)) * 1e-3).astype(np.float32)
    th = g.random(N).astype(np.float32)
    p = lbnet.init_params(2)
    p[-(3 * 64 * 9 + 3):] = g.standard_normal(3 * 64 * 9 + 3) * 0.05
    net = lbnet.Upsampler(coarse=8, max_batch=N)
    net.set_params(p)
    full = torch.zeros((N, 64, 64, 3), device="cuda")
    say("case forward batch 256")
    net.forward(dev(c), dev(th), full)
    torch.cuda.synchronize()
    full = full.cpu().numpy()
    a2_full = net.read_buffer(lbnet.BUF_A2, N)
    assert np.isfinite(full).all() and np.abs(full).max() > 0
    for lo, n in ((0, 120), (120, 64), (184, 12), (255, 1)):
        part = torch.zeros((n, 64, 64, 3), device="cuda")
        say("case forward batch", n, "samples", lo, "..", lo + n - 1)
        net.forward(dev(c[lo:lo + n]), dev(th[lo:lo + n]), part)
        torch.cuda.synchronize()
        assert np.array_equal(part.cpu().numpy(), full[lo:lo + n]), n
        assert np.array_equal(net.read_buffer(lbnet.BUF_A2, n), a2_full[lo:lo + n]), n
    net.close()


def test_gradients_and_adam_match_oracle(samples):
    c, th, truth = samples
    B = 6
    c, th, truth = c[:B], th[:B], truth[:B]
    p = lbnet.init_params(2)
    p[-(3 * 64 * 9 + 3):] = np.random.Generator(np.random.PCG64(22)).standard_normal(3 * 64 * 9 + 3) * 0.05
    net = lbnet.Upsampler(coarse=8, max_batch=16)
    net.set_params(p)
    say("case upsampler loss/grad B=6")
    loss, grad = net.loss_grad(dev(c), dev(th), dev(truth), want_loss=True, want_grad=True)
    L, g_or, _ = no.loss_grad(p.astype(np.float64), c, th, truth, bf=True)
    say("loss gpu", loss, "oracle", L)
    assert abs(loss - L) <= 1e-4 * L
    blocks = ["W1", "b1", "W2", "b2", "W3", "b3"]
    errs = {n: rel_l2(a, b) for n, a, b in zip(blocks, lbnet.split_params(grad), no.split(g_or))}
    errm = {n: max_rel(a, b) for n, a, b in zip(blocks, lbnet.split_params(grad), no.split(g_or))}
    say("gradient rel-L2 per block", errs)
    say("gradient max-norm per block", errm)
    assert max(errs.values()) < 5e-3
    # the same bf16 products summed in FP32 against FP64 (measured <= 5.3e-6)
    assert max(errm.values()) < 1e-4
    # one Adam step from the same parameters (oracle: its own gradient)
    net.adam_step(lr=1e-3)
    p1 = net.params()
    p1_or, _, _ = no.adam(p.astype(np.float64), g_or, np.zeros(p.size), np.zeros(p.size), 1, lr=1e-3)
    d_gpu, d_or = p1 - p, p1_or - p
    # the first step is ~ -lr sign(g): compare where the gradient is not tiny
    big = np.abs(g_or) > 1e-3 * np.abs(g_or).max()
    frac = np.mean(np.abs(d_gpu[big] - d_or[big]) > 1e-2 * 1e-3)
    say("Adam step: fraction of mismatched updates", frac)
    assert frac < 0.01
    net.close()


def test_loss_matches_the_forward_output_at_any_batch(samples):
    """The loss the forward's last layer forms equals the mean of
    ((u - truth) / s)^2 recomputed in FP64 on the host from lbn_forward's face
    field u and scales s, at one band per image (batch 256: one loss partial
    per image), several bands and a single image; and r after lbn_loss_grad is
    bitwise the r of lbn_forward (the same last-layer arithmetic)."""
    c, th, truth = samples
    p = lbnet.init_params(4)
    p[-(3 * 64 * 9 + 3):] = np.random.Generator(np.random.PCG64(23)).standard_normal(3 * 64 * 9 + 3) * 0.05
    net = lbnet.Upsampler(coarse=8, max_batch=256)
    net.set_params(p)
    for batch in (1, 37, 256):
        idx = np.arange(batch) % c.shape[0]
        cb, thb, tb = c[idx], th[idx], truth[idx]
        say(f"case upsampler loss at batch {batch}")
        out = torch.zeros((batch, 64, 64, 3), device="cuda")
        net.forward(dev(cb), dev(thb), out)
        torch.cuda.synchronize()
        u = out.cpu().numpy().astype(np.float64)
        s = net.read_buffer(lbnet.BUF_SCALE, batch).astype(np.float64)
        r_fwd = net.read_buffer(lbnet.BUF_R, batch)
        l_host = float(np.mean(((u - tb) / s[:, None, None, None]) ** 2))
        loss, _ = net.loss_grad(dev(cb), dev(thb), dev(tb), want_loss=True)
        say("loss gpu", loss, "host from the forward output", l_host)
        # e in FP32 on the GPU against FP64 here: rounding of e only
        assert abs(loss - l_host) <= 1e-5 * l_host
        assert np.array_equal(net.read_buffer(lbnet.BUF_R, batch), r_fwd)
    net.close()


def test_training_is_bitwise_reproducible(samples):
    """Two trainings from the same parameters on the same batches end in the
    same bits: every reduction of the backward pass runs in a fixed order."""
    c, th, truth = samples
    runs = []
    for rep in range(2):
        say(f"case upsampler training reproducibility, run {rep}")
        net = lbnet.Upsampler(coarse=8, max_batch=64)
        net.set_params(lbnet.init_params(5))
        train(net, c, th, truth, iters=40, batch=min(32, c.shape[0]), lr=3e-4, seed=3)
        runs.append(net.params())
        net.close()
    assert np.array_equal(runs[0], runs[1])


def test_window_forward_matches_gathered_samples():
    """The window entry point gathers S_{k-1..k+2} (clamped) and the phases
    itself; its result equals lbn_forward on the same inputs gathered here."""
    R, dt, ns = 8, 20, 5
    g = np.random.Generator(np.random.PCG64(7))
    hist = g.standard_normal((ns, 6, R, R, 3)).astype(np.float32) * 1e-3
    net = lbnet.Upsampler(coarse=R, max_batch=6 * dt)
    net.set_params(lbnet.init_params(3))
    for k in (0, 2, ns - 2):
        ring = torch.zeros((dt, 6, 64, 64, 3), device="cuda")
        say("case window_forward k =", k)
        net.window_forward(dev(hist), k, dt, ring)
        idx = [min(max(k - 1 + t, 0), ns - 1) for t in range(4)]
        co = hist[idx].transpose(1, 0, 4, 2, 3)                  # [6][4][3][R][R]
        c_all = np.stack([co[f] for j in range(dt) for f in range(6)])
        th_all = np.array([j / dt for j in range(dt) for f in range(6)], np.float32)
        ref = torch.zeros((6 * dt, 64, 64, 3), device="cuda")
        net.forward(dev(c_all), dev(th_all), ref)
        torch.cuda.synchronize()
        assert torch.equal(ring.reshape(6 * dt, 64, 64, 3), ref)
    net.close()


def train(net, c, th, truth, iters, batch, lr, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    n = c.shape[0]
    cd, thd, trd = dev(c), dev(th), dev(truth)
    losses = []
    for it in range(iters):
        idx = torch.from_numpy(g.choice(n, size=batch, replace=False)).cuda()
        want = it % 250 == 0 or it == iters - 1
        lr_it = lr * (0.1 ** (it / iters))          # exponential decay to lr / 10
        loss = net.train_step(cd[idx].contiguous(), thd[idx].contiguous(), trd[idx].contiguous(),
                              lr=lr_it, want_loss=want)
        if want:
            losses.append(loss)
    return losses


def face_errors(net, c, th, truth, batch=64):
    out = torch.zeros((c.shape[0], 64, 64, 3), device="cuda")
    for i in range(0, c.shape[0], batch):
        net.forward(dev(c[i:i + batch]), dev(th[i:i + batch]), out[i:i + batch])
    torch.cuda.synchronize()
    u = out.cpu().numpy()
    base = no.baseline(c, th)
    return rel_l2(u, truth), rel_l2(base, truth)


def test_training_on_gpu_beats_interpolation():
    """Train on KS faces of 48 trajectories, evaluate on 8 held-out ones: the
    learned field is closer to the dense truth than the interpolation the
    plain method uses (the network's gain), and the loss went down."""
    say("case upsampler training (48 trajectories)")
    c, th, truth = inputs.upsampler_samples(CFG_LEARNED, range(48), windows=(0, 1, 2), phases=(0, 7, 14))
    ch, thh, trh = inputs.upsampler_samples(CFG_LEARNED, range(5000, 5008), windows=(1,), phases=(3, 11))
    net = lbnet.Upsampler(coarse=8, max_batch=64)
    net.set_params(lbnet.init_params(0))
    losses = train(net, c, th, truth, iters=1500, batch=32, lr=3e-4)
    e_net, e_base = face_errors(net, ch, thh, trh)
    say("loss history", [f"{v:.3e}" for v in losses])
    say(f"held-out face rel-L2: learned {e_net:.4e}  interpolation {e_base:.4e}  gain {e_base / e_net:.2f}x")
    assert losses[-1] < 0.3 * losses[0]
    assert e_net < 0.5 * e_base
    net.close()


def test_learned_ring_equals_dense_sampled_boundary():
    """A LEARNED ring of per-step face fields (dt = 1, res = N) drives the box
    exactly like the same fields given as a SAMPLED history: bitwise."""
    n, steps = 24, 12
    g = np.random.Generator(np.random.PCG64(11))
    fields = (g.standard_normal((steps + 1, 6, n, n, 3)) * 1e-3).astype(np.float32)
    outs = []
    for mode in ("sampled", "learned"):
        # the context runs on torch's stream, so the ring refills are ordered
        # with the steps that read them
        ctx = lbm.Context([(n, n, n)], collision=lbm.MRT, tau=0.6, storage=lbm.STORE_F32,
                          stream=torch.cuda.current_stream().cuda_stream)
        if mode == "sampled":
            ctx.set_boundary(0, lbm.BC_SAMPLED, fields, t0=0, dt=1, res=n)
        else:
            ring = dev(fields[:4])                     # 4-slot ring, refilled as we go
            ctx.set_boundary(0, lbm.BC_LEARNED, ring, t0=0, dt=1, res=n)
        say("case learned ring vs sampled:", mode)
        for s0 in range(0, steps, 4):
            if mode == "learned":
                ring.copy_(dev(fields[s0:s0 + 4]))
            ctx.step(4)
        ctx.sync()
        outs.append(ctx.read(0, lbm.F_POP))
        ctx.close()
    assert np.array_equal(outs[0], outs[1])


def test_learned_boundary_rejects_fp64_contexts():
    ctx = lbm.Context([(8, 8, 8)], storage=lbm.STORE_F64)
    ring = torch.zeros((2, 6, 8, 8, 3), device="cuda")
    with pytest.raises(lbm.LBError):
        ctx.set_boundary(0, lbm.BC_LEARNED, ring, t0=0, dt=1, res=8)
    ctx.close()


def test_trained_weights_gain_downstream():
    """The committed network (trained on 2,000 trajectories by
    paper_0809_4958_amd/train_upsampler.py) against the plain interpolation on
    held-out trajectories: the face field is closer to the dense field, and so
    is the interior velocity of a 64^3 box driven by it for three windows."""
    import os
    from paper_0809_4958_amd import train_upsampler as tu
    if not os.path.exists(tu.WEIGHTS):
        pytest.skip("no trained weights committed")
    net = lbnet.Upsampler(coarse=8, max_batch=120)
    net.set_params(np.load(tu.WEIGHTS, allow_pickle=False))
    ch, thh, trh = inputs.upsampler_samples(CFG_LEARNED, range(tu.HELD_OUT_BASE + 300, tu.HELD_OUT_BASE + 308),
                                            windows=(2,), phases=(4, 13))
    u_net, u_base = tu.face_fields(net, ch, thh, 96)
    e_net, e_base = rel_l2(u_net, trh), rel_l2(u_base, trh)
    say(f"held-out face rel-L2: learned {e_net:.4e} interpolation {e_base:.4e} gain {e_base / e_net:.2f}x")
    assert e_net < 0.5 * e_base
    say("case downstream 64^3 box, 3 windows")
    e_i, e_l = tu.downstream(net, tu.HELD_OUT_BASE + 300)
    say(f"downstream interior u rel-L2 vs dense boundary: interpolation {e_i:.4e} learned {e_l:.4e}")
    assert e_l < e_i
    net.close()

