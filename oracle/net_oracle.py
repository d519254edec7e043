"""FP64 CPU oracle of the learned boundary upsampler (TEST INFRASTRUCTURE ONLY).

Plain numpy, channels-first, written from the definitions, sharing nothing
with the HIP path.  Only the tests, the smoke check and the benchmark's CPU
leg may use it.

What it computes (the upsampler of one box face, one step of a sampling
window; the interpolation it corrects is the boundary rule of Sec. 2-3,
bilinear in space on the corner-aligned sample grid x linear in time):

  lift     L(S)[y][x]: corner-aligned bilinear interpolation of an R x R
           grid to img x img (grid point p sits at node p (img-1)/(R-1))
  input    with Sb = (1 - theta) S_k + theta S_k+1 and s the RMS of the
           4 x 3 x R x R coarse values (1 if they are all 0), 15 channels:
           L(Sb)/s, L(Duu Sb)/s, L(Dvv Sb)/s, L(S_k+2 - S_k+1 - S_k + S_k-1)/s
           (3 components each; Duu, Dvv the coarse second differences along
           u and v, edge nodes taking the next node's), theta, and the cell
           position weights 4a(1-a), 4b(1-b) of the corner-aligned lift
  net      z1 = conv(x0; W1, b1), a1 = relu(z1), z2 = conv(a1; W2, b2),
           a2 = relu(z2), r = conv(a2; W3, b3)
           conv(x; W, b)[co][y][x] = b[co] + sum W[co][ci][ky][kx] x[ci][y+ky-1][x+kx-1]
           (cross-correlation, zero padding)
  output   u = base + s r, base = L(Sb) (the plain interpolation)
  loss     mean over samples, pixels and components of ((u - truth) / s)^2,
           the squared error in units of the sample's coarse RMS
  update   Adam (Kingma and Ba 2015), bias-corrected

``bf16=True`` rounds to bfloat16 (round to nearest even) where the GPU kernels
store bfloat16: the lifted input, the weights used in products, the
post-ReLU activations, the loss gradient dL/dr and the back-propagated
pre-activation gradients.  Everything else stays FP64.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ helpers
def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32; returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def lift_matrix(R: int, img: int) -> np.ndarray:
    """P [img][R]: row i holds the corner-aligned linear weights of node i."""
    P = np.zeros((img, R))
    for i in range(img):
        s = i * (R - 1)
        p = s // (img - 1)
        a = (s - p * (img - 1)) / (img - 1)
        P[i, p] += 1.0 - a
        if a > 0.0:
            P[i, p + 1] += a
    return P


def lift(S: np.ndarray, img: int) -> np.ndarray:
    """Bilinear lift of grids [..., R(v), R(u)] to [..., img, img]."""
    P = lift_matrix(S.shape[-1], img)
    return P @ S @ P.T


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray | None) -> np.ndarray:
    """x [B][Ci][H][W], W [Co][Ci][3][3] -> [B][Co][H][W] (zero padding)."""
    B, Ci, H, Wd = x.shape
    xp = np.zeros((B, Ci, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((B, W.shape[0], H, Wd))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + H, kx:kx + Wd]                      # [B][Ci][H][W]
            out += np.einsum("bihw,oi->bohw", patch, W[:, :, ky, kx])
    if b is not None:
        out += b[None, :, None, None]
    return out


def conv3x3_input_grad(dz: np.ndarray, W: np.ndarray) -> np.ndarray:
    """d/dx of sum(dz * conv3x3(x; W)): dz [B][Co][H][W] -> [B][Ci][H][W]."""
    B, Co, H, Wd = dz.shape
    dxp = np.zeros((B, W.shape[1], H + 2, Wd + 2))
    for ky in range(3):
        for kx in range(3):
            dxp[:, :, ky:ky + H, kx:kx + Wd] += np.einsum("bohw,oi->bihw", dz, W[:, :, ky, kx])
    return dxp[:, :, 1:-1, 1:-1]


def conv3x3_weight_grad(x: np.ndarray, dz: np.ndarray):
    """d/dW and d/db of sum(dz * conv3x3(x; W, b))."""
    B, Ci, H, Wd = x.shape
    xp = np.zeros((B, Ci, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dW = np.zeros((dz.shape[1], Ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.einsum("bohw,bihw->oi", dz, xp[:, :, ky:ky + H, kx:kx + Wd])
    return dW, dz.sum(axis=(0, 2, 3))


# ------------------------------------------------------------------ parameters
def split(params: np.ndarray, hidden: int = 64, n_in: int = 15, n_out: int = 3):
    """(W1, b1, W2, b2, W3, b3) views of the flat FP64 parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for co, ci in ((hidden, n_in), (hidden, hidden), (n_out, hidden)):
        out.append(p[o:o + co * ci * 9].reshape(co, ci, 3, 3))
        o += co * ci * 9
        out.append(p[o:o + co])
        o += co
    if o != p.size:
        raise ValueError("parameter vector length does not match the layer sizes")
    return tuple(out)


def join(parts) -> np.ndarray:
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in parts])


# ------------------------------------------------------------------ network
def second_difference(S: np.ndarray, axis: int) -> np.ndarray:
    """Coarse second difference along `axis` (-1 = u, -2 = v); the edge nodes
    take the value of the next node inward (zero for fewer than 3 nodes)."""
    n = S.shape[axis]
    if n < 3:
        return np.zeros_like(S)
    Sm = np.moveaxis(S, axis, -1)
    d = Sm[..., 2:] - 2.0 * Sm[..., 1:-1] + Sm[..., :-2]            # nodes 1 .. n-2
    d = np.concatenate([d[..., :1], d, d[..., -1:]], axis=-1)
    return np.moveaxis(d, -1, axis)


def cell_phase(R: int, img: int) -> np.ndarray:
    """4 a (1 - a) per fine node, a = fractional position in its coarse cell."""
    a = np.array([(i * (R - 1) - (i * (R - 1) // (img - 1)) * (img - 1)) / (img - 1) for i in range(img)])
    return 4.0 * a * (1.0 - a)


def lift_input(coarse: np.ndarray, theta: np.ndarray, img: int):
    """coarse [B][4][3][R][R], theta [B] -> (x0 [B][15][img][img], base [B][3][img][img], s [B])."""
    c = np.asarray(coarse, dtype=np.float64)
    B, R = c.shape[0], c.shape[-1]
    s = np.sqrt(np.mean(c.reshape(B, -1) ** 2, axis=1))
    s = np.where(s > 0.0, s, 1.0)
    th = np.asarray(theta, dtype=np.float64)[:, None, None, None]
    Sb = (1.0 - th) * c[:, 1] + th * c[:, 2]                          # [B][3][R][R]
    feats = [Sb, second_difference(Sb, -1), second_difference(Sb, -2),
             (c[:, 3] - c[:, 2]) - (c[:, 1] - c[:, 0])]
    L = [lift(f, img) for f in feats]                                 # 4 x [B][3][img][img]
    ph = cell_phase(R, img)
    sc = s[:, None, None, None]
    x0 = np.concatenate([L[0] / sc, L[1] / sc, L[2] / sc, L[3] / sc,
                         np.broadcast_to(th, (B, 1, img, img)),
                         np.broadcast_to(ph[None, None, None, :], (B, 1, img, img)),
                         np.broadcast_to(ph[None, None, :, None], (B, 1, img, img))], axis=1)
    return x0, L[0], s


def forward(params, coarse, theta, img: int = 64, hidden: int = 64, bf: bool = False) -> dict:
    """All intermediates of the forward pass (channels-first)."""
    W1, b1, W2, b2, W3, b3 = split(params, hidden)
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    x0, base, s = lift_input(coarse, theta, img)
    x0 = rnd(x0)
    z1 = conv3x3(x0, rnd(W1), b1)
    a1 = rnd(np.maximum(z1, 0.0))
    z2 = conv3x3(a1, rnd(W2), b2)
    a2 = rnd(np.maximum(z2, 0.0))
    r = conv3x3(a2, rnd(W3), b3)
    u = base + s[:, None, None, None] * r
    return dict(x0=x0, z1=z1, a1=a1, z2=z2, a2=a2, r=r, base=base, s=s, u=u)


def loss(u: np.ndarray, truth_chw: np.ndarray, s: np.ndarray) -> float:
    return float(np.mean(((u - truth_chw) / s[:, None, None, None]) ** 2))


def loss_grad(params, coarse, theta, truth, img: int = 64, hidden: int = 64, bf: bool = False):
    """(loss, gradient vector, forward cache); truth [B][img][img][3] (NHWC as stored)."""
    W1, b1, W2, b2, W3, b3 = split(params, hidden)
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    fw = forward(params, coarse, theta, img, hidden, bf)
    t = np.asarray(truth, dtype=np.float64).transpose(0, 3, 1, 2)
    e = (fw["u"] - t) / fw["s"][:, None, None, None]
    L = float(np.mean(e ** 2))
    dr = rnd(2.0 * e / e.size)
    dW3, db3 = conv3x3_weight_grad(fw["a2"], dr)
    dz2 = rnd(conv3x3_input_grad(dr, rnd(W3)) * (fw["z2"] > 0.0))
    dW2, db2 = conv3x3_weight_grad(fw["a1"], dz2)
    dz1 = rnd(conv3x3_input_grad(dz2, rnd(W2)) * (fw["z1"] > 0.0))
    dW1, db1 = conv3x3_weight_grad(fw["x0"], dz1)
    return L, join((dW1, db1, dW2, db2, dW3, db3)), fw


def adam(params, grad, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t = 1 for the first); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    p = params - lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return p, m, v


def baseline(coarse, theta, img: int = 64) -> np.ndarray:
    """The plain interpolation the network corrects, NHWC [B][img][img][3]."""
    _, base, _ = lift_input(coarse, theta, img)
    return base.transpose(0, 2, 3, 1)
