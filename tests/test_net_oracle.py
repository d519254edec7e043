"""Pins of the FP64 upsampler oracle against what mathematics fixes: a library
cross-correlation, exactness of the bilinear lift on affine fields, central
finite differences of the loss, the closed form of Adam's first step, and
bfloat16 rounding on exactly representable cases."""
import numpy as np
import pytest
import scipy.signal

from oracle import net_oracle as no


def rng(i):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=0x08094958, spawn_key=(77, i))))


def test_conv3x3_is_the_library_cross_correlation():
    g = rng(0)
    x = g.standard_normal((2, 3, 7, 9))
    W = g.standard_normal((4, 3, 3, 3))
    b = g.standard_normal(4)
    out = no.conv3x3(x, W, b)
    ref = np.zeros_like(out)
    for n in range(2):
        for co in range(4):
            ref[n, co] = b[co] + sum(scipy.signal.correlate2d(x[n, ci], W[co, ci], mode="same",
                                                              boundary="fill") for ci in range(3))
    assert np.max(np.abs(out - ref)) < 1e-12


@pytest.mark.parametrize("R,img", [(8, 64), (3, 10), (5, 17)])
def test_lift_exact_on_affine_fields_and_at_coinciding_nodes(R, img):
    g = rng(1)
    a, bu, bv = g.standard_normal(3)
    pu = np.arange(R) * (img - 1) / (R - 1)
    S = a + bu * pu[None, :] + bv * pu[:, None]          # [v][u] on the coarse grid
    L = no.lift(S, img)
    y = np.arange(img)
    assert np.max(np.abs(L - (a + bu * y[None, :] + bv * y[:, None]))) < 1e-12
    if (img - 1) % (R - 1) == 0:
        step = (img - 1) // (R - 1)
        T = g.standard_normal((R, R))
        assert np.max(np.abs(no.lift(T, img)[::step, ::step] - T)) < 1e-14


def test_lift_matrix_rows_are_partitions_of_unity():
    P = no.lift_matrix(8, 64)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
    assert (P >= 0).all() and (np.count_nonzero(P, axis=1) <= 2).all()


def test_base_is_the_linear_time_interpolation():
    g = rng(2)
    c = g.standard_normal((3, 4, 3, 4, 4))
    th = np.array([0.0, 0.25, 1.0])
    base = no.baseline(c, th, img=7)
    Lk = no.lift(c[:, 1], 7).transpose(0, 2, 3, 1)
    Lk1 = no.lift(c[:, 2], 7).transpose(0, 2, 3, 1)
    assert np.allclose(base[0], Lk[0], atol=1e-14)
    assert np.allclose(base[2], Lk1[2], atol=1e-14)
    assert np.allclose(base[1], 0.75 * Lk[1] + 0.25 * Lk1[1], atol=1e-14)


def test_loss_gradient_matches_central_differences():
    g = rng(3)
    hidden, img, R, B = 3, 6, 3, 2
    n = hidden * 15 * 9 + hidden + hidden * hidden * 9 + hidden + 3 * hidden * 9 + 3
    p = g.standard_normal(n) * 0.3
    c = g.standard_normal((B, 4, 3, R, R))
    th = np.array([0.1, 0.7])
    truth = g.standard_normal((B, img, img, 3))
    L, grad, _ = no.loss_grad(p, c, th, truth, img=img, hidden=hidden)
    h = 1e-6
    fd = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        lp = no.loss_grad(p + e, c, th, truth, img=img, hidden=hidden)[0]
        lm = no.loss_grad(p - e, c, th, truth, img=img, hidden=hidden)[0]
        fd[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(grad - fd) / np.linalg.norm(fd) < 1e-7
    # every parameter block carries gradient (no dropped term)
    for blk in no.split(grad, hidden):
        assert np.linalg.norm(blk) > 0


def test_input_gradient_is_the_adjoint_of_the_convolution():
    g = rng(4)
    x = g.standard_normal((2, 3, 5, 6))
    W = g.standard_normal((4, 3, 3, 3))
    dz = g.standard_normal((2, 4, 5, 6))
    lhs = np.sum(dz * no.conv3x3(x, W, None))
    rhs = np.sum(no.conv3x3_input_grad(dz, W) * x)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_adam_first_step_closed_form():
    g = rng(5)
    p = g.standard_normal(10)
    grad = g.standard_normal(10)
    p1, m, v = no.adam(p, grad, np.zeros(10), np.zeros(10), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, p - 0.01 * grad / (np.abs(grad) + 1e-8), atol=1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad * grad)


def test_bf16_rounding_nearest_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e38, 1e-40])
    r = no.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0                 # tie to even
    assert r[2] == 1 + 2 ** -6                         # tie to even (upward)
    assert r[3] == 1 + 2 ** -7 and r[4] == -2.5
    assert abs(r[5] - 3.0e38) / 3.0e38 < 2 ** -8
    assert abs(no.bf16(np.pi) - np.pi) < np.pi * 2 ** -8


def test_zero_last_layer_reproduces_the_interpolation():
    g = rng(6)
    hidden, img = 4, 9
    n = hidden * 15 * 9 + hidden + hidden * hidden * 9 + hidden + 3 * hidden * 9 + 3
    p = g.standard_normal(n)
    W1, b1, W2, b2, W3, b3 = no.split(p, hidden)
    W3[:] = 0.0
    b3[:] = 0.0
    c = g.standard_normal((2, 4, 3, 3, 3))
    th = np.array([0.3, 0.9])
    fw = no.forward(p, c, th, img=img, hidden=hidden)
    assert np.allclose(fw["u"].transpose(0, 2, 3, 1), no.baseline(c, th, img), atol=1e-15)


def test_second_difference_and_cell_phase():
    # a quadratic along u has the constant second difference 2 a h^2 (h = 1 on
    # the coarse grid), also at the edge nodes
    u = np.arange(6.0)
    S = np.broadcast_to(3.0 * u ** 2 + u, (4, 6)).copy()
    assert np.allclose(no.second_difference(S, -1), 6.0, atol=1e-12)
    assert np.allclose(no.second_difference(S, -2), 0.0, atol=1e-12)
    ph = no.cell_phase(8, 64)
    assert ph[0] == 0.0 and ph[63] == 0.0 and ph[9] == 0.0      # nodes on coarse points
    assert abs(ph[4] - 4 * (4 / 9) * (5 / 9)) < 1e-15             # 4 nodes into a 9-node cell


def test_corrected_lift_is_exact_for_quadratics():
    """The features carry what the interpolation misses: for a field quadratic
    in u and v the exact value is L(S) - (h^2/2) a(1-a) S_uu - (h^2/2) b(1-b) S_vv,
    i.e. L(S) - 1/8 (4a(1-a)) L(Duu S) - 1/8 (4b(1-b)) L(Dvv S) in coarse units."""
    R, img = 8, 64
    q = np.arange(R) * 1.0
    S = 0.3 * q[None, :] ** 2 - 0.2 * q[:, None] ** 2 + 0.1 * q[None, :] * q[:, None] + 1.0
    c = np.broadcast_to(S, (1, 4, 3, R, R)).copy()
    x0, base, s = no.lift_input(c, np.array([0.0]), img)
    y = np.arange(img) * (R - 1) / (img - 1)
    exact = 0.3 * y[None, :] ** 2 - 0.2 * y[:, None] ** 2 + 0.1 * y[None, :] * y[:, None] + 1.0
    corr = (x0[0, 0] - x0[0, 3] * x0[0, 13] / 8.0 - x0[0, 6] * x0[0, 14] / 8.0) * s[0]
    assert np.max(np.abs(corr - exact)) < 1e-12
    assert np.max(np.abs(base[0, 0] - exact)) > 1e-3             # the interpolation alone misses it

