"""Pins of the oracle's vorticity (the paper's validation observable, Sec. 3,
Figs. 1-2: |omega| = |curl u| averaged over a control volume), checked against
what the mathematics fixes rather than against itself:

* central differences are exact on fields quadratic in the coordinates, so an
  affine field gives its constant curl (A32 - A23, A13 - A31, A21 - A12), a
  rigid rotation Omega x r gives 2 Omega, and a quadratic field its curl
  evaluated at each node;
* on a periodic shear wave u_x = U sin(2 pi y / N) the central difference is
  -U cos(2 pi y / N) sin(2 pi / N) exactly (difference of sines);
* on a random field, numpy's own central-difference gradient gives the curl;
* the field is zero where a node's neighbours are not all interior, and the
  control-volume mean is the mean of the field over the volume.

The velocity is recovered from equilibrium populations set from u, so u = j/rho
is the prescribed field up to rounding.
"""
import numpy as np
import pytest

import oracle


def box_with(u, dims, pmask=0):
    ob = oracle.OracleBox(dims, collision=oracle.MRT, tau=0.7, tau_bulk=0.7, periodic_mask=pmask)
    ob.set_initial(u)
    return ob


def coords(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


def defined_mask(dims, pmask=0):
    m = np.ones(dims[::-1], dtype=bool)
    for a in range(3):
        if (pmask >> a) & 1:
            continue
        n = dims[a]
        sl = [slice(None)] * 3
        for v in (0, 1, n - 2, n - 1):
            sl[2 - a] = v
            m[tuple(sl)] = False
    return m


def test_affine_field_constant_curl():
    dims = (9, 11, 10)
    rng = np.random.default_rng(1)
    A = 1e-3 * rng.standard_normal((3, 3))
    x, y, z = coords(dims)
    r = np.stack([x - 4, y - 5, z - 4.5], -1)
    u = r @ A.T
    ob = box_with(u, dims)
    w, n = ob.vorticity()
    want = np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    m = defined_mask(dims)
    assert n == m.sum() == 5 * 7 * 6
    assert np.all(w[~m] == 0)
    assert np.abs(w[m] - want).max() < 1e-12 * want


def test_rigid_rotation_gives_twice_the_rate():
    dims = (10, 10, 10)
    om = np.array([2e-4, -3e-4, 5e-4])
    x, y, z = coords(dims)
    r = np.stack([x - 4.5, y - 4.5, z - 4.5], -1)
    u = np.cross(om[None, None, None, :], r)
    ob = box_with(u, dims)
    w, _ = ob.vorticity()
    m = defined_mask(dims)
    assert np.abs(w[m] - 2 * np.linalg.norm(om)).max() < 1e-12 * np.linalg.norm(om)


def test_quadratic_field_exact():
    """u = (a y z + b y^2, c x z, d x y + e x^2): curl = (d x - c x, a y - d y - 2 e x,
    c z - a z - 2 b y) at every node, which central differences reproduce."""
    dims = (8, 9, 7)
    a, b, c, d, e = 1e-5, -2e-5, 3e-5, -1e-5, 2e-5
    x, y, z = coords(dims)
    x, y, z = x - 3.5, y - 4.0, z - 3.0
    u = np.stack([a * y * z + b * y * y, c * x * z, d * x * y + e * x * x], -1)
    ob = box_with(u, dims)
    w, _ = ob.vorticity()
    wx = d * x - c * x
    wy = a * y - d * y - 2 * e * x
    wz = c * z - a * z - 2 * b * y
    want = np.sqrt(wx ** 2 + wy ** 2 + wz ** 2)
    m = defined_mask(dims)
    assert np.abs(w[m] - want[m]).max() < 1e-12 * np.abs(want[m]).max()


def test_periodic_shear_wave_closed_form():
    dims = (6, 16, 5)
    U = 1e-4
    x, y, z = coords(dims)
    u = np.zeros(dims[::-1] + (3,))
    u[..., 0] = U * np.sin(2 * np.pi * y / dims[1])
    ob = box_with(u, dims, pmask=7)
    w, n = ob.vorticity()
    assert n == np.prod(dims)
    want = np.abs(U * np.cos(2 * np.pi * y / dims[1]) * np.sin(2 * np.pi / dims[1]))
    assert np.abs(w - want).max() < 1e-12 * U


def test_random_field_matches_numpy_gradient_curl():
    dims = (9, 8, 10)
    rng = np.random.default_rng(4)
    u = 1e-3 * rng.standard_normal(dims[::-1] + (3,))
    ob = box_with(u, dims)
    _, uo = ob.rho_u()
    # np.gradient: central differences in the interior; axes (z, y, x) of the array
    d = {(c, a): np.gradient(uo[..., c], axis=2 - a) for c in range(3) for a in range(3)}
    want = np.sqrt((d[2, 1] - d[1, 2]) ** 2 + (d[0, 2] - d[2, 0]) ** 2 + (d[1, 0] - d[0, 1]) ** 2)
    w, _ = ob.vorticity()
    m = defined_mask(dims)
    assert np.abs(w[m] - want[m]).max() < 1e-12 * want[m].max()


def test_control_volume_mean():
    dims = (12, 12, 12)
    rng = np.random.default_rng(6)
    ob = box_with(1e-3 * rng.standard_normal(dims[::-1] + (3,)), dims)
    w, _ = ob.vorticity()
    lo, hi = (3, 2, 4), (8, 9, 6)
    mean = ob.vorticity_mean(lo, hi)
    assert mean == pytest.approx(w[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1].mean(), rel=1e-14)
    with pytest.raises(ValueError):
        ob.vorticity_mean((1, 2, 2), (5, 5, 5))
