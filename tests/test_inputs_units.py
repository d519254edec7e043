"""Synthetic inputs and the reduced-unit matching of Eq. (1), pinned to the
paper's printed numbers (tests/golden/paper_numbers.json, Sec. 3)."""
import json
import math
import os

import numpy as np

from paper_0809_4958_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def g(key):
    return GOLD[key]["value"]


def test_dns_closed_forms_match_printed_values():
    nu, eps = g("dns_nu"), g("dns_eps")
    eta = nu ** 0.75 * eps ** -0.25
    tau_eta = math.sqrt(nu / eps)
    assert abs(eta - g("dns_eta")) / g("dns_eta") < 0.005
    assert abs(tau_eta - g("dns_tau_eta")) / g("dns_tau_eta") < 0.005
    # R_lambda = sqrt(5/(3 eps nu)) u_rms^2 and Re = u_rms L / nu, L = 2 pi
    u_rms = math.sqrt(g("dns_R_lambda") / math.sqrt(5 / (3 * eps * nu)))
    assert abs(u_rms * 2 * math.pi / nu - g("dns_Re")) / g("dns_Re") < 0.001
    # eta / Delta with Delta = 2 pi / M: 3.240 computed vs 3.26 printed (0.6 %)
    delta = 2 * math.pi / g("dns_M")
    assert abs(eta / delta - g("dns_eta_over_delta")) / g("dns_eta_over_delta") < 0.01
    # (20 Delta)^3 ~ (6 eta)^3
    assert abs(g("subvolume_points") / g("dns_eta_over_delta") - g("subvolume_eta")) < 0.2


def test_mach_number_of_the_case_study():
    """Ma = eta~/(tau~_eta c_s) with eta~ = 3.26 z, tau~_eta = eta~^2/nu~; the
    printed 1.49e-2 is reproduced within 1 % by nu~ = 1/6 (tau = 1)."""
    ma = inputs.paper_mach(g("zoom"), g("dns_eta_over_delta"), 1 / 6)
    assert abs(ma - g("mach")) / g("mach") < 0.01
    # the same through UnitMap: a box of 3.26 z + 1 nodes spanning one eta
    um = inputs.UnitMap(n=int(round(g("dns_eta_over_delta") * g("zoom") * 100)) + 1, tau=1.0,
                        width_eta=100.0)
    assert abs(um.mach() - ma) / ma < 1e-3
    # LB box (120 a) = z * 20 Delta
    assert g("zoom") * g("subvolume_points") == g("lb_box_cells")


def test_unit_map_is_eq1():
    um = inputs.UnitMap(n=129, tau=0.6, width_eta=2.0)
    assert um.eta == 64.0
    assert abs(um.nu - 0.1 / 3) < 1e-16
    assert abs(um.tau_eta - 64.0 ** 2 / um.nu) < 1e-9
    # reduced velocity w~ tau~_eta / eta~ equals w tau_eta / eta = w (Kolmogorov units)
    w = 0.37
    assert abs(w * um.u_scale * um.tau_eta / um.eta - w) < 1e-15


def test_ks_field_divergence_free_and_normalised():
    ks = inputs.KSField(inputs.rng(1, 0))
    x = np.random.default_rng(0).uniform(-5, 5, size=(50, 3))
    grad = ks.gradient(x, 0.3)
    assert np.abs(np.trace(grad, axis1=-2, axis2=-1)).max() < 1e-12
    # mean squared gradient is 1 in Kolmogorov units (ensemble over modes)
    assert abs(np.sum(ks.kmag ** 2 * ks.E * ks.dk) - 1) < 1e-12
    # the tensor-grid evaluation equals the direct one
    axes = [np.linspace(-1, 1, 4), np.linspace(-0.5, 1, 3), np.linspace(0, 1, 2)]
    x0 = np.array([1.0, 2.0, -3.0])
    gv = ks.grid_velocity(x0, 0.7, axes)
    for iz, zz in enumerate(axes[2]):
        for iy, yy in enumerate(axes[1]):
            for ix, xx in enumerate(axes[0]):
                d = ks.velocity(x0 + np.array([xx, yy, zz]), 0.7)
                assert np.abs(gv[iz, iy, ix] - d).max() < 1e-12


def test_tracer_frame_field_vanishes_at_box_centre():
    """w = u - v(t) is zero at the tracer, the box centre (Sec. 2)."""
    units, u0, faces = inputs.ks_box_inputs(1, 0, n=17, tau=0.6, n_steps=40, dt=20, res=5)
    c = 8
    assert np.abs(u0[c, c, c]).max() < 1e-15
    assert faces.shape == (3, 6, 5, 5, 3)
    # faces at t = 0 equal the initial field on the face nodes (corner-aligned grid)
    assert np.abs(faces[0, 0, :, :, :] - u0[::4, ::4, 0, :]).max() < 1e-15
    assert np.abs(faces[0, 5, :, :, :] - u0[16, ::4, ::4, :]).max() < 1e-15
    assert np.abs(faces[0, 3, :, :, :] - u0[::4, 16, ::4, :]).max() < 1e-15


def test_tracer_rk4_converges():
    ks = inputs.KSField(inputs.rng(5, 0), n_modes=50)
    t = np.array([0.0, 0.5, 1.0])
    a = inputs.tracer_path(ks, np.zeros(3), t, h_max=0.05).pos
    b = inputs.tracer_path(ks, np.zeros(3), t, h_max=0.025).pos
    c = inputs.tracer_path(ks, np.zeros(3), t, h_max=0.0125).pos
    assert np.abs(b - c).max() < np.abs(a - b).max() / 8


def test_ou_strain_statistics():
    A = inputs.ou_strain(200000, inputs.rng(0, 0), corr_steps=50.0, rms=1e-3).reshape(-1, 3, 3)
    assert np.abs(np.trace(A, axis1=1, axis2=2)).max() < 1e-17
    rms = math.sqrt(np.mean(A ** 2))
    assert abs(rms - 1e-3) / 1e-3 < 0.03
    # lag-50 autocorrelation e^-1
    x = A[:, 0, 1]
    r = np.mean(x[50:] * x[:-50]) / np.mean(x * x)
    assert abs(r - math.exp(-1)) < 0.05


def test_chain_init_com_and_bonds():
    pos, vel = inputs.chain_init(32, [10.0, 11.0, 12.0], inputs.rng(2, 2))
    assert np.abs(pos.mean(axis=0) - [10, 11, 12]).max() < 1e-13
    assert np.abs(np.linalg.norm(np.diff(pos, axis=0), axis=1) - 1).max() < 1e-13
    assert not vel.any()


def test_box_sizes_uniform_choices():
    n = inputs.box_sizes(256, inputs.rng(2, 3))
    assert set(np.unique(n)) <= {32, 48, 64, 96}
    assert len(n) == 256


def test_ks_grid_vorticity_is_the_curl_of_the_analytic_gradient():
    """The tensor-grid vorticity of the KS field equals the curl taken from the
    field's analytic velocity gradient at the same points."""
    import numpy as np

    from paper_0809_4958_amd import inputs
    ks, x0 = inputs.ks_tracer(3, 1, n_modes=40)
    axes = [np.linspace(-0.5, 0.7, 4), np.linspace(-0.3, 0.2, 3), np.linspace(0.1, 0.9, 5)]
    w = ks.grid_vorticity(x0, 1.3, axes)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    pts = x0 + np.stack([x, y, z], -1)
    g = ks.gradient(pts, 1.3)  # [..., i, j] = du_i/dx_j
    curl = np.stack([g[..., 2, 1] - g[..., 1, 2], g[..., 0, 2] - g[..., 2, 0],
                     g[..., 1, 0] - g[..., 0, 1]], -1)
    assert np.abs(w - curl).max() < 1e-12 * np.abs(curl).max()
    # and the refactored per-box inputs still follow the same seeds
    ks2, x2 = inputs.ks_tracer(3, 1, n_modes=40)
    assert np.array_equal(ks2.k, ks.k) and np.array_equal(x2, x0)


def test_subvolume_writer_format(tmp_path):
    """The history file holds the documented header and arrays, bit for bit."""
    import os

    import numpy as np

    from paper_0809_4958_amd import inputs
    rng = np.random.default_rng(1)
    w = rng.standard_normal((3, 4, 4, 4, 3))
    acc = rng.standard_normal((3, 3))
    p = os.path.join(tmp_path, "h.lbsv")
    inputs.write_subvolume(p, w, dt=7, t0=-5, accel=acc)
    raw = open(p, "rb").read()
    assert raw[:8] == b"LBSUBVOL"
    hdr = np.frombuffer(raw[8:24], dtype="<i4")
    assert list(hdr) == [1, 4, 3, 7]
    assert np.frombuffer(raw[24:32], dtype="<i8")[0] == -5
    assert list(np.frombuffer(raw[32:40], dtype="<i4")) == [1, 0]
    nw = w.size * 4
    assert np.array_equal(np.frombuffer(raw[40:40 + nw], dtype="<f4").reshape(w.shape),
                          w.astype(np.float32))
    assert np.array_equal(np.frombuffer(raw[40 + nw:], dtype="<f8").reshape(3, 3), acc)


def test_tracer_acceleration_is_the_derivative_of_its_velocity():
    """The Lagrangian acceleration du/dt + (u . grad) u at the tracer equals the
    time derivative of the tracer's own velocity (central differences)."""
    import numpy as np

    from paper_0809_4958_amd import inputs
    ks, x0 = inputs.ks_tracer(2, 3, n_modes=60)
    # the central difference converges as h^2 (1.1e-5 relative at h = 1e-3)
    h = 1e-4
    tr = inputs.tracer_path(ks, x0, np.array([0.5 - h, 0.5, 0.5 + h]), h_max=1e-4)
    a = inputs.tracer_acceleration(ks, tr)[1]
    fd = (tr.vel[2] - tr.vel[0]) / (2 * h)
    assert np.abs(a - fd).max() < 1e-6 * np.abs(a).max()
