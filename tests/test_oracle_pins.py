"""Pins of the FP64 oracle against what lattice-Boltzmann theory and the paper fix.

None of these re-types the oracle's formulas: each checks a consequence
(isotropy, conservation, a closed-form flow, a linear-stability eigenvalue,
an independent brute-force implementation, an exact ODE solution).
"""
import math

import numpy as np
import pytest

import oracle
from brute_lb import BruteBox
from paper_0809_4958_amd import inputs


# ----------------------------------------------------------------- lattice
def test_lattice_isotropy():
    """D3Q19 weights and velocities: moments up to fourth order are isotropic (Sec. 3)."""
    c, w = oracle.lattice()
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-15
    assert np.abs(np.einsum('i,ia,ib->ab', w, c, c) - d / 3).max() < 1e-15
    m3 = np.einsum('i,ia,ib,ic->abc', w, c, c, c)
    assert np.abs(m3).max() < 1e-15
    m4 = np.einsum('i,ia,ib,ic,id->abcd', w, c, c, c, c)
    iso = (np.einsum('ab,cd->abcd', d, d) + np.einsum('ac,bd->abcd', d, d)
           + np.einsum('ad,bc->abcd', d, d)) / 9
    assert np.abs(m4 - iso).max() < 1e-15
    # 19 distinct velocities, |c|^2 <= 2, opposite directions adjacent
    assert len({tuple(v) for v in c}) == 19
    for i in range(1, 19, 2):
        assert np.all(c[i] == -c[i + 1])


def test_equilibrium_moments():
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        feq = oracle.equilibrium(rho, u)
        c, _ = oracle.lattice()
        assert abs(feq.sum() - rho) < 1e-14
        assert np.abs(feq @ c - rho * u).max() < 1e-15
        pi = np.einsum('i,ia,ib->ab', feq, c, c)
        assert np.abs(pi - (rho / 3 * np.eye(3) + rho * np.outer(u, u))).max() < 1e-14


def test_mrt_basis_weighted_orthogonal():
    c, w = oracle.lattice()
    e, b = oracle.mrt_basis()
    gram = e @ np.diag(w) @ e.T
    assert np.abs(gram - np.diag(b)).max() < 1e-15
    # first rows span the conserved and stress moments
    assert np.all(e[0] == 1)
    assert np.all(e[1:4] == c.T)


@pytest.mark.parametrize("coll", [oracle.BGK, oracle.MRT])
def test_collision_invariants(coll):
    """Sum f* = sum f and sum c f* = j + g (mass conserved, momentum gains g)."""
    rng = np.random.default_rng(4)
    c, _ = oracle.lattice()
    for _ in range(20):
        f = oracle.equilibrium(1.0, 0.03 * rng.standard_normal(3)) + 1e-3 * rng.standard_normal(19)
        g = 1e-3 * rng.standard_normal(3)
        out = oracle.collide(f, g, collision=coll, tau=0.6 + rng.random(), tau_bulk=0.7,
                             ghost_rate=1.2)
        assert abs(out.sum() - f.sum()) < 1e-15
        assert np.abs(out @ c - (f @ c + g)).max() < 1e-16


def test_mrt_equals_bgk_when_all_rates_equal():
    rng = np.random.default_rng(5)
    for tau in (0.55, 0.8, 1.7):
        f = oracle.equilibrium(1.02, 0.03 * rng.standard_normal(3)) + 1e-3 * rng.standard_normal(19)
        g = 1e-3 * rng.standard_normal(3)
        a = oracle.collide(f, g, collision=oracle.BGK, tau=tau)
        b = oracle.collide(f, g, collision=oracle.MRT, tau=tau, tau_bulk=tau, ghost_rate=1 / tau)
        assert np.abs(a - b).max() < 1e-15


# ------------------------------------------------- linear hydrodynamics
def _linear_operator(k, **kw):
    """Per-step linear evolution L(k) of a Fourier mode about rest (numerical
    Jacobian of the oracle's collision, then streaming phase)."""
    c, w = oracle.lattice()
    f0 = oracle.equilibrium(1.0, [0, 0, 0])
    jac = np.zeros((19, 19))
    eps = 1e-6
    for j in range(19):
        d = np.zeros(19)
        d[j] = eps
        jac[:, j] = (oracle.collide(f0 + d, **kw) - oracle.collide(f0 - d, **kw)) / (2 * eps)
    phase = np.exp(-1j * (c @ k))
    return np.diag(phase) @ jac


@pytest.mark.parametrize("coll,tau,tau_b", [(oracle.BGK, 0.8, 0.8), (oracle.MRT, 0.6, 0.6),
                                            (oracle.MRT, 0.7, 1.4)])
def test_shear_and_sound_damping_match_viscosities(coll, tau, tau_b):
    """Hydrodynamic eigenvalues of the linear LB operator at small k:
    shear |lambda| = exp(-nu k^2), nu = (tau - 1/2)/3; sound damping
    Gamma = k^2 (4 nu/3 + nu_b)/2 with nu_b = (2/9)(tau_b - 1/2)."""
    nu = (tau - 0.5) / 3
    nu_b = 2 / 9 * (tau_b - 0.5)
    for N in (64, 128):
        kk = 2 * np.pi / N
        lam = np.linalg.eigvals(_linear_operator(np.array([kk, 0, 0]), collision=coll, tau=tau,
                                                 tau_bulk=tau_b, ghost_rate=1.0))
        rate = -np.log(np.abs(lam))
        # two shear modes: real eigenvalues with rate ~ nu k^2
        shear = sorted(rate[(np.abs(lam.imag) < 1e-12) & (np.abs(lam) > 0.5)])[:2]
        assert np.allclose(shear, nu * kk * kk, rtol=0.02 * (64 / N) ** 2 + 1e-3)
        # sound pair: frequency ~ c_s k
        snd = rate[(np.abs(lam) > 0.5) & (np.abs(np.abs(np.angle(lam)) - kk / math.sqrt(3)) < 0.1 * kk)]
        assert len(snd) == 2
        gam = kk * kk * (4 * nu / 3 + nu_b) / 2
        assert np.allclose(snd, gam, rtol=0.03 * (64 / N) ** 2 + 1e-3)


def test_shear_wave_decays_at_eigenvalue():
    """Full periodic lattice run: a shear wave decays per step by the shear
    eigenvalue of the linear operator and, to O(k^2), by exp(-nu k^2)."""
    N, tau = 32, 0.8
    ob = oracle.OracleBox((4, N, 4), collision=oracle.BGK, tau=tau, periodic_mask=7)
    y = np.arange(N)
    u = np.zeros((4, N, 4, 3))
    u[..., 0] = 1e-8 * np.sin(2 * np.pi * y / N)[None, :, None]
    ob.set_initial(u)
    amp = []
    for _ in range(6):
        ob.step(50)
        _, uu = ob.rho_u()
        amp.append(np.sum(uu[0, :, 0, 0] * np.sin(2 * np.pi * y / N)))
    ratio = (amp[-1] / amp[-2]) ** (1 / 50)
    kk = 2 * np.pi / N
    lam = np.linalg.eigvals(_linear_operator(np.array([0, kk, 0]), collision=oracle.BGK, tau=tau))
    lam_shear = np.max(np.abs(lam[np.abs(lam.imag) < 1e-12]))
    assert abs(ratio - lam_shear) < 1e-9
    assert abs(ratio - math.exp(-(tau - 0.5) / 3 * kk * kk)) < 2e-5


# ------------------------------------------------------- closed forms
@pytest.mark.parametrize("coll,tau,ghost", [(oracle.BGK, 0.8, 1.0), (oracle.MRT, 0.6, 1.0),
                                            (oracle.MRT, 1.3, 1 / 1.3)])
def test_couette_closed_form(coll, tau, ghost):
    """Equilibrium-set walls at y = 0 and N-1 moving with u_x = s (y - y_c):
    the steady interior is exactly linear with slope s (N-1)/(N-3+2 tau)
    (the equilibrium wall acts at distance 1 - tau from the wall node)."""
    N, s = 12, 1e-3
    ob = oracle.OracleBox((1, N, 1), collision=coll, tau=tau, tau_bulk=tau, ghost_rate=ghost,
                          periodic_mask=5)
    A = np.zeros((2, 9))
    A[:, 1] = s
    ob.set_boundary(oracle.BC_AFFINE, A, t0=0, dt=30000)
    assert ob.step(30000) == 0
    _, u = ob.rho_u()
    yc = (N - 1) / 2
    y = np.arange(1, N - 1)
    pred = s * (N - 1) / (N - 3 + 2 * tau) * (y - yc)
    assert np.abs(u[0, 1:N - 1, 0, 0] - pred).max() < 1e-11 * np.abs(pred).max()
    assert np.abs(u[0, 1:N - 1, 0, 1:]).max() < 1e-14


def test_uniform_flow_and_rest_are_fixed_points():
    N = 10
    U = np.array([0.01, -0.02, 0.005])
    for coll in (oracle.BGK, oracle.MRT):
        ob = oracle.OracleBox((N, N, N), collision=coll, tau=0.7)
        ob.set_initial(np.broadcast_to(U, (N, N, N, 3)))
        # sampled boundary that is U everywhere
        S = np.broadcast_to(U, (3, 6, 2, 2, 3)).copy()
        ob.set_boundary(oracle.BC_SAMPLED, S, t0=0, dt=10, res=2)
        f0 = ob.pop()
        assert ob.step(20) == 0
        assert np.abs(ob.pop() - f0).max() < 1e-15
        ob2 = oracle.OracleBox((N, N, N), collision=coll, tau=0.7)
        ob2.set_boundary(oracle.BC_AFFINE, np.zeros((21, 9)))
        r0 = ob2.pop()
        assert ob2.step(20) == 0
        assert np.abs(ob2.pop() - r0).max() < 1e-15


def test_periodic_conservation_with_chain():
    """Periodic box, chain with the centre-of-mass pin off: fluid mass and
    fluid + chain momentum are conserved to rounding."""
    N = 12
    rng = np.random.default_rng(7)
    c, _ = oracle.lattice()
    for coll in (oracle.BGK, oracle.MRT):
        ob = oracle.OracleBox((N, N, N), collision=coll, tau=0.7, periodic_mask=7)
        ob.set_initial(1e-2 * rng.standard_normal((N, N, N, 3)))
        pos, _ = inputs.chain_init(6, [5.5, 6.2, 5.1], rng)
        vel = 1e-2 * rng.standard_normal((6, 3))
        ob.add_chain(pos, vel, substeps=5, fix_com=False, zeta=3.0)

        def totals():
            f = ob.pop()
            p_fl = f.sum(axis=(1, 2, 3)) @ c
            _, v = ob.beads()
            return f.sum(), p_fl + v.sum(axis=0)
        m0, p0 = totals()
        assert ob.step(15) == 0
        m1, p1 = totals()
        assert abs(m1 - m0) < 1e-11
        assert np.abs(p1 - p0).max() < 1e-13


def _run_pair(rng, coll, per, mode, chain, N=8, steps=6):
    pm = sum(1 << a for a in range(3) if per[a])
    ob = oracle.OracleBox((N, N, N), collision=oracle.BGK if coll == 'bgk' else oracle.MRT,
                          tau=0.7, tau_bulk=0.9, ghost_rate=1.3, periodic_mask=pm)
    bb = BruteBox((N, N, N), periodic=per, collision=coll, tau=0.7, tau_bulk=0.9, ghost=1.3)
    u0 = 1e-2 * rng.standard_normal((N, N, N, 3))
    ob.set_initial(u0)
    bb.set_velocity(lambda q: list(u0[q[2], q[1], q[0]]))
    if mode == 'affine':
        A = inputs.ou_strain(steps + 1, rng, corr_steps=5, rms=1e-2)
        ob.set_boundary(oracle.BC_AFFINE, A, t0=0, dt=2)
        bb.bc = ('affine', 0, 2, A.tolist(), 0)
    elif mode == 'sampled':
        R = 3
        S = 1e-2 * rng.standard_normal((4, 6, R, R, 3))
        ob.set_boundary(oracle.BC_SAMPLED, S, t0=0, dt=2, res=R)
        bb.bc = ('sampled', 0, 2, S.tolist(), R)
    if chain:
        anc = [3.7, 3.4, 3.6]
        pos, _ = inputs.chain_init(4, anc, rng)
        vel = 1e-2 * rng.standard_normal((4, 3))
        ob.add_chain(pos, vel, substeps=3, fix_com=True, zeta=2.0, anchor=anc)
        bb.add_chain(pos, vel, 3, True, 2.0, 1.0, 1.0, 2.0, anc)
    assert ob.step(steps) == 0
    for _ in range(steps):
        bb.step()
    f = ob.pop()
    err = 0.0
    for q, v in bb.f.items():
        err = max(err, np.abs(f[:, q[2], q[1], q[0]] - np.array(v)).max())
    if chain:
        pos_o, vel_o = ob.beads()
        ch = bb.chains[0]
        err = max(err, np.abs(pos_o - np.array(ch['pos'])).max(), np.abs(vel_o - np.array(ch['vel'])).max())
    return err


@pytest.mark.parametrize("coll,per,mode,chain", [
    ('bgk', (True, True, True), None, True),
    ('mrt', (True, True, True), None, True),
    ('bgk', (False, False, False), 'affine', True),
    ('mrt', (False, False, False), 'sampled', True),
    ('mrt', (True, False, True), 'sampled', False),
    ('bgk', (False, True, False), 'affine', False),
])
def test_oracle_matches_brute_force(coll, per, mode, chain):
    rng = np.random.default_rng(11)
    assert _run_pair(rng, coll, per, mode, chain) < 1e-14


# ---------------------------------------------------------- boundary
def test_sampled_boundary_exact_on_affine_data():
    """Bilinear in space x linear in time reproduces data affine in (u, v, t)."""
    N, R, dt = 9, 4, 5
    ob = oracle.OracleBox((N, N, N), tau=0.8)
    rng = np.random.default_rng(2)
    coef = rng.standard_normal((6, 4, 3))
    S = np.zeros((3, 6, R, R, 3))
    gp = np.arange(R) * (N - 1) / (R - 1)
    for k in range(3):
        for f in range(6):
            for qv in range(R):
                for pu in range(R):
                    S[k, f, qv, pu] = coef[f, 0] + coef[f, 1] * gp[pu] + coef[f, 2] * gp[qv] + coef[f, 3] * (k * dt)
    ob.set_boundary(oracle.BC_SAMPLED, S, t0=0, dt=dt, res=R)
    axes = ((1, 2), (1, 2), (0, 2), (0, 2), (0, 1), (0, 1))
    for n in (0, 3, 7, 10):
        for q in [(0, 3, 5), (8, 2, 7), (4, 0, 3), (4, 8, 1), (3, 5, 0), (2, 6, 8), (0, 0, 4), (8, 8, 8)]:
            st, u = ob.boundary_velocity(*q, n)
            assert st == 0
            # first face in -x,+x,-y,+y,-z,+z order
            f = next(f for f in range(6) if q[f // 2] == (0 if f % 2 == 0 else N - 1))
            au, av = axes[f]
            want = coef[f, 0] + coef[f, 1] * q[au] + coef[f, 2] * q[av] + coef[f, 3] * n
            assert np.abs(u - want).max() < 1e-13


def test_stepping_past_last_sample_is_an_error():
    ob = oracle.OracleBox((6, 6, 6), tau=0.8)
    ob.set_boundary(oracle.BC_AFFINE, np.zeros((3, 9)), t0=0, dt=2)   # covers steps 0..4
    assert ob.step(5) == 0
    assert ob.step(1) == oracle.ERR_ARG
    assert ob.step_index == 5


# ------------------------------------------------------------- chain
def test_single_bead_exact_friction_solution():
    """No springs, fixed fluid velocity: V(t) = u + (V0 - u) e^{-zeta t/m}."""
    u = np.array([[0.01, -0.02, 0.03]])
    v0 = np.array([[0.2, 0.1, -0.3]])
    for S in (1, 7, 10):
        st, pos, vel, dp = oracle.chain_md(np.zeros((1, 3)), v0, u, substeps=S, zeta=5.0, mass=2.0)
        assert st == 0
        want = u + (v0 - u) * math.exp(-5.0 / 2.0)
        assert np.abs(vel - want).max() < 1e-15
        assert np.abs(dp - 2.0 * (want - v0)).max() < 1e-15


def test_fene_force_is_gradient_of_potential():
    """Two beads, no friction memory (zeta -> tiny, one substep): the impulse
    balance gives the spring force; compare with -dU/dr of
    U = -(k R0^2/2) ln(1 - r^2/R0^2)."""
    k, r0 = 1.3, 2.0
    rng = np.random.default_rng(1)
    for _ in range(5):
        r = rng.standard_normal(3)
        r *= rng.uniform(0.2, 1.9) / np.linalg.norm(r)
        pos = np.array([[0, 0, 0], r])
        # with u = 0, V0 = 0, exact friction update: dp = m V' - F h  and
        # V' = F/zeta (1 - e^{-zeta h/m}), so F = (m V')/(1-e)*zeta ... invert:
        zeta, m = 2.0, 1.0
        st, p, v, dp = oracle.chain_md(pos, np.zeros((2, 3)), np.zeros((2, 3)), substeps=1,
                                       zeta=zeta, mass=m, fene_k=k, fene_r0=r0)
        F = v * zeta / (1 - math.exp(-zeta / m))

        def U(x):
            return -0.5 * k * r0 ** 2 * math.log(1 - x @ x / r0 ** 2)
        h = 1e-6
        grad = np.array([(U(r + h * e) - U(r - h * e)) / (2 * h) for e in np.eye(3)])
        assert np.abs(F[1] + grad).max() < 1e-7 * max(1, np.abs(grad).max())
        assert np.abs(F[0] - grad).max() < 1e-7 * max(1, np.abs(grad).max())


def test_dimer_converges_to_continuous_dynamics():
    """Dimer bond relaxation with the S-substep integrator approaches the
    continuous ODE (RK4 with tiny steps) as O(1/S)."""
    k, r0, zeta, m = 1.0, 2.0, 5.0, 1.0
    pos0 = np.array([[0, 0, 0], [1.5, 0.3, -0.2]])

    def rhs(y):
        r = y[1] - y[0]
        fac = k / (1 - r @ r / r0 ** 2)
        F = np.array([fac * r, -fac * r])
        return y[2:], (F - zeta * y[2:]) / m

    y = np.concatenate([pos0, np.zeros((2, 3))])
    h = 1e-4
    for _ in range(int(1 / h)):
        def f(yy):
            a, b = rhs(yy)
            return np.concatenate([a, b])
        k1 = f(y)
        k2 = f(y + h / 2 * k1)
        k3 = f(y + h / 2 * k2)
        k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    errs = []
    for S in (10, 100):
        st, p, v, dp = oracle.chain_md(pos0, np.zeros((2, 3)), np.zeros((2, 3)), substeps=S,
                                       zeta=zeta, mass=m, fene_k=k, fene_r0=r0)
        errs.append(np.abs(p - y[:2]).max())
    assert errs[1] < errs[0] / 5
    assert errs[1] < 2e-3


def test_com_pinned_and_fene_error():
    rng = np.random.default_rng(9)
    anchor = np.array([10.3, 11.1, 9.7])
    pos, vel = inputs.chain_init(16, anchor, rng)
    ub = 1e-2 * rng.standard_normal((16, 3))
    st, p, v, dp = oracle.chain_md(pos, vel, ub, substeps=10, fix_com=True, anchor=anchor)
    assert st == 0
    assert np.abs(p.mean(axis=0) - anchor).max() < 1e-14
    assert np.abs(v.mean(axis=0)).max() < 1e-17
    # overstretched bond
    bad = pos.copy()
    bad[5:] += np.array([2.5, 0, 0])
    st, *_ = oracle.chain_md(bad, vel, ub, substeps=10)
    assert st == oracle.ERR_FENE


def test_interpolation_exact_on_affine_flow_and_spreading_moments():
    """Bead in an affine flow (equilibrium populations, rho = 1): the
    velocity the bead feels is exactly a + B R.  The force spread on the
    lattice sums to -dP and its first moment is -dP (x) R (trilinear)."""
    N = 12
    rng = np.random.default_rng(12)
    a = 1e-3 * rng.standard_normal(3)
    Bm = 1e-4 * rng.standard_normal((3, 3))
    ob = oracle.OracleBox((N, N, N), tau=0.8)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing='ij')
    X = np.stack([x, y, z], axis=-1).astype(float)
    ob.set_initial(a + X @ Bm.T)
    ob.set_boundary(oracle.BC_AFFINE, np.zeros((2, 9)))
    R = np.array([[5.3, 6.71, 4.05]])
    zeta = 4.0
    ob.add_chain(R, None, substeps=4, fix_com=False, zeta=zeta)
    assert ob.step(1) == 0
    _, v = ob.beads()
    u_felt = v[0] / (1 - math.exp(-zeta))
    assert np.abs(u_felt - (a + Bm @ R[0])).max() < 1e-15
    g = ob.last_force()
    dp = v[0]                      # m (V1 - V0), no spring forces
    assert np.abs(g.sum(axis=(0, 1, 2)) + dp).max() < 1e-17
    first = np.einsum('zyxa,zyxb->ab', g, X)
    assert np.abs(first + np.outer(dp, R[0])).max() < 1e-15
    assert np.count_nonzero(np.abs(g).sum(axis=-1)) == 8


def test_bead_out_and_unstable_errors_freeze_state():
    N = 10
    ob = oracle.OracleBox((N, N, N), tau=0.8, reduce_every=2)
    ob.set_boundary(oracle.BC_AFFINE, np.zeros((50, 9)))
    ob.add_chain(np.array([[1.5, 4.0, 4.0], [8.2, 4.0, 4.0]]) * 0 + np.array([[7.9, 4, 4], [8.5, 4, 4]]),
                 None, fix_com=False)
    f0 = ob.pop()
    assert ob.step(3) == oracle.ERR_BEAD_OUT
    assert ob.error() == (oracle.ERR_BEAD_OUT, 0)
    assert np.array_equal(ob.pop(), f0) and ob.step_index == 0
    # non-finite populations are caught by the mass check
    ob2 = oracle.OracleBox((N, N, N), tau=0.8, reduce_every=2)
    ob2.set_boundary(oracle.BC_AFFINE, np.zeros((50, 9)))
    f = ob2.pop()
    f[3, 5, 5, 5] = np.nan
    ob2.set_populations(f)
    assert ob2.step(5) == oracle.ERR_UNSTABLE
    assert ob2.error() == (oracle.ERR_UNSTABLE, 1)
    assert ob2.step_index == 1


def test_mass_momentum_record():
    N = 8
    ob = oracle.OracleBox((N, N, N), tau=0.8, reduce_every=3, periodic_mask=7)
    rng = np.random.default_rng(0)
    ob.set_initial(1e-2 * rng.standard_normal((N, N, N, 3)))
    c, _ = oracle.lattice()
    ob.step(6)
    rec = ob.mass_mom()
    f = ob.pop()
    assert rec[0] == 6
    assert abs(rec[1] - f.sum()) < 1e-12
    assert np.abs(rec[2:] - f.sum(axis=(1, 2, 3)) @ c).max() < 1e-14
