"""Shared test setup: build one case on both the FP64 oracle and the GPU library
from the same seeded inputs, and compare what they return."""
from __future__ import annotations

import numpy as np

import oracle
from paper_0809_4958_amd import inputs


def bead_mass(n_beads):
    """Bead mass: the whole chain weighs half a fluid node (rho0 a^3 = 1).  The
    exact per-step friction update hands m (V - u) to the fluid; once the
    chain (kT = 0, no excluded volume) has collapsed onto a few nodes, the
    relative-velocity map multiplies by about -(n_beads m)/M with M >= 1 the
    fluid mass seen by the stencil, so n_beads m < 1 is required."""
    return 0.5 / n_beads


# Random-walk bond length of the initial chains, in lattice spacings.  With
# k = 1 and kT = 0 the chain collapses from its initial shape; bonds of 0.05
# give spring forces k b comparable to zeta times the boundary-driven flow
# (|f/w - 1| stays at the per-cent level), while unit bonds drive |f/w - 1|
# to O(1) near the chain and the lattice fluid out of its stable range.
CHAIN_BOND = 0.05


def rel_l2(a, b, mask=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a = a[mask]
        b = b[mask]
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def max_rel(a, b):
    """Per-node max-norm: the largest |a - b| over every node and component,
    relative to the largest |b| (the field's own scale; a per-node quotient
    is ill-defined where the field crosses zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    d = np.abs(a - b).max() if b.size else 0.0
    return float(d / den) if den > 0 else float(d)


def bead_errors(p_g, v_g, p_o, v_o, chains, u_scale):
    """Bead errors, element by element and as norms.

    Positions are compared relative to each chain's anchor and scaled by the
    chain's size: the rms distance of the initial beads from the anchor, or
    (a single free bead) of the oracle's final beads from it.  The kT = 0
    chain collapses toward its anchor, so R - anchor shrinks and a plain
    relative norm of it is ill-conditioned.  Velocities are scaled by the
    problem's velocity scale: the larger of the largest fluid velocity of the
    interior ``u_scale`` and the largest bead velocity.  A pinned chain's V is
    the small difference between the fluid velocity at each bead and its
    chain average, so its own magnitude would amplify rounding by |u|/|V|.
      bead_pos      rms |R_g - R_o| / size
      bead_pos_max  largest |R_g - R_o| of any bead and axis / size
      bead_vel      rms |V_g - V_o| / u_scale
      bead_vel_max  largest |V_g - V_o| of any bead and axis / u_scale
    """
    anc = np.concatenate([np.broadcast_to(c["anchor"], (len(c["pos"]), 3)) for c in chains])
    p0 = np.concatenate([np.asarray(c["pos"]) for c in chains])
    size = np.sqrt(np.mean(np.sum((p0 - anc) ** 2, axis=1)))
    if not size > 0:
        size = np.sqrt(np.mean(np.sum((np.asarray(p_o) - anc) ** 2, axis=1)))
    u_scale = max(float(u_scale), float(np.abs(v_o).max()))
    dp = np.asarray(p_g) - np.asarray(p_o)
    dv = np.asarray(v_g) - np.asarray(v_o)
    nb = len(p0)
    return {"bead_pos": float(np.sqrt(np.sum(dp ** 2) / nb) / size),
            "bead_pos_max": float(np.abs(dp).max() / size),
            "bead_vel": float(np.sqrt(np.sum(dv ** 2) / nb) / u_scale),
            "bead_vel_max": float(np.abs(dv).max() / u_scale)}


class Case:
    """Inputs of one box: dims, collision, boundary, chains, initial field."""

    def __init__(self, dims, collision=oracle.BGK, tau=0.8, tau_bulk=None, ghost_rate=1.0,
                 periodic_mask=0, bc=None, u0=None, chains=(), reduce_every=0, body=None,
                 kT=0.0, seed=0, box_index=0):
        self.dims = tuple(dims)
        self.collision = collision
        self.tau = tau
        self.tau_bulk = tau if tau_bulk is None else tau_bulk
        self.ghost_rate = ghost_rate
        self.pmask = periodic_mask
        self.bc = bc              # (mode, data, t0, dt, res)
        self.u0 = u0
        self.chains = list(chains)  # dicts: pos, vel, substeps, fix_com, zeta, fene_k, fene_r0, anchor
        self.reduce_every = reduce_every
        self.body = body            # (accel [n][3], t0, dt) or None
        self.kT, self.seed = kT, seed
        self.box_index = box_index  # the box's index in the GPU context (random counters)

    def oracle_box(self):
        ob = oracle.OracleBox(self.dims, collision=self.collision, tau=self.tau,
                              tau_bulk=self.tau_bulk, ghost_rate=self.ghost_rate,
                              periodic_mask=self.pmask, reduce_every=self.reduce_every)
        ob.set_initial(self.u0)
        if self.bc is not None:
            mode, data, t0, dt, res = self.bc
            ob.set_boundary(mode, np.asarray(data, dtype=np.float64), t0=t0, dt=dt, res=res)
        for c in self.chains:
            ob.add_chain(c["pos"], c.get("vel"), substeps=c.get("substeps", 10),
                         fix_com=c.get("fix_com", True), zeta=c.get("zeta", 5.0),
                         mass=c.get("mass", bead_mass(len(c["pos"]))),
                         fene_k=c.get("fene_k", 1.0), fene_r0=c.get("fene_r0", 2.0),
                         anchor=c.get("anchor"))
        if self.body is not None:
            accel, t0, dt = self.body
            ob.set_body_force(accel, t0=t0, dt=dt)
        if self.kT:
            assert ob.set_thermal(self.kT, self.seed, self.box_index) == 0
        return ob

    def add_to(self, ctx, box=0):
        ctx.set_initial(box, self.u0)
        if self.bc is not None:
            mode, data, t0, dt, res = self.bc
            ctx.set_boundary(box, mode, data, t0=t0, dt=dt, res=res)
        for c in self.chains:
            ctx.couple_chain(box, c["pos"], c.get("vel"), substeps=c.get("substeps", 10),
                             fix_com=c.get("fix_com", True), zeta=c.get("zeta", 5.0),
                             mass=c.get("mass", bead_mass(len(c["pos"]))),
                             fene_k=c.get("fene_k", 1.0), fene_r0=c.get("fene_r0", 2.0),
                             anchor=c.get("anchor"))
        if self.body is not None:
            accel, t0, dt = self.body
            ctx.set_body_force(box, accel, t0=t0, dt=dt)

    @property
    def n_beads(self):
        return sum(len(c["pos"]) for c in self.chains)


def cfg0_case(n_steps=200, n=32):
    """Plain FP64 configuration: n^3 BGK tau = 0.8, rest start, affine OU
    boundary (correlation 500 steps, rms 1e-3), one 16-bead FENE chain
    (k = 1, R0 = 2, zeta = 5) at the box centre."""
    A = inputs.ou_strain(n_steps, inputs.rng(0, 0), corr_steps=500.0, rms=1e-3)
    xc = np.full(3, (n - 1) / 2.0)
    pos, vel = inputs.chain_init(16, xc, inputs.rng(0, 2), bond=CHAIN_BOND)
    chain = dict(pos=pos, vel=vel, substeps=10, fix_com=True, zeta=5.0, fene_k=1.0, fene_r0=2.0,
                 anchor=xc)
    return Case((n, n, n), collision=oracle.BGK, tau=0.8, bc=(oracle.BC_AFFINE, A, 0, 1, 0),
                chains=[chain], reduce_every=50)


def ks_case(n, n_steps, dt=20, res=17, tau=0.6, n_beads=16, config_idx=1, box_idx=0,
            collision=oracle.MRT, f32_samples=True):
    """KS-driven box (tracer frame, Eq. (1) scaling, width 2 eta): MRT, sampled
    corner-aligned face grid every dt steps, one chain at the centre."""
    units, u0, faces = inputs.ks_box_inputs(config_idx, box_idx, n=n, tau=tau, n_steps=n_steps,
                                            dt=dt, res=res)
    if f32_samples:
        faces = faces.astype(np.float32)
    xc = np.full(3, (n - 1) / 2.0)
    chains = []
    if n_beads:
        pos, vel = inputs.chain_init(n_beads, xc, inputs.rng(config_idx, 2), bond=CHAIN_BOND)
        chains.append(dict(pos=pos, vel=vel, anchor=xc))
    return Case((n, n, n), collision=collision, tau=tau, tau_bulk=tau, ghost_rate=1.0,
                bc=(oracle.BC_SAMPLED, faces, 0, dt, res), u0=u0, chains=chains, reduce_every=100)
