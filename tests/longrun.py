"""Long-run and full-size parity cases: their inputs and the sites they are compared on.

Shared by the golden-value writer ``tests/golden/make_long_runs.py`` (which
runs only the FP64 oracle) and the GPU tests ``tests/test_gpu_long_runs.py``.
This module holds no lattice-Boltzmann arithmetic: it builds the seeded inputs
of each case and chooses, with host integer logic only, the interior nodes on
which the two sides are compared.

Cases (MRT tau = tau_bulk = 0.6, ghost rate 1, KS tracer boundary on a 17 x 17
corner-aligned face grid every 20 steps, KS initial field):

* ``batch16``  -- 16 boxes of the batched workload (4 of each edge 32, 48, 64,
                  96, drawn with a seeded generator from the 256 boxes of the
                  benchmark, identical inputs), one 32-bead chain each, the
                  workload's full 5,000 steps.
* ``ks128``    -- the single-box workload: 128^3, one 64-bead chain, its full
                  10,000 steps.
* ``big128``   -- the large-box setup (32 chains of 256 beads at seeded
                  anchors in [N/4, 3N/4]^3) at 128^3 over the large-box
                  workload's full 2,000 steps.
* ``big512``   -- the large-box workload itself: 512^3, 32 chains of 256
                  beads, 50 steps (the oracle's FP64 state needs about 65 GB).

Sampled sites of a box with N nodes per edge (interior coordinates 1..N-2):
  rows       every interior node of the x-rows at (y, z) in {1, 2, mid, N-3, N-2}^2:
             the rows next to the y and z faces, and the x-face neighbours
             x = 1, N-2 and wavefront edges of every row;
  columns    every interior node of the y-columns at (x, z) in {1, N-2} x {1, mid, N-2};
  cubes      the 8^3 interior nodes around each chain anchor (the nodes a
             collapsed chain spreads its force onto, and their neighbours);
  random     a seeded uniform draw of interior nodes (2,000, or all of a
             small box's interior nodes if it has fewer).
"""
from __future__ import annotations

import numpy as np

from paper_0809_4958_amd import inputs

TAU = 0.6
DT, RES = 20, 17
CHAIN_BOND = 0.05
N_RANDOM = 2000

CASES = {
    "batch16": dict(steps=5000, reduce_every=100, site_seed=0),
    "ks128": dict(steps=10000, reduce_every=100, site_seed=10000),
    "big128": dict(steps=2000, reduce_every=100, site_seed=20000),
    "big512": dict(steps=50, reduce_every=10, site_seed=30000),
}


def bead_mass(n_beads):
    """Whole chain at half a fluid node (the tests' and benchmark's reading)."""
    return 0.5 / n_beads


def batch16_indices(n_boxes=256, per_size=4, config_idx=2):
    """Indices of the 16-box subset: ``per_size`` boxes of every edge, drawn
    without replacement by a seeded generator (stream 5 of the batch)."""
    sizes = inputs.box_sizes(n_boxes, inputs.rng(config_idx, 3))
    g = inputs.rng(config_idx, 5)
    out = []
    for n in (32, 48, 64, 96):
        idx = np.flatnonzero(sizes == n)
        out.extend(int(i) for i in g.choice(idx, size=per_size, replace=False))
    return sorted(out)


def _big_box(n, steps, config_idx=4):
    units, u0, faces = inputs.ks_box_inputs(config_idx, 0, n=n, tau=TAU, n_steps=steps, dt=DT,
                                            res=RES)
    g = inputs.rng(config_idx, 2)
    anchors = inputs.anchors(32, n, g)
    chains = []
    for a in anchors:
        pos, _ = inputs.chain_init(256, a, g, bond=CHAIN_BOND)
        chains.append(dict(pos=pos, anchor=np.asarray(a, dtype=np.float64)))
    return dict(n=n, u0=u0, faces=faces.astype(np.float32), chains=chains)


def boxes(name):
    """Inputs of every box of a case: dicts with n, u0 [n][n][n][3] FP64,
    faces FP32 [samples][6][17][17][3], chains (pos, anchor), index."""
    steps = CASES[name]["steps"]
    if name == "batch16":
        import bench
        out = []
        for b in bench.batch_inputs(256, steps, TAU, only=set(batch16_indices())):
            out.append(dict(n=b["n"], u0=b["u0"], faces=b["faces"], index=b["index"],
                            chains=[dict(pos=b["pos"], anchor=b["anchor"])]))
        return out
    if name == "ks128":
        n = 128
        units, u0, faces = inputs.ks_box_inputs(1, 0, n=n, tau=TAU, n_steps=steps, dt=DT, res=RES)
        xc = np.full(3, (n - 1) / 2.0)
        pos, _ = inputs.chain_init(64, xc, inputs.rng(1, 2), bond=CHAIN_BOND)
        return [dict(n=n, u0=u0, faces=faces.astype(np.float32), index=0,
                     chains=[dict(pos=pos, anchor=xc)])]
    if name == "big128":
        b = _big_box(128, steps)
        b["index"] = 0
        return [b]
    if name == "big512":
        b = _big_box(512, steps)
        b["index"] = 0
        return [b]
    raise KeyError(name)


def sites(n, anchors, seed):
    """Sampled interior nodes of a box of edge n: int32 [k][3] (x, y, z), sorted
    by linear index (z ny + y) nx + x, without repeats."""
    mid = (n - 1) // 2
    lo, hi = 1, n - 2
    pts = []
    ys = sorted({1, 2, mid, n - 3, n - 2})
    xs_line = np.arange(lo, hi + 1)
    for y in ys:
        for z in ys:
            pts.append(np.stack([xs_line, np.full_like(xs_line, y), np.full_like(xs_line, z)], 1))
    for x in (1, n - 2):
        for z in sorted({1, mid, n - 2}):
            pts.append(np.stack([np.full_like(xs_line, x), xs_line, np.full_like(xs_line, z)], 1))
    for a in anchors:
        c = np.floor(np.asarray(a, dtype=np.float64)).astype(np.int64)
        r = [np.arange(max(lo, c[k] - 3), min(hi, c[k] + 4) + 1) for k in range(3)]
        g = np.stack(np.meshgrid(r[0], r[1], r[2], indexing="ij"), -1).reshape(-1, 3)
        pts.append(g)
    interior = (n - 2) ** 3
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        entropy=inputs.ENTROPY, spawn_key=(99, int(seed)))))
    if interior <= N_RANDOM:
        k = np.arange(interior)
    else:
        k = rng.choice(interior, size=N_RANDOM, replace=False)
    m = n - 2
    pts.append(np.stack([k % m + 1, (k // m) % m + 1, k // (m * m) + 1], 1))
    p = np.concatenate(pts).astype(np.int64)
    lin = (p[:, 2] * n + p[:, 1]) * n + p[:, 0]
    _, first = np.unique(lin, return_index=True)
    return np.ascontiguousarray(p[first], dtype=np.int32)


def golden_path(name):
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"long_{name}.npz")
