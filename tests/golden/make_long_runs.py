"""Writes the oracle's values for the long-run and full-size parity cases.

Runs only the FP64 oracle (``oracle/``) on the inputs of ``tests/longrun.py``
and stores, per box, at the sampled interior sites that module defines:

  u_<k>     float32 [sites][3]   velocity j/rho at the last step
  dev_<k>   float32 [sites][19]  population deviations f_i - w_i rho0
  bpos_<k>, bvel_<k>  float64 [beads][3]   bead positions and velocities
  mm_<k>    float64 [5]          last mass/momentum record (step, M, P)
  unorm_<k>, umax_<k>            L2 norm and largest |u| over the whole interior

into ``tests/golden/long_<case>.npz``.  Usage:

  python tests/golden/make_long_runs.py <case> [<case> ...]

The 512^3 case needs about 95 GB of host memory.  Progress is printed per
chunk of steps.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

import longrun  # noqa: E402
import oracle  # noqa: E402


def run_case(name):
    spec = longrun.CASES[name]
    steps = spec["steps"]
    t0 = time.time()
    bxs = longrun.boxes(name)
    print(f"{name}: inputs of {len(bxs)} boxes in {time.time() - t0:.1f} s", flush=True)
    _, w = oracle.lattice()
    out = {"steps": np.int64(steps), "indices": np.asarray([b["index"] for b in bxs], np.int64),
           "edges": np.asarray([b["n"] for b in bxs], np.int64)}
    for k, b in enumerate(bxs):
        n = b["n"]
        ob = oracle.OracleBox((n, n, n), collision=oracle.MRT, tau=longrun.TAU,
                              tau_bulk=longrun.TAU, ghost_rate=1.0,
                              reduce_every=spec["reduce_every"])
        ob.set_initial(b["u0"])
        ob.set_boundary(oracle.BC_SAMPLED, b["faces"].astype(np.float64), t0=0, dt=longrun.DT,
                        res=longrun.RES)
        for c in b["chains"]:
            ob.add_chain(c["pos"], None, substeps=10, fix_com=True, zeta=5.0,
                         mass=longrun.bead_mass(len(c["pos"])), fene_k=1.0, fene_r0=2.0,
                         anchor=c["anchor"])
        b.pop("u0")
        chunk = max(1, min(steps, int(2e8 // (n - 2) ** 3)))
        done, ts = 0, time.time()
        while done < steps:
            m = min(chunk, steps - done)
            st = ob.step(m)
            if st != 0:
                raise RuntimeError(f"{name} box {k}: oracle stopped with status {st} "
                                   f"at step {ob.error()[1]}")
            done += m
            print(f"{name} box {k} (edge {n}): step {done}/{steps}, "
                  f"{(n - 2) ** 3 * done / (time.time() - ts) / 1e6:.2f} MLUPS", flush=True)
        s = longrun.sites(n, [c["anchor"] for c in b["chains"]], spec["site_seed"] + b["index"])
        x, y, z = s[:, 0], s[:, 1], s[:, 2]
        _, u = ob.rho_u()
        mask = ob.interior_mask()
        out[f"unorm_{k}"] = np.float64(np.linalg.norm(u[mask]))
        out[f"umax_{k}"] = np.float64(np.abs(u[mask]).max())
        out[f"u_{k}"] = u[z, y, x].astype(np.float32)
        del u, mask
        f = ob.pop()
        out[f"dev_{k}"] = (f[:, z, y, x].T - w[None, :]).astype(np.float32)
        del f
        p, v = ob.beads()
        out[f"bpos_{k}"] = p
        out[f"bvel_{k}"] = v
        out[f"mm_{k}"] = ob.mass_mom()
        del ob
    path = longrun.golden_path(name)
    np.savez_compressed(path, **out)
    print(f"{name}: wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB) in "
          f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        run_case(name)
