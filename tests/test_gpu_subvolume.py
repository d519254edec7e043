"""Sub-volume history files (the data-on-disk coupling of the two scales,
Sec. 1-2): a KS tracer history written to a file and loaded by the library
gives the boundary history of the grid's six faces, the initial field
interpolated trilinearly from sample 0 (checked against scipy's linear
interpolator), and the tracer accelerations as the body force -- and the run
from the file equals, in FP64, the oracle run from the same arrays."""
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
from lbcase import Case
from paper_0809_4958_amd import inputs
from test_gpu_parity import check, compare

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_0809_4958_amd.lbm")


def say(*a):
    print(*a, flush=True)


def faces_of(w):
    """The six faces of a grid history [S][R][R][R][3] ([z][y][x]) in the
    SAMPLED layout [S][6][R][R][3], entry [v][u], u the lower-index axis."""
    S, R = w.shape[0], w.shape[1]
    out = np.empty((S, 6, R, R, 3))
    wx = w.transpose(0, 3, 2, 1, 4)          # [S][x][y][z][3]
    for f in range(6):
        a = f // 2
        idx = 0 if f % 2 == 0 else R - 1
        sl = [slice(None)] * 3
        sl[a] = idx
        plane = wx[(slice(None),) + tuple(sl)]  # [S][u][v][3] with u < v the remaining axes
        out[:, f] = plane.transpose(0, 2, 1, 3)
    return out


def test_subvolume_file_round_trip(tmp_path):
    n, R, dt, steps = 25, 9, 10, 40
    w, acc = inputs.ks_subvolume_history(6, 0, n=n, tau=0.7, n_steps=steps, dt=dt, grid=R)
    path = os.path.join(tmp_path, "box.lbsv")
    inputs.write_subvolume(path, w, dt=dt, t0=0, accel=acc)
    w32 = w.astype(np.float32).astype(np.float64)
    faces = faces_of(w32)
    g = np.arange(R) * (n - 1) / (R - 1)
    interp = RegularGridInterpolator((g, g, g), w32[0], method="linear")
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    u0 = interp(np.stack([zz, yy, xx], -1).reshape(-1, 3)).reshape(n, n, n, 3)
    say("case sub-volume file", n, R, "accel rms", np.sqrt((acc ** 2).mean()))
    ctx = lbm.Context([(n, n, n)], collision=lbm.MRT, tau=0.7, tau_bulk=0.7, storage=0)
    ctx.load_subvolume(0, path, lbm.SUBVOL_INITIAL | lbm.SUBVOL_BOUNDARY | lbm.SUBVOL_BODY)
    # the initial field is the trilinear interpolation of sample 0
    u_g = ctx.read(0, lbm.F_U)
    m = np.zeros((n, n, n), dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    err0 = np.abs(u_g[m] - u0[m]).max() / np.abs(u0[m]).max()
    say("initial field vs scipy", err0)
    assert err0 < 1e-13
    ctx.step(steps)
    case = Case((n, n, n), collision=oracle.MRT, tau=0.7, tau_bulk=0.7,
                bc=(oracle.BC_SAMPLED, faces, 0, dt, R), u0=u0, body=(acc, 0, dt))
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    check(compare(ctx, ob, case, "f64"), "f64", "sub-volume run")
    ctx.close()
    # malformed and truncated files are refused and change nothing
    bad = os.path.join(tmp_path, "bad.lbsv")
    with open(path, "rb") as fh:
        raw = fh.read()
    ctx2 = lbm.Context([(n, n, n)], collision=lbm.MRT, tau=0.7, tau_bulk=0.7, storage=0)
    for blob in (b"XXXXXXXX" + raw[8:], raw[:-8], raw + b"\0"):
        with open(bad, "wb") as fh:
            fh.write(blob)
        with pytest.raises(lbm.LBError) as e:
            ctx2.load_subvolume(0, bad, lbm.SUBVOL_BOUNDARY)
        assert e.value.status == lbm.ERR_ARG
    assert ctx2.step_status(1) == lbm.ERR_STATE   # still no boundary
    ctx2.close()
