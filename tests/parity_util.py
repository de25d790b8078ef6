"""Helpers shared by the GPU parity tests (comparison only, no arithmetic of the method)."""
import numpy as np


def normwise(a, b):
    """max_i |a_i - b_i| / max_i |b_i| (normwise relative error of one field)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    if den == 0.0:
        return float(np.abs(a - b).max()) if a.size else 0.0
    return float(np.abs(a - b).max() / den)


def world_positions(scene):
    """Soil positions and marker positions at the scenes' initial poses (identity
    rotations only), in FP64, in particle-id order."""
    parts = [np.asarray(scene.pos, dtype=np.float64)]
    for b in scene.bodies:
        assert np.allclose(b.quat, (1.0, 0.0, 0.0, 0.0))
        parts.append(np.asarray(b.pos, dtype=np.float64) + b.markers.astype(np.float64))
    return np.concatenate(parts)


def csr_rows(off, nbr, rows=None):
    """Dict row id -> sorted neighbour ids."""
    out = {}
    n = len(off) - 1
    for r in range(n):
        key = int(rows[r]) if rows is not None else r
        out[key] = np.sort(nbr[off[r]:off[r + 1]])
    return out


def fields_report(gpu, ref, n):
    return {k: normwise(gpu[k][:n], ref[k][:n]) for k in ("pos", "vel", "sigma", "rho")}


def check_cell_sort(got_ids, sid, cs, ce, x, tol=1e-6):
    """The GPU's slot order against the oracle's (cell order, ids ascending in
    a cell). Sec. 4.1 sorts by cell hash and leaves the order inside a cell
    open: the GPU orders a cell by x. The cells' contents must be equal, and
    inside every cell the GPU's x must ascend (x: FP64 world positions; tol
    absorbs the FP32 rounding of the stored positions)."""
    got = np.asarray(got_ids, dtype=np.int64)
    sid = np.asarray(sid, dtype=np.int64)
    assert got.shape == sid.shape
    cell = np.repeat(np.arange(cs.size), (ce - cs).astype(np.int64))
    assert cell.size == got.size
    assert np.array_equal(got[np.lexsort((got, cell))], sid)
    xs = np.asarray(x, dtype=np.float64)[got, 0]
    same = cell[1:] == cell[:-1]
    assert np.all(np.diff(xs)[same] >= -tol)


def half_ulp32(x):
    """Half the FP32 spacing at magnitude |x|: the largest error of rounding a
    value of that size to FP32."""
    return 0.5 * float(np.spacing(np.float32(abs(float(x)))))


def position_scale(scene):
    """Magnitude at which positions are stored: the largest soil coordinate for
    FP32 positions, the cell size 2h (the range of the offsets) for cell-index +
    FP32-offset positions."""
    if int(scene.params.get("pos_mode", 0)) == 1:
        return 2.0 * scene.params["h"] + float(scene.params.get("skin", 0.0))
    return float(np.abs(np.asarray(scene.pos, dtype=np.float64)).max())


def displacement_bar(steps, tol, pos_scale, disp_max):
    """Normwise bar for the displacements x_n - x_0: the fields' bar `tol` plus
    the FP32 storage of the positions, which rounds each step's position update
    once at magnitude pos_scale (at most half an ulp per step, accumulated over
    `steps` steps), relative to the largest displacement of the reference."""
    if disp_max == 0.0:
        return 0.0
    return tol + (steps + 1) * half_ulp32(pos_scale) / disp_max


def check_fields(gpu, ref, scene, steps, tol, label="", rows=None):
    """Asserts normwise parity of the soil fields (<= tol) and of the soil
    displacements from the initial positions (<= displacement_bar); rows
    selects a subset of the soil (default all). Returns the report."""
    n = scene.n_soil
    sel = slice(0, n) if rows is None else rows
    x0 = np.asarray(scene.pos, dtype=np.float64)[sel]
    rep = {k: normwise(np.asarray(gpu[k][:n])[sel], np.asarray(ref[k][:n])[sel])
           for k in ("pos", "vel", "sigma", "rho")}
    dref = np.asarray(ref["pos"][:n], dtype=np.float64)[sel] - x0
    dgot = np.asarray(gpu["pos"][:n], dtype=np.float64)[sel] - x0
    dmax = float(np.abs(dref).max()) if dref.size else 0.0
    rep["disp"] = normwise(dgot, dref) if dmax > 0.0 else float(np.abs(dgot).max() if dgot.size else 0.0)
    rep["disp_bar"] = displacement_bar(steps, tol, position_scale(scene), dmax)
    rep["disp_max"] = dmax
    print(label, steps, "steps:", {k: (f"{v:.3e}" if isinstance(v, float) else v) for k, v in rep.items()},
          flush=True)
    for k in ("pos", "vel", "sigma", "rho"):
        assert rep[k] <= tol, (label, k, rep[k])
    assert rep["disp"] <= rep["disp_bar"], (label, "displacement", rep["disp"], rep["disp_bar"])
    return rep
