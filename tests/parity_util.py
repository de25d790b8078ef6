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
