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
