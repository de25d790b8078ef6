"""Pins of the stored position form of the oracle's integer decisions (cell
index + FP32 offset, the km-scale representation of the terrain passes,
Sec. 5; cell size 2h of the linked list, Sec. 4.1).

1. The stored form of a position against exact rational arithmetic: the cell is
   floor((x - lo) / (2h)) and the offset the FP32 rounding of x - lo - c 2h,
   for coordinates on both sides of the grid origin and up to 10 km from it.
2. Translation by whole cells (a scene and its grid shifted by k 2h, every
   coordinate an exact binary fraction): the stored offsets, the neighbour
   lists and the right-hand side of the step are bit-identical, the cells move
   by k.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes

H = 2.0 ** -7          # S = 2h = 2^-6 m: whole-cell shifts are exact in FP64


def _params(lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), pos_mode=1):
    return dict(scenes.DEFAULT_PARAMS, h=H, dx=H / 1.2, domain_lo=lo, domain_hi=hi, pos_mode=pos_mode)


@pytest.mark.parametrize("lo", [0.0, -3.75, 1234.5])
def test_stored_form_against_exact_arithmetic(lo):
    p = _params(lo=(lo, lo, lo), hi=(lo + 1.0e4,) * 3)
    S = 2.0 * H
    rng = np.random.default_rng(7)
    mags = np.concatenate([rng.uniform(-5 * S, 5 * S, 300), rng.uniform(-1e4, 1e4, 300),
                           rng.uniform(0, 50 * S, 300)])
    checked = 0
    for k in range(0, mags.size, 3):
        x = lo + mags[k:k + 3]
        c, o = O.to_rep(p, x)
        for a in range(3):
            q = (Fraction(float(x[a])) - Fraction(lo)) / Fraction(S)
            fl = q.numerator // q.denominator
            if abs(q - round(q)) < Fraction(1, 10 ** 9):
                continue                      # within rounding of a cell face: either side is right
            assert c[a] == fl, (x[a], c[a], fl)
            exact = Fraction(float(x[a])) - Fraction(lo) - fl * Fraction(S)
            assert 0 <= exact < S
            want = np.float32(float(exact))
            # the offset is exact x - lo - c S rounded once to FP32 (up to the FP64
            # rounding of x - lo, far below half an FP32 ulp of the offset)
            assert abs(o[a] - float(want)) <= float(np.spacing(want)), (x[a], o[a], want)
            checked += 1
    assert checked > 800


def test_fp32_form_is_the_rounded_coordinate():
    p = _params(pos_mode=0)
    x = np.array([0.1, 9999.123456, -2.5e-3])
    c, o = O.to_rep(p, x)
    assert np.all(c == 0)
    assert np.array_equal(o, x.astype(np.float32).astype(np.float64))


def _scene(shift_cells):
    """A jittered column of 6^3 soil particles in a marker box, translated by
    shift_cells cells of 2h along x (scene and grid)."""
    S = 2.0 * H
    sh = np.array([shift_cells * S, 0.0, 0.0])
    sc = scenes.column(seed=3, n=6, dx=H / 1.2)
    sc.params.update(h=H, pos_mode=1)
    lo = np.full(3, -3 * S) + sh                # grid corners on whole cells too
    hi = np.full(3, 7 * S) + sh
    sc.params.update(domain_lo=tuple(lo), domain_hi=tuple(hi))
    sc.pos = (sc.pos.astype(np.float64) + sh)
    b = sc.bodies[0]
    b.pos = tuple(np.asarray(b.pos, dtype=np.float64) + sh)
    return sc, sh


def test_whole_cell_translation_is_exact():
    base, _ = _scene(0)
    far, sh = _scene(640000)                 # 10 km along x
    assert far.pos[:, 0].min() > 9999.0
    # every coordinate and the shift are exact binary fractions: the shift is exact
    assert np.array_equal(far.pos - sh, base.pos.astype(np.float64))
    a, b = Oracle(base, nbr_mode="cells"), Oracle(far, nbr_mode="cells")
    ra, rb = a.eval_rhs(), b.eval_rhs()
    pa, oa, na = a.lists()
    pb, ob, nb = b.lists()
    assert np.array_equal(pa, pb) and np.array_equal(oa, ob) and np.array_equal(na, nb)
    for k in ("drho", "du", "ds", "mu", "ms", "mas"):
        assert np.array_equal(ra[k], rb[k]), k
    xa, xb = a.positions(), b.positions()
    for i in range(0, xa.shape[0], 37):
        ca, oa_ = O.to_rep(base.params, xa[i])
        cb, ob_ = O.to_rep(far.params, xb[i])
        assert np.array_equal(oa_, ob_) and np.array_equal(ca, cb)     # grid moved with the scene
    # without moving the grid, the cells move by the shift and the offsets stay
    p0 = dict(base.params, domain_lo=base.params["domain_lo"], domain_hi=(60.0, 0.1, 0.1))
    for i in range(0, xa.shape[0], 37):
        ca, oa_ = O.to_rep(p0, xa[i])
        cb, ob_ = O.to_rep(p0, xa[i] + np.array([3200 * 2 * H, 0.0, 0.0]))
        assert np.array_equal(oa_, ob_) and cb[0] - ca[0] == 3200 and np.array_equal(cb[1:], ca[1:])
