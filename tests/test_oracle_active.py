"""Pins of the oracle's active domains (Sec. 4.2, Alg. 3).

Flags are checked against points constructed inside, near and outside an
oriented box; the step is checked to leave Extended-Active and Inactive
particles untouched and to equal the plain step when a box covers everything;
the capacity policy is checked on a hand-computed sequence with the paper's
constants G = 1.2, S = 0.75, S_I = 50.
"""
import numpy as np

from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes
from paper_2507_05643_amd.scenes import Body, Scene


def _quat(axis, ang):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * axis])


def _R(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_flags_match_constructed_points():
    rng = np.random.default_rng(0)
    h = 0.012
    half = np.array([0.05, 0.03, 0.04])
    q = _quat([0.3, -0.5, 0.8], 0.7)
    X = np.array([0.4, 0.5, 0.3])
    m = 1e-4
    pts, lab = [], []
    for _ in range(4000):
        kind = rng.integers(0, 3)
        if kind == 2:      # strictly inside the box
            l = rng.uniform(-half + m, half - m)
        elif kind == 1:    # inside the grown box, outside the box
            l = rng.uniform(-(half + 2 * h - m), half + 2 * h - m)
            ax = rng.integers(0, 3)
            l[ax] = np.sign(rng.uniform(-1, 1)) * rng.uniform(half[ax] + m, half[ax] + 2 * h - m)
        else:              # outside the grown box along one axis
            l = rng.uniform(-(half + 3 * h), half + 3 * h)
            ax = rng.integers(0, 3)
            l[ax] = np.sign(rng.uniform(-1, 1)) * rng.uniform(half[ax] + 2 * h + m, half[ax] + 4 * h)
        pts.append(X + _R(q) @ l)
        lab.append(kind)
    pos = np.asarray(pts, dtype=np.float32)
    p = dict(scenes.DEFAULT_PARAMS, active_domains=1, t_delay=-1.0, domain_lo=(0.0,) * 3,
             domain_hi=(1.0,) * 3, gravity=(0.0, 0.0, 0.0))
    body = Body(markers=np.zeros((0, 3), dtype=np.float32), active_half=tuple(half),
                pos=tuple(X), quat=tuple(q))
    sc = Scene("flags", p, pos, bodies=[body])
    o = Oracle(sc, nbr_mode="cells")
    o.step(1)
    assert np.array_equal(o.flags()[: len(lab)], np.asarray(lab, dtype=np.uint8))


def _strip(**kw):
    return scenes.strip(length=3.0, width=1.2, depth=0.2, dx=0.05, half=0.3, wheelbase=1.2,
                        track=0.6, **kw)


def test_inactive_and_extended_are_untouched():
    sc = _strip(seed=1, t_delay=-1.0)
    sc.params["ps_freq"] = 2
    o = Oracle(sc, nbr_mode="cells")
    s0 = o.state()
    o.step(3)
    f = o.flags()[: sc.n_soil]
    s1 = o.state()
    assert (f == 0).sum() > 100 and (f == 1).sum() > 50 and (f == 2).sum() > 50
    frozen = f != 2
    for k in ("pos", "vel", "sigma", "rho"):
        assert np.array_equal(s0[k][: sc.n_soil][frozen], s1[k][: sc.n_soil][frozen])
    moved = np.abs(s1["pos"][: sc.n_soil][f == 2] - s0["pos"][: sc.n_soil][f == 2]).max()
    assert moved > 0.0


def test_t_delay_processes_everything_before_it():
    sc = _strip(seed=2, t_delay=1.0)
    o = Oracle(sc, nbr_mode="cells")
    o.step(1)
    assert o.n_proc == o.n
    assert np.all(o.flags() == 2)


def test_covering_box_equals_no_active_domains():
    sc = scenes.column(seed=3, n=8)
    big = Body(markers=np.zeros((0, 3), dtype=np.float32), active_half=(10.0, 10.0, 10.0))
    sc.bodies.append(big)
    sc.params.update(active_domains=1, t_delay=-1.0, ps_freq=3)
    o1 = Oracle(sc, nbr_mode="cells")
    o1.step(7)
    p2 = dict(sc.params, active_domains=0)
    o2 = Oracle(sc, nbr_mode="cells", params=p2)
    o2.step(7)
    a, b = o1.state(), o2.state()
    for k in a:
        assert np.array_equal(a[k], b[k])
    Fa, Ta = o1.forces()
    Fb, Tb = o2.forces()
    assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)


def test_capacity_policy(orc):
    # grow to ceil(1.2 n) when n exceeds capacity
    assert orc.capacity_next(0, 100, 1) == 120
    assert orc.capacity_next(120, 110, 1) == 120
    assert orc.capacity_next(120, 121, 7) == 146          # ceil(145.2)
    # shrink only at multiples of S_I = 50, when n / cap < 0.75
    assert orc.capacity_next(146, 100, 49) == 146
    assert orc.capacity_next(146, 100, 50) == 100         # 0.685 < 0.75
    assert orc.capacity_next(146, 110, 50) == 146         # 0.753 >= 0.75
    assert orc.capacity_next(146, 110, 100) == 146
    assert orc.capacity_next(1000, 10, 150) == 10


def test_capacity_tracks_processed_set():
    sc = _strip(seed=0, t_delay=-1.0)
    o = Oracle(sc, nbr_mode="cells")
    o.step(1)
    n = o.n_proc
    assert n < o.n
    assert o.capacity == int(np.ceil(1.2 * n))
