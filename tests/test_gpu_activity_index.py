"""Active-domain flags from the coarse-cell index (activity_scan 0) against the
test of all N particles (activity_scan 1, Sec. 4.2 item 2): the same flags,
hence the same processed set in the same order, so every rebuild's lists and
every step's state and body forces are bit-identical. Wheels drive along a
strip, crossing several coarse cells (8 list cells per axis), with active
boxes reaching past the grid's edge, an active box wholly outside the grid,
a switch-on after t_delay, a state round trip (crm_set_state) and a
checkpoint restore in between (both rebuild the index), and a moved list
that fills up (the index is rebuilt)."""
import numpy as np
import pytest

from paper_2507_05643_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_05643_amd import crm as C
    return C


def _scene():
    sc = scenes.strip(seed=4, length=5.0, width=1.2, depth=0.2, dx=0.05, half=0.3, wheelbase=1.2, track=0.6,
                      t_delay=0.005, ps_freq=3, x0=0.2, speed=8.0)
    # a body without markers whose box lies beyond the grid's low x edge
    sc.bodies.append(scenes.Body(markers=np.zeros((0, 3), dtype=np.float32), active_half=(0.2, 0.2, 0.2),
                                 pos=(-3.0, 0.6, 0.1), name="outside"))
    return sc


class Driver:
    """Moves the wheels along x at their speed (rotating about y), the floor and
    the outside box fixed."""

    def __init__(self, sc):
        self.pos0 = np.array([b.pos for b in sc.bodies], dtype=np.float64)
        self.lin = np.array([b.linvel for b in sc.bodies], dtype=np.float64)
        self.ang = np.array([b.angvel for b in sc.bodies], dtype=np.float64)
        self.dt = sc.params["dt"]

    def bodies(self, k):
        t = k * self.dt
        p = self.pos0 + self.lin * t
        th = self.ang[:, 1] * t
        q = np.stack([np.cos(0.5 * th), np.zeros_like(th), np.sin(0.5 * th), np.zeros_like(th)], axis=1)
        return p, q, self.lin, self.ang


def _run(sim, drv, k0, n):
    for k in range(k0, k0 + n):
        sim.set_bodies(*drv.bodies(k))
        sim.step(1)
    return k0 + n


def _same_state(a, b):
    sa, sb = a.state(), b.state()
    return all(np.array_equal(sa[k], sb[k]) for k in sa)


def _same_lists(a, b):
    ea, eb = a.export(), b.export()
    for k in ("flags", "sorted_ids", "rows", "off", "nbr"):
        if not np.array_equal(ea[k], eb[k]):
            return k
    return None


# moved_cap 0: the default (16,384 entries here, never full); 6,000: the list
# fills up on the way (up to ~1,800 integrated rows a rebuild and 4,440 wheel
# markers, more soil swept over time) and the index is rebuilt; 2,000: some
# rebuilds integrate more than 1,000 rows and test all N instead, the next
# ones use a new index.
@pytest.mark.parametrize("pos_mode,moved_cap", [(0, 0), (1, 0), (0, 6000), (1, 2000)])
def test_index_flags_equal_the_scan(crm, pos_mode, moved_cap):
    sc = _scene()
    drv = Driver(sc)
    p_ix = dict(sc.params, pos_mode=pos_mode, activity_scan=0, moved_cap=moved_cap)
    p_sc = dict(sc.params, pos_mode=pos_mode, activity_scan=1)
    a = crm.Simulation(sc, params=p_ix)
    b = crm.Simulation(sc, params=p_sc)
    # 1,188 steps at 8 m/s: 2.4 m, across two to three coarse cells (0.96 m);
    # lists, flags, state and forces compared every 99 steps (a rebuild step)
    for k in range(0, 1188, 99):
        for s in (a, b):
            _run(s, drv, k, 99)
        assert a.counts()["n_proc"] == b.counts()["n_proc"], k
        bad = _same_lists(a, b)
        assert bad is None, (k, bad)
        assert _same_state(a, b), k
        Fa, Fb = a.forces(), b.forces()
        assert np.array_equal(Fa[0], Fb[0]) and np.array_equal(Fa[1], Fb[1]), k
        if k == 495:
            # a state round trip rebuilds the index
            for s in (a, b):
                st = s.state()
                n = sc.n_soil
                s.set_state(pos=st["pos"][:n], vel=st["vel"][:n], sigma=st["sigma"][:n], rho=st["rho"][:n])
    c = a.counts()
    assert 0 < c["n_proc"] < c["n_total"]
    a.close()
    b.close()


def test_index_after_checkpoint_restore(crm):
    sc = _scene()
    drv = Driver(sc)
    p_ix = dict(sc.params, activity_scan=0)
    p_sc = dict(sc.params, activity_scan=1)
    a = crm.Simulation(sc, params=p_ix)
    k = _run(a, drv, 0, 300)                    # a rebuild step (ps_freq 3)
    blob = a.save_checkpoint()
    _run(a, drv, k, 200)
    want, Fw = a.state(), a.forces()
    b = crm.Simulation(sc, params=p_ix)
    b.load_checkpoint(blob)
    _run(b, drv, k, 200)
    c = crm.Simulation(sc, params=p_sc)
    c.load_checkpoint(blob)
    _run(c, drv, k, 200)
    for s in (b, c):
        got, Fg = s.state(), s.forces()
        assert all(np.array_equal(got[q], want[q]) for q in want)
        assert np.array_equal(Fg[0], Fw[0]) and np.array_equal(Fg[1], Fw[1])
    for s in (a, b, c):
        s.close()


def test_activity_scan_flag_checked(crm):
    sc = _scene()
    with pytest.raises(crm.CrmError):
        crm.Simulation(sc, params=dict(sc.params, activity_scan=2))
    with pytest.raises(crm.CrmError):
        crm.Simulation(sc, params=dict(sc.params, moved_cap=-1))
